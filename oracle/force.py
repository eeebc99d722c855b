"""Gradient of L = Re <eta, D^-1 b> with respect to b and to the gauge links.

Not a result of the paper: it differentiates the solve whose preconditioner the
paper builds.  With x = D^-1 b and lambda = D^-dagger eta (one adjoint solve,
D^-dagger = gamma5 D^-1 gamma5):

  dL/db          = lambda                 (gradient convention dL/dRe + i dL/dIm)
  dL/dU_mu(x)    = 1/2 c_mu s_mu(x) G_mu(x)^dagger,
  G_mu(x)        = tr_spin[(1 - gamma_mu) x(x+mu) lambda(x)^dagger]
                 + tr_spin[(1 + gamma_mu) lambda(x+mu) x(x)^dagger]

obtained from dL = -Re(lambda^dagger dD x) with D of oracle.wilson.  Sums over
right-hand sides when x, lambda carry several.
"""
import numpy as np

from .gamma import GAMMA, ID4
from .geometry import neighbor_table, hop_sign
from .wilson import hop_weights


def link_force(x, lam, xi, bc_t, dims):
    """[4][V][3][3] complex gradient; x, lam [nrhs][V][4][3] or [V][4][3]."""
    if x.ndim == 3:
        x, lam = x[None], lam[None]
    nb = neighbor_table(dims)
    sg = hop_sign(dims, bc_t)
    c = hop_weights(xi)
    V = x.shape[1]
    dU = np.zeros((4, V, 3, 3), dtype=np.complex128)
    for mu in range(4):
        y = nb[:, mu]
        pm = ID4 - GAMMA[mu]
        pp = ID4 + GAMMA[mu]
        # tr_s[(1-g) x(x+mu) lam(x)^dag]_{ab} = sum_{s,t} pm[s,t] x_{t a}(x+mu) conj(lam_{s b}(x))
        g1 = np.einsum("st,rxta,rxsb->xab", pm, x[:, y], np.conj(lam))
        g2 = np.einsum("st,rxta,rxsb->xab", pp, lam[:, y], np.conj(x))
        G = g1 + g2
        dU[mu] = 0.5 * c[mu] * sg[:, mu][:, None, None] * np.conj(np.swapaxes(G, -1, -2))
    return dU


def loss(lat_solve, eta, b):
    """Re <eta, D^-1 b> given a solver callable."""
    x = lat_solve(b)
    return float(np.real(np.vdot(eta.ravel(), x.ravel())))
