"""The Wilson-Dirac operator D and its adjoint (the matrix of Eq. (1)).

The paper only calls D "the lattice Dirac operator" and depends on the gauge
field, the quark mass and the volume (Section 1).  Reading used here (unimproved
Wilson, no clover term, anisotropy xi = a_s/a_t):

  (D psi)(x) = (m + 1 + 3/xi) psi(x)
               - 1/2 sum_mu c_mu [ s_mu(x)     (1 - gamma_mu) U_mu(x)         psi(x+mu)
                                 + s_mu(x-mu)  (1 + gamma_mu) U_mu(x-mu)^dag  psi(x-mu) ]

with c_t = 1, c_x = c_y = c_z = 1/xi, and s_mu(y) = bc_t if mu = t and y_t = Lt-1,
else +1 (periodic x, y, z; bc_t = -1 gives antiperiodic time).  The free field
(U = 1) has D(p) = m + sum_mu c_mu (1 - cos p_mu) + i sum_mu c_mu gamma_mu sin p_mu.
D^dagger = gamma_5 D gamma_5, i.e. the projectors swap sign.

Fields: U [4][V][3][3], psi [nrhs][V][4][3] (or [V][4][3]); complex128.
"""
import numpy as np

from .gamma import GAMMA, GAMMA5, ID4
from .geometry import volume, neighbor_table, hop_sign

# numpy axis of direction mu inside a field reshaped to (..., Lt, Lz, Ly, Lx, ...)
_AX = {0: 3, 1: 2, 2: 1, 3: 0}


def hop_weights(xi):
    return [1.0 / xi, 1.0 / xi, 1.0 / xi, 1.0]


def diag_term(mass, xi):
    return mass + 1.0 + 3.0 / xi


def apply_wilson(U, psi, mass, xi, bc_t, dims, dagger=False):
    """D psi (or D^dagger psi) by whole-lattice shifts (np.roll)."""
    single = psi.ndim == 3
    if single:
        psi = psi[None]
    nrhs = psi.shape[0]
    Lx, Ly, Lz, Lt = dims
    P = psi.reshape(nrhs, Lt, Lz, Ly, Lx, 4, 3)
    G = U.reshape(4, Lt, Lz, Ly, Lx, 3, 3)
    c = hop_weights(xi)
    sgn = -1.0 if dagger else 1.0          # D^dag = gamma5 D gamma5 flips (1 -/+ gamma)
    out = diag_term(mass, xi) * P
    tmask = np.ones((Lt, 1, 1, 1, 1, 1))
    if bc_t == -1:
        tmask_fwd = tmask.copy(); tmask_fwd[Lt - 1] = -1.0   # s_t(x) at x_t = Lt-1
        tmask_bwd = tmask.copy(); tmask_bwd[0] = -1.0        # s_t(x-t) at x_t = 0
    else:
        tmask_fwd = tmask_bwd = tmask
    for mu in range(4):
        ax = _AX[mu] + 1
        pm = ID4 - sgn * GAMMA[mu]     # forward projector (1 - gamma_mu)
        pp = ID4 + sgn * GAMMA[mu]     # backward projector (1 + gamma_mu)
        # forward: U_mu(x) psi(x+mu)
        fwd = np.roll(P, -1, axis=ax)
        fwd = np.einsum("TZYXab,nTZYXsb->nTZYXsa", G[mu], fwd)
        fwd = np.einsum("st,nTZYXtb->nTZYXsb", pm, fwd)
        # backward: U_mu(x-mu)^dag psi(x-mu)
        w = np.einsum("TZYXba,nTZYXsb->nTZYXsa", np.conj(G[mu]), P)
        bwd = np.roll(w, 1, axis=ax)
        bwd = np.einsum("st,nTZYXtb->nTZYXsb", pp, bwd)
        if mu == 3:
            fwd = fwd * tmask_fwd
            bwd = bwd * tmask_bwd
        out = out - 0.5 * c[mu] * (fwd + bwd)
    out = out.reshape(nrhs, volume(dims), 4, 3)
    return out[0] if single else out


def apply_wilson_adj(U, psi, mass, xi, bc_t, dims):
    return apply_wilson(U, psi, mass, xi, bc_t, dims, dagger=True)


def dense_wilson(U, mass, xi, bc_t, dims):
    """Dense n x n matrix of D, n = 12 V, row/column index 12*site + 3*spin + colour.

    Built entry by entry from the site loop, independently of apply_wilson; only for
    small lattices.
    """
    V = volume(dims)
    n = 12 * V
    Dm = np.zeros((n, n), dtype=np.complex128)
    nb = neighbor_table(dims)
    sg = hop_sign(dims, bc_t)
    c = hop_weights(xi)
    a = diag_term(mass, xi)
    for x in range(V):
        Dm[12 * x:12 * x + 12, 12 * x:12 * x + 12] += a * np.eye(12)
        for mu in range(4):
            y = nb[x, mu]
            blk = -0.5 * c[mu] * sg[x, mu] * np.kron(ID4 - GAMMA[mu], U[mu, x])
            Dm[12 * x:12 * x + 12, 12 * y:12 * y + 12] += blk
            z = nb[x, 4 + mu]
            blk = -0.5 * c[mu] * sg[x, 4 + mu] * np.kron(ID4 + GAMMA[mu], np.conj(U[mu, z]).T)
            Dm[12 * x:12 * x + 12, 12 * z:12 * z + 12] += blk
    return Dm


def gamma5(psi):
    """Multiply a spinor field by gamma_5 = diag(1, 1, -1, -1) in spin."""
    return np.einsum("st,...tc->...sc", GAMMA5, psi)


def free_field_eigenvalues(mass, xi, bc_t, dims):
    """Closed-form spectrum of D at U = 1: for each momentum p,
    lambda = m + sum c_mu (1 - cos p_mu) +/- i sqrt(sum c_mu^2 sin^2 p_mu), each 6-fold.
    p_mu = 2 pi n / L_mu, with p_t shifted by pi / Lt when bc_t = -1."""
    c = hop_weights(xi)
    ps = []
    for mu in range(4):
        n = np.arange(dims[mu])
        shift = np.pi if (mu == 3 and bc_t == -1) else 0.0
        ps.append((2 * np.pi * n + shift) / dims[mu])
    P = np.meshgrid(*ps, indexing="ij")
    re = mass + sum(c[mu] * (1 - np.cos(P[mu])) for mu in range(4))
    im = np.sqrt(sum((c[mu] * np.sin(P[mu])) ** 2 for mu in range(4)))
    lam = np.concatenate([(re + 1j * im).ravel(), (re - 1j * im).ravel()])
    return np.repeat(lam, 6)


def apply_wilson_sites(U, psi, sites, mass, xi, bc_t, dims, dagger=False):
    """(D psi)(x) for the listed sites only, hop by hop from the formula above (plain loops).

    Used to check full-size lattices at sampled sites.  psi: [V][4][3]; returns [len(sites)][4][3].
    """
    nb = neighbor_table(dims)
    sg = hop_sign(dims, bc_t)
    c = hop_weights(xi)
    a = diag_term(mass, xi)
    s = -1.0 if dagger else 1.0
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    for n, x in enumerate(sites):
        acc = a * psi[x]
        for mu in range(4):
            y = nb[x, mu]
            acc = acc - 0.5 * c[mu] * sg[x, mu] * ((ID4 - s * GAMMA[mu]) @ (psi[y] @ U[mu, x].T))
            z = nb[x, 4 + mu]
            acc = acc - 0.5 * c[mu] * sg[x, 4 + mu] * ((ID4 + s * GAMMA[mu]) @ (psi[z] @ np.conj(U[mu, z])))
        out[n] = acc
    return out
