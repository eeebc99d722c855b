"""The clover (Sheikholeslami-Wohlert) term and the Wilson-clover operator.

The paper runs its multigrid on Wilson fermions with the clover term added (the
action of its experiments, Section 4) but writes no formula for it.  Reading used
here: the O(a)-improvement term of Luescher, Sint, Sommer and Weisz (1996) in the
normalisation of the Wilson operator of wilson.py,

  D_sw = D_W + T,   T(x) = sum_{mu<nu} c_{mu nu} (i/2) sigma_{mu nu} (x) Fhat_{mu nu}(x)

(which is c (i/4) sum over all ordered pairs mu != nu), with

  sigma_{mu nu}    = (i/2) [gamma_mu, gamma_nu]
  Fhat_{mu nu}(x)  = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) / 8     (no trace subtraction)
  Q_{mu nu}(x)     = the four plaquettes of the mu-nu plane that have a corner at x, each
                     a closed path from x that turns from mu to nu (the "clover leaves")
  c_{mu nu}        = c_t if mu or nu is the time direction, else c_s.

With c_s = c_t = c_sw this is the isotropic clover term; on an anisotropic lattice the
two coefficients are the caller's.  The gauge field is periodic in every direction,
so T does not see the fermion boundary condition.  T(x) is hermitian and commutes with
gamma_5, so D_sw keeps gamma_5-hermiticity (D_sw^dag = gamma_5 D_sw gamma_5) and in the
chiral basis T(x) is two hermitian 6 x 6 blocks, one per chirality.

Fields: U [4][V][3][3], T [V][12][12] with spinor index spin*3 + colour.
"""
import numpy as np

from .gamma import GAMMA, GAMMA5
from . import wilson

_AX = {0: 3, 1: 2, 2: 1, 3: 0}  # numpy axis of direction mu in a field shaped (Lt, Lz, Ly, Lx, ...)


def sigma(mu, nu):
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu] (4 x 4)."""
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


def _shift(F, mu, step):
    """The field at x + step * mu, for F shaped (Lt, Lz, Ly, Lx, 3, 3)."""
    return np.roll(F, -step, axis=_AX[mu])


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def leaves(U, dims, mu, nu):
    """Q_{mu nu}(x) [V][3][3]: the sum of the four plaquettes with a corner at x, each walked
    from x and back counter-clockwise in the (mu, nu) plane (a step along mu is followed by
    one along nu)."""
    Lx, Ly, Lz, Lt = dims
    G = U.reshape(4, Lt, Lz, Ly, Lx, 3, 3)
    Um, Un = G[mu], G[nu]
    S = _shift
    # x -> x+mu -> x+mu+nu -> x+nu -> x
    q1 = Um @ S(Un, mu, 1) @ _dag(S(Um, nu, 1)) @ _dag(Un)
    # x -> x+nu -> x+nu-mu -> x-mu -> x
    q2 = Un @ _dag(S(S(Um, nu, 1), mu, -1)) @ _dag(S(Un, mu, -1)) @ S(Um, mu, -1)
    # x -> x-mu -> x-mu-nu -> x-nu -> x
    q3 = _dag(S(Um, mu, -1)) @ _dag(S(S(Un, mu, -1), nu, -1)) @ S(S(Um, mu, -1), nu, -1) @ S(Un, nu, -1)
    # x -> x-nu -> x-nu+mu -> x+mu -> x
    q4 = _dag(S(Un, nu, -1)) @ S(Um, nu, -1) @ S(S(Un, nu, -1), mu, 1) @ _dag(Um)
    return (q1 + q2 + q3 + q4).reshape(-1, 3, 3)


def field_strength(U, dims, mu, nu):
    """Fhat_{mu nu}(x) = (Q - Q^dag) / 8, [V][3][3] anti-hermitian."""
    Q = leaves(U, dims, mu, nu)
    return (Q - _dag(Q)) / 8.0


def clover_term(U, dims, c_s, c_t):
    """T(x) [V][12][12] (spin*3 + colour), the sum over the six planes."""
    V = U.shape[1]
    T = np.zeros((V, 12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            c = c_t if (mu == 3 or nu == 3) else c_s
            F = field_strength(U, dims, mu, nu)
            T += c * 0.5j * np.einsum("st,xab->xsatb", sigma(mu, nu), F).reshape(V, 12, 12)
    return T


def apply_clover(U, T, psi, mass, xi, bc_t, dims, dagger=False):
    """D_sw psi (or D_sw^dag psi): the Wilson stencil plus T(x) psi(x); T is hermitian and
    commutes with gamma_5, so it is the same term in the adjoint."""
    out = wilson.apply_wilson(U, psi, mass, xi, bc_t, dims, dagger=dagger)
    single = psi.ndim == 3
    p = psi[None] if single else psi
    V = T.shape[0]
    add = np.einsum("xab,nxb->nxa", T, p.reshape(p.shape[0], V, 12)).reshape(p.shape)
    return out + (add[0] if single else add)


def dense_clover(U, T, mass, xi, bc_t, dims):
    """The (12V) x (12V) matrix of D_sw (small lattices only)."""
    D = wilson.dense_wilson(U, mass, xi, bc_t, dims)
    V = T.shape[0]
    for x in range(V):
        D[12 * x:12 * x + 12, 12 * x:12 * x + 12] += T[x]
    return D


def site_term(T, mass, xi):
    """A(x) = (m + 1 + 3/xi) 1 + T(x), the whole site-local part of D_sw, [V][12][12]."""
    return wilson.diag_term(mass, xi) * np.eye(12)[None] + T


def chiral_blocks(A):
    """[V][2][6][6]: the two chirality blocks of a site term that commutes with gamma_5
    (spins 0,1 for alpha = 0 and spins 2,3 for alpha = 1)."""
    return np.stack([A[:, :6, :6], A[:, 6:, 6:]], axis=1)


def gamma5_commutes(T):
    """max |[T(x), gamma_5 (x) 1]| over the lattice."""
    g5 = np.kron(GAMMA5, np.eye(3))
    return float(np.abs(T @ g5 - g5 @ T).max())
