"""Even-odd (red-black) preconditioning of the fine operator.

The paper names even-odd preconditioning among the standard accelerations of the Dirac solve
(Section 1) without writing it out.  Reading used here (the textbook Schur-complement form):
order the sites by parity p(x) = (x + y + z + t) mod 2.  The hops of D (Wilson or
Wilson-clover) join sites of opposite parity, and the site term A (the diagonal term, plus T(x)
with the clover term) is local, so

  D = [[A_ee, D_eo], [D_oe, A_oo]],

and D x = b is solved through the Schur complement on the even sites

  Dhat = A_ee - D_eo A_oo^-1 D_oe,        Dhat x_e = b_e - D_eo A_oo^-1 b_o,
  x_o  = A_oo^-1 (b_o - D_oe x_e).

A commutes with gamma_5 and is hermitian, so Dhat^dag = gamma_5 Dhat gamma_5 and the Schur
complement of D^dag is Dhat^dag.  Requires every extent even: a hop across a periodic
boundary of odd extent would join two sites of the same parity.  Each parity then holds V/2
sites, and the half-lattice index of a site is its lexicographic index divided by 2.

Fields here are full-lattice arrays [nrhs][V][4][3]; even and odd parts are selected by masks.
"""
import numpy as np

from . import wilson, krylov
from .geometry import coords, volume


def parity(dims):
    """[V] 0 for even sites, 1 for odd sites."""
    return coords(dims).sum(axis=1) % 2


def site_term(T, mass, xi, V):
    """A(x) [V][12][12]: the diagonal term, plus the clover term T if given."""
    A = wilson.diag_term(mass, xi) * np.broadcast_to(np.eye(12), (V, 12, 12)).copy()
    if T is not None:
        A = A + T
    return A


def hop(U, psi, mass, xi, bc_t, dims, dagger=False):
    """The hopping part H = D - A of the Wilson operator (it joins opposite parities)."""
    return wilson.apply_wilson(U, psi, mass, xi, bc_t, dims, dagger) - wilson.diag_term(mass, xi) * psi


def apply_site(M, psi):
    """(M psi)(x) = M(x) psi(x) for a site-local M [V][12][12] and psi [nrhs][V][4][3]."""
    n = psi.shape[0]
    V = M.shape[0]
    return np.einsum("xab,nxb->nxa", M, psi.reshape(n, V, 12)).reshape(psi.shape)


def restrict_parity(psi, par, p):
    """psi on the sites of parity p, zero elsewhere."""
    out = psi.copy()
    out[:, par != p] = 0
    return out


class EvenOdd:
    """The Schur-complement pieces of D for a gauge field, mass, anisotropy, boundary and
    optional clover term T."""

    def __init__(self, U, dims, mass, xi=1.0, bc_t=-1, T=None):
        if any(L % 2 for L in dims):
            raise ValueError("even-odd preconditioning needs every extent even")
        self.U, self.dims, self.mass, self.xi, self.bc_t = U, tuple(dims), mass, xi, bc_t
        V = volume(dims)
        self.par = parity(dims)
        self.A = site_term(T, mass, xi, V)
        self.Ainv = np.linalg.inv(self.A)

    def H(self, psi, dagger=False):
        return hop(self.U, psi, self.mass, self.xi, self.bc_t, self.dims, dagger)

    def schur(self, x_e, dagger=False):
        """Dhat x_e (or Dhat^dag x_e) for x_e supported on the even sites."""
        u = restrict_parity(self.H(x_e, dagger), self.par, 1)        # D_oe x_e
        u = apply_site(self.Ainv, u)                                   # A_oo^-1 D_oe x_e
        v = restrict_parity(self.H(u, dagger), self.par, 0)           # D_eo A_oo^-1 D_oe x_e
        return restrict_parity(apply_site(self.A, x_e), self.par, 0) - v

    def prepare(self, b, dagger=False):
        """bhat_e = b_e - D_eo A_oo^-1 b_o."""
        u = apply_site(self.Ainv, restrict_parity(b, self.par, 1))
        return restrict_parity(b, self.par, 0) - restrict_parity(self.H(u, dagger), self.par, 0)

    def reconstruct(self, x_e, b, dagger=False):
        """x = x_e + A_oo^-1 (b_o - D_oe x_e)."""
        r_o = restrict_parity(b, self.par, 1) - restrict_parity(self.H(x_e, dagger), self.par, 1)
        return x_e + apply_site(self.Ainv, r_o)

    def solve(self, b, tol=1e-12, restart=32, max_iter=5000, dagger=False):
        """D x = b (or D^dag x = b) by GMRES on the Schur complement; returns (x, iterations)."""
        bh = self.prepare(b, dagger)
        x_e, it, _ = krylov.gmres(lambda v: self.schur(v, dagger), bh, None, restart=restart, max_iter=max_iter,
                                  tol=tol)
        return self.reconstruct(x_e, b, dagger), it


def dense_schur(D, par):
    """The Schur complement from the dense (12V) x (12V) matrix of D, in even-site order."""
    e = np.repeat(par == 0, 12)
    o = ~e
    Dee, Deo, Doe, Doo = D[np.ix_(e, e)], D[np.ix_(e, o)], D[np.ix_(o, e)], D[np.ix_(o, o)]
    return Dee - Deo @ np.linalg.solve(Doo, Doe)
