"""Even-odd (red-black) form of the Galerkin coarse operator.

The paper names even-odd preconditioning among the standard accelerations of the Dirac solve
(Section 1); the coarse operator D_c = R D P (Eq. (5)) is a nine-block nearest-neighbour
stencil on the lattice of aggregates, so the same Schur-complement construction applies to it
(reading used here): colour the aggregates by the parity of their coarse coordinates,
p(j) = (j_x + j_y + j_z + j_t) mod 2.  Every hop block Y_{1+d}(j) joins j to a neighbour of the
other colour when every coarse extent is even, and Y_0(j) is local, so

  D_c = [[Y_ee, Y_eo], [Y_oe, Y_oo]],   Y_ee, Y_oo block diagonal,

  Dhat_c = Y_ee - Y_eo Y_oo^-1 Y_oe,    Dhat_c v_e = r_e - Y_eo Y_oo^-1 r_o,
  v_o = Y_oo^-1 (r_o - Y_oe v_e).

Vectors here are full coarse vectors [nrhs][d][2k]; the even and odd parts are selected by
masks, and the Schur operator returns zeros on the odd aggregates.
"""
import numpy as np

from . import krylov
from .coarse import coarse_apply
from .geometry import coords, neighbor_table


def aggregate_parity(cdims):
    """[d] 0 for even aggregates, 1 for odd ones."""
    return coords(cdims).sum(axis=1) % 2


def restrict_parity(v, par, p):
    """v on the aggregates of parity p, zero elsewhere."""
    out = v.copy()
    out[:, par != p] = 0
    return out


class CoarseEvenOdd:
    """Schur-complement pieces of the coarse stencil Y [d][9][2k][2k] on coarse extents cdims."""

    def __init__(self, Y, cdims):
        if any(L % 2 for L in cdims):
            raise ValueError("even-odd coarse operator needs every coarse extent even")
        self.Y, self.cdims = Y, tuple(cdims)
        self.par = aggregate_parity(cdims)
        self.cnb = neighbor_table(cdims)
        self.Yinv = np.linalg.inv(Y[:, 0])  # the inverse of every self block

    def block_diag(self, M, v):
        """(M v)(j) = M(j) v(j)."""
        return np.einsum("jab,rjb->rja", M, v)

    def hop(self, v):
        """The hop part of D_c: sum over d of Y_{1+d}(j) v(j + dir_d)."""
        out = np.zeros_like(v)
        for dd in range(8):
            out += np.einsum("jab,rjb->rja", self.Y[:, 1 + dd], v[:, self.cnb[:, dd]])
        return out

    def schur(self, v_e):
        """Dhat_c v_e for v_e supported on the even aggregates."""
        u = restrict_parity(self.hop(v_e), self.par, 1)   # Y_oe v_e
        u = self.block_diag(self.Yinv, u)                 # Y_oo^-1 Y_oe v_e
        w = restrict_parity(self.hop(u), self.par, 0)     # Y_eo Y_oo^-1 Y_oe v_e
        return restrict_parity(self.block_diag(self.Y[:, 0], v_e), self.par, 0) - w

    def prepare(self, r):
        """rhat_e = r_e - Y_eo Y_oo^-1 r_o."""
        u = self.block_diag(self.Yinv, restrict_parity(r, self.par, 1))
        return restrict_parity(r, self.par, 0) - restrict_parity(self.hop(u), self.par, 0)

    def reconstruct(self, v_e, r):
        """v = v_e + Y_oo^-1 (r_o - Y_oe v_e)."""
        t = restrict_parity(r, self.par, 1) - restrict_parity(self.hop(v_e), self.par, 1)
        return v_e + self.block_diag(self.Yinv, t)

    def solve(self, r, tol=1e-12, restart=32, max_iter=5000):
        """D_c v = r by GMRES on the Schur complement; returns (v, iterations)."""
        rh = self.prepare(r)
        v_e, it, _ = krylov.gmres(self.schur, rh, None, restart=restart, max_iter=max_iter, tol=tol)
        return self.reconstruct(v_e, r), it

    def apply_full(self, v):
        """D_c v through the split pieces (equals coarse_apply)."""
        return self.block_diag(self.Y[:, 0], v) + self.hop(v)


def dense_schur(Dc, par, m):
    """The Schur complement from the dense (d m) x (d m) coarse matrix, in even-aggregate order."""
    e = np.repeat(par == 0, m)
    o = ~e
    Dee, Deo, Doe, Doo = Dc[np.ix_(e, e)], Dc[np.ix_(e, o)], Dc[np.ix_(o, e)], Dc[np.ix_(o, o)]
    return Dee - Deo @ np.linalg.solve(Doo, Doe)


__all__ = ["aggregate_parity", "restrict_parity", "CoarseEvenOdd", "dense_schur", "coarse_apply"]
