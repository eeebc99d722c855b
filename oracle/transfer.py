"""Prolongation P (Eq. (6)) and restriction R = P^dagger.

P_{alpha i j}(x) = u_i^(alpha)(x) for x in Lambda_j and 0 otherwise: P is block
diagonal, one N x k block U^(alpha)_j per aggregate and chirality.  Coarse
vectors are [nrhs][d][2][k] (dof order alpha, then i by descending singular value).
"""
import numpy as np

from .icsvd import chiral_block, chiral_unblock
from .geometry import block_sites


def prolong(U, vc, dims, block):
    """fine = P vc.  U [d][2][N][k], vc [nrhs][d][2][k] -> [nrhs][V][4][3]."""
    blocks = np.einsum("janl,rjal->janr", U, vc)
    return chiral_unblock(blocks, dims, block)


def restrict(U, psi, dims, block):
    """coarse = P^dagger psi.  psi [nrhs][V][4][3] -> [nrhs][d][2][k]."""
    B = chiral_block(psi, dims, block)            # [d][2][N][nrhs]
    return np.einsum("janl,janr->rjal", np.conj(U), B)


def dense_prolongator(U, dims, block):
    """Dense 12V x 2kd matrix of Eq. (6), built entry by entry (small lattices)."""
    bs = block_sites(dims, block)
    d, nd = bs.shape
    k = U.shape[-1]
    V = d * nd
    P = np.zeros((12 * V, 2 * k * d), dtype=np.complex128)
    for j in range(d):
        for a in range(2):
            for i in range(k):
                col = (2 * j + a) * k + i
                for ib in range(nd):
                    x = bs[j, ib]
                    for sp in range(2):
                        for c in range(3):
                            P[12 * x + 3 * (2 * a + sp) + c, col] = U[j, a, 6 * ib + 3 * sp + c, i]
    return P
