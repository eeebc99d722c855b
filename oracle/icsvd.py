"""Chiral split, block gather and the (streaming) chiral SVD of the test vectors.

Section 2.1, Eq. (3): the chirality projectors split a test vector's spin
components into alpha = 0 (spins 1,2) and alpha = 1 (spins 3,4).  Blocking onto
an aggregate Lambda_j restricts it to the sites of that block.  The rows of
Psi^(alpha)(Lambda_j) are ordered (site-in-block, spin-in-chirality, colour),
N = 6 n_d rows; the columns are the test vectors.

Algorithm 3 (iCSVD, Eqs. (7)-(8)): for every stream s the r new vectors are
appended to Phi_{s-1} = U_k Sigma_k and a rank-k SVD of the concatenation is
taken; the last stream returns U_k.  Algorithm 2 (CSVD) is the one-stream case
with all m vectors at once; Algorithm 1 ("Regular") orthonormalises k vectors.
"""
import numpy as np

from .geometry import block_sites, coarse_dims, volume
from .gamma import CHIRAL_SPINS


def chiral_block(psi, dims, block):
    """psi [r][V][4][3] -> blocks [d][2][N][r] (Eq. (3) + restriction to Lambda_j)."""
    bs = block_sites(dims, block)                 # [d][n_d]
    d, nd = bs.shape
    r = psi.shape[0]
    out = np.empty((d, 2, 6 * nd, r), dtype=np.complex128)
    for a in range(2):
        sp = list(CHIRAL_SPINS[a])
        sub = psi[:, :, sp, :]                    # [r][V][2][3]
        g = sub[:, bs]                            # [r][d][n_d][2][3]
        out[:, a] = g.reshape(r, d, 6 * nd).transpose(1, 2, 0)
    return out


def chiral_unblock(blocks, dims, block):
    """Inverse of chiral_block: [d][2][N][r] -> [r][V][4][3]."""
    bs = block_sites(dims, block)
    d, nd = bs.shape
    r = blocks.shape[-1]
    out = np.zeros((r, volume(dims), 4, 3), dtype=np.complex128)
    for a in range(2):
        sp = list(CHIRAL_SPINS[a])
        g = blocks[:, a].transpose(2, 0, 1).reshape(r, d, nd, 2, 3)
        for i, s in enumerate(sp):
            out[:, bs, s, :] = g[:, :, :, i, :]
    return out


def rank_k_svd(C, k):
    """First k singular triplets of C (LAPACK gesdd via numpy), descending order."""
    U, S, Vh = np.linalg.svd(C, full_matrices=False)
    kk = min(k, S.shape[0])
    return U[:, :kk], S[:kk], Vh[:kk]


def icsvd_update(Phi, Psi, k):
    """One stream of Algorithm 3 for one (j, alpha): rank-k SVD of [Phi_{s-1}, Psi_s].

    Phi is None for the first stream (Phi_{-1} is empty).  When the concatenation has
    fewer than k columns all of them are kept.  Returns (U_k, Sigma_k).
    """
    C = Psi if Phi is None else np.concatenate([Phi, Psi], axis=1)
    U, S, _ = rank_k_svd(C, k)
    return U, S


def icsvd(streams, n_s, dims, block, k):
    """Algorithm 3 over all aggregates and both chiralities.

    streams: iterable yielding n_s arrays [r][V][4][3] (the smoothed test vectors of
    each stream), consumed one at a time so that only Phi = U_k Sigma_k is kept.
    Returns (U [d][2][N][k], Sigma [d][2][k], list of Sigma per stream).
    """
    Phi = None
    hist = []
    for s, psi in enumerate(streams):
        B = chiral_block(psi, dims, block)       # [d][2][N][r]
        d = B.shape[0]
        Us = [[None, None] for _ in range(d)]
        Ss = [[None, None] for _ in range(d)]
        for a in range(2):
            for j in range(d):
                Us[j][a], Ss[j][a] = icsvd_update(None if Phi is None else Phi[j][a], B[j, a], k)
        hist.append(np.array(Ss))
        if s == n_s - 1:
            if Us[0][0].shape[1] < k:
                raise ValueError("n_s * r must be at least k")
            return np.array(Us), hist[-1], hist
        Phi = [[Us[j][a] * Ss[j][a][None, :] for a in range(2)] for j in range(d)]
    raise ValueError("fewer streams than n_s")


def csvd(psi_all, dims, block, k):
    """Algorithm 2: one rank-k SVD of all m test vectors per (j, alpha)."""
    B = chiral_block(psi_all, dims, block)
    d = B.shape[0]
    U = np.empty((d, 2, B.shape[2], k), dtype=np.complex128)
    S = np.empty((d, 2, k))
    for j in range(d):
        for a in range(2):
            u, s, _ = rank_k_svd(B[j, a], k)
            U[j, a], S[j, a] = u, s
    return U, S


def regular(psi_k, dims, block):
    """Algorithm 1: orthonormalise the k blocked, chirally split vectors (QR)."""
    B = chiral_block(psi_k, dims, block)
    d = B.shape[0]
    U = np.empty_like(B)
    for j in range(d):
        for a in range(2):
            q, _ = np.linalg.qr(B[j, a])
            U[j, a] = q
    return U
