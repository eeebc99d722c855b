"""Pins of oracle.icsvd (Algorithm 3 and its special cases)."""
import numpy as np
import pytest

import fields
from oracle import icsvd as ic, geometry as geo, transfer
from oracle.gamma import CHIRAL_SPINS

DIMS, BLOCK = (4, 4, 2, 4), (2, 2, 2, 2)


def proj(U):
    return U @ np.conj(U.T)


def vecs(n, seed=1):
    return fields.gaussian_spinor(DIMS, n, seed)


def test_chiral_block_row_order_brute_force():
    psi = vecs(3)
    B = ic.chiral_block(psi, DIMS, BLOCK)
    bs = geo.block_sites(DIMS, BLOCK)
    for j in range(bs.shape[0]):
        for a in range(2):
            for ib in range(bs.shape[1]):
                for sp in range(2):
                    for c in range(3):
                        row = 6 * ib + 3 * sp + c
                        assert np.array_equal(B[j, a, row], psi[:, bs[j, ib], CHIRAL_SPINS[a][sp], c])
    assert np.array_equal(ic.chiral_unblock(B, DIMS, BLOCK), psi)


def test_no_truncation_equals_dense_svd():
    """k >= n_s r: the streaming SVD equals one SVD of all vectors (projector and sigma)."""
    r, ns, k = 4, 3, 12
    psis = [vecs(r, 10 + s) for s in range(ns)]
    U, S, _ = ic.icsvd(iter(psis), ns, DIMS, BLOCK, k)
    Ud, Sd = ic.csvd(np.concatenate(psis), DIMS, BLOCK, k)
    assert np.abs(S - Sd).max() < 1e-12 * Sd.max()
    for j in range(U.shape[0]):
        for a in range(2):
            assert np.linalg.norm(proj(U[j, a]) - proj(Ud[j, a])) < 1e-12


def test_one_stream_is_csvd_and_sigma_descending():
    psi = vecs(10, 3)
    U, S, _ = ic.icsvd(iter([psi]), 1, DIMS, BLOCK, 6)
    Ud, Sd = ic.csvd(psi, DIMS, BLOCK, 6)
    assert np.abs(S - Sd).max() < 1e-13
    assert np.all(np.diff(S, axis=-1) <= 0)
    # rank-k SVD is the best rank-k approximation: Eckart-Young error = sigma_{k+1}
    B = ic.chiral_block(psi, DIMS, BLOCK)
    s_all = np.linalg.svd(B[0, 0], compute_uv=False)
    Uk = U[0, 0]
    err = np.linalg.norm(B[0, 0] - Uk @ (np.conj(Uk.T) @ B[0, 0]), 2)
    assert abs(err - s_all[6]) < 1e-12


def test_exact_rank_recovery():
    """All test vectors in a fixed rank-k subspace per (j, alpha): span(U_k) equals it."""
    k, r, ns = 5, 3, 4
    rng = np.random.default_rng(7)
    N = 6 * int(np.prod(BLOCK))
    d = geo.volume(geo.coarse_dims(DIMS, BLOCK))
    basis = rng.standard_normal((d, 2, N, k)) + 1j * rng.standard_normal((d, 2, N, k))
    basis, _ = np.linalg.qr(basis)
    psis = []
    for s in range(ns):
        coef = rng.standard_normal((d, 2, k, r)) + 1j * rng.standard_normal((d, 2, k, r))
        psis.append(ic.chiral_unblock(basis @ coef, DIMS, BLOCK))
    U, S, _ = ic.icsvd(iter(psis), ns, DIMS, BLOCK, k)
    for j in range(d):
        for a in range(2):
            assert np.linalg.norm(proj(U[j, a]) - proj(basis[j, a])) < 1e-12


def test_loewner_bound_and_energy_identity():
    r, ns, k = 4, 4, 6
    psis = [vecs(r, 20 + s) for s in range(ns)]
    _, _, hist = ic.icsvd(iter(psis), ns, DIMS, BLOCK, k)
    Bs = [ic.chiral_block(p, DIMS, BLOCK) for p in psis]
    for s in range(ns):
        A = np.concatenate(Bs[:s + 1], axis=-1)
        for j in (0, 3):
            for a in range(2):
                sa = np.linalg.svd(A[j, a], compute_uv=False)
                ss = hist[s][j, a]
                assert np.all(ss <= sa[:len(ss)] * (1 + 1e-12))
                # energy: ||Phi_{s-1}||_F^2 + ||Psi_s||_F^2 = sum of all sigma_i^2 of the
                # concatenation; the kept part equals it exactly while nothing is truncated
                prev = 0.0 if s == 0 else float(np.sum(hist[s - 1][j, a] ** 2))
                energy = prev + np.linalg.norm(Bs[s][j, a]) ** 2
                ncols = (0 if s == 0 else len(hist[s - 1][j, a])) + r
                if ncols <= k:
                    assert abs(np.sum(ss ** 2) - energy) < 1e-12 * energy
                else:
                    assert np.sum(ss ** 2) <= energy * (1 + 1e-12)
                    assert np.sum(ss ** 2) >= energy * k / ncols * (1 - 1e-12)


def test_orthonormal_and_chiral_support():
    r, ns, k = 4, 3, 7
    psis = [vecs(r, 30 + s) for s in range(ns)]
    U, _, _ = ic.icsvd(iter(psis), ns, DIMS, BLOCK, k)
    for j in range(U.shape[0]):
        for a in range(2):
            assert np.abs(np.conj(U[j, a].T) @ U[j, a] - np.eye(k)).max() < 1e-13
    # gamma5 P = P sigma3 (chirality preserved), on the dense prolongator
    P = transfer.dense_prolongator(U, DIMS, BLOCK)
    V = geo.volume(DIMS)
    g5 = np.kron(np.eye(V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    d = U.shape[0]
    s3 = np.kron(np.eye(d), np.kron(np.diag([1, -1]), np.eye(k)))
    assert np.abs(g5 @ P - P @ s3).max() == 0.0


def test_least_squares_interpolation_identity():
    """Omega = I, V_f = U_k S_k V_k^dag, V_c = S_k V_k^dag gives P_j = U_k (Section 5, Eq. (9))."""
    psi = vecs(10, 4)
    B = ic.chiral_block(psi, DIMS, BLOCK)[2, 1]
    U, S, Vh = ic.rank_k_svd(B, 6)
    Vf = U @ np.diag(S) @ Vh
    Vc = np.diag(S) @ Vh
    Pj = Vf @ np.conj(Vc.T) @ np.linalg.inv(Vc @ np.conj(Vc.T))
    assert np.abs(Pj - U).max() < 1e-12


def test_span_invariant_under_unitary_mixing_within_stream():
    r, ns, k = 4, 3, 6
    psis = [vecs(r, 40 + s) for s in range(ns)]
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((r, r)) + 1j * rng.standard_normal((r, r)))
    mixed = [np.einsum("ij,jxsc->ixsc", Q.T, p) for p in psis]
    U1, S1, _ = ic.icsvd(iter(psis), ns, DIMS, BLOCK, k)
    U2, S2, _ = ic.icsvd(iter(mixed), ns, DIMS, BLOCK, k)
    assert np.abs(S1 - S2).max() < 1e-12
    for j in range(U1.shape[0]):
        for a in range(2):
            assert np.linalg.norm(proj(U1[j, a]) - proj(U2[j, a])) < 1e-10


def test_regular_same_span_as_single_stream_r_equals_k():
    k = 5
    psi = vecs(k, 6)
    Ur = ic.regular(psi, DIMS, BLOCK)
    Us, _, _ = ic.icsvd(iter([psi]), 1, DIMS, BLOCK, k)
    for j in range(Ur.shape[0]):
        for a in range(2):
            assert np.linalg.norm(proj(Ur[j, a]) - proj(Us[j, a])) < 1e-12


def test_too_few_vectors_rejected():
    with pytest.raises(ValueError):
        ic.icsvd(iter([vecs(2, 1), vecs(2, 2)]), 2, DIMS, BLOCK, 5)
