"""Pins of the next-coarser-level oracle (oracle/level.py) against facts that do not come from
the oracle itself: the published fine test-vector generator, dense Galerkin products,
sigma3-hermiticity, unitary similarity at full rank, and uniqueness of the solution."""
import numpy as np
import pytest

import fields
from oracle import coarse, geometry as geo, level, mg as omg, philox, wilson


def _sigma3(d, k):
    return np.kron(np.eye(d), np.diag(np.r_[np.ones(k), -np.ones(k)]))


@pytest.fixture(scope="module")
def c1_hier():
    """Level one of a 4^4 lattice (2^4 aggregates, k = 4) with its D_c."""
    dims = (4, 4, 4, 4)
    U = fields.random_gauge(dims, 0.3, 41)
    lat = omg.Lattice(U, dims, 0.05, 1.0, -1)
    h = omg.setup(lat, (2, 2, 2, 2), 8, 4, 4, n_setup_iter=4, seed=3)
    return h


def test_coarse_generator_reduces_to_the_fine_one():
    """Level 0 with 12 components per site is the fine test-vector generator, which the
    Philox known-answer vectors pin."""
    V = 40
    for v in (0, 7):
        a = level.gaussian_coarse_vector(14399, v, V, 12, 0)
        b = philox.gaussian_test_vector(14399, v, V).reshape(V, 12)
        assert np.array_equal(a, b)
    # another level gives other numbers
    assert not np.allclose(level.gaussian_coarse_vector(14399, 0, V, 12, 1), a)


def test_galerkin_equals_dense_product(c1_hier):
    """Stencil form of P2^dag D_c P2 equals the dense product, including coarse-coarse extents
    1 and 2 where several directional blocks reach the same aggregate."""
    h = c1_hier
    Y, cd, k = h.Y, h.cdims, h.k
    d = Y.shape[0]
    rng = np.random.default_rng(5)
    for block2 in ((2, 2, 2, 2), (1, 2, 2, 1), (2, 1, 1, 2)):
        cd2 = geo.coarse_dims(cd, block2)
        nd2 = int(np.prod(block2))
        d2 = int(np.prod(cd2))
        k2 = 3
        # orthonormal random P2 blocks
        P2 = np.empty((d2, 2, nd2 * k, k2), dtype=np.complex128)
        for J in range(d2):
            for a in range(2):
                q, _ = np.linalg.qr(rng.normal(size=(nd2 * k, k2)) + 1j * rng.normal(size=(nd2 * k, k2)))
                P2[J, a] = q
        Y2 = level.galerkin(Y, P2, cd, block2, k)
        Pd = np.zeros((d * 2 * k, d2 * 2 * k2), dtype=np.complex128)
        e = np.eye(d2 * 2 * k2)
        for c in range(d2 * 2 * k2):
            Pd[:, c] = level.prolong(P2, e[c].reshape(1, d2, 2, k2), cd, block2, k).ravel()
        dense = np.conj(Pd).T @ coarse.dense_coarse(Y, cd) @ Pd
        assert np.abs(coarse.dense_coarse(Y2, cd2) - dense).max() < 1e-12 * np.abs(dense).max()
        # restriction is the adjoint of prolongation, P2^dag P2 = I
        v = rng.normal(size=(2, d2, 2, k2)) + 1j * rng.normal(size=(2, d2, 2, k2))
        w = rng.normal(size=(2, d, 2 * k)) + 1j * rng.normal(size=(2, d, 2 * k))
        assert np.allclose(level.restrict(P2, level.prolong(P2, v, cd, block2, k), cd, block2, k), v, atol=1e-12)
        lhs = np.vdot(level.prolong(P2, v, cd, block2, k), w)
        rhs = np.vdot(v, level.restrict(P2, w, cd, block2, k))
        assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_level_setup_keeps_sigma3_hermiticity(c1_hier):
    """D_c is sigma3-hermitian (gamma5 P = P sigma3); a chirally split P2 keeps that for D_cc."""
    h = c1_hier
    d, m = h.Y.shape[0], h.Y.shape[-1]
    Dc = coarse.dense_coarse(h.Y, h.cdims)
    s3 = _sigma3(d, m // 2)
    assert np.abs(s3 @ Dc @ s3 - np.conj(Dc).T).max() < 1e-12 * np.abs(Dc).max()
    lv = level.setup(h.Y, h.cdims, (2, 2, 2, 2), 8, 4, 3, n_setup_iter=4, seed=3)
    d2, m2 = lv.Y2.shape[0], lv.Y2.shape[-1]
    Dcc = coarse.dense_coarse(lv.Y2, lv.cdims2)
    s3 = _sigma3(d2, m2 // 2)
    assert np.abs(s3 @ Dcc @ s3 - np.conj(Dcc).T).max() < 1e-12 * np.abs(Dcc).max()
    # orthonormal columns per (aggregate, chirality), singular values descending
    for J in range(d2):
        for a in range(2):
            P = lv.P[J, a]
            assert np.abs(np.conj(P).T @ P - np.eye(P.shape[1])).max() < 1e-12
            assert np.all(np.diff(lv.sigma[J, a]) <= 1e-14)


def test_full_rank_level_is_a_unitary_similarity(c1_hier):
    """Blocks of one coarse site and k2 = k: P2 is unitary per (site, chirality), so D_cc and D_c
    have the same eigenvalues."""
    h = c1_hier
    k = h.k
    lv = level.setup(h.Y, h.cdims, (1, 1, 1, 1), 8, 4, k, n_setup_iter=2, seed=4)
    def spectrum(Y, cd):  # rounded before sorting so that conjugate pairs keep their order
        ev = np.linalg.eigvals(coarse.dense_coarse(Y, cd))
        return np.sort_complex(np.round(ev.real, 8) + 1j * np.round(ev.imag, 8))

    assert np.abs(spectrum(h.Y, h.cdims) - spectrum(lv.Y2, lv.cdims2)).max() < 1e-7


def test_streaming_on_the_coarse_level_recovers_an_exact_rank():
    """Coarse test vectors inside a fixed rank-k2 subspace per (aggregate, chirality): the
    streamed basis spans exactly that subspace (no smoothing)."""
    dims = (4, 4, 4, 4)
    U = fields.random_gauge(dims, 0.3, 42)
    lat = omg.Lattice(U, dims, 0.05, 1.0, -1)
    h = omg.setup(lat, (2, 2, 2, 2), 8, 4, 4, n_setup_iter=2, seed=3)
    d, m, k = h.Y.shape[0], h.Y.shape[-1], h.k
    block2, k2 = (2, 2, 2, 2), 3
    cd2 = geo.coarse_dims(h.cdims, block2)
    d2, nd2 = int(np.prod(cd2)), 16
    rng = np.random.default_rng(8)
    basis = rng.normal(size=(d2, 2, nd2 * k, k2)) + 1j * rng.normal(size=(d2, 2, nd2 * k, k2))
    n_test = 12
    coef = rng.normal(size=(n_test, d2, 2, k2)) + 1j * rng.normal(size=(n_test, d2, 2, k2))
    tv = np.zeros((n_test, d, m), dtype=np.complex128)
    bs = geo.block_sites(h.cdims, block2)
    for v in range(n_test):
        for J in range(d2):
            for a in range(2):
                col = basis[J, a] @ coef[v, J, a]            # rows (site in block, i)
                tv[v, bs[J], a * k:(a + 1) * k] = col.reshape(nd2, k)
    lv = level.setup(h.Y, h.cdims, block2, n_test, 4, k2, n_setup_iter=0, test_vectors=tv)
    for J in range(d2):
        for a in range(2):
            q, _ = np.linalg.qr(basis[J, a])
            assert np.abs(q @ np.conj(q).T - lv.P[J, a] @ np.conj(lv.P[J, a]).T).max() < 1e-10


def test_three_level_solve_matches_the_dense_solution():
    """Three-level K-cycle solve to 1e-12: the solution equals the dense LU solution (unique)."""
    dims = (4, 4, 4, 8)
    U = fields.random_gauge(dims, 0.3, 43)
    lat = omg.Lattice(U, dims, 0.1, 1.0, -1)
    h = omg.setup(lat, (2, 2, 2, 2), 12, 4, 6, n_setup_iter=8, seed=6)
    lv = level.setup(h.Y, h.cdims, (2, 2, 1, 2), 12, 4, 4, n_setup_iter=8, seed=6)
    b = fields.gaussian_spinor(dims, 1, 44)[0]
    x, st = level.solve3(h, lv, b, tol=1e-12)
    assert st["true_rel_res"] < 1e-12
    Dd = wilson.dense_wilson(U, 0.1, 1.0, -1, dims)
    xd = np.linalg.solve(Dd, b.ravel())
    assert np.linalg.norm(x.ravel() - xd) < 1e-9 * np.linalg.norm(xd)
    assert st["coarse2"] > 0 and st["smoother1"] > 0


def test_four_level_solve_matches_the_dense_solution():
    """A fourth level set up on the third level's stencil (level word 2); the four-level solve at
    1e-12 gives the dense LU solution."""
    dims = (4, 4, 4, 8)
    U = fields.random_gauge(dims, 0.3, 45)
    lat = omg.Lattice(U, dims, 0.1, 1.0, -1)
    h = omg.setup(lat, (2, 2, 2, 2), 12, 4, 6, n_setup_iter=8, seed=6)
    lv2 = level.setup(h.Y, h.cdims, (2, 2, 1, 2), 12, 4, 4, n_setup_iter=8, seed=6, level=1)
    lv3 = level.setup(lv2.Y2, lv2.cdims2, (1, 1, 2, 1), 8, 4, 3, n_setup_iter=8, seed=6, level=2)
    assert lv3.cdims2 == (1, 1, 1, 2)
    b = fields.gaussian_spinor(dims, 1, 46)[0]
    x, st = level.solve_levels(h, [lv2, lv3], b, tol=1e-12)
    assert st["true_rel_res"] < 1e-12 and st["iters"][3] > 0 and st["smooth"][2] > 0
    xd = np.linalg.solve(wilson.dense_wilson(U, 0.1, 1.0, -1, dims), b.ravel())
    assert np.linalg.norm(x.ravel() - xd) < 1e-9 * np.linalg.norm(xd)
