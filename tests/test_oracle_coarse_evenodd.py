"""Pins of the even-odd coarse oracle (oracle/coarse_evenodd.py) on Galerkin coarse operators: the
hop blocks join opposite aggregate colours, the Schur complement equals the one cut from the
dense coarse matrix, the determinant factorises, the Schur complement keeps the
sigma3-hermiticity of D_c, the preconditioned solve equals dense LU, and the no-hop special
case."""
import numpy as np
import pytest

import fields
from oracle import icsvd as ic, coarse, coarse_evenodd as ceo, geometry as geo, krylov


def galerkin(dims, block, k, seed=41, mass=0.05, xi=2.0):
    psi = fields.gaussian_spinor(dims, k + 2, seed)
    U, _ = ic.csvd(psi, dims, block, k)
    G = fields.random_gauge(dims, 0.5, seed)
    return coarse.build_coarse(G, U, mass, xi, -1, dims, block), geo.coarse_dims(dims, block)


CASES = [((4, 4, 4, 8), (2, 2, 2, 2), 3),   # coarse 2 x 2 x 2 x 4: +mu and -mu reach one aggregate
         ((8, 4, 4, 4), (2, 2, 2, 2), 2)]   # coarse 4 x 2 x 2 x 2


@pytest.mark.parametrize("dims,block,k", CASES)
def test_hops_join_opposite_colours(dims, block, k):
    Y, cd = galerkin(dims, block, k)
    eo = ceo.CoarseEvenOdd(Y, cd)
    assert np.all(eo.par[eo.cnb] != eo.par[:, None])
    d, m = Y.shape[0], Y.shape[2]
    v = fields.gaussian_coarse(d * m, 2, 42).reshape(2, d, m)
    for p in (0, 1):
        h = eo.hop(ceo.restrict_parity(v, eo.par, p))
        assert np.abs(h[:, eo.par == p]).max() == 0.0
    # the split pieces add up to the stencil
    ref = coarse.coarse_apply(Y, v, cd)
    assert np.abs(eo.apply_full(v) - ref).max() < 1e-13 * np.abs(ref).max()


def test_odd_coarse_extent_rejected():
    Y, cd = galerkin((6, 4, 4, 4), (2, 2, 2, 2), 2)  # coarse 3 x 2 x 2 x 2
    with pytest.raises(ValueError):
        ceo.CoarseEvenOdd(Y, cd)


@pytest.mark.parametrize("dims,block,k", CASES)
def test_schur_equals_dense_and_determinant_factorises(dims, block, k):
    Y, cd = galerkin(dims, block, k)
    eo = ceo.CoarseEvenOdd(Y, cd)
    d, m = Y.shape[0], Y.shape[2]
    Dc = coarse.dense_coarse(Y, cd)
    S = ceo.dense_schur(Dc, eo.par, m)
    e = eo.par == 0
    v = fields.gaussian_coarse(d * m, 1, 43).reshape(1, d, m)
    v_e = ceo.restrict_parity(v, eo.par, 0)
    got = eo.schur(v_e)
    assert np.abs(got[:, ~e]).max() == 0.0
    ref = S @ v_e[0][e].ravel()
    assert np.abs(got[0][e].ravel() - ref).max() < 1e-12 * np.abs(ref).max()
    # det D_c = det Y_oo det Dhat_c
    o = np.repeat(eo.par == 1, m)
    s1, l1 = np.linalg.slogdet(Dc)
    s2, l2 = np.linalg.slogdet(Dc[np.ix_(o, o)])
    s3, l3 = np.linalg.slogdet(S)
    assert abs(l1 - (l2 + l3)) < 1e-9 and abs(s1 - s2 * s3) < 1e-9
    # sigma3 (diag(1, -1) over the two chirality halves of each aggregate) carries through
    s3m = np.kron(np.eye(int(e.sum())), np.kron(np.diag([1.0, -1.0]), np.eye(m // 2)))
    assert np.abs(s3m @ S @ s3m - np.conj(S.T)).max() < 1e-12 * np.abs(S).max()


@pytest.mark.parametrize("dims,block,k", CASES)
def test_schur_solve_equals_dense_lu(dims, block, k):
    Y, cd = galerkin(dims, block, k)
    eo = ceo.CoarseEvenOdd(Y, cd)
    d, m = Y.shape[0], Y.shape[2]
    r = fields.gaussian_coarse(d * m, 2, 44).reshape(2, d, m)
    v, it = eo.solve(r, tol=1e-13)
    ref = np.linalg.solve(coarse.dense_coarse(Y, cd), r.reshape(2, -1).T).T.reshape(r.shape)
    assert np.abs(v - ref).max() < 1e-10 * np.abs(ref).max()
    # the Schur system is no larger than the full one in GMRES steps
    _, it_full, _ = krylov.gmres(
        lambda x: coarse.coarse_apply(Y, x, cd), r, None, restart=32, max_iter=5000, tol=1e-13)
    assert it <= it_full


def test_no_hops_reduces_to_block_inverse():
    Y, cd = galerkin((4, 4, 4, 8), (2, 2, 2, 2), 2)
    Y = Y.copy()
    Y[:, 1:] = 0
    eo = ceo.CoarseEvenOdd(Y, cd)
    d, m = Y.shape[0], Y.shape[2]
    r = fields.gaussian_coarse(d * m, 1, 45).reshape(1, d, m)
    assert np.array_equal(eo.prepare(r), ceo.restrict_parity(r, eo.par, 0))
    v, _ = eo.solve(r, tol=1e-14)
    ref = np.stack([np.linalg.solve(Y[j, 0], r[0, j]) for j in range(d)])[None]
    assert np.abs(v - ref).max() < 1e-11 * np.abs(ref).max()
