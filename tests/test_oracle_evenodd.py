"""Pins of the even-odd oracle (oracle/evenodd.py): the hops join opposite parities, the Schur
complement equals the one cut from the dense matrix, the determinant factorises, the
preconditioned solve equals dense LU, and the adjoint and Wilson special cases."""
import numpy as np
import pytest

import fields
from oracle import clover, evenodd, wilson, geometry as geo
from oracle.gamma import GAMMA5


def _setup(dims, clov, seed=31):
    U = fields.random_gauge(dims, 0.5, seed)
    T = clover.clover_term(U, dims, 1.1, 0.9) if clov else None
    return U, T


def test_hops_join_opposite_parities():
    dims = (4, 2, 2, 4)
    U, _ = _setup(dims, False)
    par = evenodd.parity(dims)
    nb = geo.neighbor_table(dims)
    assert np.all(par[nb] != par[:, None])
    psi = fields.gaussian_spinor(dims, 1, 32)
    for p in (0, 1):
        h = evenodd.hop(U, evenodd.restrict_parity(psi, par, p), 0.1, 1.5, -1, dims)
        assert np.abs(h[:, par == p]).max() == 0.0
    with pytest.raises(ValueError):
        evenodd.EvenOdd(fields.random_gauge((4, 2, 3, 4), 0.5, 1), (4, 2, 3, 4), 0.1)


@pytest.mark.parametrize("clov", [False, True])
def test_schur_complement_equals_the_dense_one(clov):
    dims = (2, 2, 2, 4)
    U, T = _setup(dims, clov)
    mass, xi, bc = -0.1, 2.0, -1
    eo = evenodd.EvenOdd(U, dims, mass, xi, bc, T)
    D = clover.dense_clover(U, T, mass, xi, bc, dims) if clov else wilson.dense_wilson(U, mass, xi, bc, dims)
    S = evenodd.dense_schur(D, eo.par)
    e = eo.par == 0
    x = fields.gaussian_spinor(dims, 1, 33)
    x_e = evenodd.restrict_parity(x, eo.par, 0)
    for dag, M in ((False, S), (True, np.conj(S.T))):
        got = eo.schur(x_e, dagger=dag)
        assert np.abs(got[:, ~e]).max() == 0.0
        ref = M @ x_e[0][e].ravel()
        assert np.abs(got[0][e].ravel() - ref).max() < 1e-13 * np.abs(ref).max()
    # Dhat is gamma5-hermitian
    g5 = np.kron(np.eye(int(e.sum())), np.kron(GAMMA5, np.eye(3)))
    assert np.abs(g5 @ S @ g5 - np.conj(S.T)).max() < 1e-13
    # det D = det A_oo det Dhat
    o = np.repeat(eo.par == 1, 12)
    s1, l1 = np.linalg.slogdet(D)
    s2, l2 = np.linalg.slogdet(D[np.ix_(o, o)])
    s3, l3 = np.linalg.slogdet(S)
    assert abs(l1 - (l2 + l3)) < 1e-9 and abs(s1 - s2 * s3) < 1e-9


def test_wilson_schur_closed_form():
    """Without the clover term A = a 1 (a = m + 1 + 3/xi): Dhat = a - H_eo H_oe / a."""
    dims = (4, 2, 2, 2)
    U, _ = _setup(dims, False)
    mass, xi, bc = 0.07, 1.3, -1
    a = wilson.diag_term(mass, xi)
    eo = evenodd.EvenOdd(U, dims, mass, xi, bc)
    x_e = evenodd.restrict_parity(fields.gaussian_spinor(dims, 2, 34), eo.par, 0)
    h = evenodd.hop(U, evenodd.hop(U, x_e, mass, xi, bc, dims), mass, xi, bc, dims)
    ref = a * x_e - evenodd.restrict_parity(h, eo.par, 0) / a
    assert np.abs(eo.schur(x_e) - ref).max() < 1e-13


@pytest.mark.parametrize("clov", [False, True])
def test_even_odd_solve_equals_dense_lu(clov):
    dims = (4, 2, 2, 4)
    U, T = _setup(dims, clov, seed=35)
    mass, xi, bc = 0.05, 1.0, -1
    eo = evenodd.EvenOdd(U, dims, mass, xi, bc, T)
    D = clover.dense_clover(U, T, mass, xi, bc, dims) if clov else wilson.dense_wilson(U, mass, xi, bc, dims)
    b = fields.gaussian_spinor(dims, 1, 36)
    for dag, M in ((False, D), (True, np.conj(D.T))):
        x, it = eo.solve(b, tol=1e-13, dagger=dag)
        xd = np.linalg.solve(M, b.ravel())
        assert np.linalg.norm(x.ravel() - xd) < 1e-10 * np.linalg.norm(xd)
        assert it > 0
