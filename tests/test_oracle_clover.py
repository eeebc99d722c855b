"""Pins of the clover oracle (oracle/clover.py) against facts that do not come from the oracle:
the free field, closed forms for abelian backgrounds, plaquettes walked link by link, gauge
covariance, hermiticity and gamma_5 structure, the dense operator, the Galerkin product and the
unique solution of the clover multigrid solve."""
import numpy as np
import pytest

import fields
from oracle import clover, coarse, geometry as geo, icsvd as ic, mg as omg, transfer, wilson
from oracle.gamma import GAMMA5


def _abelian(dims, mu, nu, phases):
    """U_mu(x) = diag(exp(i q_c a(x_nu))) with q = (1, -1, 0), every other link 1: a U(1)
    field in the (mu, nu) plane embedded in SU(3).  phases: a[L_nu]."""
    V = geo.volume(dims)
    X = geo.coords(dims)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[:] = np.eye(3)
    q = np.array([1.0, -1.0, 0.0])
    ph = np.asarray(phases)[X[:, nu]]
    U[mu] = np.einsum("xc,cd->xcd", np.exp(1j * ph[:, None] * q[None, :]), np.eye(3))
    return U, X, q


def test_free_field_has_no_clover_term():
    dims = (2, 4, 2, 4)
    U = np.zeros((4, geo.volume(dims), 3, 3), dtype=np.complex128)
    U[:] = np.eye(3)
    assert np.abs(clover.clover_term(U, dims, 1.3, 0.7)).max() == 0.0


@pytest.mark.parametrize("mu,nu,c_s,c_t", [(0, 1, 1.7, 0.0), (2, 3, 0.0, 1.3)])
def test_abelian_background_closed_form(mu, nu, c_s, c_t):
    """One plane carries the field: the plaquettes at x - nu and x share the phase
    delta(x_nu) = q (a(x_nu) - a(x_nu + 1)), so Fhat = (i/2)(sin delta(x_nu) + sin delta(x_nu - 1))
    per colour, and T = -(c/4) (sin + sin) sigma_{mu nu} with sigma_xy = -diag(1,-1,1,-1) and
    sigma_zt = diag(1,-1,-1,1) in the chiral basis (worked out by hand from the gamma matrices).
    Each plane's coefficient is the other's zero, so a wrong c_s/c_t assignment fails."""
    dims = (4, 3, 4, 5)
    rng = np.random.default_rng(11)
    L = dims[nu]
    a = rng.uniform(-np.pi, np.pi, size=L)
    U, X, q = _abelian(dims, mu, nu, a)
    T = clover.clover_term(U, dims, c_s, c_t)
    c = c_t if nu == 3 else c_s
    eps = {(0, 1): np.array([-1, 1, -1, 1]), (2, 3): np.array([1, -1, -1, 1])}[(mu, nu)]
    y = X[:, nu]
    delta = lambda yy: np.outer(a[yy % L] - a[(yy + 1) % L], q)  # [V][colour]
    s = np.sin(delta(y)) + np.sin(delta(y - 1))
    expect = np.zeros_like(T)
    for sp in range(4):
        for col in range(3):
            expect[:, 3 * sp + col, 3 * sp + col] = -(c / 4.0) * eps[sp] * s[:, col]
    assert np.abs(T - expect).max() < 1e-14
    assert np.abs(T).max() > 0.05


def _walk(U, dims, x, steps):
    """Ordered product of links along a path of +/-(mu + 1) steps starting at coordinate x."""
    c = np.array(x)
    M = np.eye(3, dtype=np.complex128)
    for s in steps:
        mu = abs(s) - 1
        if s > 0:
            M = M @ U[mu, geo.lex(c, dims)]
            c[mu] = (c[mu] + 1) % dims[mu]
        else:
            c[mu] = (c[mu] - 1) % dims[mu]
            M = M @ np.conj(U[mu, geo.lex(c, dims)]).T
    assert np.array_equal(c, np.array(x))  # closed
    return M


def test_leaves_equal_walked_plaquettes():
    """Non-abelian field: the four leaves are the closed walks (+mu,+nu,-mu,-nu), (+nu,-mu,-nu,+mu),
    (-mu,-nu,+mu,+nu), (-nu,+mu,+nu,-mu) from x, multiplied link by link."""
    dims = (3, 4, 2, 5)
    U = fields.random_gauge(dims, 0.8, 12)
    X = geo.coords(dims)
    rng = np.random.default_rng(12)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Q = clover.leaves(U, dims, mu, nu)
            m, n = mu + 1, nu + 1
            for site in rng.choice(len(X), 6, replace=False):
                x = X[site]
                ref = sum(_walk(U, dims, x, p) for p in ([m, n, -m, -n], [n, -m, -n, m],
                                                         [-m, -n, m, n], [-n, m, n, -m]))
                assert np.abs(Q[site] - ref).max() < 1e-13


def test_clover_term_is_gauge_covariant_hermitian_and_chiral():
    """U_mu(x) -> G(x) U_mu(x) G(x+mu)^dag takes T(x) to (1 x G(x)) T(x) (1 x G(x))^dag; T(x) is
    hermitian and commutes with gamma_5 (two 6 x 6 chirality blocks)."""
    dims = (4, 2, 3, 4)
    V = geo.volume(dims)
    U = fields.random_gauge(dims, 0.7, 13)
    G = fields.random_su3(V, 14)
    nb = geo.neighbor_table(dims)
    Ug = np.einsum("xab,mxbc,mxdc->mxad", G, U, np.conj(G[nb[:, :4].T]))
    T = clover.clover_term(U, dims, 1.1, 0.9)
    Tg = clover.clover_term(Ug, dims, 1.1, 0.9)
    big = np.einsum("st,xab->xsatb", np.eye(4), G).reshape(V, 12, 12)
    assert np.abs(Tg - big @ T @ np.conj(np.swapaxes(big, 1, 2))).max() < 1e-13
    assert np.abs(T - np.conj(np.swapaxes(T, 1, 2))).max() < 1e-14
    g5 = np.kron(GAMMA5, np.eye(3))
    assert np.abs(T @ g5 - g5 @ T).max() < 1e-14
    assert np.abs(T[:, :6, 6:]).max() == 0.0 and np.abs(T).max() > 0.1


def test_operator_is_gamma5_hermitian_and_applies_the_dense_matrix():
    dims = (2, 2, 2, 4)
    U = fields.random_gauge(dims, 0.6, 15)
    T = clover.clover_term(U, dims, 1.2, 0.8)
    mass, xi, bc = -0.2, 2.0, -1
    D = clover.dense_clover(U, T, mass, xi, bc, dims)
    g5 = np.kron(np.eye(geo.volume(dims)), np.kron(GAMMA5, np.eye(3)))
    assert np.abs(g5 @ D @ g5 - np.conj(D.T)).max() < 1e-14
    psi = fields.gaussian_spinor(dims, 2, 16)
    for dag, M in ((False, D), (True, np.conj(D.T))):
        got = clover.apply_clover(U, T, psi, mass, xi, bc, dims, dagger=dag)
        ref = (M @ psi.reshape(2, -1).T).T.reshape(psi.shape)
        assert np.abs(got - ref).max() < 1e-13
    # c = 0 is the Wilson operator
    T0 = clover.clover_term(U, dims, 0.0, 0.0)
    assert np.abs(clover.dense_clover(U, T0, mass, xi, bc, dims) - wilson.dense_wilson(U, mass, xi, bc, dims)).max() == 0


def test_galerkin_with_clover_equals_dense_product():
    dims, block, k = (4, 2, 2, 4), (2, 2, 2, 2), 3
    psi = fields.gaussian_spinor(dims, k + 2, 17)
    P, _ = ic.csvd(psi, dims, block, k)
    G = fields.random_gauge(dims, 0.5, 18)
    T = clover.clover_term(G, dims, 1.4, 0.9)
    mass, xi, bc = 0.05, 1.5, -1
    Y = coarse.build_coarse(G, P, mass, xi, bc, dims, block, T=T)
    Pd = transfer.dense_prolongator(P, dims, block)
    ref = np.conj(Pd.T) @ clover.dense_clover(G, T, mass, xi, bc, dims) @ Pd
    Dc = coarse.dense_coarse(Y, geo.coarse_dims(dims, block))
    assert np.abs(Dc - ref).max() < 1e-13 * np.abs(ref).max()
    # the clover term only changes Y_0
    Yw = coarse.build_coarse(G, P, mass, xi, bc, dims, block)
    assert np.abs(Y[:, 1:] - Yw[:, 1:]).max() == 0 and np.abs(Y[:, 0] - Yw[:, 0]).max() > 1e-3


def test_clover_multigrid_solve_matches_the_dense_solution():
    dims = (4, 4, 4, 4)
    U = fields.random_gauge(dims, 0.3, 19)
    T = clover.clover_term(U, dims, 1.0, 1.0)
    lat = omg.Lattice(U, dims, 0.05, 1.0, -1, T=T)
    h = omg.setup(lat, (2, 2, 2, 2), 12, 4, 6, n_setup_iter=8, seed=6)
    b = fields.gaussian_spinor(dims, 1, 20)[0]
    x, st = omg.solve(h, b, tol=1e-12)
    assert st["true_rel_res"] < 1e-12
    xd = np.linalg.solve(clover.dense_clover(U, T, 0.05, 1.0, -1, dims), b.ravel())
    assert np.linalg.norm(x.ravel() - xd) < 1e-9 * np.linalg.norm(xd)
