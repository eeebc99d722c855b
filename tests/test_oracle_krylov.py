"""Pins of oracle.krylov: GMRES optimality against a dense least-squares problem."""
import numpy as np

import fields
from oracle import krylov, wilson, mg


def _setup(seed=3):
    dims = (2, 2, 2, 4)
    U = fields.random_gauge(dims, 0.5, seed)
    Dm = wilson.dense_wilson(U, 0.05, 1.0, -1, dims)
    return dims, U, Dm


def test_gmres_minimises_over_krylov_space():
    dims, U, Dm = _setup()
    rng = np.random.default_rng(0)
    b = rng.standard_normal(Dm.shape[0]) + 1j * rng.standard_normal(Dm.shape[0])
    x0 = rng.standard_normal(Dm.shape[0]) + 1j * rng.standard_normal(Dm.shape[0])
    for n in (1, 3, 8):
        x, it, _ = krylov.gmres(lambda v: Dm @ v, b, x0, restart=8, max_iter=n)
        r0 = b - Dm @ x0
        K = np.stack([np.linalg.matrix_power(Dm, i) @ r0 for i in range(n)], axis=1)
        c, *_ = np.linalg.lstsq(Dm @ K, r0, rcond=None)
        xbest = x0 + K @ c
        assert it == n
        assert abs(np.linalg.norm(b - Dm @ x) - np.linalg.norm(b - Dm @ xbest)) < 1e-10 * np.linalg.norm(b)
        assert np.linalg.norm(x - xbest) < 1e-8 * np.linalg.norm(xbest)


def test_gmres_restarted_residual_monotone():
    dims, U, Dm = _setup(4)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(Dm.shape[0]) + 1j * rng.standard_normal(Dm.shape[0])
    _, _, hist = krylov.gmres(lambda v: Dm @ v, b, None, restart=8, max_iter=40)
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))
    x, it, _ = krylov.gmres(lambda v: Dm @ v, b, None, restart=20, max_iter=2000, tol=1e-12)
    assert np.linalg.norm(b - Dm @ x) <= 1.01e-12 * np.linalg.norm(b)


def test_smoother_is_polynomial_with_unit_constant_term():
    """psi = q(D) phi with q(0) = 1: after n GMRES steps on D psi' = -D phi, psi - phi lies in
    span{D phi, ..., D^n phi} and ||D psi|| is minimal over that affine space."""
    dims, U, Dm = _setup(5)
    lat = mg.Lattice(U, dims, 0.05, 1.0, -1)
    rng = np.random.default_rng(2)
    phi = (rng.standard_normal((32, 4, 3)) + 1j * rng.standard_normal((32, 4, 3)))
    n = 5
    rhs = -lat.D(phi)
    dpsi, _, _ = krylov.gmres(lat.D, rhs, None, restart=8, max_iter=n)
    K = np.stack([np.linalg.matrix_power(Dm, i + 1) @ phi.ravel() for i in range(n)], axis=1)
    c, *_ = np.linalg.lstsq(Dm @ K, -(Dm @ phi.ravel()), rcond=None)
    assert np.linalg.norm(dpsi.ravel() - K @ c) < 1e-8 * np.linalg.norm(K @ c)
    psi = mg.smooth(lat, phi, n)
    assert abs(np.linalg.norm(psi) - 1) < 1e-14


def test_fgcr_with_exact_preconditioner_one_step():
    dims, U, Dm = _setup(6)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(Dm.shape[0]) + 1j * rng.standard_normal(Dm.shape[0])
    Dinv = np.linalg.inv(Dm)
    x, it, hist = krylov.fgcr(lambda v: Dm @ v, lambda r: Dinv @ r, b, tol=1e-12)
    assert it == 1 and hist[-1] < 1e-12
