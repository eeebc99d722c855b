"""Pins of oracle.mg (setup + K-cycle solve) and oracle.force (gradients)."""
import numpy as np
import pytest

import fields
from fields import workloads
from oracle import mg, wilson, force, geometry as geo


@pytest.fixture(scope="module")
def small():
    w = workloads.get("wilson4x4_fp64")
    U = fields.random_gauge(w["dims"], w["eps"], w["seed"], w["tag"])
    lat = mg.Lattice(U, w["dims"], w["mass"], w["xi"], w["bc_t"])
    h = mg.setup(lat, w["block"], w["n_test"], w["batch"], w["rank"], 16, seed=w["seed"])
    return w, lat, h


def test_solve_reaches_tolerance_and_matches_dense_lu(small):
    w, lat, h = small
    b = fields.gaussian_spinor(w["dims"], 1, w["seed"], tag=w["tag"])[0]
    x, st = mg.solve(h, b, tol=1e-12)
    assert st["true_rel_res"] <= 1e-12 * 1.5
    Dm = wilson.dense_wilson(lat.U, lat.mass, lat.xi, lat.bc_t, lat.dims)
    xd = np.linalg.solve(Dm, b.ravel())
    assert np.linalg.norm(x.ravel() - xd) <= 1e-8 * np.linalg.norm(xd)
    xa, st = mg.solve(h, b, tol=1e-12, adjoint=True)
    xad = np.linalg.solve(np.conj(Dm.T), b.ravel())
    assert np.linalg.norm(xa.ravel() - xad) <= 1e-8 * np.linalg.norm(xad)


def test_exact_two_level_preconditioner_converges_in_one_step():
    dims = (2, 2, 2, 4)
    U = fields.random_gauge(dims, 0.4, 9)
    lat = mg.Lattice(U, dims, 0.1, 1.0, -1)
    h = mg.setup(lat, (1, 1, 1, 1), 8, 4, 6, 4, seed=9)
    b = fields.gaussian_spinor(dims, 1, 9)[0]
    x, st = mg.solve(h, b, tol=1e-10, coarse_tol=1e-14, coarse_restart=400, coarse_max=400)
    assert st["outer"] == 1 and st["true_rel_res"] < 1e-10


def test_setup_invariants(small):
    w, lat, h = small
    d = h.P.shape[0]
    assert h.P.shape == (d, 2, 6 * int(np.prod(w["block"])), w["rank"])
    for j in range(d):
        for a in range(2):
            assert np.abs(np.conj(h.P[j, a].T) @ h.P[j, a] - np.eye(w["rank"])).max() < 1e-13
    assert np.all(np.diff(h.sigma, axis=-1) <= 0)


def _loss(U, dims, mass, xi, bc, eta, b):
    Dm = wilson.dense_wilson(U, mass, xi, bc, dims)
    return float(np.real(np.vdot(eta.ravel(), np.linalg.solve(Dm, b.ravel()))))


def test_link_gradient_central_differences():
    dims, mass, xi, bc = (2, 2, 2, 4), 0.05, 1.5, -1
    U = fields.random_gauge(dims, 0.5, 21)
    b = fields.gaussian_spinor(dims, 1, 21)[0]
    eta = fields.gaussian_spinor(dims, 1, 21, stream=fields.ETA_STREAM)[0]
    Dm = wilson.dense_wilson(U, mass, xi, bc, dims)
    x = np.linalg.solve(Dm, b.ravel()).reshape(b.shape)
    lam = np.linalg.solve(np.conj(Dm.T), eta.ravel()).reshape(b.shape)
    # adjoint identity <eta, D^-1 b> = <D^-dag eta, b>
    assert abs(np.vdot(eta.ravel(), x.ravel()) - np.vdot(lam.ravel(), b.ravel())) < 1e-12 * np.linalg.norm(x)
    g = force.link_force(x, lam, xi, bc, dims)
    h = 1e-5
    rng = np.random.default_rng(0)
    for _ in range(6):
        mu, s, a, c = rng.integers(4), rng.integers(geo.volume(dims)), rng.integers(3), rng.integers(3)
        for unit, part in ((1.0, "re"), (1j, "im")):
            Up, Um = U.copy(), U.copy()
            Up[mu, s, a, c] += h * unit
            Um[mu, s, a, c] -= h * unit
            fd = (_loss(Up, dims, mass, xi, bc, eta, b) - _loss(Um, dims, mass, xi, bc, eta, b)) / (2 * h)
            an = g[mu, s, a, c].real if part == "re" else g[mu, s, a, c].imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an))
    # random direction
    Dl = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    fd = (_loss(U + h * Dl, dims, mass, xi, bc, eta, b) - _loss(U - h * Dl, dims, mass, xi, bc, eta, b)) / (2 * h)
    an = float(np.real(np.vdot(g.ravel(), Dl.ravel())))
    assert abs(fd - an) < 1e-6 * abs(an)
