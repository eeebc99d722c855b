"""Pins of oracle.wilson against closed forms and symmetries of the Wilson-Dirac operator."""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import fields
from oracle import wilson, geometry as geo
from oracle.gamma import GAMMA, GAMMA5


def unit_links(dims):
    U = np.zeros((4, geo.volume(dims), 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    return U


def match(a, b):
    C = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(C)
    return C[r, c].max()


@pytest.mark.parametrize("xi,bc_t", [(1.0, -1), (3.5, -1), (2.0, 1)])
def test_free_field_spectrum_closed_form(xi, bc_t):
    dims = (2, 2, 2, 4)
    Dm = wilson.dense_wilson(unit_links(dims), 0.1, xi, bc_t, dims)
    ev = np.linalg.eigvals(Dm)
    assert match(ev, wilson.free_field_eigenvalues(0.1, xi, bc_t, dims)) < 1e-12


def test_plane_wave_4x4():
    """D e^{ipx} u = D(p) e^{ipx} u at U = 1, antiperiodic t, on 4^4."""
    dims = (4, 4, 4, 4)
    xi, m = 1.7, -0.2
    c = geo.coords(dims)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    cw = wilson.hop_weights(xi)
    for n in [(0, 0, 0, 0), (1, 2, 3, 1), (3, 0, 1, 2)]:
        p = [2 * np.pi * n[mu] / dims[mu] for mu in range(3)] + [(2 * np.pi * n[3] + np.pi) / dims[3]]
        phase = np.exp(1j * (c @ np.array(p)))
        psi = phase[:, None, None] * u[None]
        Dp = (m + sum(cw[mu] * (1 - np.cos(p[mu])) for mu in range(4))) * np.eye(4) \
            + 1j * sum(cw[mu] * np.sin(p[mu]) * GAMMA[mu] for mu in range(4))
        expect = phase[:, None, None] * (Dp @ u)[None]
        got = wilson.apply_wilson(unit_links(dims), psi, m, xi, -1, dims)
        assert np.abs(got - expect).max() < 1e-13


def test_gamma5_hermiticity():
    dims = (4, 4, 2, 4)
    U = fields.random_gauge(dims, 0.6, 7)
    psi = fields.gaussian_spinor(dims, 2, 7)
    phi = fields.gaussian_spinor(dims, 2, 8)
    a = wilson.apply_wilson(U, psi, 0.05, 3.5, -1, dims, dagger=True)
    b = wilson.gamma5(wilson.apply_wilson(U, wilson.gamma5(psi), 0.05, 3.5, -1, dims))
    assert np.abs(a - b).max() < 1e-13
    lhs = np.vdot(phi.ravel(), wilson.apply_wilson(U, psi, 0.05, 3.5, -1, dims).ravel())
    rhs = np.vdot(wilson.apply_wilson(U, phi, 0.05, 3.5, -1, dims, dagger=True).ravel(), psi.ravel())
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    assert np.allclose(GAMMA5, np.diag([1, 1, -1, -1]))


def test_gauge_covariance():
    dims = (4, 2, 4, 4)
    V = geo.volume(dims)
    U = fields.random_gauge(dims, 0.5, 11)
    g = fields.random_su3(V, 11)
    nb = geo.neighbor_table(dims)
    Ug = np.einsum("xab,mxbc,mxdc->mxad", g, U, np.conj(g[nb[:, :4].T]))
    psi = fields.gaussian_spinor(dims, 1, 12)[0]
    gpsi = np.einsum("xab,xsb->xsa", g, psi)
    lhs = wilson.apply_wilson(Ug, gpsi, 0.1, 1.3, -1, dims)
    rhs = np.einsum("xab,xsb->xsa", g, wilson.apply_wilson(U, psi, 0.1, 1.3, -1, dims))
    assert np.abs(lhs - rhs).max() < 1e-12
    # the gauge transform is nontrivial
    assert np.abs(Ug - U).max() > 0.1


def test_mass_shift_is_identity():
    dims = (2, 4, 2, 4)
    U = fields.random_gauge(dims, 0.4, 5)
    psi = fields.gaussian_spinor(dims, 1, 5)[0]
    d = wilson.apply_wilson(U, psi, 0.37, 2.0, -1, dims) - wilson.apply_wilson(U, psi, 0.0, 2.0, -1, dims)
    assert np.abs(d - 0.37 * psi).max() < 1e-13


def test_dense_equals_stencil():
    dims = (2, 2, 2, 4)
    U = fields.random_gauge(dims, 0.3, 1)
    psi = fields.gaussian_spinor(dims, 3, 1)
    Dm = wilson.dense_wilson(U, 0.05, 1.7, -1, dims)
    for dag in (False, True):
        out = wilson.apply_wilson(U, psi, 0.05, 1.7, -1, dims, dagger=dag)
        M = Dm.conj().T if dag else Dm
        assert np.abs(out.reshape(3, -1) - psi.reshape(3, -1) @ M.T).max() < 1e-13


def test_links_are_su3():
    U = fields.random_gauge((2, 2, 2, 2), 0.7, 2)
    I = np.einsum("mxab,mxcb->mxac", U, np.conj(U))
    assert np.abs(I - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13


@pytest.mark.parametrize("dims,xi,bc_t", [((3, 2, 3, 5), 1.0, -1), ((2, 3, 1, 4), 3.5, -1), ((3, 3, 2, 3), 2.0, 1)])
def test_sampled_sites_equal_dense_rows(dims, xi, bc_t):
    """apply_wilson_sites (the per-site hop loop that checks full-size GPU runs at sampled sites)
    against the rows of the dense matrix built entry by entry, for D and D^dagger, on odd
    extents, every site of the first and last time slice (the boundary wrap) and a random rest."""
    V = geo.volume(dims)
    U = fields.random_gauge(dims, 0.6, 17)
    psi = fields.gaussian_spinor(dims, 1, 17)[0]
    Dm = wilson.dense_wilson(U, -0.3, xi, bc_t, dims)
    c = geo.coords(dims)
    edge = np.nonzero((c[:, 3] == 0) | (c[:, 3] == dims[3] - 1))[0]
    rng = np.random.default_rng(5)
    sites = np.unique(np.concatenate([edge, rng.choice(V, size=min(V, 7), replace=False)]))
    for dag in (False, True):
        M = Dm.conj().T if dag else Dm
        want = (M @ psi.ravel()).reshape(V, 4, 3)[sites]
        got = wilson.apply_wilson_sites(U, psi, sites, -0.3, xi, bc_t, dims, dagger=dag)
        assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_sampled_sites_plane_wave():
    """At U = 1 a plane wave e^{ipx} u is mapped to D(p) e^{ipx} u (closed form), also at the
    sites whose t-hops cross the antiperiodic boundary; D^dagger gives D(p)^dagger."""
    dims = (4, 2, 2, 6)
    xi, m = 2.5, 0.15
    c = geo.coords(dims)
    rng = np.random.default_rng(9)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    cw = wilson.hop_weights(xi)
    sites = np.array([0, 5, 17, geo.volume(dims) - 1, int(geo.lex(np.array([1, 1, 0, 5]), dims))])
    for n in [(1, 0, 1, 2), (3, 1, 0, 5)]:
        p = [2 * np.pi * n[mu] / dims[mu] for mu in range(3)] + [(2 * np.pi * n[3] + np.pi) / dims[3]]
        phase = np.exp(1j * (c @ np.array(p)))
        psi = phase[:, None, None] * u[None]
        Dp = (m + sum(cw[mu] * (1 - np.cos(p[mu])) for mu in range(4))) * np.eye(4) \
            + 1j * sum(cw[mu] * np.sin(p[mu]) * GAMMA[mu] for mu in range(4))
        for dag, M in ((False, Dp), (True, Dp.conj().T)):
            want = phase[sites, None, None] * (M @ u)[None]
            got = wilson.apply_wilson_sites(unit_links(dims), psi, sites, m, xi, -1, dims, dagger=dag)
            assert np.abs(got - want).max() < 1e-13
