"""Pins of oracle.transfer and oracle.coarse: P/R identities and brute-force Galerkin products."""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import fields
from oracle import icsvd as ic, transfer, coarse, wilson, geometry as geo


def hierarchy(dims, block, k, seed=1, eps=0.4, nvec=None):
    psi = fields.gaussian_spinor(dims, nvec or k + 2, seed)
    U, _ = ic.csvd(psi, dims, block, k)
    G = fields.random_gauge(dims, eps, seed)
    return U, G


def test_R_is_left_inverse_and_P_isometry():
    dims, block, k = (4, 4, 2, 4), (2, 2, 2, 2), 5
    U, _ = hierarchy(dims, block, k)
    d = U.shape[0]
    vc = fields.gaussian_coarse(d * 2 * k, 2, 3).reshape(2, d, 2, k)
    f = transfer.prolong(U, vc, dims, block)
    assert np.abs(transfer.restrict(U, f, dims, block) - vc).max() < 1e-13
    assert abs(np.linalg.norm(f) - np.linalg.norm(vc)) < 1e-12 * np.linalg.norm(vc)
    psi = fields.gaussian_spinor(dims, 1, 4)
    pr = transfer.prolong(U, transfer.restrict(U, psi, dims, block), dims, block)
    pr2 = transfer.prolong(U, transfer.restrict(U, pr, dims, block), dims, block)
    assert np.abs(pr - pr2).max() < 1e-13                        # PR is a projector
    assert abs(np.vdot((psi - pr).ravel(), pr.ravel())) < 1e-12  # ... an orthogonal one


def test_dense_prolongator_matches_stencil_form():
    dims, block, k = (2, 2, 2, 4), (2, 1, 2, 2), 3
    U, _ = hierarchy(dims, block, k)
    P = transfer.dense_prolongator(U, dims, block)
    d = U.shape[0]
    vc = fields.gaussian_coarse(d * 2 * k, 1, 5).reshape(1, d, 2, k)
    assert np.abs(P @ vc.ravel() - transfer.prolong(U, vc, dims, block).ravel()).max() < 1e-13
    psi = fields.gaussian_spinor(dims, 1, 6)
    assert np.abs(np.conj(P.T) @ psi.ravel() - transfer.restrict(U, psi, dims, block).ravel()).max() < 1e-13


@pytest.mark.parametrize("dims,block,k", [((4, 4, 4, 4), (2, 2, 2, 2), 4),    # coarse extent 2
                                          ((6, 2, 4, 4), (2, 2, 2, 2), 3),    # coarse extents 3 and 1
                                          ((2, 2, 2, 4), (1, 2, 1, 2), 2)])
def test_galerkin_equals_brute_force(dims, block, k):
    U, G = hierarchy(dims, block, k, seed=2)
    mass, xi, bc = 0.07, 2.5, -1
    Y = coarse.build_coarse(G, U, mass, xi, bc, dims, block)
    cd = geo.coarse_dims(dims, block)
    Dc = coarse.dense_coarse(Y, cd)
    P = transfer.dense_prolongator(U, dims, block)
    Dm = wilson.dense_wilson(G, mass, xi, bc, dims)
    ref = np.conj(P.T) @ Dm @ P
    assert np.abs(Dc - ref).max() < 1e-13 * np.abs(ref).max()
    d = Y.shape[0]
    v = fields.gaussian_coarse(d * 2 * k, 2, 7).reshape(2, d, 2, k)
    Dv = coarse.coarse_apply(Y, v, cd)
    pdp = transfer.restrict(U, wilson.apply_wilson(G, transfer.prolong(U, v, dims, block), mass, xi, bc, dims),
                            dims, block)
    assert np.abs(Dv - pdp).max() < 1e-12 * np.abs(pdp).max()
    # sigma3-hermiticity of the coarse operator
    s3 = np.kron(np.eye(d), np.kron(np.diag([1.0, -1.0]), np.eye(k)))
    assert np.abs(s3 @ Dc @ s3 - np.conj(Dc.T)).max() < 1e-13 * np.abs(Dc).max()


def test_unit_blocks_full_rank_preserve_spectrum():
    """Blocks 1^4 with k = 6: P is unitary per site, D_c is unitarily similar to D."""
    dims, block, k = (2, 2, 2, 4), (1, 1, 1, 1), 6
    U, G = hierarchy(dims, block, k, seed=3, nvec=8)
    Y = coarse.build_coarse(G, U, 0.1, 1.0, -1, dims, block)
    ev_c = np.linalg.eigvals(coarse.dense_coarse(Y, dims))
    ev = np.linalg.eigvals(wilson.dense_wilson(G, 0.1, 1.0, -1, dims))
    C = np.abs(ev_c[:, None] - ev[None, :])
    r, c = linear_sum_assignment(C)
    assert C[r, c].max() < 1e-11
