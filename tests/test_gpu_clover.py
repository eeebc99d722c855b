"""GPU parity of the Wilson-clover operator (qmg_clover_field, qmg_clover_apply in every launch
form) and of the multigrid built on it, against oracle/clover.py."""
import numpy as np
import pytest
import torch

import fields
from oracle import clover, coarse, mg as omg
from tests._util import to_gpu, to_np, rel, projector_dist, banner

pytestmark = pytest.mark.gpu


def unpack(A):
    """Packed site term (qmg.h layout, [2,18,V] complex or [2,18,V,2] real pairs) -> [V,2,6,6]
    (decoding only)."""
    A = np.asarray(A)
    if A.ndim == 4:
        A = A[..., 0].astype(np.float64) + 1j * A[..., 1].astype(np.float64)
    V = A.shape[2]
    out = np.zeros((V, 2, 6, 6), dtype=np.complex128)
    for al in range(2):
        for e in range(3):
            out[:, al, 2 * e, 2 * e] = A[al, e].real
            out[:, al, 2 * e + 1, 2 * e + 1] = A[al, e].imag
        e = 3
        for i in range(6):
            for j in range(i + 1, 6):
                out[:, al, i, j] = A[al, e]
                out[:, al, j, i] = np.conj(A[al, e])
                e += 1
    return out


def _case(dims, seed, eps=0.7):
    U = fields.random_gauge(dims, eps, seed)
    return U


@pytest.mark.parametrize("dims", [(6, 4, 5, 8), (1, 1, 1, 4), (2, 2, 2, 2)])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-7), ("bf16", 1e-2)])
def test_clover_field_matches_oracle(qmg, dims, prec, tol):
    """960 sites (three full 256-site tiles and a ragged one), and extents 1 and 2 where leaves
    reach the site itself or wrap onto each other."""
    banner(f"clover field {dims} {prec}")
    U = _case(dims, 61)
    m, xi, cs, ct = -0.2, 2.0, 1.3, 0.9
    lat = qmg.Lattice(dims, m, xi, -1)
    A = qmg.clover_field(lat, to_gpu(U), cs, ct, prec)
    got = unpack(to_np(A.float() if prec == "bf16" else A))
    T = clover.clover_term(U, dims, cs, ct)
    ref = clover.chiral_blocks(clover.site_term(T, m, xi))
    assert rel(got, ref) < tol
    # the off-chirality blocks the packed form drops are zero in the oracle
    assert clover.gamma5_commutes(T) < 1e-14


DIMS = [(6, 4, 5, 8), (4, 4, 4, 4), (5, 3, 2, 7)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-6)])
def test_clover_apply_native_forms(qmg, dims, prec, tol):
    """Site, direction-split and t-walking forms (and the launcher's own choice), D_sw and
    D_sw^dagger, against the oracle's stencil plus T(x)."""
    nrhs = 2
    U = _case(dims, 62)
    psi = fields.gaussian_spinor(dims, nrhs, 63)
    m, xi, cs, ct = -0.3, 3.5, 1.1, 0.8
    lat = qmg.Lattice(dims, m, xi, -1)
    T = clover.clover_term(U, dims, cs, ct)
    A = qmg.clover_field(lat, to_gpu(U), cs, ct, prec)
    Un = qmg.pack_gauge(lat, to_gpu(U), prec)
    pn = qmg.pack_spinor(lat, to_gpu(psi), prec)
    try:
        for v in (0, 1, 16, 2, 4, 8):
            if v in (2, 4, 8) and dims[3] % v:
                continue
            qmg.set_dslash_variant(v)
            for dag in (False, True):
                banner(f"clover apply {dims} {prec} variant={v} dag={dag}")
                out = qmg.clover_apply(lat, Un, A, pn, layout="native", dagger=dag)
                got = to_np(qmg.unpack_spinor(lat, out, prec))
                ref = clover.apply_clover(U, T, psi, m, xi, -1, dims, dagger=dag)
                assert rel(got, ref) < tol
    finally:
        qmg.set_dslash_variant(0)


@pytest.mark.parametrize("dag", [False, True])
def test_clover_apply_canonical_and_half_storage(qmg, dag):
    dims = (6, 4, 5, 8)
    banner(f"clover apply canonical f64/f32, bf16/f16 native dag={dag}")
    U = _case(dims, 64)
    psi = fields.gaussian_spinor(dims, 3, 65)
    m, xi, cs, ct = 0.05, 1.0, 1.0, 1.0
    lat = qmg.Lattice(dims, m, xi, -1)
    T = clover.clover_term(U, dims, cs, ct)
    ref = clover.apply_clover(U, T, psi, m, xi, -1, dims, dagger=dag)
    for prec, dt, tol in (("f64", np.complex128, 1e-14), ("f32", np.complex64, 1e-6)):
        A = qmg.clover_field(lat, to_gpu(U), cs, ct, prec)
        got = to_np(qmg.clover_apply(lat, to_gpu(U.astype(dt)), A, to_gpu(psi.astype(dt)), dagger=dag))
        assert rel(got, ref) < tol
    for prec, tol in (("bf16", 1e-2), ("f16", 2e-3)):
        A = qmg.clover_field(lat, to_gpu(U), cs, ct, prec)
        Un = qmg.pack_gauge(lat, to_gpu(U), prec)
        pn = qmg.pack_spinor(lat, to_gpu(psi), prec)
        got = to_np(qmg.unpack_spinor(lat, qmg.clover_apply(lat, Un, A, pn, layout="native", dagger=dag), prec))
        assert rel(got, ref) < tol


@pytest.mark.parametrize("variant", [202, 304, 1202, 1304])
def test_clover_multi_rhs_twalk(qmg, variant):
    """t-walking with 2 or 3 right-hand sides per thread (FP32), both tile orders."""
    for dims in ((16, 16, 4, 8), (12, 10, 6, 8)):
        nrhs = 6
        banner(f"clover multi-rhs t-walk {variant} {dims}")
        U = _case(dims, 66, eps=0.6)
        psi = fields.gaussian_spinor(dims, nrhs, 67)
        m, xi, cs, ct = -0.3, 2.0, 1.2, 0.9
        lat = qmg.Lattice(dims, m, xi, -1)
        T = clover.clover_term(U, dims, cs, ct)
        A = qmg.clover_field(lat, to_gpu(U), cs, ct, "f32")
        Un = qmg.pack_gauge(lat, to_gpu(U), "f32")
        pn = qmg.pack_spinor(lat, to_gpu(psi), "f32")
        try:
            qmg.set_dslash_variant(variant)
            for dag in (False, True):
                got = to_np(qmg.unpack_spinor(lat, qmg.clover_apply(lat, Un, A, pn, layout="native", dagger=dag),
                                              "f32"))
                ref = clover.apply_clover(U, T, psi, m, xi, -1, dims, dagger=dag)
                assert rel(got, ref) < 1e-6
        finally:
            qmg.set_dslash_variant(0)


def test_clover_setup_and_galerkin_match_oracle(qmg):
    """Given test vectors: without smoothing P does not depend on D, so Y checks the Galerkin
    product with the site term in Y_0; with four smoothing iterations on D_sw the streamed
    basis and singular values match the oracle's setup on the same operator."""
    dims, block, k, r, ns = (8, 4, 4, 8), (4, 4, 4, 4), 12, 4, 3
    U = _case(dims, 68, eps=0.5)
    phi = fields.gaussian_test_vectors(dims, ns * r, 69)
    m, xi, cs, ct = -0.1, 2.0, 1.25, 0.85
    lat = qmg.Lattice(dims, m, xi, -1)
    T = clover.clover_term(U, dims, cs, ct)
    banner("clover Galerkin, no smoothing")
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, ns * r, r, k, n_setup_iter=0, inner="f64",
                                        test_vectors=to_gpu(phi), c_sw=(cs, ct))
    P = to_np(mg.prolongator()[0])
    Y = to_np(mg.coarse_blocks())
    Yo = coarse.build_coarse(U, P, m, xi, -1, dims, block, T=T)
    assert rel(Y, Yo) < 1e-13
    Yw = coarse.build_coarse(U, P, m, xi, -1, dims, block)
    assert rel(Y, Yw) > 1e-3  # the clover term is there
    mg.close()
    banner("clover setup with smoothing")
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, ns * r, r, k, n_setup_iter=4, inner="f64",
                                        test_vectors=to_gpu(phi), c_sw=(cs, ct))
    olat = omg.Lattice(U, dims, m, xi, -1, T=T)
    oh = omg.setup(olat, block, ns * r, r, k, n_setup_iter=4, test_vectors=phi)
    P, sig = mg.prolongator()
    P = to_np(P)
    assert np.abs(sig - oh.sigma).max() < 1e-10 * oh.sigma.max()
    worst = max(projector_dist(P[j, a], oh.P[j, a]) for j in range(P.shape[0]) for a in range(2))
    assert worst < 1e-9
    assert rel(to_np(mg.coarse_blocks()), coarse.build_coarse(U, P, m, xi, -1, dims, block, T=T)) < 1e-13
    mg.close()


@pytest.mark.parametrize("inner", ["f32", "f64"])
def test_clover_solve_and_checkpoint(qmg, tmp_path, inner):
    """The clover MG solve reaches 1e-10 in the oracle's D_sw residual (and for D_sw^dagger); a
    saved and reloaded hierarchy keeps the coefficients and solves identically."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    banner(f"clover solve {inner}")
    U = _case(dims, 70, eps=0.4)
    m, cs, ct = 0.02, 1.0, 1.0
    lat = qmg.Lattice(dims, m, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 24, 8, 12, n_setup_iter=16, inner=inner, seed=5,
                                        c_sw=(cs, ct))
    T = clover.clover_term(U, dims, cs, ct)
    b = fields.gaussian_spinor(dims, 2, 71)
    x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
    print(f"[clover] solve {inner}: {info[0]}")
    assert max(i["true_rel_res"] for i in info) <= 1e-10
    r = b - clover.apply_clover(U, T, to_np(x), m, 1.0, -1, dims)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-10
    xa, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-10, adjoint=True)
    r = b - clover.apply_clover(U, T, to_np(xa), m, 1.0, -1, dims, dagger=True)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-10
    path = tmp_path / "clover.qmg"
    mg.save(path)
    loaded = qmg.mg_load(path, to_gpu(U))
    assert (loaded.params.c_sw_s, loaded.params.c_sw_t) == (cs, ct)
    x1, i1 = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
    x2, i2 = qmg.mg_solve(loaded, to_gpu(b), tol=1e-10)
    assert torch.equal(x1, x2) and i1[0]["outer_iters"] == i2[0]["outer_iters"]
    loaded.close()
    mg.close()
