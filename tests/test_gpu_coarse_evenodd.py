"""GPU parity of the even-odd coarse operator (qmg_mg_set_coarse_eo, qmg_coarse_schur_apply,
qmg_coarse_eo_solve and the K-cycle's coarse solve on the Schur complement) against
oracle/coarse_evenodd.py.  Stage-wise like the other coarse tests: the oracle's Galerkin
operator is built from the hierarchy's prolongator (whose agreement with the oracle's setup is
checked elsewhere) and checked against the hierarchy's own first."""
import numpy as np
import pytest
import torch

import fields
from oracle import coarse, coarse_evenodd as ceo, geometry as geo, wilson
from tests._util import to_gpu, to_np, rel, banner

pytestmark = pytest.mark.gpu

# (dims, block, k): coarse 2^4 with 2k = 24; coarse 4 x 2 x 4 x 4 with 2k = 16; coarse
# 2 x 2 x 2 x 4 with 2k = 10 (an odd rank per chirality)
CASES = [((8, 8, 8, 8), (4, 4, 4, 4), 12),
         ((8, 4, 8, 8), (2, 2, 2, 2), 8),
         ((4, 4, 4, 8), (2, 2, 2, 2), 5)]


def _hierarchy(qmg, dims, block, k, inner, seed=81):
    U = fields.random_gauge(dims, 0.5, seed)
    m, xi = -0.1, 2.0
    lat = qmg.Lattice(dims, m, xi, -1)
    phi = fields.gaussian_test_vectors(dims, 2 * k, seed + 1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 2 * k, k, k, n_setup_iter=0, inner=inner,
                                        test_vectors=to_gpu(phi))
    P = to_np(mg.prolongator()[0])
    Yo = coarse.build_coarse(U, P, m, xi, -1, dims, block)
    assert rel(to_np(mg.coarse_blocks()), Yo) < 1e-13
    return U, mg, Yo, geo.coarse_dims(dims, block)


@pytest.mark.parametrize("dims,block,k", CASES)
@pytest.mark.parametrize("inner,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_coarse_schur_apply_matches_oracle(qmg, dims, block, k, inner, tol):
    _, mg, Yo, cd = _hierarchy(qmg, dims, block, k, inner)
    mg.set_coarse_eo(True)
    eo = ceo.CoarseEvenOdd(Yo, cd)
    d = Yo.shape[0]
    e = eo.par == 0
    cdt = torch.complex128 if inner == "f64" else torch.complex64
    for nrhs in (1, 2, 5):  # one, two and four right-hand sides per workgroup, a ragged group
        banner(f"coarse schur apply {dims} k={k} {inner} nrhs={nrhs}")
        v = fields.gaussian_coarse(d * 2 * k, nrhs, 82).reshape(nrhs, d, 2 * k)
        v_e = ceo.restrict_parity(v, eo.par, 0)
        ref = eo.schur(v_e)[:, e].reshape(nrhs, d // 2, 2, k)
        got = to_np(qmg.coarse_schur_apply(mg, to_gpu(v[:, e].reshape(nrhs, d // 2, 2, k)).to(cdt)))
        assert rel(got, ref) < tol
    mg.close()


@pytest.mark.parametrize("dims,block,k", CASES)
def test_coarse_eo_solve_matches_dense_lu(qmg, dims, block, k):
    _, mg, Yo, cd = _hierarchy(qmg, dims, block, k, "f64")
    mg.set_coarse_eo(True)
    d = Yo.shape[0]
    b = fields.gaussian_coarse(d * 2 * k, 3, 83).reshape(3, d, 2, k)
    banner(f"coarse eo solve {dims} k={k}")
    x, it = qmg.coarse_eo_solve(mg, to_gpu(b), tol=1e-12)
    ref = np.linalg.solve(coarse.dense_coarse(Yo, cd), b.reshape(3, -1).T).T.reshape(b.shape)
    print(f"[coarse-eo] {dims} k={k}: {it} Schur GMRES steps")
    assert rel(to_np(x), ref) < 1e-9
    # the oracle's Schur solve takes as many steps within a few (same Krylov space, other rounding)
    _, it_o = ceo.CoarseEvenOdd(Yo, cd).solve(b.reshape(3, d, 2 * k), tol=1e-12)
    assert abs(it - it_o) <= max(3, it_o // 10)
    mg.close()


def test_coarse_eo_after_more_streams(qmg):
    """The Yhat blocks follow a rebuilt coarse operator."""
    dims, block, k = (8, 8, 8, 8), (4, 4, 4, 4), 6
    U = fields.random_gauge(dims, 0.5, 84)
    lat = qmg.Lattice(dims, -0.1, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 12, 6, k, n_setup_iter=2, inner="f64", seed=3)
    mg.set_coarse_eo(True)
    mg.stream_more(1)
    banner("coarse eo after stream_more")
    P = to_np(mg.prolongator()[0])
    Yo = coarse.build_coarse(U, P, -0.1, 1.0, -1, dims, block)
    cd = geo.coarse_dims(dims, block)
    d = Yo.shape[0]
    b = fields.gaussian_coarse(d * 2 * k, 1, 85).reshape(1, d, 2, k)
    x, _ = qmg.coarse_eo_solve(mg, to_gpu(b), tol=1e-12)
    ref = np.linalg.solve(coarse.dense_coarse(Yo, cd), b.reshape(1, -1).T).T.reshape(b.shape)
    assert rel(to_np(x), ref) < 1e-9
    mg.close()


def test_coarse_eo_off_more_streams_on(qmg):
    """on -> off -> more streams -> on: the Yhat blocks are rebuilt from the new D_c (switching
    off releases them, so nothing of the old coarse operator survives)."""
    dims, block, k = (8, 8, 8, 8), (4, 4, 4, 4), 6
    U = fields.random_gauge(dims, 0.5, 94)
    lat = qmg.Lattice(dims, -0.1, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 12, 6, k, n_setup_iter=2, inner="f32", seed=4)
    banner("coarse eo on -> off -> stream_more -> on")
    mg.set_coarse_eo(True)
    mg.set_coarse_eo(False)
    mg.stream_more(1)
    mg.set_coarse_eo(True)
    P = to_np(mg.prolongator()[0])
    Yo = coarse.build_coarse(U, P, -0.1, 1.0, -1, dims, block)
    cd = geo.coarse_dims(dims, block)
    d = Yo.shape[0]
    b = fields.gaussian_coarse(d * 2 * k, 2, 95).reshape(2, d, 2, k)
    x, _ = qmg.coarse_eo_solve(mg, to_gpu(b), tol=1e-12)
    ref = np.linalg.solve(coarse.dense_coarse(Yo, cd), b.reshape(2, -1).T).T.reshape(b.shape)
    assert rel(to_np(x), ref) < 1e-9
    # the K-cycle's inner-precision Schur blocks follow as well: the solve reaches 1e-10
    bf = fields.gaussian_spinor(dims, 1, 96)
    xf, info = qmg.mg_solve(mg, to_gpu(bf), tol=1e-10)
    r = bf - wilson.apply_wilson(U, to_np(xf), -0.1, 1.0, -1, dims)
    assert np.linalg.norm(r) / np.linalg.norm(bf) < 2e-10
    mg.close()


@pytest.mark.parametrize("inner", ["f64", "f32", "bf16", "f16"])
def test_mg_solve_with_coarse_eo(qmg, inner):
    """The K-cycle with the coarse solve on the Schur complement reaches 1e-10 in the oracle's
    residual, with and without the even-odd fine smoother, and D^dagger too."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = fields.random_gauge(dims, 0.4, 86)
    m = 0.02
    lat = qmg.Lattice(dims, m, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 24, 8, 12, n_setup_iter=16, inner=inner, seed=5)
    b = fields.gaussian_spinor(dims, 2, 87)
    _, base = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
    mg.set_coarse_eo(True)
    for fine_eo in (False, True):
        mg.set_smoother(eo=fine_eo, sstep=fine_eo)
        banner(f"mg solve coarse eo {inner} fine_eo={fine_eo}")
        x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
        print(f"[coarse-eo] {inner} fine_eo={fine_eo}: outer {info[0]['outer_iters']} coarse "
              f"{info[0]['coarse_iters']} (full coarse operator: outer {base[0]['outer_iters']} coarse "
              f"{base[0]['coarse_iters']})")
        r = b - wilson.apply_wilson(U, to_np(x), m, 1.0, -1, dims)
        assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-10
        xa, _ = qmg.mg_solve(mg, to_gpu(b), tol=1e-10, adjoint=True)
        r = b - wilson.apply_wilson(U, to_np(xa), m, 1.0, -1, dims, dagger=True)
        assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-10
    mg.set_coarse_eo(False)
    mg.set_smoother(eo=False)
    _, again = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
    assert abs(again[0]["outer_iters"] - base[0]["outer_iters"]) <= 1
    mg.close()


def test_coarse_eo_errors(qmg):
    dims = (12, 8, 8, 8)  # coarse extent 3 in x
    U = fields.random_gauge(dims, 0.5, 88)
    lat = qmg.Lattice(dims, -0.1, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), (4, 4, 4, 4), 8, 4, 4, n_setup_iter=0, inner="f64", seed=1)
    banner("coarse eo errors")
    with pytest.raises(qmg.QmgError, match="odd"):
        mg.set_coarse_eo(True)
    d = mg.n_agg
    v = torch.zeros(1, d // 2, 2, 4, dtype=torch.complex128, device="cuda")
    with pytest.raises(qmg.QmgError, match="not set up"):
        qmg.coarse_schur_apply(mg, v)
    mg.close()
    dims = (8, 8, 8, 16)
    U = fields.random_gauge(dims, 0.5, 89)
    lat = qmg.Lattice(dims, -0.1, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), (4, 4, 4, 4), 8, 4, 4, n_setup_iter=0, inner="f64", seed=1)
    mg.add_level((1, 1, 1, 2), 8, 4, 4, n_setup_iter=0)
    with pytest.raises(qmg.QmgError, match="two-level"):
        mg.set_coarse_eo(True)
    mg.close()


def test_clover_mg_solve_with_coarse_eo(qmg):
    """The coarse Schur complement of the Wilson-clover D_c (the site term sits in every Y_0)."""
    from oracle import clover
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = fields.random_gauge(dims, 0.4, 90)
    m, cs, ct = 0.02, 1.0, 1.0
    lat = qmg.Lattice(dims, m, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 24, 8, 12, n_setup_iter=16, inner="f32", seed=5,
                                        c_sw=(cs, ct))
    T = clover.clover_term(U, dims, cs, ct)
    P = to_np(mg.prolongator()[0])
    Yo = coarse.build_coarse(U, P, m, 1.0, -1, dims, block, T=T)
    mg.set_coarse_eo(True)
    banner("clover coarse eo")
    d, k = Yo.shape[0], Yo.shape[2] // 2
    cd = geo.coarse_dims(dims, block)
    b = fields.gaussian_coarse(d * 2 * k, 1, 91).reshape(1, d, 2, k)
    x, _ = qmg.coarse_eo_solve(mg, to_gpu(b), tol=1e-12)
    ref = np.linalg.solve(coarse.dense_coarse(Yo, cd), b.reshape(1, -1).T).T.reshape(b.shape)
    assert rel(to_np(x), ref) < 1e-9
    mg.set_smoother(eo=True, sstep=True)
    bf = fields.gaussian_spinor(dims, 1, 92)
    xf, info = qmg.mg_solve(mg, to_gpu(bf), tol=1e-10)
    print(f"[coarse-eo] clover: outer {info[0]['outer_iters']} coarse {info[0]['coarse_iters']}")
    r = bf - clover.apply_clover(U, T, to_np(xf), m, 1.0, -1, dims)
    assert np.linalg.norm(r) / np.linalg.norm(bf) < 2e-10
    mg.close()
