"""GPU parity of the third level (Algorithm 4 applied to D_c) against oracle/level.py, and the
three-level solve."""
import numpy as np
import pytest
import torch

import fields
from oracle import coarse, level
from tests._util import to_gpu, to_np, rel, banner

pytestmark = pytest.mark.gpu


def _hier(qmg, dims, block, n_test, batch, k, inner, seed, mass=0.05, eps=0.3):
    U = to_gpu(fields.random_gauge(dims, eps, seed))
    lat = qmg.Lattice(dims, mass, 1.0, -1)
    return qmg.mg_setup_stream_chiral_svd(lat, U, block, n_test, batch, k, n_setup_iter=4, inner=inner, seed=seed), U


def test_level_setup_matches_oracle(qmg):
    """Coarse test vectors, FP64 smoothing on D_c, chiral split and streaming SVD of the third
    level against the oracle run on the GPU's own D_c; the coarse-coarse stencil against the
    oracle's Galerkin product with the GPU's P2."""
    banner("third level setup parity")
    mg, _ = _hier(qmg, (8, 8, 8, 8), (2, 2, 2, 2), 12, 4, 6, "f64", 51)
    block2, n2, r2, k2 = (2, 2, 2, 2), 12, 4, 5
    mg.add_level(block2, n2, r2, k2, n_setup_iter=4, seed=7)
    assert mg.level_dims == (2, 2, 2, 2) and mg.level_rank == k2
    Y1 = to_np(mg.coarse_blocks())
    cd = mg.coarse_dims
    lv = level.setup(Y1, cd, block2, n2, r2, k2, n_setup_iter=4, seed=7, level=1)
    P2, sig2 = mg.level_prolongator()
    P2 = to_np(P2)
    assert np.abs(sig2 - lv.sigma).max() < 1e-10 * lv.sigma.max()
    for J in range(P2.shape[0]):
        for a in range(2):
            g, o = P2[J, a], lv.P[J, a]
            assert np.abs(g @ np.conj(g).T - o @ np.conj(o).T).max() < 1e-9
    Y2 = to_np(mg.level_coarse_blocks())
    ref = level.galerkin(Y1, P2, cd, block2, mg.rank)
    assert rel(Y2, ref) < 1e-12
    mg.close()


@pytest.mark.parametrize("inner,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_level_transfer_and_operator(qmg, inner, tol):
    """P2, P2^dag and D_cc on coarse vectors against the oracle (with the GPU's P2 and D_cc),
    on a blocking whose coarse-coarse extents are 1 and 2."""
    banner(f"third level transfer {inner}")
    mg, _ = _hier(qmg, (8, 4, 8, 8), (2, 2, 2, 2), 12, 4, 6, inner, 52)
    block2 = (4, 1, 2, 2)
    mg.add_level(block2, 8, 4, 4, n_setup_iter=2, seed=9)
    P2 = to_np(mg.level_prolongator()[0])
    Y2 = to_np(mg.level_coarse_blocks())
    cd, k = mg.coarse_dims, mg.rank
    d, d2, k2 = mg.n_agg, mg.level_n_agg, mg.level_rank
    rng = np.random.default_rng(3)
    v2 = rng.normal(size=(3, d2, 2, k2)) + 1j * rng.normal(size=(3, d2, 2, k2))
    v1 = rng.normal(size=(3, d, 2, k)) + 1j * rng.normal(size=(3, d, 2, k))
    dt = torch.complex128 if inner == "f64" else torch.complex64
    g = lambda a: torch.from_numpy(a).to(dt).cuda()
    got = to_np(qmg.level_prolong(mg, g(v2))).reshape(3, d, 2 * k)
    assert rel(got, level.prolong(P2, v2, cd, block2, k)) < tol
    got = to_np(qmg.level_restrict(mg, g(v1)))
    assert rel(got, level.restrict(P2, v1.reshape(3, d, 2 * k), cd, block2, k)) < tol
    got = to_np(qmg.level_coarse_apply(mg, g(v2)))
    assert rel(got, coarse.coarse_apply(Y2, v2, mg.level_dims)) < tol
    mg.close()


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_three_level_solve(qmg, inner):
    """The three-level solve reaches 1e-10 and, at 1e-12, gives the two-level solution."""
    banner(f"three-level solve {inner}")
    dims = (8, 8, 8, 8)
    mg2, U = _hier(qmg, dims, (2, 2, 2, 2), 16, 8, 8, inner, 53, mass=-0.3, eps=0.4)
    b = to_gpu(fields.gaussian_spinor(dims, 1, 54))
    x2, i2 = qmg.mg_solve(mg2, b, tol=1e-12)
    mg3, _ = _hier(qmg, dims, (2, 2, 2, 2), 16, 8, 8, inner, 53, mass=-0.3, eps=0.4)
    mg3.add_level((2, 2, 2, 2), 16, 8, 8, n_setup_iter=4)
    x3, i3 = qmg.mg_solve(mg3, b, tol=1e-12)
    assert i3[0]["true_rel_res"] < 1e-12 and i3[0]["coarse2_iters"] > 0 and i3[0]["smoother1_iters"] > 0
    assert i2[0]["coarse2_iters"] == 0
    assert rel(to_np(x3), to_np(x2)) < 1e-8
    _, i = qmg.mg_solve(mg3, b, tol=1e-10)
    assert i[0]["true_rel_res"] < 1e-10
    print(f"[levels] {inner}: two levels {i2[0]['outer_iters']} outer / {i2[0]['coarse_iters']} coarse; "
          f"three levels {i3[0]['outer_iters']} / {i3[0]['coarse_iters']} / {i3[0]['coarse2_iters']}")
    mg2.close()
    mg3.close()


def test_level_errors(qmg):
    banner("third level errors")
    mg, _ = _hier(qmg, (4, 4, 4, 8), (2, 2, 2, 2), 8, 4, 4, "f64", 55)
    with pytest.raises(qmg.QmgError, match="no level 2"):
        qmg.level_coarse_apply(mg, torch.zeros(1, 1, 2, 1, dtype=torch.complex128, device="cuda"))
    with pytest.raises(qmg.QmgError, match="does not divide"):
        mg.add_level((3, 1, 1, 1), 8, 4, 4)
    with pytest.raises(qmg.QmgError, match="rank"):
        mg.add_level((2, 2, 2, 2), 8, 4, 40)
    mg.add_level((2, 2, 2, 2), 8, 4, 4, n_setup_iter=2)
    with pytest.raises(qmg.QmgError, match="host-checked"):
        mg.set_cycle(coarse_steps=12)
    mg.level_coarse_blocks(level=2)  # level 2 exists, level 3 not yet
    assert qmg.load_library().qmg_mg_level_query(mg.handle, 3, None, None, None) == -1
    assert b"no level 3" in qmg.load_library().qmg_last_error()
    mg.add_level((1, 1, 1, 2), 8, 4, 4, n_setup_iter=2)
    with pytest.raises(qmg.QmgError, match="four levels"):
        mg.add_level((1, 1, 1, 1), 8, 4, 4)
    for lv, t in ((1, 0.1), (4, 0.1), (2, 1.0), (2, -0.1)):
        with pytest.raises(qmg.QmgError):
            mg.set_level_tol(lv, t)
    mg.set_level_tol(3, 0.0)
    mg.close()


def test_more_streams_rebuild_the_third_level(qmg):
    """After qmg_mg_stream_more the third level is rebuilt on the new D_c: it equals a third level
    added to a hierarchy set up with the larger n_test from the start."""
    banner("third level after more streams")
    a, U = _hier(qmg, (4, 4, 4, 8), (2, 2, 2, 2), 8, 4, 4, "f64", 56)
    a.add_level((1, 1, 2, 2), 8, 4, 4, n_setup_iter=2, seed=3)
    a.stream_more(1)
    b, _ = _hier(qmg, (4, 4, 4, 8), (2, 2, 2, 2), 12, 4, 4, "f64", 56)
    b.add_level((1, 1, 2, 2), 8, 4, 4, n_setup_iter=2, seed=3)
    assert np.array_equal(to_np(a.level_coarse_blocks()), to_np(b.level_coarse_blocks()))
    assert np.array_equal(a.level_prolongator()[1], b.level_prolongator()[1])
    a.close()
    b.close()


def test_fourth_level_matches_oracle(qmg):
    """A fourth level on the third level's operator (Philox level word 2): its setup against the
    oracle run on the GPU's level-2 stencil, its Galerkin stencil, transfer and operator; and the
    four-level solve gives the two-level solution."""
    banner("fourth level parity and solve")
    dims = (8, 8, 8, 8)
    mg, U = _hier(qmg, dims, (2, 2, 2, 2), 12, 4, 6, "f64", 57, mass=-0.3, eps=0.4)
    mg.add_level((2, 2, 2, 2), 12, 4, 6, n_setup_iter=4, seed=5)
    block3 = (1, 2, 2, 2)
    assert mg.add_level(block3, 8, 4, 5, n_setup_iter=4, seed=5) == 3
    assert mg.levels[3]["dims"] == (2, 1, 1, 1)
    Y2 = to_np(mg.level_coarse_blocks(2))
    cd2 = mg.levels[2]["dims"]
    lv = level.setup(Y2, cd2, block3, 8, 4, 5, n_setup_iter=4, seed=5, level=2)
    P3, sig3 = mg.level_prolongator(3)
    P3 = to_np(P3)
    assert np.abs(sig3 - lv.sigma).max() < 1e-10 * lv.sigma.max()
    for J in range(P3.shape[0]):
        for a in range(2):
            g, o = P3[J, a], lv.P[J, a]
            assert np.abs(g @ np.conj(g).T - o @ np.conj(o).T).max() < 1e-9
    Y3 = to_np(mg.level_coarse_blocks(3))
    k2 = mg.levels[2]["rank"]
    assert rel(Y3, level.galerkin(Y2, P3, cd2, block3, k2)) < 1e-12
    rng = np.random.default_rng(4)
    d2, d3, k3 = mg.levels[2]["n_agg"], mg.levels[3]["n_agg"], mg.levels[3]["rank"]
    v3 = rng.normal(size=(2, d3, 2, k3)) + 1j * rng.normal(size=(2, d3, 2, k3))
    v2 = rng.normal(size=(2, d2, 2, k2)) + 1j * rng.normal(size=(2, d2, 2, k2))
    g = lambda a: torch.from_numpy(a).cuda()
    got = to_np(qmg.level_prolong(mg, g(v3), level=3)).reshape(2, d2, 2 * k2)
    assert rel(got, level.prolong(P3, v3, cd2, block3, k2)) < 1e-13
    got = to_np(qmg.level_restrict(mg, g(v2), level=3))
    assert rel(got, level.restrict(P3, v2.reshape(2, d2, 2 * k2), cd2, block3, k2)) < 1e-13
    got = to_np(qmg.level_coarse_apply(mg, g(v3), level=3))
    assert rel(got, coarse.coarse_apply(Y3, v3, mg.levels[3]["dims"])) < 1e-13
    b = to_gpu(fields.gaussian_spinor(dims, 1, 58))
    x4, i4 = qmg.mg_solve(mg, b, tol=1e-12)
    assert i4[0]["true_rel_res"] < 1e-12 and i4[0]["coarse3_iters"] > 0 and i4[0]["smoother2_iters"] > 0
    mg2, _ = _hier(qmg, dims, (2, 2, 2, 2), 12, 4, 6, "f64", 57, mass=-0.3, eps=0.4)
    x2, _ = qmg.mg_solve(mg2, b, tol=1e-12)
    assert rel(to_np(x4), to_np(x2)) < 1e-8
    print(f"[levels] four levels: {i4[0]['outer_iters']} / {i4[0]['coarse_iters']} / {i4[0]['coarse2_iters']} / "
          f"{i4[0]['coarse3_iters']}")
    # looser solves on the lower levels (0.06 on level 2, 0.6 on level 3): fewer iterations there,
    # the same solution
    mg.set_level_tol(2, 0.06)
    mg.set_level_tol(3, 0.6)
    x4l, i4l = qmg.mg_solve(mg, b, tol=1e-12)
    assert i4l[0]["true_rel_res"] < 1e-12 and rel(to_np(x4l), to_np(x2)) < 1e-8
    assert i4l[0]["coarse3_iters"] < i4[0]["coarse3_iters"]
    print(f"[levels] four levels, level tolerances 0.06 / 0.6: {i4l[0]['outer_iters']} / {i4l[0]['coarse_iters']} / "
          f"{i4l[0]['coarse2_iters']} / {i4l[0]['coarse3_iters']}")
    mg.close()
    mg2.close()
