"""GPU parity of the many-lattice hierarchy (qmg_batch_*): the setups and solves of several
independent lattices of different extents and masses run in shared launches, and each lattice is
checked against the CPU oracle run on that lattice alone: the streaming-SVD prolongator (projector
per aggregate and chirality), the Galerkin blocks of Eq. (5) (formed from P and the links on the GPU) and
the solution (dense LU where the lattice is small enough, the oracle's residual otherwise)."""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

import fields
from fields import workloads
from oracle import wilson, mg as omg, coarse
from tests._util import to_gpu, to_np, rel, projector_dist, banner

pytestmark = pytest.mark.gpu

# small enough for dense LU: block (1, 1, 2, 2) keeps every coarse extent >= 3
DENSE = [((3, 4, 6, 6), 0.07), ((4, 3, 6, 6), 0.02), ((4, 4, 6, 6), 0.045)]
DENSE_BLOCK = (1, 1, 2, 2)


@pytest.fixture(scope="module")
def dense_batch(qmg):
    lats, Us = [], []
    for i, (dims, m) in enumerate(DENSE):
        lats.append(qmg.Lattice(dims, m, 1.0, -1))
        Us.append(fields.random_gauge(dims, 0.3, 14399, 300 + i))
    lu = [sla.lu_factor(wilson.dense_wilson(U, m, 1.0, -1, dims)) for U, (dims, m) in zip(Us, DENSE)]
    return lats, Us, lu


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_batch_setup_and_solve_match_oracle_and_dense_lu(qmg, dense_batch, inner):
    lats, Us, lu = dense_batch
    banner(f"batched hierarchy of {len(lats)} lattices ({inner} inner) vs oracle and dense LU")
    bt = qmg.batch_setup(lats, [to_gpu(U) for U in Us], DENSE_BLOCK, 16, 4, 8, n_setup_iter=16, inner=inner,
                         seed=14399)
    for l, ((dims, m), U) in enumerate(zip(DENSE, Us)):
        P, sig = bt.prolongator(l)
        P = to_np(P)
        Y = to_np(bt.coarse_blocks(l))
        Yo = coarse.build_coarse(U, P, m, 1.0, -1, dims, DENSE_BLOCK)
        ey = rel(Y, Yo)
        if inner == "f64":
            # the FP64 setup follows the oracle's GMRES smoother step by step
            oh = omg.setup(omg.Lattice(U, dims, m, 1.0, -1), DENSE_BLOCK, 16, 4, 8, 16, seed=14399)
            dist = max(projector_dist(P[j, a], oh.P[j, a]) for j in range(P.shape[0]) for a in range(2))
            print(f"[parity] batch lattice {l} {dims}: projector {dist:.2e}, Galerkin blocks {ey:.2e}")
            assert dist < 1e-10
        assert ey < 1e-12
    bs = [fields.gaussian_spinor(dims, 2, 400 + l) for l, (dims, _) in enumerate(DENSE)]
    xs, info = qmg.batch_solve(bt, [to_gpu(b) for b in bs], tol=1e-12)
    for l, ((dims, m), b) in enumerate(zip(DENSE, bs)):
        x = to_np(xs[l])
        for q in range(2):
            xd = sla.lu_solve(lu[l], b[q].ravel()).reshape(b[q].shape)
            err = rel(x[q], xd)
            print(f"[precision] batch {inner} lattice {l} rhs {q}: vs dense LU {err:.2e}, res "
                  f"{info[l][q]['true_rel_res']:.2e}, outer {info[l][q]['outer_iters']}")
            assert info[l][q]["true_rel_res"] <= 1e-12
            assert err < 1e-8
    bt.close()


def test_batch_64_small_lattices(qmg):
    """The batched workload's 64 lattices (L^4, L in {8, 10, 12}, masses in [0.01, 0.1]) with FP32
    K-cycles: every lattice's solution has the oracle's residual below 2e-10; for one lattice of
    each size an FP64 batch reproduces the oracle's prolongator and its Galerkin blocks."""
    w = workloads.SMALL_LATTICES
    spec = workloads.small_lattices()
    banner(f"64 small lattices, batched setup and solve, {sum(d[0] ** 4 for d, _, _ in spec)} sites")
    lats = [qmg.Lattice(d, m, w["xi"], w["bc_t"]) for d, m, _ in spec]
    Uc = [fields.random_gauge(d, w["eps"], w["seed"], t) for d, _, t in spec]
    kw = dict(block=w["block"], n_test=w["n_test"], batch=w["batch"], rank=w["rank"], n_setup_iter=16, seed=w["seed"])
    bt = qmg.batch_setup(lats, [to_gpu(U) for U in Uc], inner=w["inner"], **kw)
    bs = [fields.gaussian_spinor(d, 1, w["seed"], tag=500 + i) for i, (d, _, _) in enumerate(spec)]
    xs, info = qmg.batch_solve(bt, [to_gpu(b) for b in bs], tol=1e-10)
    worst = 0.0
    for l, ((d, m, _), U, b) in enumerate(zip(spec, Uc, bs)):
        r = b - wilson.apply_wilson(U, to_np(xs[l]), m, w["xi"], w["bc_t"], d)
        worst = max(worst, float(np.linalg.norm(r) / np.linalg.norm(b)))
    print(f"[solve] 64 lattices FP32 inner: oracle residual worst {worst:.2e}, outer {info[0][0]['outer_iters']}, "
          f"refinements {info[0][0]['refinements']}, setup {bt.setup_times()}")
    assert worst < 2e-10
    bt.close()
    # one lattice of each size: FP64 batch against the oracle's setup of that lattice alone
    pick = [next(i for i, (d, _, _) in enumerate(spec) if d[0] == L) for L in (8, 10, 12)]
    b64 = qmg.batch_setup([lats[i] for i in pick], [to_gpu(Uc[i]) for i in pick], inner="f64", **kw)
    for l, i in enumerate(pick):
        d, m, _ = spec[i]
        oh = omg.setup(omg.Lattice(Uc[i], d, m, w["xi"], w["bc_t"]), w["block"], w["n_test"], w["batch"], w["rank"],
                       16, seed=w["seed"])
        P = to_np(b64.prolongator(l)[0])
        dist = max(projector_dist(P[j, a], oh.P[j, a]) for j in range(P.shape[0]) for a in range(2))
        ey = rel(to_np(b64.coarse_blocks(l)), coarse.build_coarse(Uc[i], P, m, w["xi"], w["bc_t"], d, w["block"]))
        print(f"[parity] small lattice {d}: projector {dist:.2e}, Galerkin blocks {ey:.2e}")
        assert dist < 1e-10 and ey < 1e-12
    b64.close()


def test_batch_errors(qmg):
    banner("batched hierarchy errors")
    dims = (4, 4, 4, 4)  # coarse extents 2 with 2^4 blocks
    lat = qmg.Lattice(dims, 0.05)
    U = to_gpu(fields.random_gauge(dims, 0.3, 1))
    with pytest.raises(qmg.QmgError) as e:
        qmg.batch_setup([lat], [U], (2, 2, 2, 2), 16, 4, 8)
    assert e.value.status == "ESHAPE"
    with pytest.raises(qmg.QmgError) as e:
        qmg.batch_setup([qmg.Lattice((6, 6, 6, 6), 0.05)], [to_gpu(fields.random_gauge((6, 6, 6, 6), 0.3, 2))],
                        (2, 2, 2, 2), 16, 4, 8, inner="bf16")
    assert e.value.status == "EDTYPE"
