"""Full-size workloads on the GPU, checked against the oracle where it can follow: the 24^3 x 64
solve with a BF16 K-cycle, the 32^3 x 64 solve of the twelve spin-colour point sources, and 64
independent small lattices (8^4 to 12^4, masses in [0.01, 0.1]) in one dslash launch.  The
oracle evaluates D site by site at sampled sites of the large lattices."""
import numpy as np
import pytest
import torch

import fields
from fields import workloads
from oracle import wilson, geometry as geo
from tests._util import to_gpu, to_np, rel, banner

pytestmark = pytest.mark.gpu


def _setup(qmg, w, U):
    lat = qmg.Lattice(w["dims"], w["mass"], w["xi"], w["bc_t"])
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), w["block"], w["n_test"], w["batch"], w["rank"],
                                        n_setup_iter=16, inner=w["inner"], seed=w["seed"])
    return lat, mg


def _sample_sites(dims, rng, n, extra=()):
    V = geo.volume(dims)
    return np.unique(np.concatenate([rng.choice(V, n, replace=False), np.asarray(extra, dtype=np.int64)]))


def test_solve_iso24x64_bf16(qmg):
    """BF16-stored K-cycle in FP32 flexible GMRES and FP64 defect correction reaches 1e-10 on 24^3 x 64."""
    w = workloads.get("iso24x64_bf16")
    banner(f"solve {w['name']} {w['dims']} m={w['mass']:.4f}")
    U = fields.random_gauge(w["dims"], w["eps"], w["seed"], w["tag"])
    lat, mg = _setup(qmg, w, U)
    b = fields.gaussian_spinor(w["dims"], 1, w["seed"], tag=w["tag"])
    x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
    print(f"[solve] {info[0]}")
    assert info[0]["true_rel_res"] <= 1e-10
    sites = _sample_sites(w["dims"], np.random.default_rng(3), 64)
    xh = to_np(x)[0]
    r = b[0][sites] - wilson.apply_wilson_sites(U, xh, sites, w["mass"], w["xi"], w["bc_t"], w["dims"])
    # the global relative residual is <= 1e-10; at 64 sampled sites against |b| there
    assert np.linalg.norm(r) / np.linalg.norm(b[0][sites]) < 1e-8
    mg.close()


def test_solve_batched32x64_point_sources(qmg):
    """The twelve spin-colour point sources of 32^3 x 64 in one multi-RHS solve."""
    w = workloads.get("batched32x64")
    dims = w["dims"]
    banner(f"solve {w['name']} {dims} 12 point sources")
    U = fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])
    lat, mg = _setup(qmg, w, U)
    V = geo.volume(dims)
    b = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device="cuda")
    for k in range(12):  # unit source at the origin in spin k // 3, colour k % 3
        b[k, 0, k // 3, k % 3] = 1.0
    x, info = qmg.mg_solve(mg, b, tol=1e-10)
    print(f"[solve] outer {[i['outer_iters'] for i in info]} worst {max(i['true_rel_res'] for i in info):.2e}")
    assert max(i["true_rel_res"] for i in info) <= 1e-10
    nb = geo.neighbor_table(dims)
    sites = _sample_sites(dims, np.random.default_rng(4), 32, extra=[0, *nb[0]])
    for k in (0, 7, 11):
        xh = x[k].cpu().numpy()
        bh = np.zeros((V, 4, 3), np.complex128)
        bh[0, k // 3, k % 3] = 1.0
        r = bh[sites] - wilson.apply_wilson_sites(U, xh, sites, w["mass"], w["xi"], w["bc_t"], dims)
        assert np.linalg.norm(r) < 1e-8  # |b| = 1
    mg.close()


@pytest.mark.parametrize("prec,tol", [("f32", 1e-6), ("bf16", 1e-2)])
def test_dslash_64_small_lattices_one_launch(qmg, prec, tol):
    """64 hypercubic lattices L^4 with L uniform in 8..12 and masses uniform in [0.01, 0.1]."""
    rng = np.random.default_rng(64)
    Ls = rng.integers(8, 13, size=64)
    masses = rng.uniform(0.01, 0.1, size=64)
    banner(f"64 small lattices in one dslash launch ({prec}), sites {int(sum(L**4 for L in Ls))}")
    lats, Us, ps, Uc, pc = [], [], [], [], []
    for i, (L, m) in enumerate(zip(Ls, masses)):
        dims = (int(L),) * 4
        lat = qmg.Lattice(dims, float(m), 1.0, -1)
        U = fields.random_gauge(dims, 0.6, 1000 + i)
        psi = fields.gaussian_spinor(dims, 1, 2000 + i)
        lats.append(lat)
        Uc.append(U)
        pc.append(psi)
        Us.append(qmg.pack_gauge(lat, to_gpu(U), prec))
        ps.append(qmg.pack_spinor(lat, to_gpu(psi), prec))
    outs = qmg.wilson_apply_batched(lats, Us, ps)
    for i in range(64):
        got = to_np(qmg.unpack_spinor(lats[i], outs[i], prec))
        ref = wilson.apply_wilson(Uc[i], pc[i], float(masses[i]), 1.0, -1, lats[i].dims)
        assert rel(got, ref) < tol, i
