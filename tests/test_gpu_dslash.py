"""GPU parity of the Wilson-Dirac stencil (qmg_wilson_apply / _adj) against the oracle."""
import numpy as np
import pytest

import fields
from oracle import wilson
from tests._util import to_gpu, to_np, rel, banner

pytestmark = pytest.mark.gpu

CASES = [
    # dims, xi, bc_t, mass, nrhs
    ((4, 4, 4, 4), 1.0, -1, 0.05, 1),
    ((6, 6, 4, 10), 3.5, -1, -0.3, 3),     # 1440 sites: several 256-site tiles + ragged tail
    ((2, 4, 6, 8), 1.7, 1, 0.2, 4),        # periodic t, extent 2, 4 rhs per thread
    ((5, 3, 2, 7), 2.0, -1, 0.0, 2),       # odd extents
    ((1, 1, 1, 4), 1.0, -1, 0.1, 1),       # degenerate extents (self-neighbours)
]


@pytest.mark.parametrize("dims,xi,bc,m,nrhs", CASES)
@pytest.mark.parametrize("dag", [False, True])
def test_dslash_f64_canonical(qmg, dims, xi, bc, m, nrhs, dag):
    banner(f"dslash f64 canonical {dims} nrhs={nrhs} dag={dag}")
    U = fields.random_gauge(dims, 0.6, 1)
    psi = fields.gaussian_spinor(dims, nrhs, 2)
    lat = qmg.Lattice(dims, m, xi, bc)
    f = qmg.wilson_apply_adj if dag else qmg.wilson_apply
    got = to_np(f(lat, to_gpu(U), to_gpu(psi)))
    ref = wilson.apply_wilson(U, psi, m, xi, bc, dims, dagger=dag)
    assert rel(got, ref) < 1e-14


@pytest.mark.parametrize("dims,xi,bc,m,nrhs", CASES)
@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-6)])
def test_dslash_native(qmg, dims, xi, bc, m, nrhs, prec, tol):
    banner(f"dslash native {prec} {dims} nrhs={nrhs}")
    U = fields.random_gauge(dims, 0.6, 3)
    psi = fields.gaussian_spinor(dims, nrhs, 4)
    lat = qmg.Lattice(dims, m, xi, bc)
    Un = qmg.pack_gauge(lat, to_gpu(U), prec)
    pn = qmg.pack_spinor(lat, to_gpu(psi), prec)
    for dag in (False, True):
        f = qmg.wilson_apply_adj if dag else qmg.wilson_apply
        got = to_np(qmg.unpack_spinor(lat, f(lat, Un, pn, layout="native"), prec))
        ref = wilson.apply_wilson(U, psi, m, xi, bc, dims, dagger=dag)
        assert rel(got, ref) < tol


def test_dslash_f32_canonical_and_bf16(qmg):
    dims = (6, 6, 4, 10)
    banner(f"dslash f32 canonical + bf16/f16 native {dims}")
    U = fields.random_gauge(dims, 0.6, 5)
    psi = fields.gaussian_spinor(dims, 2, 6)
    lat = qmg.Lattice(dims, 0.05, 3.5, -1)
    ref = wilson.apply_wilson(U, psi, 0.05, 3.5, -1, dims)
    got = to_np(qmg.wilson_apply(lat, to_gpu(U.astype(np.complex64)), to_gpu(psi.astype(np.complex64))))
    assert rel(got, ref) < 1e-6
    for prec, tol in (("bf16", 1e-2), ("f16", 2e-3)):
        Un = qmg.pack_gauge(lat, to_gpu(U), prec)
        pn = qmg.pack_spinor(lat, to_gpu(psi), prec)
        got = to_np(qmg.unpack_spinor(lat, qmg.wilson_apply(lat, Un, pn, layout="native"), prec))
        err = rel(got, ref)
        print(f"[precision] dslash {prec} storage, fp32 accumulate: rel err {err:.3e}")
        assert err < tol


@pytest.mark.parametrize("dims,nrhs", [((16, 16, 16, 32), 1), ((24, 24, 24, 64), 1), ((32, 32, 32, 64), 12)])
def test_dslash_full_size_sampled(qmg, dims, nrhs):
    """Full-size lattices in the benchmark's native FP32 launch: sampled sites vs the oracle."""
    banner(f"dslash full size {dims} nrhs={nrhs}")
    xi = 3.5 if dims[0] == 16 else 1.0
    U = fields.random_gauge(dims, 0.6, 7)
    lat = qmg.Lattice(dims, -0.2, xi, -1)
    V = lat.volume
    rng = np.random.default_rng(0)
    sites = np.unique(np.concatenate([rng.integers(0, V, 48), [0, V - 1, dims[0] - 1, V - dims[0] * dims[1]]]))
    Un = qmg.pack_gauge(lat, to_gpu(U), "f32")
    del U
    psi = fields.gaussian_spinor(dims, nrhs, 8)
    pn = qmg.pack_spinor(lat, to_gpu(psi), "f32")
    out = qmg.unpack_spinor(lat, qmg.wilson_apply(lat, Un, pn, layout="native"), "f32")
    got = to_np(out[:, sites])
    del out, pn, Un
    U = fields.random_gauge(dims, 0.6, 7)
    for r in (0, nrhs - 1):
        ref = wilson.apply_wilson_sites(U, psi[r], sites, -0.2, xi, -1, dims)
        assert rel(got[r], ref) < 1e-6


@pytest.mark.parametrize("variant", [1, 2, 4, 8, 16, 32, 64, 10002, 10008])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-6), ("bf16", 1e-2)])
def test_dslash_every_launch_variant(qmg, variant, prec, tol):
    """Each native launch form (site-parallel, t-walking with 2/4/8 sites per thread, four
    threads per site)."""
    dims, nrhs = (6, 4, 4, 16), 4
    banner(f"dslash variant {variant} {prec}")
    U = fields.random_gauge(dims, 0.6, 9)
    psi = fields.gaussian_spinor(dims, nrhs, 10)
    lat = qmg.Lattice(dims, -0.1, 2.5, -1)
    Un = qmg.pack_gauge(lat, to_gpu(U), prec)
    pn = qmg.pack_spinor(lat, to_gpu(psi), prec)
    try:
        qmg.set_dslash_variant(variant)
        for dag in (False, True):
            f = qmg.wilson_apply_adj if dag else qmg.wilson_apply
            got = to_np(qmg.unpack_spinor(lat, f(lat, Un, pn, layout="native"), prec))
            ref = wilson.apply_wilson(U, psi, -0.1, 2.5, -1, dims, dagger=dag)
            assert rel(got, ref) < tol
    finally:
        qmg.set_dslash_variant(0)


@pytest.mark.parametrize("variant", [202, 204, 208, 302, 304, 308, 1202, 1204, 1208, 1302, 1304, 1308, 10204, 11308])
def test_dslash_multi_rhs_twalk_variants(qmg, variant):
    """t-walking with 2 or 3 right-hand sides per thread (FP32), both tile orders and both
    workgroup orders (10000 +: t-chunk-major), on a lattice whose xy-planes hold whole 256-site
    tiles and on one whose planes end in a partial tile."""
    for dims in ((16, 16, 4, 8), (12, 10, 6, 8)):
        nrhs = 6
        banner(f"dslash multi-rhs t-walk {variant} {dims}")
        U = fields.random_gauge(dims, 0.6, 13)
        psi = fields.gaussian_spinor(dims, nrhs, 14)
        lat = qmg.Lattice(dims, -0.3, 2.0, -1)
        Un = qmg.pack_gauge(lat, to_gpu(U), "f32")
        pn = qmg.pack_spinor(lat, to_gpu(psi), "f32")
        try:
            qmg.set_dslash_variant(variant)
            for dag in (False, True):
                f = qmg.wilson_apply_adj if dag else qmg.wilson_apply
                got = to_np(qmg.unpack_spinor(lat, f(lat, Un, pn, layout="native"), "f32"))
                ref = wilson.apply_wilson(U, psi, -0.3, 2.0, -1, dims, dagger=dag)
                assert rel(got, ref) < 1e-6
        finally:
            qmg.set_dslash_variant(0)


def test_autotuner_cache_roundtrip(qmg, tmp_path):
    dims = (8, 8, 8, 16)
    banner("autotuner")
    U = fields.random_gauge(dims, 0.6, 11)
    psi = fields.gaussian_spinor(dims, 2, 12)
    lat = qmg.Lattice(dims, -0.1, 1.0, -1)
    Un = qmg.pack_gauge(lat, to_gpu(U), "f32")
    pn = qmg.pack_spinor(lat, to_gpu(psi), "f32")
    try:
        qmg.autotune(True)
        got = to_np(qmg.unpack_spinor(lat, qmg.wilson_apply(lat, Un, pn, layout="native"), "f32"))
        assert rel(got, wilson.apply_wilson(U, psi, -0.1, 1.0, -1, dims)) < 1e-6
        path = tmp_path / "tune.json"
        qmg.tune_save(path)
        text = path.read_text()
        assert "dslash/1/8x8x8x16/2/0" in text
        qmg.tune_load(path)
    finally:
        qmg.autotune(False)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-6), ("bf16", 1e-2)])
def test_dslash_batched_uneven_lattices(qmg, prec, tol):
    """Uneven lattices (extents, boundary, mass, anisotropy all different) in one launch, D and
    D^dagger, against the oracle lattice by lattice."""
    specs = [((4, 4, 4, 4), -1, -0.1, 1.0), ((6, 4, 2, 8), 1, 0.2, 2.5), ((8, 8, 8, 8), -1, 0.05, 1.0),
             ((2, 2, 2, 2), -1, 0.3, 3.5), ((10, 6, 4, 6), 1, -0.3, 1.5), ((3, 5, 7, 9), -1, 0.0, 1.2)]
    banner(f"batched dslash {len(specs)} lattices {prec}")
    nrhs = 2
    lats, Us, ps, Ucs, pcs = [], [], [], [], []
    for i, (dims, bc, m, xi) in enumerate(specs):
        lat = qmg.Lattice(dims, m, xi, bc)
        U = fields.random_gauge(dims, 0.6, 60 + i)
        psi = fields.gaussian_spinor(dims, nrhs, 70 + i)
        lats.append(lat)
        Ucs.append(U)
        pcs.append(psi)
        Us.append(qmg.pack_gauge(lat, to_gpu(U), prec))
        ps.append(qmg.pack_spinor(lat, to_gpu(psi), prec))
    for dag in (False, True):
        outs = qmg.wilson_apply_batched(lats, Us, ps, dagger=dag)
        for i, (dims, bc, m, xi) in enumerate(specs):
            got = to_np(qmg.unpack_spinor(lats[i], outs[i], prec))
            ref = wilson.apply_wilson(Ucs[i], pcs[i], m, xi, bc, dims, dagger=dag)
            assert rel(got, ref) < tol, (i, dag)
