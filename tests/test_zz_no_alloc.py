"""The entry point that allocates nothing (qmg_coarse_schur_apply_noalloc) against the allocating
qmg_coarse_schur_apply it mirrors, through the C ABI: two calls in a row, the second with a
smaller input, on two hierarchies (FP64 and FP32 blocks), and against the oracle's Schur
complement of the hierarchy's own D_c; a call that would need more than the fixed scratch array
is rejected before any launch."""
import numpy as np
import pytest
import torch

import fields
from oracle import coarse, coarse_evenodd as ceo, geometry as geo
from tests._util import to_gpu, to_np, rel, banner

pytestmark = pytest.mark.gpu


def _hierarchy(qmg, dims, block, k, inner, seed):
    U = fields.random_gauge(dims, 0.5, seed)
    lat = qmg.Lattice(dims, -0.1, 2.0, -1)
    phi = fields.gaussian_test_vectors(dims, 2 * k, seed + 1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 2 * k, k, k, n_setup_iter=0, inner=inner,
                                        test_vectors=to_gpu(phi))
    mg.set_coarse_eo(True)
    P = to_np(mg.prolongator()[0])
    Yo = coarse.build_coarse(U, P, -0.1, 2.0, -1, dims, block)
    return mg, Yo, geo.coarse_dims(dims, block)


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_noalloc_equals_allocating_apply(qmg, inner):
    cdt = torch.complex128 if inner == "f64" else torch.complex64
    tol = 1e-13 if inner == "f64" else 2e-6
    # the second hierarchy is smaller (fewer aggregates, lower rank), and so is its call
    for (dims, block, k), nrhs, seed in ((((8, 8, 8, 8), (4, 4, 4, 4), 12), 4, 121),
                                         (((4, 4, 4, 8), (2, 2, 2, 2), 5), 1, 123)):
        banner(f"no-alloc coarse Schur apply {inner} {dims} k={k} nrhs={nrhs}")
        mg, Yo, cd = _hierarchy(qmg, dims, block, k, inner, seed)
        d = Yo.shape[0]
        eo = ceo.CoarseEvenOdd(Yo, cd)
        e = eo.par == 0
        for n in (nrhs, 1):  # two calls in a row on this hierarchy, the second with one rhs
            v = fields.gaussian_coarse(d * 2 * k, n, seed + n).reshape(n, d, 2 * k)
            vin = to_gpu(v[:, e].reshape(n, d // 2, 2, k)).to(cdt)
            want = qmg.coarse_schur_apply(mg, vin)
            out = torch.full_like(vin, float("nan"))
            got = qmg.coarse_schur_apply_noalloc(mg, vin, out)
            torch.cuda.synchronize()
            assert torch.equal(got, want)  # the same kernels on the same inputs
            ref = eo.schur(ceo.restrict_parity(v, eo.par, 0))[:, e].reshape(n, d // 2, 2, k)
            assert rel(to_np(got), ref) < tol
        mg.close()


def test_noalloc_rejects_beyond_scratch(qmg):
    dims, block, k = (8, 8, 8, 8), (4, 4, 4, 4), 12
    mg, Yo, _ = _hierarchy(qmg, dims, block, k, "f64", 125)
    d = Yo.shape[0]
    banner("no-alloc coarse Schur apply: size beyond the scratch array")
    n = (16 << 20) // (k * d * 16) + 1  # one right-hand side more than the 16 MiB array holds
    v = torch.zeros(n, d // 2, 2, k, dtype=torch.complex128, device="cuda")
    out = torch.empty_like(v)
    with pytest.raises(qmg.QmgError) as e:
        qmg.coarse_schur_apply_noalloc(mg, v, out)
    assert e.value.status == "ESHAPE" and "scratch" in str(e.value)
    # the largest size that fits still works
    got = qmg.coarse_schur_apply_noalloc(mg, v[: n - 1].contiguous(), out[: n - 1])
    torch.cuda.synchronize()
    assert torch.count_nonzero(got) == 0
    mg.close()
