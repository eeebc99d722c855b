"""The 16-bit stencil against the oracle's low-precision emulation (oracle/lowprec.py).

With links and spinor stored in BF16 or FP16, the GPU stencil computes in FP32 and rounds its
output to the format.  The emulation rounds the same inputs to the format by the format's
definition, applies the FP64 oracle operator and rounds the result.  The inputs are made exact
in FP32 first, so that both sides round once (the GPU converts FP64 -> FP32 -> format).  The two
outputs then differ only where the FP32 arithmetic moves a value across a rounding boundary of
the format: by at most one unit in the last place of the entry, plus the FP32 rounding of the
sums (relative to the operator's scale, not to the entry: where the terms of an entry cancel,
that error is several units of the small result), in a small fraction of the entries."""
import numpy as np
import pytest

import fields
from oracle import lowprec, wilson
from tests._util import to_gpu, to_np, banner

pytestmark = pytest.mark.gpu


def _ulp(y, prec):
    """Spacing of the format at |y| (the unit in the last place of each entry's value)."""
    a = np.abs(y)
    if prec == "f16":
        return np.spacing(a.astype(np.float16)).astype(np.float64)
    # bf16: 7 stored mantissa bits, binary32's exponent range
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -126)))
    return 2.0 ** (e - 7)


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_stencil_matches_rounded_storage_emulation(qmg, prec):
    dims, nrhs, m = (8, 4, 4, 8), 2, 0.05
    banner(f"stencil {prec} against the oracle's {prec} emulation")
    U = fields.random_gauge(dims, 0.6, 21)
    psi = fields.gaussian_spinor(dims, nrhs, 22)
    U = lowprec.round_to(U, "f32")  # exact in FP32: one rounding on either side
    psi = lowprec.round_to(psi, "f32")
    lat = qmg.Lattice(dims, m, 1.0, -1)
    got = to_np(qmg.unpack_spinor(lat, qmg.wilson_apply(lat, qmg.pack_gauge(lat, to_gpu(U), prec),
                                                          qmg.pack_spinor(lat, to_gpu(psi), prec), layout="native"),
                                  prec))
    Ur, pr = lowprec.round_to(U, prec), lowprec.round_to(psi, prec)
    emu = lowprec.round_to(wilson.apply_wilson(Ur, pr, m, 1.0, -1, dims), prec)
    scale = np.abs(emu).max()
    for part in ("real", "imag"):
        g, e = getattr(got, part).ravel(), getattr(emu, part).ravel()
        diff = np.abs(g - e)
        bound = _ulp(e, prec) + 2.0 ** -20 * scale  # one unit of the entry + FP32 sums (2^-24, 16 terms)
        frac = float(np.mean(diff > 0))
        print(f"[precision] stencil {prec} {part}: entries differing from the emulation {frac:.2e}, "
              f"largest difference {(diff / _ulp(e, prec)).max():.2f} ulp, {(diff / bound).max():.2f} of the bound")
        assert np.all(diff <= bound)
        assert frac < 5e-3
    # and the emulation itself is the exact operator to the format's precision
    exact = wilson.apply_wilson(U, psi, m, 1.0, -1, dims)
    rel = np.linalg.norm((emu - exact).ravel()) / np.linalg.norm(exact.ravel())
    assert rel < {"bf16": 2e-2, "f16": 2e-3}[prec]
