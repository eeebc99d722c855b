"""Pins of the oracle's low-precision emulation (oracle/lowprec.py): the storage formats'
rounding against their definitions, the size of the error a rounded operator makes, and the
FP64 defect correction around the rounded K-cycle reaching the FP64 solution."""
import numpy as np
import pytest
import scipy.linalg as sla

import fields
from fields import workloads
from oracle import lowprec, mg as omg, wilson


def _bf16_by_distance(x):
    """bfloat16 rounding from its definition, independently of the bit arithmetic: the two
    representable neighbours of a binary32 value (mantissa truncated to 7 stored bits, and the
    next value up in magnitude), the nearer one, ties to the even stored mantissa."""
    out = np.empty_like(x)
    for i, v in enumerate(np.asarray(x, dtype=np.float32)):
        bits = int(np.array(v, dtype=np.float32).view(np.uint32))
        lo_bits = bits & 0xFFFF0000
        hi_bits = lo_bits + 0x10000
        lo = float(np.array(lo_bits, dtype=np.uint32).view(np.float32))
        hi = float(np.array(hi_bits, dtype=np.uint32).view(np.float32))
        dl, dh = abs(float(v) - lo), abs(hi - float(v))
        if dl < dh:
            out[i] = lo
        elif dh < dl:
            out[i] = hi
        else:
            out[i] = lo if ((lo_bits >> 16) & 1) == 0 else hi
    return out


def test_bf16_rounding_known_values():
    # 7 stored mantissa bits: the spacing at 1 is 2^-7
    cases = {1.0: 1.0, 1 + 2 ** -7: 1 + 2 ** -7, 1 + 2 ** -8: 1.0, 1 + 3 * 2 ** -8: 1 + 2 ** -6,
             1 + 2 ** -8 + 2 ** -20: 1 + 2 ** -7, -(1 + 3 * 2 ** -8): -(1 + 2 ** -6), 3.0: 3.0,
             256.0 + 1.0: 256.0, 0.0: 0.0}
    for x, want in cases.items():
        assert lowprec.round_to(np.array([x]), "bf16")[0] == want, x


def test_bf16_rounding_matches_nearest_neighbour_definition():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(size=400) * 10.0 ** rng.integers(-6, 6, size=400),
                        # exact ties: a bf16 value plus half its spacing
                        (1 + rng.integers(0, 128, size=100) * 2 ** -7 + 2 ** -8) * 2.0 ** rng.integers(-4, 4, 100)])
    x = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(lowprec.round_to(x, "bf16"), _bf16_by_distance(x))


def test_f32_f16_rounding_known_values():
    assert lowprec.round_to(np.array([1 + 2 ** -30]), "f32")[0] == 1.0
    assert lowprec.round_to(np.array([1 + 2 ** -23]), "f32")[0] == 1 + 2 ** -23
    assert lowprec.round_to(np.array([1 + 2 ** -11]), "f16")[0] == 1.0       # tie to even
    assert lowprec.round_to(np.array([1 + 3 * 2 ** -11]), "f16")[0] == 1 + 2 ** -9
    z = np.array([1 + 3 * 2 ** -8 - 1j * (1 + 2 ** -8)])
    assert lowprec.round_to(z, "bf16")[0] == (1 + 2 ** -6) - 1j


@pytest.fixture(scope="module")
def c1():
    w = workloads.get("wilson4x4_fp64")
    dims = w["dims"]
    U = fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])
    lat = omg.Lattice(U, dims, w["mass"], w["xi"], w["bc_t"])
    h = omg.setup(lat, w["block"], w["n_test"], w["batch"], w["rank"], 16, seed=w["seed"])
    Dm = wilson.dense_wilson(U, w["mass"], w["xi"], w["bc_t"], dims)
    return w, h, sla.lu_factor(Dm)


def test_rounded_operator_error_is_the_format_s(c1):
    """One application of D with links and output stored in the format: zero in FP64, of the
    format's unit roundoff otherwise (FP32 2^-24, BF16 2^-8, FP16 2^-11)."""
    w, h, _ = c1
    v = fields.gaussian_spinor(w["dims"], 1, 77)[0]
    assert lowprec.operator_defect(h, "f64", v) == 0.0
    e32 = lowprec.operator_defect(h, "f32", v)
    e16 = lowprec.operator_defect(h, "f16", v)
    ebf = lowprec.operator_defect(h, "bf16", v)
    assert 1e-9 < e32 < 1e-6
    assert 1e-5 < e16 < 2e-3
    assert 1e-4 < ebf < 2e-2
    assert e32 < e16 < ebf
    # P and D_c are stored in the format too: representable there, and not the FP64 arrays
    rh = lowprec.RoundedHierarchy(h, "bf16")
    for got, full in ((rh.P, h.P), (rh.Y, h.Y), (rh.U, h.lat.U)):
        assert np.array_equal(lowprec.round_to(got, "bf16"), got)
        assert 1e-4 < np.abs(got - full).max() / np.abs(full).max() < 1e-2


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_mixed_solve_reaches_the_fp64_solution(c1, prec):
    """FP64 defect correction around the rounded K-cycle: true residual 1e-12, the dense-LU
    solution to 1e-8 (kappa(D) < 1e4 on this lattice), and more refinements the coarser the
    format (FP64 inner solves to 1e-10 need two)."""
    w, h, lu = c1
    b = fields.gaussian_spinor(w["dims"], 1, 101)[0]
    x, st = lowprec.mixed_solve(h, b, prec, tol=1e-12)
    xd = sla.lu_solve(lu, b.ravel()).reshape(b.shape)
    err = np.linalg.norm((x - xd).ravel()) / np.linalg.norm(xd.ravel())
    print(f"[precision] oracle mixed solve {prec}: refinements {st['refinements']}, inner {st['inner']}, "
          f"residual {st['true_rel_res']:.2e}, error vs dense LU {err:.2e}")
    assert st["true_rel_res"] <= 1e-12
    assert err < 1e-8
    want_min = {"f64": 2, "f32": 2, "bf16": 4, "f16": 4}[prec]
    assert want_min <= st["refinements"] <= 12
