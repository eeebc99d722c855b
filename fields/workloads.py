"""Named synthetic workloads, shaped like the lattices of the paper's Section 4.

Each entry fixes lattice extents, boundary condition, gauge roughness eps,
anisotropy xi, quark mass, aggregate block shape, test-vector count, stream
batch, truncation rank per chirality and the inner precision of the solve.
A mass of None means "near critical": the left edge of the spectrum of D moved just inside
the right half plane (tests/golden/make_tuned_masses.py explains the reading and writes
tests/golden/tuned_masses.json, from which the value is read).
"""
from __future__ import annotations

import json
import os

WORKLOADS = {
    # 4^4, antiperiodic t, FP64 everywhere, GCR outer to 1e-10
    "wilson4x4_fp64": dict(dims=(4, 4, 4, 4), bc_t=-1, eps=0.3, xi=1.0, mass=0.05,
                           block=(2, 2, 2, 2), n_test=16, batch=4, rank=8,
                           inner="f64", seed=14399, tag=1),
    # 16^3x32 anisotropic, FP32 inner with FP64 refinement
    "aniso16x32_fp32": dict(dims=(16, 16, 16, 32), bc_t=-1, eps=0.6, xi=3.5, mass=None,
                            block=(4, 4, 4, 4), n_test=48, batch=8, rank=24,
                            inner="f32", seed=14399, tag=2),
    # the 16^3x32 anisotropic lattice with the clover term (unit coefficients in both plane
    # classes), mass tuned for D_sw
    "aniso16x32_clover": dict(dims=(16, 16, 16, 32), bc_t=-1, eps=0.6, xi=3.5, mass=None, c_sw=(1.0, 1.0),
                              block=(4, 4, 4, 4), n_test=48, batch=8, rank=24,
                              inner="f32", seed=14399, tag=2),
    # the same clover operator at its critical point: the leftmost eigenvalue of D_sw(0) on
    # these fields is real (searched on the full lattice), and the mass puts it 1e-3 inside
    # the right half plane, |lambda_min| = 1e-3 (the near-critical regime of the setup-method
    # comparison; four levels)
    "critical16x32_clover": dict(dims=(16, 16, 16, 32), bc_t=-1, eps=0.6, xi=3.5, mass=None, c_sw=(1.0, 1.0),
                                 block=(4, 4, 4, 4), n_test=48, batch=8, rank=24,
                                 inner="f32", seed=14399, tag=2),
    # 24^3x64 isotropic, BF16 storage with FP32 accumulation
    "iso24x64_bf16": dict(dims=(24, 24, 24, 64), bc_t=-1, eps=0.7, xi=1.0, mass=None,
                          block=(4, 4, 4, 4), n_test=96, batch=16, rank=24,
                          inner="bf16", seed=14399, tag=3),
    # 32^3x64 with the 12 spin-colour point sources at the origin solved together
    "batched32x64": dict(dims=(32, 32, 32, 64), bc_t=-1, eps=0.6, xi=1.0, mass=0.05,
                         block=(4, 4, 4, 4), n_test=48, batch=8, rank=24,
                         inner="f32", seed=14399, tag=4, rhs="point12", small_lattices=True,
                         # coarse solve on D_c itself: on this workload (4 outer iterations per
                         # source) it beats the Schur-complement coarse solve, whose blocks also
                         # cost 30 ms of setup
                         coarse_solve="full"),
    # differentiation workload
    "grad16x32": dict(dims=(16, 16, 16, 32), bc_t=-1, eps=0.5, xi=1.0, mass=0.03,
                      block=(4, 4, 4, 4), n_test=48, batch=8, rank=24,
                      inner="f32", seed=14399, tag=5),
}

# the 64 independent small lattices of the batched workload: L^4 with L uniform in {8, 10, 12}
# (even, so 2^4 aggregates divide them), masses uniform in [0.01, 0.1], roughness 0.3, xi = 1,
# antiperiodic t, the 4^4 workload's multigrid parameters (2^4 blocks; 16 / 4 / 8), FP32 inner
SMALL_LATTICES = dict(n=64, sizes=(8, 10, 12), mass_range=(0.01, 0.1), eps=0.3, xi=1.0, bc_t=-1,
                      block=(2, 2, 2, 2), n_test=16, batch=4, rank=8, inner="f32", seed=14399, tag=6)

_TUNED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "tests", "golden", "tuned_masses.json")


def rhs(w: dict):
    """The right-hand sides of a workload: the 12 point sources at the origin, or one complex
    Gaussian spinor."""
    import fields
    if w.get("rhs") == "point12":
        return fields.point_sources(w["dims"])
    return fields.gaussian_spinor(w["dims"], 1, w["seed"], tag=w["tag"])


def small_lattices(n=None):
    """[(dims, mass, gauge-field tag)] of the batched small-lattice workload (first n of them)."""
    import fields
    w = SMALL_LATTICES
    Ls, ms = fields.batched_lattice_params(w["n"], w["seed"], w["sizes"], w["mass_range"])
    out = [((L, L, L, L), m, w["tag"] * 1000 + i) for i, (L, m) in enumerate(zip(Ls, ms))]
    return out[:n] if n else out


def get(name: str) -> dict:
    w = dict(WORKLOADS[name])
    w["name"] = name
    if w["mass"] is None:
        with open(_TUNED) as f:
            w["mass"] = float(json.load(f)[name]["mass"])
    return w
