"""Solution parity of the mixed-precision solves.

The K-cycle stored in FP32, BF16 or FP16 (FP32 arithmetic) runs inside the FP64 defect
correction; the solution is compared with dense LU of D (and of D^dagger for the adjoint solve),
with both the plain GMRES(8) post-smoother on the full coarse operator and the benchmark's
even-odd s-step smoother with the coarse solve on the even-odd Schur complement of D_c.  The
solves run to a true FP64 residual of 1e-12, so the 1e-8 solution bound holds for any condition
number below 1e4 (||x - x*|| / ||x*|| <= kappa(D) * tol)."""
import numpy as np
import pytest
import scipy.linalg as sla

import fields
from fields import workloads
from oracle import wilson
from tests._util import to_gpu, to_np, rel, banner

pytestmark = pytest.mark.gpu

# (name, dims, eps, field seed, mass, block, n_test, batch, rank): the 4^4 workload, and an
# 8x4x4x4 lattice of rougher links whose mass puts the left edge of the spectrum of D
# (1.335 +- 0.424i at m = 0, from the dense eigenvalues) 0.035 inside the right half plane
CASES = {
    "wilson4x4": None,
    "edge8x4": dict(dims=(8, 4, 4, 4), eps=0.5, seed=93, tag=0, mass=-1.30, xi=1.0, bc_t=-1, block=(2, 2, 2, 2),
                    n_test=16, batch=4, rank=8),
}
_LU = {}


def _case(name):
    if name == "wilson4x4":
        w = workloads.get("wilson4x4_fp64")
    else:
        w = dict(CASES[name])
    U = fields.random_gauge(w["dims"], w["eps"], w["seed"], w["tag"])
    if name not in _LU:
        Dm = wilson.dense_wilson(U, w["mass"], w["xi"], w["bc_t"], w["dims"])
        _LU[name] = (sla.lu_factor(Dm), sla.lu_factor(np.conj(Dm.T)))
    return w, U, _LU[name]


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("form", ["plain", "evenodd"])
@pytest.mark.parametrize("inner", ["f32", "bf16", "f16"])
def test_mixed_solution_matches_dense_lu(qmg, case, form, inner):
    w, U, (lu, lua) = _case(case)
    dims = w["dims"]
    banner(f"mixed solution parity {case} {dims} inner={inner} form={form}")
    lat = qmg.Lattice(dims, w["mass"], w["xi"], w["bc_t"])
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), w["block"], w["n_test"], w["batch"], w["rank"],
                                        n_setup_iter=16, inner=inner, seed=14399)
    if form == "evenodd":
        mg.set_smoother(eo=True, sstep=True)
        mg.set_coarse_eo(True)
    b = fields.gaussian_spinor(dims, 2, 101)
    for adjoint in (False, True):
        x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-12, adjoint=adjoint)
        x = to_np(x)
        errs = []
        for q in range(2):
            xd = sla.lu_solve(lua if adjoint else lu, b[q].ravel()).reshape(b[q].shape)
            errs.append(rel(x[q], xd))
        print(f"[precision] {case} {inner} {form} {'D^dag' if adjoint else 'D'}: solution error vs dense LU "
              f"{max(errs):.2e}, true res {max(i['true_rel_res'] for i in info):.2e}, outer "
              f"{[i['outer_iters'] for i in info]}, refinements {[i['refinements'] for i in info]}")
        assert max(i["true_rel_res"] for i in info) <= 1e-12
        assert max(errs) < 1e-8
        # the oracle's own residual of the returned solution
        r = b - wilson.apply_wilson(U, x, w["mass"], w["xi"], w["bc_t"], dims, dagger=adjoint)
        assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-12
    mg.close()
