"""Low-precision emulation of the mixed-precision solve (test infrastructure, CPU only).

The GPU solve stores the K-cycle's operators and vectors in FP32, BF16 or FP16 and runs it
inside FP64 defect correction (the precision form of the method's hot path; the paper names no
precision).  This module is the plain reference for that form: the stored data are rounded to
the storage format by the format's own definition, the arithmetic stays FP64, and the outer
loop is the textbook defect correction

    r = b - D x (FP64),  solve D e = r / ||r|| to a relative tolerance with the rounded
    K-cycle,  x = x + ||r|| e,  until ||b - D x|| <= tol ||b||
(the inner right-hand side has unit norm, so the shrinking residuals stay inside the range of
the 16-bit formats).

Rounding (round to nearest, ties to even, on each real component):
  f32   IEEE binary32 (numpy's conversion)
  f16   IEEE binary16 (numpy's conversion)
  bf16  the upper 16 bits of the binary32 value: 8 exponent bits, 7 stored mantissa bits
  f64   no rounding
Stored data: the links of D, the prolongator P, the coarse blocks D_c, and every vector an
operator of the inner solve returns (its output is stored in the format before it is used).

Only tests/ call this module.
"""
import numpy as np

from . import krylov, coarse, transfer, mg

INNER_TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-2, "f16": 1e-2}


def _bf16(x):
    """float64 array -> float64 array of the nearest bfloat16 values (ties to even)."""
    f = np.ascontiguousarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def round_to(x, prec):
    """x (real or complex) rounded component-wise to the storage format `prec`."""
    x = np.asarray(x)
    if prec == "f64":
        return x.copy()
    if np.iscomplexobj(x):
        return round_to(x.real, prec) + 1j * round_to(x.imag, prec)
    if prec == "f32":
        return x.astype(np.float32).astype(np.float64)
    if prec == "f16":
        return x.astype(np.float16).astype(np.float64)
    if prec == "bf16":
        return _bf16(x)
    raise ValueError(prec)


class RoundedHierarchy:
    """The hierarchy h with its stored operators in the format prec: D on rounded links,
    P and D_c rounded; operator outputs rounded to the format."""

    def __init__(self, h, prec):
        lat = h.lat
        self.prec = prec
        self.h = h
        self.U = round_to(lat.U, prec)
        self.T = None if lat.T is None else round_to(lat.T, prec)
        self.P = round_to(h.P, prec)
        self.Y = round_to(h.Y, prec)
        self.lat = mg.Lattice(self.U, lat.dims, lat.mass, lat.xi, lat.bc_t, T=self.T)

    def D(self, v):
        return round_to(self.lat.D(v), self.prec)

    def restrict(self, v):
        return round_to(transfer.restrict(self.P, v, self.lat.dims, self.h.block), self.prec)

    def prolong(self, vc):
        return round_to(transfer.prolong(self.P, vc, self.lat.dims, self.h.block), self.prec)

    def coarse_op(self, vc):
        return round_to(coarse.coarse_apply(self.Y, vc, self.h.cdims), self.prec)


def kcycle(rh, r, coarse_tol=0.03, coarse_restart=32, coarse_max=500, n_post=8, stats=None):
    """The two-level K-cycle of oracle.mg on the rounded operators (input rounded first)."""
    r = round_to(r, rh.prec)
    rc = rh.restrict(r[None])
    ec, it_c, _ = krylov.gmres(rh.coarse_op, rc, None, restart=coarse_restart, max_iter=coarse_max, tol=coarse_tol)
    e = rh.prolong(ec)[0]
    e, it_s, _ = krylov.gmres(rh.D, r, e, restart=n_post, max_iter=n_post, tol=0.0)
    if stats is not None:
        stats["coarse"] += it_c
        stats["smoother"] += it_s
    return round_to(e, rh.prec)


def mixed_solve(h, b, prec, tol=1e-12, inner_tol=None, max_refine=40, max_inner=1000, restart=16):
    """FP64 defect correction around flexible GCR(restart) on the rounded D, preconditioned by
    the rounded K-cycle, each inner solve to inner_tol (default INNER_TOL[prec]) relative to its
    right-hand side.  Returns (x, stats) with the refinement count, the inner iterations and the
    true FP64 relative residual."""
    rh = RoundedHierarchy(h, prec)
    lat = h.lat
    it_tol = INNER_TOL[prec] if inner_tol is None else inner_tol
    bn = np.linalg.norm(b.ravel())
    x = np.zeros_like(b)
    stats = {"refinements": 0, "inner": [], "coarse": 0, "smoother": 0}
    for _ in range(max_refine):
        r = b - lat.D(x)
        rn = np.linalg.norm(r.ravel())
        if rn / bn <= tol:
            break
        e, it, _ = krylov.fgcr(rh.D, lambda v: kcycle(rh, v, stats=stats), round_to(r / rn, prec), None,
                               tol=it_tol, restart=restart, max_iter=max_inner)
        x = x + rn * e
        stats["refinements"] += 1
        stats["inner"].append(it)
    stats["true_rel_res"] = float(np.linalg.norm((b - lat.D(x)).ravel()) / bn)
    return x, stats


def operator_defect(h, prec, v):
    """||D_rounded v - D v|| / ||D v||: the relative error the stored format puts on one
    application of D (links and output rounded)."""
    rh = RoundedHierarchy(h, prec)
    d = h.lat.D(v)
    return float(np.linalg.norm((rh.D(v) - d).ravel()) / np.linalg.norm(d.ravel()))


__all__ = ["round_to", "RoundedHierarchy", "kcycle", "mixed_solve", "operator_defect", "INNER_TOL"]
