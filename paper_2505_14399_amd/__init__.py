"""Python binding of libqmg: streaming chiral-SVD multigrid for Wilson fermions on MI355X.

Argument marshalling only: every step of the computation runs in the HIP kernels of
libqmg.so (include/qmg.h).  Device memory and streams come from PyTorch; the library must
be built (``python -m paper_2505_14399_amd.build``) and fails loudly if it is missing.

Names follow the C ABI without the ``qmg_`` prefix.  Tensors are CUDA (HIP) tensors in the
canonical layouts of qmg.h: gauge [4][V][3][3], spinor [nrhs][V][4][3] (chiral basis),
coarse [nrhs][d][2][k]; complex128 is QMG_F64 and complex64 QMG_F32.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmg.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
CANONICAL, NATIVE = 0, 1
_PREC = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}

STATUS = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "EDTYPE", -4: "ENOMEM", -5: "EHIP",
          -6: "ENOCONV", -7: "EBREAKDOWN", -8: "ENONFINITE", -9: "ENOTIMPL"}


class QmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qmg {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class qmg_lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("bc_t", ctypes.c_int32),
                ("mass", ctypes.c_double), ("xi", ctypes.c_double)]


class qmg_mg_params(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32 * 4), ("n_test", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("rank", ctypes.c_int32), ("n_setup_iter", ctypes.c_int32), ("n_post_smooth", ctypes.c_int32),
                ("coarse_tol", ctypes.c_double), ("coarse_max_iter", ctypes.c_int32),
                ("inner_prec", ctypes.c_int32), ("seed", ctypes.c_uint64), ("test_vectors", ctypes.c_void_p),
                ("c_sw_s", ctypes.c_double), ("c_sw_t", ctypes.c_double)]


class qmg_solve_info(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("coarse_iters", ctypes.c_int32), ("smoother_iters", ctypes.c_int32),
                ("precision_escalations", ctypes.c_int32), ("true_rel_res", ctypes.c_double),
                ("seconds", ctypes.c_double), ("coarse2_iters", ctypes.c_int32),
                ("smoother1_iters", ctypes.c_int32), ("coarse3_iters", ctypes.c_int32),
                ("smoother2_iters", ctypes.c_int32)]


# exported symbols and their argument types (void* = device or host pointer, see qmg.h)
_P, _I, _D, _U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64
SIGNATURES = {
    "qmg_wilson_apply": [_P, _P, _P, _P, _I, _I, _I, _P],
    "qmg_wilson_apply_adj": [_P, _P, _P, _P, _I, _I, _I, _P],
    "qmg_wilson_apply_batched": [_I, _P, _P, _P, _P, _I, _I, _I, _P],
    "qmg_clover_field": [_P, _D, _D, _P, _P, _I, _P],
    "qmg_clover_apply": [_P, _P, _P, _P, _P, _I, _I, _I, _I, _P],
    "qmg_eo_pack_gauge": [_P, _P, _P, _I, _P],
    "qmg_eo_pack_spinor": [_P, _P, _P, _P, _I, _I, _P],
    "qmg_eo_unpack_spinor": [_P, _P, _P, _P, _I, _I, _P],
    "qmg_eo_site_term": [_P, _D, _D, _P, _P, _P, _I, _P],
    "qmg_schur_apply": [_P, _P, _P, _P, _P, _P, _I, _I, _I, _P],
    "qmg_eo_solve": [_P, _P, _D, _D, _P, _P, _I, _D, _I, _I, _P, _P],
    "qmg_mg_set_smoother": [_P, _I, _P],
    "qmg_mg_set_coarse_eo": [_P, _I, _P],
    "qmg_coarse_schur_apply": [_P, _P, _P, _I, _I, _P],
    "qmg_coarse_schur_apply_noalloc": [_P, _P, _P, _I, _I, _P],
    "qmg_coarse_eo_solve": [_P, _P, _P, _I, _D, _I, _P, _P],
    "qmg_pack_spinor": [_P, _P, _P, _I, _I, _P],
    "qmg_unpack_spinor": [_P, _P, _P, _I, _I, _P],
    "qmg_pack_gauge": [_P, _P, _P, _I, _P],
    "qmg_mg_setup_stream_chiral_svd": [_P, _P, _P, _P, _P],
    "qmg_prolong": [_P, _P, _P, _I, _I, _P],
    "qmg_restrict": [_P, _P, _P, _I, _I, _P],
    "qmg_coarse_apply": [_P, _P, _P, _I, _I, _P],
    "qmg_mg_solve": [_P, _P, _P, _I, _D, _I, _I, _P, _P],
    "qmg_link_force": [_P, _P, _P, _P, _I, _P],
    "qmg_random_test_vectors": [_P, _U64, _I, _I, _P, _P],
    "qmg_smooth": [_P, _P, _P, _P, _I, _I, _I, _P],
    "qmg_mg_query": [_P, _P, _P, _P],
    "qmg_mg_get_prolongator": [_P, _P, _P, _P],
    "qmg_mg_get_coarse": [_P, _P, _P],
    "qmg_mg_setup_times": [_P, _P],
    "qmg_timing_enable": [_I],
    "qmg_timing_query": [ctypes.c_char_p, _P, _P, _P, _P],
    "qmg_timing_calls": [ctypes.c_char_p, _P],
    "qmg_timing_list": [ctypes.c_char_p, _I],
    "qmg_memory_trim": [],
    "qmg_memory_cached": [_P],
    "qmg_mg_set_cycle": [_P, _I, _I],
    "qmg_autotune": [_I],
    "qmg_set_dslash_variant": [_I],
    "qmg_tune_save": [ctypes.c_char_p],
    "qmg_tune_load": [ctypes.c_char_p],
    "qmg_mg_stream_more": [_P, _I, _P],
    "qmg_mg_add_level": [_P, _P, _I, _I, _I, _I, ctypes.c_uint64, _P],
    "qmg_mg_set_level_tol": [_P, _I, ctypes.c_double],
    "qmg_mg_level_query": [_P, _I, _P, _P, _P],
    "qmg_mg_level_get": [_P, _I, _P, _P, _P, _P],
    "qmg_level_prolong": [_P, _I, _P, _P, _I, _I, _P],
    "qmg_level_restrict": [_P, _I, _P, _P, _I, _I, _P],
    "qmg_level_coarse_apply": [_P, _I, _P, _P, _I, _I, _P],
    "qmg_mg_save": [_P, ctypes.c_char_p, _P],
    "qmg_mg_load": [ctypes.c_char_p, _P, _P, _P],
    "qmg_mg_get_params": [_P, _P, _P],
    "qmg_mg_destroy": [_P],
    "qmg_batch_setup": [_I, _P, _P, _P, _P, _P],
    "qmg_batch_solve": [_P, _P, _P, _I, _D, _I, _P, _P],
    "qmg_batch_query": [_P, _I, _P, _P],
    "qmg_batch_get_prolongator": [_P, _I, _P, _P, _P],
    "qmg_batch_get_coarse": [_P, _I, _P, _P],
    "qmg_batch_setup_times": [_P, _P],
    "qmg_batch_destroy": [_P],
    "qmg_last_error": [],
    "qmg_version": [],
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libqmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libqmg.so not found at {path}: build it with "
                           "`python -m paper_2505_14399_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    lib.qmg_last_error.restype = ctypes.c_char_p
    lib.qmg_version.restype = ctypes.c_char_p
    lib.qmg_mg_destroy.restype = None
    lib.qmg_batch_destroy.restype = None
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise QmgError(rc, _lib.qmg_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _prec_of(t: torch.Tensor) -> int:
    if t.dtype == torch.complex128:
        return F64
    if t.dtype == torch.complex64:
        return F32
    if t.dtype == torch.bfloat16 and t.shape[-1] == 2:
        return BF16
    if t.dtype == torch.float16 and t.shape[-1] == 2:
        return F16
    raise TypeError(f"unsupported dtype {t.dtype}")


@dataclass
class Lattice:
    """Eq. (1)'s lattice problem: extents (Lx, Ly, Lz, Lt), time BC, mass, anisotropy."""
    dims: Sequence[int]
    mass: float
    xi: float = 1.0
    bc_t: int = -1

    @property
    def volume(self):
        v = 1
        for L in self.dims:
            v *= int(L)
        return v

    def c(self):
        s = qmg_lattice()
        for i in range(4):
            s.dims[i] = int(self.dims[i])
        s.bc_t = int(self.bc_t)
        s.mass = float(self.mass)
        s.xi = float(self.xi)
        return s


def _apply(fn, lat, U, psi, layout, out):
    lib = load_library()
    prec = _prec_of(psi)
    if _prec_of(U) != prec:
        raise TypeError("U and psi must have the same precision")
    nrhs = psi.shape[0]
    out = torch.empty_like(psi) if out is None else out
    s = lat.c()
    _check(getattr(lib, fn)(ctypes.byref(s), _ptr(U), _ptr(psi), _ptr(out), nrhs, prec,
                            CANONICAL if layout == "canonical" else NATIVE, _stream()))
    return out


def wilson_apply(lat: Lattice, U, psi, layout="canonical", out=None):
    """out = D psi.  Canonical: U [4,V,3,3], psi [nrhs,V,4,3]; native: [4,9,V], [nrhs,12,V]."""
    return _apply("qmg_wilson_apply", lat, U, psi, layout, out)


def wilson_apply_adj(lat: Lattice, U, psi, layout="canonical", out=None):
    """out = D^dagger psi."""
    return _apply("qmg_wilson_apply_adj", lat, U, psi, layout, out)


def wilson_apply_batched(lats: Sequence[Lattice], Us, psis, outs=None, dagger=False):
    """out_i = D_i psi_i (D_i^dagger if dagger) for many lattices in one launch.

    Native layout only: Us[i] [4,9,V_i], psis[i] [nrhs,12,V_i] (same precision and nrhs for all).
    """
    lib = load_library()
    n = len(lats)
    if not (len(Us) == len(psis) == n) or n == 0:
        raise ValueError("need one gauge field and one spinor block per lattice")
    prec = _prec_of(psis[0])
    nrhs = psis[0].shape[0]
    for U, p in zip(Us, psis):
        if _prec_of(U) != prec or _prec_of(p) != prec or p.shape[0] != nrhs:
            raise TypeError("all lattices need the same precision and number of right-hand sides")
    outs = [torch.empty_like(p) for p in psis] if outs is None else list(outs)
    arr = (qmg_lattice * n)(*[l.c() for l in lats])
    ptrs = torch.tensor([[_ptr(t).value for t in grp] for grp in (Us, psis, outs)], dtype=torch.int64,
                        device=psis[0].device)
    _check(lib.qmg_wilson_apply_batched(n, arr, ctypes.c_void_p(ptrs[0].data_ptr()),
                                        ctypes.c_void_p(ptrs[1].data_ptr()), ctypes.c_void_p(ptrs[2].data_ptr()),
                                        nrhs, prec, 1 if dagger else 0, _stream()))
    # the pointer table must outlive the launch: keep it until the stream has passed it
    torch.cuda.current_stream().synchronize()
    return outs


def clover_field(lat: Lattice, U, c_sw_s, c_sw_t=None, prec="f64"):
    """The packed site term (m + 1 + 3/xi) + T(x) of the Wilson-clover operator (see qmg.h:
    qmg_clover_field) from the canonical complex128 gauge field U [4,V,3,3]: [2,18,V] in `prec`
    (BF16/FP16: [2,18,V,2] real pairs).  c_sw_t defaults to c_sw_s (the isotropic term)."""
    lib = load_library()
    if U.dtype != torch.complex128:
        raise TypeError("the clover field is built from the FP64 canonical gauge field")
    p = _PREC[prec]
    shape = (2, 18, lat.volume, 2) if p in (BF16, F16) else (2, 18, lat.volume)
    out = torch.empty(shape, dtype=_dtype_of(p), device=U.device)
    s = lat.c()
    ct = c_sw_s if c_sw_t is None else c_sw_t
    _check(lib.qmg_clover_field(ctypes.byref(s), float(c_sw_s), float(ct), _ptr(U), _ptr(out), p, _stream()))
    return out


def clover_apply(lat: Lattice, U, A, psi, layout="canonical", dagger=False, out=None):
    """out = D_sw psi (D_sw^dagger psi if dagger): U and psi as in wilson_apply, A from
    clover_field in the same precision."""
    lib = load_library()
    prec = _prec_of(psi)
    if _prec_of(U) != prec or _prec_of(A) != prec:
        raise TypeError("U, A and psi must have the same precision")
    nrhs = psi.shape[0]
    out = torch.empty_like(psi) if out is None else out
    s = lat.c()
    _check(lib.qmg_clover_apply(ctypes.byref(s), _ptr(U), _ptr(A), _ptr(psi), _ptr(out), nrhs, prec,
                                CANONICAL if layout == "canonical" else NATIVE, 1 if dagger else 0, _stream()))
    return out


def _eo_prec(prec):
    return _PREC[prec]


def _eo_shape(shape, p):
    """BF16/FP16 fields carry complex numbers as a trailing pair of reals."""
    return tuple(shape) + ((2,) if p in (BF16, F16) else ())


def eo_pack_gauge(lat: Lattice, U64, prec="f64"):
    """canonical complex128 [4,V,3,3] -> half-lattice gauge [2,4,9,V/2] (parity, mu, entry, site)."""
    p = _eo_prec(prec)
    out = torch.empty(_eo_shape((2, 4, 9, lat.volume // 2), p), dtype=_dtype_of(p), device=U64.device)
    s = lat.c()
    _check(load_library().qmg_eo_pack_gauge(ctypes.byref(s), _ptr(U64), _ptr(out), p, _stream()))
    return out


def eo_pack_spinor(lat: Lattice, psi64, prec="f64"):
    """canonical complex128 [nrhs,V,4,3] -> (even, odd) half fields [nrhs,12,V/2]."""
    p = _eo_prec(prec)
    nrhs = psi64.shape[0]
    even = torch.empty(_eo_shape((nrhs, 12, lat.volume // 2), p), dtype=_dtype_of(p), device=psi64.device)
    odd = torch.empty_like(even)
    s = lat.c()
    _check(load_library().qmg_eo_pack_spinor(ctypes.byref(s), _ptr(psi64), _ptr(even), _ptr(odd), nrhs, p,
                                             _stream()))
    return even, odd


def eo_unpack_spinor(lat: Lattice, even, odd):
    p = _prec_of(even)
    nrhs = even.shape[0]
    out = torch.empty((nrhs, lat.volume, 4, 3), dtype=torch.complex128, device=even.device)
    s = lat.c()
    _check(load_library().qmg_eo_unpack_spinor(ctypes.byref(s), _ptr(even), _ptr(odd), _ptr(out), nrhs, p,
                                               _stream()))
    return out


def eo_site_term(lat: Lattice, U, c_sw_s=0.0, c_sw_t=None, prec="f64"):
    """(A_eo, Ainv_eo) [2,2,18,V/2]: the packed site term of D_sw (Wilson for zero coefficients)
    and its inverse in the half-lattice layout."""
    p = _eo_prec(prec)
    A = torch.empty(_eo_shape((2, 2, 18, lat.volume // 2), p), dtype=_dtype_of(p), device=U.device)
    Ai = torch.empty_like(A)
    s = lat.c()
    ct = c_sw_s if c_sw_t is None else c_sw_t
    _check(load_library().qmg_eo_site_term(ctypes.byref(s), float(c_sw_s), float(ct), _ptr(U), _ptr(A), _ptr(Ai), p,
                                           _stream()))
    return A, Ai


def schur_apply(lat: Lattice, U_eo, x_e, A_eo=None, Ainv_eo=None, dagger=False, out=None):
    """out_e = Dhat x_e (Dhat^dagger with dagger) on even half fields [nrhs,12,V/2]."""
    prec = _prec_of(x_e)
    out = torch.empty_like(x_e) if out is None else out
    s = lat.c()
    _check(load_library().qmg_schur_apply(ctypes.byref(s), _ptr(U_eo), _ptr(A_eo), _ptr(Ainv_eo), _ptr(x_e),
                                          _ptr(out), x_e.shape[0], prec, 1 if dagger else 0, _stream()))
    return out


def eo_solve(lat: Lattice, U, b, c_sw=None, tol=1e-10, max_iter=20000, eo=True, check=True):
    """x = D^-1 b by FP64 GMRES(32), on the even-odd Schur complement (eo) or on the full
    operator; c_sw: None (Wilson), a number or (c_sw_s, c_sw_t).  Returns (x, info)."""
    cs, ct = (0.0, 0.0) if c_sw is None else ((c_sw, c_sw) if isinstance(c_sw, (int, float)) else c_sw)
    x = torch.empty_like(b)
    info = qmg_solve_info()
    s = lat.c()
    rc = load_library().qmg_eo_solve(ctypes.byref(s), _ptr(U), float(cs), float(ct), _ptr(b), _ptr(x), b.shape[0],
                                     float(tol), int(max_iter), 1 if eo else 0, ctypes.byref(info), _stream())
    out = {f: getattr(info, f) for f, _ in qmg_solve_info._fields_}
    out["status"] = STATUS.get(rc, str(rc))
    if check:
        _check(rc)
    return x, out


def _native_spinor_shape(nrhs, V, prec):
    if prec in (BF16, F16):
        return (nrhs, 12, V, 2)
    return (nrhs, 12, V)


def _dtype_of(prec):
    return {F64: torch.complex128, F32: torch.complex64, BF16: torch.bfloat16, F16: torch.float16}[prec]


def pack_spinor(lat: Lattice, psi64, prec="f64"):
    """canonical complex128 [nrhs,V,4,3] -> native [nrhs,12,V] in `prec`."""
    lib = load_library()
    p = _PREC[prec]
    nrhs = psi64.shape[0]
    out = torch.empty(_native_spinor_shape(nrhs, lat.volume, p), dtype=_dtype_of(p), device=psi64.device)
    s = lat.c()
    _check(lib.qmg_pack_spinor(ctypes.byref(s), _ptr(psi64), _ptr(out), nrhs, p, _stream()))
    return out


def unpack_spinor(lat: Lattice, native, prec="f64"):
    lib = load_library()
    p = _PREC[prec]
    nrhs = native.shape[0]
    out = torch.empty((nrhs, lat.volume, 4, 3), dtype=torch.complex128, device=native.device)
    s = lat.c()
    _check(lib.qmg_unpack_spinor(ctypes.byref(s), _ptr(native), _ptr(out), nrhs, p, _stream()))
    return out


def pack_gauge(lat: Lattice, U64, prec="f64"):
    """canonical complex128 [4,V,3,3] -> native [4,9,V] in `prec`."""
    lib = load_library()
    p = _PREC[prec]
    shape = (4, 9, lat.volume, 2) if p in (BF16, F16) else (4, 9, lat.volume)
    out = torch.empty(shape, dtype=_dtype_of(p), device=U64.device)
    s = lat.c()
    _check(lib.qmg_pack_gauge(ctypes.byref(s), _ptr(U64), _ptr(out), p, _stream()))
    return out


class MG:
    """A two-level hierarchy built by mg_setup_stream_chiral_svd (owns the C handle)."""

    def __init__(self, handle, lat, params):
        self._h = handle
        self.lat = lat
        self.params = params
        cd = (ctypes.c_int32 * 4)()
        d = ctypes.c_int32()
        k = ctypes.c_int32()
        _check(load_library().qmg_mg_query(self._h, cd, ctypes.byref(d), ctypes.byref(k)))
        self.coarse_dims = tuple(cd)
        self.n_agg = d.value
        self.rank = k.value
        self.inner = {v: n for n, v in _PREC.items()}[params.inner_prec]
        self.levels = {}  # further levels l >= 2: dims, n_agg, rank, block

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load_library().qmg_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prolongator(self):
        """(P [d,2,N,k] complex128 on the GPU, canonical row order 6*site+3*spin+colour; sigma [d,2,k])."""
        import numpy as np
        N = 6 * int(torch.tensor(self.params.block[:]).prod())
        P = torch.empty((self.n_agg, 2, N, self.rank), dtype=torch.complex128, device="cuda")
        sig = np.empty((self.n_agg, 2, self.rank))
        _check(load_library().qmg_mg_get_prolongator(self._h, _ptr(P), sig.ctypes.data_as(ctypes.c_void_p),
                                                     _stream()))
        return P, sig

    def coarse_blocks(self):
        m = 2 * self.rank
        Y = torch.empty((self.n_agg, 9, m, m), dtype=torch.complex128, device="cuda")
        _check(load_library().qmg_mg_get_coarse(self._h, _ptr(Y), _stream()))
        return Y

    def set_cycle(self, coarse_steps=0, graph=False):
        """K-cycle form: coarse_steps > 0 gives a device-exit coarse solve with that step budget;
        graph=True captures the cycle into a hipGraph replayed at every application."""
        _check(load_library().qmg_mg_set_cycle(self._h, int(coarse_steps), 1 if graph else 0))

    def set_smoother(self, eo=False, sstep=False):
        """Even-odd (eo=True) or plain GMRES post-smoothing on the fine level; with sstep the
        even-odd GMRES steps run in s-step form (see qmg.h)."""
        _check(load_library().qmg_mg_set_smoother(self._h, (2 if sstep else 1) if eo else 0, _stream()))

    def set_coarse_eo(self, on=True):
        """Coarse solve of the K-cycle on the even-odd Schur complement of D_c (on) or on D_c
        (see qmg.h, qmg_mg_set_coarse_eo)."""
        _check(load_library().qmg_mg_set_coarse_eo(self._h, 1 if on else 0, _stream()))

    def stream_more(self, n_streams):
        """Resume the streaming SVD with n_streams more batches of test vectors (the counter RNG's
        next global indices), then rebuild P, R and D_c."""
        _check(load_library().qmg_mg_stream_more(self._h, int(n_streams), _stream()))
        self._refresh()

    def add_level(self, block, n_test, batch, rank, n_setup_iter=16, seed=None):
        """One more level on the current coarsest operator (qmg_mg_add_level): level 2 on D_c,
        then level 3; the solve then recurses over all levels.  Returns the new level's index."""
        blk = (ctypes.c_int32 * 4)(*[int(b) for b in block])
        seed = self.params.seed if seed is None else int(seed)
        _check(load_library().qmg_mg_add_level(self._h, blk, int(n_test), int(batch), int(rank), int(n_setup_iter),
                                               ctypes.c_uint64(seed), _stream()))
        lvl = 2 + len(self.levels)
        cd = (ctypes.c_int32 * 4)()
        d = ctypes.c_int32()
        k = ctypes.c_int32()
        _check(load_library().qmg_mg_level_query(self._h, lvl, cd, ctypes.byref(d), ctypes.byref(k)))
        self.levels[lvl] = {"dims": tuple(cd), "n_agg": d.value, "rank": k.value,
                            "block": tuple(int(b) for b in block)}
        return lvl

    def set_level_tol(self, level, tol):
        """Relative tolerance of the Krylov solve on level >= 2 (0: the coarse tolerance)."""
        _check(load_library().qmg_mg_set_level_tol(self._h, int(level), float(tol)))

    def _above(self, level):
        """(n_agg, rank) of the level above `level`."""
        if level == 2:
            return self.n_agg, self.rank
        a = self.levels[level - 1]
        return a["n_agg"], a["rank"]

    # level 2 (the third level) shorthands
    @property
    def level_dims(self):
        return self.levels[2]["dims"]

    @property
    def level_n_agg(self):
        return self.levels[2]["n_agg"]

    @property
    def level_rank(self):
        return self.levels[2]["rank"]

    def level_prolongator(self, level=2):
        """(P_l [d_l,2,N_l,k_l] complex128 on the GPU, rows site-in-block * k_above + i; sigma_l [d_l,2,k_l])."""
        import numpy as np
        L = self.levels[level]
        N = self._above(level)[1] * int(np.prod(L["block"]))
        P = torch.empty((L["n_agg"], 2, N, L["rank"]), dtype=torch.complex128, device="cuda")
        sig = np.empty((L["n_agg"], 2, L["rank"]))
        _check(load_library().qmg_mg_level_get(self._h, level, _ptr(P), sig.ctypes.data_as(ctypes.c_void_p), None,
                                               _stream()))
        return P, sig

    def level_coarse_blocks(self, level=2):
        L = self.levels[level]
        m = 2 * L["rank"]
        Y = torch.empty((L["n_agg"], 9, m, m), dtype=torch.complex128, device="cuda")
        _check(load_library().qmg_mg_level_get(self._h, level, None, None, _ptr(Y), _stream()))
        return Y

    def save(self, path):
        """Write the hierarchy (parameters, singular values, P in FP64) to a file."""
        _check(load_library().qmg_mg_save(self._h, os.fsencode(str(path)), _stream()))

    def _refresh(self):
        lat, p = qmg_lattice(), qmg_mg_params()
        _check(load_library().qmg_mg_get_params(self._h, ctypes.byref(lat), ctypes.byref(p)))
        self.params = p

    @property
    def streams_done(self):
        return self.params.n_test // self.params.batch

    def setup_times(self):
        t = (ctypes.c_double * 4)()
        _check(load_library().qmg_mg_setup_times(self._h, t))
        return {"smooth": t[0], "svd": t[1], "coarse": t[2], "total": t[3]}


def mg_setup_stream_chiral_svd(lat: Lattice, U, block, n_test, batch, rank, n_setup_iter=16, n_post_smooth=8,
                               coarse_tol=0.03, coarse_max_iter=500, inner="f64", seed=0, test_vectors=None,
                               c_sw=None) -> MG:
    """Algorithm 4 with Algorithm 3 (see qmg.h).  U: complex128 [4,V,3,3] on the GPU.
    c_sw: None (Wilson), a number (isotropic clover term) or (c_sw_s, c_sw_t)."""
    lib = load_library()
    if U.dtype != torch.complex128:
        raise TypeError("setup takes the FP64 canonical gauge field")
    p = qmg_mg_params()
    for i in range(4):
        p.block[i] = int(block[i])
    p.n_test, p.batch, p.rank = int(n_test), int(batch), int(rank)
    p.n_setup_iter, p.n_post_smooth = int(n_setup_iter), int(n_post_smooth)
    p.coarse_tol, p.coarse_max_iter = float(coarse_tol), int(coarse_max_iter)
    p.inner_prec = _PREC[inner]
    p.seed = int(seed)
    p.test_vectors = None if test_vectors is None else _ptr(test_vectors).value
    if c_sw is not None:
        cs, ct = (c_sw, c_sw) if isinstance(c_sw, (int, float)) else c_sw
        p.c_sw_s, p.c_sw_t = float(cs), float(ct)
    h = ctypes.c_void_p()
    s = lat.c()
    _check(lib.qmg_mg_setup_stream_chiral_svd(ctypes.byref(s), _ptr(U), ctypes.byref(p), ctypes.byref(h), _stream()))
    return MG(h, lat, p)


class Batch:
    """Multigrid hierarchies of many small lattices built and solved together (qmg_batch_*)."""

    def __init__(self, handle, lats, params):
        self._h = handle
        self.lats = list(lats)
        self.params = params

    def close(self):
        if self._h:
            load_library().qmg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, lat):
        d, k = ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().qmg_batch_query(self._h, int(lat), ctypes.byref(d), ctypes.byref(k)))
        return d.value, k.value

    def prolongator(self, lat):
        """(P [d,2,N,k] complex128 on the GPU in the canonical row order, sigma [d,2,k]) of lattice lat."""
        import numpy as np
        d, k = self.query(lat)
        N = 6 * int(torch.tensor(self.params.block[:]).prod())
        P = torch.empty((d, 2, N, k), dtype=torch.complex128, device="cuda")
        sig = np.empty((d, 2, k))
        _check(load_library().qmg_batch_get_prolongator(self._h, int(lat), _ptr(P), sig.ctypes.data_as(ctypes.c_void_p),
                                                        _stream()))
        return P, sig

    def coarse_blocks(self, lat):
        d, k = self.query(lat)
        Y = torch.empty((d, 9, 2 * k, 2 * k), dtype=torch.complex128, device="cuda")
        _check(load_library().qmg_batch_get_coarse(self._h, int(lat), _ptr(Y), _stream()))
        return Y

    def setup_times(self):
        t = (ctypes.c_double * 4)()
        _check(load_library().qmg_batch_setup_times(self._h, t))
        return {"smooth": t[0], "svd": t[1], "coarse": t[2], "total": t[3]}


def batch_setup(lats: Sequence[Lattice], Us, block, n_test, batch, rank, n_setup_iter=16, n_post_smooth=8,
                coarse_tol=0.03, coarse_max_iter=500, inner="f32", seed=0) -> Batch:
    """Hierarchies of many lattices at once (qmg_batch_setup).  Us: complex128 [4,V_l,3,3] per lattice."""
    lib = load_library()
    n = len(lats)
    if len(Us) != n or n == 0:
        raise ValueError("need one gauge field per lattice")
    for U in Us:
        if U.dtype != torch.complex128:
            raise TypeError("setup takes FP64 canonical gauge fields")
    p = qmg_mg_params()
    for i in range(4):
        p.block[i] = int(block[i])
    p.n_test, p.batch, p.rank = int(n_test), int(batch), int(rank)
    p.n_setup_iter, p.n_post_smooth = int(n_setup_iter), int(n_post_smooth)
    p.coarse_tol, p.coarse_max_iter = float(coarse_tol), int(coarse_max_iter)
    p.inner_prec = _PREC[inner]
    p.seed = int(seed)
    arr = (qmg_lattice * n)(*[l.c() for l in lats])
    ptrs = (ctypes.c_void_p * n)(*[_ptr(U).value for U in Us])
    h = ctypes.c_void_p()
    _check(lib.qmg_batch_setup(n, arr, ptrs, ctypes.byref(p), ctypes.byref(h), _stream()))
    return Batch(h, lats, p)


def batch_solve(bt: Batch, bs, tol=1e-10, max_outer=1000, check=True):
    """x_l = D_l^-1 b_l for every lattice: bs complex128 [nrhs,V_l,4,3] per lattice.  Returns (xs, info)
    with info a list (per lattice) of lists (per right-hand side) of dicts."""
    n = len(bt.lats)
    nrhs = int(bs[0].shape[0])
    xs = [torch.empty_like(b) for b in bs]
    infos = (qmg_solve_info * (n * nrhs))()
    bp = (ctypes.c_void_p * n)(*[_ptr(b).value for b in bs])
    xp = (ctypes.c_void_p * n)(*[_ptr(x).value for x in xs])
    rc = load_library().qmg_batch_solve(bt._h, bp, xp, nrhs, float(tol), int(max_outer), infos, _stream())
    out = [[{f: getattr(infos[l * nrhs + r], f) for f, _ in qmg_solve_info._fields_} for r in range(nrhs)]
           for l in range(n)]
    if check:
        _check(rc)
    return xs, out


def mg_load(path, U) -> MG:
    """Rebuild a hierarchy saved by MG.save for the gauge field U (complex128 [4,V,3,3] on the
    GPU; it must be the field the hierarchy was built for)."""
    lib = load_library()
    if U.dtype != torch.complex128:
        raise TypeError("load takes the FP64 canonical gauge field")
    h = ctypes.c_void_p()
    _check(lib.qmg_mg_load(os.fsencode(str(path)), _ptr(U), ctypes.byref(h), _stream()))
    cl, p = qmg_lattice(), qmg_mg_params()
    _check(lib.qmg_mg_get_params(h, ctypes.byref(cl), ctypes.byref(p)))
    lat = Lattice(tuple(cl.dims), cl.mass, cl.xi, cl.bc_t)
    return MG(h, lat, p)


def level_prolong(mg: MG, v2, out=None, level=2):
    """P_l v2: level-l vectors [nrhs,d_l,2,k_l] -> level-(l-1) vectors (complex128, or complex64 with FP32 inner)."""
    nrhs = v2.shape[0]
    d1, k1 = mg._above(level)
    out = torch.empty((nrhs, d1, 2, k1), dtype=v2.dtype, device=v2.device) if out is None else out
    _check(load_library().qmg_level_prolong(mg.handle, level, _ptr(v2), _ptr(out), nrhs, _prec_of(v2), _stream()))
    return out


def level_restrict(mg: MG, v1, out=None, level=2):
    """P_l^dag v1: level-(l-1) vectors -> level-l vectors [nrhs,d_l,2,k_l]."""
    nrhs = v1.shape[0]
    L = mg.levels[level]
    out = (torch.empty((nrhs, L["n_agg"], 2, L["rank"]), dtype=v1.dtype, device=v1.device)
           if out is None else out)
    _check(load_library().qmg_level_restrict(mg.handle, level, _ptr(v1), _ptr(out), nrhs, _prec_of(v1), _stream()))
    return out


def level_coarse_apply(mg: MG, v2, out=None, level=2):
    """A_l v2 on level-l vectors [nrhs,d_l,2,k_l]."""
    nrhs = v2.shape[0]
    out = torch.empty_like(v2) if out is None else out
    _check(load_library().qmg_level_coarse_apply(mg.handle, level, _ptr(v2), _ptr(out), nrhs, _prec_of(v2),
                                                 _stream()))
    return out


def _coarse_prec(t):
    return _prec_of(t)


def prolong(mg: MG, vc, out=None):
    """fine = P vc; vc [nrhs,d,2,k] complex128 (FP64 P) or complex64 (inner FP32 P)."""
    p = _prec_of(vc)
    nrhs = vc.shape[0]
    out = torch.empty((nrhs, mg.lat.volume, 4, 3), dtype=vc.dtype, device=vc.device) if out is None else out
    _check(load_library().qmg_prolong(mg.handle, _ptr(vc), _ptr(out), nrhs, p, _stream()))
    return out


def restrict(mg: MG, psi, out=None):
    """coarse = P^dagger psi; psi [nrhs,V,4,3]."""
    p = _prec_of(psi)
    nrhs = psi.shape[0]
    out = torch.empty((nrhs, mg.n_agg, 2, mg.rank), dtype=psi.dtype, device=psi.device) if out is None else out
    _check(load_library().qmg_restrict(mg.handle, _ptr(psi), _ptr(out), nrhs, p, _stream()))
    return out


def coarse_apply(mg: MG, v, out=None):
    """out = D_c v; v [nrhs,d,2,k]."""
    p = _prec_of(v)
    out = torch.empty_like(v) if out is None else out
    _check(load_library().qmg_coarse_apply(mg.handle, _ptr(v), _ptr(out), v.shape[0], p, _stream()))
    return out


def coarse_schur_apply(mg: MG, v_e, out=None):
    """out_e = Dhat_c v_e on half coarse vectors [nrhs,d/2,2,k] of the even aggregates."""
    p = _prec_of(v_e)
    out = torch.empty_like(v_e) if out is None else out
    _check(load_library().qmg_coarse_schur_apply(mg.handle, _ptr(v_e), _ptr(out), v_e.shape[0], p, _stream()))
    return out


def coarse_schur_apply_noalloc(mg: MG, v_e, out):
    """out_e = Dhat_c v_e like coarse_schur_apply, with the library's fixed scratch array instead
    of an allocated intermediate (no device allocation, no stream synchronisation): `out` must be
    given; calls that overlap on one device race (see qmg.h)."""
    p = _prec_of(v_e)
    _check(load_library().qmg_coarse_schur_apply_noalloc(mg.handle, _ptr(v_e), _ptr(out), v_e.shape[0], p,
                                                         _stream()))
    return out


def coarse_eo_solve(mg: MG, b, tol=1e-12, max_iter=5000):
    """x = D_c^-1 b (FP64, [nrhs,d,2,k]) by GMRES(32) on the even-odd Schur complement; returns
    (x, GMRES steps)."""
    x = torch.empty_like(b)
    it = ctypes.c_int32(0)
    _check(load_library().qmg_coarse_eo_solve(mg.handle, _ptr(b), _ptr(x), b.shape[0], float(tol), int(max_iter),
                                              ctypes.byref(it), _stream()))
    return x, it.value


def mg_solve(mg: MG, b, x0=None, tol=1e-10, max_outer=1000, adjoint=False, check=True):
    """Solve D x = b (D^dagger x = b if adjoint) to true FP64 relative residual tol.

    Returns (x, info) with info a list of dicts per right-hand side.  With check=False a
    non-convergence status is returned in info instead of raised.
    """
    nrhs = b.shape[0]
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    infos = (qmg_solve_info * nrhs)()
    rc = load_library().qmg_mg_solve(mg.handle, _ptr(b), _ptr(x), nrhs, float(tol), int(max_outer),
                                     1 if adjoint else 0, infos, _stream())
    out = [{f: getattr(i, f) for f, _ in qmg_solve_info._fields_} for i in infos]
    for o in out:
        o["status"] = STATUS.get(rc, str(rc))
    if check:
        _check(rc)
    return x, out


def link_force(lat: Lattice, x, lam, out=None):
    """Gradient of sum Re<eta, D^-1 b> w.r.t. the links from x = D^-1 b, lam = D^-dag eta."""
    out = torch.empty((4, lat.volume, 3, 3), dtype=torch.complex128, device=x.device) if out is None else out
    s = lat.c()
    _check(load_library().qmg_link_force(ctypes.byref(s), _ptr(x), _ptr(lam), _ptr(out), x.shape[0], _stream()))
    return out


def random_test_vectors(lat: Lattice, seed, v0, n):
    out = torch.empty((n, lat.volume, 4, 3), dtype=torch.complex128, device="cuda")
    s = lat.c()
    _check(load_library().qmg_random_test_vectors(ctypes.byref(s), int(seed), int(v0), int(n), _ptr(out),
                                                  _stream()))
    return out


def smooth(lat: Lattice, U, phi, n_iter, prec="f64"):
    """Eq. (2) smoothing of test vectors phi (canonical complex128), computed in `prec`."""
    out = torch.empty_like(phi)
    s = lat.c()
    _check(load_library().qmg_smooth(ctypes.byref(s), _ptr(U), _ptr(phi), _ptr(out), phi.shape[0], int(n_iter),
                                     _PREC[prec], _stream()))
    return out


def timing_enable(on=True, every=1):
    """Start (clearing the record; every `every`-th launch of each family is timed) or stop
    per-launch HIP-event timing of the kernel families."""
    _check(load_library().qmg_timing_enable(int(every) if on else 0))


def timing_query(family):
    """{'launches', 'ms', 'bytes', 'flops'} summed over the timed launches of `family`, and 'calls'
    (every launch since timing was enabled)."""
    n = ctypes.c_int64()
    ms, by, fl = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().qmg_timing_query(family.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                           ctypes.byref(fl)))
    calls = ctypes.c_int64()
    _check(load_library().qmg_timing_calls(family.encode(), ctypes.byref(calls)))
    return {"launches": n.value, "ms": ms.value, "bytes": by.value, "flops": fl.value, "calls": calls.value}


def timing_families():
    """Names of every kernel family launched since timing_enable."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load_library().qmg_timing_list(buf, len(buf)))
    return [f for f in buf.value.decode().split("\n") if f]


def memory_trim():
    """Return the library's cached device blocks to the runtime (see qmg.h)."""
    _check(load_library().qmg_memory_trim())


def memory_cached():
    """Bytes of device memory held by the library's cache on the current device."""
    n = ctypes.c_int64()
    _check(load_library().qmg_memory_cached(ctypes.byref(n)))
    return n.value


def autotune(on=True):
    """Enable (or disable) per-shape timing of kernel launch variants on first use."""
    _check(load_library().qmg_autotune(1 if on else 0))


def set_dslash_variant(v=0):
    """Force a native dslash launch variant (1, 2, 4, 8, 16, 32, 64, or a multi-RHS t-walking
    code 1000 z + 100 NR + TCH) or restore the automatic choice (0)."""
    _check(load_library().qmg_set_dslash_variant(int(v)))


def tune_save(path):
    _check(load_library().qmg_tune_save(os.fspath(path).encode()))


def tune_load(path):
    _check(load_library().qmg_tune_load(os.fspath(path).encode()))


def version():
    return load_library().qmg_version().decode()
