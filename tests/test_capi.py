"""CPU checks of the C ABI: the library loads, exports every function include/qmg.h declares,
and rejects invalid arguments before any device work (no GPU needed for these paths)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qmg.h")
LIB = os.path.join(ROOT, "paper_2505_14399_amd", "libqmg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qmg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libqmg.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("qmg_wilson_apply", "qmg_wilson_apply_adj", "qmg_mg_setup_stream_chiral_svd", "qmg_prolong",
                     "qmg_restrict", "qmg_coarse_apply", "qmg_mg_solve", "qmg_link_force"):
        assert required in names
    assert len(names) >= 20


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header(lib):
    import paper_2505_14399_amd as q
    assert set(declared_functions()) == set(q.SIGNATURES)
    q.load_library()
    assert q.version().startswith("qmg")


def _lat(dims=(4, 4, 4, 4), bc=-1, mass=0.1, xi=1.0):
    import paper_2505_14399_amd as q
    return q.Lattice(dims, mass, xi, bc).c()


def test_invalid_arguments_are_rejected_without_device_work():
    import paper_2505_14399_amd as q
    L = q.load_library()
    P = ctypes.c_void_p
    dummy = P(16)  # never dereferenced: validation fails first
    lat = _lat()
    # null pointers
    assert L.qmg_wilson_apply(ctypes.byref(lat), None, dummy, P(32), 1, q.F64, q.CANONICAL, None) == -1
    # aliasing
    assert L.qmg_wilson_apply(ctypes.byref(lat), dummy, P(32), P(32), 1, q.F64, q.CANONICAL, None) == -1
    # bad nrhs, bad precision, bad layout
    assert L.qmg_wilson_apply(ctypes.byref(lat), dummy, P(32), P(48), 0, q.F64, q.CANONICAL, None) == -1
    assert L.qmg_wilson_apply(ctypes.byref(lat), dummy, P(32), P(48), 1, 7, q.CANONICAL, None) == -1
    assert L.qmg_wilson_apply(ctypes.byref(lat), dummy, P(32), P(48), 1, q.F64, 5, None) == -1
    # bad lattice extents and boundary condition
    bad = _lat(dims=(4, 0, 4, 4))
    assert L.qmg_wilson_apply(ctypes.byref(bad), dummy, P(32), P(48), 1, q.F64, q.CANONICAL, None) == -2
    bad = _lat(bc=0)
    assert L.qmg_wilson_apply_adj(ctypes.byref(bad), dummy, P(32), P(48), 1, q.F64, q.CANONICAL, None) == -1
    assert b"bc_t" in L.qmg_last_error()
    # setup shape errors (block does not divide, batch / rank out of range)
    out = ctypes.c_void_p()
    for block, n_test, batch, rank in (((3, 2, 2, 2), 16, 4, 8), ((2, 2, 2, 2), 18, 4, 8),
                                       ((2, 2, 2, 2), 8, 4, 12), ((2, 2, 2, 2), 16, 0, 8),
                                       ((2, 2, 2, 2), 100, 50, 8), ((2, 2, 2, 2), 64, 16, 33)):
        p = q.qmg_mg_params()
        for i in range(4):
            p.block[i] = block[i]
        p.n_test, p.batch, p.rank = n_test, batch, rank
        p.n_setup_iter, p.n_post_smooth, p.coarse_tol, p.coarse_max_iter = 4, 8, 0.03, 100
        p.inner_prec = q.F64
        rc = L.qmg_mg_setup_stream_chiral_svd(ctypes.byref(lat), dummy, ctypes.byref(p), ctypes.byref(out), None)
        assert rc == -2, (block, n_test, batch, rank, rc)
        assert out.value is None
    # solve / transfer on a NULL handle
    assert L.qmg_mg_solve(None, dummy, P(32), 1, 1e-10, 10, 0, None, None) == -1
    assert L.qmg_prolong(None, dummy, P(32), 1, q.F64, None) == -1
    assert L.qmg_mg_query(None, None, None, None) == -1


def test_dslash_variant_codes_are_validated():
    import paper_2505_14399_amd as q
    L = q.load_library()
    try:
        for v in (0, 1, 2, 4, 8, 16, 32, 64, 202, 204, 208, 302, 304, 308, 1202, 1208, 1304, 10002, 10008, 11308,
                  501, 504, 700, 711, 744, 718, 781):
            assert L.qmg_set_dslash_variant(v) == 0, v
        for v in (-1, 3, 5, 100, 102, 108, 206, 402, 2204, 1102, 99999, 10001, 10016, 10032, 10501, 20008,
                  505, 701, 734, 770, 799, 10744):
            assert L.qmg_set_dslash_variant(v) == -1, v
    finally:
        assert L.qmg_set_dslash_variant(0) == 0


def test_hierarchy_file_errors_without_device_work(tmp_path):
    import paper_2505_14399_amd as q
    L = q.load_library()
    P = ctypes.c_void_p
    out = ctypes.c_void_p()
    dummy = P(16)  # never dereferenced: the file is rejected first
    missing = str(tmp_path / "missing.qmg").encode()
    assert L.qmg_mg_load(missing, dummy, ctypes.byref(out), None) == -1
    assert b"cannot open" in L.qmg_last_error()
    assert out.value is None
    bad = tmp_path / "bad.qmg"
    bad.write_bytes(b"NOTAHIER" + bytes(64))
    assert L.qmg_mg_load(str(bad).encode(), dummy, ctypes.byref(out), None) == -1
    assert b"not a hierarchy file" in L.qmg_last_error()
    short = tmp_path / "short.qmg"
    short.write_bytes(b"QMGHIER1" + (2).to_bytes(4, "little") + bytes(10))
    assert L.qmg_mg_load(str(short).encode(), dummy, ctypes.byref(out), None) == -1
    assert b"truncated" in L.qmg_last_error()
    old = tmp_path / "old.qmg"  # the first format had no clover coefficients
    old.write_bytes(b"QMGHIER1" + (1).to_bytes(4, "little") + bytes(200))
    assert L.qmg_mg_load(str(old).encode(), dummy, ctypes.byref(out), None) == -1
    assert b"unsupported hierarchy file version 1" in L.qmg_last_error()
    assert L.qmg_mg_load(str(bad).encode(), None, ctypes.byref(out), None) == -1
    assert L.qmg_mg_save(None, str(bad).encode(), None) == -1
    assert L.qmg_mg_stream_more(None, 1, None) == -1


def test_clover_arguments_are_rejected_without_device_work():
    import paper_2505_14399_amd as q
    L = q.load_library()
    P = ctypes.c_void_p
    D = ctypes.c_double
    dummy = P(16)  # never dereferenced: validation fails first
    lat = _lat()
    assert L.qmg_clover_field(ctypes.byref(lat), D(1.0), D(1.0), None, P(32), q.F64, None) == -1
    assert L.qmg_clover_field(ctypes.byref(lat), D(1.0), D(1.0), dummy, None, q.F64, None) == -1
    assert L.qmg_clover_field(ctypes.byref(lat), D(float("nan")), D(1.0), dummy, P(32), q.F64, None) == -1
    assert b"clover coefficients" in L.qmg_last_error()
    assert L.qmg_clover_field(ctypes.byref(lat), D(1.0), D(1.0), dummy, P(32), 9, None) == -1
    bad = _lat(dims=(4, 4, 0, 4))
    assert L.qmg_clover_field(ctypes.byref(bad), D(1.0), D(1.0), dummy, P(32), q.F64, None) == -2
    # apply: null site term, aliasing, nrhs, layout
    assert L.qmg_clover_apply(ctypes.byref(lat), dummy, None, P(32), P(48), 1, q.F64, q.CANONICAL, 0, None) == -1
    assert L.qmg_clover_apply(ctypes.byref(lat), dummy, P(24), P(32), P(32), 1, q.F64, q.CANONICAL, 0, None) == -1
    assert L.qmg_clover_apply(ctypes.byref(lat), dummy, P(24), P(32), P(48), 0, q.F64, q.CANONICAL, 0, None) == -1
    assert L.qmg_clover_apply(ctypes.byref(lat), dummy, P(24), P(32), P(48), 1, q.F64, 3, 0, None) == -1
    # setup with a non-finite clover coefficient
    p = q.qmg_mg_params()
    for i in range(4):
        p.block[i] = 2
    p.n_test, p.batch, p.rank = 8, 4, 4
    p.n_setup_iter, p.n_post_smooth, p.coarse_tol, p.coarse_max_iter = 4, 8, 0.03, 100
    p.inner_prec = q.F64
    p.c_sw_s, p.c_sw_t = 1.0, float("inf")
    out = ctypes.c_void_p()
    assert L.qmg_mg_setup_stream_chiral_svd(ctypes.byref(lat), dummy, ctypes.byref(p), ctypes.byref(out), None) == -1
    assert b"clover coefficients" in L.qmg_last_error() and out.value is None


def test_even_odd_arguments_are_rejected_without_device_work():
    import paper_2505_14399_amd as q
    L = q.load_library()
    P = ctypes.c_void_p
    D = ctypes.c_double
    dummy = P(16)  # never dereferenced: validation fails first
    lat = _lat()
    odd = _lat(dims=(4, 4, 3, 4))
    assert L.qmg_eo_pack_gauge(ctypes.byref(odd), dummy, P(32), q.F64, None) == -2
    assert b"every extent even" in L.qmg_last_error()
    assert L.qmg_eo_pack_gauge(ctypes.byref(lat), dummy, P(32), 7, None) == -1
    assert L.qmg_eo_pack_spinor(ctypes.byref(lat), dummy, P(32), None, 1, q.F64, None) == -1
    assert L.qmg_eo_unpack_spinor(ctypes.byref(lat), dummy, P(32), P(48), 0, q.F64, None) == -1
    assert L.qmg_eo_site_term(ctypes.byref(lat), D(1.0), D(float("inf")), dummy, P(32), P(48), q.F64, None) == -1
    # the Schur apply: aliasing, one of the two site-term fields missing, bad precision
    assert L.qmg_schur_apply(ctypes.byref(lat), dummy, None, None, P(32), P(32), 1, q.F64, 0, None) == -1
    assert L.qmg_schur_apply(ctypes.byref(lat), dummy, P(24), None, P(32), P(48), 1, q.F64, 0, None) == -1
    assert L.qmg_schur_apply(ctypes.byref(lat), dummy, None, None, P(32), P(48), 1, 9, 0, None) == -1
    # the solve: odd extent with eo, bad tolerance
    info = q.qmg_solve_info()
    assert L.qmg_eo_solve(ctypes.byref(odd), dummy, D(0.0), D(0.0), P(32), P(48), 1, D(1e-10), 100, 1,
                          ctypes.byref(info), None) == -2
    assert L.qmg_eo_solve(ctypes.byref(lat), dummy, D(0.0), D(0.0), P(32), P(48), 1, D(0.0), 100, 1,
                          ctypes.byref(info), None) == -1


def test_coarse_even_odd_arguments_are_rejected_without_device_work():
    import paper_2505_14399_amd as q
    L = q.load_library()
    P = ctypes.c_void_p
    D = ctypes.c_double
    it = ctypes.c_int32(0)
    assert L.qmg_mg_set_coarse_eo(None, 1, None) == -1
    assert L.qmg_coarse_schur_apply(None, P(32), P(48), 1, q.F64, None) == -1
    assert L.qmg_coarse_eo_solve(None, P(32), P(48), 1, D(1e-10), 100, ctypes.byref(it), None) == -1
    assert b"mg" in L.qmg_last_error()
