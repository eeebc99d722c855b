"""GPU parity of the even-odd (Schur complement) forms against oracle/evenodd.py: half-lattice
packing, the site term and its inverse, the Schur operator and its adjoint (Wilson and clover,
FP64 and FP32), and the preconditioned solve."""
import numpy as np
import pytest
import torch

import fields
from oracle import clover, evenodd, geometry as geo
from tests._util import to_gpu, to_np, rel, banner

pytestmark = pytest.mark.gpu


def _full(lat, qmg, even, odd=None):
    """Half fields -> canonical full-lattice array (decoding through the C ABI's unpack)."""
    odd = torch.zeros_like(even) if odd is None else odd
    return to_np(qmg.eo_unpack_spinor(lat, even, odd))


def _unpack_blocks(Ah, dims):
    """[2 parity][2 alpha][18][V/2] -> [V][2][6][6] (decoding only)."""
    Ah = to_np(Ah)
    V = int(np.prod(dims))
    par = evenodd.parity(dims)
    out = np.zeros((V, 2, 6, 6), dtype=np.complex128)
    for s_ in range(V):
        p, i = par[s_], s_ // 2
        for al in range(2):
            e18 = Ah[p, al, :, i]
            for e in range(3):
                out[s_, al, 2 * e, 2 * e] = e18[e].real
                out[s_, al, 2 * e + 1, 2 * e + 1] = e18[e].imag
            e = 3
            for a in range(6):
                for b in range(a + 1, 6):
                    out[s_, al, a, b] = e18[e]
                    out[s_, al, b, a] = np.conj(e18[e])
                    e += 1
    return out


def test_eo_packing_roundtrip(qmg):
    dims = (4, 6, 2, 8)
    banner(f"even-odd packing {dims}")
    lat = qmg.Lattice(dims, 0.1, 1.0, -1)
    psi = fields.gaussian_spinor(dims, 3, 41)
    e, o = qmg.eo_pack_spinor(lat, to_gpu(psi))
    assert np.array_equal(_full(lat, qmg, e, o), psi)
    par = evenodd.parity(dims)
    assert np.array_equal(_full(lat, qmg, e), evenodd.restrict_parity(psi, par, 0))
    U = fields.random_gauge(dims, 0.5, 42)
    Ueo = to_np(qmg.eo_pack_gauge(lat, to_gpu(U)))
    for s_ in (0, 1, 7, 100, geo.volume(dims) - 1):
        for mu in range(4):
            assert np.array_equal(Ueo[par[s_], mu, :, s_ // 2], U[mu, s_].ravel())


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_eo_site_term_and_inverse(qmg, prec, tol):
    dims = (4, 4, 2, 6)
    banner(f"even-odd site term {prec}")
    U = fields.random_gauge(dims, 0.7, 43)
    m, xi, cs, ct = -0.2, 2.0, 1.2, 0.8
    lat = qmg.Lattice(dims, m, xi, -1)
    A, Ai = qmg.eo_site_term(lat, to_gpu(U), cs, ct, prec)
    T = clover.clover_term(U, dims, cs, ct)
    ref = clover.chiral_blocks(clover.site_term(T, m, xi))
    assert rel(_unpack_blocks(A, dims), ref) < tol
    assert rel(_unpack_blocks(Ai, dims), np.linalg.inv(ref)) < tol * 10


CASES = [((4, 4, 4, 4), False, 0.05, 1.0), ((6, 4, 2, 8), True, -0.2, 2.0), ((4, 2, 4, 6), True, 0.1, 3.5)]


@pytest.mark.parametrize("dims,clov,m,xi", CASES)
@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_schur_apply_matches_oracle(qmg, dims, clov, m, xi, prec, tol):
    """Dhat and Dhat^dag on 1-3 right-hand sides against the oracle's Schur complement."""
    U = fields.random_gauge(dims, 0.6, 44)
    cs, ct = (1.1, 0.9) if clov else (0.0, 0.0)
    T = clover.clover_term(U, dims, cs, ct) if clov else None
    eo = evenodd.EvenOdd(U, dims, m, xi, -1, T)
    lat = qmg.Lattice(dims, m, xi, -1)
    Ueo = qmg.eo_pack_gauge(lat, to_gpu(U), prec)
    A, Ai = qmg.eo_site_term(lat, to_gpu(U), cs, ct, prec) if clov else (None, None)
    try:
        for form in (0, 1, 16):  # launcher's choice, one thread per site, direction split
            qmg.set_dslash_variant(form)
            for nrhs in (1, 3):
                x = fields.gaussian_spinor(dims, nrhs, 45 + nrhs)
                x_e = evenodd.restrict_parity(x, eo.par, 0)
                xe, _ = qmg.eo_pack_spinor(lat, to_gpu(x), prec)
                for dag in (False, True):
                    banner(f"schur {dims} clover={clov} {prec} form={form} nrhs={nrhs} dag={dag}")
                    got = _full(lat, qmg, qmg.schur_apply(lat, Ueo, xe, A, Ai, dagger=dag))
                    ref = eo.schur(x_e, dagger=dag)
                    assert rel(got, ref) < tol
    finally:
        qmg.set_dslash_variant(0)
    if not clov:  # the Wilson form without site-term fields equals the packed one
        Aw, Aiw = qmg.eo_site_term(lat, to_gpu(U), 0.0, 0.0, prec)
        a = qmg.schur_apply(lat, Ueo, xe, Aw, Aiw)
        b = qmg.schur_apply(lat, Ueo, xe)
        assert rel(to_np(a), to_np(b)) < tol


@pytest.mark.parametrize("dims", [(16, 32, 4, 8), (32, 16, 8, 4)])
def test_schur_apply_blocked_tile_orders(qmg, dims):
    """The hop's blocked (z, t) tile orders (launch-variant codes 7ZT) on lattices whose planes
    hold whole tiles: against the oracle's Schur complement, and bit for bit equal to the
    lexicographic order (700), since only the workgroup schedule changes; 1 to 4 right-hand
    sides (full groups of two per thread and a one-per-thread rest), Wilson and clover."""
    U = fields.random_gauge(dims, 0.6, 61)
    m, xi = -0.1, 1.5
    for clov in (False, True):
        cs, ct = (1.1, 0.9) if clov else (0.0, 0.0)
        T = clover.clover_term(U, dims, cs, ct) if clov else None
        eo = evenodd.EvenOdd(U, dims, m, xi, -1, T)
        lat = qmg.Lattice(dims, m, xi, -1)
        Ueo = qmg.eo_pack_gauge(lat, to_gpu(U), "f32")
        A, Ai = qmg.eo_site_term(lat, to_gpu(U), cs, ct, "f32") if clov else (None, None)
        for nrhs in (1, 3, 4):
            x = fields.gaussian_spinor(dims, nrhs, 62 + nrhs)
            xe, _ = qmg.eo_pack_spinor(lat, to_gpu(x), "f32")
            for dag in (False, True):
                ref = eo.schur(evenodd.restrict_parity(x, eo.par, 0), dagger=dag)
                base = None
                try:
                    for form in (700, 0, 711, 722, 744, 718, 781, 748):
                        banner(f"schur blocked order {dims} clover={clov} form={form} nrhs={nrhs} dag={dag}")
                        qmg.set_dslash_variant(form)
                        got = to_np(qmg.schur_apply(lat, Ueo, xe, A, Ai, dagger=dag))
                        if base is None:
                            base = got
                            assert rel(_full(lat, qmg, qmg.schur_apply(lat, Ueo, xe, A, Ai, dagger=dag)), ref) < 1e-6
                        assert np.array_equal(got, base), form
                finally:
                    qmg.set_dslash_variant(0)


@pytest.mark.parametrize("clov", [False, True])
def test_eo_solve(qmg, clov):
    """The preconditioned solve and the full-lattice GMRES reach 1e-10 in the oracle's residual,
    give the same solution, and the Schur system needs fewer iterations."""
    dims = (8, 8, 8, 8)
    banner(f"even-odd solve clover={clov}")
    U = fields.random_gauge(dims, 0.4, 47)
    m = 0.1
    c = (1.0, 1.0) if clov else None
    lat = qmg.Lattice(dims, m, 1.0, -1)
    b = fields.gaussian_spinor(dims, 2, 48)
    try:  # the one-site-per-thread form for the source and reconstruction forms too
        qmg.set_dslash_variant(1)
        x1, _ = qmg.eo_solve(lat, to_gpu(U), to_gpu(b), c_sw=c, tol=1e-10, eo=True)
    finally:
        qmg.set_dslash_variant(0)
    xe, ie = qmg.eo_solve(lat, to_gpu(U), to_gpu(b), c_sw=c, tol=1e-10, eo=True)
    assert rel(to_np(x1), to_np(xe)) < 1e-8
    xf, i_f = qmg.eo_solve(lat, to_gpu(U), to_gpu(b), c_sw=c, tol=1e-10, eo=False)
    print(f"[evenodd] clover={clov}: Schur {ie['outer_iters']} iterations ({ie['seconds']:.3f} s), "
          f"full {i_f['outer_iters']} ({i_f['seconds']:.3f} s)")
    T = clover.clover_term(U, dims, *c) if clov else np.zeros((geo.volume(dims), 12, 12), complex)
    for x in (xe, xf):
        r = b - clover.apply_clover(U, T, to_np(x), m, 1.0, -1, dims)
        assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-10
    assert rel(to_np(xe), to_np(xf)) < 1e-8
    assert ie["outer_iters"] < i_f["outer_iters"]


def test_eo_errors(qmg):
    dims = (4, 4, 4, 4)
    lat = qmg.Lattice(dims, 0.1, 1.0, -1)
    U = to_gpu(fields.random_gauge(dims, 0.5, 49))
    with pytest.raises(KeyError):
        qmg.eo_pack_gauge(lat, U, "fp8")
    b = to_gpu(fields.gaussian_spinor(dims, 1, 50))
    _, info = qmg.eo_solve(lat, U, b, tol=1e-12, max_iter=3, check=False)
    assert info["status"] != "OK" and info["outer_iters"] <= 3


@pytest.mark.parametrize("clov", [False, True])
def test_mg_even_odd_smoother_f64(qmg, clov):
    """FP64 K-cycle with the even-odd post-smoother: the solve to 1e-12 equals dense LU (D and
    D^dag); the captured device-exit cycle reproduces the eager one bit for bit."""
    dims, block = (4, 4, 4, 8), (2, 2, 2, 2)
    banner(f"MG even-odd smoother f64 clover={clov}")
    U = fields.random_gauge(dims, 0.3, 51)
    m = 0.05
    c = (1.0, 1.0) if clov else None
    lat = qmg.Lattice(dims, m, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 12, 4, 6, n_setup_iter=8, inner="f64", seed=3,
                                        c_sw=c)
    T = clover.clover_term(U, dims, *c) if clov else np.zeros((geo.volume(dims), 12, 12), complex)
    Dm = clover.dense_clover(U, T, m, 1.0, -1, dims)
    b = fields.gaussian_spinor(dims, 1, 52)
    _, i_plain = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
    mg.set_smoother(eo=True)
    x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
    print(f"[evenodd] MG f64 clover={clov}: even-odd smoother {info[0]['outer_iters']} outer, "
          f"plain {i_plain[0]['outer_iters']}")
    assert info[0]["true_rel_res"] <= 1e-12
    assert rel(to_np(x)[0], np.linalg.solve(Dm, b[0].ravel()).reshape(b[0].shape)) < 1e-8
    xa, _ = qmg.mg_solve(mg, to_gpu(b), tol=1e-12, adjoint=True)
    assert rel(to_np(xa)[0], np.linalg.solve(np.conj(Dm.T), b[0].ravel()).reshape(b[0].shape)) < 1e-8
    try:
        mg.set_cycle(12, graph=False)
        x_e, info_e = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
        mg.set_cycle(12, graph=True)
        x_g, info_g = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
    finally:
        mg.set_cycle(0, graph=False)
    assert info_e[0]["outer_iters"] == info_g[0]["outer_iters"] and torch.equal(x_e, x_g)
    mg.set_smoother(eo=False)
    _, i_back = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
    assert i_back[0]["outer_iters"] == i_plain[0]["outer_iters"]
    mg.close()


def test_mg_even_odd_smoother_mixed(qmg):
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    banner("MG even-odd smoother mixed f32")
    U = fields.random_gauge(dims, 0.4, 53)
    lat = qmg.Lattice(dims, 0.02, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 24, 8, 12, n_setup_iter=16, inner="f32", seed=3)
    b = fields.gaussian_spinor(dims, 2, 54)
    _, i_plain = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
    mg.set_smoother(eo=True)
    x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
    print(f"[evenodd] MG mixed: even-odd smoother {info[0]['outer_iters']} outer, plain {i_plain[0]['outer_iters']}")
    r = b - clover.apply_clover(U, np.zeros((geo.volume(dims), 12, 12), complex), to_np(x), 0.02, 1.0, -1, dims)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-10
    mg.close()


def test_mg_even_odd_smoother_errors(qmg):
    banner("MG even-odd smoother errors")
    dims = (4, 4, 4, 3)
    U = to_gpu(fields.random_gauge(dims, 0.3, 55))
    mg = qmg.mg_setup_stream_chiral_svd(qmg.Lattice(dims, 0.1, 1.0, -1), U, (2, 2, 2, 3), 8, 4, 4, n_setup_iter=2)
    with pytest.raises(qmg.QmgError, match="every extent even"):
        mg.set_smoother(eo=True)
    mg.close()
    dims = (4, 4, 4, 4)
    U = to_gpu(fields.random_gauge(dims, 0.3, 56))
    mg = qmg.mg_setup_stream_chiral_svd(qmg.Lattice(dims, 0.1, 1.0, -1), U, (2, 2, 2, 2), 8, 4, 4, n_setup_iter=2)
    with pytest.raises(qmg.QmgError, match="eo must be 0, 1 or 2"):
        qmg._check(qmg.load_library().qmg_mg_set_smoother(mg.handle, 3, None))
    mg.close()


@pytest.mark.parametrize("prec,tol", [("bf16", 1e-2), ("f16", 2e-3)])
@pytest.mark.parametrize("clov", [False, True])
def test_schur_apply_half_storage(qmg, prec, tol, clov):
    """BF16/FP16 storage with FP32 accumulation, both launch forms, against the oracle."""
    dims = (6, 4, 2, 8)
    U = fields.random_gauge(dims, 0.6, 57)
    m, xi = -0.2, 2.0
    cs, ct = (1.1, 0.9) if clov else (0.0, 0.0)
    T = clover.clover_term(U, dims, cs, ct) if clov else None
    eo = evenodd.EvenOdd(U, dims, m, xi, -1, T)
    lat = qmg.Lattice(dims, m, xi, -1)
    Ueo = qmg.eo_pack_gauge(lat, to_gpu(U), prec)
    A, Ai = qmg.eo_site_term(lat, to_gpu(U), cs, ct, prec) if clov else (None, None)
    x = fields.gaussian_spinor(dims, 2, 58)
    xe, _ = qmg.eo_pack_spinor(lat, to_gpu(x), prec)
    try:
        for form in (0, 1, 16):
            qmg.set_dslash_variant(form)
            for dag in (False, True):
                banner(f"schur {prec} clover={clov} form={form} dag={dag}")
                got = _full(lat, qmg, qmg.schur_apply(lat, Ueo, xe, A, Ai, dagger=dag))
                assert rel(got, eo.schur(evenodd.restrict_parity(x, eo.par, 0), dagger=dag)) < tol
    finally:
        qmg.set_dslash_variant(0)


@pytest.mark.parametrize("inner", ["bf16", "f16"])
def test_mg_even_odd_smoother_half_storage(qmg, inner):
    """Half-storage K-cycle with the even-odd smoother: the solve reaches 1e-10 in the oracle's
    residual."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    banner(f"MG even-odd smoother {inner}")
    U = fields.random_gauge(dims, 0.4, 59)
    lat = qmg.Lattice(dims, 0.02, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 24, 8, 12, n_setup_iter=16, inner=inner, seed=3)
    b = fields.gaussian_spinor(dims, 1, 60)
    _, i_plain = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
    mg.set_smoother(eo=True)
    x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
    print(f"[evenodd] MG {inner}: even-odd smoother {info[0]['outer_iters']} outer, plain {i_plain[0]['outer_iters']}")
    r = b - clover.apply_clover(U, np.zeros((geo.volume(dims), 12, 12), complex), to_np(x), 0.02, 1.0, -1, dims)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-10
    mg.close()


@pytest.mark.parametrize("clov", [False, True])
def test_mg_sstep_smoother(qmg, clov):
    """The s-step form of the even-odd smoother: FP64 solve equals dense LU (D and D^dag), the
    captured cycle equals the eager one, and it takes about the outer iterations of the GMRES
    form; the mixed FP32 and BF16 K-cycles reach 1e-10 in the oracle's residual."""
    dims, block = (4, 4, 4, 8), (2, 2, 2, 2)
    banner(f"MG s-step smoother clover={clov}")
    U = fields.random_gauge(dims, 0.3, 61)
    m = 0.05
    c = (1.0, 1.0) if clov else None
    lat = qmg.Lattice(dims, m, 1.0, -1)
    mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 12, 4, 6, n_setup_iter=8, inner="f64", seed=3,
                                        c_sw=c)
    T = clover.clover_term(U, dims, *c) if clov else np.zeros((geo.volume(dims), 12, 12), complex)
    Dm = clover.dense_clover(U, T, m, 1.0, -1, dims)
    b = fields.gaussian_spinor(dims, 1, 62)
    mg.set_smoother(eo=True)
    _, i_gm = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
    mg.set_smoother(eo=True, sstep=True)
    x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
    print(f"[evenodd] MG f64 clover={clov}: s-step {info[0]['outer_iters']} outer, GMRES form {i_gm[0]['outer_iters']}")
    assert info[0]["true_rel_res"] <= 1e-12
    assert info[0]["outer_iters"] <= i_gm[0]["outer_iters"] + 2
    assert rel(to_np(x)[0], np.linalg.solve(Dm, b[0].ravel()).reshape(b[0].shape)) < 1e-8
    xa, _ = qmg.mg_solve(mg, to_gpu(b), tol=1e-12, adjoint=True)
    assert rel(to_np(xa)[0], np.linalg.solve(np.conj(Dm.T), b[0].ravel()).reshape(b[0].shape)) < 1e-8
    try:
        mg.set_cycle(12, graph=False)
        x_e, info_e = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
        mg.set_cycle(12, graph=True)
        x_g, info_g = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
    finally:
        mg.set_cycle(0, graph=False)
    assert info_e[0]["outer_iters"] == info_g[0]["outer_iters"] and torch.equal(x_e, x_g)
    mg.close()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = fields.random_gauge(dims, 0.4, 63)
    lat = qmg.Lattice(dims, 0.02, 1.0, -1)
    T = clover.clover_term(U, dims, *c) if clov else np.zeros((geo.volume(dims), 12, 12), complex)
    for inner in ("f32", "bf16"):
        mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(U), block, 24, 8, 12, n_setup_iter=16, inner=inner, seed=3,
                                            c_sw=c)
        mg.set_smoother(eo=True, sstep=True)
        b = fields.gaussian_spinor(dims, 2, 64)
        x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-10)
        print(f"[evenodd] MG {inner} clover={clov}: s-step {info[0]['outer_iters']} outer")
        r = b - clover.apply_clover(U, T, to_np(x), 0.02, 1.0, -1, dims)
        assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-10
        mg.close()


def test_mg_even_odd_smoother_non_su3_links(qmg):
    """Links that are not SU(3) (scaled by 1.01) keep all nine entries in the smoother's
    half-lattice field (the third row cannot be rebuilt): the s-step and Gram-Schmidt forms still
    solve to the dense LU solution; SU(3) links (two stored rows) give the same solution too."""
    dims, block = (4, 4, 4, 8), (2, 2, 2, 2)
    banner("MG even-odd smoother, non-SU(3) links")
    U = fields.random_gauge(dims, 0.3, 65)
    b = fields.gaussian_spinor(dims, 1, 66)
    for scale in (1.0, 1.01):
        Us = U * scale
        lat = qmg.Lattice(dims, 0.1, 1.0, -1)
        mg = qmg.mg_setup_stream_chiral_svd(lat, to_gpu(Us), block, 12, 4, 6, n_setup_iter=8, inner="f64", seed=3)
        Dm = clover.dense_clover(Us, np.zeros((geo.volume(dims), 12, 12), complex), 0.1, 1.0, -1, dims)
        xd = np.linalg.solve(Dm, b[0].ravel()).reshape(b[0].shape)
        for ss in (False, True):
            mg.set_smoother(eo=True, sstep=ss)
            x, info = qmg.mg_solve(mg, to_gpu(b), tol=1e-12)
            assert info[0]["true_rel_res"] <= 1e-12 and rel(to_np(x)[0], xd) < 1e-8, (scale, ss, info[0])
        mg.close()
