// C ABI of libqmg (qmg.h): validation, the multigrid setup driver (Algorithm 4 with
// Algorithm 3), the K-cycle preconditioner and the mixed-precision MG solve.
#include <chrono>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstdarg>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>
#include <type_traits>

#include "mg.hpp"
#include "timing.hpp"
#include "tune.hpp"

struct qmg_mg {
  qmg::HierarchyDev h;
  qmg::DevBuf sigma_dev;
  qmg_lattice lat{};        // as given to the setup
  qmg_mg_params params{};   // as given to the setup (test_vectors cleared after it)
  int streams_done = 0;     // streams of the streaming SVD applied so far
  int kp = 0;               // columns of the current factor U_k
};

namespace qmg {

namespace {
thread_local char g_err[1024] = "";
}

const char* last_error_ptr() { return g_err; }

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

Geom make_geom(const qmg_lattice* lat) {
  Geom g{};
  int64_t V = 1;
  for (int m = 0; m < 4; ++m) {
    QMG_CHECK(lat->dims[m] >= 1, QMG_ESHAPE, "lattice extent %d is %d (must be >= 1)", m, lat->dims[m]);
    g.L[m] = lat->dims[m];
    V *= lat->dims[m];
  }
  QMG_CHECK(V < (int64_t(1) << 31), QMG_ESHAPE, "lattice volume %lld too large", (long long)V);
  QMG_CHECK(lat->bc_t == 1 || lat->bc_t == -1, QMG_EINVAL, "bc_t must be +1 or -1");
  QMG_CHECK(std::isfinite(lat->mass) && std::isfinite(lat->xi) && lat->xi > 0, QMG_EINVAL,
            "mass must be finite and xi positive");
  g.V = int(V);
  g.bc_t = lat->bc_t;
  g.mass = lat->mass;
  g.xi = lat->xi;
  return g;
}

namespace {

using Clock = std::chrono::steady_clock;
double secs(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

void check_prec(qmg_prec p) {
  QMG_CHECK(p == QMG_F64 || p == QMG_F32 || p == QMG_BF16 || p == QMG_F16, QMG_EINVAL, "bad precision %d", int(p));
}

// ---------------------------------------------------------------------------------------
// operators
// the fine operator: Wilson, or Wilson-clover when A (the packed site term in precision p) is set
struct WilsonOp : LinOp {
  Geom g;
  qmg_prec p;
  const void* U;
  const void* A;
  WilsonOp(const Geom& g_, qmg_prec p_, const void* U_, const void* A_) : g(g_), p(p_), U(U_), A(A_) {}
  void apply(const void* in, void* out, int nrhs, hipStream_t st, const int* = nullptr) override {
    DslashArgs a = make_dslash_args(g, nrhs, false, false);
    a.clov = A;
    launch_dslash(p, U, in, out, a, st);
  }
  size_t len() const override { return size_t(12) * g.V; }
  qmg_prec prec() const override { return p; }
};

// the even-odd Schur complement Dhat = A_ee - D_eo A_oo^-1 D_oe (Dhat^dag with dag) on even
// half fields; tmp holds the odd intermediate
struct SchurOp : LinOp {
  Geom g;
  qmg_prec p;
  const void *Ue, *Uo, *Ae, *Ao, *Aie, *Aio;
  bool dag;
  int ne;  // complex entries per stored link: 9, or 6 (two rows of SU(3) links)
  DevBuf tmp;
  SchurOp(const Geom& g_, qmg_prec p_, const void* Ueo, const void* Aeo, const void* Ainv, bool dag_, int ne_ = 9)
      : g(g_), p(p_), dag(dag_), ne(ne_) {
    const size_t half = size_t(36) * (g.V / 2) * prec_bytes(p);  // one parity's packed block
    Ue = Ueo;
    Uo = static_cast<const char*>(Ueo) + size_t(4) * ne * (g.V / 2) * prec_bytes(p);  // one parity's links
    Ae = Aeo;
    Ao = Aeo ? static_cast<const char*>(Aeo) + half : nullptr;
    Aie = Ainv;
    Aio = Ainv ? static_cast<const char*>(Ainv) + half : nullptr;
  }
  void apply(const void* in, void* out, int nrhs, hipStream_t st, const int* = nullptr) override {
    tmp.ensure(size_t(nrhs) * len() * prec_bytes(p));
    DslashArgs a = make_dslash_args(g, nrhs, dag, false);
    a.link_ne = ne;
    launch_hop_eo(p, a, Ue, Uo, 1, in, nullptr, tmp.p, nullptr, Aio, 0, 1, 1.0, st);  // A_oo^-1 D_oe in
    launch_hop_eo(p, a, Ue, Uo, 0, tmp.p, in, out, Ae, nullptr, 2, 0, -1.0, st);      // A_ee in - D_eo (...)
  }
  size_t len() const override { return size_t(12) * (g.V / 2); }
  qmg_prec prec() const override { return p; }
};

struct CoarseOp : LinOp {
  const HierarchyDev& h;
  qmg_prec p;
  const void* Y;
  CoarseOp(const HierarchyDev& h_, qmg_prec p_, const void* Y_) : h(h_), p(p_), Y(Y_) {}
  void apply(const void* in, void* out, int nrhs, hipStream_t st, const int* skip = nullptr) override {
    launch_coarse_apply(p, h, Y, in, out, nrhs, st, skip);
  }
  size_t len() const override { return size_t(2) * h.k * h.blk.d; }
  qmg_prec prec() const override { return p; }
};

// even-odd Schur complement of D_c on half coarse vectors [nrhs][d/2][2k] of the even colour:
// Y_ee v - Y_eo (Y_oo^-1 Y_oe v), the bracket with the Yhat blocks of the odd aggregates
struct CoarseSchurOp : LinOp {
  const HierarchyDev& h;
  qmg_prec p;
  const void* Y;
  const void* Yh;
  DevBuf tmp;
  CoarseSchurOp(const HierarchyDev& h_, qmg_prec p_, const void* Y_, const void* Yh_) : h(h_), p(p_), Y(Y_), Yh(Yh_) {}
  void apply(const void* in, void* out, int nrhs, hipStream_t st, const int* = nullptr) override {
    tmp.ensure(size_t(nrhs) * len() * prec_bytes(p));
    launch_coarse_eo_apply(p, h, 1, Yh, nullptr, nullptr, in, tmp.p, nrhs, 1.0, st);
    launch_coarse_eo_apply(p, h, 0, Y, nullptr, in, tmp.p, out, nrhs, -1.0, st);
  }
  size_t len() const override { return size_t(h.k) * h.blk.d; }
  qmg_prec prec() const override { return p; }
};

// D_c v = r through the Schur complement: rhat_e = r_e - Y_eo Y_oo^-1 r_o, GMRES(32) on
// Dhat_c v_e = rhat_e to tol (relative to rhat_e) within max_iter steps, v_o = Y_oo^-1 (r_o -
// Y_oe v_e).  r, v: full coarse vectors; work: six half vectors.  Returns the GMRES result.
template <class S>
typename Gmres<S>::Result coarse_eo_solve(const HierarchyDev& h, CoarseSchurOp& A, Gmres<S>& gm, const void* r,
                                          void* v, int nrhs, int max_iter, double tol, DevBuf* work, hipStream_t st,
                                          int hint = 0) {
  constexpr qmg_prec p = StoreTraits<S>::prec;
  const size_t nh = size_t(nrhs) * A.len();
  for (int i = 0; i < 6; ++i) work[i].ensure(nh * sizeof(S));
  void *re = work[0].p, *ro = work[1].p, *w = work[2].p, *rh = work[3].p, *ve = work[4].p, *vo = work[5].p;
  launch_coarse_eo_split(p, h, r, re, ro, nrhs, st);
  launch_coarse_eo_apply(p, h, 1, A.Yh, nullptr, ro, nullptr, w, nrhs, 1.0, st);  // Y_oo^-1 r_o
  launch_coarse_eo_apply(p, h, 0, A.Y, re, nullptr, w, rh, nrhs, -1.0, st);       // rhat_e
  auto res = gm.solve(A, rh, ve, true, nrhs, 32, max_iter, tol, st, nullptr, hint);
  launch_coarse_eo_apply(p, h, 1, A.Yh, nullptr, ro, ve, vo, nrhs, -1.0, st);     // v_o
  launch_coarse_eo_merge(p, h, ve, vo, v, nrhs, st);
  return res;
}

// the nine-block stencil of a further level
struct StencilOp : LinOp {
  int d, k;
  const int* cnb;
  qmg_prec p;
  const void* Y;
  StencilOp(int d_, int k_, const int* cnb_, qmg_prec p_, const void* Y_) : d(d_), k(k_), cnb(cnb_), p(p_), Y(Y_) {}
  void apply(const void* in, void* out, int nrhs, hipStream_t st, const int* skip = nullptr) override {
    launch_stencil_apply(p, d, k, cnb, Y, in, out, nrhs, st, skip);
  }
  size_t len() const override { return size_t(2) * k * d; }
  qmg_prec prec() const override { return p; }
};

// K-cycle of a coarse level l >= 1 when a further level exists (storage precision S): restrict
// to level l + 1 (h.levels[i], i = l - 1), solve there to the coarse tolerance (GMRES(32) on the
// coarsest level, else flexible GMRES(32) preconditioned by the K-cycle of level l + 1), prolong,
// GMRES post-smoothing on level l (`above`) from the prolonged correction.
template <class S>
struct KCycleC : Precond {
  const HierarchyDev& h;
  const CoarseLevel& L;
  const int d1;
  LinOp& above;
  StencilOp own;
  const void* P2;
  Gmres<S> g2, gs;
  DevBuf r2, e2;
  std::unique_ptr<KCycleC<S>> next;
  long coarse_iters = 0, smooth_iters = 0;  // Krylov iterations on level l + 1, smoothing on level l
  int last = 0;
  KCycleC(const HierarchyDev& h_, size_t i, LinOp& above_)
      : h(h_), L(*h_.levels[i]), d1(stencil_above(h_, i).d), above(above_),
        own(L.d, L.k, L.cnb.as<int>(), StoreTraits<S>::prec, StoreTraits<S>::prec == QMG_F64 ? L.Y64.p : L.Yin.p),
        P2(StoreTraits<S>::prec == QMG_F64 ? L.P64.p : L.Pin.p) {
    if (i + 1 < h.levels.size()) next.reset(new KCycleC<S>(h, i + 1, own));
  }
  void apply(const void* r1, void* z1, int nrhs, hipStream_t st) override {
    constexpr qmg_prec p = StoreTraits<S>::prec;
    const size_t n2 = size_t(nrhs) * 2 * L.k * L.d;
    r2.ensure(n2 * sizeof(S));
    e2.ensure(n2 * sizeof(S));
    launch_level_restrict(p, L, d1, P2, r1, r2.p, nrhs, st);
    const int hint = last > 1 ? last - 1 : 0;
    const double tol2 = L.tol > 0 ? L.tol : h.coarse_tol;
    auto res = g2.solve(own, r2.p, e2.p, true, nrhs, 32, h.coarse_max, tol2, st, nullptr, hint, next.get());
    coarse_iters += res.iters;
    last = res.iters;
    launch_level_prolong(p, L, d1, P2, e2.p, z1, nrhs, st);
    gs.solve(above, r1, z1, false, nrhs, std::max(1, h.n_post), h.n_post, 0.0, st);
    smooth_iters += h.n_post;
  }
};

// Two-level K-cycle with storage precision S; r and z are in the outer solver's type F.
// Eager form: restrict, coarse GMRES to the tolerance (the host reads its convergence
// estimates every few steps), prolong, fixed-length GMRES post-smoothing.  With a coarse step
// budget (h.cycle_steps > 0) the coarse solve is one device-exit cycle (convergence tested and
// acted on by the kernels themselves), so the whole cycle has no host round trip; with
// h.cycle_graph it is then captured once into a hipGraph on a private stream and replayed.
template <class F, class S>
struct KCycle : Precond {
  const HierarchyDev& h;
  WilsonOp& D;
  CoarseOp& Dc;
  const void* P;
  Gmres<S> gc, gf;
  DevBuf rc, ec, rS, zS, conv;
  std::unique_ptr<KCycleC<S>> Kc;  // level-one K-cycle when a third level exists
  std::unique_ptr<SchurOp> schur;  // even-odd post-smoother: the Schur complement and its buffers
  std::unique_ptr<CoarseSchurOp> cschur;  // even-odd coarse solve: the coarse Schur complement
  Gmres<S> gce;
  DevBuf ceo_work[6];
  DevBuf eo_t, eo_e, eo_o, eo_u, eo_b, eo_xe, eo_xo, eo_basis, eo_c, eo_part;
  long coarse_iters = 0, smooth_iters = 0, cycles = 0;
  int last_coarse = 0;             // coarse steps of the previous cycle (host-checked form)
  hipStream_t gs = nullptr;        // private stream of the captured cycle
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_nrhs = 0;
  KCycle(const HierarchyDev& h_, WilsonOp& D_, CoarseOp& Dc_, const void* P_) : h(h_), D(D_), Dc(Dc_), P(P_) {}
  ~KCycle() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gs) (void)hipStreamDestroy(gs);
  }
  // restrict -> coarse solve -> prolong -> post-smoothing, on storage-precision buffers
  void body(const void* r_s, void* z_s, int nrhs, hipStream_t st) {
    constexpr qmg_prec p = StoreTraits<S>::prec;
    launch_restrict(p, h, P, r_s, rc.p, nrhs, st);
    if (!h.levels.empty()) {
      // further levels: flexible GMRES(32) on D_c preconditioned by the level-one K-cycle
      if (!Kc) Kc.reset(new KCycleC<S>(h, 0, Dc));
      const int hint = last_coarse > 1 ? last_coarse - 1 : 0;
      auto rcs = gc.solve(Dc, rc.p, ec.p, true, nrhs, 32, h.coarse_max, h.coarse_tol, st, nullptr, hint, Kc.get());
      coarse_iters += rcs.iters;
      last_coarse = rcs.iters;
    } else if (h.cycle_steps > 0) {
      gc.solve(Dc, rc.p, ec.p, true, nrhs, h.cycle_steps, h.cycle_steps, h.coarse_tol, st, conv.as<int>());
    } else if (h.coarse_eo) {
      // the coarse solve on the even-odd Schur complement of D_c
      if (!cschur) cschur.reset(new CoarseSchurOp(h, p, Dc.Y, p == QMG_F64 ? h.Yh64.p : h.Yhin.p));
      const int hint = last_coarse > 1 ? last_coarse - 1 : 0;
      auto rcs = coarse_eo_solve<S>(h, *cschur, gce, rc.p, ec.p, nrhs, h.coarse_max, h.coarse_tol, ceo_work, st, hint);
      coarse_iters += rcs.iters;
      last_coarse = rcs.iters;
    } else {
      // first read of the convergence estimates one step before the previous cycle's count
      const int hint = last_coarse > 1 ? last_coarse - 1 : 0;
      auto rcs = gc.solve(Dc, rc.p, ec.p, true, nrhs, 32, h.coarse_max, h.coarse_tol, st, nullptr, hint);
      coarse_iters += rcs.iters;
      last_coarse = rcs.iters;
    }
    launch_prolong(p, h, P, ec.p, z_s, nrhs, st);
    if (h.eo_smoother)
      eo_smooth(r_s, z_s, nrhs, st);
    else
      gf.solve(D, r_s, z_s, false, nrhs, std::max(1, h.n_post), h.n_post, 0.0, st);
    smooth_iters += h.n_post;
  }
  // even-odd post-smoothing: t = r - D z, then n_post GMRES steps from zero on the Schur system
  // of t (Dhat e_e = t_e - D_eo A_oo^-1 t_o), e_o = A_oo^-1 (t_o - D_oe e_e), z += e
  void eo_smooth(const void* r_s, void* z_s, int nrhs, hipStream_t st) {
    constexpr qmg_prec p = StoreTraits<S>::prec;
    const int w = p == QMG_F64 ? 0 : 1;
    const size_t nf = size_t(nrhs) * 12 * h.g.V, nh = nf / 2;
    eo_t.ensure(nf * sizeof(S));
    for (DevBuf* b : {&eo_e, &eo_o, &eo_u, &eo_b, &eo_xe, &eo_xo}) b->ensure(nh * sizeof(S));
    if (!schur) schur.reset(new SchurOp(h.g, p, h.Ueo[w].p, h.Aeo[w].p, h.Aieo[w].p, false, h.eo_ne));
    D.apply(z_s, eo_t.p, nrhs, st);
    launch_eo_split_sub(p, h.g, r_s, eo_t.p, eo_e.p, eo_o.p, nrhs, st);  // t = r - D z by parity
    DslashArgs a = make_dslash_args(h.g, nrhs, false, false);
    a.link_ne = h.eo_ne;
    launch_site_eo(p, a, schur->Aio, true, eo_o.p, eo_u.p, st);
    const int ns = std::max(1, h.n_post);
    const bool sstep = h.eo_smoother == 2 && ns <= 8;
    const size_t L = size_t(12) * (h.g.V / 2);
    if (sstep) eo_basis.ensure(size_t(ns + 1) * nh * sizeof(S));
    // the Schur source goes straight into the first basis vector of the s-step form
    void* bsrc = sstep ? eo_basis.p : eo_b.p;
    launch_hop_eo(p, a, schur->Ue, schur->Uo, 0, eo_u.p, eo_e.p, bsrc, nullptr, nullptr, 1, 0, -1.0, st);
    if (sstep) {
      // the same minimisation as GMRES(ns) from zero, over the basis b, Dhat b, ..., Dhat^ns b:
      // one pass of inner products and an FP64 normal-equation solve on the device instead of
      // ns Gram-Schmidt steps; x_e = sum_j c_j p_j in one pass without clearing x_e first
      eo_c.ensure(size_t(ns) * nrhs * sizeof(double2));
      auto vec = [&](int i) { return static_cast<char*>(eo_basis.p) + size_t(i) * nh * sizeof(S); };
      for (int i = 0; i < ns; ++i) schur->apply(vec(i), vec(i + 1), nrhs, st);
      launch_sstep_coeffs(p, eo_basis.p, ns + 1, L, nrhs, eo_c.as<double2>(), eo_part, st);
      sstep_update<S>(eo_basis.p, nh, ns, eo_c.as<double2>(), 0.0, eo_xe.p, nullptr, L, nrhs, false, false, st);
    } else {
      gf.solve(*schur, eo_b.p, eo_xe.p, true, nrhs, ns, h.n_post, 0.0, st);
    }
    launch_hop_eo(p, a, schur->Ue, schur->Uo, 1, eo_xe.p, eo_o.p, eo_xo.p, nullptr, schur->Aio, 1, 1, -1.0, st);
    launch_eo_merge_add(p, h.g, eo_xe.p, eo_xo.p, z_s, nrhs, st);
  }
  void apply(const void* r, void* z, int nrhs, hipStream_t st) override {
    const size_t nc = size_t(nrhs) * 2 * h.k * h.blk.d;
    const size_t nf = size_t(nrhs) * 12 * h.g.V;
    rc.ensure(nc * sizeof(S));
    ec.ensure(nc * sizeof(S));
    if (!conv.p) {
      conv.alloc(4 * sizeof(int));
      QMG_HIP(hipMemsetAsync(conv.p, 0, 4 * sizeof(int), st));  // outside any capture
    }
    constexpr qmg_prec p = StoreTraits<S>::prec;
    constexpr qmg_prec pf = StoreTraits<F>::prec;
    constexpr bool same = std::is_same<F, S>::value;
    ++cycles;
    if (!h.cycle_graph) {
      const void* r_s = r;
      void* z_s = z;
      if (!same) {
        rS.ensure(nf * sizeof(S));
        zS.ensure(nf * sizeof(S));
        launch_convert(r, pf, rS.p, p, nf, st);
        r_s = rS.p;
        z_s = zS.p;
      }
      body(r_s, z_s, nrhs, st);
      if (!same) launch_convert(z_s, p, z, pf, nf, st);
      return;
    }
    // captured form: fixed buffers rS / zS, private stream ordered after and before st
    QMG_CHECK(h.cycle_steps > 0, QMG_EINVAL, "a captured K-cycle needs a coarse step budget");
    rS.ensure(nf * sizeof(S));
    zS.ensure(nf * sizeof(S));
    if (!gs) {
      QMG_HIP(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
      QMG_HIP(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
      QMG_HIP(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
    }
    launch_convert(r, pf, rS.p, p, nf, st);  // a copy when F == S
    QMG_HIP(hipEventRecord(ev_in, st));
    QMG_HIP(hipStreamWaitEvent(gs, ev_in, 0));
    if (!exec || graph_nrhs != nrhs) {
      if (exec) {
        QMG_HIP(hipGraphExecDestroy(exec));
        exec = nullptr;
      }
      // this cycle runs eagerly (sizing every work buffer), then the same launches are captured
      body(rS.p, zS.p, nrhs, gs);
      hipGraph_t g = nullptr;
      QMG_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed));
      try {
        body(rS.p, zS.p, nrhs, gs);
      } catch (...) {
        (void)hipStreamEndCapture(gs, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      smooth_iters -= h.n_post;  // the captured launches did not run
      QMG_HIP(hipStreamEndCapture(gs, &g));
      const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      QMG_HIP(e);
      graph_nrhs = nrhs;
    } else {
      QMG_HIP(hipGraphLaunch(exec, gs));
      smooth_iters += h.n_post;
    }
    QMG_HIP(hipEventRecord(ev_out, gs));
    QMG_HIP(hipStreamWaitEvent(st, ev_out, 0));
    launch_convert(zS.p, p, z, pf, nf, st);
  }
  // coarse steps taken in device-exit mode (read once, after the solve)
  void finish(hipStream_t st) {
    if (h.cycle_steps <= 0 || !conv.p) return;
    int c[4];
    QMG_HIP(hipStreamSynchronize(st));
    if (gs) QMG_HIP(hipStreamSynchronize(gs));
    QMG_HIP(hipMemcpy(c, conv.p, sizeof(c), hipMemcpyDeviceToHost));
    coarse_iters += c[2];
  }
};

// gamma_5 on native spinors: negate spins 2, 3
template <class S>
__global__ void k_gamma5(S* x, int V, int nrhs) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  const size_t n = size_t(nrhs) * 6 * V;
  if (g >= n) return;
  const size_t rhs = g / (size_t(6) * V), rem = g - rhs * 6 * V;
  const size_t idx = (rhs * 12 + 6) * V + rem;
  auto v = StoreTraits<S>::ld(x[idx]);
  x[idx] = StoreTraits<S>::st(-v);
}
void gamma5_f64(void* x, int V, int nrhs, hipStream_t st) {
  const size_t n = size_t(nrhs) * 6 * V;
  {
    TimedLaunch tl_("layout/gamma5", st, 2.0 * double(n) * 16, 0.0);
    launch(k_gamma5<double2>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, (double2*)x, V, nrhs);
  }
  QMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// tables
void build_tables(HierarchyDev& h) {
  const Geom& g = h.g;
  const Blocking& b = h.blk;
  std::vector<int> bsite(size_t(b.d) * b.nd), cnb(size_t(b.d) * 8);
  for (int t = 0; t < g.L[3]; ++t)
    for (int z = 0; z < g.L[2]; ++z)
      for (int y = 0; y < g.L[1]; ++y)
        for (int x = 0; x < g.L[0]; ++x) {
          const int c[4] = {x, y, z, t};
          int cj[4], ci[4];
          for (int q = 0; q < 4; ++q) {
            cj[q] = c[q] / b.b[q];
            ci[q] = c[q] % b.b[q];
          }
          const int j = cj[0] + b.cL[0] * (cj[1] + b.cL[1] * (cj[2] + b.cL[2] * cj[3]));
          const int ib = ci[0] + b.b[0] * (ci[1] + b.b[1] * (ci[2] + b.b[2] * ci[3]));
          const int site = x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
          bsite[size_t(j) * b.nd + ib] = site;
        }
  for (int j = 0; j < b.d; ++j) {
    int c[4], rem = j;
    for (int q = 0; q < 4; ++q) {
      c[q] = rem % b.cL[q];
      rem /= b.cL[q];
    }
    for (int dir = 0; dir < 8; ++dir) {
      const int mu = dir & 3, step = dir < 4 ? 1 : -1;
      int cc[4] = {c[0], c[1], c[2], c[3]};
      cc[mu] = (cc[mu] + step + b.cL[mu]) % b.cL[mu];
      cnb[size_t(j) * 8 + dir] = cc[0] + b.cL[0] * (cc[1] + b.cL[1] * (cc[2] + b.cL[2] * cc[3]));
    }
  }
  // for each hop direction, the in-block indices whose hop stays inside the block, then those
  // whose hop crosses the block face (x_mu mod b_mu = b_mu - 1 forward, = 0 backward)
  std::vector<int> lists(size_t(8) * b.nd);
  const int stride[4] = {1, b.b[0], b.b[0] * b.b[1], b.b[0] * b.b[1] * b.b[2]};
  for (int dir = 0; dir < 8; ++dir) {
    const int mu = dir & 3;
    const bool fwd = dir < 4;
    int n = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int ib = 0; ib < b.nd; ++ib) {
        const int c = (ib / stride[mu]) % b.b[mu];
        const bool face = fwd ? (c == b.b[mu] - 1) : (c == 0);
        if (face == (pass == 1)) lists[size_t(dir) * b.nd + n++] = ib;
      }
  }
  h.blists.alloc(lists.size() * sizeof(int));
  QMG_HIP(hipMemcpy(h.blists.p, lists.data(), lists.size() * sizeof(int), hipMemcpyHostToDevice));
  h.bsite.alloc(bsite.size() * sizeof(int));
  h.cnb.alloc(cnb.size() * sizeof(int));
  QMG_HIP(hipMemcpy(h.bsite.p, bsite.data(), bsite.size() * sizeof(int), hipMemcpyHostToDevice));
  QMG_HIP(hipMemcpy(h.cnb.p, cnb.data(), cnb.size() * sizeof(int), hipMemcpyHostToDevice));
}

double host_norm2(const void* dev, size_t n_complex, hipStream_t st) {
  RedWork rw;
  DevBuf out(sizeof(double));
  Blas<double2>::norm2(dev, n_complex, 1, out.as<double>(), rw, st);
  double v = 0;
  QMG_HIP(hipMemcpyAsync(&v, out.p, sizeof(double), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  return v;
}

// ---------------------------------------------------------------------------------------
// Eq. (2) smoothing of r test vectors held in native FP64 `phi` (in place: phi <- psi/|psi|),
// computed in storage precision S.
template <class S>
void smooth_native(const Geom& g, const void* Uin, const void* Ain, void* phi, int r, int n_iter, hipStream_t st,
                   Gmres<S>& gm, DevBuf& b_in, DevBuf& x_in, DevBuf& tmp64) {
  const size_t n = size_t(r) * 12 * g.V;
  constexpr qmg_prec P = StoreTraits<S>::prec;
  if (n_iter > 0) {
    b_in.ensure(n * sizeof(S));
    x_in.ensure(n * sizeof(S));
    tmp64.ensure(n * sizeof(double2));
    WilsonOp D(g, P, Uin, Ain);
    const void* phi_in = phi;
    if (P != QMG_F64) {
      launch_convert(phi, QMG_F64, x_in.p, P, n, st);
      phi_in = x_in.p;
    }
    D.apply(phi_in, b_in.p, r, st);                         // b = D phi
    Blas<S>::axpby(0.0, b_in.p, -1.0, b_in.p, n, st);      // b = -D phi
    if (P != QMG_F64 && n_iter % 8 == 0) {
      // below FP64 the cycles run in s-step form; an FP64 setup keeps the Gram-Schmidt cycles
      // that the CPU reference follows step by step
      Geom gh = g;
      gh.mass = -(1.0 + 3.0 / g.xi);  // diagonal term zero: the hopping part D - d
      WilsonOp Hop(gh, P, Uin, nullptr);
      DevBuf basis, coef, part, e;
      smooth_sstep<S>(size_t(12) * g.V, g.diag(), D, Ain ? nullptr : &Hop, r, n_iter, b_in.p, x_in.p, basis, coef,
                      part, e, st);
    } else {
      gm.solve(D, b_in.p, x_in.p, true, r, 8, n_iter, 0.0, st);  // D psi' = -D phi
    }
    if (P != QMG_F64) {
      launch_convert(x_in.p, P, tmp64.p, QMG_F64, n, st);
      Blas<double2>::axpby(1.0, tmp64.p, 1.0, phi, n, st);
    } else {
      Blas<double2>::axpby(1.0, x_in.p, 1.0, phi, n, st);
    }
  }
  RedWork rw;
  DevBuf nrm(size_t(r) * sizeof(double));
  Blas<double2>::norm2(phi, size_t(12) * g.V, r, nrm.as<double>(), rw, st);
  Blas<double2>::scale_dev(phi, nrm.as<double>(), 0, size_t(12) * g.V, r, st);
  QMG_HIP(hipStreamSynchronize(st));
}

// Streams [s0, s1) of Algorithm 3 on the handle's state (U_k in P64, Sigma in sigma_dev): test
// vectors s * r .. s * r + r - 1 (Philox by global index, or the caller's buffer), smoothed in
// storage precision S, split by chirality and folded into every (aggregate, chirality) factor.
template <class S>
void run_streams(qmg_mg* mg, int s0, int s1, const void* test_vectors, hipStream_t st) {
  HierarchyDev& h = mg->h;
  const Geom& g = h.g;
  const qmg_mg_params* p = &mg->params;
  const int r = p->batch;
  constexpr qmg_prec P = StoreTraits<S>::prec;
  const void* Uin = (P == QMG_F64) ? h.U64.p : (h.inner == QMG_F32 ? h.Uin.p : h.U32.p);
  const void* Ain = (P == QMG_F64) ? h.A64.p : (h.inner == QMG_F32 ? h.Ain.p : h.A32.p);
  DevBuf phi(size_t(r) * 12 * g.V * sizeof(double2));
  DevBuf blocks(size_t(2) * h.blk.d * r * h.blk.N * sizeof(double2));
  DevBuf b_in, x_in, tmp64;
  Gmres<S> gm;
  for (int s = s0; s < s1; ++s) {
    const auto a0 = Clock::now();
    if (test_vectors) {
      const double2* tv0 = static_cast<const double2*>(test_vectors) + size_t(s - s0) * r * 12 * g.V;
      launch_pack_spinor(tv0, QMG_F64, phi.p, QMG_F64, g.V, r, st);
    } else {
      launch_philox_native(g, p->seed, s * r, r, phi.p, st);
    }
    smooth_native<S>(g, Uin, Ain, phi.p, r, p->n_setup_iter, st, gm, b_in, x_in, tmp64);
    const auto a1 = Clock::now();
    launch_chiral_gather(h, phi.p, blocks.p, r, st);
    mg->kp = isvd_stream(h, blocks.p, r, mg->kp, mg->sigma_dev, st);
    QMG_HIP(hipStreamSynchronize(st));
    const auto a2 = Clock::now();
    h.t_smooth += secs(a0, a1);
    h.t_svd += secs(a1, a2);
    mg->streams_done = s + 1;
  }
}

// P = U_k: the Galerkin coarse operator from P64, the inner-precision copies of P and D_c and
// the host copy of Sigma (after the last stream, after a load or after more streams)
void finish_setup(qmg_mg* mg, hipStream_t st) {
  HierarchyDev& h = mg->h;
  QMG_CHECK(mg->kp == h.k, QMG_ESHAPE, "streaming SVD ended with %d < k columns", mg->kp);
  const auto c0 = Clock::now();
  const int m = 2 * h.k;
  h.Y64.alloc(size_t(h.blk.d) * 9 * m * m * sizeof(double2));
  build_coarse(h, st);
  if (h.inner != QMG_F64) {
    const size_t np = size_t(2) * h.blk.d * h.k * h.blk.N, ny = size_t(h.blk.d) * 9 * m * m;
    h.Pin.alloc(np * prec_bytes(h.inner));
    h.Yin.alloc(ny * prec_bytes(h.inner));
    launch_convert(h.P64.p, QMG_F64, h.Pin.p, h.inner, np, st);
    launch_convert(h.Y64.p, QMG_F64, h.Yin.p, h.inner, ny, st);
  }
  if (h.coarse_eo) {  // Yhat follows the rebuilt D_c; a failed build switches the Schur coarse solve off
    h.coarse_eo = 0;
    build_coarse_eo_blocks(h, st);
    h.coarse_eo = 1;
  }
  h.sigma.resize(size_t(2) * h.blk.d * h.k);
  QMG_HIP(hipMemcpyAsync(h.sigma.data(), mg->sigma_dev.p, h.sigma.size() * sizeof(double), hipMemcpyDeviceToHost,
                         st));
  QMG_HIP(hipStreamSynchronize(st));
  h.t_coarse = secs(c0, Clock::now());
}

void run_setup(qmg_mg* mg, hipStream_t st) {
  HierarchyDev& h = mg->h;
  const auto t0 = Clock::now();
  h.P64.alloc(size_t(2) * h.blk.d * h.k * h.blk.N * sizeof(double2));
  mg->sigma_dev.alloc(size_t(2) * h.blk.d * h.k * sizeof(double));
  mg->kp = 0;
  mg->streams_done = 0;
  h.t_smooth = h.t_svd = 0;
  const int ns = mg->params.n_test / mg->params.batch;
  // test-vector smoothing in FP64 for an FP64 hierarchy, else in FP32
  if (h.inner == QMG_F64) run_streams<double2>(mg, 0, ns, mg->params.test_vectors, st);
  else run_streams<float2>(mg, 0, ns, mg->params.test_vectors, st);
  finish_setup(mg, st);
  h.t_total = secs(t0, Clock::now());
}

// ---------------------------------------------------------------------------------------
// solve
struct SolveStats {
  long outer = 0, refinements = 0, coarse = 0, smooth = 0, escalations = 0;
  long iters[4] = {0, 0, 0, 0}, smooths[4] = {0, 0, 0, 0};  // per level l = 2, 3 / l = 1, 2
  template <class K>
  void add_cycle(const K& k) {
    coarse += k.coarse_iters;
    smooth += k.smooth_iters;
    int l = 2;
    for (auto* c = k.Kc.get(); c && l < 4; c = c->next.get(), ++l) {
      iters[l] += c->coarse_iters;
      smooths[l - 1] += c->smooth_iters;
    }
  }
};

// FP64 flexible GMRES(16) with the FP64 K-cycle, in place on native x64
void solve_f64(const HierarchyDev& h, const void* b64, void* x64, int nrhs, double tol, int max_iter, bool x_zero,
               hipStream_t st, SolveStats& ss, bool& converged) {
  WilsonOp D(h.g, QMG_F64, h.U64.p, h.A64.p);
  CoarseOp Dc(h, QMG_F64, h.Y64.p);
  KCycle<double2, double2> K(h, D, Dc, h.P64.p);
  Gmres<double2> f;  // flexible GMRES(16) with the K-cycle
  auto res = f.solve(D, b64, x64, x_zero, nrhs, 16, max_iter, tol, st, nullptr, 0, &K);
  K.finish(st);
  ss.outer += res.iters;
  ss.add_cycle(K);
  ss.refinements += 1;
  converged = res.converged;
}

// FP64 defect correction around an FP32 flexible GMRES(16) whose K-cycle stores in precision S
template <class S>
void solve_mixed(const HierarchyDev& h, const void* b64, void* x64, int nrhs, double tol, int max_outer,
                 hipStream_t st, SolveStats& ss, bool& converged) {
  constexpr qmg_prec P = StoreTraits<S>::prec;
  using F = float2;
  const size_t len = size_t(12) * h.g.V, n = len * nrhs;
  WilsonOp D64(h.g, QMG_F64, h.U64.p, h.A64.p);
  WilsonOp D32(h.g, QMG_F32, P == QMG_F32 ? h.Uin.p : h.U32.p, P == QMG_F32 ? h.Ain.p : h.A32.p);
  WilsonOp Din(h.g, P, h.Uin.p, h.Ain.p);
  CoarseOp Dc(h, P, h.Yin.p);
  KCycle<F, S> K(h, Din, Dc, h.Pin.p);
  Gmres<F> f;  // flexible GMRES(16) with the K-cycle
  // Two Gram-Schmidt passes in the FP32 outer solver: with a strong preconditioner each new
  // Arnoldi vector is nearly in the span of the previous ones, and one pass with the norm from
  // Pythagoras then loses orthogonality in FP32, so the least-squares estimate claims a residual
  // the iterate does not have (on 32^3 x 64 point sources: 3 to 12 outer iterations and up to
  // three refinements depending on the source; with two passes 4 and two for every source)
  f.set_cgs2(true);
  DevBuf r64(n * sizeof(double2)), rin(n * sizeof(F)), ein(n * sizeof(F)), nrm(nrhs * sizeof(double)),
      bn(nrhs * sizeof(double));
  RedWork rw;
  std::vector<double> hb(nrhs), hr(nrhs);
  Blas<double2>::norm2(b64, len, nrhs, bn.as<double>(), rw, st);
  QMG_HIP(hipMemcpyAsync(hb.data(), bn.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  const double inner_tol = (P == QMG_F32) ? 1e-5 : 1e-2;  // BF16/FP16 K-cycle limits the inner solve
  std::vector<double> hist;
  converged = false;
  struct Acc {
    SolveStats& ss;
    KCycle<F, S>& K;
    hipStream_t st;
    ~Acc() {
      try {
        K.finish(st);
      } catch (...) {
      }
      ss.add_cycle(K);
    }
  } acc{ss, K, st};
  for (int ref = 0; ref < 40 && ss.outer < max_outer; ++ref) {
    D64.apply(x64, r64.p, nrhs, st);
    dc_residual(b64, r64.p, len, nrhs, nrm.as<double>(), rw, st);  // r = b - D x in FP64 and |r|^2
    QMG_HIP(hipMemcpyAsync(hr.data(), nrm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    QMG_HIP(hipStreamSynchronize(st));
    double worst = 0;
    for (int i = 0; i < nrhs; ++i) {
      QMG_CHECK(std::isfinite(hr[i]), QMG_ENONFINITE, "non-finite residual in defect correction");
      worst = std::max(worst, hb[i] > 0 ? std::sqrt(hr[i] / hb[i]) : 0.0);
    }
    hist.push_back(worst);
    if (worst <= tol) {
      converged = true;
      return;
    }
    // stagnation: two refinements each reducing less than 2x -> finish in FP64
    const size_t H = hist.size();
    if (H >= 3 && hist[H - 1] > 0.5 * hist[H - 2] && hist[H - 2] > 0.5 * hist[H - 3]) {
      ss.escalations += 1;
      bool c = false;
      solve_f64(h, b64, x64, nrhs, tol, std::max(1, int(max_outer - ss.outer)), false, st, ss, c);
      converged = c;
      return;
    }
    // r / |r| in the inner precision
    dc_normalise(r64.p, nrm.as<double>(), rin.p, len, nrhs, st);
    auto res = f.solve(D32, rin.p, ein.p, true, nrhs, 16, int(max_outer - ss.outer), inner_tol, st, nullptr, 0, &K);
    ss.outer += res.iters;
    ss.refinements += 1;
    // x += |r| e
    dc_accumulate(ein.p, nrm.as<double>(), x64, len, nrhs, st);
  }
}

template <class F>
qmg_status guard(F&& f) {
  try {
    f();
    return QMG_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return QMG_ENOMEM;
  } catch (...) {
    set_error("unexpected exception");
    return QMG_EINVAL;
  }
}

void check_ptr(const void* p, const char* name) { QMG_CHECK(p != nullptr, QMG_EINVAL, "%s is NULL", name); }

qmg_status wilson_common(const qmg_lattice* lat, const void* U, const void* in, void* out, int32_t nrhs,
                         qmg_prec prec, qmg_layout layout, hipStream_t st, bool dag) {
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(U, "U");
    check_ptr(in, "in");
    check_ptr(out, "out");
    QMG_CHECK(in != out, QMG_EINVAL, "in and out must not alias");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    check_prec(prec);
    QMG_CHECK(layout == QMG_CANONICAL || layout == QMG_NATIVE, QMG_EINVAL, "bad layout");
    Geom g = make_geom(lat);
    DslashArgs a = make_dslash_args(g, nrhs, dag, layout == QMG_CANONICAL);
    launch_dslash(prec, U, in, out, a, st);
  });
}

Geom eo_geom_checked(const qmg_lattice* lat) {
  check_ptr(lat, "lat");
  Geom g = make_geom(lat);
  QMG_CHECK(g.L[0] % 2 == 0 && g.L[1] % 2 == 0 && g.L[2] % 2 == 0 && g.L[3] % 2 == 0, QMG_ESHAPE,
            "even-odd preconditioning needs every extent even");
  return g;
}

void check_eo_prec(qmg_prec p) { check_prec(p); }

// Device copy of the descriptor table of the last batched call (uploaded again, after the
// stream has drained, when the lattice set changes)
struct BatchCache {
  std::vector<BatchLattice> host;
  DevBuf dev;
};
BatchCache& batch_cache() {
  static BatchCache c;
  return c;
}

}  // namespace
}  // namespace qmg

using namespace qmg;

extern "C" {

qmg_status qmg_wilson_apply(const qmg_lattice* lat, const void* U, const void* in, void* out, int32_t nrhs,
                            qmg_prec prec, qmg_layout layout, hipStream_t stream) {
  return wilson_common(lat, U, in, out, nrhs, prec, layout, stream, false);
}

qmg_status qmg_wilson_apply_adj(const qmg_lattice* lat, const void* U, const void* in, void* out, int32_t nrhs,
                                qmg_prec prec, qmg_layout layout, hipStream_t stream) {
  return wilson_common(lat, U, in, out, nrhs, prec, layout, stream, true);
}

qmg_status qmg_clover_field(const qmg_lattice* lat, double c_sw_s, double c_sw_t, const void* U, void* A,
                            qmg_prec prec, hipStream_t stream) {
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(U, "U");
    check_ptr(A, "A");
    check_prec(prec);
    QMG_CHECK(std::isfinite(c_sw_s) && std::isfinite(c_sw_t), QMG_EINVAL, "clover coefficients must be finite");
    Geom g = make_geom(lat);
    const size_t na = size_t(36) * g.V;
    DevBuf U64(na * sizeof(double2));
    launch_pack_gauge(U, U64.p, QMG_F64, g.V, stream);
    if (prec == QMG_F64) {
      launch_clover_field(g, U64.p, c_sw_s, c_sw_t, A, stream);
    } else {
      DevBuf A64(na * sizeof(double2));
      launch_clover_field(g, U64.p, c_sw_s, c_sw_t, A64.p, stream);
      launch_convert(A64.p, QMG_F64, A, prec, na, stream);
      QMG_HIP(hipStreamSynchronize(stream));  // A64 is released on return
    }
  });
}

qmg_status qmg_clover_apply(const qmg_lattice* lat, const void* U, const void* A, const void* in, void* out,
                            int32_t nrhs, qmg_prec prec, qmg_layout layout, int32_t dagger, hipStream_t stream) {
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(U, "U");
    check_ptr(A, "A");
    check_ptr(in, "in");
    check_ptr(out, "out");
    QMG_CHECK(in != out, QMG_EINVAL, "in and out must not alias");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    check_prec(prec);
    QMG_CHECK(layout == QMG_CANONICAL || layout == QMG_NATIVE, QMG_EINVAL, "bad layout");
    Geom g = make_geom(lat);
    DslashArgs a = make_dslash_args(g, nrhs, dagger != 0, layout == QMG_CANONICAL);
    a.clov = A;
    launch_dslash(prec, U, in, out, a, stream);
  });
}

qmg_status qmg_eo_pack_gauge(const qmg_lattice* lat, const void* U, void* U_eo, qmg_prec prec, hipStream_t stream) {
  return guard([&] {
    const Geom g = eo_geom_checked(lat);
    check_ptr(U, "U");
    check_ptr(U_eo, "U_eo");
    check_eo_prec(prec);
    launch_eo_pack_gauge(g, U, U_eo, prec, stream);
  });
}

qmg_status qmg_eo_pack_spinor(const qmg_lattice* lat, const void* canon_f64, void* even, void* odd, int32_t nrhs,
                              qmg_prec prec, hipStream_t stream) {
  return guard([&] {
    const Geom g = eo_geom_checked(lat);
    check_ptr(canon_f64, "canon_f64");
    check_ptr(even, "even");
    check_ptr(odd, "odd");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    check_eo_prec(prec);
    launch_eo_pack_spinor(g, canon_f64, even, odd, nrhs, prec, stream);
  });
}

qmg_status qmg_eo_unpack_spinor(const qmg_lattice* lat, const void* even, const void* odd, void* canon_f64,
                                int32_t nrhs, qmg_prec prec, hipStream_t stream) {
  return guard([&] {
    const Geom g = eo_geom_checked(lat);
    check_ptr(canon_f64, "canon_f64");
    check_ptr(even, "even");
    check_ptr(odd, "odd");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    check_eo_prec(prec);
    launch_eo_unpack_spinor(g, even, odd, canon_f64, nrhs, prec, stream);
  });
}

qmg_status qmg_eo_site_term(const qmg_lattice* lat, double c_sw_s, double c_sw_t, const void* U, void* A_eo,
                            void* Ainv_eo, qmg_prec prec, hipStream_t stream) {
  return guard([&] {
    const Geom g = eo_geom_checked(lat);
    check_ptr(U, "U");
    check_ptr(A_eo, "A_eo");
    check_ptr(Ainv_eo, "Ainv_eo");
    check_eo_prec(prec);
    QMG_CHECK(std::isfinite(c_sw_s) && std::isfinite(c_sw_t), QMG_EINVAL, "clover coefficients must be finite");
    const size_t na = size_t(36) * g.V;
    DevBuf U64(na * sizeof(double2)), A64(na * sizeof(double2));
    launch_pack_gauge(U, U64.p, QMG_F64, g.V, stream);
    launch_clover_field(g, U64.p, c_sw_s, c_sw_t, A64.p, stream);
    launch_eo_site_term(g, A64.p, A_eo, Ainv_eo, prec, stream);  // synchronises
  });
}

qmg_status qmg_schur_apply(const qmg_lattice* lat, const void* U_eo, const void* A_eo, const void* Ainv_eo,
                           const void* in_e, void* out_e, int32_t nrhs, qmg_prec prec, int32_t dagger,
                           hipStream_t stream) {
  return guard([&] {
    const Geom g = eo_geom_checked(lat);
    check_ptr(U_eo, "U_eo");
    check_ptr(in_e, "in_e");
    check_ptr(out_e, "out_e");
    QMG_CHECK(in_e != out_e, QMG_EINVAL, "in_e and out_e must not alias");
    QMG_CHECK((A_eo == nullptr) == (Ainv_eo == nullptr), QMG_EINVAL, "give both A_eo and Ainv_eo, or neither");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    check_eo_prec(prec);
    SchurOp S(g, prec, U_eo, A_eo, Ainv_eo, dagger != 0);
    S.apply(in_e, out_e, nrhs, stream);
    QMG_HIP(hipStreamSynchronize(stream));  // the intermediate is released on return
  });
}

qmg_status qmg_eo_solve(const qmg_lattice* lat, const void* U, double c_sw_s, double c_sw_t, const void* b, void* x,
                        int32_t nrhs, double tol, int32_t max_iter, int32_t eo, qmg_solve_info* info,
                        hipStream_t stream) {
  return guard([&] {
    check_ptr(lat, "lat");
    const Geom g = eo ? eo_geom_checked(lat) : make_geom(lat);
    check_ptr(U, "U");
    check_ptr(b, "b");
    check_ptr(x, "x");
    QMG_CHECK(nrhs >= 1 && max_iter >= 1, QMG_EINVAL, "need nrhs >= 1, max_iter >= 1");
    QMG_CHECK(tol > 0 && tol < 1, QMG_EINVAL, "tol must be in (0, 1)");
    QMG_CHECK(std::isfinite(c_sw_s) && std::isfinite(c_sw_t), QMG_EINVAL, "clover coefficients must be finite");
    const auto t0 = Clock::now();
    const bool clov = c_sw_s != 0.0 || c_sw_t != 0.0;
    const size_t V = size_t(g.V), Vh = V / 2, len = 12 * V, n = len * nrhs;
    DevBuf U64(36 * V * sizeof(double2)), A64;
    launch_pack_gauge(U, U64.p, QMG_F64, g.V, stream);
    if (clov) {
      A64.alloc(36 * V * sizeof(double2));
      launch_clover_field(g, U64.p, c_sw_s, c_sw_t, A64.p, stream);
    }
    WilsonOp D(g, QMG_F64, U64.p, A64.p);
    DevBuf b64(n * sizeof(double2)), x64(n * sizeof(double2)), r64(n * sizeof(double2));
    launch_pack_spinor(b, QMG_F64, b64.p, QMG_F64, g.V, nrhs, stream);
    RedWork rw;
    DevBuf nb(nrhs * sizeof(double)), nr(nrhs * sizeof(double));
    Blas<double2>::norm2(b64.p, len, nrhs, nb.as<double>(), rw, stream);
    std::vector<double> hb(nrhs), hr(nrhs);
    QMG_HIP(hipMemcpyAsync(hb.data(), nb.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, stream));
    QMG_HIP(hipStreamSynchronize(stream));
    Gmres<double2> gm;
    Gmres<double2>::Result res;
    if (eo) {
      const size_t hl = 12 * Vh * nrhs;
      DevBuf Ueo(36 * V * sizeof(double2)), Aeo, Ainv;
      launch_eo_pack_gauge(g, U, Ueo.p, QMG_F64, stream);
      if (clov) {
        Aeo.alloc(36 * V * sizeof(double2));
        Ainv.alloc(36 * V * sizeof(double2));
        launch_eo_site_term(g, A64.p, Aeo.p, Ainv.p, QMG_F64, stream);
      }
      SchurOp S(g, QMG_F64, Ueo.p, Aeo.p, Ainv.p, false);
      DevBuf be(hl * sizeof(double2)), bo(hl * sizeof(double2)), bh(hl * sizeof(double2)), xe(hl * sizeof(double2)),
          xo(hl * sizeof(double2)), t(hl * sizeof(double2));
      launch_eo_pack_spinor(g, b, be.p, bo.p, nrhs, QMG_F64, stream);
      DslashArgs a = make_dslash_args(g, nrhs, false, false);
      launch_site_eo(QMG_F64, a, S.Aio, true, bo.p, t.p, stream);                                 // A_oo^-1 b_o
      launch_hop_eo(QMG_F64, a, S.Ue, S.Uo, 0, t.p, be.p, bh.p, nullptr, nullptr, 1, 0, -1.0, stream);  // bhat_e
      // Dhat x_e = bhat_e to tol ||b|| / ||bhat_e||: the even residual of the reconstructed x is
      // the Schur residual and its odd residual vanishes
      DevBuf nh(nrhs * sizeof(double));
      Blas<double2>::norm2(bh.p, 12 * Vh, nrhs, nh.as<double>(), rw, stream);
      std::vector<double> hh(nrhs);
      QMG_HIP(hipMemcpyAsync(hh.data(), nh.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, stream));
      QMG_HIP(hipStreamSynchronize(stream));
      double ratio = 1.0;
      for (int i = 0; i < nrhs; ++i)
        if (hh[i] > 0) ratio = std::min(ratio, std::sqrt(hb[i] / hh[i]));
      res = gm.solve(S, bh.p, xe.p, true, nrhs, 32, max_iter, std::min(0.5, tol * ratio), stream);
      launch_hop_eo(QMG_F64, a, S.Ue, S.Uo, 1, xe.p, bo.p, xo.p, nullptr, S.Aio, 1, 1, -1.0, stream);  // x_o
      launch_eo_unpack_spinor(g, xe.p, xo.p, x, nrhs, QMG_F64, stream);
      launch_pack_spinor(x, QMG_F64, x64.p, QMG_F64, g.V, nrhs, stream);
    } else {
      res = gm.solve(D, b64.p, x64.p, true, nrhs, 32, max_iter, tol, stream);
      launch_unpack_spinor(x64.p, QMG_F64, x, QMG_F64, g.V, nrhs, stream);
    }
    D.apply(x64.p, r64.p, nrhs, stream);
    Blas<double2>::axpby(1.0, b64.p, -1.0, r64.p, n, stream);
    Blas<double2>::norm2(r64.p, len, nrhs, nr.as<double>(), rw, stream);
    QMG_HIP(hipMemcpyAsync(hr.data(), nr.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, stream));
    QMG_HIP(hipStreamSynchronize(stream));
    double worst = 0;
    for (int i = 0; i < nrhs; ++i) worst = std::max(worst, hb[i] > 0 ? std::sqrt(hr[i] / hb[i]) : 0.0);
    if (info) {
      *info = qmg_solve_info{};
      info->outer_iters = res.iters;
      info->refinements = 1;
      info->true_rel_res = worst;
      info->seconds = secs(t0, Clock::now());
    }
    QMG_CHECK(std::isfinite(worst), QMG_ENONFINITE, "non-finite residual");
    QMG_CHECK(res.converged && worst <= 10 * tol, QMG_ENOCONV, "even-odd solve stopped at %d iterations, residual %.3g",
              res.iters, worst);
  });
}

qmg_status qmg_wilson_apply_batched(int32_t n_lat, const qmg_lattice* lats, const void* const* U,
                                    const void* const* in, void* const* out, int32_t nrhs, qmg_prec prec,
                                    int32_t dagger, hipStream_t stream) {
  return guard([&] {
    QMG_CHECK(n_lat >= 1 && n_lat <= 65536, QMG_EINVAL, "n_lat must be in [1, 65536]");
    check_ptr(lats, "lats");
    check_ptr(U, "U");
    check_ptr(in, "in");
    check_ptr(out, "out");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    QMG_CHECK(dagger == 0 || dagger == 1, QMG_EINVAL, "dagger must be 0 or 1");
    check_prec(prec);
    std::vector<BatchLattice> tab(n_lat);
    long tiles = 0;
    double sites = 0;
    for (int i = 0; i < n_lat; ++i) {
      Geom g = make_geom(&lats[i]);
      tab[i].a = make_dslash_args(g, nrhs, dagger != 0, false);
      tab[i].tile0 = int(tiles);
      tiles += long((g.V + 255) / 256) * nrhs;
      sites += double(g.V);
      QMG_CHECK(tiles < (1L << 31), QMG_ESHAPE, "batched dslash: too many workgroups");
    }
    BatchCache& c = batch_cache();
    const size_t bytes = tab.size() * sizeof(BatchLattice);
    if (c.host.size() != tab.size() || std::memcmp(c.host.data(), tab.data(), bytes) != 0) {
      QMG_HIP(hipStreamSynchronize(stream));  // the previous table may still be in use
      QMG_HIP(hipDeviceSynchronize());
      c.dev.ensure(bytes);
      QMG_HIP(hipMemcpy(c.dev.p, tab.data(), bytes, hipMemcpyHostToDevice));
      c.host = tab;
    }
    const double cb = double(prec_bytes(prec));
    launch_dslash_batched(prec, c.dev.as<BatchLattice>(), n_lat, int(tiles), U, in, out, dagger != 0,
                          sites * (24.0 * nrhs + 36.0) * cb, 1368.0 * sites * nrhs, stream);
  });
}

qmg_status qmg_pack_spinor(const qmg_lattice* lat, const void* canon, void* native, int32_t nrhs, qmg_prec prec,
                           hipStream_t stream) {
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(canon, "canon");
    check_ptr(native, "native");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    check_prec(prec);
    Geom g = make_geom(lat);
    launch_pack_spinor(canon, QMG_F64, native, prec, g.V, nrhs, stream);
  });
}

qmg_status qmg_unpack_spinor(const qmg_lattice* lat, const void* native, void* canon, int32_t nrhs, qmg_prec prec,
                             hipStream_t stream) {
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(canon, "canon");
    check_ptr(native, "native");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    check_prec(prec);
    Geom g = make_geom(lat);
    launch_unpack_spinor(native, prec, canon, QMG_F64, g.V, nrhs, stream);
  });
}

qmg_status qmg_pack_gauge(const qmg_lattice* lat, const void* canon, void* native, qmg_prec prec,
                          hipStream_t stream) {
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(canon, "canon");
    check_ptr(native, "native");
    check_prec(prec);
    Geom g = make_geom(lat);
    launch_pack_gauge(canon, native, prec, g.V, stream);
  });
}

}  // extern "C"

namespace qmg {
namespace {

// Validated blocking for a lattice and setup parameters (ESHAPE / EINVAL otherwise).
Blocking check_params(const Geom& g, const qmg_mg_params* p) {
  Blocking b{};
  b.nd = 1;
  b.d = 1;
  for (int q = 0; q < 4; ++q) {
    QMG_CHECK(p->block[q] >= 1 && g.L[q] % p->block[q] == 0, QMG_ESHAPE,
              "block extent %d (%d) does not divide lattice extent %d", q, p->block[q], g.L[q]);
    b.b[q] = p->block[q];
    b.cL[q] = g.L[q] / p->block[q];
    b.nd *= b.b[q];
    b.d *= b.cL[q];
  }
  b.N = 6 * b.nd;
  QMG_CHECK(p->batch >= 1 && p->batch <= 48, QMG_ESHAPE, "batch r must be in [1, 48]");
  QMG_CHECK(p->n_test >= p->batch && p->n_test % p->batch == 0, QMG_ESHAPE,
            "n_test must be a positive multiple of batch");
  QMG_CHECK(p->rank >= 1 && p->rank <= b.N && p->rank <= p->n_test && p->rank <= 32, QMG_ESHAPE,
            "rank k must satisfy 1 <= k <= min(6*prod(block), n_test, 32)");
  QMG_CHECK(p->n_setup_iter >= 0 && p->n_post_smooth >= 0 && p->coarse_max_iter >= 1, QMG_EINVAL,
            "iteration counts must be non-negative");
  QMG_CHECK(p->coarse_tol > 0 && p->coarse_tol < 1, QMG_EINVAL, "coarse_tol must be in (0, 1)");
  QMG_CHECK(std::isfinite(p->c_sw_s) && std::isfinite(p->c_sw_t), QMG_EINVAL, "clover coefficients must be finite");
  check_prec(p->inner_prec);
  return b;
}

// A handle with the tables and the packed gauge copies, before any stream.
std::unique_ptr<qmg_mg> new_hierarchy(const qmg_lattice* lat, const void* U, const qmg_mg_params* p,
                                      hipStream_t stream) {
  const Geom g = make_geom(lat);
  const Blocking b = check_params(g, p);
  std::unique_ptr<qmg_mg> mg(new qmg_mg());
  HierarchyDev& h = mg->h;
  h.g = g;
  h.blk = b;
  h.k = p->rank;
  h.inner = p->inner_prec;
  h.n_post = p->n_post_smooth;
  h.coarse_tol = p->coarse_tol;
  h.coarse_max = p->coarse_max_iter;
  build_tables(h);
  h.U64.alloc(size_t(36) * g.V * sizeof(double2));
  launch_pack_gauge(U, h.U64.p, QMG_F64, g.V, stream);
  const double un = host_norm2(h.U64.p, size_t(36) * g.V, stream);
  QMG_CHECK(std::isfinite(un), QMG_ENONFINITE, "gauge field has non-finite entries");
  if (h.inner != QMG_F64) {
    h.Uin.alloc(size_t(36) * g.V * prec_bytes(h.inner));
    launch_pack_gauge(U, h.Uin.p, h.inner, g.V, stream);
  }
  if (h.inner == QMG_BF16 || h.inner == QMG_F16) {
    h.U32.alloc(size_t(36) * g.V * sizeof(float2));
    launch_pack_gauge(U, h.U32.p, QMG_F32, g.V, stream);
  }
  if (p->c_sw_s != 0.0 || p->c_sw_t != 0.0) {  // Wilson-clover: the site term beside every gauge copy
    const size_t na = size_t(36) * g.V;
    h.A64.alloc(na * sizeof(double2));
    launch_clover_field(g, h.U64.p, p->c_sw_s, p->c_sw_t, h.A64.p, stream);
    if (h.inner != QMG_F64) {
      h.Ain.alloc(na * prec_bytes(h.inner));
      launch_convert(h.A64.p, QMG_F64, h.Ain.p, h.inner, na, stream);
    }
    if (h.inner == QMG_BF16 || h.inner == QMG_F16) {
      h.A32.alloc(na * sizeof(float2));
      launch_convert(h.A64.p, QMG_F64, h.A32.p, QMG_F32, na, stream);
    }
  }
  mg->lat = *lat;
  mg->params = *p;
  mg->params.test_vectors = nullptr;  // caller memory is not retained
  return mg;
}

// ---------------------------------------------------------------------------------------
// Third level: Algorithm 4 with Algorithm 3 applied to D_c.  Tables on the coarse lattice,
// streams of coarse test vectors (Philox, level word 1) smoothed in FP64 on D_c, the chiral
// split by the coarse chirality (the alpha block of every coarse site), the streaming SVD per
// (aggregate, chirality), the Galerkin stencil and the inner-precision copies.
void build_level_tables(CoarseLevel& L, const StencilRef& above) {
  const int* cL1 = above.cL;
  const int d1 = above.d;
  std::vector<int> bsite(size_t(L.d) * L.nd), cnb(size_t(L.d) * 8), agg(d1), pos(d1);
  for (int j = 0; j < d1; ++j) {
    int c[4], rem = j;
    for (int q = 0; q < 4; ++q) {
      c[q] = rem % cL1[q];
      rem /= cL1[q];
    }
    int cj[4], ci[4];
    for (int q = 0; q < 4; ++q) {
      cj[q] = c[q] / L.b[q];
      ci[q] = c[q] % L.b[q];
    }
    const int J = cj[0] + L.cL[0] * (cj[1] + L.cL[1] * (cj[2] + L.cL[2] * cj[3]));
    const int jb = ci[0] + L.b[0] * (ci[1] + L.b[1] * (ci[2] + L.b[2] * ci[3]));
    bsite[size_t(J) * L.nd + jb] = j;
    agg[j] = J;
    pos[j] = jb;
  }
  for (int J = 0; J < L.d; ++J) {
    int c[4], rem = J;
    for (int q = 0; q < 4; ++q) {
      c[q] = rem % L.cL[q];
      rem /= L.cL[q];
    }
    for (int dir = 0; dir < 8; ++dir) {
      const int mu = dir & 3, step = dir < 4 ? 1 : -1;
      int cc[4] = {c[0], c[1], c[2], c[3]};
      cc[mu] = (cc[mu] + step + L.cL[mu]) % L.cL[mu];
      cnb[size_t(J) * 8 + dir] = cc[0] + L.cL[0] * (cc[1] + L.cL[1] * (cc[2] + L.cL[2] * cc[3]));
    }
  }
  auto up = [](DevBuf& b, const std::vector<int>& v) {
    b.alloc(v.size() * sizeof(int));
    QMG_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice));
  };
  up(L.bsite, bsite);
  up(L.cnb, cnb);
  up(L.agg, agg);
  up(L.pos, pos);
}

void run_level_setup(HierarchyDev& h, size_t i, hipStream_t st) {
  CoarseLevel& L = *h.levels[i];
  const StencilRef above = stencil_above(h, i);
  const auto t0 = Clock::now();
  const int d1 = above.d, m1 = 2 * above.k, r = L.batch, ns = L.n_test / L.batch;
  const size_t len = size_t(d1) * m1, n = size_t(r) * len;
  StencilOp Dc(above.d, above.k, above.cnb, QMG_F64, above.Y64);  // the level above, FP64
  Gmres<double2> gm;
  DevBuf phi(n * sizeof(double2)), b(n * sizeof(double2)), x(n * sizeof(double2)), nrm(r * sizeof(double));
  DevBuf blocks(size_t(2) * L.d * r * L.N * sizeof(double2));
  RedWork rw;
  L.P64.alloc(size_t(2) * L.d * L.k * L.N * sizeof(double2));
  L.sigma_dev.alloc(size_t(2) * L.d * L.k * sizeof(double));
  L.kp = 0;
  for (int s = 0; s < ns; ++s) {
    launch_philox_coarse(L.seed, s * r, r, d1, m1, int(i) + 1, phi.p, st);  // level word l - 1
    if (L.n_setup_iter > 0) {  // psi = phi + psi', D_c psi' = -D_c phi by GMRES(8) from zero
      Dc.apply(phi.p, b.p, r, st);
      Blas<double2>::axpby(0.0, b.p, -1.0, b.p, n, st);
      gm.solve(Dc, b.p, x.p, true, r, 8, L.n_setup_iter, 0.0, st);
      Blas<double2>::axpby(1.0, x.p, 1.0, phi.p, n, st);
    }
    Blas<double2>::norm2(phi.p, len, r, nrm.as<double>(), rw, st);
    Blas<double2>::scale_dev(phi.p, nrm.as<double>(), 0, len, r, st);
    launch_level_gather(L, phi.p, blocks.p, r, st);
    L.kp = isvd_stream(2 * L.d, L.N, L.k, L.P64, blocks.p, r, L.kp, L.sigma_dev, st);
    L.streams_done = s + 1;
  }
  QMG_CHECK(L.kp == L.k, QMG_ESHAPE, "further level: streaming SVD ended with %d < k columns", L.kp);
  build_level_coarse(L, above, st);
  if (h.inner != QMG_F64) {
    const int m2 = 2 * L.k;
    const size_t np = size_t(2) * L.d * L.k * L.N, ny = size_t(L.d) * 9 * m2 * m2;
    L.Pin.alloc(np * prec_bytes(h.inner));
    L.Yin.alloc(ny * prec_bytes(h.inner));
    launch_convert(L.P64.p, QMG_F64, L.Pin.p, h.inner, np, st);
    launch_convert(L.Y64.p, QMG_F64, L.Yin.p, h.inner, ny, st);
  }
  L.sigma.resize(size_t(2) * L.d * L.k);
  QMG_HIP(hipMemcpyAsync(L.sigma.data(), L.sigma_dev.p, L.sigma.size() * sizeof(double), hipMemcpyDeviceToHost,
                         st));
  QMG_HIP(hipStreamSynchronize(st));
  L.t_total = secs(t0, Clock::now());
}

// level l >= 2 of the hierarchy (EINVAL when it has fewer levels)
const CoarseLevel& level_at(const qmg_mg* mg, int l) {
  check_ptr(mg, "mg");
  QMG_CHECK(l >= 2 && size_t(l - 2) < mg->h.levels.size(), QMG_EINVAL, "the hierarchy has no level %d", l);
  return *mg->h.levels[l - 2];
}
const CoarseLevel& level_for(const qmg_mg* mg, int l, qmg_prec prec) {
  const CoarseLevel& L = level_at(mg, l);
  QMG_CHECK(prec == QMG_F64 || (prec == mg->h.inner && prec == QMG_F32), QMG_EDTYPE,
            "precision must be F64 or the F32 inner precision");
  return L;
}

// ---------------------------------------------------------------------------------------
// checkpoint file: fixed little-endian fields, then Sigma and U_k (P in FP64), then a hash of
// both arrays.  The gauge field is not stored: its hash ties the file to the field it was built
// for, and the Galerkin operator is rebuilt from P and the field on load.
constexpr char kMagic[8] = {'Q', 'M', 'G', 'H', 'I', 'E', 'R', '1'};
constexpr int32_t kFileVersion = 2;

uint64_t hash_words(uint64_t h, const void* data, size_t bytes) {
  const unsigned char* c = static_cast<const unsigned char*>(data);
  size_t i = 0;
  for (; i + 8 <= bytes; i += 8) {
    uint64_t w;
    std::memcpy(&w, c + i, 8);
    h = (h ^ w) * 0x100000001b3ull;
    h ^= h >> 29;
  }
  for (; i < bytes; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
  return h;
}
constexpr uint64_t kHashSeed = 0xcbf29ce484222325ull;

// hash of a device buffer, streamed through pinned host memory
uint64_t device_hash(const void* dev, size_t bytes, hipStream_t st) {
  const size_t chunk = size_t(64) << 20;
  PinnedBuf host;
  host.ensure(std::min(chunk, bytes));
  uint64_t h = kHashSeed;
  for (size_t off = 0; off < bytes; off += chunk) {
    const size_t n = std::min(chunk, bytes - off);
    QMG_HIP(hipMemcpyAsync(host.p, static_cast<const char*>(dev) + off, n, hipMemcpyDeviceToHost, st));
    QMG_HIP(hipStreamSynchronize(st));
    h = hash_words(h, host.p, n);
  }
  return h;
}

struct File {
  std::FILE* f = nullptr;
  std::string path;
  File(const char* p, const char* mode) : f(std::fopen(p, mode)), path(p) {
    QMG_CHECK(f, QMG_EINVAL, "cannot open %s", p);
  }
  ~File() {
    if (f) std::fclose(f);
  }
  void put(const void* d, size_t n) { QMG_CHECK(std::fwrite(d, 1, n, f) == n, QMG_EINVAL, "write to %s failed", path.c_str()); }
  void get(void* d, size_t n) {
    QMG_CHECK(std::fread(d, 1, n, f) == n, QMG_EINVAL, "%s is truncated or unreadable", path.c_str());
  }
  template <class T> void put(const T& v) { put(&v, sizeof(T)); }
  template <class T> T get() {
    T v;
    get(&v, sizeof(T));
    return v;
  }
};

struct FileHeader {
  qmg_lattice lat{};
  qmg_mg_params params{};
  int32_t streams_done = 0, kp = 0;
  uint64_t gauge_hash = 0;
  uint64_t n_sigma = 0, n_p = 0;
};

void put_header(File& f, const FileHeader& hd) {
  f.put(kMagic, sizeof(kMagic));
  f.put<int32_t>(kFileVersion);
  for (int q = 0; q < 4; ++q) f.put<int32_t>(hd.lat.dims[q]);
  f.put<int32_t>(hd.lat.bc_t);
  f.put<double>(hd.lat.mass);
  f.put<double>(hd.lat.xi);
  const qmg_mg_params& p = hd.params;
  for (int q = 0; q < 4; ++q) f.put<int32_t>(p.block[q]);
  f.put<int32_t>(p.n_test);
  f.put<int32_t>(p.batch);
  f.put<int32_t>(p.rank);
  f.put<int32_t>(p.n_setup_iter);
  f.put<int32_t>(p.n_post_smooth);
  f.put<double>(p.coarse_tol);
  f.put<int32_t>(p.coarse_max_iter);
  f.put<int32_t>(int32_t(p.inner_prec));
  f.put<uint64_t>(p.seed);
  f.put<double>(p.c_sw_s);
  f.put<double>(p.c_sw_t);
  f.put<int32_t>(hd.streams_done);
  f.put<int32_t>(hd.kp);
  f.put<uint64_t>(hd.gauge_hash);
  f.put<uint64_t>(hd.n_sigma);
  f.put<uint64_t>(hd.n_p);
}

FileHeader get_header(File& f) {
  char magic[8];
  f.get(magic, sizeof(magic));
  QMG_CHECK(std::memcmp(magic, kMagic, sizeof(kMagic)) == 0, QMG_EINVAL, "%s is not a hierarchy file",
            f.path.c_str());
  const int32_t ver = f.get<int32_t>();
  QMG_CHECK(ver == kFileVersion, QMG_EINVAL, "%s: unsupported hierarchy file version %d", f.path.c_str(), ver);
  FileHeader hd;
  for (int q = 0; q < 4; ++q) hd.lat.dims[q] = f.get<int32_t>();
  hd.lat.bc_t = f.get<int32_t>();
  hd.lat.mass = f.get<double>();
  hd.lat.xi = f.get<double>();
  qmg_mg_params& p = hd.params;
  for (int q = 0; q < 4; ++q) p.block[q] = f.get<int32_t>();
  p.n_test = f.get<int32_t>();
  p.batch = f.get<int32_t>();
  p.rank = f.get<int32_t>();
  p.n_setup_iter = f.get<int32_t>();
  p.n_post_smooth = f.get<int32_t>();
  p.coarse_tol = f.get<double>();
  p.coarse_max_iter = f.get<int32_t>();
  p.inner_prec = qmg_prec(f.get<int32_t>());
  p.seed = f.get<uint64_t>();
  p.c_sw_s = f.get<double>();
  p.c_sw_t = f.get<double>();
  p.test_vectors = nullptr;
  hd.streams_done = f.get<int32_t>();
  hd.kp = f.get<int32_t>();
  hd.gauge_hash = f.get<uint64_t>();
  hd.n_sigma = f.get<uint64_t>();
  hd.n_p = f.get<uint64_t>();
  return hd;
}

}  // namespace
}  // namespace qmg

extern "C" {

qmg_status qmg_mg_setup_stream_chiral_svd(const qmg_lattice* lat, const void* U, const qmg_mg_params* p,
                                          qmg_mg** out, hipStream_t stream) {
  if (out) *out = nullptr;
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(U, "U");
    check_ptr(p, "params");
    check_ptr(out, "out");
    std::unique_ptr<qmg_mg> mg = new_hierarchy(lat, U, p, stream);
    mg->params.test_vectors = p->test_vectors;
    run_setup(mg.get(), stream);
    mg->params.test_vectors = nullptr;  // caller memory is not retained
    *out = mg.release();
  });
}

qmg_status qmg_mg_stream_more(qmg_mg* mg, int32_t n_streams, hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    QMG_CHECK(n_streams >= 1, QMG_EINVAL, "n_streams must be >= 1");
    HierarchyDev& h = mg->h;
    const auto t0 = Clock::now();
    const int s0 = mg->streams_done;
    if (h.inner == QMG_F64) run_streams<double2>(mg, s0, s0 + n_streams, nullptr, stream);
    else run_streams<float2>(mg, s0, s0 + n_streams, nullptr, stream);
    mg->params.n_test = mg->streams_done * mg->params.batch;
    finish_setup(mg, stream);
    // further levels are built on D_c and on each other: rebuild them in order (dropped if that fails)
    for (size_t i = 0; i < h.levels.size(); ++i) {
      try {
        run_level_setup(h, i, stream);
      } catch (...) {
        h.levels.clear();
        throw;
      }
    }
    h.t_total += secs(t0, Clock::now());
  });
}

qmg_status qmg_mg_add_level(qmg_mg* mg, const int32_t* block, int32_t n_test, int32_t batch, int32_t rank,
                            int32_t n_setup_iter, uint64_t seed, hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(block, "block");
    HierarchyDev& h = mg->h;
    QMG_CHECK(h.levels.size() < 2, QMG_EINVAL, "the hierarchy already has four levels");
    QMG_CHECK(h.cycle_steps == 0, QMG_EINVAL, "further levels need the host-checked K-cycle (coarse_steps = 0)");
    const size_t i = h.levels.size();
    const StencilRef above = stencil_above(h, i);
    std::unique_ptr<CoarseLevel> L(new CoarseLevel());
    L->nd = 1;
    L->d = 1;
    for (int q = 0; q < 4; ++q) {
      QMG_CHECK(block[q] >= 1 && above.cL[q] % block[q] == 0, QMG_ESHAPE,
                "level %d block extent %d (%d) does not divide extent %d of the level above", int(i) + 2, q,
                block[q], above.cL[q]);
      L->b[q] = block[q];
      L->cL[q] = above.cL[q] / block[q];
      L->nd *= block[q];
      L->d *= L->cL[q];
    }
    L->k1 = above.k;
    L->N = L->nd * above.k;
    QMG_CHECK(L->N <= 4096, QMG_ESHAPE, "further level: block of %d rows exceeds 4096", L->N);
    QMG_CHECK(batch >= 1 && batch <= 48, QMG_ESHAPE, "batch r must be in [1, 48]");
    QMG_CHECK(n_test >= batch && n_test % batch == 0, QMG_ESHAPE, "n_test must be a positive multiple of batch");
    QMG_CHECK(rank >= 1 && rank <= L->N && rank <= n_test && rank <= 32, QMG_ESHAPE,
              "rank k must satisfy 1 <= k <= min(k_above * prod(block), n_test, 32)");
    QMG_CHECK(n_setup_iter >= 0, QMG_EINVAL, "n_setup_iter must be non-negative");
    L->k = rank;
    L->n_test = n_test;
    L->batch = batch;
    L->n_setup_iter = n_setup_iter;
    L->seed = seed;
    build_level_tables(*L, above);
    h.levels.push_back(std::move(L));
    try {
      run_level_setup(h, i, stream);
    } catch (...) {
      h.levels.pop_back();
      throw;
    }
  });
}

qmg_status qmg_mg_level_query(const qmg_mg* mg, int32_t level, int32_t* coarse_dims, int32_t* n_agg,
                              int32_t* rank) {
  return guard([&] {
    const CoarseLevel& L = level_at(mg, level);
    if (coarse_dims)
      for (int q = 0; q < 4; ++q) coarse_dims[q] = L.cL[q];
    if (n_agg) *n_agg = L.d;
    if (rank) *rank = L.k;
  });
}

qmg_status qmg_mg_set_level_tol(qmg_mg* mg, int32_t level, double tol) {
  return guard([&] {
    const CoarseLevel& L = level_at(mg, level);
    QMG_CHECK(tol >= 0 && tol < 1, QMG_EINVAL, "level tolerance must be in [0, 1) (0: the coarse tolerance)");
    mg->h.levels[level - 2]->tol = tol;
    (void)L;
  });
}

qmg_status qmg_mg_level_get(const qmg_mg* mg, int32_t level, void* P, double* sigma, void* Y, hipStream_t stream) {
  return guard([&] {
    const CoarseLevel& L = level_at(mg, level);
    if (P) launch_level_export_P(L, P, stream);
    if (Y) launch_level_export_Y(L, Y, stream);
    if (sigma) std::memcpy(sigma, L.sigma.data(), L.sigma.size() * sizeof(double));
    QMG_HIP(hipStreamSynchronize(stream));
  });
}

qmg_status qmg_level_prolong(const qmg_mg* mg, int32_t level, const void* in, void* out, int32_t nrhs,
                             qmg_prec prec, hipStream_t stream) {
  return guard([&] {
    const CoarseLevel& L = level_for(mg, level, prec);
    check_ptr(in, "in");
    check_ptr(out, "out");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    const int d_above = stencil_above(mg->h, size_t(level) - 2).d;
    launch_level_prolong(prec, L, d_above, prec == QMG_F64 ? L.P64.p : L.Pin.p, in, out, nrhs, stream);
  });
}

qmg_status qmg_level_restrict(const qmg_mg* mg, int32_t level, const void* in, void* out, int32_t nrhs,
                              qmg_prec prec, hipStream_t stream) {
  return guard([&] {
    const CoarseLevel& L = level_for(mg, level, prec);
    check_ptr(in, "in");
    check_ptr(out, "out");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    const int d_above = stencil_above(mg->h, size_t(level) - 2).d;
    launch_level_restrict(prec, L, d_above, prec == QMG_F64 ? L.P64.p : L.Pin.p, in, out, nrhs, stream);
  });
}

qmg_status qmg_level_coarse_apply(const qmg_mg* mg, int32_t level, const void* in, void* out, int32_t nrhs,
                                  qmg_prec prec, hipStream_t stream) {
  return guard([&] {
    const CoarseLevel& L = level_for(mg, level, prec);
    check_ptr(in, "in");
    check_ptr(out, "out");
    QMG_CHECK(in != out, QMG_EINVAL, "in and out must not alias");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    launch_stencil_apply(prec, L.d, L.k, L.cnb.as<int>(), prec == QMG_F64 ? L.Y64.p : L.Yin.p, in, out, nrhs,
                         stream);
  });
}

qmg_status qmg_mg_save(const qmg_mg* mg, const char* path, hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(path, "path");
    const HierarchyDev& h = mg->h;
    FileHeader hd;
    hd.lat = mg->lat;
    hd.params = mg->params;
    hd.params.test_vectors = nullptr;
    hd.streams_done = mg->streams_done;
    hd.kp = mg->kp;
    hd.gauge_hash = device_hash(h.U64.p, size_t(36) * h.g.V * sizeof(double2), stream);
    hd.n_sigma = uint64_t(2) * h.blk.d * h.k;
    hd.n_p = uint64_t(2) * h.blk.d * h.k * h.blk.N;
    std::vector<double> sig(hd.n_sigma);
    QMG_HIP(hipMemcpyAsync(sig.data(), mg->sigma_dev.p, sig.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    QMG_HIP(hipStreamSynchronize(stream));
    File f(path, "wb");
    put_header(f, hd);
    f.put(sig.data(), sig.size() * sizeof(double));
    uint64_t ph = hash_words(kHashSeed, sig.data(), sig.size() * sizeof(double));
    // P in chunks through pinned memory
    const size_t bytes = hd.n_p * sizeof(double2), chunk = size_t(64) << 20;
    PinnedBuf host;
    host.ensure(std::min(chunk, bytes));
    for (size_t off = 0; off < bytes; off += chunk) {
      const size_t n = std::min(chunk, bytes - off);
      QMG_HIP(hipMemcpyAsync(host.p, static_cast<const char*>(h.P64.p) + off, n, hipMemcpyDeviceToHost, stream));
      QMG_HIP(hipStreamSynchronize(stream));
      f.put(host.p, n);
      ph = hash_words(ph, host.p, n);
    }
    f.put<uint64_t>(ph);
  });
}

qmg_status qmg_mg_load(const char* path, const void* U, qmg_mg** out, hipStream_t stream) {
  if (out) *out = nullptr;
  return guard([&] {
    check_ptr(path, "path");
    check_ptr(U, "U");
    check_ptr(out, "out");
    File f(path, "rb");
    const FileHeader hd = get_header(f);
    const Geom g = make_geom(&hd.lat);
    const Blocking b = check_params(g, &hd.params);
    QMG_CHECK(hd.kp == hd.params.rank && hd.streams_done * hd.params.batch == hd.params.n_test &&
                  hd.n_sigma == uint64_t(2) * b.d * hd.params.rank &&
                  hd.n_p == uint64_t(2) * b.d * hd.params.rank * b.N,
              QMG_EINVAL, "%s: inconsistent hierarchy header", path);
    const auto t0 = Clock::now();
    std::unique_ptr<qmg_mg> mg = new_hierarchy(&hd.lat, U, &hd.params, stream);
    HierarchyDev& h = mg->h;
    const uint64_t gh = device_hash(h.U64.p, size_t(36) * g.V * sizeof(double2), stream);
    QMG_CHECK(gh == hd.gauge_hash, QMG_EINVAL, "%s was built for a different gauge field", path);
    std::vector<double> sig(hd.n_sigma);
    f.get(sig.data(), sig.size() * sizeof(double));
    uint64_t ph = hash_words(kHashSeed, sig.data(), sig.size() * sizeof(double));
    h.P64.alloc(hd.n_p * sizeof(double2));
    mg->sigma_dev.alloc(sig.size() * sizeof(double));
    QMG_HIP(hipMemcpyAsync(mg->sigma_dev.p, sig.data(), sig.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    const size_t bytes = hd.n_p * sizeof(double2), chunk = size_t(64) << 20;
    PinnedBuf host;
    host.ensure(std::min(chunk, bytes));
    for (size_t off = 0; off < bytes; off += chunk) {
      const size_t n = std::min(chunk, bytes - off);
      QMG_HIP(hipStreamSynchronize(stream));  // the previous chunk has left the staging buffer
      f.get(host.p, n);
      ph = hash_words(ph, host.p, n);
      QMG_HIP(hipMemcpyAsync(static_cast<char*>(h.P64.p) + off, host.p, n, hipMemcpyHostToDevice, stream));
    }
    QMG_HIP(hipStreamSynchronize(stream));
    QMG_CHECK(f.get<uint64_t>() == ph, QMG_EINVAL, "%s: checksum mismatch (corrupted file)", path);
    mg->kp = hd.kp;
    mg->streams_done = hd.streams_done;
    finish_setup(mg.get(), stream);
    h.t_total = secs(t0, Clock::now());
    *out = mg.release();
  });
}

qmg_status qmg_mg_get_params(const qmg_mg* mg, qmg_lattice* lat, qmg_mg_params* params) {
  return guard([&] {
    check_ptr(mg, "mg");
    if (lat) *lat = mg->lat;
    if (params) *params = mg->params;
  });
}

qmg_status qmg_prolong(const qmg_mg* mg, const void* coarse_in, void* fine_out, int32_t nrhs, qmg_prec prec,
                       hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(coarse_in, "coarse_in");
    check_ptr(fine_out, "fine_out");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    const HierarchyDev& h = mg->h;
    QMG_CHECK(prec == QMG_F64 || (prec == h.inner && prec == QMG_F32), QMG_EDTYPE,
              "prolong: precision must be F64 or the F32 inner precision");
    const void* P = prec == QMG_F64 ? h.P64.p : h.Pin.p;
    const size_t n = size_t(nrhs) * 12 * h.g.V;
    DevBuf nat(n * prec_bytes(prec));
    launch_prolong(prec, h, P, coarse_in, nat.p, nrhs, stream);
    launch_unpack_spinor(nat.p, prec, fine_out, prec, h.g.V, nrhs, stream);
    QMG_HIP(hipStreamSynchronize(stream));
  });
}

qmg_status qmg_restrict(const qmg_mg* mg, const void* fine_in, void* coarse_out, int32_t nrhs, qmg_prec prec,
                        hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(fine_in, "fine_in");
    check_ptr(coarse_out, "coarse_out");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    const HierarchyDev& h = mg->h;
    QMG_CHECK(prec == QMG_F64 || (prec == h.inner && prec == QMG_F32), QMG_EDTYPE,
              "restrict: precision must be F64 or the F32 inner precision");
    const void* P = prec == QMG_F64 ? h.P64.p : h.Pin.p;
    const size_t n = size_t(nrhs) * 12 * h.g.V;
    DevBuf nat(n * prec_bytes(prec));
    launch_pack_spinor(fine_in, prec, nat.p, prec, h.g.V, nrhs, stream);
    launch_restrict(prec, h, P, nat.p, coarse_out, nrhs, stream);
    QMG_HIP(hipStreamSynchronize(stream));
  });
}

qmg_status qmg_coarse_apply(const qmg_mg* mg, const void* in, void* out, int32_t nrhs, qmg_prec prec,
                            hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(in, "in");
    check_ptr(out, "out");
    QMG_CHECK(in != out, QMG_EINVAL, "in and out must not alias");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    const HierarchyDev& h = mg->h;
    QMG_CHECK(prec == QMG_F64 || (prec == h.inner && prec == QMG_F32), QMG_EDTYPE,
              "coarse_apply: precision must be F64 or the F32 inner precision");
    launch_coarse_apply(prec, h, prec == QMG_F64 ? h.Y64.p : h.Yin.p, in, out, nrhs, stream);
  });
}

// bytes the outer solver's Krylov bases of one group of right-hand sides may hold (four FP32
// right-hand sides of 32^3 x 64: 26.6 GB)
constexpr size_t kBasisBudget = size_t(28) << 30;

qmg_status qmg_mg_solve(const qmg_mg* mg, const void* b, void* x, int32_t nrhs, double tol, int32_t max_outer,
                        int32_t adjoint, qmg_solve_info* info, hipStream_t stream) {
  bool converged = false;
  std::vector<SolveStats> gss;  // per group of right-hand sides
  int G = 1;
  double tr = 0, el = 0;
  std::vector<double> rel;
  qmg_status rc = guard([&] {
    check_ptr(mg, "mg");
    check_ptr(b, "b");
    check_ptr(x, "x");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    QMG_CHECK(tol > 0 && tol < 1, QMG_EINVAL, "tol must be in (0, 1)");
    QMG_CHECK(max_outer >= 1, QMG_EINVAL, "max_outer must be >= 1");
    const HierarchyDev& h = mg->h;
    const auto t0 = Clock::now();
    const size_t len = size_t(12) * h.g.V, n = len * nrhs;
    DevBuf b64(n * sizeof(double2)), x64(n * sizeof(double2)), r64(n * sizeof(double2));
    launch_pack_spinor(b, QMG_F64, b64.p, QMG_F64, h.g.V, nrhs, stream);
    launch_pack_spinor(x, QMG_F64, x64.p, QMG_F64, h.g.V, nrhs, stream);
    if (adjoint) {
      gamma5_f64(b64.p, h.g.V, nrhs, stream);
      gamma5_f64(x64.p, h.g.V, nrhs, stream);
    }
    {
      const double bn = host_norm2(b64.p, n, stream);
      QMG_CHECK(std::isfinite(bn), QMG_ENONFINITE, "right-hand side has non-finite entries");
    }
    // The right-hand sides are solved in groups whose outer-solver bases (restart + 1 basis
    // vectors and restart preconditioned ones, in the outer solver's type) fit kBasisBudget, one
    // group after another; every right-hand side has its own Krylov spaces, and a group iterates
    // until its slowest member has converged.
    const size_t per_rhs = size_t(2 * 16 + 1) * len * (h.inner == QMG_F64 ? sizeof(double2) : sizeof(float2));
    G = int(std::max<size_t>(1, std::min<size_t>(size_t(nrhs), kBasisBudget / per_rhs)));
    converged = true;
    for (int g0 = 0; g0 < nrhs; g0 += G) {
      const int ng = std::min(G, nrhs - g0);
      void* bg = b64.as<double2>() + size_t(g0) * len;
      void* xg = x64.as<double2>() + size_t(g0) * len;
      gss.emplace_back();
      SolveStats& ss = gss.back();
      bool c = false;
      if (h.inner == QMG_F64) solve_f64(h, bg, xg, ng, tol, max_outer, false, stream, ss, c);
      else if (h.inner == QMG_F32) solve_mixed<float2>(h, bg, xg, ng, tol, max_outer, stream, ss, c);
      else if (h.inner == QMG_BF16) solve_mixed<cbf16>(h, bg, xg, ng, tol, max_outer, stream, ss, c);
      else solve_mixed<chalf>(h, bg, xg, ng, tol, max_outer, stream, ss, c);
      converged = converged && c;
    }
    // true residual in FP64
    WilsonOp D(h.g, QMG_F64, h.U64.p, h.A64.p);
    D.apply(x64.p, r64.p, nrhs, stream);
    Blas<double2>::axpby(1.0, b64.p, -1.0, r64.p, n, stream);
    RedWork rw;
    DevBuf nr(2 * nrhs * sizeof(double));
    Blas<double2>::norm2(r64.p, len, nrhs, nr.as<double>(), rw, stream);
    Blas<double2>::norm2(b64.p, len, nrhs, nr.as<double>() + nrhs, rw, stream);
    std::vector<double> hn(2 * nrhs);
    QMG_HIP(hipMemcpyAsync(hn.data(), nr.p, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, stream));
    QMG_HIP(hipStreamSynchronize(stream));
    rel.resize(nrhs);
    for (int i = 0; i < nrhs; ++i) {
      rel[i] = hn[nrhs + i] > 0 ? std::sqrt(hn[i] / hn[nrhs + i]) : 0.0;
      tr = std::max(tr, rel[i]);
    }
    QMG_CHECK(std::isfinite(tr), QMG_ENONFINITE, "non-finite final residual");
    if (adjoint) gamma5_f64(x64.p, h.g.V, nrhs, stream);
    launch_unpack_spinor(x64.p, QMG_F64, x, QMG_F64, h.g.V, nrhs, stream);
    QMG_HIP(hipStreamSynchronize(stream));
    el = secs(t0, Clock::now());
    QMG_CHECK(tr <= tol, QMG_ENOCONV, "solve stopped at relative residual %.3e > tol %.3e", tr, tol);
  });
  if (info) {
    for (int i = 0; i < nrhs; ++i) {
      const size_t gi = size_t(i / G);
      const SolveStats ss = gi < gss.size() ? gss[gi] : SolveStats{};
      info[i].outer_iters = int(ss.outer);
      info[i].refinements = int(ss.refinements);
      info[i].coarse_iters = int(ss.coarse);
      info[i].smoother_iters = int(ss.smooth);
      info[i].precision_escalations = int(ss.escalations);
      info[i].true_rel_res = i < int(rel.size()) ? rel[i] : tr;
      info[i].seconds = el;
      info[i].coarse2_iters = int(ss.iters[2]);
      info[i].smoother1_iters = int(ss.smooths[1]);
      info[i].coarse3_iters = int(ss.iters[3]);
      info[i].smoother2_iters = int(ss.smooths[2]);
    }
  }
  return rc;
}

qmg_status qmg_link_force(const qmg_lattice* lat, const void* xv, const void* lam, void* dU, int32_t nrhs,
                          hipStream_t stream) {
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(xv, "x");
    check_ptr(lam, "lambda");
    check_ptr(dU, "dU");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    Geom g = make_geom(lat);
    launch_link_force(g, xv, lam, dU, nrhs, stream);
  });
}

qmg_status qmg_random_test_vectors(const qmg_lattice* lat, uint64_t seed, int32_t v0, int32_t n, void* out,
                                   hipStream_t stream) {
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(out, "out");
    QMG_CHECK(n >= 1 && v0 >= 0, QMG_EINVAL, "need n >= 1 and v0 >= 0");
    Geom g = make_geom(lat);
    DevBuf nat(size_t(n) * 12 * g.V * sizeof(double2));
    launch_philox_native(g, seed, v0, n, nat.p, stream);
    launch_unpack_spinor(nat.p, QMG_F64, out, QMG_F64, g.V, n, stream);
    QMG_HIP(hipStreamSynchronize(stream));
  });
}

qmg_status qmg_smooth(const qmg_lattice* lat, const void* U, const void* phi, void* psi, int32_t nrhs,
                      int32_t n_iter, qmg_prec prec, hipStream_t stream) {
  return guard([&] {
    check_ptr(lat, "lat");
    check_ptr(U, "U");
    check_ptr(phi, "phi");
    check_ptr(psi, "psi");
    QMG_CHECK(nrhs >= 1 && n_iter >= 0, QMG_EINVAL, "need nrhs >= 1, n_iter >= 0");
    QMG_CHECK(prec == QMG_F64 || prec == QMG_F32, QMG_EDTYPE, "smooth: precision must be F64 or F32");
    Geom g = make_geom(lat);
    DevBuf Un(size_t(36) * g.V * prec_bytes(prec)), ph(size_t(nrhs) * 12 * g.V * sizeof(double2));
    launch_pack_gauge(U, Un.p, prec, g.V, stream);
    launch_pack_spinor(phi, QMG_F64, ph.p, QMG_F64, g.V, nrhs, stream);
    DevBuf b_in, x_in, tmp64;
    if (prec == QMG_F64) {
      Gmres<double2> gm;
      smooth_native<double2>(g, Un.p, nullptr, ph.p, nrhs, n_iter, stream, gm, b_in, x_in, tmp64);
    } else {
      Gmres<float2> gm;
      smooth_native<float2>(g, Un.p, nullptr, ph.p, nrhs, n_iter, stream, gm, b_in, x_in, tmp64);
    }
    launch_unpack_spinor(ph.p, QMG_F64, psi, QMG_F64, g.V, nrhs, stream);
    QMG_HIP(hipStreamSynchronize(stream));
  });
}

qmg_status qmg_mg_query(const qmg_mg* mg, int32_t* coarse_dims, int32_t* n_agg, int32_t* rank) {
  return guard([&] {
    check_ptr(mg, "mg");
    if (coarse_dims)
      for (int q = 0; q < 4; ++q) coarse_dims[q] = mg->h.blk.cL[q];
    if (n_agg) *n_agg = mg->h.blk.d;
    if (rank) *rank = mg->h.k;
  });
}

qmg_status qmg_mg_get_prolongator(const qmg_mg* mg, void* P, double* sigma, hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    if (P) launch_export_P(mg->h, P, stream);
    if (sigma) std::memcpy(sigma, mg->h.sigma.data(), mg->h.sigma.size() * sizeof(double));
    QMG_HIP(hipStreamSynchronize(stream));
  });
}

qmg_status qmg_mg_get_coarse(const qmg_mg* mg, void* Y, hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(Y, "Y");
    launch_export_Y(mg->h, Y, stream);
    QMG_HIP(hipStreamSynchronize(stream));
  });
}

qmg_status qmg_mg_setup_times(const qmg_mg* mg, double* t) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(t, "t");
    t[0] = mg->h.t_smooth;
    t[1] = mg->h.t_svd;
    t[2] = mg->h.t_coarse;
    t[3] = mg->h.t_total;
  });
}

qmg_status qmg_timing_enable(int32_t on) {
  return guard([&] {
    QMG_CHECK(on >= 0, QMG_EINVAL, "timing_enable: on must be >= 0");
    timing_enable(on);
  });
}

qmg_status qmg_timing_query(const char* family, int64_t* launches, double* total_ms, double* algo_bytes,
                            double* algo_flops) {
  return guard([&] {
    check_ptr(family, "family");
    check_ptr(launches, "launches");
    check_ptr(total_ms, "total_ms");
    double b = 0, f = 0;
    timing_query(family, launches, total_ms, &b, &f);
    if (algo_bytes) *algo_bytes = b;
    if (algo_flops) *algo_flops = f;
  });
}

qmg_status qmg_mg_set_cycle(qmg_mg* mg, int32_t coarse_steps, int32_t graph) {
  return guard([&] {
    check_ptr(mg, "mg");
    QMG_CHECK(coarse_steps >= 0 && coarse_steps <= 63, QMG_EINVAL, "coarse_steps must be in [0, 63]");
    QMG_CHECK(graph == 0 || graph == 1, QMG_EINVAL, "graph must be 0 or 1");
    QMG_CHECK(!graph || coarse_steps > 0, QMG_EINVAL, "a captured K-cycle needs coarse_steps > 0");
    QMG_CHECK(coarse_steps == 0 || mg->h.levels.empty(), QMG_EINVAL,
              "with further levels the K-cycle is host-checked (coarse_steps must be 0)");
    mg->h.cycle_steps = coarse_steps;
    mg->h.cycle_graph = graph != 0;
  });
}

qmg_status qmg_mg_set_smoother(qmg_mg* mg, int32_t eo, hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    QMG_CHECK(eo >= 0 && eo <= 2, QMG_EINVAL, "eo must be 0, 1 or 2");
    HierarchyDev& h = mg->h;
    if (!eo) {
      h.eo_smoother = 0;
      return;
    }
    const Geom& g = h.g;
    QMG_CHECK(g.L[0] % 2 == 0 && g.L[1] % 2 == 0 && g.L[2] % 2 == 0 && g.L[3] % 2 == 0, QMG_ESHAPE,
              "even-odd preconditioning needs every extent even");
    const size_t n = size_t(36) * g.V;
    if (!h.Ueo[0].p) {
      // SU(3) links (to 1e-12) are stored as their first two rows: the hop kernels rebuild the
      // third, and read two thirds of the link bytes
      h.eo_ne = launch_su3_row_defect(g, h.U64.p, stream) < 1e-12 ? 6 : 9;
    }
    for (int w = 0; w < (h.inner != QMG_F64 ? 2 : 1); ++w) {
      const qmg_prec p = w ? h.inner : QMG_F64;
      if (!h.Ueo[w].p) {
        h.Ueo[w].alloc(size_t(4) * h.eo_ne * g.V * prec_bytes(p));
        launch_eo_gauge_from_native(g, h.U64.p, h.Ueo[w].p, p, stream, h.eo_ne);
      }
      if (h.A64.p && !h.Aeo[w].p) {
        h.Aeo[w].alloc(n * prec_bytes(p));
        h.Aieo[w].alloc(n * prec_bytes(p));
        launch_eo_site_term(g, h.A64.p, h.Aeo[w].p, h.Aieo[w].p, p, stream);
      }
    }
    QMG_HIP(hipStreamSynchronize(stream));
    h.eo_smoother = eo;
  });
}

qmg_status qmg_mg_set_coarse_eo(qmg_mg* mg, int32_t on, hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    QMG_CHECK(on == 0 || on == 1, QMG_EINVAL, "on must be 0 or 1");
    HierarchyDev& h = mg->h;
    h.coarse_eo = 0;
    if (!on) {  // the blocks belong to the current D_c only: rebuilt when switched on again
      h.Yh64.release();
      h.Yhin.release();
      return;
    }
    QMG_CHECK(h.levels.empty(), QMG_EINVAL, "the even-odd coarse solve needs a two-level hierarchy");
    if (!h.ceo_tab.p) build_coarse_eo_tables(h, stream);
    build_coarse_eo_blocks(h, stream);  // always from the current D_c; releases them on failure
    QMG_HIP(hipStreamSynchronize(stream));
    h.coarse_eo = 1;
  });
}

qmg_status qmg_coarse_schur_apply(const qmg_mg* mg, const void* in, void* out, int32_t nrhs, qmg_prec prec,
                                  hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(in, "in");
    check_ptr(out, "out");
    QMG_CHECK(in != out, QMG_EINVAL, "in and out must not alias");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    const HierarchyDev& h = mg->h;
    QMG_CHECK(h.coarse_eo, QMG_EINVAL, "coarse_schur_apply: the even-odd coarse operator is not set up");
    QMG_CHECK(prec == QMG_F64 || (prec == h.inner && prec == QMG_F32), QMG_EDTYPE,
              "coarse_schur_apply: precision must be F64 or the F32 inner precision");
    const bool d64 = prec == QMG_F64;
    CoarseSchurOp A(h, prec, d64 ? h.Y64.p : h.Yin.p, d64 ? h.Yh64.p : h.Yhin.p);
    A.apply(in, out, nrhs, stream);
    QMG_HIP(hipStreamSynchronize(stream));  // A's work buffer is released on return
  });
}

// ---------------------------------------------------------------------------------------
// qmg_coarse_schur_apply_noalloc: the Schur apply with its intermediate half vector (the
// Yhat-hops of the input on the odd colour) in a file-scope device array instead of an
// allocated buffer.  The array's host-side name is no device address: its address on each
// device is taken once, on the first call on that device, and only that address is passed to
// the kernels.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(QMG_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_on_current_device() {
  int dev = 0;
  QMG_HIP(hipGetDevice(&dev));
  QMG_CHECK(dev >= 0 && dev < kMaxDevices, QMG_EINVAL, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    QMG_CHECK(e == hipSuccess && ptr, QMG_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
              hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

qmg_status qmg_coarse_schur_apply_noalloc(const qmg_mg* mg, const void* in, void* out, int32_t nrhs, qmg_prec prec,
                                          hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(in, "in");
    check_ptr(out, "out");
    QMG_CHECK(in != out, QMG_EINVAL, "in and out must not alias");
    QMG_CHECK(nrhs >= 1, QMG_EINVAL, "nrhs must be >= 1");
    const HierarchyDev& h = mg->h;
    QMG_CHECK(h.coarse_eo, QMG_EINVAL, "coarse_schur_apply_noalloc: the even-odd coarse operator is not set up");
    QMG_CHECK(prec == QMG_F64 || (prec == h.inner && prec == QMG_F32), QMG_EDTYPE,
              "coarse_schur_apply_noalloc: precision must be F64 or the F32 inner precision");
    const size_t need = size_t(nrhs) * size_t(h.k) * size_t(h.blk.d) * prec_bytes(prec);
    QMG_CHECK(need <= kNoAllocScratchBytes, QMG_ESHAPE,
              "coarse_schur_apply_noalloc: %d right-hand sides of %d half coarse entries need %zu bytes of scratch, "
              "above the library's fixed %zu bytes (use qmg_coarse_schur_apply or fewer right-hand sides)",
              nrhs, h.k * h.blk.d, need, kNoAllocScratchBytes);
    void* tmp = scratch_on_current_device();
    const bool d64 = prec == QMG_F64;
    const void* Y = d64 ? h.Y64.p : h.Yin.p;
    const void* Yh = d64 ? h.Yh64.p : h.Yhin.p;
    // the first launch writes every entry of the intermediate, so nothing needs clearing
    launch_coarse_eo_apply(prec, h, 1, Yh, nullptr, nullptr, in, tmp, nrhs, 1.0, stream);
    launch_coarse_eo_apply(prec, h, 0, Y, nullptr, in, tmp, out, nrhs, -1.0, stream);
  });
}

qmg_status qmg_coarse_eo_solve(const qmg_mg* mg, const void* b, void* x, int32_t nrhs, double tol, int32_t max_iter,
                               int32_t* iters, hipStream_t stream) {
  return guard([&] {
    check_ptr(mg, "mg");
    check_ptr(b, "b");
    check_ptr(x, "x");
    check_ptr(iters, "iters");
    QMG_CHECK(b != x, QMG_EINVAL, "b and x must not alias");
    QMG_CHECK(nrhs >= 1 && max_iter >= 1, QMG_EINVAL, "need nrhs >= 1, max_iter >= 1");
    QMG_CHECK(tol > 0 && tol < 1, QMG_EINVAL, "tol must be in (0, 1)");
    const HierarchyDev& h = mg->h;
    QMG_CHECK(h.coarse_eo, QMG_EINVAL, "coarse_eo_solve: the even-odd coarse operator is not set up");
    CoarseSchurOp A(h, QMG_F64, h.Y64.p, h.Yh64.p);
    Gmres<double2> gm;
    DevBuf work[6];
    auto res = coarse_eo_solve<double2>(h, A, gm, b, x, nrhs, max_iter, tol, work, stream);
    QMG_HIP(hipStreamSynchronize(stream));
    *iters = res.iters;
    QMG_CHECK(res.converged, QMG_ENOCONV, "coarse_eo_solve: no convergence in %d steps", max_iter);
  });
}

qmg_status qmg_timing_calls(const char* family, int64_t* calls) {
  return guard([&] {
    check_ptr(family, "family");
    check_ptr(calls, "calls");
    *calls = timing_calls(family);
  });
}

qmg_status qmg_timing_list(char* buf, int32_t len) {
  return guard([&] {
    check_ptr(buf, "buf");
    QMG_CHECK(len >= 1, QMG_EINVAL, "len must be >= 1");
    const std::string names = timing_families();
    QMG_CHECK(names.size() + 1 <= size_t(len), QMG_ESHAPE, "timing_list: %zu bytes needed", names.size() + 1);
    std::memcpy(buf, names.c_str(), names.size() + 1);
  });
}

qmg_status qmg_memory_trim(void) {
  return guard([&] { dev_trim(); });
}

qmg_status qmg_memory_cached(int64_t* bytes) {
  return guard([&] {
    check_ptr(bytes, "bytes");
    *bytes = int64_t(dev_cached());
  });
}

qmg_status qmg_autotune(int32_t on) {
  return guard([&] { tune_enable(on != 0); });
}

qmg_status qmg_set_dslash_variant(int32_t v) {
  return guard([&] {
    const int cm = v >= 10000 ? 1 : 0, u = v % 10000;  // 10000 + a t-walking code: t-chunk-major order
    const int z = u / 1000, nr = (u % 1000) / 100, tch = u % 100;
    const bool tw = u > 100 && z <= 1 && (nr == 2 || nr == 3) && (tch == 2 || tch == 4 || tch == 8);
    const bool hop_nr = !cm && v >= 501 && v <= 504;  // even-odd hop: 1 .. 4 right-hand sides per thread
    auto p2 = [](int q) { return q == 1 || q == 2 || q == 4 || q == 8; };
    const bool hop_order = !cm && (v == 700 || (v > 700 && v < 800 && p2((v / 10) % 10) && p2(v % 10)));
    const bool plain = !cm && (v == 0 || v == 1 || v == 16 || v == 32 || v == 64);
    QMG_CHECK(v < 20000 && (tw || hop_nr || hop_order || plain || u == 2 || u == 4 || u == 8), QMG_EINVAL,
              "dslash variant must be 0, 1, 2, 4, 8, 16, 32, 64, an even-odd hop code 500 + NR (NR in 1..4) or "
              "7ZT (tile order over patches of Z x T planes, Z and T in {1, 2, 4, 8}; 700 lexicographic), a "
              "multi-rhs t-walking code 1000 z + 100 NR + TCH (z in {0,1}, NR in {2,3}, TCH in {2,4,8}), or "
              "10000 + a t-walking code (2, 4, 8 or multi-rhs) for the t-chunk-major workgroup order");
    set_dslash_variant(v);
  });
}

qmg_status qmg_tune_save(const char* path) {
  return guard([&] {
    check_ptr(path, "path");
    QMG_CHECK(tune_save(path) == 0, QMG_EINVAL, "cannot write tuning cache %s", path);
  });
}

qmg_status qmg_tune_load(const char* path) {
  return guard([&] {
    check_ptr(path, "path");
    QMG_CHECK(tune_load(path) >= 0, QMG_EINVAL, "cannot read tuning cache %s", path);
  });
}

void qmg_mg_destroy(qmg_mg* mg) { delete mg; }

const char* qmg_last_error(void) { return last_error_ptr(); }

const char* qmg_version(void) { return "qmg 0.1 (gfx950)"; }

}  // extern "C"
