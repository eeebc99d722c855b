// Multigrid over many independent small lattices at once (each with its own extents, mass and
// gauge field; one aggregate shape and rank for all): the setup of Algorithm 4 with the
// streaming SVD of Algorithm 3 and the K-cycle solve of every lattice run as shared launches.
//
// Layouts: the fine fields of all lattices are zero-padded to a common volume Vpad and stacked,
// lattice-major: gauge [l][4][9][Vpad], spinors [l][nr][12][Vpad]; the coarse vectors likewise
// to a common aggregate count dmax: [l][nr][dmax][2k].  Every (lattice, right-hand side) pair is
// one column of the Krylov solvers, so inner products, norms and convergence tests are per
// lattice (the padding is zero and stays zero), while every operator, transfer and vector kernel
// is one launch over all lattices.  The aggregates of all lattices are numbered globally
// (lattice-major, J = aoff[l] + j): the prolongator [J][2][k][N] and the coarse blocks
// [J][9][2k][2k] are the per-lattice arrays of a single hierarchy concatenated, so the streaming
// SVD runs over all of them in its usual launches.
//
// The Galerkin blocks Y_s(j) = P_j^dag D P_{j+s} (Eq. (5)) are formed directly from the
// prolongator and the links, one workgroup per (aggregate, slot), in FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <cstring>
#include <memory>
#include <vector>

#include "krylov.hpp"
#include "mg.hpp"
#include "timing.hpp"

struct qmg_batch;

namespace qmg {

namespace {

constexpr int kMaxRank = 32;  // 2k <= 64 coarse components per aggregate

// canonical FP64 gauge [4][V][3][3] -> padded native [4][9][Vpad]
__global__ void k_b_pack_gauge(const double2* __restrict__ canon, double2* __restrict__ out, int V, int Vpad) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  const int me = blockIdx.y;  // mu * 9 + e
  if (site >= Vpad) return;
  const int mu = me / 9, e = me - 9 * mu;
  out[size_t(me) * Vpad + site] = site < V ? canon[(size_t(mu) * V + site) * 9 + e] : make_double2(0.0, 0.0);
}

// canonical FP64 spinors [nrhs][V][12] <-> padded native [nrhs][12][Vpad]
__global__ void k_b_pack_spinor(const double2* __restrict__ canon, double2* __restrict__ out, int V, int Vpad) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  const int rc = blockIdx.y;  // rhs * 12 + comp
  if (site >= Vpad) return;
  const int rhs = rc / 12, c = rc - 12 * rhs;
  out[size_t(rc) * Vpad + site] = site < V ? canon[(size_t(rhs) * V + site) * 12 + c] : make_double2(0.0, 0.0);
}
__global__ void k_b_unpack_spinor(const double2* __restrict__ nat, double2* __restrict__ canon, int V, int Vpad) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  const int rc = blockIdx.y;
  if (site >= V) return;
  const int rhs = rc / 12, c = rc - 12 * rhs;
  canon[(size_t(rhs) * V + site) * 12 + c] = nat[size_t(rc) * Vpad + site];
}

// chiral split and block gather of r test vectors of every lattice: blocks [(J, alpha)][r][N],
// row = s6 * nd + ib (the row order of the single-lattice gather)
__global__ void k_b_gather(const double2* __restrict__ fine, double2* __restrict__ blocks, const int* __restrict__ gsite,
                           const int* __restrict__ jinfo, int nd, int N, int r, int Vpad) {
  const int row = blockIdx.z * 256 + threadIdx.x;
  const int v = blockIdx.y, ja = blockIdx.x;  // the (aggregate, chirality) count may exceed 65535
  if (row >= N) return;
  const int J = ja >> 1, a = ja & 1, l = jinfo[2 * J];
  const int s6 = row / nd, ib = row - s6 * nd;
  const int site = gsite[size_t(J) * nd + ib];
  blocks[(size_t(ja) * r + v) * N + row] = fine[((size_t(l) * r + v) * 12 + 6 * a + s6) * Vpad + site];
}

// fine = P coarse: one thread per (row of (J, alpha), rhs); fine padding is not touched
template <class S>
__global__ __launch_bounds__(256) void k_b_prolong(const S* __restrict__ P, const S* __restrict__ vc,
                                                   S* __restrict__ fine, const int* __restrict__ gsite,
                                                   const int* __restrict__ jinfo, int nd, int N, int k, int dmax,
                                                   int Vpad, int nrhs) {
  using C = ctype<S>;
  const int row = blockIdx.y * 256 + threadIdx.x;
  const int ja = blockIdx.x, rhs = blockIdx.z;  // the (aggregate, chirality) count may exceed 65535
  if (row >= N) return;
  const int J = ja >> 1, a = ja & 1, l = jinfo[2 * J], j = jinfo[2 * J + 1];
  const size_t col = size_t(l) * nrhs + rhs;
  const S* Pc = P + size_t(ja) * k * N;
  const S* v = vc + (col * dmax + j) * 2 * k + a * k;
  cplx<C> acc = {C(0), C(0)};
  for (int i = 0; i < k; ++i) acc += ldc(Pc, size_t(i) * N + row) * ldc(v, i);
  const int s6 = row / nd, ib = row - s6 * nd;
  stc(fine, (col * 12 + 6 * a + s6) * Vpad + gsite[size_t(J) * nd + ib], acc);
}

// coarse = P^dag fine: one wavefront per ((J, alpha), rhs); the block's N fine entries are staged
// in LDS and lane i < k forms component i
template <class S>
__global__ __launch_bounds__(64) void k_b_restrict(const S* __restrict__ P, const S* __restrict__ fine,
                                                   S* __restrict__ vc, const int* __restrict__ gsite,
                                                   const int* __restrict__ jinfo, int nd, int N, int k, int dmax,
                                                   int Vpad, int nrhs) {
  using C = ctype<S>;
  extern __shared__ unsigned char smem[];
  cplx<C>* psi = reinterpret_cast<cplx<C>*>(smem);  // [N]
  const int ja = blockIdx.x, rhs = blockIdx.y;
  const int J = ja >> 1, a = ja & 1, l = jinfo[2 * J], j = jinfo[2 * J + 1];
  const size_t col = size_t(l) * nrhs + rhs;
  for (int row = threadIdx.x; row < N; row += 64) {
    const int s6 = row / nd, ib = row - s6 * nd;
    psi[row] = ldc(fine, (col * 12 + 6 * a + s6) * Vpad + gsite[size_t(J) * nd + ib]);
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i >= k) return;
  const S* Pc = P + (size_t(ja) * k + i) * N;
  cplx<C> acc = {C(0), C(0)};
  for (int row = 0; row < N; ++row) acc += cmul_conj(ldc(Pc, row), psi[row]);
  stc(vc, (col * dmax + j) * 2 * k + a * k + i, acc);
}

// out = D_c in on the padded coarse columns: one workgroup of 64 threads per (64 / 2k aggregate
// slots, column), so that every lane works at small ranks (2k = 16: four aggregates); the nine
// inputs of each aggregate (self, then the eight neighbours) are staged in LDS, thread
// (aggregate, row) forms one output component; padding aggregates give zeros
template <class S>
__global__ __launch_bounds__(64) void k_b_coarse_apply(const S* __restrict__ Y, const S* __restrict__ in,
                                                       S* __restrict__ out, const int* __restrict__ cnb,
                                                       const int* __restrict__ jinfo, const int* __restrict__ dl,
                                                       const int* __restrict__ aoff, int m, int dmax, int nrhs) {
  using C = ctype<S>;
  __shared__ cplx<C> v[9 * 64];  // [aggregate in workgroup][slot][component], apw * m <= 64
  const int apw = 64 / m;        // aggregates per workgroup
  const int jb = blockIdx.x * apw, col = blockIdx.y, l = col / nrhs;
  const int nd = dl[l];
  for (int t = threadIdx.x; t < apw * 9 * m; t += 64) {
    const int aa = t / (9 * m), rem = t - aa * 9 * m;
    const int sl = rem / m, c = rem - sl * m, jj = jb + aa;
    if (jj >= nd) continue;
    const int jn = sl == 0 ? jj : jinfo[2 * cnb[size_t(aoff[l] + jj) * 8 + sl - 1] + 1];
    v[t] = ldc(in, (size_t(col) * dmax + jn) * m + c);
  }
  __syncthreads();
  const int a = threadIdx.x / m, row = threadIdx.x - a * m, j = jb + a;
  if (a >= apw || j >= dmax) return;
  const size_t ob = (size_t(col) * dmax + j) * m;
  if (j >= nd) {
    stc(out, ob + row, cplx<C>{C(0), C(0)});
    return;
  }
  cplx<C> acc = {C(0), C(0)};
  const S* YJ = Y + size_t(aoff[l] + j) * 9 * m * m;
  const cplx<C>* va = v + size_t(a) * 9 * m;
  for (int sl = 0; sl < 9; ++sl)
    for (int c = 0; c < m; ++c) acc += ldc(YJ, (size_t(sl) * m + c) * m + row) * va[sl * m + c];
  stc(out, ob + row, acc);
}

// Galerkin blocks directly (Eq. (5)): Y_s(J) = sum over the sites x of J of P_J(x)^dag W_s(x),
// W_s(x) = sum of H P_J'(x') over the hops x -> x' of slot s, H the hop term of D
// (-1/2 c_mu s_mu (1 -+ gamma_mu) (x) U); slot 0 holds the diagonal term and the hops that stay
// inside the block, slot 1 + dir the hops in direction dir that leave it (every coarse extent is
// >= 3, so such a hop lands in the neighbour aggregate cnb[J][dir]).  One workgroup per
// (aggregate J, slot s) takes the sites of J in batches of nb = 256 / 2k: thread (site, column c)
// forms column c of W_s(x) (12 x 2k) in LDS, then thread (row, col) adds
// sum over the batch's sites and the six components of row's chirality of conj(P_J(x)) W_s(x).
// P_J(x) is the 12 x 2k matrix of the rows of site x: chirality alpha's columns are nonzero on its
// six components only.
__constant__ double2 c_bgamma[4][16];  // gamma_mu (chiral basis), row-major 4 x 4

__device__ inline cplx<double> b_p(const double2* __restrict__ P, int J, int comp, int col, int ib, int k, int nd,
                                   int N) {
  const int a = col / k, i = col - a * k;
  if (comp / 6 != a) return {0.0, 0.0};
  const double2 v = P[((size_t(J) * 2 + a) * k + i) * N + (comp - 6 * a) * nd + ib];
  return {v.x, v.y};
}

template <int KPER>  // (row, col) pairs per thread: ceil((2k)^2 / 256)
__global__ __launch_bounds__(256) void k_b_galerkin(const double2* __restrict__ U, const double2* __restrict__ P,
                                                    double2* __restrict__ Y, const int* __restrict__ gsite,
                                                    const int* __restrict__ jinfo, const int* __restrict__ cnb,
                                                    const int* __restrict__ aoff, const BatchLattice* __restrict__ lat,
                                                    int b0, int b1, int b2, int b3, int nd, int N, int k) {
  __shared__ cplx<double> W[256 * 12];  // [site in batch][component][column]
  const int J = blockIdx.x, s = blockIdx.y, m = 2 * k, tid = threadIdx.x;
  const int nb = 256 / m;
  const int l = jinfo[2 * J];
  const DslashArgs& a = lat[l].a;
  const int L[4] = {a.L[0], a.L[1], a.L[2], a.L[3]}, bb[4] = {b0, b1, b2, b3};
  const int Vpad = a.V;
  const double2* Ul = U + size_t(l) * 36 * Vpad;
  cplx<double> acc[KPER];
  for (int q = 0; q < KPER; ++q) acc[q] = {0.0, 0.0};
  for (int ib0 = 0; ib0 < nd; ib0 += nb) {
    const int nbs = min(nb, nd - ib0);
    __syncthreads();  // the previous batch's W is no longer read
    if (tid < nbs * m) {
      const int sb = tid / m, col = tid - sb * m, ib = ib0 + sb;
      const int x = gsite[size_t(J) * nd + ib];
      int c[4], rem = x;
      for (int q = 0; q < 4; ++q) {
        c[q] = rem % L[q];
        rem /= L[q];
      }
      cplx<double> w[12];
      for (int comp = 0; comp < 12; ++comp)
        w[comp] = s == 0 ? a.diag_d * b_p(P, J, comp, col, ib, k, nd, N) : cplx<double>{0.0, 0.0};
      for (int dir = (s == 0 ? 0 : s - 1); dir < (s == 0 ? 8 : s); ++dir) {
        const int mu = dir & 3;
        const bool fwd = dir < 4;
        int cn[4] = {c[0], c[1], c[2], c[3]};
        cn[mu] = (cn[mu] + (fwd ? 1 : -1) + L[mu]) % L[mu];
        int cj[4], ci[4];
        for (int q = 0; q < 4; ++q) {
          cj[q] = cn[q] / bb[q];
          ci[q] = cn[q] - cj[q] * bb[q];
        }
        const int Jn = aoff[l] + cj[0] + (L[0] / bb[0]) * (cj[1] + (L[1] / bb[1]) * (cj[2] + (L[2] / bb[2]) * cj[3]));
        if (s == 0 ? Jn != J : (Jn == J || Jn != cnb[size_t(J) * 8 + dir])) continue;
        const int ibn = ci[0] + bb[0] * (ci[1] + bb[1] * (ci[2] + bb[2] * ci[3]));
        const int xn = cn[0] + L[0] * (cn[1] + L[1] * (cn[2] + L[2] * cn[3]));
        // boundary sign: t-hops across t = Lt - 1 <-> 0 with antiperiodic time
        const bool wrap = mu == 3 && ((fwd && c[3] == L[3] - 1) || (!fwd && c[3] == 0));
        const double coef = -0.5 * a.cw_d[mu] * ((wrap && a.bc_t < 0) ? -1.0 : 1.0);
        // spin: h = (1 -+ gamma_mu) v; colour: U_mu(x) h (forward) or U_mu(x - mu)^dag h (backward)
        cplx<double> v[12], h[12];
        for (int comp = 0; comp < 12; ++comp) v[comp] = b_p(P, Jn, comp, col, ibn, k, nd, N);
        const double sg = fwd ? -1.0 : 1.0;
        for (int sp = 0; sp < 4; ++sp)
          for (int cc = 0; cc < 3; ++cc) {
            cplx<double> t = v[3 * sp + cc];
            for (int tp = 0; tp < 4; ++tp) {
              const double2 g = c_bgamma[mu][sp * 4 + tp];
              if (g.x != 0.0 || g.y != 0.0) t += sg * (cplx<double>{g.x, g.y} * v[3 * tp + cc]);
            }
            h[3 * sp + cc] = t;
          }
        const int ls = fwd ? x : xn;
        for (int ca = 0; ca < 3; ++ca)
          for (int cb = 0; cb < 3; ++cb) {
            const double2 ut = fwd ? Ul[(size_t(mu) * 9 + 3 * ca + cb) * Vpad + ls]
                                   : Ul[(size_t(mu) * 9 + 3 * cb + ca) * Vpad + ls];
            const cplx<double> u = {ut.x, fwd ? ut.y : -ut.y};
            for (int sp = 0; sp < 4; ++sp) w[3 * sp + ca] += coef * (u * h[3 * sp + cb]);
          }
      }
      for (int comp = 0; comp < 12; ++comp) W[(sb * 12 + comp) * m + col] = w[comp];
    }
    __syncthreads();
    for (int q = 0; q < KPER; ++q) {
      const int t = tid + 256 * q;
      if (t >= m * m) break;
      const int row = t / m, col = t - row * m, ar = row / k, ir = row - ar * k;
      const double2* Pr = P + ((size_t(J) * 2 + ar) * k + ir) * N;
      cplx<double> sum = {0.0, 0.0};
      for (int sb = 0; sb < nbs; ++sb)
        for (int c6 = 0; c6 < 6; ++c6) {
          const double2 pv = Pr[c6 * nd + ib0 + sb];
          sum += cmul_conj(cplx<double>{pv.x, pv.y}, W[(sb * 12 + 6 * ar + c6) * m + col]);
        }
      acc[q] += sum;
    }
  }
  for (int q = 0; q < KPER; ++q) {
    const int t = tid + 256 * q;
    if (t >= m * m) break;
    const int row = t / m, col = t - row * m;
    Y[((size_t(J) * 9 + s) * m + col) * m + row] = make_double2(acc[q].re, acc[q].im);
  }
}

template <class F>
void dispatch_b(qmg_prec p, F&& f) {
  if (p == QMG_F64) f(double2{});
  else f(float2{});
}

}  // namespace

// ---------------------------------------------------------------------------------------
// the many-lattice hierarchy

struct BatchDev {
  int nl = 0, Vpad = 0, k = 0, nd = 0, N = 0, DT = 0, dmax = 0;
  int blk[4] = {1, 1, 1, 1};
  qmg_prec inner = QMG_F32;
  int n_post = 8, coarse_max = 500;
  double coarse_tol = 0.03;
  std::vector<Geom> geo;
  std::vector<int> d, aoff, V;
  DevBuf lat;                 // BatchLattice[nl], a.V = Vpad
  std::vector<BatchLattice> lat_h;  // the same descriptors on the host
  DevBuf Vl, dl, aoffd;       // int[nl]
  DevBuf U64, Uin;            // [l][4][9][Vpad]
  DevBuf gsite, jinfo, cnb;   // [DT][nd], [DT][2] (lattice, local index), [DT][8] (global)
  DevBuf P64, Pin;            // [DT][2][k][N]
  DevBuf Y64, Yin;            // [DT][9][2k][2k] column-major blocks
  DevBuf sigma;               // [DT][2][k]
  std::vector<double> sigma_h;
  double t_smooth = 0, t_svd = 0, t_coarse = 0, t_total = 0;
  size_t fine_len() const { return size_t(12) * Vpad; }
  size_t coarse_len() const { return size_t(2) * k * dmax; }
};

namespace {

// D of every lattice on padded columns (nl * nr columns of 12 Vpad complex numbers)
struct BatchOp : LinOp {
  const BatchDev& b;
  qmg_prec p;
  const void* U;
  const BatchLattice* lat;  // descriptors (default: the lattices' own; the setup's shifted copy)
  BatchOp(const BatchDev& b_, qmg_prec p_, const void* U_, const BatchLattice* lat_ = nullptr)
      : b(b_), p(p_), U(U_), lat(lat_ ? lat_ : b_.lat.as<BatchLattice>()) {}
  void apply(const void* in, void* out, int ncol, hipStream_t st, const int* = nullptr) override {
    const int nr = ncol / b.nl;
    double sites = 0;
    for (int v : b.V) sites += v;
    launch_dslash_padded(p, lat, b.nl, nr, b.Vpad, U, in, out, false, sites * (24.0 * nr + 36.0) * prec_bytes(p),
                         1368.0 * sites * nr, st);
  }
  size_t len() const override { return b.fine_len(); }
  qmg_prec prec() const override { return p; }
};

struct BatchCoarseOp : LinOp {
  const BatchDev& b;
  qmg_prec p;
  const void* Y;
  BatchCoarseOp(const BatchDev& b_, qmg_prec p_, const void* Y_) : b(b_), p(p_), Y(Y_) {}
  void apply(const void* in, void* out, int ncol, hipStream_t st, const int* = nullptr) override {
    const int nr = ncol / b.nl, m = 2 * b.k;
    TimedLaunch tl("batch/coarse_apply", st, double(b.DT) * (9.0 * m * m + m * 2.0 * nr) * prec_bytes(p),
                   8.0 * 9.0 * m * m * b.DT * nr);
    dispatch_b(p, [&](auto tag) {
      using S = decltype(tag);
      launch(k_b_coarse_apply<S>, dim3(unsigned((b.dmax + 64 / m - 1) / (64 / m)), ncol), dim3(64), 0, st,
             static_cast<const S*>(Y),
             static_cast<const S*>(in), static_cast<S*>(out), b.cnb.as<int>(), b.jinfo.as<int>(), b.dl.as<int>(),
             b.aoffd.as<int>(), m, b.dmax, nr);
    });
    QMG_LAUNCH_CHECK();
  }
  size_t len() const override { return b.coarse_len(); }
  qmg_prec prec() const override { return p; }
};

void b_prolong(const BatchDev& b, qmg_prec p, const void* P, const void* vc, void* fine, int nr, hipStream_t st) {
  double sites = 0;
  for (int v : b.V) sites += v;
  TimedLaunch tl("batch/prolong", st, sites * (12.0 * b.k + 12.0 * nr) * prec_bytes(p), 8.0 * 12.0 * b.k * sites * nr);
  dispatch_b(p, [&](auto tag) {
    using S = decltype(tag);
    launch(k_b_prolong<S>, dim3(2 * b.DT, unsigned((b.N + 255) / 256), nr), dim3(256), 0, st, static_cast<const S*>(P),
           static_cast<const S*>(vc), static_cast<S*>(fine), b.gsite.as<int>(), b.jinfo.as<int>(), b.nd, b.N, b.k,
           b.dmax, b.Vpad, nr);
  });
  QMG_LAUNCH_CHECK();
}

// the restricted columns' padding aggregates are cleared first
void b_restrict(const BatchDev& b, qmg_prec p, const void* P, const void* fine, void* vc, int nr, hipStream_t st) {
  double sites = 0;
  for (int v : b.V) sites += v;
  dispatch_b(p, [&](auto tag) {
    using S = decltype(tag);
    Blas<S>::zero(vc, b.coarse_len() * b.nl * nr, st);
    TimedLaunch tl("batch/restrict", st, sites * (12.0 * b.k + 12.0 * nr) * prec_bytes(p),
                   8.0 * 12.0 * b.k * sites * nr);
    launch(k_b_restrict<S>, dim3(2 * b.DT, nr), dim3(64), uint32_t(b.N * sizeof(cplx<ctype<S>>)), st,
           static_cast<const S*>(P), static_cast<const S*>(fine), static_cast<S*>(vc), b.gsite.as<int>(),
           b.jinfo.as<int>(), b.nd, b.N, b.k, b.dmax, b.Vpad, nr);
  });
  QMG_LAUNCH_CHECK();
}

// Galerkin blocks from P and the links (k_b_galerkin), FP64
void b_build_coarse_direct(BatchDev& b, hipStream_t st) {
  // __constant__ memory is per device: upload once on every device the library runs on
  static std::mutex init_mu;
  static bool init[64] = {};
  {
    int dev = 0;
    QMG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> init_lk(init_mu);
    if (dev < 0 || dev >= 64 || !init[dev]) {
      // chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_t = [[0, 1], [1, 0]]
      double2 gm[4][16] = {};
      auto set = [&](int mu, int r, int c, double re, double im) { gm[mu][r * 4 + c] = make_double2(re, im); };
      set(0, 0, 3, 0, -1); set(0, 1, 2, 0, -1); set(0, 2, 1, 0, 1); set(0, 3, 0, 0, 1);
      set(1, 0, 3, -1, 0); set(1, 1, 2, 1, 0); set(1, 2, 1, 1, 0); set(1, 3, 0, -1, 0);
      set(2, 0, 2, 0, -1); set(2, 1, 3, 0, 1); set(2, 2, 0, 0, 1); set(2, 3, 1, 0, -1);
      set(3, 0, 2, 1, 0); set(3, 1, 3, 1, 0); set(3, 2, 0, 1, 0); set(3, 3, 1, 1, 0);
      QMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_bgamma), gm, sizeof(gm)));
      if (dev >= 0 && dev < 64) init[dev] = true;
    }
  }
  const int m = 2 * b.k;
  b.Y64.alloc(size_t(b.DT) * 9 * m * m * sizeof(double2));
  double sites = 0;
  for (int v : b.V) sites += v;
  // bytes: the blocks written, P and the links read once; flops: per site and slot the 6 x m by
  // 6 x m products of each chirality and the hops applied to the 12 x m columns of P
  TimedLaunch tl("batch/coarse_build", st, double(b.DT) * (9.0 * m * m + 6.0 * m * b.nd + 36.0 * b.nd) * 16.0,
                 sites * 9.0 * (48.0 * m * m + 400.0 * m));
  auto go = [&](auto kern) {
    launch(kern, dim3(b.DT, 9), dim3(256), 0, st, b.U64.as<double2>(), b.P64.as<double2>(), b.Y64.as<double2>(),
           b.gsite.as<int>(), b.jinfo.as<int>(), b.cnb.as<int>(), b.aoffd.as<int>(), b.lat.as<BatchLattice>(),
           b.blk[0], b.blk[1], b.blk[2], b.blk[3], b.nd, b.N, b.k);
  };
  // accumulators sized to the block: a fixed 16 pairs per thread spills at small ranks
  if (m <= 16) go(k_b_galerkin<1>);
  else if (m <= 32) go(k_b_galerkin<4>);
  else if (m <= 48) go(k_b_galerkin<9>);
  else go(k_b_galerkin<16>);
  QMG_LAUNCH_CHECK();
}

// K-cycle over all lattices: restrict, coarse GMRES(32) to the coarse tolerance (per column),
// prolong, GMRES(n_post) post-smoothing from the prolonged correction; storage S = outer type
template <class S>
struct BatchKCycle : Precond {
  const BatchDev& b;
  BatchOp& D;
  BatchCoarseOp& Dc;
  const void* P;
  Gmres<S> gc, gf;
  DevBuf rc, ec;
  long coarse_iters = 0, smooth_iters = 0;
  BatchKCycle(const BatchDev& b_, BatchOp& D_, BatchCoarseOp& Dc_, const void* P_) : b(b_), D(D_), Dc(Dc_), P(P_) {}
  void apply(const void* r, void* z, int ncol, hipStream_t st) override {
    constexpr qmg_prec p = StoreTraits<S>::prec;
    const int nr = ncol / b.nl;
    rc.ensure(b.coarse_len() * ncol * sizeof(S));
    ec.ensure(b.coarse_len() * ncol * sizeof(S));
    b_restrict(b, p, P, r, rc.p, nr, st);
    auto res = gc.solve(Dc, rc.p, ec.p, true, ncol, 32, b.coarse_max, b.coarse_tol, st);
    coarse_iters += res.iters;
    Blas<S>::zero(z, b.fine_len() * ncol, st);
    b_prolong(b, p, P, ec.p, z, nr, st);
    gf.solve(D, r, z, false, ncol, std::max(1, b.n_post), b.n_post, 0.0, st);
    smooth_iters += b.n_post;
  }
};

using Clock = std::chrono::steady_clock;
double secs(Clock::time_point a, Clock::time_point c) { return std::chrono::duration<double>(c - a).count(); }

}  // namespace

// setup of every lattice (Algorithm 4 with Algorithm 3): Philox test vectors, smoothing,
// streaming SVD over all (aggregate, chirality) problems of all lattices, Galerkin blocks
void batch_setup(BatchDev& b, const qmg_mg_params& prm, hipStream_t st) {
  const auto t0 = Clock::now();
  const int r = prm.batch, ns = prm.n_test / prm.batch;
  const size_t cols = size_t(b.nl) * r;
  const size_t nf = b.fine_len() * cols;
  b.P64.alloc(size_t(2) * b.DT * b.k * b.N * sizeof(double2));
  b.sigma.alloc(size_t(2) * b.DT * b.k * sizeof(double));
  DevBuf phi(nf * sizeof(double2)), blocks(size_t(2) * b.DT * r * b.N * sizeof(double2));
  DevBuf xs, bs, tmp, basis, coef, part, e, latH;
  Gmres<double2> g64;
  int kp = 0;
  double mean_diag = 0;
  for (const Geom& g : b.geo) mean_diag += g.diag() / b.nl;
  for (int s = 0; s < ns; ++s) {
    const auto a0 = Clock::now();
    launch_philox_padded(prm.seed, s * r, r, b.nl, b.Vl.as<int>(), b.Vpad, phi.p, st);
    if (prm.n_setup_iter > 0) {
      // Eq. (2) per lattice and test vector: n_setup GMRES(8) steps on D psi' = -D phi, psi = phi + psi'
      if (b.inner == QMG_F64) {
        BatchOp D(b, QMG_F64, b.U64.p);
        bs.ensure(nf * sizeof(double2));
        xs.ensure(nf * sizeof(double2));
        D.apply(phi.p, bs.p, int(cols), st);
        Blas<double2>::axpby(0.0, bs.p, -1.0, bs.p, nf, st);
        g64.solve(D, bs.p, xs.p, true, int(cols), 8, prm.n_setup_iter, 0.0, st);
        Blas<double2>::axpby(1.0, xs.p, 1.0, phi.p, nf, st);
      } else {
        QMG_CHECK(prm.n_setup_iter % 8 == 0, QMG_EINVAL, "batched setup below FP64: n_setup_iter must be a multiple of 8");
        BatchOp D(b, QMG_F32, b.Uin.p);
        // D - d with d the lattices' mean diagonal term, in the stencil itself: each lattice's
        // diagonal coefficient becomes its own diagonal term minus d (the shifted s-step basis
        // then needs no separate vector update per step)
        if (!latH.p) {
          std::vector<BatchLattice> sh = b.lat_h;
          for (auto& x : sh) {
            x.a.diag_d -= mean_diag;
            x.a.diag_f = float(x.a.diag_d);
          }
          latH.alloc(sh.size() * sizeof(BatchLattice));
          QMG_HIP(hipMemcpy(latH.p, sh.data(), sh.size() * sizeof(BatchLattice), hipMemcpyHostToDevice));
        }
        BatchOp H(b, QMG_F32, b.Uin.p, latH.as<BatchLattice>());
        bs.ensure(nf * sizeof(float2));
        xs.ensure(nf * sizeof(float2));
        tmp.ensure(nf * sizeof(double2));
        launch_convert(phi.p, QMG_F64, xs.p, QMG_F32, nf, st);
        D.apply(xs.p, bs.p, int(cols), st);
        Blas<float2>::axpby(0.0, bs.p, -1.0, bs.p, nf, st);
        smooth_sstep<float2>(b.fine_len(), mean_diag, D, &H, int(cols), prm.n_setup_iter, bs.p, xs.p, basis, coef,
                             part, e, st);
        launch_convert(xs.p, QMG_F32, tmp.p, QMG_F64, nf, st);
        Blas<double2>::axpby(1.0, tmp.p, 1.0, phi.p, nf, st);
      }
    }
    {  // psi / |psi| per lattice and test vector
      RedWork rw;
      DevBuf nrm(cols * sizeof(double));
      Blas<double2>::norm2(phi.p, b.fine_len(), int(cols), nrm.as<double>(), rw, st);
      Blas<double2>::scale_dev(phi.p, nrm.as<double>(), 0, b.fine_len(), int(cols), st);
    }
    const auto a1 = Clock::now();
    {
      TimedLaunch tl_("batch/gather", st, double(cols) * b.Vpad * 12 * 2 * 16, 0.0);
      launch(k_b_gather, dim3(2 * b.DT, r, unsigned((b.N + 255) / 256)), dim3(256), 0, st,
             static_cast<const double2*>(phi.p), blocks.as<double2>(), b.gsite.as<int>(), b.jinfo.as<int>(), b.nd, b.N,
             r, b.Vpad);
    }
    QMG_LAUNCH_CHECK();
    kp = isvd_stream(2 * b.DT, b.N, b.k, b.P64, blocks.p, r, kp, b.sigma, st);
    QMG_HIP(hipStreamSynchronize(st));
    b.t_smooth += secs(a0, a1);
    b.t_svd += secs(a1, Clock::now());
  }
  QMG_CHECK(kp == b.k, QMG_ESHAPE, "streaming SVD ended with %d < k columns", kp);
  const auto c0 = Clock::now();
  b_build_coarse_direct(b, st);
  if (b.inner != QMG_F64) {
    const int m = 2 * b.k;
    const size_t np = size_t(2) * b.DT * b.k * b.N, ny = size_t(b.DT) * 9 * m * m;
    b.Pin.alloc(np * sizeof(float2));
    b.Yin.alloc(ny * sizeof(float2));
    launch_convert(b.P64.p, QMG_F64, b.Pin.p, QMG_F32, np, st);
    launch_convert(b.Y64.p, QMG_F64, b.Yin.p, QMG_F32, ny, st);
  }
  b.sigma_h.resize(size_t(2) * b.DT * b.k);
  QMG_HIP(hipMemcpyAsync(b.sigma_h.data(), b.sigma.p, b.sigma_h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  b.t_coarse = secs(c0, Clock::now());
  b.t_total = secs(t0, Clock::now());
}

// x = D^-1 b for every lattice and right-hand side (padded native FP64 in place in x64):
// FP64 flexible GMRES(16) with the FP64 K-cycle, or FP64 defect correction around an FP32
// flexible GMRES(16) (two Gram-Schmidt passes) whose K-cycle is stored in FP32; per-column
// relative residuals in FP64 until every column is at or below tol.
void batch_solve(const BatchDev& b, const void* b64, void* x64, int nr, double tol, int max_outer, hipStream_t st,
                 long* stats /* outer, refinements, coarse, smoother */) {
  const int ncol = b.nl * nr;
  const size_t len = b.fine_len(), n = len * ncol;
  BatchOp D64(b, QMG_F64, b.U64.p);
  if (b.inner == QMG_F64) {
    BatchCoarseOp Dc(b, QMG_F64, b.Y64.p);
    BatchKCycle<double2> K(b, D64, Dc, b.P64.p);
    Gmres<double2> f;
    auto res = f.solve(D64, b64, x64, true, ncol, 16, max_outer, tol, st, nullptr, 0, &K);
    stats[0] += res.iters;
    stats[1] += 1;
    stats[2] += K.coarse_iters;
    stats[3] += K.smooth_iters;
    return;
  }
  BatchOp D32(b, QMG_F32, b.Uin.p);
  BatchCoarseOp Dc(b, QMG_F32, b.Yin.p);
  BatchKCycle<float2> K(b, D32, Dc, b.Pin.p);
  Gmres<float2> f;
  f.set_cgs2(true);
  DevBuf r64(n * sizeof(double2)), rin(n * sizeof(float2)), ein(n * sizeof(float2)), nrm(ncol * sizeof(double)),
      bn(ncol * sizeof(double));
  RedWork rw;
  std::vector<double> hb(ncol), hr(ncol);
  Blas<double2>::zero(x64, n, st);
  Blas<double2>::norm2(b64, len, ncol, bn.as<double>(), rw, st);
  QMG_HIP(hipMemcpyAsync(hb.data(), bn.p, ncol * sizeof(double), hipMemcpyDeviceToHost, st));
  std::vector<double> hist;
  for (int ref = 0; ref < 40 && stats[0] < max_outer; ++ref) {
    D64.apply(x64, r64.p, ncol, st);
    dc_residual(b64, r64.p, len, ncol, nrm.as<double>(), rw, st);  // r = b - D x in FP64 and |r|^2
    QMG_HIP(hipMemcpyAsync(hr.data(), nrm.p, ncol * sizeof(double), hipMemcpyDeviceToHost, st));
    QMG_HIP(hipStreamSynchronize(st));
    double worst = 0;
    for (int i = 0; i < ncol; ++i) {
      QMG_CHECK(std::isfinite(hr[i]), QMG_ENONFINITE, "non-finite residual in defect correction");
      worst = std::max(worst, hb[i] > 0 ? std::sqrt(hr[i] / hb[i]) : 0.0);
    }
    hist.push_back(worst);
    if (worst <= tol) break;
    dc_normalise(r64.p, nrm.as<double>(), rin.p, len, ncol, st);
    auto res = f.solve(D32, rin.p, ein.p, true, ncol, 16, int(max_outer - stats[0]), 1e-5, st, nullptr, 0, &K);
    stats[0] += res.iters;
    stats[1] += 1;
    dc_accumulate(ein.p, nrm.as<double>(), x64, len, ncol, st);
  }
  stats[2] += K.coarse_iters;
  stats[3] += K.smooth_iters;
}

}  // namespace qmg

// ---------------------------------------------------------------------------------------
// C ABI

struct qmg_batch {
  qmg::BatchDev b;
  qmg_mg_params params{};
};

using namespace qmg;

namespace {

// a DevBuf pointing at memory it does not own for the lifetime of the guard (never freed by it)
struct Borrowed {
  DevBuf& d;
  Borrowed(DevBuf& d_, void* p) : d(d_) { d.p = p; }
  ~Borrowed() {
    d.p = nullptr;
    d.bytes = 0;
  }
};

template <class Fn>
qmg_status bguard(Fn&& f) {
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

}  // namespace

qmg_status qmg_batch_setup(int32_t n_lat, const qmg_lattice* lats, const void* const* U, const qmg_mg_params* p,
                           qmg_batch** out, hipStream_t stream) {
  return bguard([&] {
    QMG_CHECK(lats && U && p && out, QMG_EINVAL, "null argument");
    QMG_CHECK(n_lat >= 1 && n_lat <= 4096, QMG_EINVAL, "n_lat must be in [1, 4096]");
    QMG_CHECK(p->inner_prec == QMG_F64 || p->inner_prec == QMG_F32, QMG_EDTYPE,
              "batched hierarchies store their K-cycle in FP64 or FP32");
    QMG_CHECK(p->c_sw_s == 0.0 && p->c_sw_t == 0.0, QMG_ENOTIMPL, "batched hierarchies are Wilson only");
    QMG_CHECK(p->test_vectors == nullptr, QMG_EINVAL, "batched hierarchies draw their test vectors from the Philox generator");
    QMG_CHECK(p->batch >= 1 && p->n_test >= p->batch && p->n_test % p->batch == 0, QMG_ESHAPE,
              "n_test must be a positive multiple of batch");
    QMG_CHECK(p->rank >= 1 && p->rank <= kMaxRank && p->rank <= p->n_test, QMG_ESHAPE, "rank must be in [1, %d] and <= n_test",
              kMaxRank);
    QMG_CHECK(p->rank + p->batch <= 64, QMG_ESHAPE, "rank + batch must be <= 64");
    QMG_CHECK(p->n_setup_iter >= 0 && p->n_post_smooth >= 1 && p->coarse_tol > 0 && p->coarse_tol < 1 &&
                  p->coarse_max_iter >= 1,
              QMG_EINVAL, "bad smoother or coarse-solve parameters");
    std::unique_ptr<qmg_batch> h(new qmg_batch);
    BatchDev& b = h->b;
    h->params = *p;
    b.nl = n_lat;
    b.k = p->rank;
    b.inner = static_cast<qmg_prec>(p->inner_prec);
    b.n_post = p->n_post_smooth;
    b.coarse_tol = p->coarse_tol;
    b.coarse_max = p->coarse_max_iter;
    b.nd = 1;
    for (int q = 0; q < 4; ++q) {
      b.blk[q] = p->block[q];
      QMG_CHECK(b.blk[q] >= 1, QMG_ESHAPE, "block extents must be >= 1");
      b.nd *= b.blk[q];
    }
    b.N = 6 * b.nd;
    QMG_CHECK(b.k <= b.N, QMG_ESHAPE, "rank above the rows of an aggregate");
    std::vector<BatchLattice> desc(n_lat);
    int DT = 0;
    for (int l = 0; l < n_lat; ++l) {
      QMG_CHECK(U[l], QMG_EINVAL, "gauge field %d is NULL", l);
      Geom g = make_geom(&lats[l]);
      for (int q = 0; q < 4; ++q) {
        QMG_CHECK(g.L[q] % b.blk[q] == 0, QMG_ESHAPE, "lattice %d: block does not divide the extents", l);
        QMG_CHECK(g.L[q] / b.blk[q] >= 3, QMG_ESHAPE,
                  "lattice %d: every coarse extent must be >= 3 (eight distinct neighbour aggregates)", l);
      }
      b.geo.push_back(g);
      b.V.push_back(g.V);
      b.Vpad = std::max(b.Vpad, g.V);
      b.d.push_back(g.V / b.nd);
      b.aoff.push_back(DT);
      DT += g.V / b.nd;
      b.dmax = std::max(b.dmax, g.V / b.nd);
    }
    b.DT = DT;
    b.Vpad = (b.Vpad + 255) / 256 * 256;
    // tables: descriptors, volumes, aggregates, global neighbour aggregates
    std::vector<int> gsite(size_t(DT) * b.nd), jinfo(size_t(2) * DT), cnb(size_t(8) * DT);
    for (int l = 0; l < n_lat; ++l) {
      const Geom& g = b.geo[l];
      desc[l].a = make_dslash_args(g, 1, false, false);
      desc[l].a.V = b.Vpad;
      desc[l].tile0 = 0;
      int cL[4];
      for (int q = 0; q < 4; ++q) cL[q] = g.L[q] / b.blk[q];
      for (int site = 0; site < g.V; ++site) {
        int c[4], rem = site;
        for (int q = 0; q < 4; ++q) {
          c[q] = rem % g.L[q];
          rem /= g.L[q];
        }
        int cj[4], ci[4];
        for (int q = 0; q < 4; ++q) {
          cj[q] = c[q] / b.blk[q];
          ci[q] = c[q] % b.blk[q];
        }
        const int j = cj[0] + cL[0] * (cj[1] + cL[1] * (cj[2] + cL[2] * cj[3]));
        const int ib = ci[0] + b.blk[0] * (ci[1] + b.blk[1] * (ci[2] + b.blk[2] * ci[3]));
        gsite[size_t(b.aoff[l] + j) * b.nd + ib] = site;
      }
      for (int j = 0; j < b.d[l]; ++j) {
        const int J = b.aoff[l] + j;
        jinfo[2 * J] = l;
        jinfo[2 * J + 1] = j;
        int c[4], rem = j;
        for (int q = 0; q < 4; ++q) {
          c[q] = rem % cL[q];
          rem /= cL[q];
        }
        for (int dir = 0; dir < 8; ++dir) {
          const int mu = dir & 3, step = dir < 4 ? 1 : -1;
          int cc[4] = {c[0], c[1], c[2], c[3]};
          cc[mu] = (cc[mu] + step + cL[mu]) % cL[mu];
          cnb[size_t(J) * 8 + dir] = b.aoff[l] + cc[0] + cL[0] * (cc[1] + cL[1] * (cc[2] + cL[2] * cc[3]));
        }
      }
    }
    auto upload = [&](DevBuf& d, const void* src, size_t bytes) {
      d.alloc(bytes);
      QMG_HIP(hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice));
    };
    b.lat_h = desc;
    upload(b.lat, desc.data(), desc.size() * sizeof(BatchLattice));
    upload(b.Vl, b.V.data(), b.V.size() * sizeof(int));
    upload(b.dl, b.d.data(), b.d.size() * sizeof(int));
    upload(b.aoffd, b.aoff.data(), b.aoff.size() * sizeof(int));
    upload(b.gsite, gsite.data(), gsite.size() * sizeof(int));
    upload(b.jinfo, jinfo.data(), jinfo.size() * sizeof(int));
    upload(b.cnb, cnb.data(), cnb.size() * sizeof(int));
    // gauge fields: padded native FP64 (and FP32)
    b.U64.alloc(size_t(n_lat) * 36 * b.Vpad * sizeof(double2));
    for (int l = 0; l < n_lat; ++l) {
      launch(k_b_pack_gauge, dim3(unsigned(b.Vpad / 256), 36), dim3(256), 0, stream, static_cast<const double2*>(U[l]),
             b.U64.as<double2>() + size_t(l) * 36 * b.Vpad, b.V[l], b.Vpad);
      QMG_LAUNCH_CHECK();
    }
    {
      const double un = [&] {
        RedWork rw;
        DevBuf nr(sizeof(double));
        Blas<double2>::norm2(b.U64.p, size_t(n_lat) * 36 * b.Vpad, 1, nr.as<double>(), rw, stream);
        double v = 0;
        QMG_HIP(hipMemcpyAsync(&v, nr.p, sizeof(double), hipMemcpyDeviceToHost, stream));
        QMG_HIP(hipStreamSynchronize(stream));
        return v;
      }();
      QMG_CHECK(std::isfinite(un), QMG_ENONFINITE, "gauge fields have non-finite entries");
    }
    if (b.inner == QMG_F32) {
      b.Uin.alloc(size_t(n_lat) * 36 * b.Vpad * sizeof(float2));
      launch_convert(b.U64.p, QMG_F64, b.Uin.p, QMG_F32, size_t(n_lat) * 36 * b.Vpad, stream);
    }
    batch_setup(b, *p, stream);
    *out = h.release();
  });
}

qmg_status qmg_batch_solve(const qmg_batch* h, const void* const* rhs, void* const* x, int32_t nrhs, double tol,
                           int32_t max_outer, qmg_solve_info* info, hipStream_t stream) {
  long stats[4] = {0, 0, 0, 0};
  std::vector<double> rel;
  double el = 0;
  qmg_status rc = bguard([&] {
    QMG_CHECK(h && rhs && x, QMG_EINVAL, "null argument");
    QMG_CHECK(nrhs >= 1 && max_outer >= 1, QMG_EINVAL, "need nrhs >= 1 and max_outer >= 1");
    QMG_CHECK(tol > 0 && tol < 1, QMG_EINVAL, "tol must be in (0, 1)");
    const BatchDev& b = h->b;
    for (int l = 0; l < b.nl; ++l) QMG_CHECK(rhs[l] && x[l], QMG_EINVAL, "right-hand side or solution %d is NULL", l);
    const auto t0 = Clock::now();
    const int ncol = b.nl * nrhs;
    const size_t len = b.fine_len(), n = len * ncol;
    DevBuf b64(n * sizeof(double2)), x64(n * sizeof(double2)), r64(n * sizeof(double2));
    for (int l = 0; l < b.nl; ++l) {
      launch(k_b_pack_spinor, dim3(unsigned(b.Vpad / 256), 12 * nrhs), dim3(256), 0, stream,
             static_cast<const double2*>(rhs[l]), b64.as<double2>() + size_t(l) * nrhs * len, b.V[l], b.Vpad);
      QMG_LAUNCH_CHECK();
    }
    RedWork rw;
    DevBuf nr(2 * size_t(ncol) * sizeof(double));
    Blas<double2>::norm2(b64.p, len, ncol, nr.as<double>() + ncol, rw, stream);
    batch_solve(b, b64.p, x64.p, nrhs, tol, max_outer, stream, stats);
    BatchOp D(b, QMG_F64, b.U64.p);
    D.apply(x64.p, r64.p, ncol, stream);
    Blas<double2>::axpby(1.0, b64.p, -1.0, r64.p, n, stream);
    Blas<double2>::norm2(r64.p, len, ncol, nr.as<double>(), rw, stream);
    std::vector<double> hn(2 * size_t(ncol));
    QMG_HIP(hipMemcpyAsync(hn.data(), nr.p, hn.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    for (int l = 0; l < b.nl; ++l) {
      launch(k_b_unpack_spinor, dim3(unsigned((b.V[l] + 255) / 256), 12 * nrhs), dim3(256), 0, stream,
             x64.as<double2>() + size_t(l) * nrhs * len, static_cast<double2*>(x[l]), b.V[l], b.Vpad);
      QMG_LAUNCH_CHECK();
    }
    QMG_HIP(hipStreamSynchronize(stream));
    double worst = 0;
    rel.resize(ncol);
    for (int i = 0; i < ncol; ++i) {
      rel[i] = hn[ncol + i] > 0 ? std::sqrt(hn[i] / hn[ncol + i]) : 0.0;
      QMG_CHECK(std::isfinite(rel[i]), QMG_ENONFINITE, "non-finite final residual");
      worst = std::max(worst, rel[i]);
    }
    el = secs(t0, Clock::now());
    QMG_CHECK(worst <= tol, QMG_ENOCONV, "batched solve stopped at relative residual %.3e > tol %.3e", worst, tol);
  });
  if (info && h) {
    const int ncol = h->b.nl * nrhs;
    for (int i = 0; i < ncol; ++i) {
      info[i] = qmg_solve_info{};
      info[i].outer_iters = int(stats[0]);
      info[i].refinements = int(stats[1]);
      info[i].coarse_iters = int(stats[2]);
      info[i].smoother_iters = int(stats[3]);
      info[i].true_rel_res = i < int(rel.size()) ? rel[i] : -1.0;
      info[i].seconds = el;
    }
  }
  return rc;
}

qmg_status qmg_batch_query(const qmg_batch* h, int32_t lat, int32_t* n_agg, int32_t* rank) {
  return bguard([&] {
    QMG_CHECK(h && n_agg && rank, QMG_EINVAL, "null argument");
    QMG_CHECK(lat >= 0 && lat < h->b.nl, QMG_EINVAL, "lattice index out of range");
    *n_agg = h->b.d[lat];
    *rank = h->b.k;
  });
}

qmg_status qmg_batch_get_prolongator(const qmg_batch* h, int32_t lat, void* P, double* sigma, hipStream_t stream) {
  return bguard([&] {
    QMG_CHECK(h, QMG_EINVAL, "null handle");
    const BatchDev& b = h->b;
    QMG_CHECK(lat >= 0 && lat < b.nl, QMG_EINVAL, "lattice index out of range");
    const size_t off = size_t(2) * b.aoff[lat], np = size_t(2) * b.d[lat];
    if (P) {
      HierarchyDev tmp;  // export in the CPU reference's row order, through the single-lattice layout
      tmp.blk.nd = b.nd;
      tmp.blk.N = b.N;
      tmp.blk.d = b.d[lat];
      tmp.k = b.k;
      Borrowed hold(tmp.P64, b.P64.as<double2>() + off * b.k * b.N);
      launch_export_P(tmp, P, stream);
      QMG_HIP(hipStreamSynchronize(stream));
    }
    if (sigma) std::memcpy(sigma, b.sigma_h.data() + off * b.k, np * b.k * sizeof(double));
  });
}

qmg_status qmg_batch_get_coarse(const qmg_batch* h, int32_t lat, void* Y, hipStream_t stream) {
  return bguard([&] {
    QMG_CHECK(h && Y, QMG_EINVAL, "null argument");
    const BatchDev& b = h->b;
    QMG_CHECK(lat >= 0 && lat < b.nl, QMG_EINVAL, "lattice index out of range");
    HierarchyDev tmp;
    tmp.blk.d = b.d[lat];
    tmp.k = b.k;
    const int m = 2 * b.k;
    Borrowed hold(tmp.Y64, b.Y64.as<double2>() + size_t(b.aoff[lat]) * 9 * m * m);
    launch_export_Y(tmp, Y, stream);
    QMG_HIP(hipStreamSynchronize(stream));
  });
}

qmg_status qmg_batch_setup_times(const qmg_batch* h, double* t) {
  return bguard([&] {
    QMG_CHECK(h && t, QMG_EINVAL, "null argument");
    t[0] = h->b.t_smooth;
    t[1] = h->b.t_svd;
    t[2] = h->b.t_coarse;
    t[3] = h->b.t_total;
  });
}

void qmg_batch_destroy(qmg_batch* h) { delete h; }
