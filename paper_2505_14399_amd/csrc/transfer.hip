// Transfer operators P and R = P^dagger (Eq. (6)), the Galerkin coarse operator D_c = R D P
// (Eq. (5)) and its application, plus the layout kernels of the hierarchy.
#include <cmath>
#include <mutex>
#include <type_traits>

#include "mg.hpp"
#include "timing.hpp"

namespace qmg {

namespace {

inline unsigned cdiv(size_t a, size_t b) { return unsigned((a + b - 1) / b); }

// XCD-local index of workgroup b of nb: the hardware deals workgroups to the eight XCDs round
// robin (b % 8), so this numbering gives each XCD one contiguous range.  The transfers use it
// so that neighbouring aggregates, whose blocks share cache lines of the fine vectors (4 sites
// of a 128-byte line of 16 in FP32), run on one XCD and meet those lines in its L2.
__device__ inline int xcd_local(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
  return x * q + min(x, rem) + i;
}

// ---------------------------------------------------------------------------------------
// prolong: one thread per pack of PR rows of a (j, alpha) block, for NR right-hand sides; the
// k coarse coefficients of those right-hand sides are staged in LDS, so P is read once per
// group of right-hand sides.  Rows are s6 * nd + ib; the fine site is bsite[j][ib].
// Grid: one dimension of npack * 2d * groups workgroups, in XCD-local order (row packs of a
// block, then the blocks, then the groups of right-hand sides).
template <class S, int PR, int NR>
__global__ __launch_bounds__(256) void k_prolong(const S* __restrict__ P, const S* __restrict__ vc,
                                                 S* __restrict__ fine, const int* __restrict__ bsite, int nd, int N,
                                                 int k, int d, int V, int nrhs, int npack) {
  using C = ctype<S>;
  __shared__ cplx<C> cv[NR][64];
  const int wg = xcd_local(blockIdx.x, gridDim.x);
  const int pk = wg % npack, rest = wg / npack;
  const int ja = rest % (2 * d);  // j * 2 + alpha
  const int rhs0 = (rest / (2 * d)) * NR;
  const int nr = min(NR, nrhs - rhs0);
  const int j = ja >> 1, a = ja & 1;
  for (int t = threadIdx.x; t < NR * k; t += 256) {
    const int r = t / k, i = t - r * k;
    cv[r][i] = r < nr ? ldc(vc, (size_t(rhs0 + r) * d + j) * 2 * k + a * k + i) : cplx<C>{C(0), C(0)};
  }
  __syncthreads();
  const int rp = pk * 256 + threadIdx.x;  // row pack
  if (rp * PR >= N) return;
  const S* Pc = P + size_t(ja) * k * N;
  const size_t np = N / PR;
  cplx<C> acc[NR][PR];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int u = 0; u < PR; ++u) acc[r][u] = {C(0), C(0)};
  int i = 0;
  for (; i + 4 <= k; i += 4) {
    Pk<S, PR> pv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) pv[q] = ldp<S, PR>(Pc, size_t(i + q) * np + rp);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < PR; ++u) {
        const cplx<C> pe = StoreTraits<S>::ld(pv[q].v[u]);
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r][u] += pe * cv[r][i + q];
      }
  }
  for (; i < k; ++i) {
    const Pk<S, PR> pv = ldp<S, PR>(Pc, size_t(i) * np + rp);
#pragma unroll
    for (int u = 0; u < PR; ++u) {
      const cplx<C> pe = StoreTraits<S>::ld(pv.v[u]);
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r][u] += pe * cv[r][i];
    }
  }
#pragma unroll
  for (int u = 0; u < PR; ++u) {
    const int row = rp * PR + u;
    const int s6 = row / nd, ib = row - s6 * nd;
    const int site = bsite[size_t(j) * nd + ib];
    const int comp = 6 * a + s6;
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nr) stc(fine, (size_t(rhs0 + r) * 12 + comp) * V + site, acc[r][u]);
  }
}

// restrict: one workgroup per (j, alpha, group of NR right-hand sides).  The block of each fine
// vector is gathered into LDS; thread t takes row packs t, t + 256, ... and accumulates
// conj(P) psi for eight columns at a time, which are then summed over the workgroup (wavefront
// shuffles, then LDS across the four wavefronts).  P is read once per group.
template <class S, int PR, int NR>
__global__ __launch_bounds__(256) void k_restrict(const S* __restrict__ P, const S* __restrict__ fine,
                                                  S* __restrict__ vc, const int* __restrict__ bsite, int nd, int N,
                                                  int k, int d, int V, int nrhs) {
  using C = ctype<S>;
  constexpr int KC = 8;
  extern __shared__ unsigned char smem[];
  cplx<C>* psi = reinterpret_cast<cplx<C>*>(smem);  // [NR][N]
  __shared__ cplx<C> red[4][KC * NR];
  const int ja = xcd_local(blockIdx.x, gridDim.x), rhs0 = blockIdx.y * NR;
  const int nr = min(NR, nrhs - rhs0);
  const int j = ja >> 1, a = ja & 1;
  // the gather: GU rows per thread and pass, their fine sites first and then all GU x NR spinor
  // components, so that the loads of a pass are in flight together (two memory round trips per
  // pass rather than two per element)
  constexpr int GU = 6;
  for (int base = 0; base < N; base += 256 * GU) {
    size_t off[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int row = base + u * 256 + threadIdx.x;
      off[u] = 0;
      if (row < N) {
        const int s6 = row / nd, ib = row - s6 * nd;
        off[u] = size_t(6 * a + s6) * V + bsite[size_t(j) * nd + ib];
      }
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int row = base + u * 256 + threadIdx.x;
      if (row < N) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          psi[size_t(r) * N + row] = r < nr ? ldc(fine, size_t(rhs0 + r) * 12 * V + off[u]) : cplx<C>{C(0), C(0)};
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const size_t np = N / PR;
  const S* Pb = P + size_t(ja) * k * N;
  for (int i0 = 0; i0 < k; i0 += KC) {
    const int kc = min(KC, k - i0);
    cplx<C> acc[KC][NR];
#pragma unroll
    for (int q = 0; q < KC; ++q)
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[q][r] = {C(0), C(0)};
    // P loads one row pack ahead of the arithmetic
    Pk<S, PR> pv[KC], pn[KC];
    if (threadIdx.x < np) {
#pragma unroll
      for (int q = 0; q < KC; ++q)
        if (q < kc) pv[q] = ldp<S, PR>(Pb, size_t(i0 + q) * np + threadIdx.x);
    }
    for (size_t rp = threadIdx.x; rp < np; rp += 256) {
      if (rp + 256 < np) {
#pragma unroll
        for (int q = 0; q < KC; ++q)
          if (q < kc) pn[q] = ldp<S, PR>(Pb, size_t(i0 + q) * np + rp + 256);
      }
#pragma unroll
      for (int u = 0; u < PR; ++u) {
        cplx<C> ps[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) ps[r] = psi[size_t(r) * N + rp * PR + u];
#pragma unroll
        for (int q = 0; q < KC; ++q) {
          if (q < kc) {
            const cplx<C> pe = StoreTraits<S>::ld(pv[q].v[u]);
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[q][r] += cmul_conj(pe, ps[r]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < KC; ++q) pv[q] = pn[q];
    }
#pragma unroll
    for (int q = 0; q < KC; ++q)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const cplx<C> v = {wave_sum(acc[q][r].re), wave_sum(acc[q][r].im)};
        if (lane == 0) red[w][q * NR + r] = v;
      }
    __syncthreads();
    if (threadIdx.x < kc * NR) {
      const int q = threadIdx.x / NR, r = threadIdx.x - q * NR;
      cplx<C> s = red[0][threadIdx.x];
#pragma unroll
      for (int ww = 1; ww < 4; ++ww) s += red[ww][threadIdx.x];
      if (r < nr) stc(vc, (size_t(rhs0 + r) * d + j) * 2 * k + a * k + i0 + q, s);
    }
    __syncthreads();
  }
}

// coarse apply: one workgroup per (aggregate, group of NR right-hand sides).  The nine input
// vectors v(j + slot) are staged in LDS.  Thread (h, slot, row pack) forms PR rows of
// Y_slot(j) times v(j + slot) over column chunk h of H (each Y entry read once per group of
// right-hand sides; PR consecutive rows of a column-major block are one 16-byte load); the
// 9 H partial rows are summed in LDS.  H splits the columns so that a workgroup has enough
// wavefronts to keep the Y stream in flight.
template <class S, int NR, int PR>
__global__ __launch_bounds__(1024) void k_coarse_apply(const S* __restrict__ Y, const S* __restrict__ in,
                                                       S* __restrict__ out, const int* __restrict__ cnb, int d, int m,
                                                       int nrhs, int H, const int* __restrict__ skip) {
  using C = ctype<S>;
  if (skip && *skip) return;  // device-side early exit of a converged coarse solve
  extern __shared__ unsigned char smem_raw[];
  cplx<C>* vin = reinterpret_cast<cplx<C>*>(smem_raw);  // [NR][9][m]
  cplx<C>* part = vin + size_t(NR) * 9 * m;              // [NR][9 H][m]
  const int j = blockIdx.x, rhs0 = blockIdx.y * NR;
  const int nr = min(NR, nrhs - rhs0);
  for (int t = threadIdx.x; t < NR * 9 * m; t += blockDim.x) {
    const int r = t / (9 * m), rem = t - r * 9 * m, slot = rem / m, col = rem - slot * m;
    const int nbj = slot == 0 ? j : cnb[j * 8 + slot - 1];
    vin[t] = r < nr ? ldc(in, (size_t(rhs0 + r) * d + nbj) * m + col) : cplx<C>{C(0), C(0)};
  }
  __syncthreads();
  const int mp = m / PR;           // row packs per column
  const int cc = (m + H - 1) / H;  // columns per chunk
  for (int t = threadIdx.x; t < H * 9 * mp; t += blockDim.x) {
    const int hs = t / mp, rp = t - hs * mp;  // hs = h * 9 + slot
    const int h = hs / 9, slot = hs - h * 9;
    const int c0 = h * cc, c1 = min(m, c0 + cc);
    const S* Yb = Y + (size_t(j) * 9 + slot) * m * m;
    cplx<C> acc[NR][PR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int u = 0; u < PR; ++u) acc[r][u] = {C(0), C(0)};
#pragma unroll 6
    for (int col = c0; col < c1; ++col) {
      const Pk<S, PR> y = ldp<S, PR>(Yb, size_t(col) * mp + rp);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const cplx<C> v = vin[(r * 9 + slot) * m + col];
#pragma unroll
        for (int u = 0; u < PR; ++u) acc[r][u] += StoreTraits<S>::ld(y.v[u]) * v;
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int u = 0; u < PR; ++u) part[(size_t(r) * 9 * H + hs) * m + rp * PR + u] = acc[r][u];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nr * m; t += blockDim.x) {
    const int r = t / m, row = t - r * m;
    cplx<C> s = {C(0), C(0)};
    for (int q = 0; q < 9 * H; ++q) s += part[(size_t(r) * 9 * H + q) * m + row];
    stc(out, (size_t(rhs0 + r) * d + j) * m + row, s);
  }
}

// ---------------------------------------------------------------------------------------
// Galerkin build (FP64).  One workgroup per (aggregate j, forward direction mu).  For every
// site x of the block the hop term H(x, mu) is applied to the 2k columns of P at the neighbour
// y and contracted with P(x)^dag; hops leaving the block through its face go to Y_{1+mu}(j),
// the others to the partial self block W_mu(j) (workgroup mu = 0 also forms the diagonal
// term).  The backward directions follow from sigma3-hermiticity (k_sum_self,
// k_fill_backward).
struct BuildArgs {
  int L[4], b[4], cL[4];
  int V, nd, N, k, d, bc_t;
  double diag, cw[4];
  const double2* clov;  // packed FP64 site term with the clover term (nullptr: diag)
};

__device__ inline int lex4(const int* c, const int* L) { return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3])); }

// chi (12 comps, chirality beta only) -> H chi  for direction dir with link u (already U or U^dag)
template <int MU>
__device__ inline void hop_col(const cplx<double>* q, int beta, double sg, const cplx<double>* u, double coef,
                               cplx<double>* out) {
  // h = chi_up + sg A chi_dn
  cplx<double> h[6];
  for (int c = 0; c < 3; ++c) {
    cplx<double> u0, u1, d0, d1;
    if (beta == 0) {
      u0 = q[c]; u1 = q[3 + c]; d0 = {0, 0}; d1 = {0, 0};
    } else {
      u0 = {0, 0}; u1 = {0, 0}; d0 = q[c]; d1 = q[3 + c];
    }
    if (MU == 0) { h[c] = u0 + sg * times_mi(d1); h[3 + c] = u1 + sg * times_mi(d0); }
    else if (MU == 1) { h[c] = u0 - sg * d1; h[3 + c] = u1 + sg * d0; }
    else if (MU == 2) { h[c] = u0 + sg * times_mi(d0); h[3 + c] = u1 + sg * times_i(d1); }
    else { h[c] = u0 + sg * d0; h[3 + c] = u1 + sg * d1; }
  }
  cplx<double> w[6];
  for (int sp = 0; sp < 2; ++sp)
    for (int a = 0; a < 3; ++a) {
      cplx<double> t = {0, 0};
      for (int bb = 0; bb < 3; ++bb) t += u[3 * a + bb] * h[3 * sp + bb];
      w[3 * sp + a] = t;
    }
  for (int c = 0; c < 3; ++c) {
    cplx<double> w0 = w[c], w1 = w[3 + c];
    out[c] = coef * w0;
    out[3 + c] = coef * w1;
    cplx<double> l0, l1;
    if (MU == 0) { l0 = times_i(w1); l1 = times_i(w0); }
    else if (MU == 1) { l0 = w1; l1 = -w0; }
    else if (MU == 2) { l0 = times_i(w0); l1 = times_mi(w1); }
    else { l0 = w0; l1 = w1; }
    out[6 + c] = (coef * sg) * l0;
    out[9 + c] = (coef * sg) * l1;
  }
}

constexpr int kMaxM = 64;        // 2k <= 64

// grid (d, 8): workgroup (j, dir) forms, for the hops of direction dir leaving the sites of
// aggregate j, the sum over sites of P_j(x)^dag H(x, dir) P_{j'}(x + dir) as a small GEMM:
// rows (alpha, i) of P_j(x)^dag, columns (beta, l) of H P at the neighbour, reduction over
// the sites and the 6 spin-colour components of chirality alpha.  The sites of the block are
// visited by class from a host-built list: hops that stay inside the block (accumulated into
// the partial W[dir][j] of Y_0), then, for dir 0 only, the diagonal term (m+1+3/xi) P^dag P
// (also into W), then the hops through the face (written to Y_{1+dir}(j)).  NS sites are
// staged per phase; each thread owns a TS x TS tile of the (2k) x (2k) block.
template <int TS>
__global__ __launch_bounds__(256) void k_build_coarse(const double2* __restrict__ U, const double2* __restrict__ P,
                                                      const int* __restrict__ bsite, const int* __restrict__ lists,
                                                      double2* __restrict__ Y, double2* __restrict__ W, BuildArgs a,
                                                      int NS) {
  extern __shared__ unsigned char smem_raw[];
  const int k = a.k, m = 2 * k, N = a.N, nd = a.nd, V = a.V;
  cplx<double>* Px = reinterpret_cast<cplx<double>*>(smem_raw);  // [NS][12][k]
  cplx<double>* HP = Px + size_t(NS) * 12 * k;                    // [NS][12][m]
  cplx<double>* lnk = HP + size_t(NS) * 12 * m;                   // [NS][9]
  double* scoef = reinterpret_cast<double*>(lnk + size_t(NS) * 9); // [NS]
  int* sinfo = reinterpret_cast<int*>(scoef + NS);                // [NS][5]: ib, x, y, jy, iby
  const int j = blockIdx.x, dir = blockIdx.y;
  const int mu = dir & 3;
  const bool fwd = dir < 4;
  const double sg = fwd ? -1.0 : 1.0;
  const int tid = threadIdx.x;
  const int nrk = (k + TS - 1) / TS;        // row tiles per chirality
  const int nct = (m + TS - 1) / TS;        // column tiles
  const bool active = tid < 2 * nrk * nct;
  const int rt = tid / nct, ct = tid - (tid / nct) * nct;
  const int al = rt / nrk, i0 = (rt - al * nrk) * TS, c0 = ct * TS;
  const int nface = nd / a.b[mu];
  const int* list = lists + size_t(dir) * nd;  // intra sites, then face sites
  const int nent = m * m;
  cplx<double> acc[TS][TS];

  for (int cls = 0; cls < 3; ++cls) {
    // cls 0: intra hops, cls 1: diagonal term (dir 0 only), cls 2: face hops
    if (cls == 1 && dir != 0) continue;
    const int count = cls == 0 ? nd - nface : (cls == 1 ? nd : nface);
    const int base = cls == 2 ? nd - nface : 0;
#pragma unroll
    for (int t = 0; t < TS; ++t)
#pragma unroll
      for (int u = 0; u < TS; ++u) acc[t][u] = {0, 0};
    for (int n0 = 0; n0 < count; n0 += NS) {
      const int ns = min(NS, count - n0);
      if (tid < ns) {
        const int ib = cls == 1 ? n0 + tid : list[base + n0 + tid];
        const int x = bsite[size_t(j) * nd + ib];
        int c[4];
        int rem = x;
        for (int q = 0; q < 4; ++q) { c[q] = rem % a.L[q]; rem /= a.L[q]; }
        int cy[4] = {c[0], c[1], c[2], c[3]};
        if (cls != 1) cy[mu] = fwd ? (c[mu] + 1) % a.L[mu] : (c[mu] + a.L[mu] - 1) % a.L[mu];
        int cj[4], ci[4];
        for (int q = 0; q < 4; ++q) { cj[q] = cy[q] / a.b[q]; ci[q] = cy[q] % a.b[q]; }
        int* si = sinfo + tid * 5;
        si[0] = ib;
        si[1] = x;
        si[2] = lex4(cy, a.L);
        si[3] = lex4(cj, a.cL);
        si[4] = lex4(ci, a.b);
        double sgnbc = 1.0;
        if (mu == 3 && a.bc_t < 0) {
          if (fwd && c[3] == a.L[3] - 1) sgnbc = -1.0;
          if (!fwd && c[3] == 0) sgnbc = -1.0;
        }
        scoef[tid] = -0.5 * a.cw[mu] * sgnbc;
      }
      __syncthreads();
      // links and the rows of P at the staged sites
      for (int t = tid; t < ns * 9; t += 256) {
        const int q = t / 9, e = t - q * 9;
        const int* si = sinfo + q * 5;
        if (fwd) {
          const double2 v = U[(size_t(mu) * 9 + e) * V + si[1]];
          lnk[q * 9 + e] = {v.x, v.y};
        } else {
          const int rr = e / 3, cc = e - rr * 3;
          const double2 v = U[(size_t(mu) * 9 + cc * 3 + rr) * V + si[2]];
          lnk[q * 9 + e] = {v.x, -v.y};
        }
      }
      for (int t = tid; t < ns * 12 * k; t += 256) {
        const int q = t % ns, rem = t / ns;
        const int comp = rem / k, i = rem - comp * k;
        const int alc = comp / 6, s6 = comp - alc * 6;
        const double2 v = P[((size_t(j) * 2 + alc) * k + i) * N + size_t(s6) * nd + sinfo[q * 5]];
        Px[(size_t(q) * 12 + comp) * k + i] = {v.x, v.y};
      }
      __syncthreads();
      // H P at the neighbour (cls 1: the diagonal term times P at the site itself)
      for (int t = tid; t < ns * m; t += 256) {
        const int q = t / m, col = t - q * m;
        const int beta = col / k, l = col - beta * k;
        cplx<double>* hp = HP + size_t(q) * 12 * m + col;
        if (cls == 1 && a.clov) {
          // the chirality-beta block of the site term at the staged site times P's column
          const double2* blk = a.clov + size_t(beta) * 18 * V + sinfo[q * 5 + 1];
          cplx<double> x[6];
          for (int s6 = 0; s6 < 6; ++s6) x[s6] = Px[(size_t(q) * 12 + 6 * beta + s6) * k + l];
          cplx<double> y[6];
          for (int e = 0; e < 3; ++e) {
            const double2 dd = blk[size_t(e) * V];
            y[2 * e] = dd.x * x[2 * e];
            y[2 * e + 1] = dd.y * x[2 * e + 1];
          }
          int e = 3;
          for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j, ++e) {
              const double2 ov = blk[size_t(e) * V];
              const cplx<double> o = {ov.x, ov.y};
              y[i] += o * x[j];
              y[j] += cmul_conj(o, x[i]);
            }
          for (int comp = 0; comp < 12; ++comp)
            hp[comp * m] = (comp / 6 == beta) ? y[comp - 6 * beta] : cplx<double>{0, 0};
        } else if (cls == 1) {
          for (int comp = 0; comp < 12; ++comp)
            hp[comp * m] = (comp / 6 == beta) ? a.diag * Px[(size_t(q) * 12 + comp) * k + l] : cplx<double>{0, 0};
        } else {
          const int* si = sinfo + q * 5;
          cplx<double> qv[6];
          for (int s6 = 0; s6 < 6; ++s6) {
            const double2 v = P[((size_t(si[3]) * 2 + beta) * k + l) * N + size_t(s6) * nd + si[4]];
            qv[s6] = {v.x, v.y};
          }
          cplx<double> out[12];
          switch (mu) {
            case 0: hop_col<0>(qv, beta, sg, lnk + q * 9, scoef[q], out); break;
            case 1: hop_col<1>(qv, beta, sg, lnk + q * 9, scoef[q], out); break;
            case 2: hop_col<2>(qv, beta, sg, lnk + q * 9, scoef[q], out); break;
            default: hop_col<3>(qv, beta, sg, lnk + q * 9, scoef[q], out); break;
          }
          for (int comp = 0; comp < 12; ++comp) hp[comp * m] = out[comp];
        }
      }
      __syncthreads();
      if (active) {
        for (int q = 0; q < ns; ++q) {
#pragma unroll 2
          for (int s6 = 0; s6 < 6; ++s6) {
            const int comp = 6 * al + s6;
            const cplx<double>* pr = Px + (size_t(q) * 12 + comp) * k;
            const cplx<double>* hr = HP + (size_t(q) * 12 + comp) * m;
            cplx<double> pa[TS], hb[TS];
#pragma unroll
            for (int t = 0; t < TS; ++t) pa[t] = (i0 + t < k) ? pr[i0 + t] : cplx<double>{0, 0};
#pragma unroll
            for (int u = 0; u < TS; ++u) hb[u] = (c0 + u < m) ? hr[c0 + u] : cplx<double>{0, 0};
#pragma unroll
            for (int t = 0; t < TS; ++t)
#pragma unroll
              for (int u = 0; u < TS; ++u) acc[t][u] += cmul_conj(pa[t], hb[u]);
          }
        }
      }
      __syncthreads();
    }
    // write: intra hops to W[dir], the diagonal term to W[4], face hops to Y_{1+dir}
    if (active) {
      for (int t = 0; t < TS; ++t)
        for (int u = 0; u < TS; ++u) {
          const int i = i0 + t, col = c0 + u;
          if (i >= k || col >= m) continue;
          const int idx = col * m + al * k + i;
          const double2 v = make_double2(acc[t][u].re, acc[t][u].im);
          if (cls == 2) Y[(size_t(j) * 9 + 1 + dir) * nent + idx] = v;
          else W[(size_t(cls == 1 ? 4 : dir) * a.d + j) * nent + idx] = v;
        }
    }
  }
}

// D_c is sigma3-hermitian (gamma5 P = P sigma3 and gamma5 D gamma5 = D^dag), so the hops
// along -mu are the sigma3-adjoints of those along +mu: inside a block, the -mu intra-block
// part of Y_0 is sigma3 W_mu^dag sigma3, and across faces Y_{-mu}(j) = sigma3 Y_{+mu}(j-mu)^dag
// sigma3.  Only the four forward directions are built; sigma3 = diag(+1 (alpha = 0), -1).
__device__ inline double2 s3adj(const double2* B, int m, int k, int row, int col) {
  const double2 v = B[size_t(row) * m + col];  // B(col, row), column-major
  const double s = ((row < k) == (col < k)) ? 1.0 : -1.0;
  return make_double2(s * v.x, -s * v.y);
}

// Y_0(j) = diagonal term + sum over the four forward directions of (W_mu + sigma3 W_mu^dag sigma3)
__global__ void k_sum_self(const double2* __restrict__ W, double2* __restrict__ Y, int d, int m, int k) {
  const int nent = m * m;
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= size_t(d) * nent) return;
  const size_t j = g / nent, idx = g - j * nent;
  const int col = int(idx / m), row = int(idx - size_t(col) * m);
  double2 s = W[(size_t(4) * d + j) * nent + idx];
  for (int dir = 0; dir < 4; ++dir) {
    const double2* B = W + (size_t(dir) * d + j) * nent;
    const double2 v = B[idx], a = s3adj(B, m, k, row, col);
    s.x += v.x + a.x;
    s.y += v.y + a.y;
  }
  Y[(j * 9) * nent + idx] = s;
}

// Y_{1+4+mu}(j) = sigma3 Y_{1+mu}(j - mu)^dag sigma3
__global__ void k_fill_backward(double2* __restrict__ Y, const int* __restrict__ cnb, int d, int m, int k) {
  const int nent = m * m;
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= size_t(d) * 4 * nent) return;
  const size_t jm = g / nent, idx = g - jm * nent;
  const int j = int(jm / 4), mu = int(jm - size_t(j) * 4);
  const int col = int(idx / m), row = int(idx - size_t(col) * m);
  const int jb = cnb[j * 8 + 4 + mu];
  Y[(size_t(j) * 9 + 5 + mu) * nent + idx] = s3adj(Y + (size_t(jb) * 9 + 1 + mu) * nent, m, k, row, col);
}

// ---------------------------------------------------------------------------------------
__global__ void k_chiral_gather(const double2* __restrict__ fine, double2* __restrict__ blocks,
                                const int* __restrict__ bsite, int nd, int N, int r, int V) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  const int v = blockIdx.y, ja = blockIdx.z;
  if (row >= N) return;
  const int j = ja >> 1, a = ja & 1;
  const int s6 = row / nd, ib = row - s6 * nd;
  const int site = bsite[size_t(j) * nd + ib];
  blocks[(size_t(ja) * r + v) * N + row] = fine[(size_t(v) * 12 + 6 * a + s6) * V + site];
}

__global__ void k_export_P(const double2* __restrict__ P, double2* __restrict__ out, int nd, int N, int k, size_t n) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= n) return;
  // out [ja][row_c][i], row_c = 6 ib + s6
  const int i = int(g % k);
  const size_t t = g / k;
  const int rowc = int(t % N);
  const size_t ja = t / N;
  const int ib = rowc / 6, s6 = rowc - 6 * ib;
  out[g] = P[(ja * k + i) * N + size_t(s6) * nd + ib];
}

__global__ void k_export_Y(const double2* __restrict__ Y, double2* __restrict__ out, int m, size_t n) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= n) return;
  const int col = int(g % m);
  const size_t t = g / m;
  const int row = int(t % m);
  const size_t blk = t / m;
  out[g] = Y[(blk * m + col) * m + row];
}

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = uint64_t(M0) * c[0], p1 = uint64_t(M1) * c[2];
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0), hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ void k_philox(double2* __restrict__ out, uint64_t seed, int v0, int V) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  const int vi = blockIdx.y;
  if (site >= V) return;
  const uint32_t k0 = uint32_t(seed & 0xffffffffu), k1 = uint32_t(seed >> 32);
  const double twopi = 2.0 * M_PI;
  for (int g = 0; g < 6; ++g) {
    uint32_t c[4] = {uint32_t(site), uint32_t(g), uint32_t(v0 + vi), 0u};
    philox4x32_10(c, k0, k1);
    double u[4];
    for (int q = 0; q < 4; ++q) u[q] = (double(c[q]) + 0.5) * 0x1p-32;
    const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    const double t0 = twopi * u[1], t1 = twopi * u[3];
    out[(size_t(vi) * 12 + 2 * g) * V + site] = make_double2(r0 * cos(t0), r0 * sin(t0));
    out[(size_t(vi) * 12 + 2 * g + 1) * V + site] = make_double2(r1 * cos(t1), r1 * sin(t1));
  }
}

// The same generator for many lattices in padded layouts: vector v of lattice l (blockIdx.z)
// at [(l n + v) 12 + comp][Vpad]; sites at and beyond the lattice's volume are zero.
__global__ void k_philox_padded(double2* __restrict__ out, uint64_t seed, int v0, int n, const int* __restrict__ Vl,
                                int Vpad) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  const int vi = blockIdx.y, l = blockIdx.z;
  if (site >= Vpad) return;
  double2* o = out + size_t(l) * n * 12 * Vpad;
  if (site >= Vl[l]) {
    for (int c = 0; c < 12; ++c) o[(size_t(vi) * 12 + c) * Vpad + site] = make_double2(0.0, 0.0);
    return;
  }
  const uint32_t k0 = uint32_t(seed & 0xffffffffu), k1 = uint32_t(seed >> 32);
  const double twopi = 2.0 * M_PI;
  for (int g = 0; g < 6; ++g) {
    uint32_t c[4] = {uint32_t(site), uint32_t(g), uint32_t(v0 + vi), 0u};
    philox4x32_10(c, k0, k1);
    double u[4];
    for (int q = 0; q < 4; ++q) u[q] = (double(c[q]) + 0.5) * 0x1p-32;
    const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    const double t0 = twopi * u[1], t1 = twopi * u[3];
    o[(size_t(vi) * 12 + 2 * g) * Vpad + site] = make_double2(r0 * cos(t0), r0 * sin(t0));
    o[(size_t(vi) * 12 + 2 * g + 1) * Vpad + site] = make_double2(r1 * cos(t1), r1 * sin(t1));
  }
}

// ---------------------------------------------------------------------------------------
// link force, canonical FP64
__constant__ double2 c_gamma[4][16];  // gamma_mu, row-major 4x4

__global__ void k_link_force(const double2* __restrict__ x, const double2* __restrict__ lam, double2* __restrict__ dU,
                             int L0, int L1, int L2, int L3, int bc_t, double cws, double cwt, int nrhs, int V) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  const int mu = blockIdx.y;
  if (site >= V) return;
  const int Ls[4] = {L0, L1, L2, L3};
  int c[4];
  {
    int rem = site;
    for (int q = 0; q < 4; ++q) { c[q] = rem % Ls[q]; rem /= Ls[q]; }
  }
  int cy[4] = {c[0], c[1], c[2], c[3]};
  cy[mu] = (c[mu] + 1) % Ls[mu];
  const int y = cy[0] + L0 * (cy[1] + L1 * (cy[2] + L2 * cy[3]));
  cplx<double> G[9];
  for (int e = 0; e < 9; ++e) G[e] = {0, 0};
  for (int r = 0; r < nrhs; ++r) {
    const double2* xx = x + (size_t(r) * V + site) * 12;
    const double2* xy = x + (size_t(r) * V + y) * 12;
    const double2* lx = lam + (size_t(r) * V + site) * 12;
    const double2* ly = lam + (size_t(r) * V + y) * 12;
    for (int s = 0; s < 4; ++s)
      for (int t = 0; t < 4; ++t) {
        const double2 gm = c_gamma[mu][s * 4 + t];
        const cplx<double> pm = {(s == t ? 1.0 : 0.0) - gm.x, -gm.y};  // (1 - gamma)_{st}
        const cplx<double> pp = {(s == t ? 1.0 : 0.0) + gm.x, gm.y};   // (1 + gamma)_{st}
        if (pm.re == 0 && pm.im == 0 && pp.re == 0 && pp.im == 0) continue;
        for (int aa = 0; aa < 3; ++aa)
          for (int bb = 0; bb < 3; ++bb) {
            const double2 x1 = xy[3 * t + aa], l1 = lx[3 * s + bb];
            const double2 l2 = ly[3 * t + aa], x2 = xx[3 * s + bb];
            G[3 * aa + bb] += pm * cmul_conj(cplx<double>{l1.x, l1.y}, cplx<double>{x1.x, x1.y});
            G[3 * aa + bb] += pp * cmul_conj(cplx<double>{x2.x, x2.y}, cplx<double>{l2.x, l2.y});
          }
      }
  }
  double sg = 1.0;
  if (mu == 3 && bc_t < 0 && c[3] == L3 - 1) sg = -1.0;
  const double f = 0.5 * (mu == 3 ? cwt : cws) * sg;
  for (int aa = 0; aa < 3; ++aa)
    for (int bb = 0; bb < 3; ++bb) {
      const cplx<double> gba = G[3 * bb + aa];  // (G^dag)_{ab} = conj(G_{ba})
      dU[(size_t(mu) * V + site) * 9 + 3 * aa + bb] = make_double2(f * gba.re, -f * gba.im);
    }
}

// ---------------------------------------------------------------------------------------
// layout conversion
template <class Sc, class Sn>
__global__ void k_pack_spinor(const Sc* __restrict__ in, Sn* __restrict__ out, int V, size_t n) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;  // canonical index
  if (g >= n) return;
  const int comp = int(g % 12);
  const size_t t = g / 12;
  const int site = int(t % V);
  const size_t rhs = t / V;
  stc(out, (rhs * 12 + comp) * V + site, ldc(in, g));
}
template <class Sn, class Sc>
__global__ void k_unpack_spinor(const Sn* __restrict__ in, Sc* __restrict__ out, int V, size_t n) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= n) return;
  const int comp = int(g % 12);
  const size_t t = g / 12;
  const int site = int(t % V);
  const size_t rhs = t / V;
  stc(out, g, ldc(in, (rhs * 12 + comp) * V + site));
}
template <class S>
__global__ void k_pack_gauge(const double2* __restrict__ in, S* __restrict__ out, int V, size_t n) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= n) return;
  const int e = int(g % 9);
  const size_t t = g / 9;
  const int site = int(t % V);
  const size_t mu = t / V;
  const double2 v = in[g];
  stc(out, (mu * 9 + e) * V + site, cplx<double>{v.x, v.y});
}
template <class Si, class So>
__global__ void k_convert(const Si* __restrict__ in, So* __restrict__ out, size_t n) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= n) return;
  auto v = ldc(in, g);
  stc(out, g, v);
}

// ---------------------------------------------------------------------------------------
// Third level (Algorithm 4 applied to the coarse stencil D_c)

// coarse test vectors [n][d][m] FP64: Philox counter (j, g, v, level), components 2g, 2g + 1
__global__ void k_philox_coarse(double2* __restrict__ out, uint64_t seed, int v0, int d, int m, int level) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int vi = blockIdx.y;
  if (j >= d) return;
  const uint32_t k0 = uint32_t(seed & 0xffffffffu), k1 = uint32_t(seed >> 32);
  const double twopi = 2.0 * M_PI;
  for (int g = 0; g < m / 2; ++g) {
    uint32_t c[4] = {uint32_t(j), uint32_t(g), uint32_t(v0 + vi), uint32_t(level)};
    philox4x32_10(c, k0, k1);
    double u[4];
    for (int q = 0; q < 4; ++q) u[q] = (double(c[q]) + 0.5) * 0x1p-32;
    const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    const double t0 = twopi * u[1], t1 = twopi * u[3];
    double2* o = out + (size_t(vi) * d + j) * m;
    o[2 * g] = make_double2(r0 * cos(t0), r0 * sin(t0));
    o[2 * g + 1] = make_double2(r1 * cos(t1), r1 * sin(t1));
  }
}

// chiral split + block gather of coarse vectors: blocks[(2J + alpha) * r + v][row], row = i * nd + jb,
// from v[v][j][alpha * k1 + i] with j = bsite[J][jb]
__global__ void k_level_gather(const double2* __restrict__ v, double2* __restrict__ blocks,
                               const int* __restrict__ bsite, int nd, int k1, int d1, int r) {
  const int N = nd * k1;
  const int row = blockIdx.x * 256 + threadIdx.x;
  const int vi = blockIdx.y, ja = blockIdx.z;  // ja = 2J + alpha
  if (row >= N) return;
  const int J = ja >> 1, a = ja & 1;
  const int i = row / nd, jb = row - i * nd;
  const int j = bsite[J * nd + jb];
  blocks[(size_t(ja) * r + vi) * N + row] = v[(size_t(vi) * d1 + j) * (2 * k1) + a * k1 + i];
}

// v1[rhs][j][alpha k1 + i] = sum_l P[(2J + alpha) k + l][row] v2[rhs][J][alpha k + l]
template <class S>
__global__ __launch_bounds__(256) void k_level_prolong(const S* __restrict__ P, const S* __restrict__ v2,
                                                       S* __restrict__ v1, const int* __restrict__ bsite, int nd,
                                                       int k1, int k, int d1, int d) {
  using C = ctype<S>;
  const int N = nd * k1;
  const int row = blockIdx.x * 256 + threadIdx.x;
  const int ja = blockIdx.y, rhs = blockIdx.z;
  if (row >= N) return;
  const int J = ja >> 1, a = ja & 1;
  const S* Pc = P + size_t(ja) * k * N;
  const S* c = v2 + (size_t(rhs) * d + J) * (2 * k) + a * k;
  cplx<C> acc = {C(0), C(0)};
  for (int l = 0; l < k; ++l) acc += ldc(Pc, size_t(l) * N + row) * ldc(c, l);
  const int i = row / nd, jb = row - i * nd;
  const int j = bsite[J * nd + jb];
  stc(v1, (size_t(rhs) * d1 + j) * (2 * k1) + a * k1 + i, acc);
}

// v2[rhs][J][alpha k + l] = sum_row conj(P[(2J + alpha) k + l][row]) v1[rhs][j(row)][alpha k1 + i(row)]
// one workgroup per (J, alpha, rhs): the block's N entries of v1 staged in LDS, one wavefront per l
template <class S>
__global__ __launch_bounds__(256) void k_level_restrict(const S* __restrict__ P, const S* __restrict__ v1,
                                                        S* __restrict__ v2, const int* __restrict__ bsite, int nd,
                                                        int k1, int k, int d1, int d) {
  using C = ctype<S>;
  extern __shared__ unsigned char smem_raw[];
  cplx<C>* vb = reinterpret_cast<cplx<C>*>(smem_raw);  // [N]
  const int N = nd * k1;
  const int ja = blockIdx.x, rhs = blockIdx.y;
  const int J = ja >> 1, a = ja & 1;
  for (int row = threadIdx.x; row < N; row += blockDim.x) {
    const int i = row / nd, jb = row - i * nd;
    const int j = bsite[J * nd + jb];
    vb[row] = ldc(v1, (size_t(rhs) * d1 + j) * (2 * k1) + a * k1 + i);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const S* Pc = P + size_t(ja) * k * N;
  for (int l = w; l < k; l += nw) {
    double sr = 0.0, si = 0.0;
    for (int row = lane; row < N; row += 64) {
      const cplx<C> p = ldc(Pc, size_t(l) * N + row), x = vb[row];
      sr += double(p.re) * double(x.re) + double(p.im) * double(x.im);
      si += double(p.re) * double(x.im) - double(p.im) * double(x.re);
    }
    for (int off = 32; off > 0; off >>= 1) {
      sr += __shfl_xor(sr, off, 64);
      si += __shfl_xor(si, off, 64);
    }
    if (lane == 0) stc(v2, (size_t(rhs) * d + J) * (2 * k) + a * k + l, cplx<double>{sr, si});
  }
}

// Y2[J][slot] = sum over the (site jb, term dir1) pairs of this slot of R(j)^dag Y1_dir1(j) R(t),
// R(x)[(alpha, i), (alpha, l)] = P[(2 J(x) + alpha) k + l][i nd + jb(x)] (block diagonal in alpha).
// Workgroup (J, slot): slot 0 takes the self terms and the hops that stay inside the block, slot
// 1 + dir the hops in direction dir that leave it through its face.  T = Y1 R(t) is staged in
// LDS, then every thread adds its entries of R(j)^dag T.  FP64.
struct LevelBuildArgs {
  int cL1[4], b[4];
  int nd, k1, k, d1, d;
};

__global__ __launch_bounds__(256) void k_level_build(const double2* __restrict__ Y1, const int* __restrict__ cnb1,
                                                     const double2* __restrict__ P, const int* __restrict__ bsite,
                                                     const int* __restrict__ agg, const int* __restrict__ pos,
                                                     double2* __restrict__ Y2, LevelBuildArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int m1 = 2 * a.k1, m2 = 2 * a.k, N = a.nd * a.k1;
  cplx<double>* T = reinterpret_cast<cplx<double>*>(smem_raw);  // [m1][m2] column-major (row (beta, i'))
  cplx<double>* Rj = T + size_t(m1) * m2;                        // [2][k][k1]: conj P rows of site j
  cplx<double>* Rt = Rj + size_t(2) * a.k * a.k1;                // [2][k][k1]: P rows of site t
  const int J = blockIdx.x, slot = blockIdx.y;
  constexpr int MAXE = 16;  // (2k)^2 / 256 entries per thread, 2k <= 64
  cplx<double> acc[MAXE];
#pragma unroll
  for (int q = 0; q < MAXE; ++q) acc[q] = {0.0, 0.0};
  const int ne = m2 * m2;
  for (int jb = 0; jb < a.nd; ++jb) {
    const int j = bsite[J * a.nd + jb];
    int c[4], rem = j;
    for (int q = 0; q < 4; ++q) {
      c[q] = rem % a.cL1[q];
      rem /= a.cL1[q];
    }
    for (int dir1 = 0; dir1 < 9; ++dir1) {
      int target;  // slot this term belongs to
      if (dir1 == 0) {
        target = 0;
      } else {
        const int dd = dir1 - 1, mu = dd & 3;
        const bool face = dd < 4 ? (c[mu] % a.b[mu] == a.b[mu] - 1) : (c[mu] % a.b[mu] == 0);
        target = face ? dir1 : 0;
      }
      if (target != slot) continue;
      const int t = dir1 == 0 ? j : cnb1[j * 8 + dir1 - 1];
      const int Jt = agg[t], jbt = pos[t];
      __syncthreads();  // the previous pair is done with T, Rj, Rt
      for (int e = threadIdx.x; e < 2 * a.k * a.k1; e += blockDim.x) {
        const int al = e / (a.k * a.k1), rem2 = e - al * a.k * a.k1, l = rem2 / a.k1, i = rem2 - l * a.k1;
        const double2 pj = P[(size_t(2 * J + al) * a.k + l) * N + i * a.nd + jb];
        const double2 pt = P[(size_t(2 * Jt + al) * a.k + l) * N + i * a.nd + jbt];
        Rj[e] = {pj.x, -pj.y};
        Rt[e] = {pt.x, pt.y};
      }
      __syncthreads();
      // T[(beta, i'), (alpha, l)] = sum_i Y1[(beta, i'), (alpha, i)] Rt[alpha][l][i]
      const double2* Yb = Y1 + (size_t(j) * 9 + dir1) * m1 * m1;  // column-major
      for (int e = threadIdx.x; e < m1 * m2; e += blockDim.x) {
        const int col = e / m1, row = e - col * m1;  // col = (alpha, l), row = (beta, i')
        const int al = col / a.k, l = col - al * a.k;
        cplx<double> v = {0.0, 0.0};
        for (int i = 0; i < a.k1; ++i) {
          const double2 y = Yb[size_t(al * a.k1 + i) * m1 + row];
          v += cplx<double>{y.x, y.y} * Rt[(al * a.k + l) * a.k1 + i];
        }
        T[e] = v;
      }
      __syncthreads();
      // acc[(beta, l'), (alpha, l)] += sum_i' Rj[beta][l'][i'] T[(beta, i'), (alpha, l)]
#pragma unroll
      for (int q = 0; q < MAXE; ++q) {
        const int e = threadIdx.x + q * 256;
        if (e < ne) {
          const int col = e / m2, row = e - col * m2;  // row = (beta, l'), col = (alpha, l)
          const int be = row / a.k, lp = row - be * a.k;
          cplx<double> v = {0.0, 0.0};
          for (int ip = 0; ip < a.k1; ++ip) v += Rj[(be * a.k + lp) * a.k1 + ip] * T[size_t(col) * m1 + be * a.k1 + ip];
          acc[q] += v;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < MAXE; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e < ne) Y2[(size_t(J) * 9 + slot) * ne + e] = make_double2(acc[q].re, acc[q].im);  // column-major
  }
}

// canonical export of the third level's P: [d][2][N][k] with rows (jb * k1 + i)
__global__ void k_level_export_P(const double2* __restrict__ P, double2* __restrict__ out, int nd, int k1, int k,
                                 size_t n) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= n) return;
  const int N = nd * k1;
  const int l = int(g % k);
  const size_t t = g / k;
  const int crow = int(t % N);            // canonical row jb * k1 + i
  const size_t ja = t / N;
  const int jb = crow / k1, i = crow - jb * k1;
  out[g] = P[(ja * k + l) * N + size_t(i) * nd + jb];
}

template <class F>
void dispatch_prec(qmg_prec p, F&& f) {
  switch (p) {
    case QMG_F64: f(double2{}); break;
    case QMG_F32: f(float2{}); break;
    case QMG_BF16: f(cbf16{}); break;
    case QMG_F16: f(chalf{}); break;
  }
}

}  // namespace

// pack width over the rows of P (N rows per column; every column starts at a multiple of N)
template <class S>
static int row_pack(int N) {
  return (N % kPack<S> == 0) ? kPack<S> : 1;
}

void launch_prolong(qmg_prec prec, const HierarchyDev& h, const void* P, const void* coarse, void* fine, int nrhs,
                    hipStream_t st) {
  TimedLaunch tl("prolong", st, double(h.g.V) * (12.0 * h.k + 12.0 * nrhs) * prec_bytes(prec),
                 8.0 * 12.0 * h.k * h.g.V * nrhs);
  QMG_CHECK(h.k <= 64, QMG_EINVAL, "prolong: rank above 64");
  dispatch_prec(prec, [&](auto tag) {
    using S = decltype(tag);
    constexpr int PK = kPack<S>;
    const bool packed = row_pack<S>(h.blk.N) == PK;
    auto go = [&](auto pr, auto nrt) {
      constexpr int PR = decltype(pr)::value, NR = decltype(nrt)::value;
      const int npack = int(cdiv(h.blk.N / PR, 256));
      const size_t nwg = size_t(npack) * 2 * h.blk.d * cdiv(nrhs, NR);
      QMG_CHECK(nwg < (size_t(1) << 31), QMG_EINVAL, "prolong: grid too large");
      launch(k_prolong<S, PR, NR>, dim3(unsigned(nwg)), dim3(256), 0, st, P, coarse, fine, h.bsite.as<int>(),
             h.blk.nd, h.blk.N, h.k, h.blk.d, h.g.V, nrhs, npack);
    };
    using one = std::integral_constant<int, 1>;
    using four = std::integral_constant<int, 4>;
    using pk = std::integral_constant<int, PK>;
    // groups of four right-hand sides (the last one ragged) read P once per group: already
    // from two right-hand sides on, since P is larger than the vectors
    if (packed) {
      if (nrhs >= 2) go(pk{}, four{});
      else go(pk{}, one{});
    } else {
      if (nrhs >= 2) go(one{}, four{});
      else go(one{}, one{});
    }
  });
  QMG_LAUNCH_CHECK();
}

void launch_restrict(qmg_prec prec, const HierarchyDev& h, const void* P, const void* fine, void* coarse, int nrhs,
                     hipStream_t st) {
  TimedLaunch tl("restrict", st, double(h.g.V) * (12.0 * h.k + 12.0 * nrhs) * prec_bytes(prec),
                 8.0 * 12.0 * h.k * h.g.V * nrhs);
  dispatch_prec(prec, [&](auto tag) {
    using S = decltype(tag);
    constexpr int PK = kPack<S>;
    const bool packed = row_pack<S>(h.blk.N) == PK;
    auto go = [&](auto pr, auto nrt) {
      constexpr int PR = decltype(pr)::value, NR = decltype(nrt)::value;
      const size_t lds = size_t(NR) * h.blk.N * sizeof(cplx<ctype<S>>);
      QMG_CHECK(lds <= 96 * 1024, QMG_EINVAL, "restrict: aggregate too large for LDS staging");
      launch(k_restrict<S, PR, NR>, dim3(2 * h.blk.d, cdiv(nrhs, NR)), dim3(256), uint32_t(lds), st, P, fine,
             coarse, h.bsite.as<int>(), h.blk.nd, h.blk.N, h.k, h.blk.d, h.g.V, nrhs);
    };
    using one = std::integral_constant<int, 1>;
    using four = std::integral_constant<int, 4>;
    using pk = std::integral_constant<int, PK>;
    const bool multi = nrhs >= 2 && size_t(4) * h.blk.N * sizeof(cplx<ctype<S>>) <= 96 * 1024;
    if (packed) {
      if (multi) go(pk{}, four{});
      else go(pk{}, one{});
    } else {
      if (multi) go(one{}, four{});
      else go(one{}, one{});
    }
  });
  QMG_LAUNCH_CHECK();
}

void launch_coarse_apply(qmg_prec prec, const HierarchyDev& h, const void* Y, const void* in, void* out, int nrhs,
                         hipStream_t st, const int* skip) {
  TimedLaunch tl("coarse_apply", st, double(h.blk.d) * (9.0 * 4 * h.k * h.k + 4.0 * h.k * nrhs) * prec_bytes(prec),
                 8.0 * 9.0 * 4 * h.k * h.k * h.blk.d * nrhs);
  launch_stencil_apply(prec, h.blk.d, h.k, h.cnb.as<int>(), Y, in, out, nrhs, st, skip);
}

void launch_stencil_apply(qmg_prec prec, int d, int k, const int* cnb, const void* Y, const void* in, void* out,
                          int nrhs, hipStream_t st, const int* skip) {
  const int m = 2 * k;
  dispatch_prec(prec, [&](auto tag) {
    using S = decltype(tag);
    constexpr int PK = kPack<S>;
    auto go = [&](auto kern, int NR, int PR) {
      const int mp = m / PR;
      const int H = std::max(1, std::min(8, 1024 / (9 * mp)));
      const int threads = int(std::min<size_t>(1024, ((size_t(9) * mp * H + 63) / 64) * 64));
      const size_t lds = size_t(NR) * 9 * m * (1 + H) * sizeof(cplx<ctype<S>>);
      QMG_CHECK(lds <= 160 * 1024, QMG_EINVAL, "coarse apply: block too large for LDS staging");
      if (lds > 64 * 1024)
        QMG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
      launch(kern, dim3(d, (nrhs + NR - 1) / NR), dim3(threads), uint32_t(lds), st, Y, in, out, cnb, d, m, nrhs, H,
             skip);
    };
    const bool packed = m % PK == 0;
    if (packed) {
      if (nrhs >= 3) go(k_coarse_apply<S, 4, PK>, 4, PK);
      else if (nrhs == 2) go(k_coarse_apply<S, 2, PK>, 2, PK);
      else go(k_coarse_apply<S, 1, PK>, 1, PK);
    } else {
      if (nrhs >= 3) go(k_coarse_apply<S, 4, 1>, 4, 1);
      else if (nrhs == 2) go(k_coarse_apply<S, 2, 1>, 2, 1);
      else go(k_coarse_apply<S, 1, 1>, 1, 1);
    }
  });
  QMG_LAUNCH_CHECK();
}

void build_coarse(HierarchyDev& h, hipStream_t st) {
  QMG_CHECK(2 * h.k <= kMaxM && h.k <= 32, QMG_ESHAPE, "coarse build supports k <= 32");
  BuildArgs a{};
  for (int q = 0; q < 4; ++q) {
    a.L[q] = h.g.L[q];
    a.b[q] = h.blk.b[q];
    a.cL[q] = h.blk.cL[q];
    a.cw[q] = h.g.cw(q);
  }
  a.V = h.g.V;
  a.nd = h.blk.nd;
  a.N = h.blk.N;
  a.k = h.k;
  a.d = h.blk.d;
  a.bc_t = h.g.bc_t;
  a.diag = h.g.diag();
  a.clov = static_cast<const double2*>(h.A64.p);
  TimedLaunch tl("coarse_build", st, double(h.g.V) * 12.0 * h.k * 16.0 + 9.0 * h.blk.d * 4.0 * h.k * h.k * 16.0,
                 double(h.g.V) * 4.0 * (2.0 * h.k) * (2.0 * h.k) * 6.0 * 8.0, false);
  const int nent = 4 * h.k * h.k;
  DevBuf W(size_t(8) * h.blk.d * nent * sizeof(double2));
  // per site: Px (12 k) + HP (24 k) + link (9) complex, + coefficient and 5 ints
  const size_t per_site = size_t(12 * h.k + 24 * h.k + 9) * sizeof(cplx<double>) + sizeof(double) + 5 * sizeof(int);
  // sites staged per phase within 76 KB of LDS, so that two workgroups share a CU (their
  // register use allows two) and one's loads overlap the other's products: at 32^3 x 64, k = 24
  // (5 sites) 70 ms against 106 ms with 110 KB (one workgroup per CU); smaller budgets are slower
  const int NS = int(std::max<size_t>(1, std::min<size_t>(16, (76 * 1024) / per_site)));
  const size_t lds = per_site * NS;
  auto go = [&](auto kern) {
    if (lds > 64 * 1024) QMG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     int(lds)));
    kern<<<dim3(h.blk.d, 4), 256, lds, st>>>(h.U64.as<double2>(), h.P64.as<double2>(), h.bsite.as<int>(),
                                             h.blists.as<int>(), h.Y64.as<double2>(), W.as<double2>(), a, NS);
  };
  if (h.k <= 24) go(k_build_coarse<3>);
  else go(k_build_coarse<4>);
  QMG_LAUNCH_CHECK();
  k_sum_self<<<cdiv(size_t(h.blk.d) * nent, 256), 256, 0, st>>>(W.as<double2>(), h.Y64.as<double2>(), h.blk.d,
                                                                2 * h.k, h.k);
  QMG_LAUNCH_CHECK();
  k_fill_backward<<<cdiv(size_t(h.blk.d) * 4 * nent, 256), 256, 0, st>>>(h.Y64.as<double2>(), h.cnb.as<int>(),
                                                                        h.blk.d, 2 * h.k, h.k);
  QMG_LAUNCH_CHECK();
  QMG_HIP(hipStreamSynchronize(st));  // W is released on return
}

void launch_chiral_gather(const HierarchyDev& h, const void* fine, void* blocks, int r, hipStream_t st) {
  dim3 grid(cdiv(h.blk.N, 256), r, 2 * h.blk.d);
  {
    TimedLaunch tl_("setup/gather", st, double(r) * h.g.V * 12 * 2 * 16, 0.0);
    launch(k_chiral_gather, dim3(grid), dim3(256), 0, st, (const double2*)fine, (double2*)blocks, h.bsite.as<int>(),
           h.blk.nd, h.blk.N, r, h.g.V);
  }
  QMG_LAUNCH_CHECK();
}

void launch_export_P(const HierarchyDev& h, void* out, hipStream_t st) {
  const size_t n = size_t(h.blk.d) * 2 * h.blk.N * h.k;
  {
    TimedLaunch tl_("export", st, 2.0 * double(n) * 16, 0.0);
    launch(k_export_P, dim3(cdiv(n, 256)), dim3(256), 0, st, h.P64.as<double2>(), (double2*)out, h.blk.nd, h.blk.N,
           h.k, n);
  }
  QMG_LAUNCH_CHECK();
}

void launch_export_Y(const HierarchyDev& h, void* out, hipStream_t st) {
  const int m = 2 * h.k;
  const size_t n = size_t(h.blk.d) * 9 * m * m;
  {
    TimedLaunch tl_("export", st, 2.0 * double(n) * 16, 0.0);
    launch(k_export_Y, dim3(cdiv(n, 256)), dim3(256), 0, st, h.Y64.as<double2>(), (double2*)out, m, n);
  }
  QMG_LAUNCH_CHECK();
}

void launch_philox_padded(uint64_t seed, int v0, int n, int nl, const int* Vl, int Vpad, void* out, hipStream_t st) {
  {
    TimedLaunch tl_("batch/philox", st, double(nl) * n * Vpad * 12 * 16, 0.0);
    launch(k_philox_padded, dim3(cdiv(Vpad, 256), n, nl), dim3(256), 0, st, (double2*)out, seed, v0, n, Vl, Vpad);
  }
  QMG_LAUNCH_CHECK();
}

void launch_philox_native(const Geom& g, uint64_t seed, int v0, int n, void* out, hipStream_t st) {
  {
    TimedLaunch tl_("setup/philox", st, double(n) * g.V * 12 * 16, 0.0);
    launch(k_philox, dim3(cdiv(g.V, 256), n), dim3(256), 0, st, (double2*)out, seed, v0, g.V);
  }
  QMG_LAUNCH_CHECK();
}

void launch_link_force(const Geom& g, const void* x, const void* lam, void* dU, int nrhs, hipStream_t st) {
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
      // -i sigma_1 = [[0,-i],[-i,0]] ; i sigma_1 = [[0,i],[i,0]]
      set(0, 0, 3, 0, -1); set(0, 1, 2, 0, -1); set(0, 2, 1, 0, 1); set(0, 3, 0, 0, 1);
      // -i sigma_2 = [[0,-1],[1,0]] ; i sigma_2 = [[0,1],[-1,0]]
      set(1, 0, 3, -1, 0); set(1, 1, 2, 1, 0); set(1, 2, 1, 1, 0); set(1, 3, 0, -1, 0);
      // -i sigma_3 = [[-i,0],[0,i]] ; i sigma_3 = [[i,0],[0,-i]]
      set(2, 0, 2, 0, -1); set(2, 1, 3, 0, 1); set(2, 2, 0, 0, 1); set(2, 3, 1, 0, -1);
      // gamma_t
      set(3, 0, 2, 1, 0); set(3, 1, 3, 1, 0); set(3, 2, 0, 1, 0); set(3, 3, 1, 1, 0);
      QMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gamma), gm, sizeof(gm)));
      if (dev >= 0 && dev < 64) init[dev] = true;
    }
  }
  {
    TimedLaunch tl_("force", st, double(g.V) * (nrhs * 48.0 + 72.0) * 8, 0.0);
    launch(k_link_force, dim3(cdiv(g.V, 256), 4), dim3(256), 0, st, (const double2*)x, (const double2*)lam,
           (double2*)dU, g.L[0], g.L[1], g.L[2], g.L[3], g.bc_t, g.cw(0), g.cw(3), nrhs, g.V);
  }
  QMG_LAUNCH_CHECK();
}

void launch_pack_spinor(const void* canon, qmg_prec pc, void* native, qmg_prec pn, int V, int nrhs,
                        hipStream_t st) {
  const size_t n = size_t(nrhs) * V * 12;
  dispatch_prec(pc, [&](auto tc) {
    using Sc = decltype(tc);
    dispatch_prec(pn, [&](auto tn) {
      using Sn = decltype(tn);
      {
        TimedLaunch tl_("layout/spinor", st, double(n) * (sizeof(Sc) + sizeof(Sn)), 0.0);
        launch(k_pack_spinor<Sc, Sn>, dim3(cdiv(n, 256)), dim3(256), 0, st, (const Sc*)canon, (Sn*)native, V, n);
      }
    });
  });
  QMG_LAUNCH_CHECK();
}
void launch_unpack_spinor(const void* native, qmg_prec pn, void* canon, qmg_prec pc, int V, int nrhs,
                          hipStream_t st) {
  const size_t n = size_t(nrhs) * V * 12;
  dispatch_prec(pn, [&](auto tn) {
    using Sn = decltype(tn);
    dispatch_prec(pc, [&](auto tc) {
      using Sc = decltype(tc);
      {
        TimedLaunch tl_("layout/spinor", st, double(n) * (sizeof(Sc) + sizeof(Sn)), 0.0);
        launch(k_unpack_spinor<Sn, Sc>, dim3(cdiv(n, 256)), dim3(256), 0, st, (const Sn*)native, (Sc*)canon, V, n);
      }
    });
  });
  QMG_LAUNCH_CHECK();
}
void launch_pack_gauge(const void* canon, void* native, qmg_prec prec, int V, hipStream_t st) {
  const size_t n = size_t(4) * V * 9;
  dispatch_prec(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("layout/gauge", st, double(n) * (16.0 + sizeof(S)), 0.0);
      launch(k_pack_gauge<S>, dim3(cdiv(n, 256)), dim3(256), 0, st, (const double2*)canon, (S*)native, V, n);
    }
  });
  QMG_LAUNCH_CHECK();
}
void launch_convert(const void* in, qmg_prec pin, void* out, qmg_prec pout, size_t n, hipStream_t st) {
  if (!n) return;
  dispatch_prec(pin, [&](auto ti) {
    using Si = decltype(ti);
    dispatch_prec(pout, [&](auto to) {
      using So = decltype(to);
      {
        TimedLaunch tl_("layout/convert", st, double(n) * (sizeof(Si) + sizeof(So)), 0.0);
        launch(k_convert<Si, So>, dim3(cdiv(n, 256)), dim3(256), 0, st, (const Si*)in, (So*)out, n);
      }
    });
  });
  QMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// third level: launchers
void launch_philox_coarse(uint64_t seed, int v0, int n, int d, int m, int level, void* out, hipStream_t st) {
  {
    TimedLaunch tl_("level/philox", st, double(n) * d * m * 16, 0.0);
    launch(k_philox_coarse, dim3(cdiv(d, 256), n), dim3(256), 0, st, (double2*)out, seed, v0, d, m, level);
  }
  QMG_LAUNCH_CHECK();
}

void launch_level_gather(const CoarseLevel& L, const void* v, void* blocks, int r, hipStream_t st) {
  const int d1 = L.d * L.nd;
  {
    TimedLaunch tl_("level/gather", st, double(r) * d1 * L.k1 * 2 * 2 * 16, 0.0);
    launch(k_level_gather, dim3(cdiv(L.N, 256), r, 2 * L.d), dim3(256), 0, st, (const double2*)v, (double2*)blocks,
           L.bsite.as<int>(), L.nd, L.k1, d1, r);
  }
  QMG_LAUNCH_CHECK();
}

void launch_level_prolong(qmg_prec prec, const CoarseLevel& L, int d1, const void* P, const void* v2, void* v1,
                          int nrhs, hipStream_t st) {
  TimedLaunch tl("level_prolong", st, (2.0 * L.d * L.k * L.N + double(nrhs) * (2.0 * L.d * L.k + 2.0 * d1 * L.k1)) *
                                          prec_bytes(prec),
                 8.0 * 2.0 * L.d * L.k * L.N * nrhs);
  dispatch_prec(prec, [&](auto tag) {
    using S = decltype(tag);
    launch(k_level_prolong<S>, dim3(cdiv(L.N, 256), 2 * L.d, nrhs), dim3(256), 0, st, (const S*)P, (const S*)v2,
           (S*)v1, L.bsite.as<int>(), L.nd, L.k1, L.k, d1, L.d);
  });
  QMG_LAUNCH_CHECK();
}

void launch_level_restrict(qmg_prec prec, const CoarseLevel& L, int d1, const void* P, const void* v1, void* v2,
                           int nrhs, hipStream_t st) {
  TimedLaunch tl("level_restrict", st, (2.0 * L.d * L.k * L.N + double(nrhs) * (2.0 * L.d * L.k + 2.0 * d1 * L.k1)) *
                                           prec_bytes(prec),
                 8.0 * 2.0 * L.d * L.k * L.N * nrhs);
  dispatch_prec(prec, [&](auto tag) {
    using S = decltype(tag);
    const size_t lds = size_t(L.N) * sizeof(cplx<ctype<S>>);
    QMG_CHECK(lds <= 64 * 1024, QMG_ESHAPE, "level restrict: block of %d rows too large", L.N);
    launch(k_level_restrict<S>, dim3(2 * L.d, nrhs), dim3(256), uint32_t(lds), st, (const S*)P, (const S*)v1,
           (S*)v2, L.bsite.as<int>(), L.nd, L.k1, L.k, d1, L.d);
  });
  QMG_LAUNCH_CHECK();
}

void build_level_coarse(CoarseLevel& L, const StencilRef& h, hipStream_t st) {
  const int m2 = 2 * L.k, m1 = 2 * L.k1;
  QMG_CHECK(m2 <= 64 && m1 <= 64, QMG_ESHAPE, "third level: 2k <= 64 on both levels");
  LevelBuildArgs a{};
  for (int q = 0; q < 4; ++q) {
    a.cL1[q] = h.cL[q];
    a.b[q] = L.b[q];
  }
  a.nd = L.nd;
  a.k1 = L.k1;
  a.k = L.k;
  a.d1 = h.d;
  a.d = L.d;
  L.Y64.alloc(size_t(L.d) * 9 * m2 * m2 * sizeof(double2));
  const size_t lds = (size_t(m1) * m2 + size_t(4) * L.k * L.k1) * sizeof(cplx<double>);
  QMG_CHECK(lds <= 160 * 1024, QMG_ESHAPE, "third level: coarse build needs too much LDS");
  if (lds > 64 * 1024)
    QMG_HIP(hipFuncSetAttribute((const void*)k_level_build, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  TimedLaunch tl("level_build", st, 0.0, 8.0 * 2.0 * double(m1) * m2 * (m1 / 2 + m2 / 2) * h.d * 9, false);
  k_level_build<<<dim3(L.d, 9), 256, lds, st>>>((const double2*)h.Y64, h.cnb, L.P64.as<double2>(),
                                                 L.bsite.as<int>(), L.agg.as<int>(), L.pos.as<int>(),
                                                 L.Y64.as<double2>(), a);
  QMG_LAUNCH_CHECK();
}

void launch_level_export_P(const CoarseLevel& L, void* out, hipStream_t st) {
  const size_t n = size_t(2) * L.d * L.N * L.k;
  {
    TimedLaunch tl_("export", st, 2.0 * double(n) * 16, 0.0);
    launch(k_level_export_P, dim3(cdiv(n, 256)), dim3(256), 0, st, L.P64.as<double2>(), (double2*)out, L.nd, L.k1,
           L.k, n);
  }
  QMG_LAUNCH_CHECK();
}

void launch_level_export_Y(const CoarseLevel& L, void* out, hipStream_t st) {
  const int m = 2 * L.k;
  const size_t n = size_t(L.d) * 9 * m * m;
  {
    TimedLaunch tl_("export", st, 2.0 * double(n) * 16, 0.0);
    launch(k_export_Y, dim3(cdiv(n, 256)), dim3(256), 0, st, L.Y64.as<double2>(), (double2*)out, m, n);
  }
  QMG_LAUNCH_CHECK();
}

}  // namespace qmg
