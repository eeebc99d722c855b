// Even-odd form of the Galerkin coarse operator D_c = R D P (Eq. (5)) on the colouring of the
// aggregates by the parity of their coarse coordinates (every coarse extent even, so every hop
// block joins aggregates of opposite colour):
//
//   Dhat_c = Y_ee - Y_eo Y_oo^-1 Y_oe,
//   rhat_e = r_e - Y_eo Y_oo^-1 r_o,   v_o = Y_oo^-1 (r_o - Y_oe v_e).
//
// Everything is written with one kernel form applied to one colour of half vectors
// [nrhs][d/2][2k] (aggregates of a colour in increasing index order):
//
//   out(h) = [y(h)] + [B_0(j) a(h)] + sgn sum_{s=1..8} B_s(j) b(nbh(j, s)),   j = list(h),
//
// with B the blocks Y, or Yhat = Y_0^-1 Y whose slot 0 holds Y_0^-1 (so Yhat_s = Y_0^-1 Y_s for
// the hops).  Yhat folds the inverse self blocks into the odd hops: the Schur apply is two
// launches (u_o = Yhat-hops of v_e; out_e = Y_0 v_e - Y-hops of u_o) that each stream half of
// the blocks once.
#include <cstring>
#include <vector>

#include "mg.hpp"
#include "timing.hpp"

namespace qmg {

namespace {

// Yhat(j) = Y_0(j)^-1 Y(j) with slot 0 = Y_0(j)^-1, FP64: one workgroup per aggregate,
// Gauss-Jordan with partial pivoting on [Y_0 | 1] (row-major, m x 2m) in LDS; the left half
// then stages each hop block for the product.  Column-major blocks in and out.
// A pivot below 1e-13 of the largest entry of Y_0 (in modulus) marks the block as numerically
// singular (flag[0] = 1); the largest modulus of a real or imaginary part written to Yhat is
// returned in flag[1..2] (the bits of a non-negative double, which order like the double).
__global__ __launch_bounds__(256) void k_coarse_eo_blocks(const double2* __restrict__ Y, double2* __restrict__ Yh,
                                                          int m, int* __restrict__ flag) {
  extern __shared__ unsigned char smem_raw[];
  cplx<double>* a = reinterpret_cast<cplx<double>*>(smem_raw);  // [m][2m]
  cplx<double>* f = a + size_t(m) * 2 * m;                       // [m] elimination factors
  __shared__ int piv, bad;
  __shared__ double ymax2;
  __shared__ unsigned long long omax;
  const int j = blockIdx.x, w = 2 * m, tid = threadIdx.x;
  const double2* Yj = Y + size_t(j) * 9 * m * m;
  for (int t = tid; t < m * w; t += 256) {
    const int i = t / w, c = t - i * w;
    if (c < m) {
      const double2 v = Yj[size_t(c) * m + i];
      a[t] = {v.x, v.y};
    } else {
      a[t] = {c - m == i ? 1.0 : 0.0, 0.0};
    }
  }
  if (tid == 0) {
    bad = 0;
    omax = 0ull;
  }
  __syncthreads();
  if (tid == 0) {
    double v = 0.0;
    for (int i = 0; i < m; ++i)
      for (int c = 0; c < m; ++c) v = fmax(v, norm2(a[i * w + c]));
    ymax2 = v;
  }
  __syncthreads();
  const double tiny2 = 1e-26 * ymax2;  // (1e-13 max |Y_0|)^2
  for (int p = 0; p < m; ++p) {
    if (tid == 0) {
      int best = p;
      double bv = norm2(a[p * w + p]);
      for (int i = p + 1; i < m; ++i) {
        const double v = norm2(a[i * w + p]);
        if (v > bv) {
          bv = v;
          best = i;
        }
      }
      piv = best;
      if (!(bv > tiny2) || !(bv > 1e-280) || !isfinite(bv)) bad = 1;
    }
    __syncthreads();
    if (bad) break;  // uniform: every thread reads the same shared value
    const int pr = piv;
    if (pr != p)
      for (int c = tid; c < w; c += 256) {
        const cplx<double> t = a[p * w + c];
        a[p * w + c] = a[pr * w + c];
        a[pr * w + c] = t;
      }
    __syncthreads();
    const cplx<double> dp = a[p * w + p];
    const double dn = norm2(dp);
    const cplx<double> inv = {dp.re / dn, -dp.im / dn};
    __syncthreads();  // every thread has read the pivot before row p is scaled
    for (int c = tid; c < w; c += 256) a[p * w + c] = a[p * w + c] * inv;
    __syncthreads();
    for (int i = tid; i < m; i += 256) f[i] = i == p ? cplx<double>{0.0, 0.0} : a[i * w + p];
    __syncthreads();
    for (int t = tid; t < m * w; t += 256) {
      const int i = t / w, c = t - i * w;
      if (i != p) a[t] -= f[i] * a[p * w + c];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) atomicMax(flag, 1);
    return;
  }
  double2* out = Yh + size_t(j) * 9 * m * m;
  double lmax = 0.0;
  for (int t = tid; t < m * m; t += 256) {  // slot 0: the inverse
    const int c = t / m, i = t - c * m;
    const cplx<double> v = a[i * w + m + c];
    out[t] = make_double2(v.re, v.im);
    lmax = fmax(lmax, fmax(fabs(v.re), fabs(v.im)));
  }
  for (int s = 1; s < 9; ++s) {
    __syncthreads();
    const double2* Ys = Yj + size_t(s) * m * m;
    for (int t = tid; t < m * m; t += 256) {
      const int c = t / m, i = t - c * m;
      const double2 v = Ys[t];
      a[i * w + c] = {v.x, v.y};
    }
    __syncthreads();
    for (int t = tid; t < m * m; t += 256) {
      const int c = t / m, i = t - c * m;
      cplx<double> acc = {0.0, 0.0};
      for (int l = 0; l < m; ++l) acc += a[i * w + m + l] * a[l * w + c];
      out[size_t(s) * m * m + t] = make_double2(acc.re, acc.im);
      lmax = fmax(lmax, fmax(fabs(acc.re), fabs(acc.im)));
    }
  }
  if (!(lmax == lmax)) lmax = 1e308;  // a NaN entry counts as an overflow
  atomicMax(&omax, static_cast<unsigned long long>(__double_as_longlong(lmax)));
  __syncthreads();
  if (tid == 0) atomicMax(reinterpret_cast<unsigned long long*>(flag + 2), omax);
}

// One colour of the even-odd coarse operator (the form in the file header).  One workgroup per
// (aggregate of the colour, group of NR right-hand sides); the staged inputs and the column
// chunking over H follow the full coarse apply: thread (h, slot, row pack) forms PR rows of
// B_slot(j) times its input over column chunk h, the partial rows are summed in LDS.  Slots
// lo .. lo + ns - 1 are applied (lo = 0 with a self input a, lo + ns = 9 with a hop input b).
// Splitting the rows of an aggregate over several workgroups (to give each colour more than
// d/2 workgroups) measured slower: each workgroup then reads short row segments of every
// column-major block instead of whole columns.
template <class S, int NR, int PR>
__global__ __launch_bounds__(1024) void k_coarse_eo_apply(const S* __restrict__ B, const S* __restrict__ y,
                                                          const S* __restrict__ a, const S* __restrict__ b,
                                                          S* __restrict__ out, const int* __restrict__ list,
                                                          const int* __restrict__ nbh, int dh, int m, int nrhs, int H,
                                                          int lo, int ns, double sgn) {
  using C = ctype<S>;
  extern __shared__ unsigned char smem_raw[];
  cplx<C>* vin = reinterpret_cast<cplx<C>*>(smem_raw);  // [NR][ns][m]
  cplx<C>* part = vin + size_t(NR) * ns * m;             // [NR][ns H][m]
  const int h = blockIdx.x, j = list[h], rhs0 = blockIdx.y * NR;
  const int nr = min(NR, nrhs - rhs0);
  for (int t = threadIdx.x; t < NR * ns * m; t += blockDim.x) {
    const int r = t / (ns * m), rem = t - r * ns * m, q = rem / m, col = rem - q * m;
    const int slot = lo + q;
    cplx<C> v = {C(0), C(0)};
    if (r < nr) {
      if (slot == 0)
        v = ldc(a, (size_t(rhs0 + r) * dh + h) * m + col);
      else
        v = ldc(b, (size_t(rhs0 + r) * dh + nbh[j * 8 + slot - 1]) * m + col);
    }
    vin[t] = v;
  }
  __syncthreads();
  const int mp = m / PR;
  const int cc = (m + H - 1) / H;
  for (int t = threadIdx.x; t < H * ns * mp; t += blockDim.x) {
    const int hq = t / mp, rp = t - hq * mp;  // hq = hc * ns + q
    const int hc = hq / ns, q = hq - hc * ns;
    const int c0 = hc * cc, c1 = min(m, c0 + cc);
    const S* Bb = B + (size_t(j) * 9 + lo + q) * m * m;
    cplx<C> acc[NR][PR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int u = 0; u < PR; ++u) acc[r][u] = {C(0), C(0)};
#pragma unroll 6
    for (int col = c0; col < c1; ++col) {
      const Pk<S, PR> yv = ldp<S, PR>(Bb, size_t(col) * mp + rp);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const cplx<C> v = vin[(r * ns + q) * m + col];
#pragma unroll
        for (int u = 0; u < PR; ++u) acc[r][u] += StoreTraits<S>::ld(yv.v[u]) * v;
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int u = 0; u < PR; ++u) part[(size_t(r) * ns * H + hq) * m + rp * PR + u] = acc[r][u];
  }
  __syncthreads();
  // each output row is summed by kG consecutive lanes (partials hq = g, g + kG, ...), then a
  // fixed butterfly over the kG lanes: the same order on every call.  The loop bound is a
  // multiple of kG and blockDim.x of 64, so a group's lanes are all active together.
  constexpr int kG = 16;
  const C sg = C(sgn);
  const int nq = ns * H;
  for (int t = threadIdx.x; t < nr * m * kG; t += blockDim.x) {
    const int g = t % kG, rr = t / kG;
    const int r = rr / m, row = rr - r * m;
    cplx<C> s = {C(0), C(0)};
    for (int hq = g; hq < nq; hq += kG) {
      const cplx<C> v = part[(size_t(r) * nq + hq) * m + row];
      if (lo + hq % ns == 0)
        s += v;
      else
        s += sg * v;
    }
#pragma unroll
    for (int off = kG / 2; off > 0; off >>= 1) {
      s.re += __shfl_xor(s.re, off);
      s.im += __shfl_xor(s.im, off);
    }
    if (g == 0) {
      const size_t o = (size_t(rhs0 + r) * dh + h) * m + row;
      if (y) s += ldc(y, o);
      stc(out, o, s);
    }
  }
}

// full coarse vectors [nrhs][d][m] <-> the two colours [nrhs][d/2][m]
template <class S>
__global__ __launch_bounds__(256) void k_coarse_eo_split(const S* __restrict__ full, S* __restrict__ ev,
                                                         S* __restrict__ od, const int* __restrict__ tab, int d, int m,
                                                         size_t n) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= n) return;
  const size_t rj = g / m;
  const int row = int(g - rj * m);
  const int r = int(rj / d), j = int(rj - size_t(r) * d);
  const size_t o = (size_t(r) * (d / 2) + tab[d + j]) * m + row;
  (tab[j] ? od : ev)[o] = full[g];
}

template <class S>
__global__ __launch_bounds__(256) void k_coarse_eo_merge(const S* __restrict__ ev, const S* __restrict__ od,
                                                         S* __restrict__ full, const int* __restrict__ tab, int d, int m,
                                                         size_t n) {
  const size_t g = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= n) return;
  const size_t rj = g / m;
  const int row = int(g - rj * m);
  const int r = int(rj / d), j = int(rj - size_t(r) * d);
  const size_t o = (size_t(r) * (d / 2) + tab[d + j]) * m + row;
  full[g] = (tab[j] ? od : ev)[o];
}

template <class F>
void dispatch_ceo(qmg_prec p, F&& f) {
  switch (p) {
    case QMG_F64: f(double2{}); break;
    case QMG_F32: f(float2{}); break;
    case QMG_BF16: f(cbf16{}); break;
    case QMG_F16: f(chalf{}); break;
  }
}

inline unsigned nblk256(size_t n) { return unsigned((n + 255) / 256); }

}  // namespace

void build_coarse_eo_tables(HierarchyDev& h, hipStream_t st) {
  const int d = h.blk.d;
  const int* cL = h.blk.cL;
  for (int q = 0; q < 4; ++q)
    QMG_CHECK(cL[q] % 2 == 0, QMG_ESHAPE, "even-odd coarse operator: coarse extent %d in direction %d is odd",
              cL[q], q);
  std::vector<int> cnb(size_t(8) * d);
  QMG_HIP(hipMemcpyAsync(cnb.data(), h.cnb.p, cnb.size() * sizeof(int), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  // tab: [0, d) colour, [d, 2d) index within the colour, [2d, 3d) the aggregates of colour 0
  // then colour 1, [3d, 11d) the colour index of every neighbour
  std::vector<int> tab(size_t(11) * d);
  int cnt[2] = {0, 0};
  for (int j = 0; j < d; ++j) {
    int rem = j, s = 0;
    for (int q = 0; q < 4; ++q) {
      s += rem % cL[q];
      rem /= cL[q];
    }
    const int p = s & 1;
    tab[j] = p;
    tab[d + j] = cnt[p]++;
  }
  QMG_CHECK(cnt[0] == d / 2 && cnt[1] == d / 2, QMG_ESHAPE, "even-odd coarse colouring is unbalanced");
  for (int j = 0; j < d; ++j) tab[2 * d + tab[j] * (d / 2) + tab[d + j]] = j;
  for (int j = 0; j < d; ++j)
    for (int s = 0; s < 8; ++s) {
      const int nb = cnb[size_t(j) * 8 + s];
      QMG_CHECK(tab[nb] != tab[j], QMG_ESHAPE, "coarse hop between aggregates of one colour");
      tab[3 * d + j * 8 + s] = tab[d + nb];
    }
  h.ceo_tab.alloc(tab.size() * sizeof(int));
  QMG_HIP(hipMemcpyAsync(h.ceo_tab.p, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice, st));
  QMG_HIP(hipStreamSynchronize(st));
}

void build_coarse_eo_blocks(HierarchyDev& h, hipStream_t st) {
  const int d = h.blk.d, m = 2 * h.k;
  QMG_CHECK(m <= 64, QMG_EINVAL, "even-odd coarse operator supports 2k <= 64");
  const size_t nblk = size_t(d) * 9 * m * m;
  // a failed or partial build leaves no blocks behind (the caller's coarse_eo flag stays off)
  h.Yh64.release();
  h.Yhin.release();
  h.Yh64.alloc(nblk * sizeof(double2));
  DevBuf flag(4 * sizeof(int));  // [0] singular block, [2..3] largest |entry| of Yhat (double bits)
  QMG_HIP(hipMemsetAsync(flag.p, 0, 4 * sizeof(int), st));
  const size_t lds = (size_t(m) * 2 * m + m) * sizeof(double2);
  if (lds > 64 * 1024)
    QMG_HIP(hipFuncSetAttribute((const void*)k_coarse_eo_blocks, hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(lds)));
  {
    TimedLaunch tl_("setup/coarse_eo_blocks", st, double(d) * 18 * m * m * 16, 0.0);
    launch(k_coarse_eo_blocks, dim3(d), dim3(256), lds, st, h.Y64.as<double2>(), h.Yh64.as<double2>(), m,
           flag.as<int>());
  }
  QMG_LAUNCH_CHECK();
  int fl[4] = {0, 0, 0, 0};
  QMG_HIP(hipMemcpyAsync(fl, flag.p, sizeof(fl), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  double ymax = 0.0;
  std::memcpy(&ymax, fl + 2, sizeof(double));
  // largest finite value of the inner storage type, with a factor 2 of headroom for the sums
  const double lim = h.inner == QMG_F16 ? 65504.0 / 2 : 3.0e38 / 2;
  if (fl[0] != 0 || !(ymax < lim)) {
    h.Yh64.release();
    QMG_CHECK(fl[0] == 0, QMG_EBREAKDOWN,
              "a coarse self block is numerically singular (pivot below 1e-13 of its largest entry)");
    QMG_CHECK(false, QMG_EBREAKDOWN, "Y_0^-1 Y has entries of modulus %.3g, beyond the %s storage range", ymax,
              h.inner == QMG_F16 ? "FP16" : "inner");
  }
  if (h.inner != QMG_F64) {
    h.Yhin.alloc(nblk * prec_bytes(h.inner));
    launch_convert(h.Yh64.p, QMG_F64, h.Yhin.p, h.inner, nblk, st);
  } else {
    h.Yhin.release();
  }
}

void launch_coarse_eo_apply(qmg_prec prec, const HierarchyDev& h, int colour, const void* B, const void* y,
                            const void* a, const void* b, void* out, int nrhs, double sgn, hipStream_t st) {
  const int d = h.blk.d, dh = d / 2, m = 2 * h.k;
  const int lo = a ? 0 : 1, hi = b ? 9 : 1, ns = hi - lo;
  QMG_CHECK(ns >= 1, QMG_ESHAPE, "even-odd coarse apply without inputs");
  const int* tab = h.ceo_tab.as<int>();
  const int* list = tab + 2 * d + colour * dh;
  const int* nbh = tab + 3 * d;
  TimedLaunch tl("coarse_eo", st,
                 double(dh) * (double(ns) * m * m + double(m) * nrhs * (ns + 1 + (y ? 1 : 0))) * prec_bytes(prec),
                 8.0 * ns * double(m) * m * dh * nrhs);
  dispatch_ceo(prec, [&](auto tag) {
    using S = decltype(tag);
    constexpr int PK = kPack<S>;
    auto go = [&](auto kern, int NR, int PR) {
      const int mp = m / PR;
      const int H = std::max(1, std::min(8, 1024 / (ns * mp)));
      const int threads = int(std::min<size_t>(1024, ((size_t(ns) * mp * H + 63) / 64) * 64));
      const size_t lds = size_t(NR) * ns * m * (1 + H) * sizeof(cplx<ctype<S>>);
      QMG_CHECK(lds <= 160 * 1024, QMG_EINVAL, "even-odd coarse apply: block too large for LDS staging");
      if (lds > 64 * 1024)
        QMG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
      launch(kern, dim3(dh, (nrhs + NR - 1) / NR), dim3(threads), uint32_t(lds), st, static_cast<const S*>(B),
             static_cast<const S*>(y), static_cast<const S*>(a), static_cast<const S*>(b), static_cast<S*>(out), list,
             nbh, dh, m, nrhs, H, lo, ns, sgn);
    };
    if (m % PK == 0) {
      if (nrhs >= 3) go(k_coarse_eo_apply<S, 4, PK>, 4, PK);
      else if (nrhs == 2) go(k_coarse_eo_apply<S, 2, PK>, 2, PK);
      else go(k_coarse_eo_apply<S, 1, PK>, 1, PK);
    } else {
      if (nrhs >= 3) go(k_coarse_eo_apply<S, 4, 1>, 4, 1);
      else if (nrhs == 2) go(k_coarse_eo_apply<S, 2, 1>, 2, 1);
      else go(k_coarse_eo_apply<S, 1, 1>, 1, 1);
    }
  });
  QMG_LAUNCH_CHECK();
}

void launch_coarse_eo_split(qmg_prec prec, const HierarchyDev& h, const void* full, void* ev, void* od, int nrhs,
                            hipStream_t st) {
  const int d = h.blk.d, m = 2 * h.k;
  const size_t n = size_t(nrhs) * d * m;
  dispatch_ceo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("coarse_eo_layout", st, 2.0 * double(n) * sizeof(S), 0.0);
      launch(k_coarse_eo_split<S>, dim3(nblk256(n)), dim3(256), 0, st, static_cast<const S*>(full),
             static_cast<S*>(ev), static_cast<S*>(od), h.ceo_tab.as<int>(), d, m, n);
    }
  });
  QMG_LAUNCH_CHECK();
}

void launch_coarse_eo_merge(qmg_prec prec, const HierarchyDev& h, const void* ev, const void* od, void* full, int nrhs,
                            hipStream_t st) {
  const int d = h.blk.d, m = 2 * h.k;
  const size_t n = size_t(nrhs) * d * m;
  dispatch_ceo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("coarse_eo_layout", st, 2.0 * double(n) * sizeof(S), 0.0);
      launch(k_coarse_eo_merge<S>, dim3(nblk256(n)), dim3(256), 0, st, static_cast<const S*>(ev),
             static_cast<const S*>(od), static_cast<S*>(full), h.ceo_tab.as<int>(), d, m, n);
    }
  });
  QMG_LAUNCH_CHECK();
}

}  // namespace qmg
