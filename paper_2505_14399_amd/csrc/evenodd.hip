// Even-odd (Schur complement) preconditioning of the fine operator: half-lattice layouts and the
// inverse of the site term.
//
// With every extent even, the hops of D join sites of opposite parity p = (x + y + z + t) mod 2
// and the site term A (the diagonal term, plus the clover term) is local, so D x = b is solved
// through Dhat = A_ee - D_eo A_oo^-1 D_oe on the even sites: Dhat x_e = b_e - D_eo A_oo^-1 b_o,
// then x_o = A_oo^-1 (b_o - D_oe x_e).  A site's half-lattice index is its lexicographic index
// divided by 2.  The hop kernels are in dslash.hip; this file moves fields between the full and
// the half-lattice layouts and inverts the packed 6 x 6 blocks of the site term.
#include <algorithm>
#include <cstring>

#include "qmg_internal.hpp"
#include "timing.hpp"

namespace qmg {

namespace {

inline unsigned nblk(size_t n) { return unsigned((n + 255) / 256); }

struct EoGeom {
  int L[4];
  int V;
};

__device__ inline int site_parity(int s, const EoGeom& g) {
  const int x = s % g.L[0];
  s /= g.L[0];
  const int y = s % g.L[1];
  s /= g.L[1];
  const int z = s % g.L[2];
  const int t = s / g.L[2];
  return (x + y + z + t) & 1;
}

// canonical FP64 gauge [mu][V][9] -> [parity][mu][9][V/2]
template <class S>
__global__ void k_eo_pack_gauge(const double2* __restrict__ in, S* __restrict__ out, EoGeom g, size_t n) {
  const size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= n) return;
  const int e = int(q % 9);
  const size_t t = q / 9;
  const int site = int(t % g.V);
  const int mu = int(t / g.V);
  const int Vh = g.V >> 1;
  const int p = site_parity(site, g);
  const double2 v = in[q];
  stc(out, ((size_t(p) * 4 + mu) * 9 + e) * Vh + (site >> 1), cplx<double>{v.x, v.y});
}

// canonical FP64 spinors [rhs][V][12] <-> half fields [rhs][12][V/2] of each parity
template <class S>
__global__ void k_eo_pack_spinor(const double2* __restrict__ in, S* __restrict__ even, S* __restrict__ odd,
                                 EoGeom g, size_t n) {
  const size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= n) return;
  const int k = int(q % 12);
  const size_t t = q / 12;
  const int site = int(t % g.V);
  const size_t r = t / g.V;
  const int Vh = g.V >> 1;
  S* dst = site_parity(site, g) ? odd : even;
  const double2 v = in[q];
  stc(dst, (r * 12 + k) * Vh + (site >> 1), cplx<double>{v.x, v.y});
}

template <class S>
__global__ void k_eo_unpack_spinor(const S* __restrict__ even, const S* __restrict__ odd, double2* __restrict__ out,
                                   EoGeom g, size_t n) {
  const size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= n) return;
  const int k = int(q % 12);
  const size_t t = q / 12;
  const int site = int(t % g.V);
  const size_t r = t / g.V;
  const int Vh = g.V >> 1;
  const S* src = site_parity(site, g) ? odd : even;
  const auto v = ldc(src, (r * 12 + k) * Vh + (site >> 1));
  out[q] = make_double2(double(v.re), double(v.im));
}

// packed FP64 site term [alpha][18][V] (full lattice) -> the same and its inverse in the
// half-lattice layout [parity][alpha][18][V/2]; one thread per (site, chirality).  The inverse
// is Gauss-Jordan elimination with partial pivoting in FP64 on the unpacked block (the block is
// hermitian but need not be definite); the inverse is hermitian and is packed from its upper
// triangle and the real parts of its diagonal.
template <class S>
__global__ __launch_bounds__(128) void k_eo_site_term(const double2* __restrict__ A, S* __restrict__ Aeo,
                                                      S* __restrict__ Ainv, EoGeom g, int* __restrict__ singular) {
  const int site = blockIdx.x * 128 + threadIdx.x;
  if (site >= g.V) return;
  const int al = blockIdx.y;
  const int V = g.V, Vh = V >> 1;
  const int p = site_parity(site, g);
  const size_t dst0 = (size_t(p) * 2 + al) * 18 * Vh + (site >> 1);
  cplx<double> M[6][6], R[6][6];
  const double2* src = A + size_t(al) * 18 * V + site;
  for (int e = 0; e < 18; ++e) {
    const double2 v = src[size_t(e) * V];
    stc(Aeo, dst0 + size_t(e) * Vh, cplx<double>{v.x, v.y});
  }
  for (int e = 0; e < 3; ++e) {
    const double2 d = src[size_t(e) * V];
    M[2 * e][2 * e] = {d.x, 0.0};
    M[2 * e + 1][2 * e + 1] = {d.y, 0.0};
  }
  {
    int e = 3;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j, ++e) {
        const double2 o = src[size_t(e) * V];
        M[i][j] = {o.x, o.y};
        M[j][i] = {o.x, -o.y};
      }
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) R[i][j] = {i == j ? 1.0 : 0.0, 0.0};
  bool ok = true;
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    double best = norm2(M[c][c]);
    for (int r = c + 1; r < 6; ++r) {
      const double v = norm2(M[r][c]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (!(best > 0.0)) {
      ok = false;
      break;
    }
    if (piv != c) {
      for (int j = 0; j < 6; ++j) {
        const cplx<double> a = M[c][j], b = R[c][j];
        M[c][j] = M[piv][j];
        R[c][j] = R[piv][j];
        M[piv][j] = a;
        R[piv][j] = b;
      }
    }
    const cplx<double> pv = M[c][c];
    const double inv_n = 1.0 / norm2(pv);
    const cplx<double> ip = {pv.re * inv_n, -pv.im * inv_n};  // 1 / pivot
    for (int j = 0; j < 6; ++j) {
      M[c][j] = ip * M[c][j];
      R[c][j] = ip * R[c][j];
    }
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const cplx<double> f = M[r][c];
      for (int j = 0; j < 6; ++j) {
        M[r][j] -= f * M[c][j];
        R[r][j] -= f * R[c][j];
      }
    }
  }
  if (!ok) {
    atomicOr(singular, 1);
    return;
  }
  for (int e = 0; e < 3; ++e)
    stc(Ainv, dst0 + size_t(e) * Vh, cplx<double>{R[2 * e][2 * e].re, R[2 * e + 1][2 * e + 1].re});
  int e = 3;
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j, ++e) stc(Ainv, dst0 + size_t(e) * Vh, R[i][j]);
}

// native FP64 gauge [mu][9][V] -> [parity][mu][ne][V/2] (ne = 9, or 6: rows 0 and 1)
template <class S>
__global__ void k_eo_gauge_from_native(const double2* __restrict__ in, S* __restrict__ out, EoGeom g, size_t n,
                                       int ne) {
  const size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= n) return;
  const int site = int(q % g.V);
  const size_t me = q / g.V;  // mu * 9 + e
  const int mu = int(me / 9), e = int(me % 9);
  if (e >= ne) return;
  const int Vh = g.V >> 1;
  const int p = site_parity(site, g);
  const double2 v = in[q];
  stc(out, ((size_t(p) * 4 + mu) * ne + e) * Vh + (site >> 1), cplx<double>{v.x, v.y});
}

// max over links of |row 2 - conj(row 0 x row 1)| (FP64), as the bits of a non-negative double
__global__ void k_su3_row_defect(const double2* __restrict__ U, int V, unsigned long long* __restrict__ out) {
  const size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= size_t(4) * V) return;
  const int site = int(q % V), mu = int(q / V);
  cplx<double> u[9];
  for (int e = 0; e < 9; ++e) {
    const double2 v = U[(size_t(mu) * 9 + e) * V + site];
    u[e] = {v.x, v.y};
  }
  double d = 0;
  for (int c = 0; c < 3; ++c) {
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    const cplx<double> r = conj(u[c1] * u[3 + c2] - u[c2] * u[3 + c1]);
    d = fmax(d, sqrt(norm2(u[6 + c] - r)));
  }
  if (!(d == d)) d = 1e300;  // a non-finite link is no SU(3) link
  unsigned long long bits;
  memcpy(&bits, &d, sizeof(bits));
  atomicMax(out, bits);
}

// native spinors [rhs][12][V] (storage S) <-> half fields of each parity.  Split: the half fields
// of r - t, the difference rounded to the storage type once (as a subtraction pass followed by a
// split would); merge: full += the two halves.
template <class S>
__global__ void k_eo_split_sub(const S* __restrict__ r, const S* __restrict__ t, S* __restrict__ even,
                               S* __restrict__ odd, EoGeom g, size_t n) {
  const size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= n) return;
  const int site = int(q % g.V);
  const size_t rk = q / g.V;  // rhs * 12 + component
  const int Vh = g.V >> 1;
  S* dst = site_parity(site, g) ? odd : even;
  stc(dst, rk * Vh + (site >> 1), ldc(r, q) - ldc(t, q));
}

template <class S>
__global__ void k_eo_merge_add(const S* __restrict__ even, const S* __restrict__ odd, S* __restrict__ full, EoGeom g,
                               size_t n) {
  const size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= n) return;
  const int site = int(q % g.V);
  const size_t rk = q / g.V;
  const int Vh = g.V >> 1;
  const S* src = site_parity(site, g) ? odd : even;
  const auto a = ldc(full, q);
  const auto b = ldc(src, rk * Vh + (site >> 1));
  stc(full, q, a + b);
}

// s-step residual minimisation over a Krylov basis p_0 .. p_{m-1} (m <= kSMax; vector i of rhs r
// at P[(i * nrhs + r) * len]): with p_{j+1} = A p_j, the x = sum_j c_j p_j minimising
// ||p_0 - A x|| solves the normal equations sum_j <p_{i+1}, p_{j+1}> c_j = <p_{i+1}, p_0>.  One
// pass forms every inner product <p_i, p_j> (i <= j), accumulated in FP64 for every storage
// type: the normal equations square the condition number of the basis, and FP32 sums (relative
// error ~1e-7 times the terms per thread) left only the first few basis directions resolvable,
// which weakened the FP32 K-cycle's smoother (more outer iterations than the FP64 path).
constexpr int kSMax = 9;
constexpr int kPairs = kSMax * (kSMax + 1) / 2;

template <class S>
__global__ __launch_bounds__(256) void k_sstep_gram(const S* __restrict__ P, int m, size_t len, int nrhs,
                                                    double2* __restrict__ part) {
  using C = ctype<S>;
  const int r = blockIdx.y;
  cplx<double> acc[kPairs];
#pragma unroll
  for (int q = 0; q < kPairs; ++q) acc[q] = {0.0, 0.0};
  // storage below FP64: the next element's values are loaded before this element's products
  // (one element ahead), so each wavefront has a load in flight while its FP64 products run
  // (FP64 storage has no registers to spare for it)
  constexpr bool kAhead = sizeof(C) < 8;
  const size_t stride = size_t(gridDim.x) * 256;
  size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
  cplx<C> nx[kSMax];
  if constexpr (kAhead) {
#pragma unroll
    for (int i = 0; i < kSMax; ++i)
      nx[i] = (i < m && e < len) ? ldc(P, (size_t(i) * nrhs + r) * len + e) : cplx<C>{C(0), C(0)};
  }
  for (; e < len; e += stride) {
    cplx<double> v[kSMax];
    if constexpr (kAhead) {
#pragma unroll
      for (int i = 0; i < kSMax; ++i) v[i] = {double(nx[i].re), double(nx[i].im)};
      const size_t en = e + stride;
#pragma unroll
      for (int i = 0; i < kSMax; ++i)
        nx[i] = (i < m && en < len) ? ldc(P, (size_t(i) * nrhs + r) * len + en) : cplx<C>{C(0), C(0)};
    } else {
#pragma unroll
      for (int i = 0; i < kSMax; ++i) {
        const cplx<C> t = i < m ? ldc(P, (size_t(i) * nrhs + r) * len + e) : cplx<C>{C(0), C(0)};
        v[i] = {double(t.re), double(t.im)};
      }
    }
    int q = 0;
#pragma unroll
    for (int i = 0; i < kSMax; ++i)
#pragma unroll
      for (int j = i; j < kSMax; ++j, ++q) acc[q] += cmul_conj(v[i], v[j]);
  }
  __shared__ double2 red[4][kPairs];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kPairs; ++q) {
    double re = acc[q].re, im = acc[q].im;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off);
      im += __shfl_xor(im, off);
    }
    if (lane == 0) red[wave][q] = make_double2(re, im);
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < kPairs) {
    double2 sum = red[0][t];
    for (int w = 1; w < 4; ++w) {
      sum.x += red[w][t].x;
      sum.y += red[w][t].y;
    }
    part[(size_t(r) * gridDim.x + blockIdx.x) * kPairs + t] = sum;
  }
}

// one workgroup per right-hand side: the workgroup partials of k_sstep_gram summed by 22 slices
// x 45 pair threads through LDS into Gout[r][pair]
__global__ __launch_bounds__(1024) void k_sstep_reduce(const double2* __restrict__ part, int nblk,
                                                       double2* __restrict__ Gout) {
  constexpr int kSlices = 1024 / kPairs;
  __shared__ double2 red[kSlices][kPairs];
  const int r = blockIdx.x, t = threadIdx.x;
  const int q = t % kPairs, sl = t / kPairs;
  if (sl < kSlices) {
    double re = 0, im = 0;
    for (int b = sl; b < nblk; b += kSlices) {
      const double2 v = part[(size_t(r) * nblk + b) * kPairs + q];
      re += v.x;
      im += v.y;
    }
    red[sl][q] = make_double2(re, im);
  }
  __syncthreads();
  if (t < kPairs) {
    double re = 0, im = 0;
    for (int w = 0; w < kSlices; ++w) {
      re += red[w][t].x;
      im += red[w][t].y;
    }
    Gout[size_t(r) * kPairs + t] = make_double2(re, im);
  }
}

// one wavefront per right-hand side, one thread solving the s x s normal equations (s = m - 1),
// equilibrated by the diagonal, by Cholesky in FP64 with compile-time indices (the unused rows
// of the 8 x 8 factor are predicated off, so it stays in registers); a pivot below 1e-13 of the
// unit diagonal ends the factor and the remaining coefficients are zero (the basis vectors beyond
// it add nothing resolvable)
// With a shifted basis p_{j+1} = (A - d) p_j the images are w_j = A p_j = p_{j+1} + d p_j, and
// the products <w_i, w_j>, <w_i, p_0> follow from the same inner products of the p's (d real;
// d = 0 is the plain basis).
__global__ __launch_bounds__(64) void k_sstep_solve(const double2* __restrict__ Gin, int m, int nrhs,
                                                    double2* __restrict__ c, double d) {
  constexpr int kS = kSMax - 1;
  const int r = blockIdx.x;
  if (threadIdx.x != 0) return;
  const double2* G = Gin + size_t(r) * kPairs;
  const int s = m - 1;
  auto gp = [&](int i, int j) {  // <p_i, p_j>
    if (i <= j) {
      const double2 v = G[i * kSMax - i * (i - 1) / 2 + (j - i)];
      return cplx<double>{v.x, v.y};
    }
    const double2 v = G[j * kSMax - j * (j - 1) / 2 + (i - j)];
    return cplx<double>{v.x, -v.y};
  };
  // inner(i + 1, j + 1) = <w_i, w_j>, inner(i + 1, 0) = <w_i, p_0>
  auto inner = [&](int i, int j) {
    if (j == 0) return gp(i, 0) + d * gp(i - 1, 0);
    return gp(i, j) + d * (gp(i, j - 1) + gp(i - 1, j)) + (d * d) * gp(i - 1, j - 1);
  };
  double dsc[kS];
#pragma unroll
  for (int a = 0; a < kS; ++a) {
    const double d = a < s ? inner(a + 1, a + 1).re : 0.0;
    dsc[a] = d > 0 ? 1.0 / sqrt(d) : 0.0;
  }
  cplx<double> L[kS][kS];
  double Ld[kS];
  int se = s;
#pragma unroll
  for (int k = 0; k < kS; ++k) {
    cplx<double> d = k < s ? dsc[k] * dsc[k] * inner(k + 1, k + 1) : cplx<double>{1.0, 0.0};
#pragma unroll
    for (int j = 0; j < k; ++j) d -= L[k][j] * conj(L[k][j]);
    const bool good = !(k < se) || d.re > 1e-13;
    if (k < se && !good) se = k;
    Ld[k] = (k < se) ? sqrt(d.re) : 1.0;
    L[k][k] = {Ld[k], 0.0};
#pragma unroll
    for (int i = k + 1; i < kS; ++i) {
      cplx<double> v = i < s ? dsc[i] * dsc[k] * inner(i + 1, k + 1) : cplx<double>{0.0, 0.0};
#pragma unroll
      for (int j = 0; j < k; ++j) v -= L[i][j] * conj(L[k][j]);
      L[i][k] = (1.0 / Ld[k]) * v;
    }
  }
  cplx<double> y[kS];
#pragma unroll
  for (int i = 0; i < kS; ++i) {  // L y = D g
    cplx<double> v = i < se ? dsc[i] * inner(i + 1, 0) : cplx<double>{0.0, 0.0};
#pragma unroll
    for (int j = 0; j < i; ++j) v -= L[i][j] * y[j];
    y[i] = i < se ? (1.0 / Ld[i]) * v : cplx<double>{0.0, 0.0};
  }
#pragma unroll
  for (int i = kS - 1; i >= 0; --i) {  // L^dag chat = y, c = D chat
    cplx<double> v = y[i];
#pragma unroll
    for (int j = i + 1; j < kS; ++j) v -= cmul_conj(L[j][i], y[j]);
    y[i] = i < se ? (1.0 / Ld[i]) * v : cplx<double>{0.0, 0.0};
  }
#pragma unroll
  for (int a = 0; a < kS; ++a)
    if (a < s) c[size_t(a) * nrhs + r] = make_double2(dsc[a] * y[a].re, dsc[a] * y[a].im);
}

template <class F>
void dispatch_eo(qmg_prec p, F&& f) {
  switch (p) {
    case QMG_F64: f(double2{}); break;
    case QMG_F32: f(float2{}); break;
    case QMG_BF16: f(cbf16{}); break;
    case QMG_F16: f(chalf{}); break;
  }
}

EoGeom eo_geom(const Geom& g) {
  EoGeom e{};
  for (int q = 0; q < 4; ++q) e.L[q] = g.L[q];
  e.V = g.V;
  return e;
}

}  // namespace

void launch_eo_pack_gauge(const Geom& g, const void* canon, void* out, qmg_prec prec, hipStream_t st) {
  const size_t n = size_t(36) * g.V;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("layout/eo_gauge", st, double(n) * (16.0 + sizeof(S)), 0.0);
      launch(k_eo_pack_gauge<S>, dim3(nblk(n)), dim3(256), 0, st, static_cast<const double2*>(canon),
             static_cast<S*>(out), eo_geom(g), n);
    }
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_pack_spinor(const Geom& g, const void* canon, void* even, void* odd, int nrhs, qmg_prec prec,
                           hipStream_t st) {
  const size_t n = size_t(12) * g.V * nrhs;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("layout/eo_spinor", st, double(n) * (16.0 + sizeof(S)), 0.0);
      launch(k_eo_pack_spinor<S>, dim3(nblk(n)), dim3(256), 0, st, static_cast<const double2*>(canon),
             static_cast<S*>(even), static_cast<S*>(odd), eo_geom(g), n);
    }
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_unpack_spinor(const Geom& g, const void* even, const void* odd, void* canon, int nrhs, qmg_prec prec,
                             hipStream_t st) {
  const size_t n = size_t(12) * g.V * nrhs;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("layout/eo_spinor", st, double(n) * (16.0 + sizeof(S)), 0.0);
      launch(k_eo_unpack_spinor<S>, dim3(nblk(n)), dim3(256), 0, st, static_cast<const S*>(even),
             static_cast<const S*>(odd), static_cast<double2*>(canon), eo_geom(g), n);
    }
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_gauge_from_native(const Geom& g, const void* U64, void* out, qmg_prec prec, hipStream_t st, int ne) {
  QMG_CHECK(ne == 9 || ne == 6, QMG_EINVAL, "links carry 9 or 6 complex entries");
  const size_t n = size_t(36) * g.V;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("layout/eo_gauge", st, double(n) * (16.0 + sizeof(S)), 0.0);
      launch(k_eo_gauge_from_native<S>, dim3(nblk(n)), dim3(256), 0, st, static_cast<const double2*>(U64),
             static_cast<S*>(out), eo_geom(g), n, ne);
    }
  });
  QMG_LAUNCH_CHECK();
}

double launch_su3_row_defect(const Geom& g, const void* U64, hipStream_t st) {
  DevBuf m(sizeof(unsigned long long));
  QMG_HIP(hipMemsetAsync(m.p, 0, sizeof(unsigned long long), st));
  {
    TimedLaunch tl_("setup/su3_check", st, double(g.V) * 4 * 9 * 16, 0.0);
    launch(k_su3_row_defect, dim3(nblk(size_t(4) * g.V)), dim3(256), 0, st, static_cast<const double2*>(U64), g.V,
           static_cast<unsigned long long*>(m.p));
  }
  QMG_LAUNCH_CHECK();
  unsigned long long bits = 0;
  QMG_HIP(hipMemcpyAsync(&bits, m.p, sizeof(bits), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  double d;
  std::memcpy(&d, &bits, sizeof(d));
  return d;
}

void launch_eo_split_sub(qmg_prec prec, const Geom& g, const void* r, const void* t, void* even, void* odd, int nrhs,
                         hipStream_t st) {
  const size_t n = size_t(12) * g.V * nrhs;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("eo_layout/split", st, 3.0 * double(n) * sizeof(S), 0.0);
      launch(k_eo_split_sub<S>, dim3(nblk(n)), dim3(256), 0, st, static_cast<const S*>(r), static_cast<const S*>(t),
             static_cast<S*>(even), static_cast<S*>(odd), eo_geom(g), n);
    }
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_merge_add(qmg_prec prec, const Geom& g, const void* even, const void* odd, void* full, int nrhs,
                         hipStream_t st) {
  const size_t n = size_t(12) * g.V * nrhs;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("eo_layout/merge", st, 3.0 * double(n) * sizeof(S), 0.0);
      launch(k_eo_merge_add<S>, dim3(nblk(n)), dim3(256), 0, st, static_cast<const S*>(even),
             static_cast<const S*>(odd), static_cast<S*>(full), eo_geom(g), n);
    }
  });
  QMG_LAUNCH_CHECK();
}

void launch_sstep_coeffs(qmg_prec prec, const void* P, int m, size_t len, int nrhs, double2* c, DevBuf& part,
                         hipStream_t st, double shift) {
  QMG_CHECK(m >= 2 && m <= kSMax, QMG_EINVAL, "s-step basis of %d vectors (2 .. %d)", m, kSMax);
  const int nblk = int(std::max<size_t>(1, std::min<size_t>(512, len / (256 * 8))));
  part.ensure(size_t(nrhs) * (nblk + 1) * kPairs * sizeof(double2));  // partials, then the reduced pairs
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("sstep/gram", st, double(m + 1) * len * nrhs * sizeof(S), 0.0);
      launch(k_sstep_gram<S>, dim3(nblk, nrhs), dim3(256), 0, st, static_cast<const S*>(P), m, len, nrhs,
             part.as<double2>());
    }
  });
  QMG_LAUNCH_CHECK();
  {
    TimedLaunch tl_("sstep/reduce", st, double(nblk) * nrhs * kPairs * sizeof(double2), 0.0);
    launch(k_sstep_reduce, dim3(nrhs), dim3(1024), 0, st, part.as<double2>(), nblk,
           part.as<double2>() + size_t(nrhs) * nblk * kPairs);
  }
  QMG_LAUNCH_CHECK();
  {
    TimedLaunch tl_("sstep/solve", st, double(nrhs) * kPairs * sizeof(double2), 0.0);
    launch(k_sstep_solve, dim3(nrhs), dim3(64), 0, st, part.as<double2>() + size_t(nrhs) * nblk * kPairs, m, nrhs, c,
           shift);
  }
  QMG_LAUNCH_CHECK();
}

void launch_eo_site_term(const Geom& g, const void* A64, void* Aeo, void* Ainv, qmg_prec prec, hipStream_t st) {
  DevBuf flag(sizeof(int));
  QMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    {
      TimedLaunch tl_("setup/eo_site_term", st, double(g.V) * 36 * (16.0 + 2 * sizeof(S)), 0.0);
      launch(k_eo_site_term<S>, dim3(unsigned((g.V + 127) / 128), 2), dim3(128), 0, st,
             static_cast<const double2*>(A64), static_cast<S*>(Aeo), static_cast<S*>(Ainv), eo_geom(g),
             flag.as<int>());
    }
  });
  QMG_LAUNCH_CHECK();
  int h = 0;
  QMG_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  QMG_CHECK(h == 0, QMG_EBREAKDOWN, "the site term is singular at some site: no even-odd preconditioning");
}

}  // namespace qmg
