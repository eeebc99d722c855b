// BLAS-1 kernels (deterministic double-accumulated reductions) and the multi-RHS Krylov
// solvers used by the smoother, the coarse solve and the outer solve.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <initializer_list>
#include <type_traits>

#include "krylov.hpp"
#include "timing.hpp"

namespace qmg {

namespace {

constexpr int RB = 256;  // threads per reduction workgroup (4 wavefronts)

__device__ inline double2 warp_sum(double2 v) {  // total in every lane
  return make_double2(wave_sum(v.x), wave_sum(v.y));
}

__device__ inline double2 block_sum(double2 v) {
  __shared__ double2 red[RB / 64];
  v = warp_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < RB / 64; ++i) {
      s.x += red[i].x;
      s.y += red[i].y;
    }
  }
  return s;  // valid in thread 0
}

// Vectors are read and written in packs of P consecutive complex numbers (16 bytes for every
// storage type when the length and the pointers allow it, else P = 1).  Index arithmetic below
// is in packs: a vector of len complex numbers holds np = len / P packs.

}  // namespace

// out[c] = sum over b < nblk of partial[c * nblk + b], fixed order per thread + tree
__global__ __launch_bounds__(RB) void k_finalize2(const double2* __restrict__ partial, int nblk,
                                                  double2* __restrict__ out, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a device-side early exit (converged)
  const int c = blockIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (int b = threadIdx.x; b < nblk; b += RB) {
    acc.x += partial[size_t(c) * nblk + b].x;
    acc.y += partial[size_t(c) * nblk + b].y;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) out[c] = acc;
}

__global__ __launch_bounds__(RB) void k_finalize1(const double2* __restrict__ partial, int nblk,
                                                  double* __restrict__ out, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a device-side early exit (converged)
  const int c = blockIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (int b = threadIdx.x; b < nblk; b += RB) acc.x += partial[size_t(c) * nblk + b].x;
  acc = block_sum(acc);
  if (threadIdx.x == 0) out[c] = acc.x;
}

namespace {

// workgroups for a reduction over np packs with ncols independent outputs: at most about one
// resident wave of workgroups (256 CUs x 4 workgroups of the fused kernels), so that no
// partial second round of workgroups trails the first
int pick_nblk(size_t np, int ncols) {
  size_t nb = (np + RB * 2 - 1) / (RB * 2);
  size_t cap = std::max<size_t>(1, 1024 / std::max(1, ncols));
  nb = std::min(nb, cap);
  return int(std::max<size_t>(nb, 1));
}

inline unsigned nb256(size_t n) { return unsigned((n + 255) / 256); }

template <class S, int P>
__global__ void k_zero(S* x, size_t np) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  Pk<S, P> z;
#pragma unroll
  for (int u = 0; u < P; ++u) z.v[u] = StoreTraits<S>::st({ctype<S>(0), ctype<S>(0)});
  stp<S, P>(x, i, z);
}

template <class S, int P>
__global__ void k_copy(const S* __restrict__ x, S* __restrict__ y, size_t np) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < np) stp<S, P>(y, i, ldp<S, P>(x, i));
}

template <class S, int P>
__global__ void k_axpby(double a, const S* __restrict__ x, double b, S* __restrict__ y, size_t np) {
  using C = ctype<S>;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const auto xv = ldp<S, P>(x, i);
  auto yv = ldp<S, P>(y, i);
#pragma unroll
  for (int u = 0; u < P; ++u)
    yv.v[u] = StoreTraits<S>::st(C(a) * StoreTraits<S>::ld(xv.v[u]) + C(b) * StoreTraits<S>::ld(yv.v[u]));
  stp<S, P>(y, i, yv);
}

// w[r] += sgn * sum_i c[i * nrhs + r] X_i[r], accumulated in order of i; the basis loads are
// issued eight at a time so that their latencies overlap
template <class S, int P>
__global__ void k_axpy_multi(const S* __restrict__ X, size_t xstride_p, int m, const double2* __restrict__ c,
                             double sgn, S* __restrict__ w, size_t np, int nrhs, const int* __restrict__ skip,
                             const int* __restrict__ mcount) {
  if (skip && *skip) return;  // a device-side early exit (converged)
  using C = ctype<S>;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= np) return;
  if (mcount) m = min(m, mcount[r]);  // only the vectors this rhs actually built
  const size_t off = size_t(r) * np + e;
  auto wv = ldp<S, P>(w, off);
  cplx<C> acc[P];
#pragma unroll
  for (int u = 0; u < P; ++u) acc[u] = StoreTraits<S>::ld(wv.v[u]);
  int i = 0;
  for (; i + 8 <= m; i += 8) {
    Pk<S, P> xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xv[q] = ldp<S, P>(X, (i + q) * xstride_p + off);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double2 ci = c[size_t(i + q) * nrhs + r];
      const cplx<C> cc = {C(sgn * ci.x), C(sgn * ci.y)};
#pragma unroll
      for (int u = 0; u < P; ++u) acc[u] += cc * StoreTraits<S>::ld(xv[q].v[u]);
    }
  }
  for (; i < m; ++i) {
    const double2 ci = c[size_t(i) * nrhs + r];
    const cplx<C> cc = {C(sgn * ci.x), C(sgn * ci.y)};
    const auto xv = ldp<S, P>(X, i * xstride_p + off);
#pragma unroll
    for (int u = 0; u < P; ++u) acc[u] += cc * StoreTraits<S>::ld(xv.v[u]);
  }
#pragma unroll
  for (int u = 0; u < P; ++u) wv.v[u] = StoreTraits<S>::st(acc[u]);
  stp<S, P>(w, off, wv);
}

template <class S, int P>
__global__ void k_scale_dev(S* __restrict__ w, const double* __restrict__ n2, int mode, size_t np, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a device-side early exit (converged)
  using C = ctype<S>;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= np) return;
  const double v = n2[r];
  double f;
  if (mode == 0) f = (v > 0.0) ? 1.0 / sqrt(v) : 0.0;
  else if (mode == 1) f = sqrt(v);
  else f = v;
  const size_t off = size_t(r) * np + e;
  auto wv = ldp<S, P>(w, off);
#pragma unroll
  for (int u = 0; u < P; ++u) wv.v[u] = StoreTraits<S>::st(C(f) * StoreTraits<S>::ld(wv.v[u]));
  stp<S, P>(w, off, wv);
}

template <class S, int P>
__global__ void k_scale_cdev(S* __restrict__ w, const double2* __restrict__ c, double sgn, size_t np) {
  using C = ctype<S>;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= np) return;
  const cplx<C> cc = {C(sgn * c[r].x), C(sgn * c[r].y)};
  const size_t off = size_t(r) * np + e;
  auto wv = ldp<S, P>(w, off);
#pragma unroll
  for (int u = 0; u < P; ++u) wv.v[u] = StoreTraits<S>::st(cc * StoreTraits<S>::ld(wv.v[u]));
  stp<S, P>(w, off, wv);
}

template <class S, int P>
__global__ void k_caxpy_dev(const double2* __restrict__ c, double sgn, const S* __restrict__ y, S* __restrict__ x,
                            size_t np) {
  using C = ctype<S>;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= np) return;
  const cplx<C> cc = {C(sgn * c[r].x), C(sgn * c[r].y)};
  const size_t off = size_t(r) * np + e;
  auto xv = ldp<S, P>(x, off);
  const auto yv = ldp<S, P>(y, off);
#pragma unroll
  for (int u = 0; u < P; ++u)
    xv.v[u] = StoreTraits<S>::st(StoreTraits<S>::ld(xv.v[u]) + cc * StoreTraits<S>::ld(yv.v[u]));
  stp<S, P>(x, off, xv);
}

// ---------------------------------------------------------------------------------------
// Reductions.  Workgroup b of rhs r covers packs b*RB + tid, stepping by nblk*RB, and writes
// one partial sum per output column c at partial[c * nblk + b] (c = i * nrhs + r for basis
// vector i); a finalise kernel or the consuming kernel sums the partials in fixed order.

// partial <X_i, w> for the single basis vector i = blockIdx.z
template <class S, int P>
__global__ __launch_bounds__(RB) void k_dot_partial(const S* __restrict__ X, size_t xstride_p,
                                                    const S* __restrict__ w, size_t np, int nrhs, int nblk,
                                                    double2* __restrict__ partial) {
  const int b = blockIdx.x, r = blockIdx.y, i = blockIdx.z;
  const S* xi = X + i * xstride_p * P;
  double2 acc = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < np; e += size_t(nblk) * RB) {
    const auto a = ldp<S, P>(xi, size_t(r) * np + e);
    const auto c = ldp<S, P>(w, size_t(r) * np + e);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const auto av = StoreTraits<S>::ld(a.v[u]);
      const auto cv = StoreTraits<S>::ld(c.v[u]);
      const double ar = av.re, ai = av.im, cr = cv.re, ci = cv.im;
      acc.x += ar * cr + ai * ci;
      acc.y += ar * ci - ai * cr;
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[(size_t(i) * nrhs + r) * nblk + b] = acc;
}

template <class S, int P>
__global__ __launch_bounds__(RB) void k_norm_partial(const S* __restrict__ w, size_t np, int nblk,
                                                     double2* __restrict__ partial) {
  const int b = blockIdx.x, r = blockIdx.y;
  double2 acc = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < np; e += size_t(nblk) * RB) {
    const auto a = ldp<S, P>(w, size_t(r) * np + e);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const auto av = StoreTraits<S>::ld(a.v[u]);
      const double ar = av.re, ai = av.im;
      acc.x += ar * ar + ai * ai;
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[size_t(r) * nblk + b] = acc;
}

// Fused multi-vector kernels for the Arnoldi/GCR orthogonalisation: each reads the target
// vector w once for up to MG basis vectors (grid.z = group of MG vectors).
constexpr int MG = 8;
constexpr int kMaxCoef = 72;  // coefficients per right-hand side a fused consumer stages in LDS

template <class S>
__device__ inline void store_partials(double2 (&acc)[MG], int mi, double2* partial, int i0, int nrhs, int r, int b,
                                      int nblk) {
  __shared__ double2 red[MG][RB / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < MG; ++i) {
    if (i < mi) {  // uniform: only the live accumulators
      const double2 v = warp_sum(acc[i]);
      if (lane == 0) red[i][wid] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < mi) {
    const int i = threadIdx.x;
    double2 sacc = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < RB / 64; ++q) {
      sacc.x += red[i][q].x;
      sacc.y += red[i][q].y;
    }
    partial[(size_t(i0 + i) * nrhs + r) * nblk + b] = sacc;
  }
}

// Least-squares state of restarted GMRES, one thread per right-hand side, kept on the device
// so that a fixed-length cycle needs no host round trip.  Per rhs (double2 slots):
//   cs[m] (real in .x), sn[m], g[m+1], R[m*m] (upper triangle, column-major), {valid, stopped}
//   and |b| (in .x).
__host__ __device__ inline size_t gv_stride(int m) { return size_t(m) * m + 3 * size_t(m) + 3; }

struct GvView {
  double2* base;
  int m;
  __device__ double2* cs() const { return base; }
  __device__ double2* sn() const { return base + m; }
  __device__ double2* g() const { return base + 2 * m; }
  __device__ double2* R() const { return base + 3 * m + 1; }
  __device__ double2& flags() const { return base[size_t(m) * m + 3 * m + 1]; }
  __device__ double2& bn() const { return base[size_t(m) * m + 3 * m + 2]; }
};

__device__ inline double cabs2(double2 a) { return sqrt(a.x * a.x + a.y * a.y); }
__device__ inline double2 cmul2(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cconj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 cscale2(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ inline double2 cadd2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cdiv2(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

__device__ inline double2 shfl2(double2 v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

// One Givens step of the GMRES least-squares problem, executed by one whole wavefront (lane
// i holds entry i of Hessenberg column j in hl, i <= j; hsub = h[j+1]): applies the previous
// rotations in order through lane broadcasts, forms rotation j, stores column j of R and
// updates g; lane 0 writes (|g[j]|, |g[j+1]|) / |b| to *est.  m <= 64.
__device__ inline void gv_apply(GvView v, double2 hl, double2 hsub, int j, int lane, double2* est, double tol = 0.0,
                                int* conv = nullptr, int nrhs = 1, int r = 0) {
  double2* g = v.g();
  const double2 fl = v.flags();
  const int valid = int(fl.x);
  const double bn = v.bn().x;
  const double inv_bn = bn > 0.0 ? 1.0 / bn : 0.0;
  const double before = cabs2(g[valid]) * inv_bn;
  if (fl.y != 0.0) {  // stopped earlier in this cycle
    if (lane == 0) *est = make_double2(before, before);
    return;
  }
  double2 csl = make_double2(0.0, 0.0), snl = make_double2(0.0, 0.0);
  if (lane < j) {
    csl = v.cs()[lane];
    snl = v.sn()[lane];
  }
  double2* R = v.R();
  const int m = v.m;
  // cur = h[i] after rotations 0..i-1; rotation i mixes it with h[i+1]
  double2 cur = shfl2(hl, 0);
  for (int i = 0; i < j; ++i) {
    const double2 nxt = shfl2(hl, i + 1);
    const double ci = __shfl(csl.x, i, 64);
    const double2 si = shfl2(snl, i);
    const double2 t = cadd2(cscale2(ci, cur), cmul2(si, nxt));
    cur = cadd2(cscale2(-1.0, cmul2(cconj2(si), cur)), cscale2(ci, nxt));
    if (lane == 0) R[size_t(j) * m + i] = t;
  }
  if (lane != 0) return;
  const double2 a = cur, b = hsub;
  const double aa = cabs2(a), bb = cabs2(b);
  const double den = sqrt(aa * aa + bb * bb);
  if (den == 0.0 || !isfinite(den)) {  // singular column: the cycle stops before it
    v.flags() = make_double2(double(valid), 1.0);
    *est = make_double2(before, isfinite(den) ? before : den);
    return;
  }
  double2 c, sn;
  if (aa == 0.0) {
    c = make_double2(0.0, 0.0);
    sn = cscale2(1.0 / bb, cconj2(b));
  } else {
    c = make_double2(aa / den, 0.0);
    sn = cscale2(1.0 / den, cmul2(cscale2(1.0 / aa, a), cconj2(b)));
  }
  v.cs()[j] = c;
  v.sn()[j] = sn;
  R[size_t(j) * m + j] = cadd2(cscale2(c.x, a), cmul2(sn, b));
  const double2 gj = g[j];
  g[j + 1] = cscale2(-1.0, cmul2(cconj2(sn), gj));
  g[j] = cscale2(c.x, gj);
  const double after = cabs2(g[j + 1]) * inv_bn;
  bool stop = bb == 0.0;  // exact breakdown
  if (conv) {
    if (r == 0) atomicAdd(conv + 2, 1);
    if (after <= tol) {  // converged: this rhs stops; the last one to converge raises the skip flag
      stop = true;
      if (atomicAdd(conv, 1) == nrhs - 1) atomicExch(conv + 1, 1);
    }
  }
  v.flags() = make_double2(double(j + 1), stop ? 1.0 : 0.0);
  *est = make_double2(before, after);
}

// Givens step fused into the last kernel of an Arnoldi step (gst == nullptr: none)
struct GvFuse {
  double2* gst;
  int m, j;
  double2* est;
  double tol;  // with conv: device-side convergence test est <= tol
  int* conv;   // {rhs converged, all converged (the skip flag), steps of rhs 0}, or nullptr
  int nrhs;
};

// Where a kernel finds its per-rhs coefficients c_i (i < n): finalised values fin[i * nrhs + r],
// or, when partial is set, the per-workgroup partial sums partial[(i * nrhs + r) * nblk + q]
// (q < nblk) of the previous kernel, which every consumer workgroup sums itself in the same
// fixed order; workgroup (0, r) then stores the sums to fin_out[i * nrhs + r] (if set).
struct CoefSrc {
  const double2* fin;
  const double2* partial;
  int nblk;
  double2* fin_out;
};

__device__ inline void load_coefs(double2* s_c, int n, int r, int nrhs, const CoefSrc& src) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (src.partial) {
    for (int i = wid; i < n; i += nw) {
      const double2* p = src.partial + (size_t(i) * nrhs + r) * src.nblk;
      double2 a = make_double2(0.0, 0.0);
      for (int q = lane; q < src.nblk; q += 64) {
        a.x += p[q].x;
        a.y += p[q].y;
      }
      a = warp_sum(a);
      if (lane == 0) {
        s_c[i] = a;
        if (blockIdx.x == 0 && blockIdx.z == 0 && src.fin_out) src.fin_out[size_t(i) * nrhs + r] = a;
      }
    }
  } else {
    for (int i = threadIdx.x; i < n; i += blockDim.x) s_c[i] = src.fin[size_t(i) * nrhs + r];
  }
  __syncthreads();
}

// v[u] += sgn * sum_{i < m} c_i X_i[off] for the P entries of one pack, accumulated in order
// of i; loads are issued eight at a time so that their latencies overlap
template <class S, int P>
__device__ inline void acc_basis(cplx<ctype<S>> (&v)[P], const S* __restrict__ X, size_t xstride_p, size_t off,
                                 const double2* c, int m, double sgn) {
  using C = ctype<S>;
  int i = 0;
  for (; i + 8 <= m; i += 8) {
    Pk<S, P> xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xv[q] = ldp<S, P>(X, (i + q) * xstride_p + off);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const cplx<C> cc = {C(sgn * c[i + q].x), C(sgn * c[i + q].y)};
#pragma unroll
      for (int u = 0; u < P; ++u) v[u] += cc * StoreTraits<S>::ld(xv[q].v[u]);
    }
  }
  for (; i < m; ++i) {
    const cplx<C> cc = {C(sgn * c[i].x), C(sgn * c[i].y)};
    const auto xv = ldp<S, P>(X, i * xstride_p + off);
#pragma unroll
    for (int u = 0; u < P; ++u) v[u] += cc * StoreTraits<S>::ld(xv.v[u]);
  }
}

// acc[i] += <X_{i0+i}[off], w> over the P entries of one pack (cw: the entries of w)
template <class S, int P>
__device__ inline void acc_dots(double2 (&acc)[MG], const S* __restrict__ X, size_t xstride_p, size_t off, int i0,
                                int mi, const double (&cr)[P], const double (&ci)[P]) {
  Pk<S, P> xv[MG];
#pragma unroll
  for (int i = 0; i < MG; ++i)
    if (i < mi) xv[i] = ldp<S, P>(X, (i0 + i) * xstride_p + off);
#pragma unroll
  for (int i = 0; i < MG; ++i) {
    if (i < mi) {
#pragma unroll
      for (int u = 0; u < P; ++u) {
        const auto a = StoreTraits<S>::ld(xv[i].v[u]);
        const double ar = a.re, ai = a.im;
        acc[i].x += ar * cr[u] + ai * ci[u];
        acc[i].y += ar * ci[u] - ai * cr[u];
      }
    }
  }
}

// partial <X_i, w> for i in [i0, i0 + MG) of this z-group
template <class S, int P>
__global__ __launch_bounds__(RB) void k_mdot(const S* __restrict__ X, size_t xstride_p, int m,
                                             const S* __restrict__ w, size_t np, int nrhs, int nblk,
                                             double2* __restrict__ partial, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a device-side early exit (converged)
  const int b = blockIdx.x, r = blockIdx.y, i0 = blockIdx.z * MG;
  const int mi = min(MG, m - i0);
  double2 acc[MG];
#pragma unroll
  for (int i = 0; i < MG; ++i) acc[i] = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < np; e += size_t(nblk) * RB) {
    const size_t off = size_t(r) * np + e;
    const auto c = ldp<S, P>(w, off);
    double cr[P], ci[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const auto cv = StoreTraits<S>::ld(c.v[u]);
      cr[u] = cv.re;
      ci[u] = cv.im;
    }
    acc_dots<S, P>(acc, X, xstride_p, off, i0, mi, cr, ci);
  }
  store_partials<S>(acc, mi, partial, i0, nrhs, r, b, nblk);
}

// wout <- w + sgn * sum_i c_i X_i (all m vectors), then partial <X_i, wout> (grid.z groups) or
// partial |wout|^2 (mode 1, grid.z = 1).  Each z-group recomputes the same update; only z = 0
// stores it, so wout may alias w only with a single z-group.
template <class S, int MODE, int P>
__global__ __launch_bounds__(RB) void k_axpy_then(const S* __restrict__ X, size_t xstride_p, int m, CoefSrc csrc,
                                                  double sgn, const S* w, S* wout, size_t np, int nrhs, int nblk,
                                                  double2* __restrict__ partial, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a device-side early exit (converged)
  using C = ctype<S>;
  const int b = blockIdx.x, r = blockIdx.y, i0 = blockIdx.z * MG;
  const int mi = MODE == 0 ? min(MG, m - i0) : 1;
  __shared__ double2 s_c[kMaxCoef];
  load_coefs(s_c, m, r, nrhs, csrc);
  double2 acc[MG];
#pragma unroll
  for (int i = 0; i < MG; ++i) acc[i] = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < np; e += size_t(nblk) * RB) {
    const size_t off = size_t(r) * np + e;
    auto wv = ldp<S, P>(w, off);
    cplx<C> v[P];
#pragma unroll
    for (int u = 0; u < P; ++u) v[u] = StoreTraits<S>::ld(wv.v[u]);
    acc_basis<S, P>(v, X, xstride_p, off, s_c, m, sgn);
    double cr[P], ci[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      wv.v[u] = StoreTraits<S>::st(v[u]);
      const auto vv = StoreTraits<S>::ld(wv.v[u]);  // the stored (rounded) value
      cr[u] = vv.re;
      ci[u] = vv.im;
    }
    if (blockIdx.z == 0) stp<S, P>(wout, off, wv);
    if (MODE == 0) {
      acc_dots<S, P>(acc, X, xstride_p, off, i0, mi, cr, ci);
    } else {
#pragma unroll
      for (int u = 0; u < P; ++u) acc[0].x += cr[u] * cr[u] + ci[u] * ci[u];
    }
  }
  store_partials<S>(acc, mi, partial, i0, nrhs, r, b, nblk);
}

// partial <X_i, w> (grid.z groups of MG) and, in group 0, partial |w|^2 stored at slot m
template <class S, int P>
__global__ __launch_bounds__(RB) void k_mdot_norm(const S* __restrict__ X, size_t xstride_p, int m,
                                                  const S* __restrict__ w, size_t np, int nrhs, int nblk,
                                                  double2* __restrict__ partial, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a device-side early exit (converged)
  const int b = blockIdx.x, r = blockIdx.y, i0 = blockIdx.z * MG;
  const int mi = min(MG, m - i0);
  double2 acc[MG];
  double nn = 0.0;
#pragma unroll
  for (int i = 0; i < MG; ++i) acc[i] = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < np; e += size_t(nblk) * RB) {
    const size_t off = size_t(r) * np + e;
    const auto c = ldp<S, P>(w, off);
    double cr[P], ci[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const auto cv = StoreTraits<S>::ld(c.v[u]);
      cr[u] = cv.re;
      ci[u] = cv.im;
      nn += cr[u] * cr[u] + ci[u] * ci[u];
    }
    acc_dots<S, P>(acc, X, xstride_p, off, i0, mi, cr, ci);
  }
  store_partials<S>(acc, mi, partial, i0, nrhs, r, b, nblk);
  if (blockIdx.z == 0) {
    double2 t = block_sum(make_double2(nn, 0.0));
    if (threadIdx.x == 0) partial[(size_t(m) * nrhs + r) * nblk + b] = t;
  }
}

// w <- (w - sum_i c_i X_i) / beta with beta^2 = |w|^2 - sum_i |c_i|^2 (Pythagoras, c = X^dag w
// for orthonormal X); coefficient slot m holds |w|^2 before the update; beta^2 is written to
// out_n2 (workgroup 0).
template <class S, int P>
__global__ __launch_bounds__(256) void k_axpy_scale(const S* __restrict__ X, size_t xstride_p, int m, CoefSrc csrc,
                                                    S* __restrict__ w, size_t np, int nrhs,
                                                    double* __restrict__ out_n2, GvFuse gf, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a device-side early exit (converged)
  using C = ctype<S>;
  const int r = blockIdx.y;
  __shared__ double2 s_c[kMaxCoef];
  load_coefs(s_c, m + 1, r, nrhs, csrc);
  double b2 = s_c[m].x;
  for (int i = 0; i < m; ++i) b2 -= s_c[i].x * s_c[i].x + s_c[i].y * s_c[i].y;
  b2 = fmax(b2, 0.0);
  const double inv = b2 > 0.0 ? 1.0 / sqrt(b2) : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) out_n2[r] = b2;
  if (gf.gst && blockIdx.x == 0 && threadIdx.x < 64) {  // Hessenberg column j = (h, beta)
    const int lane = threadIdx.x;
    const double2 hl = lane <= gf.j ? s_c[lane] : make_double2(0.0, 0.0);
    gv_apply(GvView{gf.gst + r * gv_stride(gf.m), gf.m}, hl, make_double2(sqrt(b2), 0.0), gf.j, lane,
             gf.est + r, gf.tol, gf.conv, gf.nrhs, r);
  }
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= np) return;
  const size_t off = size_t(r) * np + e;
  auto wv = ldp<S, P>(w, off);
  cplx<C> v[P];
#pragma unroll
  for (int u = 0; u < P; ++u) v[u] = StoreTraits<S>::ld(wv.v[u]);
  acc_basis<S, P>(v, X, xstride_p, off, s_c, m, -1.0);
#pragma unroll
  for (int u = 0; u < P; ++u) wv.v[u] = StoreTraits<S>::st(C(inv) * v[u]);
  stp<S, P>(w, off, wv);
}

// w[r] /= sqrt(n2) with n2 = the real part of the single coefficient of rhs r (zero norm gives
// a zero vector); workgroup 0 stores n2 to out_n2[r]
template <class S, int P>
__global__ __launch_bounds__(256) void k_scale_norm(S* __restrict__ w, CoefSrc csrc, size_t np, int nrhs,
                                                    double* __restrict__ out_n2, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a device-side early exit (converged)
  using C = ctype<S>;
  const int r = blockIdx.y;
  __shared__ double2 s_c[1];
  load_coefs(s_c, 1, r, nrhs, csrc);
  const double v = s_c[0].x;
  if (blockIdx.x == 0 && threadIdx.x == 0) out_n2[r] = v;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= np) return;
  const double f = (v > 0.0) ? 1.0 / sqrt(v) : 0.0;
  const size_t off = size_t(r) * np + e;
  auto wv = ldp<S, P>(w, off);
#pragma unroll
  for (int u = 0; u < P; ++u) wv.v[u] = StoreTraits<S>::st(C(f) * StoreTraits<S>::ld(wv.v[u]));
  stp<S, P>(w, off, wv);
}

// Pack width usable for vectors of len complex numbers at the given pointers (and basis
// stride): the full 16-byte pack when everything is a multiple of it, else 1.
template <class S>
bool packable(size_t len, size_t xstride, std::initializer_list<const void*> ptrs) {
  constexpr int P = kPack<S>;
  if (P == 1) return true;
  if (len % P || xstride % P) return false;
  for (const void* p : ptrs)
    if (reinterpret_cast<uintptr_t>(p) % 16) return false;
  return true;
}

template <class S>
bool packable_vec(size_t len, const void* p) {
  return packable<S>(len, 0, {p});
}

// Short vectors (the coarse level) are latency bound: there the consumer of a reduction sums
// the producer's partials itself instead of a separate finalise launch, with at most
// kSmallBlk partials per coefficient.
constexpr size_t kSmallLen = size_t(RB) * 128 * 8;
constexpr int kSmallBlk = 128;
inline int small_nblk(size_t np) { return int(std::min<size_t>(kSmallBlk, std::max<size_t>(1, (np + RB - 1) / RB))); }

// Host side of every operation, for one pack width.
template <class S, int P>
struct BlasP {
  static void zero(void* x, size_t n, hipStream_t st) {
    {
      TimedLaunch tl_("blas/zero", st, double(n) * sizeof(S), 0.0);
      launch(k_zero<S, P>, dim3(nb256(n / P)), dim3(256), 0, st, (S*)x, n / P);
    }
    QMG_LAUNCH_CHECK();
  }
  static void copy(const void* x, void* y, size_t n, hipStream_t st) {
    {
      TimedLaunch tl_("blas/copy", st, 2.0 * double(n) * sizeof(S), 0.0);
      launch(k_copy<S, P>, dim3(nb256(n / P)), dim3(256), 0, st, (const S*)x, (S*)y, n / P);
    }
    QMG_LAUNCH_CHECK();
  }
  static void axpby(double a, const void* x, double b, void* y, size_t n, hipStream_t st) {
    {
      TimedLaunch tl_("blas/axpby", st, 3.0 * double(n) * sizeof(S), 0.0);
      launch(k_axpby<S, P>, dim3(nb256(n / P)), dim3(256), 0, st, a, (const S*)x, b, (S*)y, n / P);
    }
    QMG_LAUNCH_CHECK();
  }
  static void dot_multi(const void* X, size_t xstride, int m, const void* w, size_t len, int nrhs, double2* out,
                        RedWork& rw, hipStream_t st) {
    const int* skip = nullptr;
    const size_t np = len / P;
    const int nblk = pick_nblk(np, m * nrhs);
    rw.ensure(size_t(nblk) * m * nrhs, 0);
    {
      TimedLaunch tl_("blas/dot", st, double(m + 1) * len * nrhs * sizeof(S), 0.0);
      launch(k_dot_partial<S, P>, dim3(nblk, nrhs, m), dim3(RB), 0, st, (const S*)X, xstride / P, (const S*)w, np,
             nrhs, nblk, rw.partial.as<double2>());
    }
    QMG_LAUNCH_CHECK();
    {
      TimedLaunch tl_("blas/finalize", st, double(nblk) * (m + 1) * nrhs * sizeof(double2), 0.0);
      launch(k_finalize2, dim3(m * nrhs), dim3(RB), 0, st, rw.partial.as<double2>(), nblk, out, skip);
    }
    QMG_LAUNCH_CHECK();
  }
  static void norm2(const void* w, size_t len, int nrhs, double* out, RedWork& rw, hipStream_t st) {
    const size_t np = len / P;
    const int nblk = pick_nblk(np, nrhs);
    rw.ensure(size_t(nblk) * nrhs, 0);
    {
      TimedLaunch tl_("blas/norm", st, double(len) * nrhs * sizeof(S), 0.0);
      launch(k_norm_partial<S, P>, dim3(nblk, nrhs), dim3(RB), 0, st, (const S*)w, np, nblk,
             rw.partial.as<double2>());
    }
    QMG_LAUNCH_CHECK();
    {
      TimedLaunch tl_("blas/finalize", st, double(nblk) * nrhs * sizeof(double2), 0.0);
      launch(k_finalize1, dim3(nrhs), dim3(RB), 0, st, rw.partial.as<double2>(), nblk, out, nullptr);
    }
    QMG_LAUNCH_CHECK();
  }
  static void axpy_multi(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w, size_t len,
                         int nrhs, hipStream_t st, const int* skip, const int* mcount) {
    const size_t np = len / P;
    {
      TimedLaunch tl_("blas/axpy_multi", st, double(m + 2) * len * nrhs * sizeof(S), 0.0);
      launch(k_axpy_multi<S, P>, dim3(nb256(np), nrhs), dim3(256), 0, st, (const S*)X, xstride / P, m, c, sgn, (S*)w,
             np, nrhs, skip, mcount);
    }
    QMG_LAUNCH_CHECK();
  }
  static void scale_dev(void* w, const double* n2, int mode, size_t len, int nrhs, hipStream_t st,
                        const int* skip) {
    {
      TimedLaunch tl_("blas/scale", st, 2.0 * len * nrhs * sizeof(S), 0.0);
      launch(k_scale_dev<S, P>, dim3(nb256(len / P), nrhs), dim3(256), 0, st, (S*)w, n2, mode, len / P, skip);
    }
    QMG_LAUNCH_CHECK();
  }
  static void scale_cdev(void* w, const double2* c, double sgn, size_t len, int nrhs, hipStream_t st) {
    {
      TimedLaunch tl_("blas/scale", st, 2.0 * len * nrhs * sizeof(S), 0.0);
      launch(k_scale_cdev<S, P>, dim3(nb256(len / P), nrhs), dim3(256), 0, st, (S*)w, c, sgn, len / P);
    }
    QMG_LAUNCH_CHECK();
  }
  static void caxpy_dev(const double2* c, double sgn, const void* y, void* x, size_t len, int nrhs,
                        hipStream_t st) {
    {
      TimedLaunch tl_("blas/caxpy", st, 3.0 * len * nrhs * sizeof(S), 0.0);
      launch(k_caxpy_dev<S, P>, dim3(nb256(len / P), nrhs), dim3(256), 0, st, c, sgn, (const S*)y, (S*)x, len / P);
    }
    QMG_LAUNCH_CHECK();
  }
  static void mdot(const void* X, size_t xstride, int m, const void* w, size_t len, int nrhs, double2* out,
                   RedWork& rw, hipStream_t st, const int* skip) {
    const size_t np = len / P;
    const int ng = (m + MG - 1) / MG;
    const int nblk = pick_nblk(np, ng * nrhs);
    rw.ensure(size_t(nblk) * m * nrhs, 0);
    {
      TimedLaunch tl_("blas/mdot", st, double(m + 1) * len * nrhs * sizeof(S), 0.0);
      launch(k_mdot<S, P>, dim3(nblk, nrhs, ng), dim3(RB), 0, st, (const S*)X, xstride / P, m, (const S*)w, np, nrhs,
             nblk, rw.partial.as<double2>(), skip);
    }
    QMG_LAUNCH_CHECK();
    {
      TimedLaunch tl_("blas/finalize", st, double(nblk) * (m + 1) * nrhs * sizeof(double2), 0.0);
      launch(k_finalize2, dim3(m * nrhs), dim3(RB), 0, st, rw.partial.as<double2>(), nblk, out, skip);
    }
    QMG_LAUNCH_CHECK();
  }
  static void axpy_then(int mode, const void* X, size_t xstride, int m, const double2* c, double sgn, void* w,
                        size_t len, int nrhs, void* out, RedWork& rw, hipStream_t st, const int* skip) {
    const size_t np = len / P;
    const int nblk = pick_nblk(np, nrhs);
    rw.ensure(size_t(nblk) * std::max(m, 1) * nrhs, 0);
    const CoefSrc src{c, nullptr, 0, nullptr};
    if (mode == 0) {
      {
        TimedLaunch tl_("blas/axpy_then", st, double(m + 2) * len * nrhs * sizeof(S), 0.0);
        launch(k_axpy_then<S, 0, P>, dim3(nblk, nrhs, 1), dim3(RB), 0, st, (const S*)X, xstride / P, m, src, sgn,
               (const S*)w, (S*)w, np, nrhs, nblk, rw.partial.as<double2>(), skip);
      }
      QMG_LAUNCH_CHECK();
      {
        TimedLaunch tl_("blas/finalize", st, double(nblk) * (m + 1) * nrhs * sizeof(double2), 0.0);
        launch(k_finalize2, dim3(m * nrhs), dim3(RB), 0, st, rw.partial.as<double2>(), nblk, (double2*)out, skip);
      }
    } else {
      {
        TimedLaunch tl_("blas/axpy_then", st, double(m + 2) * len * nrhs * sizeof(S), 0.0);
        launch(k_axpy_then<S, 1, P>, dim3(nblk, nrhs, 1), dim3(RB), 0, st, (const S*)X, xstride / P, m, src, sgn,
               (const S*)w, (S*)w, np, nrhs, nblk, rw.partial.as<double2>(), skip);
      }
      QMG_LAUNCH_CHECK();
      {
        TimedLaunch tl_("blas/finalize", st, double(nblk) * nrhs * sizeof(double2), 0.0);
        launch(k_finalize1, dim3(nrhs), dim3(RB), 0, st, rw.partial.as<double2>(), nblk, (double*)out, skip);
      }
    }
    QMG_LAUNCH_CHECK();
  }
  static void cgs1(const void* X, size_t xstride, int m, void* w, size_t len, int nrhs, double2* h, double* n2,
                   RedWork& rw, hipStream_t st, GvFuse gf, const int* skip) {
    const size_t np = len / P;
    const int ng = (m + MG - 1) / MG;
    const bool small = len <= kSmallLen;
    const int nblk = small ? small_nblk(np) : pick_nblk(np, ng * nrhs);
    rw.ensure(size_t(nblk) * (m + 1) * nrhs, size_t(nrhs));
    double2* part = rw.partial.as<double2>();
    {
      TimedLaunch tl_("blas/mdot_norm", st, double(m + 1) * len * nrhs * sizeof(S), 0.0);
      launch(k_mdot_norm<S, P>, dim3(nblk, nrhs, ng), dim3(RB), 0, st, (const S*)X, xstride / P, m, (const S*)w, np,
             nrhs, nblk, part, skip);
    }
    QMG_LAUNCH_CHECK();
    CoefSrc src{h, nullptr, 0, nullptr};
    if (small) {
      src = CoefSrc{nullptr, part, nblk, h};
    } else {
      {
        TimedLaunch tl_("blas/finalize", st, double(nblk) * (m + 1) * nrhs * sizeof(double2), 0.0);
        launch(k_finalize2, dim3((m + 1) * nrhs), dim3(RB), 0, st, part, nblk, h, skip);
      }
      QMG_LAUNCH_CHECK();
    }
    {
      TimedLaunch tl_("blas/axpy_scale", st, double(m + 2) * len * nrhs * sizeof(S), 0.0);
      launch(k_axpy_scale<S, P>, dim3(nb256(np), nrhs), dim3(256), 0, st, (const S*)X, xstride / P, m, src, (S*)w, np,
             nrhs, n2, gf, skip);
    }
    QMG_LAUNCH_CHECK();
  }
  static void cgs2_small(const void* X, size_t xstride, int m, void* w, size_t len, int nrhs, double2* h1,
                         double2* h2, double* n2, RedWork& rw, hipStream_t st, const int* skip) {
    const size_t np = len / P;
    const int ng = (m + MG - 1) / MG;
    const int nblk = small_nblk(np);
    rw.ensure(size_t(nblk) * m * nrhs, 0);
    // second buffer: partials, then w' (16-byte aligned after the partials)
    rw.ensure2(size_t(nblk) * m * nrhs + (len * nrhs * sizeof(S) + sizeof(double2) - 1) / sizeof(double2));
    double2* pa = rw.partial.as<double2>();
    double2* pb = rw.partial2.as<double2>();
    S* wtmp = reinterpret_cast<S*>(pb + size_t(nblk) * m * nrhs);
    // pass 1: partials of X^dag w
    {
      TimedLaunch tl_("blas/mdot", st, double(m + 1) * len * nrhs * sizeof(S), 0.0);
      launch(k_mdot<S, P>, dim3(nblk, nrhs, ng), dim3(RB), 0, st, (const S*)X, xstride / P, m, (const S*)w, np, nrhs,
             nblk, pa, skip);
    }
    QMG_LAUNCH_CHECK();
    // w' = w - X h1 (h1 summed from pa) into wtmp, partials of X^dag w' into pb
    {
      TimedLaunch tl_("blas/axpy_then", st, double(m + 2) * len * nrhs * sizeof(S), 0.0);
      launch(k_axpy_then<S, 0, P>, dim3(nblk, nrhs, ng), dim3(RB), 0, st, (const S*)X, xstride / P, m,
             CoefSrc{nullptr, pa, nblk, h1}, -1.0, (const S*)w, wtmp, np, nrhs, nblk, pb, skip);
    }
    QMG_LAUNCH_CHECK();
    // w = w' - X h2 (h2 summed from pb), partial |w|^2 into pa
    {
      TimedLaunch tl_("blas/axpy_then", st, double(m + 2) * len * nrhs * sizeof(S), 0.0);
      launch(k_axpy_then<S, 1, P>, dim3(nblk, nrhs, 1), dim3(RB), 0, st, (const S*)X, xstride / P, m,
             CoefSrc{nullptr, pb, nblk, h2}, -1.0, (const S*)wtmp, (S*)w, np, nrhs, nblk, pa, skip);
    }
    QMG_LAUNCH_CHECK();
    {
      TimedLaunch tl_("blas/scale", st, 2.0 * len * nrhs * sizeof(S), 0.0);
      launch(k_scale_norm<S, P>, dim3(nb256(np), nrhs), dim3(256), 0, st, (S*)w, CoefSrc{nullptr, pa, nblk, nullptr},
             np, nrhs, n2, skip);
    }
    QMG_LAUNCH_CHECK();
  }
};

}  // namespace

// ---------------------------------------------------------------------------------------
// Blas<S>: pick the pack width, then dispatch
#define QMG_PACKED(cond, call)             \
  do {                                     \
    if (cond) BlasP<S, kPack<S>>::call;    \
    else BlasP<S, 1>::call;                \
  } while (0)

template <class S>
void Blas<S>::zero(void* x, size_t n, hipStream_t st) {
  if (!n) return;
  QMG_PACKED(packable<S>(n, 0, {x}), zero(x, n, st));
}
template <class S>
void Blas<S>::copy(const void* x, void* y, size_t n, hipStream_t st) {
  if (!n) return;
  QMG_PACKED(packable<S>(n, 0, {x, y}), copy(x, y, n, st));
}
template <class S>
void Blas<S>::axpby(double a, const void* x, double b, void* y, size_t n, hipStream_t st) {
  if (!n) return;
  QMG_PACKED(packable<S>(n, 0, {x, y}), axpby(a, x, b, y, n, st));
}
template <class S>
void Blas<S>::dot_multi(const void* X, size_t xstride, int m, const void* w, size_t len, int nrhs, double2* out,
                        RedWork& rw, hipStream_t st) {
  if (m <= 0) return;
  QMG_PACKED(packable<S>(len, xstride, {X, w}), dot_multi(X, xstride, m, w, len, nrhs, out, rw, st));
}
template <class S>
void Blas<S>::norm2(const void* w, size_t len, int nrhs, double* out, RedWork& rw, hipStream_t st) {
  QMG_PACKED(packable<S>(len, 0, {w}), norm2(w, len, nrhs, out, rw, st));
}
template <class S>
void Blas<S>::axpy_multi(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w, size_t len,
                         int nrhs, hipStream_t st, const int* skip, const int* mcount) {
  if (m <= 0) return;
  QMG_PACKED(packable<S>(len, xstride, {X, w}), axpy_multi(X, xstride, m, c, sgn, w, len, nrhs, st, skip, mcount));
}
template <class S>
void Blas<S>::scale_dev(void* w, const double* n2, int mode, size_t len, int nrhs, hipStream_t st,
                        const int* skip) {
  QMG_PACKED(packable<S>(len, 0, {w}), scale_dev(w, n2, mode, len, nrhs, st, skip));
}
template <class S>
void Blas<S>::scale_cdev(void* w, const double2* c, double sgn, size_t len, int nrhs, hipStream_t st) {
  QMG_PACKED(packable<S>(len, 0, {w}), scale_cdev(w, c, sgn, len, nrhs, st));
}
template <class S>
void Blas<S>::caxpy_dev(const double2* c, double sgn, const void* y, void* x, size_t len, int nrhs,
                        hipStream_t st) {
  QMG_PACKED(packable<S>(len, 0, {x, y}), caxpy_dev(c, sgn, y, x, len, nrhs, st));
}
template <class S>
void Blas<S>::mdot(const void* X, size_t xstride, int m, const void* w, size_t len, int nrhs, double2* out,
                   RedWork& rw, hipStream_t st, const int* skip) {
  if (m <= 0) return;
  QMG_PACKED(packable<S>(len, xstride, {X, w}), mdot(X, xstride, m, w, len, nrhs, out, rw, st, skip));
}
template <class S>
void Blas<S>::axpy_mdot(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w, size_t len,
                        int nrhs, double2* out, RedWork& rw, hipStream_t st, const int* skip) {
  if (m <= 0) return;
  // the update must be complete before other z-groups read w: one group only when m > MG
  if (m > MG) {
    axpy_multi(X, xstride, m, c, sgn, w, len, nrhs, st, skip);
    mdot(X, xstride, m, w, len, nrhs, out, rw, st, skip);
    return;
  }
  QMG_PACKED(packable<S>(len, xstride, {X, w}), axpy_then(0, X, xstride, m, c, sgn, w, len, nrhs, out, rw, st, skip));
}
template <class S>
void Blas<S>::axpy_norm(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w, size_t len,
                        int nrhs, double* out, RedWork& rw, hipStream_t st, const int* skip) {
  if (m > kMaxCoef) {
    QMG_CHECK(!skip, QMG_EINVAL, "device early exit needs at most 72 basis vectors");
    axpy_multi(X, xstride, m, c, sgn, w, len, nrhs, st);
    norm2(w, len, nrhs, out, rw, st);
    return;
  }
  QMG_PACKED(packable<S>(len, xstride, {X, w}), axpy_then(1, X, xstride, m, c, sgn, w, len, nrhs, out, rw, st, skip));
}
template <class S>
bool Blas<S>::cgs1_step(const void* X, size_t xstride, int m, void* w, size_t len, int nrhs, double2* h, double* n2,
                        RedWork& rw, hipStream_t st, double2* gst, int gm, double2* est, double tol, int* conv) {
  QMG_CHECK(m >= 1, QMG_EINVAL, "Gram-Schmidt step: no basis vectors");
  const int* skip = conv ? conv + 1 : nullptr;
  if (m + 1 > kMaxCoef || m > 64) {  // long bases: explicit update and norm instead of Pythagoras
    QMG_CHECK(!conv, QMG_EINVAL, "device early exit needs at most 63 basis vectors");
    mdot(X, xstride, m, w, len, nrhs, h, rw, st);
    axpy_multi(X, xstride, m, h, -1.0, w, len, nrhs, st);
    norm2(w, len, nrhs, n2, rw, st);
    scale_dev(w, n2, 0, len, nrhs, st);
    return false;
  }
  const GvFuse gf{gst, gm, m - 1, est, tol, conv, nrhs};
  QMG_PACKED(packable<S>(len, xstride, {X, w}), cgs1(X, xstride, m, w, len, nrhs, h, n2, rw, st, gf, skip));
  return gst != nullptr;
}
template <class S>
void Blas<S>::cgs2_step(const void* X, size_t xstride, int m, void* w, size_t len, int nrhs, double2* h1,
                        double2* h2, double* n2, RedWork& rw, hipStream_t st, const int* skip) {
  QMG_CHECK(m >= 1, QMG_EINVAL, "Gram-Schmidt step: no basis vectors");
  if (len > kSmallLen || m > kMaxCoef) {
    mdot(X, xstride, m, w, len, nrhs, h1, rw, st, skip);
    axpy_mdot(X, xstride, m, h1, -1.0, w, len, nrhs, h2, rw, st, skip);
    axpy_norm(X, xstride, m, h2, -1.0, w, len, nrhs, n2, rw, st, skip);
    scale_dev(w, n2, 0, len, nrhs, st, skip);
    return;
  }
  QMG_PACKED(packable<S>(len, xstride, {X, w}), cgs2_small(X, xstride, m, w, len, nrhs, h1, h2, n2, rw, st, skip));
}
#undef QMG_PACKED

template struct Blas<double2>;
template struct Blas<float2>;
template struct Blas<cbf16>;
template struct Blas<chalf>;

// The update that closes one s-step cycle, in one pass over the basis p_0 .. p_s of each
// right-hand side (p_0 is the residual): x += sum_j c_j p_j (x = ... when add is 0, without
// reading x) and, unless it is the last cycle,
// p_0 <- p_0 - sum_j c_j D p_j with D p_j = p_{j+1} + d p_j (the shifted basis), accumulated in
// the storage type's arithmetic precision.  Each thread reads and writes only its own element,
// so p_0 is updated in place.
template <class S>
__global__ __launch_bounds__(256) void k_sstep_update(const S* basis, size_t vstride, int s,
                                                      const double2* __restrict__ c, double d, S* __restrict__ x,
                                                      S* p0, size_t len, int nrhs, int res, int add) {
  using C = ctype<S>;
  const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= len) return;
  const size_t off = size_t(r) * len + e;
  cplx<C> p[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) p[i] = i <= s ? ldc(basis, size_t(i) * vstride + off) : cplx<C>{C(0), C(0)};
  cplx<C> ax = add ? ldc(x, off) : cplx<C>{C(0), C(0)}, ar = p[0];
  const C dd = C(d);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (j >= s) break;
    const double2 cj = c[size_t(j) * nrhs + r];
    const cplx<C> cc = {C(cj.x), C(cj.y)};
    ax += cc * p[j];
    ar -= cc * (p[j + 1] + dd * p[j]);
  }
  stc(x, off, ax);
  if (res) stc(p0, off, ar);
}

// s-step form of the smoothing GMRES(8) cycles (storage below FP64): per cycle, from the
// residual r, the shifted basis p_0 = r, p_{i+1} = (D - d) p_i (d the diagonal term m + 1 + 3/xi,
// which centres the spectrum and keeps the powers better conditioned; the Krylov space is
// that of D) is formed with the same eight operator applications as eight GMRES steps, one pass
// gives every <p_i, p_j>, and the 8 x 8 normal equations of min ||r - D sum_j c_j p_j|| are
// solved in FP64 on the device: the minimisation of GMRES(8) over the same space, with one
// reduction instead of eight Gram-Schmidt steps over a growing basis.  The next cycle's residual
// r - sum_j c_j (p_{j+1} + d p_j) comes from the basis, without another operator application;
// it and the update of x are one pass over the basis (k_sstep_update).
template <class S>
void smooth_sstep(size_t len, double d, LinOp& D, LinOp* H, int r, int n_iter, const void* b, void* x, DevBuf& basis,
                  DevBuf& coef, DevBuf& part, DevBuf& e, hipStream_t st) {
  constexpr qmg_prec P = StoreTraits<S>::prec;
  constexpr int s = 8;
  const size_t n = len * r, vb = n * sizeof(S);
  basis.ensure((s + 1) * vb);
  coef.ensure(size_t(s) * r * sizeof(double2));
  (void)e;
  auto vec = [&](int i) { return static_cast<char*>(basis.p) + size_t(i) * vb; };
  if (n_iter / s == 0) Blas<S>::zero(x, n, st);  // otherwise the first cycle writes x
  Blas<S>::copy(b, vec(0), n, st);
  for (int cyc = 0; cyc < n_iter / s; ++cyc) {
    for (int i = 0; i < s; ++i) {
      if (H) {
        H->apply(vec(i), vec(i + 1), r, st);  // the hopping part: D - d directly
      } else {
        D.apply(vec(i), vec(i + 1), r, st);
        Blas<S>::axpby(-d, vec(i), 1.0, vec(i + 1), n, st);
      }
    }
    launch_sstep_coeffs(P, basis.p, s + 1, len, r, coef.as<double2>(), part, st, d);
    sstep_update<S>(basis.p, n, s, coef.as<double2>(), d, x, vec(0), len, r, cyc + 1 < n_iter / s, cyc > 0, st);
  }
}

template <class S>
void sstep_update(const void* basis, size_t vstride, int s, const double2* c, double d, void* x, void* p0, size_t len,
                  int nrhs, bool res, bool add, hipStream_t st) {
  const double n = double(len) * nrhs;
  {
    TimedLaunch tl_("sstep/update", st, double(s + 2 + (add ? 1 : 0) + (res ? 2 : 0)) * n * sizeof(S),
                    8.0 * (res ? 2 : 1) * s * n);
    launch(k_sstep_update<S>, dim3(unsigned((len + 255) / 256), nrhs), dim3(256), 0, st, static_cast<const S*>(basis),
           vstride, s, c, d, static_cast<S*>(x), static_cast<S*>(p0), len, nrhs, res ? 1 : 0, add ? 1 : 0);
  }
  QMG_LAUNCH_CHECK();
}
template void sstep_update<double2>(const void*, size_t, int, const double2*, double, void*, void*, size_t, int, bool,
                                    bool, hipStream_t);
template void sstep_update<float2>(const void*, size_t, int, const double2*, double, void*, void*, size_t, int, bool,
                                   bool, hipStream_t);
template void sstep_update<cbf16>(const void*, size_t, int, const double2*, double, void*, void*, size_t, int, bool,
                                  bool, hipStream_t);
template void sstep_update<chalf>(const void*, size_t, int, const double2*, double, void*, void*, size_t, int, bool,
                                  bool, hipStream_t);

template void smooth_sstep<float2>(size_t, double, LinOp&, LinOp*, int, int, const void*, void*, DevBuf&, DevBuf&,
                                   DevBuf&, DevBuf&, hipStream_t);
template void smooth_sstep<cbf16>(size_t, double, LinOp&, LinOp*, int, int, const void*, void*, DevBuf&, DevBuf&,
                                  DevBuf&, DevBuf&, hipStream_t);
template void smooth_sstep<chalf>(size_t, double, LinOp&, LinOp*, int, int, const void*, void*, DevBuf&, DevBuf&,
                                  DevBuf&, DevBuf&, hipStream_t);

// ---------------------------------------------------------------------------------------
// GMRES

using zc = std::complex<double>;

template <class S>
void Gmres<S>::ensure(size_t len, int nrhs, int restart) {
  if (len == len_ && nrhs <= nrhs_ && restart <= restart_) return;
  len_ = len;
  nrhs_ = std::max(nrhs, nrhs_);
  restart_ = std::max(restart, restart_);
  V_.ensure(size_t(restart_ + 1) * nrhs_ * len_ * sizeof(S));
  h1_.ensure(size_t(restart_ + 1) * nrhs_ * sizeof(double2));
  h2_.ensure(size_t(restart_ + 1) * nrhs_ * sizeof(double2));
  nrm_.ensure(size_t(2 * nrhs_) * sizeof(double));
  y_.ensure(size_t(restart_ + 1) * nrhs_ * sizeof(double2) + size_t(nrhs_) * sizeof(int));  // y, then valid counts
  r_.ensure(size_t(nrhs_) * len_ * sizeof(S));
}

namespace {
// Start of a cycle, fused with the normalisation of the first basis vector:
// w[r] /= beta_r with beta_r^2 = nr2[r]; workgroup (0, r) resets the rotations of rhs r with
// g = (beta_r, 0, ...) and, when nb2 is given, stores |b_r| = sqrt(nb2[r]).
template <class S, int P>
__global__ void k_gv_start(S* __restrict__ w, const double* __restrict__ nr2, size_t np, double2* st, int m,
                           const double* __restrict__ nb2, int* conv) {
  using C = ctype<S>;
  const int r = blockIdx.y;
  const double beta2 = nr2[r];
  const double beta = sqrt(beta2);
  if (conv && blockIdx.x == 0 && r == 0 && threadIdx.x == 0) {  // device-exit counters of this cycle
    conv[0] = 0;
    conv[1] = 0;
  }
  if (blockIdx.x == 0) {
    GvView v{st + r * gv_stride(m), m};
    for (int i = threadIdx.x; i <= m; i += blockDim.x) v.g()[i] = make_double2(i == 0 ? beta : 0.0, 0.0);
    if (threadIdx.x == 0) {
      v.flags() = make_double2(0.0, beta == 0.0 ? 1.0 : 0.0);
      if (nb2) v.bn() = make_double2(sqrt(nb2[r]), 0.0);
    }
  }
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= np) return;
  const double f = beta2 > 0.0 ? 1.0 / beta : 0.0;
  const size_t off = size_t(r) * np + e;
  auto wv = ldp<S, P>(w, off);
#pragma unroll
  for (int u = 0; u < P; ++u) wv.v[u] = StoreTraits<S>::st(C(f) * StoreTraits<S>::ld(wv.v[u]));
  stp<S, P>(w, off, wv);
}

// Arnoldi column j of rhs r, staged in a separate buffer (h1 [(m+1) nrhs], h2 [(m+1) nrhs] if
// two passes, |w|^2 [nrhs] as doubles) -> rotations; one wavefront per rhs.
__global__ __launch_bounds__(64) void k_gv_step(double2* st, int m, int nrhs, int j, const double2* col,
                                                int two_pass, double2* est, double tol, int* conv) {
  if (conv && conv[1]) return;  // every rhs converged
  const int r = blockIdx.x, lane = threadIdx.x;
  const double2* h1 = col;
  const double2* h2 = col + size_t(m + 1) * nrhs;
  const double* cn = reinterpret_cast<const double*>(col + size_t(2 * (m + 1)) * nrhs);
  double2 hl = make_double2(0.0, 0.0);
  if (lane <= j) {
    hl = h1[size_t(lane) * nrhs + r];
    if (two_pass) hl = cadd2(hl, h2[size_t(lane) * nrhs + r]);
  }
  gv_apply(GvView{st + r * gv_stride(m), m}, hl, make_double2(sqrt(cn[r]), 0.0), j, lane, est + r, tol, conv, nrhs,
           r);
}

// y = R^-1 g over the first min(n, valid) columns, zero beyond; y[i * nrhs + r].  One
// wavefront per rhs: R is staged in LDS, lane l holds y[l], each row is a wavefront sum.
__global__ __launch_bounds__(64) void k_gv_solve(const double2* st, int m, int nrhs, int n, double2* y,
                                                 int* nvalid) {
  __shared__ double2 Rs[64 * 64];
  const int r = blockIdx.x, lane = threadIdx.x;
  GvView v{const_cast<double2*>(st) + r * gv_stride(m), m};
  const int nv = min(n, int(v.flags().x));
  const double2* R = v.R();
  for (int t = lane; t < nv * nv; t += 64) {
    const int col = t / nv, row = t - col * nv;
    Rs[col * 64 + row] = R[size_t(col) * m + row];
  }
  const double2 gl = lane < nv ? v.g()[lane] : make_double2(0.0, 0.0);
  __syncthreads();
  double2 yl = make_double2(0.0, 0.0);
  for (int i = nv - 1; i >= 0; --i) {
    // s = g[i] - sum_{l > i} R[i][l] y[l]
    double2 p = lane > i && lane < nv ? cmul2(Rs[lane * 64 + i], yl) : make_double2(0.0, 0.0);
    p = warp_sum(p);
    const double2 gi = shfl2(gl, i);
    const double2 yi = cdiv2(cadd2(gi, cscale2(-1.0, p)), Rs[i * 64 + i]);
    if (lane == i) yl = yi;
  }
  if (lane < m) y[size_t(lane) * nrhs + r] = lane < nv ? yl : make_double2(0.0, 0.0);  // m <= 64
  if (lane == 0) nvalid[r] = nv;  // basis vectors beyond nv were never built for this rhs
}

}  // namespace

template <class S>
typename Gmres<S>::Result Gmres<S>::solve(LinOp& A, const void* b, void* x, bool x_zero, int nrhs, int m,
                                          int max_iter, double tol, hipStream_t st, int* conv, int first_check,
                                          Precond* M) {
  // FP64 keeps two Gram-Schmidt passes (parity with the FP64 reference to ~1e-12); lower
  // storage precisions use one pass with the Pythagorean norm, which halves the basis traffic
  const bool kCgs2 = cgs2_;
  // with a tolerance the host reads the convergence estimates once per kBatch Arnoldi steps
  // (steps past the converged one are discarded); without one (fixed step count) the cycle
  // runs without any host round trip: rotations and the small triangular solve are on the device
  constexpr int kBatch = 4;
  QMG_CHECK(m >= 1 && m <= 64, QMG_EINVAL, "GMRES restart length must be in [1, 64]");
  // device-side exit (conv given): one cycle of at most m steps, convergence tested by the
  // Givens kernels, every later kernel of the cycle returns at once; no host round trip
  const bool dev_exit = conv != nullptr;
  QMG_CHECK(!dev_exit || (x_zero && tol > 0 && max_iter <= m && m + 1 <= kMaxCoef && !M), QMG_EINVAL,
            "device-exit GMRES needs a zero guess, a tolerance, no preconditioner and one cycle of at most 63 steps");
  // flexible form: z_j = M v_j is kept (Z), the Arnoldi vector is A z_j and the solution is
  // updated with Z instead of V; each step is a preconditioner application, so the estimates
  // are read after every step
  const int* skip = dev_exit ? conv + 1 : nullptr;
  const size_t len = A.len();
  ensure(len, nrhs, m);
  S* V = V_.as<S>();
  const size_t vs = size_t(nrhs) * len;  // stride between basis vectors
  S* Z = nullptr;
  if (M) {
    Z_.ensure(size_t(m) * vs * sizeof(S));
    Z = Z_.as<S>();
  }
  // per-column device staging: h1 [(m+1) nrhs], h2 [(m+1) nrhs], |w|^2 [nrhs], estimates [nrhs]
  const size_t per_col = size_t(2 * (m + 1) + 2) * nrhs;
  const size_t est_off = size_t(2 * (m + 1) + 1) * nrhs;
  cols_.ensure(size_t(m) * per_col * sizeof(double2));
  gst_.ensure(size_t(nrhs) * gv_stride(m) * sizeof(double2));
  double2* colsd = cols_.as<double2>();
  double2* gst = gst_.as<double2>();
  double* nrm = nrm_.as<double>();
  double2* yd = y_.as<double2>();
  PinnedBuf& hb = hb_;
  hb.ensure(size_t(m) * per_col * sizeof(double2));
  double2* hcols = hb.as<double2>();

  Result res;
  res.rel_est.assign(nrhs, -1.0);  // unknown without a tolerance
  double* nb = nrm + nrhs;  // |b|^2 (only needed apart from |r0|^2 when x is not zero)
  if (!x_zero) Blas<S>::norm2(b, len, nrhs, nb, rw_, st);
  if (x_zero) Blas<S>::zero(x, vs, st);
  auto start = [&](bool first_cycle) {  // normalise V_0, reset the rotations (and |b|)
    const double* nb2 = first_cycle ? (x_zero ? nrm : nb) : nullptr;
    if (packable_vec<S>(len, V)) {
      constexpr int P = kPack<S>;
      {
        TimedLaunch tl_("krylov/givens", st, double(len) * nrhs * sizeof(S), 0.0);
        launch(k_gv_start<S, P>, dim3(unsigned((len / P + 255) / 256), nrhs), dim3(256), 0, st, V, nrm, len / P, gst,
               m, nb2, conv);
      }
    } else {
      {
        TimedLaunch tl_("krylov/givens", st, double(len) * nrhs * sizeof(S), 0.0);
        launch(k_gv_start<S, 1>, dim3(unsigned((len + 255) / 256), nrhs), dim3(256), 0, st, V, nrm, len, gst, m, nb2,
               conv);
      }
    }
    QMG_LAUNCH_CHECK();
  };

  int it = 0;
  bool first = true;
  bool all_conv = false;
  while (it < max_iter) {
    if (first && x_zero) {
      Blas<S>::copy(b, V, vs, st);
    } else {
      A.apply(x, V, nrhs, st);
      Blas<S>::axpby(1.0, b, -1.0, V, vs, st);
    }
    Blas<S>::norm2(V, len, nrhs, nrm, rw_, st);
    start(first);
    first = false;
    const int mc = std::min(m, max_iter - it);
    int jdone = 0, processed = 0, copied = 0;
    for (int j = 0; j < mc; ++j) {
      S* vj = V + size_t(j) * vs;
      S* vn = V + size_t(j + 1) * vs;
      double2* col = colsd + size_t(j) * per_col;
      double2* h1 = col;
      double2* h2 = col + size_t(m + 1) * nrhs;
      double* cn = reinterpret_cast<double*>(col + size_t(2 * (m + 1)) * nrhs);
      if (M) {
        S* zj = Z + size_t(j) * vs;
        M->apply(vj, zj, nrhs, st);
        A.apply(zj, vn, nrhs, st, skip);
      } else {
        A.apply(vj, vn, nrhs, st, skip);
      }
      bool fused = false;
      if (kCgs2) {
        // CGS2: h1 = V^dag w ; w -= V h1 and h2 = V^dag w ; w -= V h2 and |w|^2 ; w /= |w|
        Blas<S>::cgs2_step(V, vs, j + 1, vn, len, nrhs, h1, h2, cn, rw_, st, skip);
      } else {
        // one classical Gram-Schmidt pass with the norm from Pythagoras; scaling and the
        // Givens step fused into its last kernel
        fused = Blas<S>::cgs1_step(V, vs, j + 1, vn, len, nrhs, h1, cn, rw_, st, gst, m, col + est_off, tol, conv);
      }
      if (!fused) {
        {
          TimedLaunch tl_("krylov/givens", st, 0.0, 0.0);
          launch(k_gv_step, dim3(nrhs), dim3(64), 0, st, gst, m, nrhs, j, col, kCgs2 ? 1 : 0, col + est_off, tol,
                 conv);
        }
        QMG_LAUNCH_CHECK();
      }
      jdone = j + 1;
      // read points: every kBatch steps, or (with a hint, in the first cycle) at first_check and
      // every second step after it
      const bool read_now = M ? true
                              : first_check > 0 && it == 0
                                  ? (j + 1 >= first_check && (j + 1 - first_check) % 2 == 0)
                                  : (j + 1) % kBatch == 0;
      if (!dev_exit && tol > 0 && (read_now || j == mc - 1)) {
        // the columns since the last read travel to the host in one copy
        QMG_HIP(hipMemcpyAsync(hcols + size_t(copied) * per_col, colsd + size_t(copied) * per_col,
                               size_t(j + 1 - copied) * per_col * sizeof(double2), hipMemcpyDeviceToHost, st));
        copied = j + 1;
        QMG_HIP(hipStreamSynchronize(st));
        for (; processed <= j; ++processed) {
          const double2* e = hcols + size_t(processed) * per_col + est_off;
          bool before = true, after = true;
          for (int r = 0; r < nrhs; ++r) {
            QMG_CHECK(std::isfinite(e[r].x) && std::isfinite(e[r].y), QMG_ENONFINITE,
                      "GMRES: non-finite Hessenberg entry");
            res.rel_est[r] = e[r].y;
            if (!(e[r].x <= tol)) before = false;
            if (!(e[r].y <= tol)) after = false;
          }
          if (processed == 0 && before) {  // already converged at the start of the cycle
            jdone = 0;
            all_conv = true;
            break;
          }
          if (after) {
            jdone = processed + 1;
            all_conv = true;
            break;
          }
        }
        if (all_conv) break;
      }
    }
    it += jdone;
    if (jdone > 0) {
      // x += V y with y = R^-1 g over the accepted columns (zero beyond each rhs's last valid one)
      int* nvd = reinterpret_cast<int*>(yd + size_t(m + 1) * nrhs);
      {
        TimedLaunch tl_("krylov/givens", st, 0.0, 0.0);
        launch(k_gv_solve, dim3(nrhs), dim3(64), 0, st, gst, m, nrhs, jdone, yd, nvd);
      }
      QMG_LAUNCH_CHECK();
      Blas<S>::axpy_multi(M ? Z : V, vs, jdone, yd, 1.0, x, len, nrhs, st, nullptr, nvd);
    }
    if (dev_exit || all_conv || jdone == 0) break;
  }
  res.iters = dev_exit ? -1 : it;  // device-exit steps are counted in conv[2]
  res.converged = (tol <= 0) || all_conv || dev_exit;
  return res;
}

// ---------------------------------------------------------------------------------------
// Defect correction between the FP64 outer residual and the FP32 inner solve: each step is one
// pass over its vectors instead of two or three (subtraction then norm; scale then conversion;
// conversion, scale and update), with the same roundings as the separate passes.
namespace {

// r = b - r with the partial sums of |r|^2 over the slices and in the order of k_norm_partial
// (FP64 packs are single complex numbers), so the norms equal those of a separate norm pass
__global__ __launch_bounds__(RB) void k_dc_residual(const double2* __restrict__ b, double2* __restrict__ r,
                                                    size_t len, int nblk, double2* __restrict__ partial) {
  const int blk = blockIdx.x, c = blockIdx.y;
  double2 acc = make_double2(0.0, 0.0);
  for (size_t e = size_t(blk) * RB + threadIdx.x; e < len; e += size_t(nblk) * RB) {
    const size_t i = size_t(c) * len + e;
    const double2 bv = b[i], rv = r[i];
    const double ar = bv.x - rv.x, ai = bv.y - rv.y;
    r[i] = make_double2(ar, ai);
    acc.x += ar * ar + ai * ai;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[size_t(c) * nblk + blk] = acc;
}

// out = FP32(r / sqrt(n2)) per column (zero for a zero norm): the scaled value is rounded to
// FP64 first, as a scale pass followed by a conversion would
__global__ void k_dc_normalise(const double2* __restrict__ r, const double* __restrict__ n2, float2* __restrict__ out,
                               size_t len) {
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (e >= len) return;
  const double v = n2[c];
  const double f = (v > 0.0) ? 1.0 / sqrt(v) : 0.0;
  const size_t i = size_t(c) * len + e;
  const double2 x = r[i];
  const double xr = f * x.x, xi = f * x.y;
  out[i] = make_float2(float(xr), float(xi));
}

// x += sqrt(n2) e per column, e in FP32: the product is rounded before the sum (no fused
// multiply-add), as a scale pass followed by an update pass would
__global__ void k_dc_accumulate(const float2* __restrict__ ev, const double* __restrict__ n2, double2* __restrict__ x,
                                size_t len) {
#pragma clang fp contract(off)
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (e >= len) return;
  const double f = sqrt(n2[c]);
  const size_t i = size_t(c) * len + e;
  const float2 u = ev[i];
  const double tr = f * double(u.x), ti = f * double(u.y);
  double2 xv = x[i];
  xv.x = tr + xv.x;
  xv.y = ti + xv.y;
  x[i] = xv;
}

}  // namespace

void dc_residual(const void* b64, void* r64, size_t len, int nrhs, double* n2, RedWork& rw, hipStream_t st) {
  const int nblk = pick_nblk(len, nrhs);
  rw.ensure(size_t(nblk) * nrhs, 0);
  {
    TimedLaunch tl_("blas/dc_residual", st, 3.0 * double(len) * nrhs * sizeof(double2), 0.0);
    launch(k_dc_residual, dim3(nblk, nrhs), dim3(RB), 0, st, (const double2*)b64, (double2*)r64, len, nblk,
           rw.partial.as<double2>());
  }
  QMG_LAUNCH_CHECK();
  {
    TimedLaunch tl_("blas/finalize", st, double(nblk) * nrhs * sizeof(double2), 0.0);
    launch(k_finalize1, dim3(nrhs), dim3(RB), 0, st, rw.partial.as<double2>(), nblk, n2, nullptr);
  }
  QMG_LAUNCH_CHECK();
}

void dc_normalise(const void* r64, const double* n2, void* rin, size_t len, int nrhs, hipStream_t st) {
  {
    TimedLaunch tl_("blas/dc_normalise", st, double(len) * nrhs * (sizeof(double2) + sizeof(float2)), 0.0);
    launch(k_dc_normalise, dim3(nb256(len), nrhs), dim3(256), 0, st, (const double2*)r64, n2, (float2*)rin, len);
  }
  QMG_LAUNCH_CHECK();
}

void dc_accumulate(const void* ein, const double* n2, void* x64, size_t len, int nrhs, hipStream_t st) {
  {
    TimedLaunch tl_("blas/dc_accumulate", st, double(len) * nrhs * (sizeof(float2) + 2.0 * sizeof(double2)), 0.0);
    launch(k_dc_accumulate, dim3(nb256(len), nrhs), dim3(256), 0, st, (const float2*)ein, n2, (double2*)x64, len);
  }
  QMG_LAUNCH_CHECK();
}

template class Gmres<double2>;
template class Gmres<float2>;
template class Gmres<cbf16>;
template class Gmres<chalf>;

}  // namespace qmg
