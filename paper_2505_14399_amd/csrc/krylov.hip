// BLAS-1 kernels (deterministic double-accumulated reductions) and the multi-RHS Krylov
// solvers used by the smoother, the coarse solve and the outer solve.
#include <cmath>
#include <complex>
#include <cstring>
#include <type_traits>

#include "krylov.hpp"

namespace qmg {

namespace {

constexpr int RB = 256;  // threads per reduction workgroup (4 wavefronts)


__device__ inline double2 warp_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_down(v.x, off, 64);
    v.y += __shfl_down(v.y, off, 64);
  }
  return v;
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

template <class S>
__global__ __launch_bounds__(RB) void k_dot_partial(const S* __restrict__ X, size_t xstride, const S* __restrict__ w,
                                                    size_t len, int nrhs, int nblk, double2* __restrict__ partial) {
  const int b = blockIdx.x, r = blockIdx.y, i = blockIdx.z;
  const S* xi = X + i * xstride + size_t(r) * len;
  const S* wr = w + size_t(r) * len;
  double2 acc = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < len; e += size_t(nblk) * RB) {
    auto a = StoreTraits<S>::ld(xi[e]);
    auto c = StoreTraits<S>::ld(wr[e]);
    const double ar = a.re, ai = a.im, cr = c.re, ci = c.im;
    acc.x += ar * cr + ai * ci;
    acc.y += ar * ci - ai * cr;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[(size_t(i) * nrhs + r) * nblk + b] = acc;
}

template <class S>
__global__ __launch_bounds__(RB) void k_norm_partial(const S* __restrict__ w, size_t len, int nblk,
                                                     double2* __restrict__ partial) {
  const int b = blockIdx.x, r = blockIdx.y;
  const S* wr = w + size_t(r) * len;
  double2 acc = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < len; e += size_t(nblk) * RB) {
    auto a = StoreTraits<S>::ld(wr[e]);
    const double ar = a.re, ai = a.im;
    acc.x += ar * ar + ai * ai;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[size_t(r) * nblk + b] = acc;
}

// out[c] = sum over b < nblk of partial[c * nblk + b], fixed order per thread + tree
__global__ __launch_bounds__(RB) void k_finalize2(const double2* __restrict__ partial, int nblk,
                                                  double2* __restrict__ out) {
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
                                                  double* __restrict__ out) {
  const int c = blockIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (int b = threadIdx.x; b < nblk; b += RB) acc.x += partial[size_t(c) * nblk + b].x;
  acc = block_sum(acc);
  if (threadIdx.x == 0) out[c] = acc.x;
}

int pick_nblk(size_t len, int ncols) {
  size_t nb = (len + RB * 4 - 1) / (RB * 4);
  size_t cap = std::max<size_t>(1, 4096 / std::max(1, ncols));
  nb = std::min(nb, cap);
  return int(std::max<size_t>(nb, 1));
}

template <class S>
__global__ void k_zero(S* x, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = StoreTraits<S>::st({ctype<S>(0), ctype<S>(0)});
}

template <class S>
__global__ void k_copy(const S* __restrict__ x, S* __restrict__ y, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

template <class S>
__global__ void k_axpby(double a, const S* __restrict__ x, double b, S* __restrict__ y, size_t n) {
  using C = ctype<S>;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    auto xv = StoreTraits<S>::ld(x[i]);
    auto yv = StoreTraits<S>::ld(y[i]);
    y[i] = StoreTraits<S>::st(C(a) * xv + C(b) * yv);
  }
}

template <class S>
__global__ void k_axpy_multi(const S* __restrict__ X, size_t xstride, int m, const double2* __restrict__ c,
                             double sgn, S* __restrict__ w, size_t len, int nrhs) {
  using C = ctype<S>;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= len) return;
  const size_t off = size_t(r) * len + e;
  auto acc = StoreTraits<S>::ld(w[off]);
  for (int i = 0; i < m; ++i) {
    const double2 ci = c[size_t(i) * nrhs + r];
    const cplx<C> cc = {C(sgn * ci.x), C(sgn * ci.y)};
    acc += cc * StoreTraits<S>::ld(X[i * xstride + off]);
  }
  w[off] = StoreTraits<S>::st(acc);
}

template <class S>
__global__ void k_scale_dev(S* __restrict__ w, const double* __restrict__ n2, int mode, size_t len) {
  using C = ctype<S>;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= len) return;
  const double v = n2[r];
  double f;
  if (mode == 0) f = (v > 0.0) ? 1.0 / sqrt(v) : 0.0;
  else if (mode == 1) f = sqrt(v);
  else f = v;
  const size_t off = size_t(r) * len + e;
  w[off] = StoreTraits<S>::st(C(f) * StoreTraits<S>::ld(w[off]));
}

template <class S>
__global__ void k_scale_cdev(S* __restrict__ w, const double2* __restrict__ c, double sgn, size_t len) {
  using C = ctype<S>;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= len) return;
  const cplx<C> cc = {C(sgn * c[r].x), C(sgn * c[r].y)};
  const size_t off = size_t(r) * len + e;
  w[off] = StoreTraits<S>::st(cc * StoreTraits<S>::ld(w[off]));
}

template <class S>
__global__ void k_caxpy_dev(const double2* __restrict__ c, double sgn, const S* __restrict__ y, S* __restrict__ x,
                            size_t len) {
  using C = ctype<S>;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= len) return;
  const cplx<C> cc = {C(sgn * c[r].x), C(sgn * c[r].y)};
  const size_t off = size_t(r) * len + e;
  x[off] = StoreTraits<S>::st(StoreTraits<S>::ld(x[off]) + cc * StoreTraits<S>::ld(y[off]));
}

inline unsigned nb256(size_t n) { return unsigned((n + 255) / 256); }

// ---------------------------------------------------------------------------------------
// Fused multi-vector kernels for the Arnoldi/GCR orthogonalisation: each reads the target
// vector w once for up to MG basis vectors (grid.z = group of MG vectors).
constexpr int MG = 8;

template <class S>
__device__ inline void store_partials(double2 (&acc)[MG], int mi, double2* partial, int i0, int nrhs, int r, int b,
                                      int nblk) {
  __shared__ double2 red[MG][RB / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < MG; ++i) {
    const double2 v = warp_sum(acc[i]);
    if (lane == 0) red[i][wid] = v;
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

// partial <X_i, w> for i in [i0, i0 + MG) of this z-group
template <class S>
__global__ __launch_bounds__(RB) void k_mdot(const S* __restrict__ X, size_t xstride, int m, const S* __restrict__ w,
                                             size_t len, int nrhs, int nblk, double2* __restrict__ partial) {
  const int b = blockIdx.x, r = blockIdx.y, i0 = blockIdx.z * MG;
  const int mi = min(MG, m - i0);
  const S* wr = w + size_t(r) * len;
  double2 acc[MG];
#pragma unroll
  for (int i = 0; i < MG; ++i) acc[i] = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < len; e += size_t(nblk) * RB) {
    const auto c = StoreTraits<S>::ld(wr[e]);
    const double cr = c.re, ci = c.im;
#pragma unroll
    for (int i = 0; i < MG; ++i) {
      if (i < mi) {
        const auto a = StoreTraits<S>::ld(X[(i0 + i) * xstride + size_t(r) * len + e]);
        const double ar = a.re, ai = a.im;
        acc[i].x += ar * cr + ai * ci;
        acc[i].y += ar * ci - ai * cr;
      }
    }
  }
  store_partials<S>(acc, mi, partial, i0, nrhs, r, b, nblk);
}

// w <- w + sgn * sum_i c_i X_i (all m vectors), then partial <X_i, w> (grid.z groups) or
// partial |w|^2 (mode 1, grid.z = 1).  Each z-group recomputes the same w update; only z = 0
// stores it.
template <class S, int MODE>
__global__ __launch_bounds__(RB) void k_axpy_then(const S* __restrict__ X, size_t xstride, int m,
                                                  const double2* __restrict__ c, double sgn, S* __restrict__ w,
                                                  size_t len, int nrhs, int nblk, double2* __restrict__ partial) {
  using C = ctype<S>;
  const int b = blockIdx.x, r = blockIdx.y, i0 = blockIdx.z * MG;
  const int mi = MODE == 0 ? min(MG, m - i0) : 1;
  S* wr = w + size_t(r) * len;
  double2 acc[MG];
#pragma unroll
  for (int i = 0; i < MG; ++i) acc[i] = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < len; e += size_t(nblk) * RB) {
    auto v = StoreTraits<S>::ld(wr[e]);
    for (int i = 0; i < m; ++i) {
      const double2 ci = c[size_t(i) * nrhs + r];
      const cplx<C> cc = {C(sgn * ci.x), C(sgn * ci.y)};
      v += cc * StoreTraits<S>::ld(X[i * xstride + size_t(r) * len + e]);
    }
    const S vs = StoreTraits<S>::st(v);
    if (blockIdx.z == 0) wr[e] = vs;
    const auto vv = StoreTraits<S>::ld(vs);  // the stored (rounded) value
    const double cr = vv.re, cim = vv.im;
    if (MODE == 0) {
#pragma unroll
      for (int i = 0; i < MG; ++i) {
        if (i < mi) {
          const auto a = StoreTraits<S>::ld(X[(i0 + i) * xstride + size_t(r) * len + e]);
          const double ar = a.re, ai = a.im;
          acc[i].x += ar * cr + ai * cim;
          acc[i].y += ar * cim - ai * cr;
        }
      }
    } else {
      acc[0].x += cr * cr + cim * cim;
    }
  }
  store_partials<S>(acc, mi, partial, i0, nrhs, r, b, nblk);
}

// partial <X_i, w> (grid.z groups of MG) and, in group 0, partial |w|^2 stored at slot m
template <class S>
__global__ __launch_bounds__(RB) void k_mdot_norm(const S* __restrict__ X, size_t xstride, int m,
                                                  const S* __restrict__ w, size_t len, int nrhs, int nblk,
                                                  double2* __restrict__ partial) {
  const int b = blockIdx.x, r = blockIdx.y, i0 = blockIdx.z * MG;
  const int mi = min(MG, m - i0);
  const S* wr = w + size_t(r) * len;
  double2 acc[MG];
  double nn = 0.0;
#pragma unroll
  for (int i = 0; i < MG; ++i) acc[i] = make_double2(0.0, 0.0);
  for (size_t e = size_t(b) * RB + threadIdx.x; e < len; e += size_t(nblk) * RB) {
    const auto c = StoreTraits<S>::ld(wr[e]);
    const double cr = c.re, ci = c.im;
    nn += cr * cr + ci * ci;
#pragma unroll
    for (int i = 0; i < MG; ++i) {
      if (i < mi) {
        const auto a = StoreTraits<S>::ld(X[(i0 + i) * xstride + size_t(r) * len + e]);
        const double ar = a.re, ai = a.im;
        acc[i].x += ar * cr + ai * ci;
        acc[i].y += ar * ci - ai * cr;
      }
    }
  }
  store_partials<S>(acc, mi, partial, i0, nrhs, r, b, nblk);
  if (blockIdx.z == 0) {
    double2 t = block_sum(make_double2(nn, 0.0));
    if (threadIdx.x == 0) partial[(size_t(m) * nrhs + r) * nblk + b] = t;
  }
}

// w <- (w - sum_i c_i X_i) / beta with beta^2 = |w|^2 - sum_i |c_i|^2 (Pythagoras, c = X^dag w
// for orthonormal X); beta^2 is also written to out_n2 (block 0).  n2 = |w|^2 before the update.
template <class S>
__global__ __launch_bounds__(RB) void k_axpy_scale(const S* __restrict__ X, size_t xstride, int m,
                                                   const double2* __restrict__ c, const double2* __restrict__ n2,
                                                   S* __restrict__ w, size_t len, int nrhs, double* __restrict__ out_n2) {
  using C = ctype<S>;
  const int r = blockIdx.y;
  double b2 = n2[r].x;
  for (int i = 0; i < m; ++i) {
    const double2 ci = c[size_t(i) * nrhs + r];
    b2 -= ci.x * ci.x + ci.y * ci.y;
  }
  b2 = fmax(b2, 0.0);
  const double inv = b2 > 0.0 ? 1.0 / sqrt(b2) : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) out_n2[r] = b2;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= len) return;
  S* wr = w + size_t(r) * len;
  auto v = StoreTraits<S>::ld(wr[e]);
  for (int i = 0; i < m; ++i) {
    const double2 ci = c[size_t(i) * nrhs + r];
    const cplx<C> cc = {C(-ci.x), C(-ci.y)};
    v += cc * StoreTraits<S>::ld(X[i * xstride + size_t(r) * len + e]);
  }
  wr[e] = StoreTraits<S>::st(C(inv) * v);
}

}  // namespace

// ---------------------------------------------------------------------------------------
template <class S>
void Blas<S>::zero(void* x, size_t n, hipStream_t st) {
  if (!n) return;
  k_zero<S><<<nb256(n), 256, 0, st>>>((S*)x, n);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::copy(const void* x, void* y, size_t n, hipStream_t st) {
  if (!n) return;
  k_copy<S><<<nb256(n), 256, 0, st>>>((const S*)x, (S*)y, n);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::axpby(double a, const void* x, double b, void* y, size_t n, hipStream_t st) {
  if (!n) return;
  k_axpby<S><<<nb256(n), 256, 0, st>>>(a, (const S*)x, b, (S*)y, n);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::dot_multi(const void* X, size_t xstride, int m, const void* w, size_t len, int nrhs, double2* out,
                        RedWork& rw, hipStream_t st) {
  if (m <= 0) return;
  const int nblk = pick_nblk(len, m * nrhs);
  rw.ensure(size_t(nblk) * m * nrhs, 0);
  k_dot_partial<S><<<dim3(nblk, nrhs, m), RB, 0, st>>>((const S*)X, xstride, (const S*)w, len, nrhs, nblk,
                                                        rw.partial.as<double2>());
  QMG_LAUNCH_CHECK();
  k_finalize2<<<m * nrhs, RB, 0, st>>>(rw.partial.as<double2>(), nblk, out);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::norm2(const void* w, size_t len, int nrhs, double* out, RedWork& rw, hipStream_t st) {
  const int nblk = pick_nblk(len, nrhs);
  rw.ensure(size_t(nblk) * nrhs, 0);
  k_norm_partial<S><<<dim3(nblk, nrhs), RB, 0, st>>>((const S*)w, len, nblk, rw.partial.as<double2>());
  QMG_LAUNCH_CHECK();
  k_finalize1<<<nrhs, RB, 0, st>>>(rw.partial.as<double2>(), nblk, out);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::axpy_multi(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w, size_t len,
                         int nrhs, hipStream_t st) {
  if (m <= 0) return;
  k_axpy_multi<S><<<dim3(nb256(len), nrhs), 256, 0, st>>>((const S*)X, xstride, m, c, sgn, (S*)w, len, nrhs);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::scale_dev(void* w, const double* n2, int mode, size_t len, int nrhs, hipStream_t st) {
  k_scale_dev<S><<<dim3(nb256(len), nrhs), 256, 0, st>>>((S*)w, n2, mode, len);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::scale_cdev(void* w, const double2* c, double sgn, size_t len, int nrhs, hipStream_t st) {
  k_scale_cdev<S><<<dim3(nb256(len), nrhs), 256, 0, st>>>((S*)w, c, sgn, len);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::caxpy_dev(const double2* c, double sgn, const void* y, void* x, size_t len, int nrhs,
                        hipStream_t st) {
  k_caxpy_dev<S><<<dim3(nb256(len), nrhs), 256, 0, st>>>(c, sgn, (const S*)y, (S*)x, len);
  QMG_LAUNCH_CHECK();
}

template <class S>
void Blas<S>::mdot(const void* X, size_t xstride, int m, const void* w, size_t len, int nrhs, double2* out,
                   RedWork& rw, hipStream_t st) {
  if (m <= 0) return;
  const int ng = (m + MG - 1) / MG;
  const int nblk = pick_nblk(len, ng * nrhs);
  rw.ensure(size_t(nblk) * m * nrhs, 0);
  k_mdot<S><<<dim3(nblk, nrhs, ng), RB, 0, st>>>((const S*)X, xstride, m, (const S*)w, len, nrhs, nblk,
                                                 rw.partial.as<double2>());
  QMG_LAUNCH_CHECK();
  k_finalize2<<<m * nrhs, RB, 0, st>>>(rw.partial.as<double2>(), nblk, out);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::axpy_mdot(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w, size_t len,
                        int nrhs, double2* out, RedWork& rw, hipStream_t st) {
  if (m <= 0) return;
  // the update must be complete before other z-groups read w: one group only when m > MG
  if (m > MG) {
    axpy_multi(X, xstride, m, c, sgn, w, len, nrhs, st);
    mdot(X, xstride, m, w, len, nrhs, out, rw, st);
    return;
  }
  const int nblk = pick_nblk(len, nrhs);
  rw.ensure(size_t(nblk) * m * nrhs, 0);
  k_axpy_then<S, 0><<<dim3(nblk, nrhs, 1), RB, 0, st>>>((const S*)X, xstride, m, c, sgn, (S*)w, len, nrhs, nblk,
                                                         rw.partial.as<double2>());
  QMG_LAUNCH_CHECK();
  k_finalize2<<<m * nrhs, RB, 0, st>>>(rw.partial.as<double2>(), nblk, out);
  QMG_LAUNCH_CHECK();
}
template <class S>
void Blas<S>::axpy_norm(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w, size_t len,
                        int nrhs, double* out, RedWork& rw, hipStream_t st) {
  const int nblk = pick_nblk(len, nrhs);
  rw.ensure(size_t(nblk) * nrhs, 0);
  k_axpy_then<S, 1><<<dim3(nblk, nrhs, 1), RB, 0, st>>>((const S*)X, xstride, m, c, sgn, (S*)w, len, nrhs, nblk,
                                                         rw.partial.as<double2>());
  QMG_LAUNCH_CHECK();
  k_finalize1<<<nrhs, RB, 0, st>>>(rw.partial.as<double2>(), nblk, out);
  QMG_LAUNCH_CHECK();
}

template <class S>
void Blas<S>::cgs1_step(const void* X, size_t xstride, int m, void* w, size_t len, int nrhs, double2* h, double* n2,
                        RedWork& rw, hipStream_t st) {
  const int ng = (m + MG - 1) / MG;
  const int nblk = pick_nblk(len, ng * nrhs);
  rw.ensure(size_t(nblk) * (m + 1) * nrhs, size_t(nrhs));
  k_mdot_norm<S><<<dim3(nblk, nrhs, ng), RB, 0, st>>>((const S*)X, xstride, m, (const S*)w, len, nrhs, nblk,
                                                      rw.partial.as<double2>());
  QMG_LAUNCH_CHECK();
  k_finalize2<<<m * nrhs, RB, 0, st>>>(rw.partial.as<double2>(), nblk, h);
  QMG_LAUNCH_CHECK();
  double2* wn = rw.result.as<double2>();
  k_finalize2<<<nrhs, RB, 0, st>>>(rw.partial.as<double2>() + size_t(m) * nrhs * nblk, nblk, wn);
  QMG_LAUNCH_CHECK();
  k_axpy_scale<S><<<dim3(nb256(len), nrhs), 256, 0, st>>>((const S*)X, xstride, m, h, wn, (S*)w, len, nrhs, n2);
  QMG_LAUNCH_CHECK();
}

template struct Blas<double2>;
template struct Blas<float2>;
template struct Blas<cbf16>;
template struct Blas<chalf>;

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
  nrm_.ensure(size_t(nrhs_) * sizeof(double));
  y_.ensure(size_t(restart_ + 1) * nrhs_ * sizeof(double2));
  r_.ensure(size_t(nrhs_) * len_ * sizeof(S));
}

namespace {
// one Givens step on column j of a Hessenberg matrix (column-major h[0..j+1])
struct GivensState {
  std::vector<double> cs;
  std::vector<zc> sn, g, R;  // R: upper triangle, column-major (m x m)
  int m = 0, valid = 0;
  bool stopped = false;
  void init(int m_, double beta) {
    m = m_;
    cs.assign(m, 0.0);
    sn.assign(m, 0.0);
    g.assign(m + 1, 0.0);
    R.assign(size_t(m) * m, 0.0);
    g[0] = beta;
    valid = 0;
    stopped = (beta == 0.0);
  }
  // h has j+2 entries; returns |g[j+1]|
  double step(int j, zc* h) {
    if (stopped) return std::abs(g[valid]);
    for (int i = 0; i < j; ++i) {
      zc t = cs[i] * h[i] + sn[i] * h[i + 1];
      h[i + 1] = -std::conj(sn[i]) * h[i] + cs[i] * h[i + 1];
      h[i] = t;
    }
    const zc a = h[j], b = h[j + 1];
    const double den = std::sqrt(std::norm(a) + std::norm(b));
    if (den == 0.0 || !std::isfinite(den)) {  // singular column: stop this cycle before it
      stopped = true;
      return std::abs(g[valid]);
    }
    if (std::abs(a) == 0.0) {
      cs[j] = 0.0;
      sn[j] = std::conj(b) / std::abs(b);
    } else {
      cs[j] = std::abs(a) / den;
      sn[j] = (a / std::abs(a)) * std::conj(b) / den;
    }
    h[j] = cs[j] * a + sn[j] * b;
    for (int i = 0; i <= j; ++i) R[size_t(j) * m + i] = h[i];
    g[j + 1] = -std::conj(sn[j]) * g[j];
    g[j] = cs[j] * g[j];
    valid = j + 1;
    if (std::abs(b) == 0.0) stopped = true;  // exact (lucky) breakdown
    return std::abs(g[j + 1]);
  }
  void solve(std::vector<zc>& y) const {
    y.assign(m, 0.0);
    for (int i = valid - 1; i >= 0; --i) {
      zc s = g[i];
      for (int l = i + 1; l < valid; ++l) s -= R[size_t(l) * m + i] * y[l];
      y[i] = s / R[size_t(i) * m + i];
    }
  }
};
}  // namespace

template <class S>
typename Gmres<S>::Result Gmres<S>::solve(LinOp& A, const void* b, void* x, bool x_zero, int nrhs, int m,
                                          int max_iter, double tol, hipStream_t st) {
  // FP64 keeps two Gram-Schmidt passes (parity with the FP64 reference to ~1e-12); lower
  // storage precisions use one pass with the Pythagorean norm, which halves the basis traffic
  constexpr bool kCgs2 = std::is_same<S, double2>::value;
  // with a tolerance, Arnoldi steps are issued in batches of kBatch before the host reads the
  // Hessenberg columns; steps past the converged one are discarded
  constexpr int kBatch = 4;
  const size_t len = A.len();
  ensure(len, nrhs, m);
  S* V = V_.as<S>();
  const size_t vs = size_t(nrhs) * len;  // stride between basis vectors
  // per-column device staging: h1 [(m+1) nrhs], h2 [(m+1) nrhs], nrm [nrhs] (as double2 slots)
  const size_t per_col = size_t(2 * (m + 1) + 1) * nrhs;
  cols_.ensure(size_t(m) * per_col * sizeof(double2));
  double2* colsd = cols_.as<double2>();
  double* nrm = nrm_.as<double>();
  PinnedBuf& hb = hb_;
  hb.ensure((size_t(m) * per_col + 2 * nrhs + size_t(m + 1) * nrhs) * sizeof(double2));
  double2* hcols = hb.as<double2>();
  double* hnrm0 = reinterpret_cast<double*>(hcols + size_t(m) * per_col);

  Result res;
  res.rel_est.assign(nrhs, 0.0);
  std::vector<double> bn(nrhs, 0.0);
  Blas<S>::norm2(b, len, nrhs, nrm, rw_, st);
  QMG_HIP(hipMemcpyAsync(hnrm0, nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  for (int r = 0; r < nrhs; ++r) bn[r] = std::sqrt(hnrm0[r]);
  if (x_zero) Blas<S>::zero(x, vs, st);

  int it = 0;
  bool first = true;
  std::vector<GivensState> gs(nrhs);
  std::vector<zc> y, hcol(m + 2);
  std::vector<double2> yh(size_t(m) * nrhs);
  bool all_conv = false;
  auto process = [&](int j) {  // host Givens step on column j; true if every rhs converged
    const double2* snap = hcols + size_t(j) * per_col;
    bool conv = true;
    for (int r = 0; r < nrhs; ++r) {
      for (int i = 0; i <= j; ++i) {
        const double2 a = snap[size_t(i) * nrhs + r];
        double2 c = make_double2(0.0, 0.0);
        if (kCgs2) c = snap[size_t(m + 1 + i) * nrhs + r];
        hcol[i] = zc(a.x + c.x, a.y + c.y);
      }
      hcol[j + 1] = std::sqrt(reinterpret_cast<const double*>(snap + size_t(2 * (m + 1)) * nrhs)[r]);
      const double est = gs[r].step(j, hcol.data());
      QMG_CHECK(std::isfinite(est), QMG_ENONFINITE, "GMRES: non-finite Hessenberg entry");
      res.rel_est[r] = bn[r] > 0 ? est / bn[r] : 0.0;
      if (!(tol > 0 && est <= tol * bn[r])) conv = false;
    }
    return conv;
  };
  while (it < max_iter) {
    if (first && x_zero) {
      Blas<S>::copy(b, V, vs, st);
    } else {
      A.apply(x, V, nrhs, st);
      Blas<S>::axpby(1.0, b, -1.0, V, vs, st);
    }
    first = false;
    Blas<S>::norm2(V, len, nrhs, nrm, rw_, st);
    QMG_HIP(hipMemcpyAsync(hnrm0, nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    QMG_HIP(hipStreamSynchronize(st));
    all_conv = true;
    for (int r = 0; r < nrhs; ++r) {
      const double beta = std::sqrt(hnrm0[r]);
      QMG_CHECK(std::isfinite(beta), QMG_ENONFINITE, "GMRES: non-finite residual norm");
      res.rel_est[r] = bn[r] > 0 ? beta / bn[r] : 0.0;
      if (!(tol > 0 && beta <= tol * bn[r]) && beta > 0) all_conv = false;
    }
    if (all_conv) break;
    Blas<S>::scale_dev(V, nrm, 0, len, nrhs, st);
    const int mc = std::min(m, max_iter - it);
    for (int r = 0; r < nrhs; ++r) gs[r].init(mc, std::sqrt(hnrm0[r]));
    int jdone = 0, processed = 0;
    for (int j = 0; j < mc; ++j) {
      S* vj = V + size_t(j) * vs;
      S* vn = V + size_t(j + 1) * vs;
      double2* col = colsd + size_t(j) * per_col;
      double2* h1 = col;
      double2* h2 = col + size_t(m + 1) * nrhs;
      double* cn = reinterpret_cast<double*>(col + size_t(2 * (m + 1)) * nrhs);
      A.apply(vj, vn, nrhs, st);
      if (kCgs2) {
        // CGS2: h1 = V^dag w ; w -= V h1 and h2 = V^dag w ; w -= V h2 and |w|^2 ; w /= |w|
        Blas<S>::mdot(V, vs, j + 1, vn, len, nrhs, h1, rw_, st);
        Blas<S>::axpy_mdot(V, vs, j + 1, h1, -1.0, vn, len, nrhs, h2, rw_, st);
        Blas<S>::axpy_norm(V, vs, j + 1, h2, -1.0, vn, len, nrhs, cn, rw_, st);
        Blas<S>::scale_dev(vn, cn, 0, len, nrhs, st);
      } else {
        // one classical Gram-Schmidt pass with the norm from Pythagoras, scaling fused
        Blas<S>::cgs1_step(V, vs, j + 1, vn, len, nrhs, h1, cn, rw_, st);
      }
      QMG_HIP(hipMemcpyAsync(hcols + size_t(j) * per_col, col, per_col * sizeof(double2), hipMemcpyDeviceToHost,
                             st));
      jdone = j + 1;
      if (tol > 0 && ((j + 1) % kBatch == 0 || j == mc - 1)) {
        QMG_HIP(hipStreamSynchronize(st));
        for (; processed <= j; ++processed) {
          if (process(processed)) {
            jdone = processed + 1;
            all_conv = true;
            break;
          }
        }
        if (all_conv) break;
      }
    }
    if (tol <= 0) {
      QMG_HIP(hipStreamSynchronize(st));
      for (int j = 0; j < jdone; ++j) process(j);
    }
    it += jdone;
    // x += sum_i y_i V_i
    for (int r = 0; r < nrhs; ++r) {
      gs[r].solve(y);
      for (int i = 0; i < jdone; ++i) yh[size_t(i) * nrhs + r] = make_double2(y[i].real(), y[i].imag());
    }
    double2* yd = y_.as<double2>();
    QMG_HIP(hipMemcpyAsync(yd, yh.data(), size_t(jdone) * nrhs * sizeof(double2), hipMemcpyHostToDevice, st));
    Blas<S>::axpy_multi(V, vs, jdone, yd, 1.0, x, len, nrhs, st);
    // the host vector yh must outlive the async copy
    QMG_HIP(hipStreamSynchronize(st));
    if (all_conv) break;
  }
  res.iters = it;
  res.converged = (tol <= 0) || all_conv;
  return res;
}

// ---------------------------------------------------------------------------------------
// flexible GCR

template <class S>
void Fgcr<S>::ensure(size_t len, int nrhs, int restart) {
  if (len == len_ && nrhs <= nrhs_ && restart <= restart_) return;
  len_ = len;
  nrhs_ = std::max(nrhs, nrhs_);
  restart_ = std::max(restart, restart_);
  Z_.ensure(size_t(restart_) * nrhs_ * len_ * sizeof(S));
  W_.ensure(size_t(restart_) * nrhs_ * len_ * sizeof(S));
  r_.ensure(size_t(nrhs_) * len_ * sizeof(S));
  tmp_.ensure(size_t(nrhs_) * len_ * sizeof(S));
  beta_.ensure(size_t(restart_ + 1) * nrhs_ * sizeof(double2));
  nrm_.ensure(size_t(2 * nrhs_) * sizeof(double));
}

template <class S>
typename Fgcr<S>::Result Fgcr<S>::solve(LinOp& A, Precond& M, const void* b, void* x, bool x_zero, int nrhs,
                                        int restart, int max_iter, double tol, hipStream_t st) {
  const size_t len = A.len();
  ensure(len, nrhs, restart);
  const size_t vs = size_t(nrhs) * len;
  S* Z = Z_.as<S>();
  S* W = W_.as<S>();
  S* r = r_.as<S>();
  double2* beta = beta_.as<double2>();
  double* nrm = nrm_.as<double>();
  PinnedBuf& hb = hb_;
  hb.ensure(size_t(2 * nrhs) * sizeof(double));
  double* hn = hb.as<double>();

  Result res;
  res.rel_res.assign(nrhs, 0.0);
  std::vector<double> bn(nrhs);
  Blas<S>::norm2(b, len, nrhs, nrm, rw_, st);
  QMG_HIP(hipMemcpyAsync(hn, nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < nrhs; ++i) {
    bn[i] = std::sqrt(hn[i]);
    QMG_CHECK(std::isfinite(bn[i]), QMG_ENONFINITE, "FGCR: non-finite right-hand side");
  }
  auto residual = [&]() {  // r = b - A x, returns true if all converged
    if (x_zero && res.iters == 0) {
      Blas<S>::copy(b, r, vs, st);
    } else {
      A.apply(x, r, nrhs, st);
      Blas<S>::axpby(1.0, b, -1.0, r, vs, st);
    }
    Blas<S>::norm2(r, len, nrhs, nrm, rw_, st);
    QMG_HIP(hipMemcpyAsync(hn, nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    QMG_HIP(hipStreamSynchronize(st));
    bool conv = true;
    for (int i = 0; i < nrhs; ++i) {
      const double rn = std::sqrt(hn[i]);
      QMG_CHECK(std::isfinite(rn), QMG_ENONFINITE, "FGCR: non-finite residual");
      res.rel_res[i] = bn[i] > 0 ? rn / bn[i] : 0.0;
      if (res.rel_res[i] > tol) conv = false;
    }
    return conv;
  };
  if (x_zero) Blas<S>::zero(x, vs, st);
  bool conv = residual();
  while (!conv && res.iters < max_iter) {
    int k = 0;
    for (; k < restart && res.iters < max_iter; ++k) {
      S* zk = Z + size_t(k) * vs;
      S* wk = W + size_t(k) * vs;
      M.apply(r, zk, nrhs, st);
      A.apply(zk, wk, nrhs, st);
      for (int pass = 0; pass < 2 && k > 0; ++pass) {
        Blas<S>::mdot(W, vs, k, wk, len, nrhs, beta, rw_, st);
        Blas<S>::axpy_multi(W, vs, k, beta, -1.0, wk, len, nrhs, st);
        Blas<S>::axpy_multi(Z, vs, k, beta, -1.0, zk, len, nrhs, st);
      }
      Blas<S>::norm2(wk, len, nrhs, nrm, rw_, st);
      Blas<S>::scale_dev(wk, nrm, 0, len, nrhs, st);
      Blas<S>::scale_dev(zk, nrm, 0, len, nrhs, st);
      Blas<S>::dot_multi(wk, 0, 1, r, len, nrhs, beta, rw_, st);  // alpha = <w_k, r>
      Blas<S>::caxpy_dev(beta, 1.0, zk, x, len, nrhs, st);
      Blas<S>::caxpy_dev(beta, -1.0, wk, r, len, nrhs, st);
      Blas<S>::norm2(r, len, nrhs, nrm + nrhs, rw_, st);
      QMG_HIP(hipMemcpyAsync(hn, nrm, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
      QMG_HIP(hipStreamSynchronize(st));
      ++res.iters;
      bool c2 = true;
      for (int i = 0; i < nrhs; ++i) {
        const double rn = std::sqrt(hn[nrhs + i]);
        QMG_CHECK(std::isfinite(rn) && std::isfinite(hn[i]), QMG_ENONFINITE, "FGCR: non-finite residual");
        const double rel = bn[i] > 0 ? rn / bn[i] : 0.0;
        if (rel > tol) {
          c2 = false;
          QMG_CHECK(hn[i] > 0.0, QMG_EBREAKDOWN, "FGCR: preconditioned direction has zero image");
        }
      }
      if (c2) {
        ++k;
        break;
      }
    }
    conv = residual();
  }
  res.converged = conv;
  return res;
}

template class Gmres<double2>;
template class Gmres<float2>;
template class Gmres<cbf16>;
template class Gmres<chalf>;
template class Fgcr<double2>;
template class Fgcr<float2>;

}  // namespace qmg
