// Even-odd (Schur complement) preconditioning of the fine operator: half-lattice layouts and the
// inverse of the site term.
//
// With every extent even, the hops of D join sites of opposite parity p = (x + y + z + t) mod 2
// and the site term A (the diagonal term, plus the clover term) is local, so D x = b is solved
// through Dhat = A_ee - D_eo A_oo^-1 D_oe on the even sites: Dhat x_e = b_e - D_eo A_oo^-1 b_o,
// then x_o = A_oo^-1 (b_o - D_oe x_e).  A site's half-lattice index is its lexicographic index
// divided by 2.  The hop kernels are in dslash.hip; this file moves fields between the full and
// the half-lattice layouts and inverts the packed 6 x 6 blocks of the site term.
#include "qmg_internal.hpp"

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

// native FP64 gauge [mu][9][V] -> [parity][mu][9][V/2]
template <class S>
__global__ void k_eo_gauge_from_native(const double2* __restrict__ in, S* __restrict__ out, EoGeom g, size_t n) {
  const size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= n) return;
  const int site = int(q % g.V);
  const size_t me = q / g.V;  // mu * 9 + e
  const int Vh = g.V >> 1;
  const int p = site_parity(site, g);
  const double2 v = in[q];
  stc(out, (size_t(p) * 36 + me) * Vh + (site >> 1), cplx<double>{v.x, v.y});
}

// native spinors [rhs][12][V] (storage S) -> half fields of each parity, and back (added)
template <class S>
__global__ void k_eo_split(const S* __restrict__ full, S* __restrict__ even, S* __restrict__ odd, EoGeom g,
                           size_t n) {
  const size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= n) return;
  const int site = int(q % g.V);
  const size_t rk = q / g.V;  // rhs * 12 + component
  const int Vh = g.V >> 1;
  S* dst = site_parity(site, g) ? odd : even;
  dst[rk * Vh + (site >> 1)] = full[q];
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
    k_eo_pack_gauge<S><<<nblk(n), 256, 0, st>>>(static_cast<const double2*>(canon), static_cast<S*>(out), eo_geom(g),
                                                n);
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_pack_spinor(const Geom& g, const void* canon, void* even, void* odd, int nrhs, qmg_prec prec,
                           hipStream_t st) {
  const size_t n = size_t(12) * g.V * nrhs;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    k_eo_pack_spinor<S><<<nblk(n), 256, 0, st>>>(static_cast<const double2*>(canon), static_cast<S*>(even),
                                                 static_cast<S*>(odd), eo_geom(g), n);
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_unpack_spinor(const Geom& g, const void* even, const void* odd, void* canon, int nrhs, qmg_prec prec,
                             hipStream_t st) {
  const size_t n = size_t(12) * g.V * nrhs;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    k_eo_unpack_spinor<S><<<nblk(n), 256, 0, st>>>(static_cast<const S*>(even), static_cast<const S*>(odd),
                                                   static_cast<double2*>(canon), eo_geom(g), n);
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_gauge_from_native(const Geom& g, const void* U64, void* out, qmg_prec prec, hipStream_t st) {
  const size_t n = size_t(36) * g.V;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    k_eo_gauge_from_native<S><<<nblk(n), 256, 0, st>>>(static_cast<const double2*>(U64), static_cast<S*>(out),
                                                        eo_geom(g), n);
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_split(qmg_prec prec, const Geom& g, const void* full, void* even, void* odd, int nrhs, hipStream_t st) {
  const size_t n = size_t(12) * g.V * nrhs;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    k_eo_split<S><<<nblk(n), 256, 0, st>>>(static_cast<const S*>(full), static_cast<S*>(even), static_cast<S*>(odd),
                                           eo_geom(g), n);
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_merge_add(qmg_prec prec, const Geom& g, const void* even, const void* odd, void* full, int nrhs,
                         hipStream_t st) {
  const size_t n = size_t(12) * g.V * nrhs;
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    k_eo_merge_add<S><<<nblk(n), 256, 0, st>>>(static_cast<const S*>(even), static_cast<const S*>(odd),
                                               static_cast<S*>(full), eo_geom(g), n);
  });
  QMG_LAUNCH_CHECK();
}

void launch_eo_site_term(const Geom& g, const void* A64, void* Aeo, void* Ainv, qmg_prec prec, hipStream_t st) {
  DevBuf flag(sizeof(int));
  QMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
  dispatch_eo(prec, [&](auto tag) {
    using S = decltype(tag);
    k_eo_site_term<S><<<dim3(unsigned((g.V + 127) / 128), 2), 128, 0, st>>>(
        static_cast<const double2*>(A64), static_cast<S*>(Aeo), static_cast<S*>(Ainv), eo_geom(g), flag.as<int>());
  });
  QMG_LAUNCH_CHECK();
  int h = 0;
  QMG_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  QMG_HIP(hipStreamSynchronize(st));
  QMG_CHECK(h == 0, QMG_EBREAKDOWN, "the site term is singular at some site: no even-odd preconditioning");
}

}  // namespace qmg
