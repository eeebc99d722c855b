// Internal definitions shared by the HIP translation units of libqmg.
//
// Native layouts (structure of arrays, one complex plane per component, so that a
// wavefront reading one component of 64 consecutive sites issues one coalesced load):
//   spinor  [nrhs][12 = 3*spin + colour][V]   complex
//   gauge   [4 mu][9 = 3*row + col][V]        complex (physical links, no boundary sign)
//   coarse  [nrhs][d][2k]                     complex (dof order chirality, then rank index)
//   P       [d][2][k][N]                      complex, N = 6 n_d rows per (aggregate, chirality)
//                                             row = s6 * n_d + site_in_block, s6 = 3*spin_in_chirality + colour
//   Y       [d][9][2k col][2k row]            complex (slot 0 self, 1+d the hop direction d)
// Site index is lexicographic, x fastest; direction d < 4 is +mu, d >= 4 is -mu.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qmg.h"

namespace qmg {

// ----------------------------------------------------------------------------------------
// errors

void set_error(const char* fmt, ...);
const char* last_error_ptr();

struct Error {
  qmg_status code;
};

#define QMG_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      ::qmg::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call, hipGetErrorString(e_));  \
      throw ::qmg::Error{QMG_EHIP};                                                         \
    }                                                                                       \
  } while (0)

#define QMG_CHECK(cond, code, ...)      \
  do {                                  \
    if (!(cond)) {                      \
      ::qmg::set_error(__VA_ARGS__);    \
      throw ::qmg::Error{code};         \
    }                                   \
  } while (0)

#define QMG_LAUNCH_CHECK() QMG_HIP(hipGetLastError())

// ----------------------------------------------------------------------------------------
// complex arithmetic (compute types: float, double)

template <class T>
struct cplx {
  T re, im;
};

template <class T> __host__ __device__ inline cplx<T> mk(T r, T i) { return {r, i}; }
template <class T> __host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __host__ __device__ inline cplx<T> operator-(cplx<T> a) { return {-a.re, -a.im}; }
template <class T> __host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __host__ __device__ inline cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <class T> __host__ __device__ inline cplx<T>& operator+=(cplx<T>& a, cplx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <class T> __host__ __device__ inline cplx<T>& operator-=(cplx<T>& a, cplx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <class T> __host__ __device__ inline cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <class T> __host__ __device__ inline cplx<T> cmul_conj(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class T> __host__ __device__ inline T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
// i * a, -i * a
template <class T> __host__ __device__ inline cplx<T> times_i(cplx<T> a) { return {-a.im, a.re}; }
template <class T> __host__ __device__ inline cplx<T> times_mi(cplx<T> a) { return {a.im, -a.re}; }

// ----------------------------------------------------------------------------------------
// storage types: complex numbers as stored in memory

// 4-byte aligned, so that one complex number is one 32-bit access
struct alignas(4) cbf16 {  // two bfloat16 (upper halves of IEEE binary32), round to nearest even
  uint16_t re, im;
};
struct alignas(4) chalf {
  _Float16 re, im;
};

__host__ __device__ inline float bf16_to_f(uint16_t h) {
  uint32_t u = uint32_t(h) << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
__host__ __device__ inline uint16_t f_to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffff) ? 0x40 : 0));  // inf/nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

template <class S> struct StoreTraits;
template <> struct StoreTraits<double2> {
  using C = double;
  static constexpr qmg_prec prec = QMG_F64;
  __host__ __device__ static cplx<double> ld(double2 v) { return {v.x, v.y}; }
  __host__ __device__ static double2 st(cplx<double> v) { return make_double2(v.re, v.im); }
};
template <> struct StoreTraits<float2> {
  using C = float;
  static constexpr qmg_prec prec = QMG_F32;
  __host__ __device__ static cplx<float> ld(float2 v) { return {v.x, v.y}; }
  __host__ __device__ static float2 st(cplx<float> v) { return make_float2(v.re, v.im); }
};
template <> struct StoreTraits<cbf16> {
  using C = float;
  static constexpr qmg_prec prec = QMG_BF16;
  __host__ __device__ static cplx<float> ld(cbf16 v) { return {bf16_to_f(v.re), bf16_to_f(v.im)}; }
  __host__ __device__ static cbf16 st(cplx<float> v) { return {f_to_bf16(v.re), f_to_bf16(v.im)}; }
};
template <> struct StoreTraits<chalf> {
  using C = float;
  static constexpr qmg_prec prec = QMG_F16;
  __host__ __device__ static cplx<float> ld(chalf v) { return {float(v.re), float(v.im)}; }
  __host__ __device__ static chalf st(cplx<float> v) { return {_Float16(v.re), _Float16(v.im)}; }
};

template <class S> using ctype = typename StoreTraits<S>::C;

template <class S, class T>
__device__ inline cplx<ctype<S>> ldc(const S* p, T i) {
  return StoreTraits<S>::ld(p[i]);
}
template <class S, class T, class U>
__device__ inline void stc(S* p, T i, cplx<U> v) {
  using C = ctype<S>;
  p[i] = StoreTraits<S>::st(cplx<C>{C(v.re), C(v.im)});
}

// The same store with the non-temporal hint: for outputs a kernel streams out and never reads
// back, so that the inputs it re-reads (a stencil's neighbour spinors) keep the cache (the
// t-walking stencil at 32^3 x 64 FP32: 8 rhs 1541 -> 1475 us, 12 rhs 2314 -> 2193 us per launch)
template <int B> struct NtWord;
template <> struct NtWord<4> { typedef unsigned int T; };
template <> struct NtWord<8> { typedef unsigned long long T; };
template <> struct NtWord<16> { typedef unsigned long long T __attribute__((ext_vector_type(2))); };
template <class S, class T, class U>
__device__ inline void stc_stream(S* p, T i, cplx<U> v) {
  using C = ctype<S>;
  const S sv = StoreTraits<S>::st(cplx<C>{C(v.re), C(v.im)});
  typename NtWord<sizeof(S)>::T w;
  __builtin_memcpy(&w, &sv, sizeof(S));
  __builtin_nontemporal_store(w, reinterpret_cast<typename NtWord<sizeof(S)>::T*>(p + i));
}

// Wavefront sums through DPP row operations (gfx9 family: quad permutations and row rotations
// within each 16-lane row, then the row broadcasts of lanes 15 and 31), a few cycles per step
// instead of an LDS-crossbar shuffle.  The additions happen in a fixed order, so every call
// gives the same bits.  All 64 lanes must be active; wave_sum returns the total in every lane.
template <int CTRL, int ROWMASK>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}
template <int CTRL, int ROWMASK>
__device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline float lane63(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }
__device__ inline double lane63(double v) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}
template <class T>
__device__ inline T wave_sum(T v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124, 0xF>(v);  // row_ror:4
  v += dpp_move<0x128, 0xF>(v);  // row_ror:8  (every lane: its 16-lane row)
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3 (lane 63: all 64)
  return lane63(v);
}

// P consecutive complex numbers moved as one 16-byte (or, for FP64, one-number) access;
// pointers are to elements, indices to packs
template <class S, int P>
struct alignas(sizeof(S) * P) Pk {
  S v[P];
};
template <class S>
constexpr int kPack = sizeof(S) >= 16 ? 1 : int(16 / sizeof(S));

template <class S, int P>
__device__ inline Pk<S, P> ldp(const S* p, size_t pe) {
  return reinterpret_cast<const Pk<S, P>*>(p)[pe];
}
template <class S, int P>
__device__ inline void stp(S* p, size_t pe, const Pk<S, P>& v) {
  reinterpret_cast<Pk<S, P>*>(p)[pe] = v;
}

inline size_t prec_bytes(qmg_prec p) {  // bytes per complex number
  switch (p) {
    case QMG_F64: return 16;
    case QMG_F32: return 8;
    case QMG_BF16: return 4;
    case QMG_F16: return 4;
  }
  return 0;
}

// ----------------------------------------------------------------------------------------
// geometry

struct Geom {
  int L[4];      // extents x, y, z, t
  int V;         // volume
  int bc_t;      // +1 periodic, -1 antiperiodic in t
  double mass, xi;
  double diag() const { return mass + 1.0 + 3.0 / xi; }
  double cw(int mu) const { return mu == 3 ? 1.0 : 1.0 / xi; }
};

Geom make_geom(const qmg_lattice* lat);

struct Blocking {
  int b[4];     // block extents
  int cL[4];    // coarse extents
  int nd;       // sites per block
  int d;        // number of aggregates
  int N;        // rows per (aggregate, chirality) = 6 nd
};

// ----------------------------------------------------------------------------------------
// device memory owned by the library

// the library's device allocator (alloc.hip): a per-device cache of freed blocks in front of
// hipMalloc; dev_free waits for the device before a block can be handed out again
void* dev_alloc(size_t n);  // throws ENOMEM
void dev_free(void* p);
void dev_trim();            // release the cache of the current device
size_t dev_cached();        // bytes held by the cache of the current device

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    p = dev_alloc(n);
    bytes = n;
  }
  void ensure(size_t n) { if (n > bytes) alloc(n); }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// pinned host staging memory (for asynchronous device-to-host reads of small scalars)
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  void ensure(size_t n) {
    if (n <= bytes) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(&p, n, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      set_error("hipHostMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
      throw Error{QMG_ENOMEM};
    }
    bytes = n;
  }
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  template <class T> T* as() { return static_cast<T*>(p); }
};

// ----------------------------------------------------------------------------------------
// kernels exposed across translation units (host launchers)

struct DslashArgs {
  int L[4];
  int V;
  int bc_t;
  float  diag_f, cw_f[4];
  double diag_d, cw_d[4];
  int nrhs;
  int dagger;
  int canonical;  // 1: AoS canonical layouts, 0: native SoA
  int tchunk;     // native kernel: sites per thread along t (0: chosen by the launcher)
  // site term with the clover term, in the storage precision of U: per chirality alpha the 18
  // complex entries of a hermitian 6 x 6 block at [(alpha * 18 + e) * V + site] (e = 0..2: the
  // real diagonal in pairs, 3..17: the upper triangle row by row); nullptr: the scalar
  // diagonal term of the Wilson operator
  const void* clov;
  // complex entries stored per link in the half-lattice gauge field of the even-odd forms: 9, or
  // 6 (the first two rows of SU(3) links; the third is rebuilt in the kernel)
  int link_ne;
};
DslashArgs make_dslash_args(const Geom& g, int nrhs, bool dagger, bool canonical);

// one lattice of a batched launch: its operator arguments and its first workgroup
struct BatchLattice {
  DslashArgs a;
  int tile0;
};
// out[i] = D_i in[i] for n_lat lattices in one launch (native layout; U, in, out: device arrays
// of device pointers; lat_dev: device array of descriptors with prefix-summed tile0)
void launch_dslash_batched(qmg_prec prec, const BatchLattice* lat_dev, int n_lat, int total_tiles,
                           const void* const* U, const void* const* in, void* const* out, bool dagger,
                           double bytes, double flops, hipStream_t st);
// many lattices in padded layouts (see k_dslash_padded): nl lattices of nr spinors each
void launch_dslash_padded(qmg_prec prec, const BatchLattice* lat_dev, int nl, int nr, int Vpad, const void* U,
                          const void* in, void* out, bool dagger, double bytes, double flops, hipStream_t st);
void set_dslash_variant(int v);

// out = D in (or D^dag) ; U in the same storage type and layout as the spinors
void launch_dslash(qmg_prec prec, const void* U, const void* in, void* out, const DslashArgs& a,
                   hipStream_t st);

// layout conversion (canonical FP64 <-> native storage), spinors and gauge
// canonical [nrhs][V][12] in precision pc <-> native [nrhs][12][V] in precision pn
void launch_pack_spinor(const void* canon, qmg_prec pc, void* native, qmg_prec pn, int V, int nrhs, hipStream_t st);
void launch_unpack_spinor(const void* native, qmg_prec pn, void* canon, qmg_prec pc, int V, int nrhs, hipStream_t st);
void launch_pack_gauge(const void* canon_f64, void* native, qmg_prec prec, int V, hipStream_t st);
// precision conversion between native buffers of n complex numbers
void launch_convert(const void* in, qmg_prec pin, void* out, qmg_prec pout, size_t n, hipStream_t st);
// A64 = the packed FP64 site term (layout of DslashArgs::clov) of the Wilson-clover operator with
// clover coefficients cs (spatial planes) and ct (planes containing t), from the native FP64
// gauge field U64; synchronises st before returning (it frees a temporary)
void launch_clover_field(const Geom& g, const void* U64, double cs, double ct, void* A64, hipStream_t st);
// Even-odd forms (every extent even; half-lattice index = lexicographic index / 2).  Layouts:
// spinor [rhs][12][V/2] per parity, gauge [parity][mu][9][V/2], packed site term and inverse
// [parity][alpha][18][V/2] (nullptr: the scalar diagonal term).  Every storage precision.
// out (parity p) = POST(YM(y) + sgn H in): ym 0 nothing, 1 y, 2 A_p y; post 0 nothing, 1 A_p^-1;
// the forms (ym, post) = (0, 1), (2, 0), (1, 0), (1, 1) are built.  a.nrhs, a.dagger apply.
void launch_hop_eo(qmg_prec prec, const DslashArgs& a, const void* Ue, const void* Uo, int p, const void* in,
                   const void* y, void* out, const void* Ap, const void* Aip, int ym, int post, double sgn,
                   hipStream_t st);
// out = M in (M = A_p, or A_p^-1 with inv) on one parity's half fields
void launch_site_eo(qmg_prec prec, const DslashArgs& a, const void* M, bool inv, const void* in, void* out,
                    hipStream_t st);
void launch_eo_pack_gauge(const Geom& g, const void* canon, void* out, qmg_prec prec, hipStream_t st);
void launch_eo_pack_spinor(const Geom& g, const void* canon, void* even, void* odd, int nrhs, qmg_prec prec,
                           hipStream_t st);
void launch_eo_unpack_spinor(const Geom& g, const void* even, const void* odd, void* canon, int nrhs, qmg_prec prec,
                             hipStream_t st);
// native FP64 gauge [mu][9][V] -> [parity][mu][ne][V/2] in prec (ne = 9, or 6: the first two rows)
void launch_eo_gauge_from_native(const Geom& g, const void* U64, void* out, qmg_prec prec, hipStream_t st,
                                 int ne = 9);
// largest |third row - conj(row0 x row1)| over the native FP64 gauge field (synchronises)
double launch_su3_row_defect(const Geom& g, const void* U64, hipStream_t st);
// native spinors [rhs][12][V] in prec: full += the two half fields of each parity
void launch_eo_merge_add(qmg_prec prec, const Geom& g, const void* even, const void* odd, void* full, int nrhs,
                         hipStream_t st);
// half fields of r - t, rounded once to the storage type
void launch_eo_split_sub(qmg_prec prec, const Geom& g, const void* r, const void* t, void* even, void* odd, int nrhs,
                         hipStream_t st);
// s-step residual minimisation: c[j * nrhs + r] (device, j < m - 1) minimising
// ||p_0 - sum_j c_j w_j||, w_j = p_{j+1} + shift p_j, over a basis p_0 .. p_{m-1} (m <= 9, vector
// i of rhs r at P + (i * nrhs + r) * len, storage prec); with p_{j+1} = (A - shift) p_j,
// x = sum_j c_j p_j minimises ||p_0 - A x|| over the Krylov space.  part: work buffer (sized here)
void launch_sstep_coeffs(qmg_prec prec, const void* P, int m, size_t len, int nrhs, double2* c, DevBuf& part,
                         hipStream_t st, double shift = 0.0);
// the full-lattice packed FP64 site term -> its half-lattice copy and inverse in prec (synchronises;
// EBREAKDOWN if a block is singular)
void launch_eo_site_term(const Geom& g, const void* A64, void* Aeo, void* Ainv, qmg_prec prec, hipStream_t st);

}  // namespace qmg
