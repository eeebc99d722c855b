// Wilson-Dirac stencil D and D^dagger (the operator of Eq. (1)), site-parallel.
//
// Every hop uses the rank-2 spin projection of (1 +/- gamma_mu) in the chiral basis
// gamma_mu = [[0, A_mu], [A_mu^dag, 0]] (A_x = -i sigma_1, A_y = -i sigma_2,
// A_z = -i sigma_3, A_t = 1):
//   (1 + s gamma_mu) chi = [ h ; s A_mu^dag h ],  h = chi_up + s A_mu chi_down,
// so a hop multiplies two colour vectors by the link instead of four.  Bandwidth bound:
// per site and right-hand side the algorithm reads the spinor once (24 reals), the four
// forward links once (72 reals, shared across right-hand sides) and writes 24 reals.
//
// With the clover term the site-local part of the operator, (m + 1 + 3/xi) + T(x), is two
// hermitian 6 x 6 blocks per site (T commutes with gamma_5); every form then applies them in
// its epilogue in place of the scalar diagonal term (kernels instantiated with CLOV = true).
//
// Launch: one thread per (site, group of NR right-hand sides), 256 threads per workgroup.
// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X; the tile index is
// remapped so that each XCD walks a contiguous range of sites, keeping the +-t neighbour
// slices of a tile inside that XCD's L2.
#include <string>
#include <type_traits>

#include "timing.hpp"
#include "tune.hpp"

namespace qmg {

namespace {
int g_variant = 0;  // forced native-layout launch variant (0: heuristic or tuned)
}

void set_dslash_variant(int v) { g_variant = v; }

DslashArgs make_dslash_args(const Geom& g, int nrhs, bool dagger, bool canonical) {
  DslashArgs a{};
  a.tchunk = g_variant;
  for (int m = 0; m < 4; ++m) a.L[m] = g.L[m];
  a.V = g.V;
  a.bc_t = g.bc_t;
  a.diag_d = g.diag();
  a.diag_f = float(a.diag_d);
  for (int m = 0; m < 4; ++m) {
    a.cw_d[m] = g.cw(m);
    a.cw_f[m] = float(a.cw_d[m]);
  }
  a.nrhs = nrhs;
  a.dagger = dagger ? 1 : 0;
  a.canonical = canonical ? 1 : 0;
  a.clov = nullptr;
  a.link_ne = 9;
  return a;
}

namespace {

constexpr int kBlock = 256;

// XCD-aware tile index: hardware hands workgroup b to XCD b % 8.
__device__ inline int xcd_tile(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
  return x * q + min(x, rem) + i;
}

template <bool CANON>
__device__ inline size_t sp_idx(int rhs, int comp, int site, int V) {
  return CANON ? (size_t(rhs) * V + site) * 12 + comp : (size_t(rhs) * 12 + comp) * V + site;
}
template <bool CANON>
__device__ inline size_t g_idx(int mu, int e, int site, int V) {
  return CANON ? (size_t(mu) * V + site) * 9 + e : (size_t(mu) * 9 + e) * V + site;
}

// h = chi_up + s A_mu chi_dn   (2 spin x 3 colour), components index 3*spin + colour
template <int MU, class C>
__device__ inline void project(const cplx<C>* chi, C s, cplx<C>* h) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cplx<C> u0 = chi[c], u1 = chi[3 + c], d0 = chi[6 + c], d1 = chi[9 + c];
    if (MU == 0) {         // A = -i sigma_1: (A d) = (-i d1, -i d0)
      h[c] = u0 + s * times_mi(d1);
      h[3 + c] = u1 + s * times_mi(d0);
    } else if (MU == 1) {  // A = -i sigma_2 = [[0,-1],[1,0]]: (A d) = (-d1, d0)
      h[c] = u0 - s * d1;
      h[3 + c] = u1 + s * d0;
    } else if (MU == 2) {  // A = -i sigma_3 = diag(-i, i)
      h[c] = u0 + s * times_mi(d0);
      h[3 + c] = u1 + s * times_i(d1);
    } else {               // A = 1
      h[c] = u0 + s * d0;
      h[3 + c] = u1 + s * d1;
    }
  }
}

// acc += coef * [ w ; s A_mu^dag w ]
template <int MU, class C>
__device__ inline void reconstruct(cplx<C>* acc, const cplx<C>* w, C s, C coef) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cplx<C> w0 = coef * w[c], w1 = coef * w[3 + c];
    acc[c] += w0;
    acc[3 + c] += w1;
    const C cs = s;
    if (MU == 0) {         // A^dag = i sigma_1: (i w1, i w0)
      acc[6 + c] += cs * times_i(w1);
      acc[9 + c] += cs * times_i(w0);
    } else if (MU == 1) {  // A^dag = [[0,1],[-1,0]]: (w1, -w0)
      acc[6 + c] += cs * w1;
      acc[9 + c] -= cs * w0;
    } else if (MU == 2) {  // A^dag = diag(i, -i)
      acc[6 + c] += cs * times_i(w0);
      acc[9 + c] += cs * times_mi(w1);
    } else {
      acc[6 + c] += cs * w0;
      acc[9 + c] += cs * w1;
    }
  }
}

template <class C, bool ADJ>
__device__ inline void su3_mul(const cplx<C>* u, const cplx<C>* h, cplx<C>* w) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<C> t = {C(0), C(0)};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (ADJ) t += cmul_conj(u[3 * b + a], h[3 * sp + b]);
        else t += u[3 * a + b] * h[3 * sp + b];
      }
      w[3 * sp + a] = t;
    }
  }
}

// NE = 6: native links stored as their first two rows ([mu][6][V]); the third row of an SU(3)
// matrix is the complex conjugate of the cross product of the first two
template <class S, bool CANON, int NR, int MU, bool FWD, bool DAG, int NE = 9>
__device__ inline void do_hop(const S* __restrict__ U, const S* __restrict__ in, cplx<ctype<S>> (*acc)[12],
                              int link_site, int nb_site, int rhs0, int V, ctype<S> coef) {
  using C = ctype<S>;
  cplx<C> u[9];
  if constexpr (NE == 9) {
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ldc(U, g_idx<CANON>(MU, e, link_site, V));
  } else {
    static_assert(!CANON && NE == 6, "two-row links exist in the native half-lattice layout only");
#pragma unroll
    for (int e = 0; e < 6; ++e) u[e] = ldc(U, (size_t(MU) * 6 + e) * V + link_site);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      u[6 + c] = conj(u[c1] * u[3 + c2] - u[c2] * u[3 + c1]);
    }
  }
  // forward hop uses (1 - gamma), backward (1 + gamma); D^dag swaps them
  const C s = (FWD != DAG) ? C(-1) : C(1);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    cplx<C> chi[12], h[6], w[6];
#pragma unroll
    for (int k = 0; k < 12; ++k) chi[k] = ldc(in, sp_idx<CANON>(rhs0 + r, k, nb_site, V));
    project<MU>(chi, s, h);
    su3_mul<C, !FWD>(u, h, w);
    reconstruct<MU>(acc[r], w, s, coef);
  }
}

// acc[r] += A(x) v[r] for NR right-hand sides, A(x) the site's packed site term: per chirality
// 18 complex entries at A[(alpha * 18 + e) * V + x], e = 0..2 the real diagonal in pairs
// (re: entry 2e, im: entry 2e+1) and e = 3..17 the upper triangle row by row; the lower
// triangle is its conjugate.  Each entry is loaded once for all NR right-hand sides.
template <class S, int NR>
__device__ inline void clover_acc(const S* __restrict__ A, int site, int V, const cplx<ctype<S>> (*v)[12],
                                  cplx<ctype<S>> (*acc)[12]) {
  using C = ctype<S>;
#pragma unroll
  for (int al = 0; al < 2; ++al) {
    const S* b = A + size_t(al) * 18 * V + site;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const cplx<C> d = ldc(b, size_t(e) * V);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        acc[r][6 * al + 2 * e] += d.re * v[r][6 * al + 2 * e];
        acc[r][6 * al + 2 * e + 1] += d.im * v[r][6 * al + 2 * e + 1];
      }
    }
    int e = 3;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i + 1; j < 6; ++j, ++e) {
        const cplx<C> o = ldc(b, size_t(e) * V);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          acc[r][6 * al + i] += o * v[r][6 * al + j];
          acc[r][6 * al + j] += cmul_conj(o, v[r][6 * al + i]);
        }
      }
  }
}

// D (or D^dag) at one site for NR right-hand sides starting at rhs0
template <class S, bool CANON, int NR, bool DAG, bool CLOV = false>
__device__ inline void site_dslash(const S* __restrict__ U, const S* __restrict__ in, S* __restrict__ out,
                                   const DslashArgs& a, int site, int rhs0) {
  using C = ctype<S>;
  const int V = a.V;
  const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  int rem = site;
  const int x = rem % L0; rem /= L0;
  const int y = rem % L1; rem /= L1;
  const int z = rem % L2;
  const int t = rem / L2;
  const int s1 = L0, s2 = L0 * L1, s3 = L0 * L1 * L2;
  const int xp = (x + 1 == L0) ? site - (L0 - 1) : site + 1;
  const int xm = (x == 0) ? site + (L0 - 1) : site - 1;
  const int yp = (y + 1 == L1) ? site - (L1 - 1) * s1 : site + s1;
  const int ym = (y == 0) ? site + (L1 - 1) * s1 : site - s1;
  const int zp = (z + 1 == L2) ? site - (L2 - 1) * s2 : site + s2;
  const int zm = (z == 0) ? site + (L2 - 1) * s2 : site - s2;
  const int tp = (t + 1 == L3) ? site - (L3 - 1) * s3 : site + s3;
  const int tm = (t == 0) ? site + (L3 - 1) * s3 : site - s3;

  C cw[4], diag;
  if constexpr (sizeof(C) == 8) {
    for (int m = 0; m < 4; ++m) cw[m] = a.cw_d[m];
    diag = a.diag_d;
  } else {
    for (int m = 0; m < 4; ++m) cw[m] = a.cw_f[m];
    diag = a.diag_f;
  }
  const C bt_f = (a.bc_t < 0 && t == L3 - 1) ? C(-1) : C(1);
  const C bt_b = (a.bc_t < 0 && t == 0) ? C(-1) : C(1);

  cplx<C> acc[NR][12];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[r][k] = {C(0), C(0)};

  const C mh = C(-0.5);
  do_hop<S, CANON, NR, 0, true, DAG>(U, in, acc, site, xp, rhs0, V, mh * cw[0]);
  do_hop<S, CANON, NR, 0, false, DAG>(U, in, acc, xm, xm, rhs0, V, mh * cw[0]);
  do_hop<S, CANON, NR, 1, true, DAG>(U, in, acc, site, yp, rhs0, V, mh * cw[1]);
  do_hop<S, CANON, NR, 1, false, DAG>(U, in, acc, ym, ym, rhs0, V, mh * cw[1]);
  do_hop<S, CANON, NR, 2, true, DAG>(U, in, acc, site, zp, rhs0, V, mh * cw[2]);
  do_hop<S, CANON, NR, 2, false, DAG>(U, in, acc, zm, zm, rhs0, V, mh * cw[2]);
  do_hop<S, CANON, NR, 3, true, DAG>(U, in, acc, site, tp, rhs0, V, mh * cw[3] * bt_f);
  do_hop<S, CANON, NR, 3, false, DAG>(U, in, acc, tm, tm, rhs0, V, mh * cw[3] * bt_b);

  if constexpr (CLOV) {
    cplx<C> v[NR][12];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int k = 0; k < 12; ++k) v[r][k] = ldc(in, sp_idx<CANON>(rhs0 + r, k, site, V));
    clover_acc<S, NR>(static_cast<const S*>(a.clov), site, V, v, acc);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int k = 0; k < 12; ++k) stc(out, sp_idx<CANON>(rhs0 + r, k, site, V), acc[r][k]);
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const size_t i = sp_idx<CANON>(rhs0 + r, k, site, V);
        cplx<C> v = ldc(in, i);
        stc(out, i, diag * v + acc[r][k]);
      }
    }
  }
}

template <class S, bool CANON, int NR, bool DAG, bool CLOV = false>
__global__ __launch_bounds__(kBlock) void k_dslash(const S* __restrict__ U, const S* __restrict__ in,
                                                   S* __restrict__ out, DslashArgs a) {
  // flattened grid over (tile, rhs group) with the rhs groups of a tile adjacent in the
  // XCD-local order, so that they share the tile's links in L2
  const int ng = a.nrhs / NR;
  const int wg = xcd_tile(blockIdx.x, gridDim.x);
  const int tile = wg / ng;
  const int site = tile * kBlock + threadIdx.x;
  if (site >= a.V) return;
  site_dslash<S, CANON, NR, DAG, CLOV>(U, in, out, a, site, (wg - tile * ng) * NR);
}

// Many lattices in one launch: workgroup (after the XCD remap) w belongs to the lattice whose
// tile range [tile0, tile0 + ntiles * nrhs) holds it; every lattice has its own extents,
// coefficients, gauge field and spinors (native layout).
template <class S, bool DAG>
__global__ __launch_bounds__(kBlock) void k_dslash_batched(const BatchLattice* __restrict__ lat, int n_lat,
                                                           const S* const* __restrict__ U,
                                                           const S* const* __restrict__ in,
                                                           S* const* __restrict__ out) {
  const int wg = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = n_lat - 1;  // last lattice with tile0 <= wg
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (lat[mid].tile0 <= wg) lo = mid;
    else hi = mid - 1;
  }
  const BatchLattice& b = lat[lo];
  const int local = wg - b.tile0;
  const int ntile = (b.a.V + kBlock - 1) / kBlock;
  const int rhs = local / ntile, tile = local - rhs * ntile;
  const int site = tile * kBlock + threadIdx.x;
  if (site >= b.a.V) return;
  site_dslash<S, false, 1, DAG>(U[lo], in[lo], out[lo], b.a, site, rhs);
}

// Many lattices in padded layouts (one hierarchy over many small lattices): lattice l's links at
// U + l * 36 Vpad ([4][9][Vpad]) and its nr spinors at in / out + l * nr * 12 Vpad
// ([nr][12][Vpad]); lat[l].a carries the lattice's extents and coefficients with a.V = Vpad (the
// stride).  Grid: nl * nr * ceil(Vpad / 256) workgroups; sites at and beyond the lattice's
// volume are written as zeros, so every output column is zero-padded.
// A thread forms NR right-hand sides of its site (links loaded once for all of them); the
// groups of a tile are adjacent in the schedule.
template <class S, bool DAG, int NR>
__global__ __launch_bounds__(kBlock) void k_dslash_padded(const BatchLattice* __restrict__ lat, const S* __restrict__ U,
                                                          const S* __restrict__ in, S* __restrict__ out, int nr,
                                                          int ntile) {
  const int wg = xcd_tile(blockIdx.x, gridDim.x);
  const int ng = nr / NR;
  const int g = wg % ng, tc = wg / ng;
  const int tile = tc % ntile, l = tc / ntile;
  const int rhs0 = g * NR;
  const DslashArgs& a = lat[l].a;
  const int Vpad = a.V;
  const int site = tile * kBlock + threadIdx.x;
  if (site >= Vpad) return;
  const size_t base = size_t(l) * nr * 12 * Vpad;
  if (site >= a.L[0] * a.L[1] * a.L[2] * a.L[3]) {
    for (int r = 0; r < NR; ++r)
      for (int k = 0; k < 12; ++k) stc(out + base, sp_idx<false>(rhs0 + r, k, site, Vpad), cplx<ctype<S>>{0, 0});
    return;
  }
  site_dslash<S, false, NR, DAG>(U + size_t(l) * 36 * Vpad, in + base, out + base, a, site, rhs0);
}

// Native-layout kernel that walks along t.  Thread (spatial site, t-chunk, group of NR
// right-hand sides) computes the TCH sites t0 .. t0+TCH-1 of its column for NR right-hand
// sides; each link is loaded once for all NR of them.  The spinor of the next slice, loaded
// for the forward t-hop, becomes the own spinor of the next step, and the backward t-hop
// U_t(x, t-1)^dag (1 + gamma_t) psi(x, t-1) is formed from the own spinor and forward t-link
// of the previous step, so t-neighbours and t-links are read once.  Workgroups are 256
// spatial sites of one (t-chunk, rhs group); the rhs groups of a tile are adjacent in the
// XCD-local schedule so that they share its links in L2.  Tiles are 256 consecutive spatial
// sites, or (zfast) 256-site pieces of one xy-plane with z fastest in the schedule, so that
// the tiles holding a site's z-neighbours run next to it.
template <class S, int TCH, int NR, bool DAG, bool CLOV = false>
__global__ __launch_bounds__(kBlock) void k_dslash_t(const S* __restrict__ U, const S* __restrict__ in,
                                                     S* __restrict__ out, DslashArgs a, int ntile_s, int zfast,
                                                     int cmaj) {
  using C = ctype<S>;
  const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  const int Vs = L0 * L1 * L2, V = a.V;
  const int ng = a.nrhs / NR;
  const int per_chunk = ntile_s * ng;
  int wg;
  if (cmaj) {  // t-chunk major in dispatch order (all XCDs on one chunk), XCD-local tiles within it
    const int ch = blockIdx.x / per_chunk;
    wg = ch * per_chunk + xcd_tile(blockIdx.x - ch * per_chunk, per_chunk);
  } else {
    wg = xcd_tile(blockIdx.x, gridDim.x);
  }
  const int chunk = wg / per_chunk, r0 = wg - chunk * per_chunk;
  const int ts = r0 / ng, g = r0 - ts * ng;
  int xs;  // spatial site
  if (zfast) {
    const int Pxy = L0 * L1;
    const int z = ts % L2, piece = ts / L2;
    const int xy = piece * kBlock + threadIdx.x;
    if (xy >= Pxy) return;
    xs = xy + z * Pxy;
  } else {
    xs = ts * kBlock + threadIdx.x;
    if (xs >= Vs) return;
  }
  const int rhs0 = g * NR;
  const int t0 = chunk * TCH;
  int rem = xs;
  const int x = rem % L0; rem /= L0;
  const int y = rem % L1;
  const int z = rem / L1;
  const int s1 = L0, s2 = L0 * L1;
  const int dxp = (x + 1 == L0) ? -(L0 - 1) : 1, dxm = (x == 0) ? (L0 - 1) : -1;
  const int dyp = (y + 1 == L1) ? -(L1 - 1) * s1 : s1, dym = (y == 0) ? (L1 - 1) * s1 : -s1;
  const int dzp = (z + 1 == L2) ? -(L2 - 1) * s2 : s2, dzm = (z == 0) ? (L2 - 1) * s2 : -s2;
  C cw[4], diag;
  if constexpr (sizeof(C) == 8) {
    for (int m = 0; m < 4; ++m) cw[m] = a.cw_d[m];
    diag = a.diag_d;
  } else {
    for (int m = 0; m < 4; ++m) cw[m] = a.cw_f[m];
    diag = a.diag_f;
  }
  const C mh = C(-0.5);
  const C sf = DAG ? C(1) : C(-1);  // forward projector sign: (1 + sf gamma)
  const C sb = -sf;                  // backward projector sign

  // own spinors of the first site and the backward t-hops carried into them
  cplx<C> psi[NR][12], hb[NR][6];
  {
    const int tm = (t0 == 0) ? L3 - 1 : t0 - 1;
    const int sm = xs + tm * Vs;
    cplx<C> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ldc(U, size_t(3 * 9 + e) * V + sm);
    const int s0 = xs + t0 * Vs;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      cplx<C> chi[12], h[6];
#pragma unroll
      for (int k = 0; k < 12; ++k) chi[k] = ldc(in, sp_idx<false>(rhs0 + r, k, sm, V));
      project<3>(chi, sb, h);
      su3_mul<C, true>(u, h, hb[r]);
#pragma unroll
      for (int k = 0; k < 12; ++k) psi[r][k] = ldc(in, sp_idx<false>(rhs0 + r, k, s0, V));
    }
  }
#pragma unroll 1
  for (int dt = 0; dt < TCH; ++dt) {
    const int t = t0 + dt;
    const int site = xs + t * Vs;
    const int tp = (t + 1 == L3) ? 0 : t + 1;
    const int sp = xs + tp * Vs;
    cplx<C> acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[r][k] = {C(0), C(0)};
    // the site term first, from the own spinors that are live anyway: each of its entries is
    // loaded once for all NR right-hand sides and nothing more stays live for the epilogue
    if constexpr (CLOV) clover_acc<S, NR>(static_cast<const S*>(a.clov), site, V, psi, acc);
    do_hop<S, false, NR, 0, true, DAG>(U, in, acc, site, site + dxp, rhs0, V, mh * cw[0]);
    do_hop<S, false, NR, 0, false, DAG>(U, in, acc, site + dxm, site + dxm, rhs0, V, mh * cw[0]);
    do_hop<S, false, NR, 1, true, DAG>(U, in, acc, site, site + dyp, rhs0, V, mh * cw[1]);
    do_hop<S, false, NR, 1, false, DAG>(U, in, acc, site + dym, site + dym, rhs0, V, mh * cw[1]);
    do_hop<S, false, NR, 2, true, DAG>(U, in, acc, site, site + dzp, rhs0, V, mh * cw[2]);
    do_hop<S, false, NR, 2, false, DAG>(U, in, acc, site + dzm, site + dzm, rhs0, V, mh * cw[2]);
    // backward t-hop (carried), boundary sign at t = 0
    const C bt_b = (a.bc_t < 0 && t == 0) ? C(-1) : C(1);
    const C bt_f = (a.bc_t < 0 && t == L3 - 1) ? C(-1) : C(1);
    // forward t-hop: this site's t-link and the next spinors
    cplx<C> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ldc(U, size_t(3 * 9 + e) * V + site);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      reconstruct<3>(acc[r], hb[r], sb, mh * cw[3] * bt_b);
      cplx<C> nxt[12], h[6], w[6];
#pragma unroll
      for (int k = 0; k < 12; ++k) nxt[k] = ldc(in, sp_idx<false>(rhs0 + r, k, sp, V));
      project<3>(nxt, sf, h);
      su3_mul<C, false>(u, h, w);
      reconstruct<3>(acc[r], w, sf, mh * cw[3] * bt_f);
      // backward t-hop of the next site from this site's spinor and t-link
      project<3>(psi[r], sb, h);
      su3_mul<C, true>(u, h, hb[r]);
      if constexpr (CLOV) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          stc_stream(out, sp_idx<false>(rhs0 + r, k, site, V), acc[r][k]);
          psi[r][k] = nxt[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          stc_stream(out, sp_idx<false>(rhs0 + r, k, site, V), diag * psi[r][k] + acc[r][k]);
          psi[r][k] = nxt[k];
        }
      }
    }
  }
}

// Rows I0 .. I0+2 of one chirality block of the packed site term (layout of clover_acc)
// applied to that chirality's six spinor components x; compile-time row indices.
template <class S, int I0>
__device__ inline void site_term_rows(const S* __restrict__ b, int V, const cplx<ctype<S>> (&x)[6],
                                      cplx<ctype<S>> (&y)[3]) {
  using C = ctype<S>;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int i = I0 + q;
    const cplx<C> dd = ldc(b, size_t(i >> 1) * V);
    cplx<C> v = ((i & 1) ? dd.im : dd.re) * x[i];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (j == i) continue;
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      const cplx<C> o = ldc(b, size_t(3 + lo * (11 - lo) / 2 + (hi - lo - 1)) * V);
      v += (i < j) ? o * x[j] : cmul_conj(o, x[j]);
    }
    y[q] = v;
  }
}

// Direction-split native kernel: a workgroup covers 64 consecutive sites, wavefront mu forms
// the forward and backward hops along mu for those sites (mu is uniform in the wavefront, so
// there is no divergence), the four partial sums meet in LDS, and wavefront w then writes
// spinor components 3w .. 3w+2 of the 64 sites.  Four times as many threads as the site
// kernel, each with two hops in flight: for lattices too small to fill the GPU with one
// thread per site.
template <class S, bool DAG, bool CLOV = false>
__global__ __launch_bounds__(kBlock) void k_dslash_dir(const S* __restrict__ U, const S* __restrict__ in,
                                                       S* __restrict__ out, DslashArgs a) {
  using C = ctype<S>;
  constexpr int TS = kBlock / 4;  // sites per workgroup
  __shared__ cplx<C> part[4][12][TS];
  const int wg = xcd_tile(blockIdx.x, gridDim.x);
  const int ntile = (a.V + TS - 1) / TS;
  const int tile = wg % ntile, rhs = wg / ntile;
  const int lane = threadIdx.x & (TS - 1), mu = threadIdx.x / TS;
  const int site = tile * TS + lane;
  const bool live = site < a.V;
  const int V = a.V;
  const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  const S* inr = in + size_t(rhs) * 12 * V;
  S* outr = out + size_t(rhs) * 12 * V;
  C cw, diag;
  if constexpr (sizeof(C) == 8) {
    cw = a.cw_d[mu];
    diag = a.diag_d;
  } else {
    cw = a.cw_f[mu];
    diag = a.diag_f;
  }
  const C mh = C(-0.5);
  cplx<C> acc[1][12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[0][k] = {C(0), C(0)};
  if (live) {
    int rem = site;
    const int x = rem % L0; rem /= L0;
    const int y = rem % L1; rem /= L1;
    const int z = rem % L2;
    const int t = rem / L2;
    int c, L, st;
    if (mu == 0) { c = x; L = L0; st = 1; }
    else if (mu == 1) { c = y; L = L1; st = L0; }
    else if (mu == 2) { c = z; L = L2; st = L0 * L1; }
    else { c = t; L = L3; st = L0 * L1 * L2; }
    const int fp = (c + 1 == L) ? site - (L - 1) * st : site + st;
    const int bm = (c == 0) ? site + (L - 1) * st : site - st;
    C cf = mh * cw, cb = mh * cw;
    if (mu == 3 && a.bc_t < 0) {
      if (t == L3 - 1) cf = -cf;
      if (t == 0) cb = -cb;
    }
    switch (mu) {  // uniform within the wavefront
      case 0:
        do_hop<S, false, 1, 0, true, DAG>(U, inr, acc, site, fp, 0, V, cf);
        do_hop<S, false, 1, 0, false, DAG>(U, inr, acc, bm, bm, 0, V, cb);
        break;
      case 1:
        do_hop<S, false, 1, 1, true, DAG>(U, inr, acc, site, fp, 0, V, cf);
        do_hop<S, false, 1, 1, false, DAG>(U, inr, acc, bm, bm, 0, V, cb);
        break;
      case 2:
        do_hop<S, false, 1, 2, true, DAG>(U, inr, acc, site, fp, 0, V, cf);
        do_hop<S, false, 1, 2, false, DAG>(U, inr, acc, bm, bm, 0, V, cb);
        break;
      default:
        do_hop<S, false, 1, 3, true, DAG>(U, inr, acc, site, fp, 0, V, cf);
        do_hop<S, false, 1, 3, false, DAG>(U, inr, acc, bm, bm, 0, V, cb);
        break;
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) part[mu][k][lane] = acc[0][k];
  __syncthreads();
  if (!live) return;
  if constexpr (CLOV) {
    // wavefront mu writes rows 3 (mu & 1) .. +2 of chirality mu >> 1 (uniform in the wavefront)
    const int al = mu >> 1;
    cplx<C> x[6], y[3];
#pragma unroll
    for (int j = 0; j < 6; ++j) x[j] = ldc(inr, size_t(6 * al + j) * V + site);
    const S* b = static_cast<const S*>(a.clov) + size_t(al) * 18 * V + site;
    if (mu & 1) site_term_rows<S, 3>(b, V, x, y);
    else site_term_rows<S, 0>(b, V, x, y);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int k = 3 * mu + q;
      cplx<C> v = y[q];
#pragma unroll
      for (int m = 0; m < 4; ++m) v += part[m][k][lane];
      stc(outr, size_t(k) * V + site, v);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int k = 3 * mu + q;
      const size_t i = size_t(k) * V + site;
      cplx<C> v = diag * ldc(inr, i);
#pragma unroll
      for (int m = 0; m < 4; ++m) v += part[m][k][lane];
      stc(outr, i, v);
    }
  }
}

template <class S>
void launch_dir(const void* U, const void* in, void* out, const DslashArgs& a, hipStream_t st) {
  dim3 grid(unsigned((a.V + kBlock / 4 - 1) / (kBlock / 4)) * unsigned(a.nrhs));
  if (a.clov) {
    if (a.dagger)
      launch(k_dslash_dir<S, true, true>, grid, dim3(kBlock), 0, st, U, in, out, a);
    else
      launch(k_dslash_dir<S, false, true>, grid, dim3(kBlock), 0, st, U, in, out, a);
  } else if (a.dagger) {
    launch(k_dslash_dir<S, true>, grid, dim3(kBlock), 0, st, U, in, out, a);
  } else {
    launch(k_dslash_dir<S, false>, grid, dim3(kBlock), 0, st, U, in, out, a);
  }
  QMG_LAUNCH_CHECK();
}

template <class S, bool CANON, int NR>
void launch_t(const void* U, const void* in, void* out, const DslashArgs& a, hipStream_t st) {
  dim3 grid(unsigned((a.V + kBlock - 1) / kBlock) * unsigned(a.nrhs / NR));
  if constexpr (NR == 1) {
    if (a.clov) {
      if (a.dagger)
        launch(k_dslash<S, CANON, 1, true, true>, grid, dim3(kBlock), 0, st, U, in, out, a);
      else
        launch(k_dslash<S, CANON, 1, false, true>, grid, dim3(kBlock), 0, st, U, in, out, a);
      QMG_LAUNCH_CHECK();
      return;
    }
  }
  if (a.dagger)
    launch(k_dslash<S, CANON, NR, true>, grid, dim3(kBlock), 0, st, U, in, out, a);
  else
    launch(k_dslash<S, CANON, NR, false>, grid, dim3(kBlock), 0, st, U, in, out, a);
  QMG_LAUNCH_CHECK();
}

template <class S, int TCH, int NR>
void launch_tw(const void* U, const void* in, void* out, const DslashArgs& a, int zfast, hipStream_t st,
               int cmaj = 0) {
  const int Vs = a.L[0] * a.L[1] * a.L[2];
  const int ntile_s = zfast ? ((a.L[0] * a.L[1] + kBlock - 1) / kBlock) * a.L[2] : (Vs + kBlock - 1) / kBlock;
  const int nchunk = a.L[3] / TCH;
  dim3 grid(unsigned(ntile_s * nchunk * (a.nrhs / NR)));
  if constexpr (sizeof(S) >= 8) {  // the site-term forms exist for FP32 and FP64 storage
    if (a.clov) {
      if (a.dagger)
        launch(k_dslash_t<S, TCH, NR, true, true>, grid, dim3(kBlock), 0, st, U, in, out, a, ntile_s, zfast, cmaj);
      else
        launch(k_dslash_t<S, TCH, NR, false, true>, grid, dim3(kBlock), 0, st, U, in, out, a, ntile_s, zfast,
               cmaj);
      QMG_LAUNCH_CHECK();
      return;
    }
  }
  if (a.dagger)
    launch(k_dslash_t<S, TCH, NR, true>, grid, dim3(kBlock), 0, st, U, in, out, a, ntile_s, zfast, cmaj);
  else
    launch(k_dslash_t<S, TCH, NR, false>, grid, dim3(kBlock), 0, st, U, in, out, a, ntile_s, zfast, cmaj);
  QMG_LAUNCH_CHECK();
}

// Multi-RHS t-walking forms, code 1000 * zfast + 100 * NR + TCH (NR = 2 or 3 right-hand sides
// per thread; FP32 storage only: the NR accumulators, own spinors and carried hops take
// 190-250 VGPRs)
inline bool twx_code(int v) {
  const int z = v / 1000, nr = (v % 1000) / 100, tch = v % 100;
  return v > 100 && z <= 1 && (nr == 2 || nr == 3) && (tch == 2 || tch == 4 || tch == 8);
}

template <class S>
void run_twx(int v, const void* U, const void* in, void* out, const DslashArgs& a, hipStream_t st, int cm) {
  if constexpr (sizeof(S) != 8) {
    set_error("dslash launch form %d needs FP32 storage", v);
  } else {
    const int z = v / 1000, nr = (v % 1000) / 100, tch = v % 100;
    auto go = [&](auto nrc) {
      constexpr int NR = decltype(nrc)::value;
      if (tch == 2) launch_tw<S, 2, NR>(U, in, out, a, z, st, cm);
      else if (tch == 4) launch_tw<S, 4, NR>(U, in, out, a, z, st, cm);
      else launch_tw<S, 8, NR>(U, in, out, a, z, st, cm);
    };
    if (nr == 2) go(std::integral_constant<int, 2>{});
    else go(std::integral_constant<int, 3>{});
  }
}

template <class S>
void launch_s(const void* U, const void* in, void* out, const DslashArgs& a, hipStream_t st) {
  const bool clov = a.clov != nullptr;
  // algorithmic traffic: spinor in + out (2 x 12 complex per site and rhs) + 4 links per site
  // (+ the site term's 2 x 18 complex entries with the clover term); flops: 1368 per site and
  // rhs for the stencil, 504 more for the two 6 x 6 hermitian blocks
  const double cb = double(sizeof(S));
  const double bytes = double(a.V) * (24.0 * a.nrhs + 36.0 + (clov ? 36.0 : 0.0)) * cb;
  const double flops = (clov ? 1872.0 : 1368.0) * a.V * a.nrhs;
  if (a.canonical) {
    TimedLaunch tl(clov ? "clover/canonical" : "dslash/canonical", st, bytes, flops);
    launch_t<S, true, 1>(U, in, out, a, st);
    return;
  }
  // Launch variants for the native layout: 1 = one site per thread, 2/4/8 = t-walking with
  // that many sites per thread along t, 16 = direction-split (four threads per site), 32/64 =
  // one site per thread for 2/4 right-hand sides at once (links loaded once for all of them),
  // 1000 z + 100 NR + TCH = t-walking with NR = 2 or 3 right-hand sides per thread (FP32; z:
  // z-fastest tile order); 10000 + a t-walking code: the same in t-chunk-major workgroup order.  Default heuristic: for several right-hand sides in FP32 the
  // multi-RHS t-walk (3 per thread when nrhs is a multiple of 3, else 2); otherwise the longest
  // t-chunk that still gives >= 1024 workgroups, else the direction split when one thread per
  // site would leave the GPU short of wavefronts.  With the autotuner enabled every valid
  // variant is timed on first use of (precision, extents, nrhs, adjoint) and the fastest is
  // kept.  With the clover term: forms 1, 16, 2, 4, 8 and the multi-RHS t-walks (FP32 and FP64
  // storage), the direction split alone for BF16/FP16 storage.
  const int Vs = a.L[0] * a.L[1] * a.L[2];
  const long wg1 = long((Vs + kBlock - 1) / kBlock) * a.nrhs;  // workgroups per t-slice
  const int Lt = a.L[3];
  auto run = [&](int v) {
    const int cm = v / 10000;  // 10000 + code: the t-walks in t-chunk-major workgroup order
    v %= 10000;
    const int f = v == 16 ? 0 : (v == 1 || v == 32 || v == 64) ? 1 : 2;
    static const char* const fams[2][3] = {{"dslash/dir", "dslash/site", "dslash/twalk"},
                                           {"clover/dir", "clover/site", "clover/twalk"}};
    TimedLaunch tl(fams[clov ? 1 : 0][f], st, bytes, flops);
    switch (v) {
      case 8: launch_tw<S, 8, 1>(U, in, out, a, 0, st, cm); break;
      case 4: launch_tw<S, 4, 1>(U, in, out, a, 0, st, cm); break;
      case 2: launch_tw<S, 2, 1>(U, in, out, a, 0, st, cm); break;
      case 16: launch_dir<S>(U, in, out, a, st); break;
      case 32: launch_t<S, false, 2>(U, in, out, a, st); break;
      case 64: launch_t<S, false, 4>(U, in, out, a, st); break;
      default:
        if (v > 100) run_twx<S>(v, U, in, out, a, st, cm);
        else launch_t<S, false, 1>(U, in, out, a, st);
        break;
    }
  };
  auto valid = [&](int v) {
    if (v >= 10000) {
      v -= 10000;
      if (v < 2 || v == 16 || v == 32 || v == 64 || v >= 10000) return false;
    }
    if (v == 16) return true;
    if (clov && (sizeof(S) == 4 || v == 32 || v == 64)) return false;
    if (v == 1) return true;
    if (v == 32) return a.nrhs % 2 == 0;
    if (v == 64) return a.nrhs % 4 == 0;
    if (v > 100) {
      const int nr = (v % 1000) / 100, tch = v % 100;
      return sizeof(S) == 8 && twx_code(v) && a.nrhs % nr == 0 && Lt % tch == 0;
    }
    return (v == 2 || v == 4 || v == 8) && Lt % v == 0;
  };
  if (a.tchunk > 0 && valid(a.tchunk)) {
    run(a.tchunk);
    return;
  }
  auto fits = [&](int tch) { return Lt % tch == 0 && wg1 * (Lt / tch) >= 1024; };
  // one thread per site fills 256 CUs x 32 wavefronts only from 2^18 sites x rhs on
  const bool small = long(a.V) * a.nrhs < (1L << 19);
  int choice = fits(8) ? 8 : fits(4) ? 4 : fits(2) ? 2 : small ? 16 : 1;
  // 4-byte storage (BF16/FP16): the one-thread-per-site forms hold every hop's loads in
  // registers (up to 256 VGPRs, one wavefront per SIMD); the direction split needs 64-70
  if (sizeof(S) == 4) choice = 16;
  if (!valid(choice)) choice = 16;
  if (sizeof(S) == 8 && a.nrhs >= 2) {
    // measured at 16^3x32 (8 rhs), 24^3x64 (16) and 32^3x64 (12): 10-20% faster than the
    // one-rhs-per-thread forms; z-fastest tiles only where 256-site pieces tile an xy-plane
    const int nr = a.nrhs % 3 == 0 ? 3 : a.nrhs % 2 == 0 ? 2 : 0;
    const int z = (a.L[0] * a.L[1]) % kBlock == 0 ? 1 : 0;
    const int tch = (nr == 3 && Lt % 8 == 0) ? 8 : Lt % 4 == 0 ? 4 : 2;
    if (nr && valid(1000 * z + 100 * nr + tch)) choice = 1000 * z + 100 * nr + tch;
  }
  // t-walks in t-chunk-major order: every XCD works on the same t-chunk, so the neighbour
  // re-reads that miss an XCD's L2 meet the chunk in the last-level cache (measured at
  // 32^3x64: 4 rhs 824 -> 773 us, 1 and 12 rhs within 2-4%)
  if ((choice == 2 || choice == 4 || choice == 8 || choice > 100) && valid(10000 + choice)) choice += 10000;
  if (tune_enabled()) {
    const std::string key = "dslash/" + std::to_string(int(StoreTraits<S>::prec)) + "/" + std::to_string(a.L[0]) +
                            "x" + std::to_string(a.L[1]) + "x" + std::to_string(a.L[2]) + "x" +
                            std::to_string(a.L[3]) + "/" + std::to_string(a.nrhs) + "/" + std::to_string(a.dagger) +
                            (clov ? "/clover" : "");
    const int cached = tune_lookup(key);
    if (cached > 0) {
      choice = cached;
    } else {
      int cand[48], n = 0;
      for (int v : {1, 16, 2, 4, 8, 32, 64, 202, 204, 208, 302, 304, 308, 1202, 1204, 1208, 1302, 1304, 1308})
        for (int c : {0, 10000})
          if ((c == 0 || (v != 1 && v != 16 && v != 32 && v != 64)) && valid(c + v)) cand[n++] = c + v;
      choice = tune_measure(key, cand, n, st, run);
    }
  }
  run(choice);
}


// ---------------------------------------------------------------------------------------
// Even-odd (Schur complement) forms on half-lattice fields.  Every extent is even; a site of
// parity p = (x + y + z + t) mod 2 has the half-lattice index i = lex / 2, so within a row of
// fixed (y, z, t) the sites of one parity are every other x.  Layouts: spinor [rhs][12][V/2]
// per parity, gauge [parity][mu][9][V/2] (U_mu(x) stored at x's parity), site term and its
// inverse [parity][alpha][18][V/2] in the packed form of clover_acc (nullptr: the scalar
// diagonal term of the Wilson operator).

// out (parity p) = POST( YM(y) + sgn * H in ), H the hopping part of D (of D^dag with DAG),
// in on parity 1 - p.  YM: 0 nothing, 1 y, 2 A_p y.  POST: 0 nothing, 1 A_p^-1.
// Each thread forms NR right-hand sides rhs_base + NR g .. + NR - 1 of its site, so every link
// is loaded once for all NR of them; the NR-groups of a tile are adjacent in the (XCD-aware)
// workgroup order, so the groups of one tile run on one XCD and meet its links in that L2.
template <class S, bool DAG, int YM, int POST, int NE = 9, int NR = 1>
__global__ __launch_bounds__(kBlock) void k_hop_eo(const S* __restrict__ Ue, const S* __restrict__ Uo,
                                                   const S* __restrict__ in, const S* __restrict__ y,
                                                   S* __restrict__ out, const S* __restrict__ Ap,
                                                   const S* __restrict__ Aip, DslashArgs a, int p, float sgn,
                                                   int rhs_base, int ngroup, int bzt) {
  using C = ctype<S>;
  const int Vh = a.V >> 1;
  const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  const int wg = xcd_tile(blockIdx.x, gridDim.x);
  int tile = wg / ngroup;
  const int rhs = rhs_base + NR * (wg % ngroup);
  if (bzt) {
    // blocked order over the (z, t) planes: the tiles of a patch of BZ planes x BT slices are
    // adjacent in the schedule (t fastest, then z, then the tiles of a plane), so the slices a
    // site's t-hops read are loaded by tiles running close in time (lexicographic order runs a
    // whole t-slice between them); needs whole tiles per plane, BZ | L2 and BT | L3
    const int BZ = bzt & 0xff, BT = bzt >> 8, tpp = (L0 * L1) / (2 * kBlock);
    const int h = tile % tpp;
    int r = tile / tpp;
    const int tt = r % BT;
    r /= BT;
    const int zz = r % BZ;
    r /= BZ;
    const int nbz = L2 / BZ;
    tile = h + tpp * ((r % nbz) * BZ + zz + L2 * ((r / nbz) * BT + tt));
  }
  const int i = tile * kBlock + threadIdx.x;
  if (i >= Vh) return;
  const int Lxh = L0 >> 1;
  const int xh = i % Lxh;
  int row = i / Lxh;
  const int yy = row % L1;
  row /= L1;
  const int z = row % L2;
  const int t = row / L2;
  const int x = 2 * xh + ((yy + z + t + p) & 1);
  auto cb = [&](int cx, int cy, int cz, int ct) { return (cx + L0 * (cy + L1 * (cz + L2 * ct))) >> 1; };
  const int xp = cb(x + 1 == L0 ? 0 : x + 1, yy, z, t), xm = cb(x == 0 ? L0 - 1 : x - 1, yy, z, t);
  const int yp = cb(x, yy + 1 == L1 ? 0 : yy + 1, z, t), ym = cb(x, yy == 0 ? L1 - 1 : yy - 1, z, t);
  const int zp = cb(x, yy, z + 1 == L2 ? 0 : z + 1, t), zm = cb(x, yy, z == 0 ? L2 - 1 : z - 1, t);
  const int tp = cb(x, yy, z, t + 1 == L3 ? 0 : t + 1), tm = cb(x, yy, z, t == 0 ? L3 - 1 : t - 1);
  const S* Uown = p ? Uo : Ue;  // links leaving this site
  const S* Uoth = p ? Ue : Uo;  // links arriving from the backward neighbours
  C cw[4], diag;
  if constexpr (sizeof(C) == 8) {
    for (int m = 0; m < 4; ++m) cw[m] = a.cw_d[m];
    diag = a.diag_d;
  } else {
    for (int m = 0; m < 4; ++m) cw[m] = a.cw_f[m];
    diag = a.diag_f;
  }
  const C bt_f = (a.bc_t < 0 && t == L3 - 1) ? C(-1) : C(1);
  const C bt_b = (a.bc_t < 0 && t == 0) ? C(-1) : C(1);
  cplx<C> w[NR][12];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) w[r][k] = {C(0), C(0)};
  const C mh = C(-0.5) * C(sgn);
  do_hop<S, false, NR, 0, true, DAG, NE>(Uown, in, w, i, xp, rhs, Vh, mh * cw[0]);
  do_hop<S, false, NR, 0, false, DAG, NE>(Uoth, in, w, xm, xm, rhs, Vh, mh * cw[0]);
  do_hop<S, false, NR, 1, true, DAG, NE>(Uown, in, w, i, yp, rhs, Vh, mh * cw[1]);
  do_hop<S, false, NR, 1, false, DAG, NE>(Uoth, in, w, ym, ym, rhs, Vh, mh * cw[1]);
  do_hop<S, false, NR, 2, true, DAG, NE>(Uown, in, w, i, zp, rhs, Vh, mh * cw[2]);
  do_hop<S, false, NR, 2, false, DAG, NE>(Uoth, in, w, zm, zm, rhs, Vh, mh * cw[2]);
  do_hop<S, false, NR, 3, true, DAG, NE>(Uown, in, w, i, tp, rhs, Vh, mh * cw[3] * bt_f);
  do_hop<S, false, NR, 3, false, DAG, NE>(Uoth, in, w, tm, tm, rhs, Vh, mh * cw[3] * bt_b);
  if constexpr (YM == 1) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int k = 0; k < 12; ++k) w[r][k] += ldc(y, sp_idx<false>(rhs + r, k, i, Vh));
  } else if constexpr (YM == 2) {
    if (Ap) {
      cplx<C> yv[NR][12];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) yv[r][k] = ldc(y, sp_idx<false>(rhs + r, k, i, Vh));
      clover_acc<S, NR>(Ap, i, Vh, yv, w);
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) w[r][k] += diag * ldc(y, sp_idx<false>(rhs + r, k, i, Vh));
    }
  }
  if constexpr (POST == 1) {
    if (Aip) {
      cplx<C> o[NR][12];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) o[r][k] = {C(0), C(0)};
      clover_acc<S, NR>(Aip, i, Vh, w, o);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) w[r][k] = o[r][k];
    } else {
      const C inv = C(1) / diag;
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) w[r][k] = inv * w[r][k];
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) stc_stream(out, sp_idx<false>(rhs + r, k, i, Vh), w[r][k]);
}

// Rows I0 .. I0+2 of one chirality of the even-odd epilogue: x holds sgn H in (+ y with YM = 1)
// on the six components of the chirality; YM = 2 adds A_p y, POST = 1 applies A_p^-1
template <class S, int YM, int POST, int I0>
__device__ inline void eo_rows(const S* __restrict__ Ab, const S* __restrict__ Aib, const S* __restrict__ y,
                               size_t ybase, int Vh, ctype<S> diag, cplx<ctype<S>> (&x)[6], cplx<ctype<S>> (&r)[3]) {
  using C = ctype<S>;
  if constexpr (YM == 2) {
    cplx<C> yv[6], ay[3];
#pragma unroll
    for (int j = 0; j < 6; ++j) yv[j] = ldc(y, ybase + size_t(j) * Vh);
    if (Ab) {
      site_term_rows<S, I0>(Ab, Vh, yv, ay);
    } else {
#pragma unroll
      for (int q = 0; q < 3; ++q) ay[q] = diag * yv[I0 + q];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) r[q] = x[I0 + q] + ay[q];
  } else if constexpr (POST == 1) {
    if (Aib) {
      site_term_rows<S, I0>(Aib, Vh, x, r);
    } else {
      const C inv = C(1) / diag;
#pragma unroll
      for (int q = 0; q < 3; ++q) r[q] = inv * x[I0 + q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 3; ++q) r[q] = x[I0 + q];
  }
}

// Direction-split form of k_hop_eo for half lattices too small to fill the GPU with one thread
// per site: a workgroup covers 64 half-lattice sites, wavefront mu forms the two hops along mu,
// the partial spinors meet in LDS, and wavefront w then finishes output components
// 3w .. 3w+2 (rows 3 (w & 1) .. +2 of chirality w >> 1) with the epilogue of k_hop_eo.
template <class S, bool DAG, int YM, int POST, int NE = 9>
__global__ __launch_bounds__(kBlock) void k_hop_eo_dir(const S* __restrict__ Ue, const S* __restrict__ Uo,
                                                       const S* __restrict__ in, const S* __restrict__ y,
                                                       S* __restrict__ out, const S* __restrict__ Ap,
                                                       const S* __restrict__ Aip, DslashArgs a, int p, float sgn) {
  using C = ctype<S>;
  constexpr int TS = kBlock / 4;
  __shared__ cplx<C> part[4][12][TS];
  const int Vh = a.V >> 1;
  const int ntile = (Vh + TS - 1) / TS;
  const int wg = xcd_tile(blockIdx.x, gridDim.x);
  const int tile = wg % ntile, rhs = wg / ntile;
  const int lane = threadIdx.x & (TS - 1), mu = threadIdx.x / TS;
  const int i = tile * TS + lane;
  const bool live = i < Vh;
  const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  C cw, diag;
  if constexpr (sizeof(C) == 8) {
    cw = a.cw_d[mu];
    diag = a.diag_d;
  } else {
    cw = a.cw_f[mu];
    diag = a.diag_f;
  }
  cplx<C> acc[1][12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[0][k] = {C(0), C(0)};
  if (live) {
    const int Lxh = L0 >> 1;
    const int xh = i % Lxh;
    int row = i / Lxh;
    const int yy = row % L1;
    row /= L1;
    const int z = row % L2;
    const int t = row / L2;
    int c[4] = {2 * xh + ((yy + z + t + p) & 1), yy, z, t};
    const int L = a.L[mu];
    const int cmu = c[mu];
    auto cb = [&](int v) {
      int d[4] = {c[0], c[1], c[2], c[3]};
      d[mu] = v;
      return (d[0] + L0 * (d[1] + L1 * (d[2] + L2 * d[3]))) >> 1;
    };
    const int fp = cb(cmu + 1 == L ? 0 : cmu + 1), bm = cb(cmu == 0 ? L - 1 : cmu - 1);
    const C mh = C(-0.5);
    C cf = mh * cw, cbk = mh * cw;
    if (mu == 3 && a.bc_t < 0) {
      if (t == L3 - 1) cf = -cf;
      if (t == 0) cbk = -cbk;
    }
    const S* Uown = p ? Uo : Ue;
    const S* Uoth = p ? Ue : Uo;
    switch (mu) {  // uniform within the wavefront
      case 0:
        do_hop<S, false, 1, 0, true, DAG, NE>(Uown, in, acc, i, fp, rhs, Vh, cf);
        do_hop<S, false, 1, 0, false, DAG, NE>(Uoth, in, acc, bm, bm, rhs, Vh, cbk);
        break;
      case 1:
        do_hop<S, false, 1, 1, true, DAG, NE>(Uown, in, acc, i, fp, rhs, Vh, cf);
        do_hop<S, false, 1, 1, false, DAG, NE>(Uoth, in, acc, bm, bm, rhs, Vh, cbk);
        break;
      case 2:
        do_hop<S, false, 1, 2, true, DAG, NE>(Uown, in, acc, i, fp, rhs, Vh, cf);
        do_hop<S, false, 1, 2, false, DAG, NE>(Uoth, in, acc, bm, bm, rhs, Vh, cbk);
        break;
      default:
        do_hop<S, false, 1, 3, true, DAG, NE>(Uown, in, acc, i, fp, rhs, Vh, cf);
        do_hop<S, false, 1, 3, false, DAG, NE>(Uoth, in, acc, bm, bm, rhs, Vh, cbk);
        break;
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) part[mu][k][lane] = acc[0][k];
  __syncthreads();
  if (!live) return;
  const int al = mu >> 1;
  const C sg = C(sgn);
  cplx<C> x6[6], r[3];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int k = 6 * al + j;
    cplx<C> h = part[0][k][lane];
#pragma unroll
    for (int m = 1; m < 4; ++m) h += part[m][k][lane];
    x6[j] = sg * h;
    if constexpr (YM == 1) x6[j] += ldc(y, sp_idx<false>(rhs, k, i, Vh));
  }
  const size_t ybase = sp_idx<false>(rhs, 6 * al, i, Vh);
  const S* Ab = Ap ? Ap + size_t(al) * 18 * Vh + i : nullptr;
  const S* Aib = Aip ? Aip + size_t(al) * 18 * Vh + i : nullptr;
  if (mu & 1) eo_rows<S, YM, POST, 3>(Ab, Aib, y, ybase, Vh, diag, x6, r);
  else eo_rows<S, YM, POST, 0>(Ab, Aib, y, ybase, Vh, diag, x6, r);
#pragma unroll
  for (int q = 0; q < 3; ++q) stc(out, sp_idx<false>(rhs, 3 * mu + q, i, Vh), r[q]);
}

// out = M in on one parity's half field, M the packed site term (or its inverse) of that
// parity, or the scalar diag (or 1 / diag) when M is nullptr
template <class S, bool INV>
__global__ __launch_bounds__(kBlock) void k_site_eo(const S* __restrict__ M, const S* __restrict__ in,
                                                    S* __restrict__ out, DslashArgs a) {
  using C = ctype<S>;
  const int Vh = a.V >> 1;
  const int ntile = (Vh + kBlock - 1) / kBlock;
  const int wg = blockIdx.x;
  const int tile = wg % ntile, rhs = wg / ntile;
  const int i = tile * kBlock + threadIdx.x;
  if (i >= Vh) return;
  cplx<C> v[1][12], r[1][12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    v[0][k] = ldc(in, sp_idx<false>(rhs, k, i, Vh));
    r[0][k] = {C(0), C(0)};
  }
  if (M) {
    clover_acc<S, 1>(M, i, Vh, v, r);
  } else {
    const C d = sizeof(C) == 8 ? C(a.diag_d) : C(a.diag_f);
    const C f = INV ? C(1) / d : d;
#pragma unroll
    for (int k = 0; k < 12; ++k) r[0][k] = f * v[0][k];
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) stc(out, sp_idx<false>(rhs, k, i, Vh), r[0][k]);
}

}  // namespace

void launch_dslash_batched(qmg_prec prec, const BatchLattice* lat_dev, int n_lat, int total_tiles,
                           const void* const* U, const void* const* in, void* const* out, bool dagger,
                           double bytes, double flops, hipStream_t st) {
  TimedLaunch tl("dslash/batched", st, bytes, flops);
  auto go = [&](auto tag) {
    using S = decltype(tag);
    if (dagger)
      launch(k_dslash_batched<S, true>, dim3(total_tiles), dim3(kBlock), 0, st, lat_dev, n_lat, U, in, out);
    else
      launch(k_dslash_batched<S, false>, dim3(total_tiles), dim3(kBlock), 0, st, lat_dev, n_lat, U, in, out);
  };
  switch (prec) {
    case QMG_F64: go(double2{}); break;
    case QMG_F32: go(float2{}); break;
    case QMG_BF16: go(cbf16{}); break;
    case QMG_F16: go(chalf{}); break;
  }
  QMG_LAUNCH_CHECK();
}

void launch_dslash_padded(qmg_prec prec, const BatchLattice* lat_dev, int nl, int nr, int Vpad, const void* U,
                          const void* in, void* out, bool dagger, double bytes, double flops, hipStream_t st) {
  TimedLaunch tl("batch/dslash", st, bytes, flops);
  const int ntile = (Vpad + kBlock - 1) / kBlock;
  auto go = [&](auto tag) {
    using S = decltype(tag);
    auto run = [&](auto nrc) {
      constexpr int NR = decltype(nrc)::value;
      const dim3 g(unsigned(ntile) * unsigned(nl) * unsigned(nr / NR));
      if (dagger)
        launch(k_dslash_padded<S, true, NR>, g, dim3(kBlock), 0, st, lat_dev, static_cast<const S*>(U),
               static_cast<const S*>(in), static_cast<S*>(out), nr, ntile);
      else
        launch(k_dslash_padded<S, false, NR>, g, dim3(kBlock), 0, st, lat_dev, static_cast<const S*>(U),
               static_cast<const S*>(in), static_cast<S*>(out), nr, ntile);
    };
    // several right-hand sides per thread in FP32 storage (the setup's test-vector batches)
    if constexpr (sizeof(S) == 8) {
      if (nr % 4 == 0) return run(std::integral_constant<int, 4>{});
      if (nr % 2 == 0) return run(std::integral_constant<int, 2>{});
    }
    run(std::integral_constant<int, 1>{});
  };
  switch (prec) {
    case QMG_F64: go(double2{}); break;
    case QMG_F32: go(float2{}); break;
    case QMG_BF16: go(cbf16{}); break;
    case QMG_F16: go(chalf{}); break;
  }
  QMG_LAUNCH_CHECK();
}

void launch_dslash(qmg_prec prec, const void* U, const void* in, void* out, const DslashArgs& a,
                   hipStream_t st) {
  switch (prec) {
    case QMG_F64: launch_s<double2>(U, in, out, a, st); break;
    case QMG_F32: launch_s<float2>(U, in, out, a, st); break;
    case QMG_BF16: launch_s<cbf16>(U, in, out, a, st); break;
    case QMG_F16: launch_s<chalf>(U, in, out, a, st); break;
  }
}

// right-hand sides per thread of the even-odd hop for several right-hand sides (links loaded
// once for all of them)
constexpr int kHopNR = 2;
// (z, t) patch of the hop's blocked tile order for two or more right-hand sides (measured at
// 32^3 x 64 FP32, four right-hand sides: 4 x 4 planes 522 us per launch against 543-551 us in
// lexicographic order, the other patches with 4 or 8 slices within 1 %; at one right-hand side
// the blocked orders are slower, 191 against 197-215 us, so it keeps the lexicographic order)
constexpr int kHopBZ = 4, kHopBT = 4;

void launch_hop_eo(qmg_prec prec, const DslashArgs& a, const void* Ue, const void* Uo, int p, const void* in,
                   const void* y, void* out, const void* Ap, const void* Aip, int ym, int post, double sgn,
                   hipStream_t st) {
  const int Vh = a.V / 2;
  // direction split for the clover forms on half lattices too small to fill the GPU with one
  // thread per site (measured FP32, one RHS: clover 23.1 against 25.1 us at 16^3 x 32 and 43.4
  // against 48.7 us at 24^3 x 32; the Wilson forms are faster one site per thread at every size,
  // 12.3 against 21.3 us at 16^3 x 32).  Forced with the launch-variant codes 1 = one site per
  // thread, 16 = direction split.
  // The same holds for BF16/FP16 storage (BF16 at 16^3 x 32: Wilson 8.7 against 17.8 us, clover
  // 21.0 against 18.5 us; the forms tie at 24^3 x 64).
  const bool with_site_term = (ym == 2 && Ap) || (post == 1 && Aip);
  const bool split =
      a.tchunk == 16 || (a.tchunk != 1 && with_site_term && long(Vh) * a.nrhs < (1L << 19));
  const int per_wg = split ? kBlock / 4 : kBlock;
  const unsigned ntile = unsigned((Vh + per_wg - 1) / per_wg);
  const dim3 grid(ntile * unsigned(a.nrhs));
  // right-hand sides per thread of the one-site-per-thread form: forced with the launch-variant
  // codes 501 .. 504, else HOP_NR (FP32 storage and below) once there are enough of them
  int nr = 1;
  if (!split) {
    if (a.tchunk >= 501 && a.tchunk <= 504) nr = a.tchunk - 500;
    else if (prec != QMG_F64 && a.nrhs >= 2) nr = std::min(a.nrhs, kHopNR);
  }
  // tile order of the one-site-per-thread form: blocked over patches of BZ x BT (z, t) planes
  // where whole tiles fill a plane (kHopBZ x kHopBT from two right-hand sides on, or forced
  // with the launch-variant codes 7ZT: BZ = Z, BT = T planes; 700 = lexicographic)
  int bz = a.nrhs >= 2 ? kHopBZ : 0, bt = a.nrhs >= 2 ? kHopBT : 0;
  if (a.tchunk >= 700 && a.tchunk < 800) {
    bz = (a.tchunk / 10) % 10;
    bt = a.tchunk % 10;
  }
  const bool blocked = !split && bz > 0 && bt > 0 && (a.L[0] * a.L[1]) % (2 * kBlock) == 0 && a.L[2] % bz == 0 &&
                       a.L[3] % bt == 0;
  const int bzt = blocked ? bz | (bt << 8) : 0;
  // algorithmic traffic: the other parity's spinors and both parities' links once per site of
  // this parity, y when used, the output, and the packed blocks when used
  const double cb = double(prec_bytes(prec));
  const double bytes = double(Vh) * (a.nrhs * (12.0 + 12.0 + (ym ? 12.0 : 0.0)) + 8.0 * a.link_ne +
                                     ((ym == 2 && Ap) ? 36.0 : 0.0) + ((post && Aip) ? 36.0 : 0.0)) * cb;
  // full groups of nr right-hand sides and a one-per-thread rest are two launches: time the pair
  // as one (events on the stream around both) rather than the first launch alone
  const bool two = nr > 1 && a.nrhs >= nr && a.nrhs % nr != 0;
  TimedLaunch tl("evenodd/hop", st, bytes, 1320.0 * Vh * a.nrhs, !two);
  auto go = [&](auto tag) {
    using S = decltype(tag);
    auto run = [&](auto kern) {
      launch(kern, grid, dim3(kBlock), 0, st, static_cast<const S*>(Ue), static_cast<const S*>(Uo),
             static_cast<const S*>(in), static_cast<const S*>(y), static_cast<S*>(out), static_cast<const S*>(Ap),
             static_cast<const S*>(Aip), a, p, float(sgn));
    };
    // one-site-per-thread form: full groups of NR right-hand sides, then the rest one per thread
    auto run_nr = [&](auto k_nr, auto k_1) {
      const int ng = a.nrhs / nr, done = ng * nr;
      auto go1 = [&](auto kern, int base, int groups) {
        launch(kern, dim3(ntile * unsigned(groups)), dim3(kBlock), 0, st, static_cast<const S*>(Ue),
               static_cast<const S*>(Uo), static_cast<const S*>(in), static_cast<const S*>(y), static_cast<S*>(out),
               static_cast<const S*>(Ap), static_cast<const S*>(Aip), a, p, float(sgn), base, groups, bzt);
      };
      if (nr > 1 && ng > 0) go1(k_nr, 0, ng);
      if (nr == 1) go1(k_1, 0, a.nrhs);
      else if (done < a.nrhs) go1(k_1, done, a.nrhs - done);
    };
    const int form = ym * 2 + post;  // forms used by the Schur operator, the source and the reconstruction
    auto pick = [&](auto dag, auto ne) {
      constexpr bool D = decltype(dag)::value;
      constexpr int NE = decltype(ne)::value;
      if (split) {
        if (form == 1) run(k_hop_eo_dir<S, D, 0, 1, NE>);
        else if (form == 4) run(k_hop_eo_dir<S, D, 2, 0, NE>);
        else if (form == 2) run(k_hop_eo_dir<S, D, 1, 0, NE>);
        else run(k_hop_eo_dir<S, D, 1, 1, NE>);
        return;
      }
      auto by_nr = [&](auto ym_c, auto post_c) {
        constexpr int YM = decltype(ym_c)::value, PO = decltype(post_c)::value;
        auto k1 = k_hop_eo<S, D, YM, PO, NE, 1>;
        if (nr == 2) run_nr(k_hop_eo<S, D, YM, PO, NE, 2>, k1);
        else if (nr == 3) run_nr(k_hop_eo<S, D, YM, PO, NE, 3>, k1);
        else if (nr == 4) run_nr(k_hop_eo<S, D, YM, PO, NE, 4>, k1);
        else run_nr(k1, k1);
      };
      using I0 = std::integral_constant<int, 0>;
      using I1 = std::integral_constant<int, 1>;
      using I2 = std::integral_constant<int, 2>;
      if (form == 1) by_nr(I0{}, I1{});
      else if (form == 4) by_nr(I2{}, I0{});
      else if (form == 2) by_nr(I1{}, I0{});
      else by_nr(I1{}, I1{});
    };
    using N9 = std::integral_constant<int, 9>;
    using N6 = std::integral_constant<int, 6>;
    if (a.link_ne == 6) {
      if (a.dagger) pick(std::true_type{}, N6{});
      else pick(std::false_type{}, N6{});
    } else {
      if (a.dagger) pick(std::true_type{}, N9{});
      else pick(std::false_type{}, N9{});
    }
  };
  QMG_CHECK((ym == 0 && post == 1) || (ym == 2 && post == 0) || (ym == 1 && post == 0) || (ym == 1 && post == 1),
            QMG_EINVAL, "even-odd hop form (%d, %d) is not built", ym, post);
  switch (prec) {
    case QMG_F64: go(double2{}); break;
    case QMG_F32: go(float2{}); break;
    case QMG_BF16: go(cbf16{}); break;
    case QMG_F16: go(chalf{}); break;
  }
  QMG_LAUNCH_CHECK();
}

void launch_site_eo(qmg_prec prec, const DslashArgs& a, const void* M, bool inv, const void* in, void* out,
                    hipStream_t st) {
  const int Vh = a.V / 2;
  const dim3 grid(unsigned((Vh + kBlock - 1) / kBlock) * unsigned(a.nrhs));
  auto go = [&](auto tag) {
    using S = decltype(tag);
    if (inv)
      launch(k_site_eo<S, true>, grid, dim3(kBlock), 0, st, static_cast<const S*>(M), static_cast<const S*>(in),
             static_cast<S*>(out), a);
    else
      launch(k_site_eo<S, false>, grid, dim3(kBlock), 0, st, static_cast<const S*>(M), static_cast<const S*>(in),
             static_cast<S*>(out), a);
  };
  switch (prec) {
    case QMG_F64: go(double2{}); break;
    case QMG_F32: go(float2{}); break;
    case QMG_BF16: go(cbf16{}); break;
    case QMG_F16: go(chalf{}); break;
  }
  QMG_LAUNCH_CHECK();
}

}  // namespace qmg
