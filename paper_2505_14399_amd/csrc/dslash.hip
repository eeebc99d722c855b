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
// Launch: one thread per (site, group of NR right-hand sides), 256 threads per workgroup.
// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X; the tile index is
// remapped so that each XCD walks a contiguous range of sites, keeping the +-t neighbour
// slices of a tile inside that XCD's L2.
#include "qmg_internal.hpp"

namespace qmg {

DslashArgs make_dslash_args(const Geom& g, int nrhs, bool dagger, bool canonical) {
  DslashArgs a{};
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

template <class S, bool CANON, int NR, int MU, bool FWD, bool DAG>
__device__ inline void do_hop(const S* __restrict__ U, const S* __restrict__ in, cplx<ctype<S>> (*acc)[12],
                              int link_site, int nb_site, int rhs0, int V, ctype<S> coef) {
  using C = ctype<S>;
  cplx<C> u[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = ldc(U, g_idx<CANON>(MU, e, link_site, V));
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

template <class S, bool CANON, int NR, bool DAG>
__global__ __launch_bounds__(kBlock) void k_dslash(const S* __restrict__ U, const S* __restrict__ in,
                                                   S* __restrict__ out, DslashArgs a) {
  using C = ctype<S>;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int site = tile * kBlock + threadIdx.x;
  if (site >= a.V) return;
  const int rhs0 = blockIdx.y * NR;
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

template <class S, bool CANON, int NR>
void launch_t(const void* U, const void* in, void* out, const DslashArgs& a, hipStream_t st) {
  dim3 grid((a.V + kBlock - 1) / kBlock, a.nrhs / NR);
  if (a.dagger)
    k_dslash<S, CANON, NR, true><<<grid, kBlock, 0, st>>>((const S*)U, (const S*)in, (S*)out, a);
  else
    k_dslash<S, CANON, NR, false><<<grid, kBlock, 0, st>>>((const S*)U, (const S*)in, (S*)out, a);
  QMG_LAUNCH_CHECK();
}

template <class S>
void launch_s(const void* U, const void* in, void* out, const DslashArgs& a, hipStream_t st) {
  if (a.canonical) {
    launch_t<S, true, 1>(U, in, out, a, st);
    return;
  }
  if (a.nrhs % 4 == 0) launch_t<S, false, 4>(U, in, out, a, st);
  else if (a.nrhs % 2 == 0) launch_t<S, false, 2>(U, in, out, a, st);
  else launch_t<S, false, 1>(U, in, out, a, st);
}

}  // namespace

void launch_dslash(qmg_prec prec, const void* U, const void* in, void* out, const DslashArgs& a,
                   hipStream_t st) {
  switch (prec) {
    case QMG_F64: launch_s<double2>(U, in, out, a, st); break;
    case QMG_F32: launch_s<float2>(U, in, out, a, st); break;
    case QMG_BF16: launch_s<cbf16>(U, in, out, a, st); break;
    case QMG_F16: launch_s<chalf>(U, in, out, a, st); break;
  }
}

}  // namespace qmg
