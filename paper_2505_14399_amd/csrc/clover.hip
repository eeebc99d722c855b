// The clover term T(x) of the Wilson-clover operator and the packed site term
// A(x) = (m + 1 + 3/xi) 1 + T(x) that the dslash kernels apply in their epilogue.
//
// T(x) = sum over the six planes mu < nu of c_{mu nu} (i/2) sigma_{mu nu} (x) Fhat_{mu nu}(x), the
// O(a)-improvement term of Luescher, Sint, Sommer and Weisz in the normalisation of the Wilson
// operator used here; Fhat = (Q - Q^dag)/8 with Q the four plaquettes ("leaves") of the plane
// with a corner at x, all walked counter-clockwise (mu before nu); c_{mu nu} = c_t for planes
// that contain t, c_s for the three spatial planes.  In the chiral basis
// gamma_mu = [[0, A_mu], [A_mu^dag, 0]] (A_k = -i sigma_k, A_t = 1), sigma_{mu nu} = i gamma_mu
// gamma_nu is block diagonal with blocks i A_mu A_nu^dag (alpha = 0) and i A_mu^dag A_nu
// (alpha = 1); working the products out gives, per chirality (s_0 = +1, s_1 = -1),
//   T_alpha = sigma_1 (x) G1 + sigma_2 (x) G2 + sigma_3 (x) G3,
//   G1 = (i/2)(-c_s F_yz + s_alpha c_t F_xt), G2 = (i/2)(c_s F_xz + s_alpha c_t F_yt),
//   G3 = (i/2)(-c_s F_xy + s_alpha c_t F_zt),
// each G hermitian (Fhat is anti-hermitian), so each chirality block is a hermitian 6 x 6
// matrix over (spin within the chirality, colour).
//
// Setup work in FP64: one thread per (site, plane) forms the leaves from the native gauge field
// (links at x and seven neighbours, twelve 3 x 3 products), then one thread per (site,
// chirality) assembles and packs the block.
#include "qmg_internal.hpp"
#include "timing.hpp"

namespace qmg {

namespace {

using Z = cplx<double>;

struct M3 {
  Z e[9];
};

__device__ inline M3 ld_link(const double2* __restrict__ U, int mu, int site, int V) {
  M3 m;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    const double2 v = U[(size_t(mu) * 9 + e) * V + site];
    m.e[e] = {v.x, v.y};
  }
  return m;
}

// a b, a b^dag, a^dag b
__device__ inline M3 mul_nn(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Z t = a.e[3 * i] * b.e[j];
      t += a.e[3 * i + 1] * b.e[3 + j];
      t += a.e[3 * i + 2] * b.e[6 + j];
      c.e[3 * i + j] = t;
    }
  return c;
}
__device__ inline M3 mul_nd(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Z t = a.e[3 * i] * conj(b.e[3 * j]);
      t += a.e[3 * i + 1] * conj(b.e[3 * j + 1]);
      t += a.e[3 * i + 2] * conj(b.e[3 * j + 2]);
      c.e[3 * i + j] = t;
    }
  return c;
}
__device__ inline M3 mul_dn(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Z t = cmul_conj(a.e[i], b.e[j]);
      t += cmul_conj(a.e[3 + i], b.e[3 + j]);
      t += cmul_conj(a.e[6 + i], b.e[6 + j]);
      c.e[3 * i + j] = t;
    }
  return c;
}

struct PlaneArgs {
  int L[4];
  int V;
};

// the six planes in the order xy, xz, xt, yz, yt, zt
__device__ inline void plane_dirs(int p, int& mu, int& nu) {
  mu = p < 3 ? 0 : (p < 5 ? 1 : 2);
  nu = p < 3 ? p + 1 : (p < 5 ? p - 1 : 3);
}

// F[(p * 9 + e) * V + x] = Fhat_p(x)
__global__ __launch_bounds__(256) void k_clover_leaves(const double2* __restrict__ U, double2* __restrict__ F,
                                                       PlaneArgs a) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  if (site >= a.V) return;
  const int p = blockIdx.y;
  int mu, nu;
  plane_dirs(p, mu, nu);
  int c[4], rem = site;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c[q] = rem % a.L[q];
    rem /= a.L[q];
  }
  // lexicographic index of x + dm mu + dn nu (periodic)
  auto at = [&](int dm, int dn) {
    int cc[4] = {c[0], c[1], c[2], c[3]};
    cc[mu] = (cc[mu] + dm + a.L[mu]) % a.L[mu];
    cc[nu] = (cc[nu] + dn + a.L[nu]) % a.L[nu];
    return cc[0] + a.L[0] * (cc[1] + a.L[1] * (cc[2] + a.L[2] * cc[3]));
  };
  const int V = a.V;
  const M3 um = ld_link(U, mu, site, V), un = ld_link(U, nu, site, V);
  M3 q;
  {  // x -> x+mu -> x+mu+nu -> x+nu -> x
    M3 t = mul_nn(um, ld_link(U, nu, at(1, 0), V));
    t = mul_nd(t, ld_link(U, mu, at(0, 1), V));
    q = mul_nd(t, un);
  }
  {  // x -> x+nu -> x+nu-mu -> x-mu -> x
    const int xm = at(-1, 0);
    M3 t = mul_nd(un, ld_link(U, mu, at(-1, 1), V));
    t = mul_nd(t, ld_link(U, nu, xm, V));
    t = mul_nn(t, ld_link(U, mu, xm, V));
#pragma unroll
    for (int e = 0; e < 9; ++e) q.e[e] += t.e[e];
  }
  {  // x -> x-mu -> x-mu-nu -> x-nu -> x: the first two steps are (U_nu(x-mu-nu) U_mu(x-mu))^dag
    const int xmm = at(-1, -1);
    const M3 w = mul_nn(ld_link(U, nu, xmm, V), ld_link(U, mu, at(-1, 0), V));
    M3 t = mul_dn(w, ld_link(U, mu, xmm, V));
    t = mul_nn(t, ld_link(U, nu, at(0, -1), V));
#pragma unroll
    for (int e = 0; e < 9; ++e) q.e[e] += t.e[e];
  }
  {  // x -> x-nu -> x-nu+mu -> x+mu -> x
    const int xn = at(0, -1);
    M3 t = mul_dn(ld_link(U, nu, xn, V), ld_link(U, mu, xn, V));
    t = mul_nn(t, ld_link(U, nu, at(1, -1), V));
    t = mul_nd(t, um);
#pragma unroll
    for (int e = 0; e < 9; ++e) q.e[e] += t.e[e];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const Z f = q.e[3 * i + j] - conj(q.e[3 * j + i]);
      F[(size_t(p) * 9 + 3 * i + j) * V + site] = make_double2(0.125 * f.re, 0.125 * f.im);
    }
}

struct AssembleArgs {
  int V;
  double diag, cs, ct;
};

// A[(alpha * 18 + e) * V + x]: the packed hermitian block of chirality alpha (blockIdx.y)
__global__ __launch_bounds__(256) void k_clover_assemble(const double2* __restrict__ F, double2* __restrict__ A,
                                                         AssembleArgs a) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  if (site >= a.V) return;
  const int al = blockIdx.y;
  const double sa = al == 0 ? 1.0 : -1.0;
  const int V = a.V;
  auto f = [&](int p, int e) {
    const double2 v = F[(size_t(p) * 9 + e) * V + site];
    return Z{v.x, v.y};
  };
  // G_k = (i/2) (spatial part + s_alpha temporal part); planes xy 0, xz 1, xt 2, yz 3, yt 4, zt 5
  Z G[3][9];
  const int sp[3] = {3, 1, 0}, tp[3] = {2, 4, 5};
  const double ss[3] = {-a.cs, a.cs, -a.cs};
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      const Z s = ss[k] * f(sp[k], e) + (sa * a.ct) * f(tp[k], e);
      G[k][e] = 0.5 * times_i(s);
    }
  // block entry (i, j), i = s * 3 + colour: sigma_1 G1 + sigma_2 G2 + sigma_3 G3
  auto entry = [&](int i, int j) {
    const int s = i / 3, ca = i % 3, t = j / 3, cb = j % 3;
    const int e = 3 * ca + cb;
    if (s == t) return s == 0 ? G[2][e] : -G[2][e];
    // (0,1): G1 - i G2 ; (1,0): G1 + i G2
    return s == 0 ? G[0][e] + times_mi(G[1][e]) : G[0][e] + times_i(G[1][e]);
  };
  double2* out = A + size_t(al) * 18 * V + site;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const double d0 = a.diag + entry(2 * e, 2 * e).re, d1 = a.diag + entry(2 * e + 1, 2 * e + 1).re;
    out[size_t(e) * V] = make_double2(d0, d1);
  }
  int e = 3;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j, ++e) {
      const Z v = entry(i, j);
      out[size_t(e) * V] = make_double2(v.re, v.im);
    }
}

}  // namespace

void launch_clover_field(const Geom& g, const void* U64, double cs, double ct, void* A64, hipStream_t st) {
  DevBuf F(size_t(6) * 9 * g.V * sizeof(double2));
  PlaneArgs pa{};
  for (int q = 0; q < 4; ++q) pa.L[q] = g.L[q];
  pa.V = g.V;
  const unsigned nb = unsigned((g.V + 255) / 256);
  {
    TimedLaunch tl_("setup/clover", st, double(g.V) * 6 * 9 * 16 * 4, 0.0);
    launch(k_clover_leaves, dim3(nb, 6), dim3(256), 0, st, static_cast<const double2*>(U64), F.as<double2>(), pa);
  }
  QMG_LAUNCH_CHECK();
  AssembleArgs aa{g.V, g.diag(), cs, ct};
  {
    TimedLaunch tl_("setup/clover", st, double(g.V) * (6 * 9 + 36) * 16, 0.0);
    launch(k_clover_assemble, dim3(nb, 2), dim3(256), 0, st, F.as<double2>(), static_cast<double2*>(A64), aa);
  }
  QMG_LAUNCH_CHECK();
  QMG_HIP(hipStreamSynchronize(st));  // F is released on return
}

}  // namespace qmg
