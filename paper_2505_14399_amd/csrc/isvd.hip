// Streaming chiral SVD update (Algorithm 3, Eqs. (7)-(8)) for all (aggregate, chirality)
// problems of one stream, in FP64.
//
// For each problem the state is Phi_{s-1} = U Sigma (U: N x kp orthonormal) and the new block
// Psi (N x r).  The rank-k SVD of [U Sigma, Psi] is obtained without forming it:
//   X  = U^dag Psi,  R = Psi - U X,  X2 = U^dag R,  G = R^dag R        (Gram kernel: two row
//        passes, the projection done twice, i.e. classical Gram-Schmidt with one re-projection)
//   G2 = G - X2^dag X2 = T^dag T        (Cholesky; a column whose remaining norm falls below
//        1e-12 of its original norm is dropped: its row of T is zero)
//   [U Sigma, Psi] = [U, Q] K,  K = [[Sigma, X + X2], [0, T]],  Q = (Psi - U (X + X2)) T^-1
//   K = Y S Z^dag by one-sided Jacobi on the columns of K^dag with the rotations accumulated,
//        so Y (the left singular vectors of K) is unitary even where S is zero   (small kernel,
//        one wavefront per problem)
//   U_new = [U, Q] Y_k = U A + Psi B,   B = T^-1 Y_bot,   A = Y_top - (X + X2) B  (rotation
//        kernel, in place, row-local)
// Singular values are sorted descending with ties broken by the lower index.
//
// The row passes stream N rows through LDS in chunks of CH rows; the next chunk is prefetched
// into registers while the current one is used.  Each thread owns a 2 x 2 tile of the small
// output (up to four tiles when there are more tiles than threads) and a subset of the rows
// (split-K), the partial tiles are summed once per pass.
#include <algorithm>
#include <cmath>

#include "mg.hpp"
#include "timing.hpp"

namespace qmg {

namespace {

using cd = cplx<double>;
constexpr int T = 256;                 // threads of the row-pass kernels
constexpr int CH = 64;                 // rows per chunk
constexpr int CHP = CH + 1;            // padded LDS column stride
constexpr int MAXW = 64;               // k + r <= MAXW
constexpr int PF = (MAXW * CH) / T;    // prefetch registers per thread (complex), upper bound
constexpr double kJacobiTol = 1e-14;   // |<m_p, m_q>| <= tol |m_p| |m_q| counts as orthogonal

struct IsvdArgs {
  int nprob, N, k, r, kp, w, kn;
};

__device__ inline cd ld2(const double2* p, size_t i) {
  const double2 v = p[i];
  return {v.x, v.y};
}
__device__ inline void st2(double2* p, size_t i, cd v) { p[i] = make_double2(v.re, v.im); }

// scratch per problem: X [kp][r], X2 [kp][r], G [r][r], pn [r]   (complex)
__host__ __device__ inline size_t small_stride(int kp, int r) { return size_t(2) * kp * r + size_t(r) * r + r; }

// Load chunk rows [r0, r0+CH) of the w columns (U then Psi) into registers (NPF per thread).
template <int NPF>
__device__ inline void prefetch(cd* reg, const double2* U, const double2* Psi, int kp, int w, int N, int r0,
                                int tid) {
#pragma unroll
  for (int q = 0; q < NPF; ++q) {
    const int t = tid + q * T;
    const int col = t / CH, row = t - col * CH;
    const int gr = r0 + row;
    cd v = {0, 0};
    if (col < w && gr < N) v = col < kp ? ld2(U, size_t(col) * N + gr) : ld2(Psi, size_t(col - kp) * N + gr);
    reg[q] = v;
  }
}
template <int NPF>
__device__ inline void stage(cd* chunk, const cd* reg, int w, int tid) {
#pragma unroll
  for (int q = 0; q < NPF; ++q) {
    const int t = tid + q * T;
    const int col = t / CH, row = t - col * CH;
    if (col < w) chunk[col * CHP + row] = reg[q];
  }
}

// Gram kernel: rows of the result are the w columns [U, Psi or R], columns the r columns of
// Psi (pass 1) or R (pass 2).  2x2 tiles over (a, b), row groups over the chunk rows.
template <int NPF, int TPT>
__global__ __launch_bounds__(T) void k_isvd_gram(const double2* __restrict__ Ug, const double2* __restrict__ Psig,
                                                 double2* __restrict__ small, IsvdArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int N = a.N, kp = a.kp, r = a.r, w = a.w, k = a.k;
  const int tid = threadIdx.x;
  cd* chunk = reinterpret_cast<cd*>(smem_raw);   // [w][CHP]
  cd* Xs = chunk + size_t(w) * CHP;              // [kp][r]  X of pass 1
  cd* red = Xs + size_t(kp) * r;                 // reduction buffer [nrg][w][r]
  const int ta = (w + 1) / 2, tb = (r + 1) / 2, ntile = ta * tb;
  // TPT == 1: one tile per thread and the chunk rows split over T / ntile row groups;
  // TPT > 1 (more tiles than threads): tiles tid, tid + T, ... per thread, one row group
  const int nrg = TPT == 1 ? max(1, T / ntile) : 1;
  const int rg = TPT == 1 ? tid / ntile : 0;
  int a0[TPT], b0[TPT];
  bool active[TPT];
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int tile = TPT == 1 ? tid % ntile : tid + q * T;
    active[q] = TPT == 1 ? (rg < nrg && tid < ntile * nrg) : tile < ntile;
    a0[q] = 2 * (tile / tb);
    b0[q] = 2 * (tile % tb);
  }
  const size_t sstride = small_stride(kp, r);

  for (int p = blockIdx.x; p < a.nprob; p += gridDim.x) {
    const double2* U = Ug + size_t(p) * k * N;
    const double2* Psi = Psig + size_t(p) * r * N;
    double2* sm = small + size_t(p) * sstride;
    for (int pass = 0; pass < 2; ++pass) {
      cd acc[TPT][2][2];
#pragma unroll
      for (int q = 0; q < TPT; ++q) acc[q][0][0] = acc[q][0][1] = acc[q][1][0] = acc[q][1][1] = {0, 0};
      cd reg[NPF];
      prefetch<NPF>(reg, U, Psi, kp, w, N, 0, tid);
      for (int r0 = 0; r0 < N; r0 += CH) {
        stage<NPF>(chunk, reg, w, tid);
        __syncthreads();
        if (r0 + CH < N) prefetch<NPF>(reg, U, Psi, kp, w, N, r0 + CH, tid);
        if (pass == 1 && kp > 0) {
          // residual R = Psi - U X in place over the Psi columns of the chunk
          for (int t = tid; t < r * CH; t += T) {
            const int b = t / CH, row = t - b * CH;
            cd v = chunk[(kp + b) * CHP + row];
#pragma unroll 4
            for (int aa = 0; aa < kp; ++aa) v -= chunk[aa * CHP + row] * Xs[aa * r + b];
            chunk[(kp + b) * CHP + row] = v;
          }
          __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
          if (!active[q]) continue;
          const int a1 = min(a0[q] + 1, w - 1), b1 = min(b0[q] + 1, r - 1);
          const cd* A0 = chunk + a0[q] * CHP;
          const cd* A1 = chunk + a1 * CHP;
          const cd* B0 = chunk + (kp + b0[q]) * CHP;
          const cd* B1 = chunk + (kp + b1) * CHP;
#pragma unroll 4
          for (int row = rg; row < CH; row += nrg) {
            const cd x0 = A0[row], x1 = A1[row], y0 = B0[row], y1 = B1[row];
            acc[q][0][0] += cmul_conj(x0, y0);
            acc[q][0][1] += cmul_conj(x0, y1);
            acc[q][1][0] += cmul_conj(x1, y0);
            acc[q][1][1] += cmul_conj(x1, y1);
          }
        }
        __syncthreads();
      }
      // sum the partial tiles over the row groups
#pragma unroll
      for (int q = 0; q < TPT; ++q) {
        if (!active[q]) continue;
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            const int aa = a0[q] + i, bb = b0[q] + j;
            if (aa < w && bb < r) red[(size_t(rg) * w + aa) * r + bb] = acc[q][i][j];
          }
      }
      __syncthreads();
      for (int e = tid; e < w * r; e += T) {
        cd s = {0, 0};
        for (int g = 0; g < nrg; ++g) s += red[size_t(g) * w * r + e];
        const int aa = e / r, bb = e - aa * r;
        if (pass == 0) {
          if (aa < kp) {
            Xs[e] = s;
            st2(sm, e, s);                                          // X
          } else if (aa - kp == bb) {
            st2(sm, size_t(2) * kp * r + size_t(r) * r + bb, s);    // pn = |Psi_b|^2
          }
        } else {
          if (aa < kp) st2(sm, size_t(kp) * r + e, s);              // X2
          else st2(sm, size_t(2) * kp * r + size_t(aa - kp) * r + bb, s);  // G
        }
      }
      __syncthreads();
    }
  }
}

// Gram kernel on the FP64 matrix cores: C = W^dag B with W the w columns [U, Psi or R] and B
// the r columns of Psi or R, as real 16x16x4 products (Re C = Wr^T Br + Wi^T Bi, Im C =
// Wr^T Bi - Wi^T Br); TM row tiles of 16 (w <= 16 TM) by one column tile (r <= 16).  Wavefront v
// takes the 4-row steps v, v + 4, ... of every chunk (split-K); the four partial tiles are summed
// in LDS as in the vector kernel.  Operand layout of the 16x16x4 FP64 instruction: lane l holds
// A(l % 16, l / 16) and B(l / 16, l % 16); result register q of lane l is C(l / 16 + 4 q, l % 16).
typedef double v4d __attribute__((ext_vector_type(4)));

template <int NPF, int TM>
__global__ __launch_bounds__(T) void k_isvd_gram_mfma(const double2* __restrict__ Ug, const double2* __restrict__ Psig,
                                                      double2* __restrict__ small, IsvdArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int N = a.N, kp = a.kp, r = a.r, w = a.w, k = a.k;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int NW = T / 64;                     // wavefronts (row groups of the reduction)
  cd* chunk = reinterpret_cast<cd*>(smem_raw);   // [w][CHP]
  cd* Xs = chunk + size_t(w) * CHP;              // [kp][r]  X of pass 1
  cd* red = Xs + size_t(kp) * r;                 // reduction buffer [NW][w][r]
  const size_t sstride = small_stride(kp, r);

  for (int p = blockIdx.x; p < a.nprob; p += gridDim.x) {
    const double2* U = Ug + size_t(p) * k * N;
    const double2* Psi = Psig + size_t(p) * r * N;
    double2* sm = small + size_t(p) * sstride;
    for (int pass = 0; pass < 2; ++pass) {
      v4d cr[TM], ci[TM];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        cr[tm] = v4d{0.0, 0.0, 0.0, 0.0};
        ci[tm] = v4d{0.0, 0.0, 0.0, 0.0};
      }
      cd reg[NPF];
      prefetch<NPF>(reg, U, Psi, kp, w, N, 0, tid);
      for (int r0 = 0; r0 < N; r0 += CH) {
        stage<NPF>(chunk, reg, w, tid);
        __syncthreads();
        if (r0 + CH < N) prefetch<NPF>(reg, U, Psi, kp, w, N, r0 + CH, tid);
        if (pass == 1 && kp > 0) {
          // residual R = Psi - U X in place over the Psi columns of the chunk
          for (int t = tid; t < r * CH; t += T) {
            const int b = t / CH, row = t - b * CH;
            cd v = chunk[(kp + b) * CHP + row];
#pragma unroll 4
            for (int aa = 0; aa < kp; ++aa) v -= chunk[aa * CHP + row] * Xs[aa * r + b];
            chunk[(kp + b) * CHP + row] = v;
          }
          __syncthreads();
        }
        for (int ks = wv; ks < CH / 4; ks += NW) {
          const int row = 4 * ks + lk;
          const cd bv = li < r ? chunk[(kp + li) * CHP + row] : cd{0.0, 0.0};
#pragma unroll
          for (int tm = 0; tm < TM; ++tm) {
            const int aa = tm * 16 + li;
            const cd av = aa < w ? chunk[aa * CHP + row] : cd{0.0, 0.0};
            cr[tm] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.re, cr[tm], 0, 0, 0);
            cr[tm] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.im, bv.im, cr[tm], 0, 0, 0);
            ci[tm] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.im, ci[tm], 0, 0, 0);
            ci[tm] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.im, bv.re, ci[tm], 0, 0, 0);
          }
        }
        __syncthreads();
      }
      // this wavefront's partial tiles -> red[wv]
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int aa = tm * 16 + lk + 4 * q, bb = li;
          if (aa < w && bb < r) red[(size_t(wv) * w + aa) * r + bb] = cd{cr[tm][q], ci[tm][q]};
        }
      __syncthreads();
      for (int e = tid; e < w * r; e += T) {
        cd s = {0, 0};
        for (int g = 0; g < NW; ++g) s += red[size_t(g) * w * r + e];
        const int aa = e / r, bb = e - aa * r;
        if (pass == 0) {
          if (aa < kp) {
            Xs[e] = s;
            st2(sm, e, s);                                          // X
          } else if (aa - kp == bb) {
            st2(sm, size_t(2) * kp * r + size_t(r) * r + bb, s);    // pn = |Psi_b|^2
          }
        } else {
          if (aa < kp) st2(sm, size_t(kp) * r + e, s);              // X2
          else st2(sm, size_t(2) * kp * r + size_t(aa - kp) * r + bb, s);  // G
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------------
// small dense part: one wavefront per problem
// Sum over the lpp lanes of a pair's group (lpp a power of two, groups aligned, every lane of
// a group active): DPP quad permutations and row mirrors within a 16-lane row, a few cycles per
// step instead of an LDS-crossbar shuffle, then shuffles across rows.  Each step adds the
// partner's partial as the butterfly lane ^ off would (the partials are uniform within the
// half already summed), so the bits are those of the butterfly.
__device__ inline double pair_sum(double v, int lpp) {
  if (lpp >= 2) v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  if (lpp >= 4) v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  if (lpp >= 8) v += dpp_move<0x141, 0xF>(v);  // row_half_mirror: the other quad of 8 lanes
  if (lpp >= 16) v += dpp_move<0x140, 0xF>(v); // row_mirror: the other half of 16 lanes
  for (int off = 16; off < lpp; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int TW = 128;  // two wavefronts per small problem

__device__ inline int rr_pos(int i, int t, int w) {  // round-robin tournament position
  return i == 0 ? 0 : 1 + (i - 1 + t) % (w - 1);
}

__global__ __launch_bounds__(TW) void k_isvd_small(const double2* __restrict__ small, double* __restrict__ sig,
                                                   double2* __restrict__ AB, IsvdArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int kp = a.kp, r = a.r, w = a.w, kn = a.kn, k = a.k;
  const int we = w + (w & 1);
  const int lane = threadIdx.x;
  // J (the accumulated rotations) takes G's space: G is last read by the Cholesky step, J is
  // first written after it
  const int gj = max(r * r, we * we);
  // T and T^-1 take X2's space once X2 has been added into X when they fit there (2r <= kp):
  // 2 KB less per problem at k = 24, r = 8, so that four problems share a CU's LDS, not three
  const bool t_in_x2 = 2 * r <= kp;
  cd* X = reinterpret_cast<cd*>(smem_raw);        // [kp][r]  (X + X2 after the first step)
  cd* X2 = X + size_t(kp) * r;                    // [kp][r]
  cd* G = X2 + size_t(kp) * r;                    // [r][r]
  cd* J = G;                                      // [we][we]
  cd* Tm = t_in_x2 ? X2 : G + size_t(gj);         // [r][r] upper, row-major
  cd* Ti = Tm + size_t(r) * r;                    // [r][r]
  cd* M = t_in_x2 ? G + size_t(gj) : Ti + size_t(r) * r;  // [we][we] column-major
  double* s = reinterpret_cast<double*>(M + size_t(we) * we);  // [we]
  double* pn = s + we;                      // [r]
  int* keep = reinterpret_cast<int*>(pn + r);  // [r]
  int* perm = keep + r;                     // [we]
  const size_t sstride = small_stride(kp, r);
  __shared__ double wmax[TW / 64];
  const int npairs = we / 2;
  int lpp = 1;  // lanes per pair (power of two)
  while (lpp * 2 * npairs <= TW) lpp *= 2;
  const int grp = lane / lpp, gl = lane % lpp;

  for (int p = blockIdx.x; p < a.nprob; p += gridDim.x) {
    const double2* sm = small + size_t(p) * sstride;
    double* sg = sig + size_t(p) * k;
    double2* ab = AB + size_t(p) * w * kn;
    for (int e = lane; e < 2 * kp * r + r * r; e += TW) {
      const double2 v = sm[e];
      X[e] = {v.x, v.y};  // X, X2, G are contiguous in both layouts
    }
    for (int b = lane; b < r; b += TW) pn[b] = sm[size_t(2) * kp * r + size_t(r) * r + b].x;
    __syncthreads();
    // G2 = G - X2^dag X2 ; X <- X + X2
    for (int e = lane; e < r * r; e += TW) {
      const int i = e / r, l = e - i * r;
      cd v = G[e];
      for (int aa = 0; aa < kp; ++aa) v -= cmul_conj(X2[aa * r + i], X2[aa * r + l]);
      G[e] = v;
      if (!t_in_x2) {
        Tm[e] = {0, 0};
        Ti[e] = {0, 0};
      }
    }
    __syncthreads();
    for (int e = lane; e < kp * r; e += TW) X[e] += X2[e];
    if (t_in_x2) {  // X2 is dead once every lane has added it: clear T and T^-1 in its place
      __syncthreads();
      for (int e = lane; e < r * r; e += TW) {
        Tm[e] = {0, 0};
        Ti[e] = {0, 0};
      }
      __syncthreads();
    }
    // Cholesky with dropping: G2 = T^dag T
    for (int jj = 0; jj < r; ++jj) {
      if (lane == 0) {
        double dj = G[jj * r + jj].re;
        for (int i = 0; i < jj; ++i) dj -= norm2(Tm[i * r + jj]);
        const bool ok = dj > 1e-24 * pn[jj] && dj > 0.0;
        keep[jj] = ok ? 1 : 0;
        Tm[jj * r + jj] = {ok ? sqrt(dj) : 0.0, 0.0};
      }
      __syncthreads();
      if (keep[jj]) {
        const double inv = 1.0 / Tm[jj * r + jj].re;
        for (int l = jj + 1 + lane; l < r; l += TW) {
          cd v = G[jj * r + l];
          for (int i = 0; i < jj; ++i) v -= cmul_conj(Tm[i * r + jj], Tm[i * r + l]);
          Tm[jj * r + l] = inv * v;
        }
      }
      __syncthreads();
    }
    // Ti = T^-1 on the kept rows/columns: column l by lane l
    for (int l = lane; l < r; l += TW) {
      if (!keep[l]) continue;
      for (int i = l; i >= 0; --i) {
        if (!keep[i]) continue;
        cd v = (i == l) ? cd{1.0, 0.0} : cd{0.0, 0.0};
        for (int q = i + 1; q <= l; ++q)
          if (keep[q]) v -= Tm[i * r + q] * Ti[q * r + l];
        Ti[i * r + l] = (1.0 / Tm[i * r + i].re) * v;
      }
    }
    // M = K^dag: M(row, c) = conj(K(c, row)), column-major; J = I
    for (int e = lane; e < we * we; e += TW) {
      const int c = e / we, row = e - c * we;
      cd kv = {0, 0};
      if (c < w && row < w) {
        if (c < kp) {
          if (row < kp) kv = (c == row) ? cd{sg[c], 0.0} : cd{0, 0};
          else kv = X[c * r + (row - kp)];
        } else if (row >= kp) {
          kv = Tm[(c - kp) * r + (row - kp)];
        }
      }
      M[e] = conj(kv);
      J[e] = (c == row) ? cd{1.0, 0.0} : cd{0.0, 0.0};
    }
    __syncthreads();
    // one-sided Jacobi on the columns of M, rotations accumulated in J
    for (int sweep = 0; sweep < 40; ++sweep) {
      double offmax = 0.0;
      for (int t = 0; t < we - 1; ++t) {
        if (grp < npairs) {
          int pp = rr_pos(grp, t, we), qq = rr_pos(we - 1 - grp, t, we);
          if (pp > qq) {
            const int tmp = pp;
            pp = qq;
            qq = tmp;
          }
          cd* Mp = M + size_t(pp) * we;
          cd* Mq = M + size_t(qq) * we;
          double al = 0, be = 0;
          cd ga = {0, 0};
          for (int row = gl; row < we; row += lpp) {
            const cd u = Mp[row], v = Mq[row];
            al += norm2(u);
            be += norm2(v);
            ga += cmul_conj(u, v);
          }
          al = pair_sum(al, lpp);
          be = pair_sum(be, lpp);
          ga.re = pair_sum(ga.re, lpp);
          ga.im = pair_sum(ga.im, lpp);
          // the test and the rotation in squared quantities and reciprocal square roots: four
          // dependent FP64 square roots and divisions per round instead of eight
          const double g2 = norm2(ga), ab = al * be;
          if (al > 0.0 && be > 0.0 && g2 > 1e-300) {
            offmax = fmax(offmax, g2 / ab);  // squared relative off-diagonal
            if (g2 > kJacobiTol * kJacobiTol * ab) {
              const double ig = rsqrt(g2);  // 1 / |<m_p, m_q>|
              const double zeta = 0.5 * (be - al) * ig;
              const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
              const double cs = rsqrt(1.0 + tt * tt), sn = tt * cs;
              const cd e = {ga.re * ig, -ga.im * ig};  // exp(-i theta)
              cd* Jp = J + size_t(pp) * we;
              cd* Jq = J + size_t(qq) * we;
              for (int row = gl; row < we; row += lpp) {
                const cd u = Mp[row], v = e * Mq[row];
                Mp[row] = cs * u - sn * v;
                Mq[row] = sn * u + cs * v;
                const cd u2 = Jp[row], v2 = e * Jq[row];
                Jp[row] = cs * u2 - sn * v2;
                Jq[row] = sn * u2 + cs * v2;
              }
            }
          }
        }
        __syncthreads();
      }
      for (int off = 1; off < 64; off <<= 1) offmax = fmax(offmax, __shfl_xor(offmax, off, 64));
      if ((lane & 63) == 0) wmax[lane >> 6] = offmax;
      __syncthreads();
      for (int q = 0; q < TW / 64; ++q) offmax = fmax(offmax, wmax[q]);
      __syncthreads();
      if (offmax <= kJacobiTol * kJacobiTol) break;
    }
    // singular values = column norms of M, sorted descending (stable)
    for (int c = lane; c < we; c += TW) {
      double v = 0;
      for (int row = 0; row < we; ++row) v += norm2(M[size_t(c) * we + row]);
      s[c] = (c < w) ? sqrt(v) : -1.0;
    }
    __syncthreads();
    for (int c = lane; c < we; c += TW) {
      int rank = 0;
      for (int q = 0; q < we; ++q) rank += (s[q] > s[c] || (s[q] == s[c] && q < c)) ? 1 : 0;
      perm[rank] = c;
    }
    __syncthreads();
    // AB = [A; B] (w x kn, row-major): B = Ti Y_bot, A = Y_top - X B with Y = J[:, perm]
    for (int e = lane; e < r * kn; e += TW) {
      const int b = e / kn, i = e - b * kn;
      const cd* Yc = J + size_t(perm[i]) * we;
      cd v = {0, 0};
      for (int q = 0; q < r; ++q) v += Ti[b * r + q] * Yc[kp + q];
      M[e] = v;  // M is free now: B staged at M[0 .. r*kn)
      st2(ab, size_t(kp + b) * kn + i, v);
    }
    __syncthreads();
    for (int e = lane; e < kp * kn; e += TW) {
      const int aa = e / kn, i = e - aa * kn;
      const cd* Yc = J + size_t(perm[i]) * we;
      cd v = Yc[aa];
      for (int b = 0; b < r; ++b) v -= X[aa * r + b] * M[b * kn + i];
      st2(ab, size_t(aa) * kn + i, v);
    }
    for (int i = lane; i < kn; i += TW) sg[i] = s[perm[i]];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// rotation: U_new = [U, Psi] AB, in place.  Thread owns 2 rows x (kn / 8) columns.
template <int NPF>
__global__ __launch_bounds__(T) void k_isvd_rotate(double2* __restrict__ Ug, const double2* __restrict__ Psig,
                                                   const double2* __restrict__ AB, IsvdArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int N = a.N, kp = a.kp, r = a.r, w = a.w, kn = a.kn, k = a.k;
  const int tid = threadIdx.x;
  cd* chunk = reinterpret_cast<cd*>(smem_raw);  // [w][CHP]
  cd* Ms = chunk + size_t(w) * CHP;             // [w][kn]
  constexpr int NG = T / (CH / 2);              // column groups
  const int rp = tid % (CH / 2), ig = tid / (CH / 2);
  for (int p = blockIdx.x; p < a.nprob; p += gridDim.x) {
    double2* U = Ug + size_t(p) * k * N;
    const double2* Psi = Psig + size_t(p) * r * N;
    const double2* ab = AB + size_t(p) * w * kn;
    for (int e = tid; e < w * kn; e += T) Ms[e] = ld2(ab, e);
    cd reg[NPF];
    prefetch<NPF>(reg, U, Psi, kp, w, N, 0, tid);
    for (int r0 = 0; r0 < N; r0 += CH) {
      stage<NPF>(chunk, reg, w, tid);
      __syncthreads();
      if (r0 + CH < N) prefetch<NPF>(reg, U, Psi, kp, w, N, r0 + CH, tid);
      const int row0 = 2 * rp, row1 = 2 * rp + 1;
      for (int i = ig; i < kn; i += NG) {
        cd v0 = {0, 0}, v1 = {0, 0};
#pragma unroll 4
        for (int c = 0; c < w; ++c) {
          const cd m = Ms[c * kn + i];
          v0 += chunk[c * CHP + row0] * m;
          v1 += chunk[c * CHP + row1] * m;
        }
        if (r0 + row0 < N) st2(U, size_t(i) * N + r0 + row0, v0);
        if (r0 + row1 < N) st2(U, size_t(i) * N + r0 + row1, v1);
      }
      __syncthreads();
    }
  }
}

// Rotation, row-parallel form: U_new = [U, Psi] M (M = [A; B], w x kn) is independent per row,
// so a workgroup takes 256 rows of one problem (one row per thread, its w inputs held in
// registers before any output of that row is written, which makes the in-place update safe)
// and M is staged in LDS.  Every input and output element moves once, and all rows of all
// problems are in flight at once instead of one problem per workgroup.
template <int WM>
__global__ __launch_bounds__(T) void k_isvd_rotate_rows(double2* __restrict__ Ug, const double2* __restrict__ Psig,
                                                        const double2* __restrict__ AB, IsvdArgs a) {
  __shared__ cd Ms[WM * MAXW];
  const int N = a.N, kp = a.kp, w = a.w, kn = a.kn, k = a.k, r = a.r;
  const int p = blockIdx.x;  // problems on x: their count may exceed the 65535 of a y extent
  const double2* ab = AB + size_t(p) * w * kn;
  for (int e = threadIdx.x; e < w * kn; e += T) Ms[e] = ld2(ab, e);
  __syncthreads();
  const int row = blockIdx.y * T + threadIdx.x;
  if (row >= N) return;
  double2* U = Ug + size_t(p) * k * N;
  const double2* Psi = Psig + size_t(p) * r * N;
  cd in[WM];
#pragma unroll
  for (int c = 0; c < WM; ++c) {
    if (c < w) in[c] = c < kp ? ld2(U, size_t(c) * N + row) : ld2(Psi, size_t(c - kp) * N + row);
  }
  for (int i0 = 0; i0 < kn; i0 += 8) {
    cd acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = {0, 0};
#pragma unroll
    for (int c = 0; c < WM; ++c) {
      if (c < w) {
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (i0 + t < kn) acc[t] += in[c] * Ms[c * kn + i0 + t];
      }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (i0 + t < kn) st2(U, size_t(i0 + t) * N + row, acc[t]);
  }
}

// the matrix-core Gram kernel takes one column tile (r <= 16) and 16 < w <= 64 (for w <= 16 a
// 16 x 16 tile wastes most of its products and the vector kernel is faster)
inline bool gram_on_mfma(int w, int r) { return r <= 16 && w > 16 && w <= 64; }
size_t gram_lds(int kp, int r) {
  const int w = kp + r;
  const int ta = (w + 1) / 2, tb = (r + 1) / 2, ntile = ta * tb;
  // row groups of the reduction: the wavefronts (matrix-core kernel) or T / tiles (vector kernel)
  const int nrg = gram_on_mfma(w, r) ? T / 64 : std::max(1, T / ntile);
  return (size_t(w) * CHP + size_t(kp) * r + size_t(nrg) * w * r) * sizeof(cd);
}
size_t small_lds(int kp, int r) {
  const int w = kp + r, we = w + (w & 1);
  // X, X2, G / J, T and T^-1 (inside X2 when 2r <= kp), M: the layout of k_isvd_small
  const size_t tt = (2 * r <= kp) ? 0 : 2 * size_t(r) * r;
  const size_t n = 2 * size_t(kp) * r + std::max(size_t(r) * r, size_t(we) * we) + tt + size_t(we) * we;
  return n * sizeof(cd) + (we + r) * sizeof(double) + (r + we) * sizeof(int);
}
size_t rotate_lds(int kp, int r, int kn) {
  const int w = kp + r;
  return (size_t(w) * CHP + size_t(w) * kn) * sizeof(cd);
}

void set_lds(const void* f, size_t lds) {
  if (lds > 64 * 1024) QMG_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
}

template <int NPF>
void launch_rows(const IsvdArgs& a, int ncu, size_t lg, size_t lr, DevBuf& P64, const void* blocks,
                 DevBuf& small, DevBuf& AB, DevBuf& sigma_dev, size_t ls, hipStream_t st) {
  set_lds((const void*)k_isvd_small, ls);
  set_lds((const void*)k_isvd_rotate<NPF>, lr);
  const int grid = std::min(a.nprob, 4 * ncu);
  const int ntile = ((a.w + 1) / 2) * ((a.r + 1) / 2);
  const double Nn = double(a.N) * a.nprob;
  double2* U = P64.as<double2>();
  const double2* Psi = static_cast<const double2*>(blocks);
  {
    // two row passes over U (kp columns) and Psi (r columns); the Gram products of both passes
    // and the residual R = Psi - U X
    TimedLaunch tl("isvd/gram", st, Nn * 16.0 * 2.0 * (a.kp + a.r),
                   Nn * 8.0 * (2.0 * double(a.w) * a.r + double(a.kp) * a.r));
    auto go = [&](auto kern) {
      set_lds((const void*)kern, lg);
      launch(kern, dim3(grid), dim3(T), uint32_t(lg), st, U, Psi, small.as<double2>(), a);
    };
    if (gram_on_mfma(a.w, a.r)) {
      if (a.w <= 32) go(k_isvd_gram_mfma<NPF, 2>);
      else go(k_isvd_gram_mfma<NPF, 4>);
    } else if (ntile <= T) {
      go(k_isvd_gram<NPF, 1>);
    } else {
      go(k_isvd_gram<NPF, 4>);
    }
  }
  QMG_LAUNCH_CHECK();
  {
    // the w x w core per problem: Cholesky and one-sided Jacobi, counted as six sweeps of
    // w (w - 1) / 2 rotations of two length-w columns of K^dag and of the rotation accumulator
    const double w3 = double(a.w) * a.w * a.w;
    TimedLaunch tl("isvd/small", st, double(a.nprob) * (small_stride(a.kp, a.r) + double(a.w) * a.kn) * 16.0,
                   double(a.nprob) * 120.0 * w3);
    launch(k_isvd_small, dim3(a.nprob), dim3(TW), uint32_t(ls), st, static_cast<const double2*>(small.as<double2>()),
           sigma_dev.as<double>(), AB.as<double2>(), a);
  }
  QMG_LAUNCH_CHECK();
  {
    // U_new = U A + Psi B in place: U and Psi read once, U_new written
    TimedLaunch tl("isvd/rotate", st, Nn * 16.0 * (a.kp + a.r + a.kn), Nn * 8.0 * double(a.w) * a.kn);
    const dim3 rgrid(a.nprob, (a.N + T - 1) / T);
    const double2* ABc = AB.as<double2>();
    if (a.w <= 32) launch(k_isvd_rotate_rows<32>, rgrid, dim3(T), 0, st, U, Psi, ABc, a);
    else if (a.w <= 48) launch(k_isvd_rotate_rows<48>, rgrid, dim3(T), 0, st, U, Psi, ABc, a);
    else launch(k_isvd_rotate<NPF>, dim3(grid), dim3(T), uint32_t(lr), st, U, Psi, ABc, a);
  }
  QMG_LAUNCH_CHECK();
}

}  // namespace

int isvd_stream(HierarchyDev& h, const void* blocks, int r, int kp, DevBuf& sigma_dev, hipStream_t st) {
  return isvd_stream(2 * h.blk.d, h.blk.N, h.k, h.P64, blocks, r, kp, sigma_dev, st);
}

int isvd_stream(int nprob, int N, int k, DevBuf& P64, const void* blocks, int r, int kp, DevBuf& sigma_dev,
                hipStream_t st) {
  const int w = kp + r;
  const int kn = std::min(k, w);
  QMG_CHECK(r >= 1 && w <= MAXW, QMG_ESHAPE, "streaming SVD: k + r = %d exceeds %d", w, MAXW);
  QMG_CHECK(((w + 1) / 2) * ((r + 1) / 2) <= 4 * T, QMG_ESHAPE,
            "streaming SVD: ceil((k+r)/2) * ceil(r/2) = %d exceeds %d", ((w + 1) / 2) * ((r + 1) / 2), 4 * T);
  const size_t lg = gram_lds(kp, r), ls = small_lds(kp, r), lr = rotate_lds(kp, r, kn);
  QMG_CHECK(lg <= 160 * 1024 && ls <= 160 * 1024 && lr <= 160 * 1024, QMG_ESHAPE,
            "streaming SVD: k + r = %d needs more than 160 KiB of LDS", w);
  IsvdArgs a{nprob, N, k, r, kp, w, kn};
  int dev = 0, ncu = 256;
  QMG_HIP(hipGetDevice(&dev));
  QMG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  DevBuf small(size_t(a.nprob) * small_stride(kp, r) * sizeof(double2));
  DevBuf AB(size_t(a.nprob) * w * kn * sizeof(double2));
  // algorithmic: read U (kp cols) and Psi (r cols) in the two Gram passes and the rotation,
  // write U (kn cols); flops of the Gram passes, the residual and the rotation
  const int need = (w * CH + T - 1) / T;  // prefetch registers needed
  if (need <= 4) launch_rows<4>(a, ncu, lg, lr, P64, blocks, small, AB, sigma_dev, ls, st);
  else if (need <= 8) launch_rows<8>(a, ncu, lg, lr, P64, blocks, small, AB, sigma_dev, ls, st);
  else launch_rows<PF>(a, ncu, lg, lr, P64, blocks, small, AB, sigma_dev, ls, st);
  QMG_HIP(hipStreamSynchronize(st));  // scratch buffers are released on return
  return kn;
}

}  // namespace qmg
