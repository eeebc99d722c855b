// Streaming chiral SVD update (Algorithm 3, Eqs. (7)-(8)) for all (aggregate, chirality)
// problems of one stream, in FP64.
//
// For each problem the state is Phi_{s-1} = U Sigma (U: N x kp orthonormal) and the new block
// Psi (N x r).  The rank-k SVD of [U Sigma, Psi] is obtained without forming it:
//   X  = U^dag Psi,  R = Psi - U X,  X2 = U^dag R,  G = R^dag R        (row passes 1 and 2;
//        projection done twice, classical Gram-Schmidt)
//   G2 = G - X2^dag X2 = T^dag T        (Cholesky; a column whose remaining norm falls below
//        1e-12 of its original norm is dropped: its row of T is zero)
//   [U Sigma, Psi] = [U, Q] K,  K = [[Sigma, X + X2], [0, T]],  Q = (Psi - U (X + X2)) T^-1
//   K = Y S Z^dag by one-sided Jacobi on the columns of K^dag with the rotations accumulated,
//        so Y (the left singular vectors of K) is unitary even where S is zero
//   U_new = [U, Q] Y_k = U A + Psi B,   B = T^-1 Y_bot,   A = Y_top - (X + X2) B   (pass 3)
// Singular values are sorted descending with ties broken by the lower index.
//
// Launch: persistent grid, one 256-thread workgroup per problem at a time; rows are streamed
// through LDS in chunks, the small dense matrices (at most (k+r)^2) live in LDS.
#include <cmath>

#include "mg.hpp"

namespace qmg {

namespace {

using cd = cplx<double>;
constexpr int T = 256;
constexpr int CH = 32;       // rows per chunk
constexpr int CHP = CH + 1;  // padded LDS stride

struct IsvdArgs {
  int nprob, N, k, r, kp, w, kn;
};

__device__ inline cd ld2(const double2* p, size_t i) {
  const double2 v = p[i];
  return {v.x, v.y};
}
__device__ inline void st2(double2* p, size_t i, cd v) { p[i] = make_double2(v.re, v.im); }

__device__ inline int rr_pos(int i, int t, int w) {  // round-robin tournament position
  return i == 0 ? 0 : 1 + (i - 1 + t) % (w - 1);
}

__global__ __launch_bounds__(T) void k_isvd(double2* __restrict__ Ug, double* __restrict__ sig,
                                            const double2* __restrict__ Psig, IsvdArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int N = a.N, kp = a.kp, r = a.r, w = a.w, kn = a.kn, k = a.k;
  const int tid = threadIdx.x;
  // LDS regions
  cd* chunk = reinterpret_cast<cd*>(smem_raw);      // [w][CHP]: U columns then Psi columns
  cd* X = chunk + size_t(w) * CHP;                  // [kp][r]
  cd* X2 = X + size_t(kp) * r;                      // [kp][r]
  cd* G = X2 + size_t(kp) * r;                      // [r][r]
  cd* Tm = G + size_t(r) * r;                       // [r][r] upper triangular, row-major
  cd* Ti = Tm + size_t(r) * r;                      // [r][r]
  const int we = w + (w & 1);                       // even size for the tournament
  cd* M = Ti + size_t(r) * r;                       // [we][we] column-major: column p at M + p*we
  cd* J = M + size_t(we) * we;                      // [we][we]
  double* s = reinterpret_cast<double*>(J + size_t(we) * we);  // [we]
  double* pn = s + we;                              // [r]
  double* offg = pn + r;                            // [32]
  int* keep = reinterpret_cast<int*>(offg + 32);    // [r]
  int* perm = keep + r;                             // [we]
  __shared__ int s_flag;

  const int nown1 = kp * r + r;       // pass-1 outputs: X entries then |Psi_b|^2
  const int nown2 = kp * r + r * r;   // pass-2 outputs: X2 entries then G entries
  constexpr int MAXO = 4;             // outputs per thread (kp*r + r*r <= 4 * 256)

  for (int p = blockIdx.x; p < a.nprob; p += gridDim.x) {
    double2* U = Ug + size_t(p) * k * N;
    const double2* Psi = Psig + size_t(p) * r * N;
    double* sg = sig + size_t(p) * k;

    // ---------------- pass 1: X = U^dag Psi, pn = |Psi_b|^2
    cd acc[MAXO];
    for (int q = 0; q < MAXO; ++q) acc[q] = {0, 0};
    for (int r0 = 0; r0 < N; r0 += CH) {
      for (int t = tid; t < w * CH; t += T) {
        const int col = t / CH, row = t - col * CH;
        const int gr = r0 + row;
        cd v = {0, 0};
        if (gr < N) v = col < kp ? ld2(U, size_t(col) * N + gr) : ld2(Psi, size_t(col - kp) * N + gr);
        chunk[col * CHP + row] = v;
      }
      __syncthreads();
      for (int q = 0; q < MAXO; ++q) {
        const int e = tid + q * T;
        if (e >= nown1) break;
        const cd* x;
        const cd* y;
        if (e < kp * r) {
          x = chunk + (e / r) * CHP;
          y = chunk + (kp + e % r) * CHP;
        } else {
          x = y = chunk + (kp + e - kp * r) * CHP;
        }
        cd sum = {0, 0};
        for (int row = 0; row < CH; ++row) sum += cmul_conj(x[row], y[row]);
        acc[q] += sum;
      }
      __syncthreads();
    }
    for (int q = 0; q < MAXO; ++q) {
      const int e = tid + q * T;
      if (e >= nown1) break;
      if (e < kp * r) X[e] = acc[q];
      else pn[e - kp * r] = acc[q].re;
    }
    __syncthreads();

    // ---------------- pass 2: R = Psi - U X ; X2 = U^dag R ; G = R^dag R
    for (int q = 0; q < MAXO; ++q) acc[q] = {0, 0};
    for (int r0 = 0; r0 < N; r0 += CH) {
      for (int t = tid; t < w * CH; t += T) {
        const int col = t / CH, row = t - col * CH;
        const int gr = r0 + row;
        cd v = {0, 0};
        if (gr < N) v = col < kp ? ld2(U, size_t(col) * N + gr) : ld2(Psi, size_t(col - kp) * N + gr);
        chunk[col * CHP + row] = v;
      }
      __syncthreads();
      if (kp > 0) {
        // residual in registers, then written over the Psi part of the chunk
        cd res[(CH * 48 + T - 1) / T];
        int nres = 0;
        for (int t = tid; t < r * CH; t += T, ++nres) {
          const int b = t / CH, row = t - b * CH;
          cd v = chunk[(kp + b) * CHP + row];
          for (int aa = 0; aa < kp; ++aa) v -= chunk[aa * CHP + row] * X[aa * r + b];
          res[nres] = v;
        }
        __syncthreads();
        nres = 0;
        for (int t = tid; t < r * CH; t += T, ++nres) {
          const int b = t / CH, row = t - b * CH;
          chunk[(kp + b) * CHP + row] = res[nres];
        }
        __syncthreads();
      }
      for (int q = 0; q < MAXO; ++q) {
        const int e = tid + q * T;
        if (e >= nown2) break;
        const cd* x;
        const cd* y;
        if (e < kp * r) {
          x = chunk + (e / r) * CHP;
          y = chunk + (kp + e % r) * CHP;
        } else {
          const int f = e - kp * r;
          x = chunk + (kp + f / r) * CHP;
          y = chunk + (kp + f % r) * CHP;
        }
        cd sum = {0, 0};
        for (int row = 0; row < CH; ++row) sum += cmul_conj(x[row], y[row]);
        acc[q] += sum;
      }
      __syncthreads();
    }
    for (int q = 0; q < MAXO; ++q) {
      const int e = tid + q * T;
      if (e >= nown2) break;
      if (e < kp * r) X2[e] = acc[q];
      else G[e - kp * r] = acc[q];
    }
    __syncthreads();

    // ---------------- small dense part
    // G2 = G - X2^dag X2 (in G), X += X2
    for (int e = tid; e < r * r; e += T) {
      const int i = e / r, l = e - i * r;
      cd v = G[e];
      for (int aa = 0; aa < kp; ++aa) v -= cmul_conj(X2[aa * r + i], X2[aa * r + l]);
      G[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < kp * r; e += T) X[e] += X2[e];
    for (int e = tid; e < r * r; e += T) {
      Tm[e] = {0, 0};
      Ti[e] = {0, 0};
    }
    __syncthreads();
    // Cholesky with dropping: G2 = T^dag T, T upper, row-major Tm[i*r + l]
    for (int jj = 0; jj < r; ++jj) {
      if (tid == 0) {
        double dj = G[jj * r + jj].re;
        for (int i = 0; i < jj; ++i) dj -= norm2(Tm[i * r + jj]);
        const bool ok = dj > 1e-24 * pn[jj] && dj > 0.0;
        keep[jj] = ok ? 1 : 0;
        Tm[jj * r + jj] = {ok ? sqrt(dj) : 0.0, 0.0};
      }
      __syncthreads();
      if (keep[jj]) {
        const double djj = Tm[jj * r + jj].re;
        for (int l = jj + 1 + tid; l < r; l += T) {
          cd v = G[jj * r + l];
          for (int i = 0; i < jj; ++i) v -= cmul_conj(Tm[i * r + jj], Tm[i * r + l]);
          Tm[jj * r + l] = (1.0 / djj) * v;
        }
      }
      __syncthreads();
    }
    // Ti = T^-1 on the kept rows/columns (zero elsewhere): column l solved by thread l
    if (tid < r) {
      const int l = tid;
      if (keep[l]) {
        for (int i = l; i >= 0; --i) {
          if (!keep[i]) continue;
          cd v = (i == l) ? cd{1.0, 0.0} : cd{0.0, 0.0};
          for (int q = i + 1; q <= l; ++q)
            if (keep[q]) v -= Tm[i * r + q] * Ti[q * r + l];
          Ti[i * r + l] = (1.0 / Tm[i * r + i].re) * v;
        }
      }
    }
    // M = K^dag (column-major, M[c*we + row] = conj(K[row][c])), J = I
    for (int e = tid; e < we * we; e += T) {
      const int c = e / we, row = e - c * we;
      cd kv = {0, 0};  // K[row][c]... M column c = conj of K row c
      // M[c][row] (column c, entry row) = conj(K[c][row])
      const int kr = c, kc = row;
      if (kr < w && kc < w) {
        if (kr < kp) {
          if (kc < kp) kv = (kr == kc) ? cd{sg[kr], 0.0} : cd{0, 0};
          else kv = X[kr * r + (kc - kp)];
        } else if (kc >= kp) {
          kv = Tm[(kr - kp) * r + (kc - kp)];
        }
      }
      M[e] = conj(kv);
      J[e] = (c == row) ? cd{1.0, 0.0} : cd{0.0, 0.0};
    }
    __syncthreads();

    // one-sided Jacobi on the columns of M, rotations accumulated in J
    const int npairs = we / 2;
    const int grp = tid >> 3, gl = tid & 7;
    for (int sweep = 0; sweep < 40; ++sweep) {
      double offmax = 0.0;
      for (int t = 0; t < we - 1; ++t) {
        if (grp < npairs) {
          int pp = rr_pos(grp, t, we), qq = rr_pos(we - 1 - grp, t, we);
          if (pp > qq) { const int tmp = pp; pp = qq; qq = tmp; }
          cd* Mp = M + size_t(pp) * we;
          cd* Mq = M + size_t(qq) * we;
          double al = 0, be = 0;
          cd ga = {0, 0};
          for (int row = gl; row < we; row += 8) {
            al += norm2(Mp[row]);
            be += norm2(Mq[row]);
            ga += cmul_conj(Mp[row], Mq[row]);
          }
#pragma unroll
          for (int off = 1; off < 8; off <<= 1) {
            al += __shfl_xor(al, off, 64);
            be += __shfl_xor(be, off, 64);
            ga.re += __shfl_xor(ga.re, off, 64);
            ga.im += __shfl_xor(ga.im, off, 64);
          }
          const double g = sqrt(norm2(ga));
          if (al > 0.0 && be > 0.0 && g > 1e-300) {
            const double rel = g / sqrt(al * be);
            offmax = fmax(offmax, rel);
            if (rel > 1e-16) {
              const double zeta = (be - al) / (2.0 * g);
              const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
              const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = tt * cs;
              const cd e = {ga.re / g, -ga.im / g};  // exp(-i theta)
              for (int row = gl; row < we; row += 8) {
                const cd u = Mp[row], v = e * Mq[row];
                Mp[row] = cs * u - sn * v;
                Mq[row] = sn * u + cs * v;
              }
              cd* Jp = J + size_t(pp) * we;
              cd* Jq = J + size_t(qq) * we;
              for (int row = gl; row < we; row += 8) {
                const cd u = Jp[row], v = e * Jq[row];
                Jp[row] = cs * u - sn * v;
                Jq[row] = sn * u + cs * v;
              }
            }
          }
        }
        __syncthreads();
      }
      if (gl == 0 && grp < 32) offg[grp] = (grp < npairs) ? offmax : 0.0;
      __syncthreads();
      if (tid == 0) {
        double mx = 0.0;
        for (int q = 0; q < npairs && q < 32; ++q) mx = fmax(mx, offg[q]);
        s_flag = (mx < 1e-15) ? 1 : 0;
      }
      __syncthreads();
      if (s_flag) break;
    }
    // singular values = column norms of M, sorted descending (stable)
    for (int c = tid; c < we; c += T) {
      double v = 0;
      for (int row = 0; row < we; ++row) v += norm2(M[size_t(c) * we + row]);
      s[c] = (c < w) ? sqrt(v) : -1.0;
    }
    __syncthreads();
    for (int c = tid; c < we; c += T) {
      int rank = 0;
      for (int q = 0; q < we; ++q) rank += (s[q] > s[c] || (s[q] == s[c] && q < c)) ? 1 : 0;
      perm[rank] = c;
    }
    __syncthreads();
    // B = Ti Y_bot (r x kn), A = Y_top - X B (kp x kn); Y = J[:, perm], stored over M:
    // M[0 .. kp*kn) = A (row-major [a][i]), then B ([b][i])
    cd* Am = M;
    cd* Bm = M + size_t(kp) * kn;
    // M is no longer needed; write B first from J (J untouched)
    for (int e = tid; e < r * kn; e += T) {
      const int b = e / kn, i = e - b * kn;
      const cd* Yc = J + size_t(perm[i]) * we;
      cd v = {0, 0};
      for (int q = 0; q < r; ++q) v += Ti[b * r + q] * Yc[kp + q];
      Bm[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < kp * kn; e += T) {
      const int aa = e / kn, i = e - aa * kn;
      const cd* Yc = J + size_t(perm[i]) * we;
      cd v = Yc[aa];
      for (int b = 0; b < r; ++b) v -= X[aa * r + b] * Bm[b * kn + i];
      Am[e] = v;
    }
    for (int i = tid; i < kn; i += T) sg[i] = s[perm[i]];
    __syncthreads();

    // ---------------- pass 3: U_new = U A + Psi B (row-local, in place)
    for (int r0 = 0; r0 < N; r0 += CH) {
      for (int t = tid; t < w * CH; t += T) {
        const int col = t / CH, row = t - col * CH;
        const int gr = r0 + row;
        cd v = {0, 0};
        if (gr < N) v = col < kp ? ld2(U, size_t(col) * N + gr) : ld2(Psi, size_t(col - kp) * N + gr);
        chunk[col * CHP + row] = v;
      }
      __syncthreads();
      for (int t = tid; t < kn * CH; t += T) {
        const int i = t / CH, row = t - i * CH;
        const int gr = r0 + row;
        if (gr >= N) continue;
        cd v = {0, 0};
        for (int aa = 0; aa < kp; ++aa) v += chunk[aa * CHP + row] * Am[aa * kn + i];
        for (int b = 0; b < r; ++b) v += chunk[(kp + b) * CHP + row] * Bm[b * kn + i];
        st2(U, size_t(i) * N + gr, v);
      }
      __syncthreads();
    }
  }
}

size_t isvd_lds_bytes(int kp, int r) {
  const int w = kp + r, we = w + (w & 1);
  const size_t n = size_t(w) * CHP + 2 * size_t(kp) * r + 3 * size_t(r) * r + 2 * size_t(we) * we;
  return n * sizeof(cd) + (we + r + 32) * sizeof(double) + (r + we) * sizeof(int);
}

}  // namespace

int isvd_stream(HierarchyDev& h, const void* blocks, int r, int kp, DevBuf& sigma_dev, hipStream_t st) {
  const int w = kp + r;
  const int kn = std::min(h.k, w);
  QMG_CHECK(kp * r + r * r <= 4 * T && kp * r + r <= 4 * T, QMG_ESHAPE, "streaming SVD: k*r + r*r too large");
  QMG_CHECK(r >= 1 && r <= 48, QMG_ESHAPE, "streaming SVD: batch r must be in [1, 48]");
  const size_t lds = isvd_lds_bytes(kp, r);
  QMG_CHECK(lds <= 160 * 1024, QMG_ESHAPE, "streaming SVD: k + r = %d needs %zu bytes of LDS (> 160 KiB)", w, lds);
  IsvdArgs a{2 * h.blk.d, h.blk.N, h.k, r, kp, w, kn};
  int dev = 0, ncu = 256;
  QMG_HIP(hipGetDevice(&dev));
  QMG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = std::min(a.nprob, ncu * 2);
  if (lds > 64 * 1024) QMG_HIP(hipFuncSetAttribute((const void*)k_isvd, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  k_isvd<<<grid, T, lds, st>>>(h.P64.as<double2>(), sigma_dev.as<double>(), (const double2*)blocks, a);
  QMG_LAUNCH_CHECK();
  return kn;
}

}  // namespace qmg
