// The two-level hierarchy owned by a qmg_mg handle, and the kernels that act on it.
#pragma once

#include <memory>
#include <vector>

#include "krylov.hpp"

namespace qmg {

// Aggregate-local tables (device, int32):
//   bsite [d][nd]   fine site of (aggregate j, in-block index ib), ib lexicographic in the block
//   cnb   [d][8]    coarse neighbour of aggregate j in direction dir
// P row order inside (j, alpha): row = s6 * nd + ib with s6 = 3 * spin_in_chirality + colour;
// this component-major order lets consecutive threads read consecutive P entries.

// A further level built on the coarse stencil of the level above (Algorithm 4 applied to D_c):
// sites J of the lattice cL, each a block b of nd sites of the level above (k1 degrees of
// freedom per chirality there).  Rows of a (J, alpha) block: row = i * nd + jb (i < k1 the dof
// index inside chirality alpha, jb the site in the block), N = nd * k1.
struct CoarseLevel {
  int cL[4] = {1, 1, 1, 1}, b[4] = {1, 1, 1, 1};
  int nd = 1, d = 1, N = 0, k = 0, k1 = 0;
  DevBuf bsite, cnb;         // [d][nd] site of the level above; [d][8] neighbours on cL
  DevBuf agg, pos;           // [d1] aggregate J and in-block index jb of every site above
  DevBuf P64, Pin;           // [d][2][k][N]
  DevBuf Y64, Yin;           // [d][9][2k][2k] column-major blocks
  DevBuf sigma_dev;          // [d][2][k]
  std::vector<double> sigma;
  int n_test = 0, batch = 0, n_setup_iter = 0, streams_done = 0, kp = 0;
  uint64_t seed = 0;
  double t_total = 0;
  double tol = 0;  // relative tolerance of the Krylov solve on this level (0: the hierarchy's coarse_tol)
};

struct HierarchyDev {
  Geom g;
  Blocking blk;
  int k = 0;                 // rank per chirality
  qmg_prec inner = QMG_F64;  // inner storage precision

  DevBuf U64, Uin;           // native gauge, FP64 and inner precision
  DevBuf U32;                // FP32 gauge when the inner precision is below FP32 (outer GCR, setup)
  DevBuf A64, Ain, A32;      // packed site term with the clover term, beside U64, Uin, U32 (empty: Wilson)
  // even-odd smoother (qmg_mg_set_smoother): half-lattice gauge, site term and its inverse in
  // FP64 ([0]) and in the inner precision ([1], when it is not F64); site terms empty for Wilson
  int eo_smoother = 0;  // 0: GMRES on D, 1: even-odd with GMRES, 2: even-odd with the s-step form
  DevBuf Ueo[2], Aeo[2], Aieo[2];
  int eo_ne = 9;  // complex entries per link in Ueo: 9, or 6 for SU(3) links (two rows stored)
  DevBuf bsite, cnb;         // tables
  DevBuf blists;             // [8][nd]: in-block sites per hop direction, intra-block hops first
  DevBuf P64, Pin;           // [d][2][k][N]
  DevBuf Y64, Yin;           // [d][9][2k][2k] column-major blocks
  // even-odd coarse solve (qmg_mg_set_coarse_eo): the colouring tables and Yhat = Y_0^-1 Y
  // (slot 0: Y_0^-1) in FP64 and, below FP64, in the inner precision
  int coarse_eo = 0;
  DevBuf ceo_tab;            // [d] colour, [d] index in colour, [2][d/2] aggregates, [d][8] neighbour index
  DevBuf Yh64, Yhin;
  std::vector<double> sigma; // [d][2][k]
  double t_smooth = 0, t_svd = 0, t_coarse = 0, t_total = 0;
  int n_post = 8, coarse_max = 500;
  double coarse_tol = 0.03;
  int cycle_steps = 0;       // > 0: device-exit coarse solve with this step budget
  bool cycle_graph = false;  // capture the K-cycle into a hipGraph (needs cycle_steps > 0)
  std::vector<std::unique_ptr<CoarseLevel>> levels;  // further levels (l = 2, 3), each on the one above
};

// The nine-block stencil that a further level is built on: the first coarse level's D_c, or the
// operator of the previous further level.
struct StencilRef {
  int cL[4];
  int d, k;
  const int* cnb;
  const void* Y64;
};
inline StencilRef stencil_above(const HierarchyDev& h, size_t i) {
  StencilRef s{};
  if (i == 0) {
    for (int q = 0; q < 4; ++q) s.cL[q] = h.blk.cL[q];
    s.d = h.blk.d;
    s.k = h.k;
    s.cnb = h.cnb.as<int>();
    s.Y64 = h.Y64.p;
  } else {
    const CoarseLevel& L = *h.levels[i - 1];
    for (int q = 0; q < 4; ++q) s.cL[q] = L.cL[q];
    s.d = L.d;
    s.k = L.k;
    s.cnb = L.cnb.as<int>();
    s.Y64 = L.Y64.p;
  }
  return s;
}

// prolong: fine[rhs] (native, storage S) = P coarse[rhs]
void launch_prolong(qmg_prec prec, const HierarchyDev& h, const void* P, const void* coarse, void* fine, int nrhs,
                    hipStream_t st);
// restrict: coarse[rhs] = P^dag fine[rhs]
void launch_restrict(qmg_prec prec, const HierarchyDev& h, const void* P, const void* fine, void* coarse, int nrhs,
                     hipStream_t st);
// out = D_c in, coarse vectors [nrhs][d][2k]
void launch_coarse_apply(qmg_prec prec, const HierarchyDev& h, const void* Y, const void* in, void* out, int nrhs,
                         hipStream_t st, const int* skip = nullptr);  // skip: device early-exit flag
// the same for any nine-block stencil: d sites, 2k dof per site, neighbour table cnb [d][8]
void launch_stencil_apply(qmg_prec prec, int d, int k, const int* cnb, const void* Y, const void* in, void* out,
                          int nrhs, hipStream_t st, const int* skip = nullptr);
// third level: Philox coarse test vectors [n][d][m] FP64 (counter (j, g, v0 + n, level))
void launch_philox_coarse(uint64_t seed, int v0, int n, int d, int m, int level, void* out, hipStream_t st);
// chiral split of r coarse vectors [r][d1][2k1] FP64 into blocks [2d][r][N] FP64
void launch_level_gather(const CoarseLevel& L, const void* v, void* blocks, int r, hipStream_t st);
// v1 [nrhs][d1][2k1] = P2 v2 [nrhs][d][2k]; v2 = P2^dag v1 (storage precision prec)
void launch_level_prolong(qmg_prec prec, const CoarseLevel& L, int d1, const void* P, const void* v2, void* v1,
                          int nrhs, hipStream_t st);
void launch_level_restrict(qmg_prec prec, const CoarseLevel& L, int d1, const void* P, const void* v1, void* v2,
                           int nrhs, hipStream_t st);
// Y2 = P2^dag A P2 in FP64 from the stencil A of the level above
void build_level_coarse(CoarseLevel& L, const StencilRef& above, hipStream_t st);
// canonical exports of the third level: P [d][2][N][k] with rows (jb * k1 + i), Y [d][9][2k][2k]
void launch_level_export_P(const CoarseLevel& L, void* out, hipStream_t st);
void launch_level_export_Y(const CoarseLevel& L, void* out, hipStream_t st);
// even-odd coarse operator: colouring tables (ESHAPE if a coarse extent is odd) and Yhat from Y64
// (EBREAKDOWN if a self block is singular)
void build_coarse_eo_tables(HierarchyDev& h, hipStream_t st);
void build_coarse_eo_blocks(HierarchyDev& h, hipStream_t st);
// one colour of half vectors [nrhs][d/2][2k]: out = [y] + [B_0 a] + sgn sum_s B_s b(nbh), B = Y or
// Yhat; a null a or b drops the self or the hop slots
void launch_coarse_eo_apply(qmg_prec prec, const HierarchyDev& h, int colour, const void* B, const void* y,
                            const void* a, const void* b, void* out, int nrhs, double sgn, hipStream_t st);
// full coarse vectors [nrhs][d][2k] <-> colours [nrhs][d/2][2k]
void launch_coarse_eo_split(qmg_prec prec, const HierarchyDev& h, const void* full, void* ev, void* od, int nrhs,
                            hipStream_t st);
void launch_coarse_eo_merge(qmg_prec prec, const HierarchyDev& h, const void* ev, const void* od, void* full, int nrhs,
                            hipStream_t st);
// Galerkin build in FP64 from U64 and P64 into Y64 (needs a workspace of 8 * d * (2k)^2 double2)
void build_coarse(HierarchyDev& h, hipStream_t st);
// chiral split + block gather: fine FP64 native [r][12][V] -> blocks [2d][r][N] FP64
void launch_chiral_gather(const HierarchyDev& h, const void* fine, void* blocks, int r, hipStream_t st);
// one streaming-SVD stream for all (aggregate, chirality) problems, in place on P64 / sigma
// kp: current columns (0 on the first stream), returns the new column count
int isvd_stream(HierarchyDev& h, const void* blocks, int r, int kp, DevBuf& sigma_dev, hipStream_t st);
// the same for nprob problems of N rows and rank k with the factor U in P64
int isvd_stream(int nprob, int N, int k, DevBuf& P64, const void* blocks, int r, int kp, DevBuf& sigma_dev,
                hipStream_t st);
// canonical P export [d][2][N][k] with canonical row order 6*ib + 3*sp + c
void launch_export_P(const HierarchyDev& h, void* out, hipStream_t st);
// canonical Y export [d][9][2k row][2k col]
void launch_export_Y(const HierarchyDev& h, void* out, hipStream_t st);
// Philox4x32-10 Gaussian test vectors into native FP64 [n][12][V]
void launch_philox_native(const Geom& g, uint64_t seed, int v0, int n, void* out, hipStream_t st);
// the same test vectors for nl lattices of volumes Vl (device int[nl]) in the padded layout
// [l][n][12][Vpad] (zero beyond each lattice's volume)
void launch_philox_padded(uint64_t seed, int v0, int n, int nl, const int* Vl, int Vpad, void* out, hipStream_t st);
// link force: canonical FP64 x, lambda -> canonical FP64 dU
void launch_link_force(const Geom& g, const void* x, const void* lam, void* dU, int nrhs, hipStream_t st);

}  // namespace qmg
