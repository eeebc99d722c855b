/* qmg.h -- C ABI of libqmg: Wilson-Dirac stencil, streaming chiral-SVD multigrid setup,
 * transfer operators, coarse operator and the multigrid-preconditioned solve on one AMD
 * Instinct MI355X (gfx950).
 *
 * The method is the adaptive multigrid setup with a streaming SVD of the chirally split
 * test vectors of Whyte, Stathopoulos and Romero, "Accelerating multigrid with streaming
 * chiral SVD for Wilson fermions in lattice QCD" (arXiv 2505.14399): Eq. (1) (D x = b),
 * Eq. (2) (test vectors), Eq. (3) (chiral split), Eq. (5) (Galerkin coarse operator),
 * Eq. (6) (chiral-SVD prolongator), Eqs. (7)-(8) and Algorithms 3-4 (streaming update).
 * Beyond the two-level path: up to four levels (qmg_mg_add_level), the clover term of the
 * action used in Section 4 (qmg_clover_*; mg params c_sw_s / c_sw_t), even-odd (Schur
 * complement) preconditioning of the fine operator named in Section 1 (qmg_eo_*,
 * qmg_schur_apply, qmg_eo_solve, the even-odd post-smoother of qmg_mg_set_smoother) and of
 * the coarse operator (qmg_mg_set_coarse_eo, qmg_coarse_schur_apply, qmg_coarse_eo_solve),
 * hierarchy checkpoints and resumable streams (qmg_mg_save / _load / _stream_more).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns qmg_status; 0 is success, a negative value an error.
 *   Inputs are validated before any launch; on error nothing has been written unless the
 *   description says otherwise, and qmg_last_error() holds a message (per thread).
 * Memory: every pointer argument named "device" is caller-owned device memory of the
 *   current HIP device (for example a torch CUDA tensor's data_ptr()).  The library never
 *   retains or frees a caller pointer after returning.  Handles (qmg_mg) are library-owned
 *   until qmg_mg_destroy; one handle must not be used by two calls at the same time.
 * Streams: all work is enqueued on the given stream.  Apply, transfer and force calls are
 *   asynchronous.  Setup and solve make host decisions and synchronize the stream before
 *   returning.
 * Complex numbers are interleaved (re, im) in the given precision.
 * Canonical layouts (row-major, lexicographic site = x + Lx*(y + Ly*(z + Lz*t))):
 *   gauge   [4 mu][V][3][3]        U_mu(x), the physical link from x to x+mu
 *   spinor  [nrhs][V][4 spin][3 colour] in the chiral basis, gamma_5 = diag(1,1,-1,-1)
 *   coarse  [nrhs][d][2 chirality][k]   aggregates d in coarse lexicographic order,
 *                                        rank index by descending singular value
 * Native layouts (QMG_NATIVE) are the structure-of-arrays forms the kernels stream:
 *   spinor  [nrhs][12 = 3*spin + colour][V]
 *   gauge   [4 mu][9 = 3*row + col][V]
 */
#ifndef QMG_H
#define QMG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qmg_status;
enum {
  QMG_OK = 0,
  QMG_EINVAL = -1,      /* null pointer, bad enum, non-positive count              */
  QMG_ESHAPE = -2,      /* lattice / block / rank / batch sizes inconsistent       */
  QMG_EDTYPE = -3,      /* precision not supported by this entry point             */
  QMG_ENOMEM = -4,      /* device allocation failed                                */
  QMG_EHIP = -5,        /* a HIP runtime call or launch failed                     */
  QMG_ENOCONV = -6,     /* solve stopped at max iterations; x holds the best iterate */
  QMG_EBREAKDOWN = -7,  /* Krylov breakdown (zero or non-finite norm)              */
  QMG_ENONFINITE = -8,  /* NaN or Inf in an input or a residual                    */
  QMG_ENOTIMPL = -9
};

typedef enum { QMG_F64 = 0, QMG_F32 = 1, QMG_BF16 = 2, QMG_F16 = 3 } qmg_prec;
typedef enum { QMG_CANONICAL = 0, QMG_NATIVE = 1 } qmg_layout;

/* The lattice problem of Eq. (1): extents, time boundary condition, quark mass, anisotropy.
 * D is the Wilson-Dirac operator
 *   (D psi)(x) = (m + 1 + 3/xi) psi(x)
 *     - 1/2 sum_mu c_mu [ s_mu(x) (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                       + s_mu(x-mu) (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 * with c_t = 1, c_x = c_y = c_z = 1/xi and s_mu(y) = bc_t for mu = t, y_t = Lt-1, else 1.
 * Extents must be >= 1 and V = Lx Ly Lz Lt < 2^31. */
typedef struct {
  int32_t dims[4]; /* Lx, Ly, Lz, Lt */
  int32_t bc_t;    /* +1 periodic, -1 antiperiodic in t (x, y, z periodic) */
  double mass;     /* m */
  double xi;       /* anisotropy a_s / a_t, > 0 */
} qmg_lattice;

/* out = D in (Eq. (1)'s operator), for nrhs spinors at once.
 * U, in, out: device buffers in precision `prec` and layout `layout` (gauge and spinor
 *   forms above); out must not alias in.  F64 computes in double, F32/BF16/F16 store in
 *   that precision and accumulate in float.
 * Errors: EINVAL (null, nrhs < 1, bad enum), ESHAPE (bad extents), EHIP. */
qmg_status qmg_wilson_apply(const qmg_lattice* lat, const void* U, const void* in, void* out,
                            int32_t nrhs, qmg_prec prec, qmg_layout layout, hipStream_t stream);
/* out = D^dagger in = gamma_5 D gamma_5 in; arguments as qmg_wilson_apply. */
qmg_status qmg_wilson_apply_adj(const qmg_lattice* lat, const void* U, const void* in, void* out,
                                int32_t nrhs, qmg_prec prec, qmg_layout layout, hipStream_t stream);

/* Many independent lattices in one launch (for example 64 small lattices of 4,096 to 20,736
 * sites with different extents): out_i = D_i in_i (D_i^dagger if dagger = 1) for i < n_lat,
 * each lattice with its own extents, boundary, mass, anisotropy, gauge field and nrhs spinors,
 * the operator of qmg_wilson_apply in the native layout.  Workgroups are assigned to lattices
 * by a prefix sum of their site tiles, so uneven lattices share one launch.
 * lats: host array of n_lat descriptors.  U, in, out: DEVICE arrays of n_lat device pointers
 *   (native gauge [4][9][V_i], native spinors [nrhs][12][V_i] in precision prec); out_i must
 *   not alias in_i.
 * The descriptor table is uploaded on the first call for a given set of lattices (after the
 * stream has drained) and reused while the set is unchanged; calls with different sets on
 * several streams at once are not supported.
 * Errors: EINVAL (null, n_lat outside [1, 65536], nrhs < 1, bad enum), ESHAPE (extents), EHIP. */
qmg_status qmg_wilson_apply_batched(int32_t n_lat, const qmg_lattice* lats, const void* const* U,
                                    const void* const* in, void* const* out, int32_t nrhs, qmg_prec prec,
                                    int32_t dagger, hipStream_t stream);

/* Wilson-clover operator D_sw = D + T, the operator of the paper's experiments (Section 4: Wilson
 * fermions with the clover term), which the paper names but does not write out.  The reading
 * implemented: the O(a)-improvement term of Luescher, Sint, Sommer and Weisz (1996) in the
 * normalisation of D above,
 *   T(x) = sum_{mu<nu} c_{mu nu} (i/2) sigma_{mu nu} (x) Fhat_{mu nu}(x),
 *   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],  Fhat_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag)/8,
 * Q_{mu nu}(x) the four plaquettes of the mu-nu plane with a corner at x, each walked
 * counter-clockwise (a mu step before a nu step), no trace subtraction; c_{mu nu} = c_sw_t for
 * the three planes containing t and c_sw_s for the spatial planes (c_sw_s = c_sw_t = c_sw: the
 * isotropic term).  The gauge field is periodic in every direction, so T ignores bc_t.  T(x) is
 * hermitian and commutes with gamma_5, so D_sw^dagger = gamma_5 D_sw gamma_5.
 *
 * qmg_clover_field: A = the site-local part (m + 1 + 3/xi) 1 + T(x) of D_sw, packed.
 * U: device, canonical FP64 gauge field.  A: device, 36 V complex numbers in precision prec
 *   (written): per chirality alpha (spins 0,1 for alpha = 0, spins 2,3 for alpha = 1) a
 *   hermitian 6 x 6 block over (spin within the chirality, colour), stored site-fastest at
 *   A[(alpha*18 + e)*V + x]; e = 0, 1, 2 hold the real diagonal entries (2e, 2e+1) as the (re, im)
 *   pair of one complex number, e = 3 .. 17 the upper triangle (i < j) row by row.  The
 *   computation is FP64 whatever prec is; it synchronizes the stream (it frees a temporary).
 * Errors: EINVAL (null, bad enum, non-finite coefficient), ESHAPE (extents), ENOMEM, EHIP. */
qmg_status qmg_clover_field(const qmg_lattice* lat, double c_sw_s, double c_sw_t, const void* U, void* A,
                            qmg_prec prec, hipStream_t stream);
/* out = D_sw in (dagger = 0) or D_sw^dagger in (dagger = 1): the stencil of qmg_wilson_apply with
 * the packed site term A (from qmg_clover_field, device, precision prec) in place of its
 * diagonal term, fused into the same kernels.  U, in, out as in qmg_wilson_apply; out must
 * not alias in.  Errors: EINVAL (null, nrhs < 1, bad enum, aliasing), ESHAPE, EHIP. */
qmg_status qmg_clover_apply(const qmg_lattice* lat, const void* U, const void* A, const void* in, void* out,
                            int32_t nrhs, qmg_prec prec, qmg_layout layout, int32_t dagger, hipStream_t stream);

/* Layout/precision conversion: canonical FP64 <-> native `prec` (device buffers, no aliasing). */
qmg_status qmg_pack_spinor(const qmg_lattice* lat, const void* canon_f64, void* native, int32_t nrhs,
                           qmg_prec prec, hipStream_t stream);
qmg_status qmg_unpack_spinor(const qmg_lattice* lat, const void* native, void* canon_f64, int32_t nrhs,
                             qmg_prec prec, hipStream_t stream);
qmg_status qmg_pack_gauge(const qmg_lattice* lat, const void* canon_f64, void* native, qmg_prec prec,
                          hipStream_t stream);

/* Parameters of the setup, Algorithms 3 and 4: block shape of the aggregates Lambda_j,
 * the number of test vectors sampled (n_s streams of r = batch vectors each), the rank k
 * kept per chirality, the smoother and the K-cycle. */
typedef struct {
  int32_t block[4];      /* aggregate extents; each must divide the lattice extent            */
  int32_t n_test;        /* total test vectors sampled, n_s * batch                           */
  int32_t batch;         /* r, test vectors per stream                                        */
  int32_t rank;          /* k per chirality: 1 <= k <= 6*prod(block), k <= n_test, k+r <= 64  */
  int32_t n_setup_iter;  /* GMRES(8) iterations smoothing each test vector (0: psi = phi)     */
  int32_t n_post_smooth; /* GMRES post-smoothing iterations in the K-cycle (Section 4: 8)     */
  double coarse_tol;     /* coarse solve to ||r_c|| <= coarse_tol ||b_c|| (Section 4: 0.03)   */
  int32_t coarse_max_iter; /* cap on coarse GMRES iterations per cycle (e.g. 500)             */
  qmg_prec inner_prec;   /* storage precision of D, P, D_c and vectors inside the K-cycle    */
  uint64_t seed;         /* Philox4x32-10 key for the random initial guesses phi             */
  const void* test_vectors; /* optional device buffer, canonical FP64 [n_test][V][4][3]: the
                               initial guesses phi (NULL: internal counter RNG)               */
  double c_sw_s;         /* clover coefficients of the fine operator (qmg_clover_field): spatial */
  double c_sw_t;         /*   planes and planes containing t; both 0 (default): Wilson          */
} qmg_mg_params;

typedef struct qmg_mg qmg_mg; /* opaque two-level hierarchy: P (FP64 and inner copy), D_c */

/* Multigrid setup with the streaming chiral SVD (Algorithm 4 with Algorithm 3).  For every
 * stream s: r initial guesses phi are smoothed on D psi ~ 0 (Eq. (2)), normalised, split by
 * chirality and blocked (Eq. (3)), and every (aggregate, chirality) block updates its rank-k
 * SVD of [Phi_{s-1}, Psi_s] (Eq. (8)); the last stream gives P = U_k (Eq. (6)), R = P^dag and
 * D_c = R D P (Eq. (5)).
 * U: device, canonical FP64 gauge field; it is copied into the handle.  With a non-zero clover
 * coefficient in params the fine operator is D_sw (qmg_clover_field's site term is built from U
 * and kept beside every gauge copy): smoothing, the Galerkin product (the site term enters
 * Y_0), the smoother and the outer solve all use it.
 * Errors: EINVAL, ESHAPE (block does not divide, k or r out of range, n_test % batch,
 *   n_test < k), ENOMEM, EHIP, ENONFINITE (non-finite links). On error *out is NULL. */
qmg_status qmg_mg_setup_stream_chiral_svd(const qmg_lattice* lat, const void* U, const qmg_mg_params* params,
                                          qmg_mg** out, hipStream_t stream);

/* fine_out = P coarse_in (Eq. (6)), canonical layouts, prec F64 or F32. */
qmg_status qmg_prolong(const qmg_mg* mg, const void* coarse_in, void* fine_out, int32_t nrhs, qmg_prec prec,
                       hipStream_t stream);
/* coarse_out = R fine_in = P^dag fine_in, canonical layouts, prec F64 or F32. */
qmg_status qmg_restrict(const qmg_mg* mg, const void* fine_in, void* coarse_out, int32_t nrhs, qmg_prec prec,
                        hipStream_t stream);
/* out = D_c in (Eq. (5)) as the nine-block coarse stencil, canonical coarse layout,
 * prec F64 (the FP64 operator) or F32 (the inner copy when inner_prec is F32). */
qmg_status qmg_coarse_apply(const qmg_mg* mg, const void* in, void* out, int32_t nrhs, qmg_prec prec,
                            hipStream_t stream);

typedef struct {
  int32_t outer_iters;      /* outer flexible GMRES iterations, summed over refinements      */
  int32_t refinements;      /* FP64 defect-correction steps                                  */
  int32_t coarse_iters;     /* coarse GMRES iterations, summed                               */
  int32_t smoother_iters;   /* fine GMRES post-smoothing iterations, summed                  */
  int32_t precision_escalations;
  double true_rel_res;      /* ||b - D x|| / ||b|| recomputed in FP64 at the end              */
  double seconds;
  int32_t coarse2_iters;    /* Krylov iterations on level 2 (the third level), summed; 0 if none */
  int32_t smoother1_iters;  /* GMRES post-smoothing iterations on D_c (level 1), summed        */
  int32_t coarse3_iters;    /* Krylov iterations on level 3 (the fourth level), summed; 0 if none */
  int32_t smoother2_iters;  /* GMRES post-smoothing iterations on level 2, summed              */
} qmg_solve_info;

/* Solve D x = b (or D^dag x = b when adjoint != 0, as gamma5 D^-1 gamma5) to a true FP64
 * relative residual <= tol with flexible GMRES(16) preconditioned by the two-level K-cycle
 * (Section 2.1: restrict, coarse GMRES to coarse_tol, prolong, post-smooth; Section 4: FGMRES
 * as the outer solver).  With an inner precision below F64 the K-cycle runs in that precision
 * and the flexible GMRES in FP32, inside an FP64 defect-correction loop.  With further levels
 * (qmg_mg_add_level) the coarse solve is a flexible GMRES(32) on D_c to coarse_tol
 * preconditioned by the K-cycle of the first coarse level, recursively.
 * b, x: device, canonical FP64 [nrhs][V][4][3]; x is the initial guess on entry (zeros
 *   allowed) and the solution on return.  info: host array of nrhs entries (may be NULL).
 * Errors: ENOCONV (x holds the best iterate, info filled), ENONFINITE, EBREAKDOWN, EHIP. */
qmg_status qmg_mg_solve(const qmg_mg* mg, const void* b, void* x, int32_t nrhs, double tol, int32_t max_outer,
                        int32_t adjoint, qmg_solve_info* info, hipStream_t stream);

/* Further levels (the paper's hierarchies have three and four levels, Section 4): each call
 * applies Algorithm 4 with Algorithm 3 to the operator of the current coarsest level (D_c of
 * the hierarchy for level l = 2, then level 2's operator for l = 3; at most four levels).  Test
 * vectors phi_v (v < n_test) on that level are complex Gaussian from Philox4x32-10 keyed by seed
 * with counter (site, g, v, l - 1) (components 2g, 2g+1), smoothed by n_setup_iter GMRES(8)
 * iterations on A psi' = -A phi in FP64 and normalised; the chirality is sigma3 (the alpha block
 * of every site); blocks of `block` sites (each extent must divide the extent of the level
 * above) are folded into a rank-`rank` streaming SVD per (aggregate, chirality) in batches of
 * `batch`; P_l = U_k and A_l = P_l^dag A P_l as a nine-block stencil (hops leaving an aggregate
 * through its face kept in their directional block).  qmg_mg_solve then recurses: level l - 1
 * solves level l by flexible GMRES(32) to coarse_tol preconditioned by level l's K-cycle (plain
 * GMRES(32) on the coarsest level), with n_post_smooth post-smoothing steps on level l - 1.
 * Limits: k_above * prod(block) <= 4096, 1 <= batch <= 48, rank <= min(k_above * prod(block),
 * n_test, 32).  Not combined with the device-exit / captured K-cycle (qmg_mg_set_cycle with
 * coarse_steps > 0: EINVAL either way), not stored by qmg_mg_save (a loaded hierarchy has two
 * levels); qmg_mg_stream_more rebuilds them.
 * Errors: EINVAL (null, already four levels, device-exit cycle set), ESHAPE, ENOMEM, EHIP. */
qmg_status qmg_mg_add_level(qmg_mg* mg, const int32_t* block, int32_t n_test, int32_t batch, int32_t rank,
                            int32_t n_setup_iter, uint64_t seed, hipStream_t stream);
/* Relative tolerance of the Krylov solve on level l >= 2 inside the K-cycle of level l - 1
 * (default 0: the hierarchy's coarse_tol, which level 1 always uses).  Near the critical mass
 * the lower levels of a deep hierarchy are solved more loosely (Section 4: 0.06 on l = 2 and
 * 0.6 on l = 3 for four levels).  A solve-time setting: not stored by qmg_mg_save, kept by
 * qmg_mg_stream_more.  Errors: EINVAL (null, no level l, tol outside [0, 1)). */
qmg_status qmg_mg_set_level_tol(qmg_mg* mg, int32_t level, double tol);
/* Level l >= 2: extents [4], aggregate count and rank (EINVAL when the hierarchy has no level l). */
qmg_status qmg_mg_level_query(const qmg_mg* mg, int32_t level, int32_t* coarse_dims, int32_t* n_agg,
                              int32_t* rank);
/* Level l >= 2: P_l as FP64 blocks [d_l][2][N_l][k_l] with rows (site in block * k_above + i)
 * (device, may be NULL), singular values [d_l][2][k_l] (host, may be NULL), A_l blocks
 * [d_l][9][2k_l][2k_l] FP64 (device, may be NULL; slot 0 self, 1 + dir hops, row-major blocks). */
qmg_status qmg_mg_level_get(const qmg_mg* mg, int32_t level, void* P, double* sigma, void* Y, hipStream_t stream);
/* Level l >= 2 transfer and operator on coarse vectors (device, [nrhs][d][2][k] layouts, prec F64
 * or the F32 inner precision): out = P_l in (level l -> level l - 1), out = P_l^dag in, out = A_l in. */
qmg_status qmg_level_prolong(const qmg_mg* mg, int32_t level, const void* in, void* out, int32_t nrhs,
                             qmg_prec prec, hipStream_t stream);
qmg_status qmg_level_restrict(const qmg_mg* mg, int32_t level, const void* in, void* out, int32_t nrhs,
                              qmg_prec prec, hipStream_t stream);
qmg_status qmg_level_coarse_apply(const qmg_mg* mg, int32_t level, const void* in, void* out, int32_t nrhs,
                                  qmg_prec prec, hipStream_t stream);

/* Gradient of L = sum_rhs Re <eta, D^-1 b> with respect to the gauge links, from the
 * solution x = D^-1 b and the adjoint solution lambda = D^-dag eta:
 *   dL/dU_mu(x) = 1/2 c_mu s_mu(x) G^dag,
 *   G = tr_spin[(1-gamma_mu) x(x+mu) lambda(x)^dag] + tr_spin[(1+gamma_mu) lambda(x+mu) x(x)^dag]
 * (gradient convention dL/dRe + i dL/dIm).  x, lambda: device canonical FP64 spinors;
 * dU: device canonical FP64 gauge field, overwritten. */
qmg_status qmg_link_force(const qmg_lattice* lat, const void* x, const void* lambda, void* dU, int32_t nrhs,
                          hipStream_t stream);

/* Test-vector initial guesses phi_v, v = v0 .. v0+n-1, from Philox4x32-10 keyed by seed
 * (counter (site, g, v, 0), Box-Muller), canonical FP64 [n][V][4][3] into device `out`. */
qmg_status qmg_random_test_vectors(const qmg_lattice* lat, uint64_t seed, int32_t v0, int32_t n, void* out,
                                   hipStream_t stream);

/* Smooth test vectors (Eq. (2)): psi = phi + psi', psi' from n_iter GMRES(8) iterations on
 * D psi' = -D phi from zero, then psi /= ||psi||.  U, phi, psi: device canonical FP64;
 * computed in `prec` (F64 or F32). */
qmg_status qmg_smooth(const qmg_lattice* lat, const void* U, const void* phi, void* psi, int32_t nrhs,
                      int32_t n_iter, qmg_prec prec, hipStream_t stream);

/* Read the hierarchy: coarse extents [4], d and k; P as canonical FP64 blocks
 * [d][2][N][k] (device, may be NULL), singular values [d][2][k] (host, may be NULL),
 * Galerkin blocks [d][9][2k][2k] FP64 (device, may be NULL; slot 0 self, 1+dir hops). */
qmg_status qmg_mg_query(const qmg_mg* mg, int32_t* coarse_dims, int32_t* n_agg, int32_t* rank);
qmg_status qmg_mg_get_prolongator(const qmg_mg* mg, void* P, double* sigma, hipStream_t stream);
qmg_status qmg_mg_get_coarse(const qmg_mg* mg, void* Y, hipStream_t stream);

/* The lattice and setup parameters of a hierarchy (either pointer may be NULL).  n_test is the
 * number of test vectors folded in so far (streams done * batch); test_vectors is NULL. */
qmg_status qmg_mg_get_params(const qmg_mg* mg, qmg_lattice* lat, qmg_mg_params* params);

/* Resumable streams: Algorithm 3 continues from the current factor U_k Sigma_k with n_streams
 * more streams of `batch` test vectors (the counter RNG with the setup's seed at the next global
 * indices streams_done * batch, ..., smoothed as in the setup), then P, R and D_c are rebuilt.
 * The result equals a setup with the larger n_test.  A third level (qmg_mg_add_level) is
 * rebuilt on the new D_c with its own parameters.  Errors: EINVAL (null, n_streams < 1),
 * ENOMEM, EHIP. */
qmg_status qmg_mg_stream_more(qmg_mg* mg, int32_t n_streams, hipStream_t stream);

/* Hierarchy checkpoint.  qmg_mg_save writes the lattice, the setup parameters (with the clover
 * coefficients), the number of
 * streams done, a 64-bit hash of the gauge field, the singular values and the factor U_k (= P)
 * in FP64 to `path` (a little-endian binary file ending in a hash of its arrays).
 * qmg_mg_load rebuilds the hierarchy from such a file for the gauge field U (device, canonical
 * FP64): the Galerkin operator and the inner-precision copies are recomputed, so the loaded
 * hierarchy solves exactly as the saved one, and qmg_mg_stream_more continues the streaming SVD
 * from it.  The file does not hold U.
 * Errors: EINVAL (null, unreadable / truncated / corrupted file, wrong magic or version,
 *   inconsistent header, U differs from the field the file was built for), ESHAPE, ENOMEM, EHIP.
 *   On error *out is NULL. */
qmg_status qmg_mg_save(const qmg_mg* mg, const char* path, hipStream_t stream);
qmg_status qmg_mg_load(const char* path, const void* U, qmg_mg** out, hipStream_t stream);

/* Even-odd (red-black) preconditioning of the fine operator, which the paper names among the
 * standard accelerations of the solve (Section 1) without writing it out.  Reading: with every
 * extent even, the hops of D (or D_sw) join sites of opposite parity p = (x+y+z+t) mod 2 and
 * the site term A (the diagonal term, plus T with the clover term) is local, so D x = b is
 * solved through the Schur complement on the even sites,
 *   Dhat = A_ee - D_eo A_oo^-1 D_oe,   Dhat x_e = b_e - D_eo A_oo^-1 b_o,
 *   x_o = A_oo^-1 (b_o - D_oe x_e);
 * Dhat^dagger = gamma_5 Dhat gamma_5 is the Schur complement of D^dagger.
 * Half-lattice layouts (device, any qmg_prec; BF16/FP16 store and FP32 accumulate): a site's
 * half index is its lexicographic index / 2;
 *   spinor      [nrhs][12 = 3*spin + colour][V/2] for one parity
 *   gauge       [2 parity][4 mu][9][V/2]        U_mu(x) stored at the parity of x
 *   site term   [2 parity][2 alpha][18][V/2]    the packed blocks of qmg_clover_field
 * Errors of every entry below: EINVAL (null, bad count, aliasing, bad enum), ESHAPE (an odd
 * extent), ENOMEM, EHIP. */
qmg_status qmg_eo_pack_gauge(const qmg_lattice* lat, const void* U, void* U_eo, qmg_prec prec, hipStream_t stream);
qmg_status qmg_eo_pack_spinor(const qmg_lattice* lat, const void* canon_f64, void* even, void* odd, int32_t nrhs,
                              qmg_prec prec, hipStream_t stream);
qmg_status qmg_eo_unpack_spinor(const qmg_lattice* lat, const void* even, const void* odd, void* canon_f64,
                                int32_t nrhs, qmg_prec prec, hipStream_t stream);
/* A_eo = the packed site term of D_sw with coefficients (c_sw_s, c_sw_t) (both 0: the Wilson
 * diagonal term) in the half-lattice layout, and Ainv_eo its inverse (per site and chirality,
 * Gauss-Jordan with partial pivoting in FP64).  U: device, canonical FP64 gauge field.
 * Synchronizes the stream.  Extra error: EBREAKDOWN if a block is singular. */
qmg_status qmg_eo_site_term(const qmg_lattice* lat, double c_sw_s, double c_sw_t, const void* U, void* A_eo,
                            void* Ainv_eo, qmg_prec prec, hipStream_t stream);
/* out_e = Dhat in_e (dagger = 0) or Dhat^dagger in_e (dagger = 1) on even half fields: two hop
 * launches, A_oo^-1 D_oe in_e on the odd sites, then A_ee in_e - D_eo (...).  A_eo and Ainv_eo
 * from qmg_eo_site_term, or both NULL for the Wilson operator (the scalar diagonal term).
 * Synchronizes the stream (it frees the odd intermediate). */
qmg_status qmg_schur_apply(const qmg_lattice* lat, const void* U_eo, const void* A_eo, const void* Ainv_eo,
                           const void* in_e, void* out_e, int32_t nrhs, qmg_prec prec, int32_t dagger,
                           hipStream_t stream);
/* x = D^-1 b (D = D_sw when a clover coefficient is non-zero) by FP64 GMRES(32): with eo = 1 on
 * the Schur complement (source preparation, Dhat solve to tol ||b|| / ||bhat_e||,
 * reconstruction), with eo = 0 on the full-lattice operator (the same Krylov method, for
 * comparison).  U: device canonical FP64 gauge field; b, x: device canonical FP64
 * [nrhs][V][4][3].  info (host, optional): outer_iters = GMRES iterations, true_rel_res =
 * ||b - D x|| / ||b|| in FP64 (worst over right-hand sides), seconds.  Extra errors: ENOCONV
 * (not converged within max_iter; x holds the last iterate), ENONFINITE. */
qmg_status qmg_eo_solve(const qmg_lattice* lat, const void* U, double c_sw_s, double c_sw_t, const void* b, void* x,
                        int32_t nrhs, double tol, int32_t max_iter, int32_t eo, qmg_solve_info* info,
                        hipStream_t stream);

/* Setup timings in seconds: smoother, streaming SVD, coarse build, total (host array [4]). */
qmg_status qmg_mg_setup_times(const qmg_mg* mg, double* t);

/* Form of the K-cycle used by later qmg_mg_solve calls on this hierarchy.
 * coarse_steps = 0 (default): the coarse GMRES(32) runs to its tolerance with the host reading
 *   its convergence estimates every few steps (restarted up to coarse_max_iter steps).
 * coarse_steps in [1, 63]: the coarse solve is one GMRES cycle of at most coarse_steps steps
 *   whose convergence test is made on the device: once every right-hand side is below the
 *   tolerance the remaining launches of the cycle return at once, and the whole K-cycle needs
 *   no host round trip (a weaker coarse solve if the budget is short: the outer solver is
 *   flexible, so the solve still converges, possibly in more iterations).
 * graph = 1 (needs coarse_steps > 0): the K-cycle is captured into a hipGraph on a private
 *   stream at its first application in each solve and replayed for every later one.
 * Errors: EINVAL (null, coarse_steps outside [0, 63], graph not 0/1, graph without steps). */
qmg_status qmg_mg_set_cycle(qmg_mg* mg, int32_t coarse_steps, int32_t graph);

/* Fine-level post-smoother of the K-cycle (later qmg_mg_solve calls on this hierarchy).
 * eo = 0 (default): n_post_smooth GMRES steps on D e = r from the prolonged correction.
 * eo = 1: even-odd smoothing: t = r - D z for the prolonged correction z, n_post_smooth GMRES
 *   steps from zero on the Schur system of t (Dhat e_e = t_e - D_eo A_oo^-1 t_o, the operator
 *   of qmg_schur_apply), e_o = A_oo^-1 (t_o - D_oe e_e), z += e.
 * eo = 2: as eo = 1, with the GMRES steps in s-step form (n_post_smooth <= 8; otherwise as 1):
 *   the same minimisation of ||bhat - Dhat e_e|| over the Krylov space of dimension
 *   n_post_smooth, from the basis bhat, Dhat bhat, ..., one pass of inner products and an FP64
 *   normal-equation solve (equilibrated Cholesky; a pivot below 1e-13 ends the basis) on the
 *   device, instead of n_post_smooth Gram-Schmidt steps.  The half-lattice gauge field,
 *   site term and its inverse are built once (FP64, and in the inner precision when that is
 *   not FP64) from the handle's fields; when every link is SU(3) to 1e-12 (third row = complex
 *   conjugate of the cross product of the first two) only the first two rows are stored and
 *   the hop kernels rebuild the third.  Synchronizes the stream.  Works with every form of
 *   qmg_mg_set_cycle.  The choice is not stored by qmg_mg_save.
 * Errors: EINVAL (null, eo not 0/1/2), ESHAPE (an odd extent), EBREAKDOWN (a singular site
 *   block), ENOMEM, EHIP. */
qmg_status qmg_mg_set_smoother(qmg_mg* mg, int32_t eo, hipStream_t stream);

/* Even-odd coarse solve (Section 1 names even-odd preconditioning; here it is applied to the
 * Galerkin operator D_c of Eq. (5)).  The aggregates are coloured by the parity of their coarse
 * coordinates (every coarse extent must be even, so every hop block of D_c joins aggregates of
 * opposite colour) and the coarse solve of the K-cycle runs GMRES on the Schur complement
 *   Dhat_c = Y_ee - Y_eo Y_oo^-1 Y_oe,   rhat_e = r_e - Y_eo Y_oo^-1 r_o,
 *   v_o = Y_oo^-1 (r_o - Y_oe v_e),
 * to the coarse tolerance relative to rhat_e.  on = 1 builds Y_0(j)^-1 Y(j) for every
 * aggregate from the current D_c in FP64 (self blocks inverted by Gauss-Jordan with partial
 * pivoting) and its inner-precision copy, and rebuilds them whenever the coarse operator is
 * rebuilt (qmg_mg_stream_more); on = 0 returns to the full coarse operator and releases them.
 * When a build fails (here or inside qmg_mg_stream_more) the blocks are released and the
 * Schur coarse solve is off.  Synchronizes the stream.  Applies to the host-checked coarse solve of
 * a two-level hierarchy (qmg_mg_set_cycle with coarse_steps = 0; a further level added later
 * takes precedence).  Not stored by qmg_mg_save.  With an FP64 K-cycle it reduced the outer
 * iterations on every operator tried; with a lower-precision K-cycle the outer count can move
 * either way with the operator (rounding-sensitive), so it is off by default.
 * Errors: EINVAL (null, on not 0/1, further levels exist), ESHAPE (an odd coarse extent),
 *   EBREAKDOWN (a self block whose pivot falls below 1e-13 of its largest entry, or entries
 *   of Y_0^-1 Y beyond half the largest finite value of the inner storage type), ENOMEM, EHIP. */
qmg_status qmg_mg_set_coarse_eo(qmg_mg* mg, int32_t on, hipStream_t stream);

/* out_e = Dhat_c in_e (above) on half coarse vectors [nrhs][d/2][2k] (device, canonical coarse
 * order within the half: the even-coloured aggregates in increasing index order), prec F64 or
 * the F32 inner precision.  Needs qmg_mg_set_coarse_eo(mg, 1).  Synchronizes the stream.
 * Errors: EINVAL (null, aliasing, nrhs < 1, even-odd coarse operator not set up), EDTYPE, ENOMEM,
 *   EHIP. */
qmg_status qmg_coarse_schur_apply(const qmg_mg* mg, const void* in, void* out, int32_t nrhs, qmg_prec prec,
                                  hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): qmg_coarse_schur_apply with the same arguments,
 * result and errors, but its intermediate half vector lives in a fixed device array of the
 * library (QMG_NOALLOC_SCRATCH_BYTES bytes, one per device, held until the process ends), so
 * the call makes no hipMalloc / hipFree and does not synchronize the stream (asynchronous, like
 * the apply calls).  The array's address on a device is looked up on the first call on that
 * device.  Every call on one device shares that array: calls that overlap on one device (on
 * different streams, or from different threads) race and must be ordered by the caller.
 * Limit: nrhs * k * d * (16 bytes for F64, 8 for F32) <= QMG_NOALLOC_SCRATCH_BYTES (d
 * aggregates, k per chirality).  Additional error: ESHAPE when a call needs more than that. */
#define QMG_NOALLOC_SCRATCH_BYTES (16u << 20)
qmg_status qmg_coarse_schur_apply_noalloc(const qmg_mg* mg, const void* in, void* out, int32_t nrhs,
                                          qmg_prec prec, hipStream_t stream);

/* D_c x = b (full coarse vectors [nrhs][d][2k], device, FP64) through the Schur complement
 * above: GMRES(32) from zero on Dhat_c to tol relative to rhat_e within max_iter steps, then the
 * odd part; *iters = GMRES steps.  Needs qmg_mg_set_coarse_eo(mg, 1).  Synchronizes the stream.
 * Errors: EINVAL (null, aliasing, bad counts or tol, not set up), ENOCONV (x holds the last
 *   iterate), ENOMEM, EHIP. */
qmg_status qmg_coarse_eo_solve(const qmg_mg* mg, const void* b, void* x, int32_t nrhs, double tol,
                               int32_t max_iter, int32_t* iters, hipStream_t stream);

/* Many independent small lattices in one hierarchy object (batching form 2: many lattices of
 * uneven size, each with its own extents, boundary, mass, anisotropy and gauge field; one aggregate
 * shape, test-vector count, batch and rank for all).  Every step of Algorithm 4 with Algorithm 3
 * (Philox test vectors, the Eq. (2) smoothing, the chiral split and gather, the streaming SVD over
 * all (aggregate, chirality) problems of all lattices, the Galerkin blocks of Eq. (5)) and every
 * step of the K-cycle solve runs as shared launches over all lattices: the fine fields of the
 * lattices are zero-padded to a common volume and stacked, each (lattice, right-hand side) pair is
 * one column of the Krylov solvers (inner products, norms and convergence per lattice).  The
 * Galerkin blocks are formed by probing (colour-separated unit coarse vectors prolonged, the fine
 * operator applied, restricted) in FP64.  Wilson operator only; K-cycle in FP64 or FP32 (then
 * inside FP64 defect correction, the smoothing below FP64 in s-step form as in the single-lattice
 * setup); plain GMRES post-smoothing on D; coarse GMRES(32).
 * qmg_batch_setup: lats host array of n_lat descriptors; U host array of n_lat device pointers to
 *   canonical FP64 gauge fields [4][V_l][3][3]; params as qmg_mg_setup_stream_chiral_svd (block
 *   dividing every lattice's extents with every coarse extent >= 3, test_vectors NULL, no clover
 *   coefficients, inner_prec F64 or F32, rank <= 32, rank + batch <= 64).  Test vector i of
 *   every lattice is the counter-based generator's vector i for that lattice's volume, as in the
 *   single-lattice setup with the same seed.  Synchronizes the stream.
 * qmg_batch_solve: rhs, x host arrays of n_lat device pointers to canonical FP64 spinors
 *   [nrhs][V_l][4][3] (x written); every lattice and right-hand side to a true FP64 relative
 *   residual tol; info (optional) [n_lat * nrhs], lattice-major (the iteration counts are those of
 *   the shared solve).  Synchronizes the stream.
 * qmg_batch_get_prolongator / _get_coarse: lattice lat's P [d_l][2][N][k] (rows in the canonical
 *   order of qmg_mg_get_prolongator) and sigma [d_l][2][k] (host), and its Galerkin blocks
 *   [d_l][9][2k][2k] (row-major, FP64, device).  qmg_batch_query: d_l and k.
 *   qmg_batch_setup_times: seconds of smoothing, streaming SVD, coarse build and the whole setup.
 * Errors: EINVAL (null, counts), ESHAPE (extents, block, rank), EDTYPE, ENOTIMPL (clover),
 *   ENONFINITE (non-finite links or residuals), ENOCONV, ENOMEM, EHIP. */
typedef struct qmg_batch qmg_batch;
qmg_status qmg_batch_setup(int32_t n_lat, const qmg_lattice* lats, const void* const* U,
                           const qmg_mg_params* params, qmg_batch** out, hipStream_t stream);
qmg_status qmg_batch_solve(const qmg_batch* b, const void* const* rhs, void* const* x, int32_t nrhs,
                           double tol, int32_t max_outer, qmg_solve_info* info, hipStream_t stream);
qmg_status qmg_batch_query(const qmg_batch* b, int32_t lat, int32_t* n_agg, int32_t* rank);
qmg_status qmg_batch_get_prolongator(const qmg_batch* b, int32_t lat, void* P, double* sigma,
                                     hipStream_t stream);
qmg_status qmg_batch_get_coarse(const qmg_batch* b, int32_t lat, void* Y, hipStream_t stream);
qmg_status qmg_batch_setup_times(const qmg_batch* b, double* t);
void qmg_batch_destroy(qmg_batch* b);

/* Measurement hooks.  qmg_timing_enable(n), n >= 1, clears the record and times the first later
 * launch of each kernel family and then about one in n (picked by a hash of the call index)
 * with a pair of HIP events attached to the dispatch (its own start and end).  Every
 * kernel of the library belongs to a family: the operators ("dslash/site", "dslash/twalk",
 * "dslash/dir", "dslash/canonical", "dslash/batched", "clover/...", "evenodd/hop",
 * "coarse_apply", "coarse_eo", "prolong", "restrict", "level_..."), the Krylov vector kernels
 * ("blas/mdot_norm", "blas/axpy_scale", "blas/axpy_multi", ..., "krylov/givens", "sstep/..."),
 * the setup ("setup/philox", "setup/gather", "isvd/...", "coarse_build", ...), layout
 * conversions ("layout/...", "eo_layout/...") and the many-lattice hierarchy ("batch/dslash",
 * "batch/prolong", "batch/restrict", "batch/coarse_apply", "batch/coarse_build", "batch/gather",
 * "batch/philox").  0 stops recording.  qmg_timing_query returns, for one family, the launches timed, their
 * summed duration (ms, it synchronizes on the events) and their summed algorithmic bytes and
 * flops; a name without '/' also sums its sub-families ("dslash").  Errors: EINVAL (n < 0). */
qmg_status qmg_timing_enable(int32_t on);
qmg_status qmg_timing_query(const char* family, int64_t* launches, double* total_ms, double* algo_bytes,
                            double* algo_flops);
/* Every launch of the family (timed or not) since qmg_timing_enable.  Errors: EINVAL (null). */
qmg_status qmg_timing_calls(const char* family, int64_t* calls);
/* The names of every family launched since qmg_timing_enable, newline-separated, into buf
 * (host, len bytes, NUL-terminated).  Errors: EINVAL (null, len < 1), ESHAPE (buf too short). */
qmg_status qmg_timing_list(char* buf, int32_t len);

/* Device memory.  The library's buffers (hierarchies, solver workspaces) come from a cache of
 * freed blocks per device in front of hipMalloc, so repeated setups and solves reuse their
 * blocks; a block is cached only after the device has finished its work (the wait hipFree
 * performs), the cache holds at most half of the device memory (environment QMG_CACHE_GB
 * overrides, 0 disables caching), and a failed hipMalloc releases it and retries.
 * qmg_memory_trim returns the cache of the current device to the runtime (synchronizes the
 * device); qmg_memory_cached reports its size in bytes.  Errors: EINVAL (null). */
qmg_status qmg_memory_trim(void);
qmg_status qmg_memory_cached(int64_t* bytes);

/* Autotuner.  qmg_autotune(1) (or QMG_TUNE=1 in the environment) makes every kernel with
 * launch variants (the native-layout dslash: one site per thread, 2/4/8 sites per thread
 * along t, four threads per site, or 2-3 right-hand sides per thread along t) time each variant with HIP events on its first call for a given (precision,
 * extents, right-hand sides, adjoint) and keep the fastest; 0 returns to the built-in
 * heuristic.  Tuning never runs while the stream is being captured into a graph.
 * qmg_tune_save / qmg_tune_load write / read the choices as JSON {"key": variant}. */
qmg_status qmg_autotune(int32_t on);
/* Force one native-layout dslash variant for every later call (1: one site per thread; 2, 4, 8:
 * sites per thread along t, used when Lt is a multiple; 16: four threads per site, one per
 * direction; 32, 64: one site per thread for 2 or 4 right-hand sides at once, used when nrhs is
 * a multiple; 1000 z + 100 NR + TCH with z in {0, 1}, NR in {2, 3}, TCH in {2, 4, 8}: TCH sites
 * along t for NR right-hand sides per thread, FP32 storage only, z = 1 orders the tiles z-fastest;
 * 10000 + a t-walking code: the same with the workgroups in t-chunk-major order; for the
 * even-odd hop, 500 + NR (NR in 1..4 right-hand sides per thread) or 7ZT (tiles in patches of
 * Z x T (z, t) planes, Z and T in {1, 2, 4, 8}, where whole tiles fill a plane; 700:
 * lexicographic order); a variant that does not apply to a call falls back to the automatic
 * choice); 0 restores the automatic choice.  Any other value gives QMG_EINVAL.
 * For tests and tuning studies. */
qmg_status qmg_set_dslash_variant(int32_t variant);
qmg_status qmg_tune_save(const char* path);
qmg_status qmg_tune_load(const char* path);

void qmg_mg_destroy(qmg_mg* mg);
const char* qmg_last_error(void);
const char* qmg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QMG_H */
