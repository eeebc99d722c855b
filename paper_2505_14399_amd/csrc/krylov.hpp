// Vector kernels and Krylov solvers over native complex arrays [nrhs][len].
//
// Reductions accumulate in double and are deterministic: each workgroup reduces a fixed
// slice (wavefront shuffles, then LDS), partial sums are combined in fixed order by a
// second pass.  Coefficients produced by one kernel (inner products, norms) stay on the
// device and are consumed by the next, so a Krylov iteration needs no host round trip
// except the one that reads the small Hessenberg column for the convergence test.
#pragma once

#include <type_traits>

#include "qmg_internal.hpp"

namespace qmg {

struct LinOp {
  virtual ~LinOp() = default;
  // out = A in, nrhs vectors of len() complex numbers each, storage prec().  skip: a device
  // flag; an operator may return at once when it is set (device-side early exit), or ignore it
  virtual void apply(const void* in, void* out, int nrhs, hipStream_t st, const int* skip = nullptr) = 0;
  virtual size_t len() const = 0;
  virtual qmg_prec prec() const = 0;
};

struct Precond {
  virtual ~Precond() = default;
  // z ~ A^-1 r (may vary between calls: flexible outer solver required)
  virtual void apply(const void* r, void* z, int nrhs, hipStream_t st) = 0;
};

// scratch for two-pass reductions; the second buffer lets a kernel that sums one set of
// partials (from the previous kernel) write the next set in the same launch
struct RedWork {
  DevBuf partial;   // double2 partial sums
  DevBuf partial2;  // second partial buffer
  DevBuf result;    // double2 results
  void ensure(size_t npart, size_t nres) {
    partial.ensure(npart * sizeof(double2));
    result.ensure(nres * sizeof(double2));
  }
  void ensure2(size_t npart) { partial2.ensure(npart * sizeof(double2)); }
};

template <class S>
struct Blas {
  static void zero(void* x, size_t n, hipStream_t st);
  static void copy(const void* x, void* y, size_t n, hipStream_t st);
  // y = a x + b y (real scalars)
  static void axpby(double a, const void* x, double b, void* y, size_t n, hipStream_t st);
  // out[i * nrhs + r] = <X_i[r], w[r]>, X_i = X + i * xstride complex entries, i < m
  static void dot_multi(const void* X, size_t xstride, int m, const void* w, size_t len, int nrhs,
                        double2* out, RedWork& rw, hipStream_t st);
  // as dot_multi, reading w once per group of up to 8 vectors
  static void mdot(const void* X, size_t xstride, int m, const void* w, size_t len, int nrhs, double2* out,
                   RedWork& rw, hipStream_t st, const int* skip = nullptr);
  // w[r] += sgn * sum_i c[i * nrhs + r] X_i[r], then out = <X_i[r], w[r]> (fused)
  static void axpy_mdot(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w, size_t len,
                        int nrhs, double2* out, RedWork& rw, hipStream_t st, const int* skip = nullptr);
  // w[r] += sgn * sum_i c[i * nrhs + r] X_i[r], then out[r] = ||w[r]||^2 (fused)
  static void axpy_norm(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w, size_t len,
                        int nrhs, double* out, RedWork& rw, hipStream_t st, const int* skip = nullptr);
  // one Gram-Schmidt step: h = X^dag w (m vectors), w <- (w - X h) / beta with
  // beta^2 = |w|^2 - |h|^2, n2[r] = beta^2 (device); h needs (m + 1) * nrhs slots, slot m
  // receives |w|^2 before the update.  With gst, the GMRES Givens step for Hessenberg column
  // m - 1 (restart length gm) runs in the same launch and writes its estimates to est; returns
  // whether it did.
  // With conv (device counters, see Gmres::solve) the Givens step also tests est <= tol and the
  // kernels return at once once every rhs has converged.
  static bool cgs1_step(const void* X, size_t xstride, int m, void* w, size_t len, int nrhs, double2* h, double* n2,
                        RedWork& rw, hipStream_t st, double2* gst = nullptr, int gm = 0, double2* est = nullptr,
                        double tol = 0.0, int* conv = nullptr);
  // two Gram-Schmidt passes: h1 = X^dag w ; w -= X h1 ; h2 = X^dag w ; w -= X h2 ;
  // n2[r] = |w|^2 ; w /= |w| (h1, h2, n2 on the device)
  static void cgs2_step(const void* X, size_t xstride, int m, void* w, size_t len, int nrhs, double2* h1,
                        double2* h2, double* n2, RedWork& rw, hipStream_t st, const int* skip = nullptr);
  // out[r] = ||w[r]||^2
  static void norm2(const void* w, size_t len, int nrhs, double* out, RedWork& rw, hipStream_t st);
  // w[r] += sgn * sum_i c[i * nrhs + r] X_i[r]
  // (mcount: optional device int per rhs capping m for that rhs)
  static void axpy_multi(const void* X, size_t xstride, int m, const double2* c, double sgn, void* w,
                         size_t len, int nrhs, hipStream_t st, const int* skip = nullptr, const int* mcount = nullptr);
  // w[r] *= f(n2[r]) with f = 1/sqrt (mode 0) or sqrt (mode 1) or a direct factor (mode 2,
  // n2 then holds the factor); a zero norm gives a zero vector in mode 0
  static void scale_dev(void* w, const double* n2, int mode, size_t len, int nrhs, hipStream_t st,
                        const int* skip = nullptr);
  // w[r] *= c[r] (complex, device)
  static void scale_cdev(void* w, const double2* c, double sgn, size_t len, int nrhs, hipStream_t st);
  // x[r] += sgn * c[r] * y[r]  (complex scalar per rhs, on device)
  static void caxpy_dev(const double2* c, double sgn, const void* y, void* x, size_t len, int nrhs,
                        hipStream_t st);
};

// Restarted GMRES(m) and flexible GMRES(m), multi right-hand side: Arnoldi with classical
// Gram-Schmidt (twice in FP64) and the Givens least-squares update on the device; with a
// tolerance the host reads the residual estimates once per few steps (after every step in the
// flexible form), without one a cycle has no host round trip.
template <class S>
class Gmres {
 public:
  struct Result {
    int iters = 0;           // Arnoldi steps taken (max over rhs)
    bool converged = true;
    std::vector<double> rel_est;  // final residual estimate / ||b|| per rhs
  };
  // x: initial guess if !x_zero, solution on return.  tol <= 0: exactly max_iter steps.
  // conv (device int[3], optional): device-side exit for graph capture: one cycle of max_iter
  // <= restart steps from a zero guess; conv[0] counts converged rhs, conv[1] is raised when
  // all have converged (later kernels of the cycle return at once), conv[2] accumulates the
  // steps of rhs 0.  No host round trip; iters is then -1.
  // first_check (host-checked mode): Arnoldi step after which the host first reads the
  // estimates (later every two steps); 0 = every four steps.  A caller that knows the typical
  // count (the previous solve's) saves host round trips without changing the result.
  // M (optional): flexible GMRES, z_j = M v_j with a preconditioner that may change between
  // applications (the solution is updated with the z_j).
  Result solve(LinOp& A, const void* b, void* x, bool x_zero, int nrhs, int restart, int max_iter, double tol,
               hipStream_t st, int* conv = nullptr, int first_check = 0, Precond* M = nullptr);
  // Arnoldi orthogonalisation: two classical Gram-Schmidt passes (default in FP64) or one pass
  // with the norm from Pythagoras (default below FP64)
  void set_cgs2(bool on) { cgs2_ = on; }

 private:
  bool cgs2_ = std::is_same<S, double2>::value;
  void ensure(size_t len, int nrhs, int restart);
  DevBuf V_, Z_, H_, h1_, h2_, nrm_, y_, r_, cols_, gst_;
  PinnedBuf hb_;
  RedWork rw_;
  size_t len_ = 0;
  int nrhs_ = 0, restart_ = 0;
};

// s-step form of n_iter (a multiple of 8) restarted GMRES(8) steps on D x = b from zero, with the
// shifted basis p_{i+1} = (D - d) p_i (H, when given, applies D - d directly); r right-hand sides
// of len complex numbers; the buffers are work space (sized here).  Instantiated below FP64.
template <class S>
void smooth_sstep(size_t len, double d, LinOp& D, LinOp* H, int r, int n_iter, const void* b, void* x, DevBuf& basis,
                  DevBuf& coef, DevBuf& part, DevBuf& e, hipStream_t st);

// One pass over the s-step basis p_0 .. p_s (vectors vstride apart, nrhs right-hand sides of len
// complex numbers each, coefficients c[j * nrhs + rhs]): x += sum_j c_j p_j (x = ... without
// add) and, with res, p_0 -= sum_j c_j (p_{j+1} + d p_j) in place.  s <= 8.
template <class S>
void sstep_update(const void* basis, size_t vstride, int s, const double2* c, double d, void* x, void* p0, size_t len,
                  int nrhs, bool res, bool add, hipStream_t st);

// Defect correction between an FP64 outer residual and an FP32 inner solve, nrhs columns of len
// complex numbers, one pass over the vectors per call:
//   dc_residual:   r = b - r (r holds D x on entry) and n2[c] = |r_c|^2, FP64 (device);
//   dc_normalise:  rin = FP32(r / |r|) per column (zero for a zero norm), from n2;
//   dc_accumulate: x += |r| e per column, e the FP32 inner solution, x in FP64.
void dc_residual(const void* b64, void* r64, size_t len, int nrhs, double* n2, RedWork& rw, hipStream_t st);
void dc_normalise(const void* r64, const double* n2, void* rin, size_t len, int nrhs, hipStream_t st);
void dc_accumulate(const void* ein, const double* n2, void* x64, size_t len, int nrhs, hipStream_t st);

}  // namespace qmg
