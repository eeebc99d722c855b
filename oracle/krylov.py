"""Krylov solvers: restarted GMRES (smoother and coarse solver) and flexible GCR.

The paper uses FGMRES as smoother and solver on every level and a flexible outer
solver (FGMRES or GCR) preconditioned by a K-cycle (Section 2.1, Section 4).  The
smoother and the coarse solver here are unpreconditioned, so FGMRES reduces to
GMRES; the outer solver is flexible GCR.  GMRES uses the Arnoldi process with
modified Gram-Schmidt and Givens rotations for the small least-squares problem.

Vectors are numpy complex arrays of any shape; inner products are over all entries.
"""
import numpy as np


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _nrm(a):
    return float(np.linalg.norm(a.ravel()))


def gmres(A, b, x0=None, restart=8, max_iter=16, tol=0.0):
    """Restarted GMRES(restart) on A x = b.

    Runs until `max_iter` Arnoldi steps in total, or until the Givens residual
    estimate is <= tol * ||b||.  Returns (x, iterations, history of residual estimates).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnrm = _nrm(b)
    target = tol * bnrm
    it = 0
    hist = []
    while it < max_iter:
        r = b - A(x) if (x0 is not None or it > 0) else b.copy()
        beta = _nrm(r)
        hist.append(beta)
        if beta == 0.0 or beta <= target:
            break
        m = min(restart, max_iter - it)
        Vb = [r / beta]
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.float64)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        j_done = 0
        for j in range(m):
            w = A(Vb[j])
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = _dot(Vb[i], w)
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = _nrm(w)
            for i in range(j):                           # apply previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]                  # new rotation zeroing H[j+1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den if abs(a) > 0 else 1.0
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= target:
                break
            Vb.append(w / _nrm(w) if _nrm(w) > 0 else w)
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        for i in range(j_done):
            x = x + y[i] * Vb[i]
        if abs(g[j_done]) <= target:
            break
    return x, it, hist


def fgcr(A, M, b, x0=None, tol=1e-10, restart=16, max_iter=1000):
    """Flexible GCR: z_k = M(r_k) may change from step to step (K-cycle preconditioner).

    Stops when ||r|| <= tol ||b|| where r is the recursively updated residual; the
    true residual b - A x is recomputed at every restart.  Returns (x, iterations, history).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnrm = _nrm(b)
    r = b - A(x) if x0 is not None else b.copy()
    hist = [_nrm(r) / bnrm]
    it = 0
    while it < max_iter and hist[-1] > tol:
        Z, W = [], []
        for _ in range(restart):
            z = M(r)
            w = A(z)
            for zi, wi in zip(Z, W):                     # modified Gram-Schmidt on w
                beta = _dot(wi, w)
                w = w - beta * wi
                z = z - beta * zi
            nw = _nrm(w)
            w, z = w / nw, z / nw
            alpha = _dot(w, r)
            x = x + alpha * z
            r = r - alpha * w
            Z.append(z)
            W.append(w)
            it += 1
            hist.append(_nrm(r) / bnrm)
            if hist[-1] <= tol or it >= max_iter:
                break
        r = b - A(x)                                     # true residual at restart
        hist[-1] = _nrm(r) / bnrm
    return x, it, hist
