"""Test-vector smoothing, the iCSVD multigrid setup and the two-level K-cycle solve.

Setup (Algorithm 4 with Algorithm 3): for every stream s, r random initial
guesses phi_i are smoothed on D psi ~ 0 (Eq. (2): psi = phi + psi' with
D psi' ~ -D phi), the chirally split, blocked vectors update the streaming rank-k
SVD, and after the last stream P = U_k, R = P^dagger and D_c = R D P (Eq. (5)).

Readings where the paper gives no value (Section 4 gives FGMRES, 8 post-smoothing
iterations and coarse solves to 0.03 ||b||):
  smoother      GMRES(8), n_setup iterations in total from a zero guess; psi is then
                normalised to unit 2-norm
  cycle         two levels; the coarse system R r is solved by GMRES(32) to a residual
                of 0.03 of its right-hand side (at most 500 iterations); the coarse
                correction is prolonged and followed by 8 GMRES post-smoothing
                iterations on D e = r; no pre-smoothing
  outer solver  flexible GCR(16) in FP64 to ||b - D x|| <= tol ||b||
"""
import numpy as np

from . import wilson, clover, krylov, icsvd as ic, transfer, coarse, philox
from .geometry import volume, coarse_dims


class Lattice:
    """The fine operator: Wilson, or Wilson-clover when the clover term T [V][12][12]
    (clover.clover_term) is given."""

    def __init__(self, U, dims, mass, xi=1.0, bc_t=-1, T=None):
        self.U, self.dims, self.mass, self.xi, self.bc_t = U, tuple(dims), mass, xi, bc_t
        self.T = T

    def D(self, psi):
        if self.T is not None:
            return clover.apply_clover(self.U, self.T, psi, self.mass, self.xi, self.bc_t, self.dims)
        return wilson.apply_wilson(self.U, psi, self.mass, self.xi, self.bc_t, self.dims)

    def Ddag(self, psi):
        if self.T is not None:
            return clover.apply_clover(self.U, self.T, psi, self.mass, self.xi, self.bc_t, self.dims, dagger=True)
        return wilson.apply_wilson(self.U, psi, self.mass, self.xi, self.bc_t, self.dims, dagger=True)


def smooth(lat, phi, n_iter, restart=8):
    """Eq. (2): psi = phi + psi', psi' from n_iter GMRES iterations on D psi' = -D phi."""
    if n_iter == 0:
        psi = phi.copy()
    else:
        rhs = -lat.D(phi)
        dpsi, _, _ = krylov.gmres(lat.D, rhs, None, restart=restart, max_iter=n_iter, tol=0.0)
        psi = phi + dpsi
    return psi / np.linalg.norm(psi.ravel())


def initial_guess(seed, v, V, test_vectors=None):
    if test_vectors is not None:
        return test_vectors[v].copy()
    return philox.gaussian_test_vector(seed, v, V)


class Hierarchy:
    pass


def setup(lat, block, n_test, batch, rank, n_setup_iter=16, seed=0, test_vectors=None, restart=8):
    """Algorithm 4 (one level) with Algorithm 3 as the basis generator."""
    if n_test % batch != 0:
        raise ValueError("n_test must be a multiple of the stream batch r")
    n_s = n_test // batch
    V = volume(lat.dims)

    def streams():
        for s in range(n_s):
            psi = np.stack([smooth(lat, initial_guess(seed, s * batch + i, V, test_vectors),
                                   n_setup_iter, restart) for i in range(batch)])
            yield psi

    h = Hierarchy()
    h.lat, h.block, h.k = lat, tuple(block), rank
    h.cdims = coarse_dims(lat.dims, block)
    h.P, h.sigma, h.sigma_hist = ic.icsvd(streams(), n_s, lat.dims, block, rank)
    h.Y = coarse.build_coarse(lat.U, h.P, lat.mass, lat.xi, lat.bc_t, lat.dims, block, T=lat.T)
    return h


def prolong(h, vc):
    return transfer.prolong(h.P, vc, h.lat.dims, h.block)


def restrict(h, psi):
    return transfer.restrict(h.P, psi, h.lat.dims, h.block)


def coarse_op(h, vc):
    return coarse.coarse_apply(h.Y, vc, h.cdims)


def kcycle(h, r, coarse_tol=0.03, coarse_restart=32, coarse_max=500, n_post=8, stats=None):
    """Two-level K-cycle preconditioner M(r) (Section 2.1; parameters of Section 4)."""
    rc = restrict(h, r[None])
    ec, it_c, _ = krylov.gmres(lambda v: coarse_op(h, v), rc, None, restart=coarse_restart,
                               max_iter=coarse_max, tol=coarse_tol)
    e = prolong(h, ec)[0]
    e, it_s, _ = krylov.gmres(h.lat.D, r, e, restart=n_post, max_iter=n_post, tol=0.0)
    if stats is not None:
        stats["coarse"] += it_c
        stats["smoother"] += it_s
        stats["cycles"] += 1
    return e


def solve(h, b, tol=1e-10, max_iter=1000, restart=16, adjoint=False, **kw):
    """MG-preconditioned flexible GCR in FP64.  Returns (x, stats).

    adjoint=True solves D^dagger x = b as gamma5 D^-1 gamma5 b with the same hierarchy.
    """
    if adjoint:
        x, st = solve(h, wilson.gamma5(b), tol, max_iter, restart, **kw)
        return wilson.gamma5(x), st
    stats = {"coarse": 0, "smoother": 0, "cycles": 0}
    x, it, hist = krylov.fgcr(h.lat.D, lambda r: kcycle(h, r, stats=stats, **kw), b,
                              None, tol=tol, restart=restart, max_iter=max_iter)
    stats["outer"] = it
    stats["hist"] = hist
    stats["true_rel_res"] = float(np.linalg.norm((b - h.lat.D(x)).ravel()) / np.linalg.norm(b.ravel()))
    return x, stats
