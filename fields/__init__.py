"""Seeded synthetic inputs shared by the oracle, the GPU tests and the benchmark.

This module only *generates fields*: gauge links, sources, gauge transforms.
It holds none of the multigrid method's arithmetic (no Dirac operator, no
smoother, no SVD, no transfer or coarse operator), so both the CPU oracle and
the HIP path can take their inputs from here without sharing any of the
computation they are compared on.

Canonical layouts (complex128, row-major):
  gauge   [4 mu][V][3][3]        U_mu(x): link from x to x+mu (physical, no BC sign)
  spinor  [nrhs][V][4 spin][3 colour]
Site index: x + Lx*(y + Ly*(z + Lz*t)), mu = 0,1,2,3 = x,y,z,t.

Random streams: numpy PCG64 seeded with SeedSequence([seed, stream, tag]):
  stream 0 gauge field, 1 right-hand sides, 2 gauge transforms, 3 eta (adjoint
  source), 4 per-lattice parameters of batched workloads.
"""
from __future__ import annotations

import numpy as np

GAUGE_STREAM, RHS_STREAM, GT_STREAM, ETA_STREAM, PARAM_STREAM = 0, 1, 2, 3, 4


def rng(seed: int, stream: int, tag: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream, tag])))


def volume(dims) -> int:
    return int(np.prod(dims))


def _hermitian_traceless(g: np.random.Generator, n: int) -> np.ndarray:
    a = g.standard_normal((n, 3, 3)) + 1j * g.standard_normal((n, 3, 3))
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h -= tr[:, None, None] * np.eye(3)
    return h


def _exp_i(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*h) for a batch of Hermitian 3x3 matrices, via eigh (FP64)."""
    lam, q = np.linalg.eigh(h)
    ph = np.exp(1j * eps * lam)
    return np.einsum("nij,nj,nkj->nik", q, ph, np.conj(q))


def random_gauge(dims, eps: float, seed: int, tag: int = 0, chunk: int = 1 << 20) -> np.ndarray:
    """U_mu(x) = exp(i*eps*H), H Gaussian traceless Hermitian; eps = 0 is the free field.

    Draw order is site-lexicographic with mu innermost.  Returns [4][V][3][3] complex128.
    """
    V = volume(dims)
    g = rng(seed, GAUGE_STREAM, tag)
    out = np.empty((V, 4, 3, 3), dtype=np.complex128)
    flat = out.reshape(V * 4, 3, 3)
    n = V * 4
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        flat[s:e] = _exp_i(_hermitian_traceless(g, e - s), eps)
    return np.ascontiguousarray(out.transpose(1, 0, 2, 3))


def random_su3(n: int, seed: int, tag: int = 0) -> np.ndarray:
    """n random SU(3) matrices exp(iH) (used as gauge transformations g(x))."""
    g = rng(seed, GT_STREAM, tag)
    return _exp_i(_hermitian_traceless(g, n), 1.0)


def gaussian_spinor(dims, nrhs: int, seed: int, stream: int = RHS_STREAM, tag: int = 0) -> np.ndarray:
    """Complex Gaussian spinors, Re and Im ~ N(0,1).  [nrhs][V][4][3]."""
    V = volume(dims)
    g = rng(seed, stream, tag)
    return g.standard_normal((nrhs, V, 4, 3)) + 1j * g.standard_normal((nrhs, V, 4, 3))


def point_sources(dims, site: int = 0) -> np.ndarray:
    """The 12 spin-colour unit sources at one site.  [12][V][4][3]."""
    V = volume(dims)
    b = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for s in range(4):
        for c in range(3):
            b[3 * s + c, site, s, c] = 1.0
    return b


def gaussian_coarse(n_coarse: int, nrhs: int, seed: int, tag: int = 0) -> np.ndarray:
    """Complex Gaussian coarse vectors [nrhs][n_coarse]."""
    g = rng(seed, RHS_STREAM, 1000 + tag)
    return g.standard_normal((nrhs, n_coarse)) + 1j * g.standard_normal((nrhs, n_coarse))


def gaussian_test_vectors(dims, n: int, seed: int, tag: int = 0) -> np.ndarray:
    """Explicit initial test-vector guesses phi (for the test hook that bypasses the counter RNG)."""
    return gaussian_spinor(dims, n, seed, stream=RHS_STREAM, tag=2000 + tag)


def batched_lattice_params(n_lat: int, seed: int, sizes=(8, 10, 12), mass_range=(0.01, 0.1)):
    """Per-lattice extents and masses of a many-small-lattices workload."""
    g = rng(seed, PARAM_STREAM, 0)
    L = g.choice(np.asarray(sizes), size=n_lat)
    m = g.uniform(mass_range[0], mass_range[1], size=n_lat)
    return [int(v) for v in L], [float(v) for v in m]
