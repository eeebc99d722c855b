"""The next coarser level of a coarse stencil operator (a third multigrid level).

Test infrastructure: only tests/, the smoke check and the benchmark's CPU baseline use
this package (see oracle/__init__.py).

The paper's hierarchies have three and four levels (Section 4, Tables 1-3): the setup of
Algorithm 4 with Algorithm 3 is applied again to the coarse operator D_c of Eq. (5).  On
a coarse level:

  sites        the coarse sites j of D_c (aggregates of the level below), lexicographic
               on the coarse lattice
  components   the 2k coarse degrees of freedom (alpha, i) of a site
  chirality    the coarse gamma5 is sigma3 (+1 on alpha = 0, Section 2.1): the chiral split
               of Eq. (3) keeps the alpha block of every site
  test vectors random complex Gaussian coarse vectors, Philox counter (j, g, v, level)
               giving components 2g and 2g + 1 (the fine generator is the case level = 0,
               2k = 12); n_setup GMRES(8) iterations on D_c psi' = -D_c phi from zero,
               psi = phi + psi', normalised to unit 2-norm
  aggregates   blocks of b2 coarse sites; the rows of a (J, alpha) block are ordered
               (site in block, i), N2 = k n_d2
  basis        Algorithm 3 per (J, alpha); P2 = U_k2
  operator     D_cc = P2^dag D_c P2 as a nine-block stencil (Eq. (5) one level down): for
               coarse site j and each term of D_c (the self block, or the hop block towards
               t = j + dir), P2(j)^dag Y_dir(j) P2(t) goes to the self block of j's aggregate
               for the self term and for hops that stay inside the aggregate, and to the
               directional block dir for hops that leave it through its face
               (c_mu mod b2_mu = b2_mu - 1 forward, = 0 backward), also when that face leads
               back into the same aggregate (coarse-coarse extent 1 or 2)

Readings (the paper only says that every level is set up the same way): the smoother, the
setup iteration count, the chirality convention and the coarse tolerance of level one are
used on every level; the K-cycle of level l solves level l + 1 by a flexible Krylov method to
0.03 of its right-hand side (at most 500 iterations, restart 32) preconditioned by the
K-cycle of level l + 1, the coarsest level by GMRES(32) to 0.03, followed by 8 GMRES
post-smoothing iterations on level l.
"""
import numpy as np

from . import krylov, philox, icsvd as ic, coarse, mg
from .geometry import block_sites, coarse_dims, coords, neighbor_table, volume, check_block


def gaussian_coarse_vector(seed, v, d, m, level):
    """phi_v on a coarse level: [d][m] complex128, Philox counter (j, g, v, level)."""
    if m % 2:
        raise ValueError("coarse vectors have an even number of components per site")
    site = np.arange(d, dtype=np.uint64)
    out = np.empty((d, m), dtype=np.complex128)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    for g in range(m // 2):
        ctr = np.zeros((d, 4), dtype=np.uint64)
        ctr[:, 0] = site
        ctr[:, 1] = g
        ctr[:, 2] = v
        ctr[:, 3] = level
        x = philox.philox4x32_10(ctr, key).astype(np.float64)
        u = (x + 0.5) * 2.0 ** -32
        r0 = np.sqrt(-2.0 * np.log(u[:, 0]))
        r1 = np.sqrt(-2.0 * np.log(u[:, 2]))
        out[:, 2 * g] = r0 * np.cos(2 * np.pi * u[:, 1]) + 1j * r0 * np.sin(2 * np.pi * u[:, 1])
        out[:, 2 * g + 1] = r1 * np.cos(2 * np.pi * u[:, 3]) + 1j * r1 * np.sin(2 * np.pi * u[:, 3])
    return out


def chiral_block(vs, cdims, block2, k):
    """Coarse vectors vs [r][d][2k] -> blocks [d2][2][N2][r], rows (site in block, i)."""
    bs = block_sites(cdims, block2)                 # [d2][n_d2] coarse sites
    d2, nd2 = bs.shape
    r = vs.shape[0]
    v = vs.reshape(r, -1, 2, k)
    out = np.empty((d2, 2, nd2 * k, r), dtype=np.complex128)
    for a in range(2):
        g = v[:, bs, a, :]                          # [r][d2][n_d2][k]
        out[:, a] = g.reshape(r, d2, nd2 * k).transpose(1, 2, 0)
    return out


def rows(P2, cdims, block2, k):
    """[d][2k][2k2]: the rows of P2 at every coarse site (zero across chiralities)."""
    bs = block_sites(cdims, block2)
    d2, nd2 = bs.shape
    k2 = P2.shape[-1]
    d = volume(cdims)
    R = np.zeros((d, 2 * k, 2 * k2), dtype=np.complex128)
    for J in range(d2):
        for jb in range(nd2):
            j = bs[J, jb]
            for a in range(2):
                R[j, a * k:(a + 1) * k, a * k2:(a + 1) * k2] = P2[J, a, jb * k:(jb + 1) * k, :]
    return R


def aggregate_of(cdims, block2):
    bs = block_sites(cdims, block2)
    agg = np.empty(volume(cdims), dtype=np.int64)
    for J in range(bs.shape[0]):
        agg[bs[J]] = J
    return agg


def prolong(P2, v2, cdims, block2, k):
    """v1 = P2 v2: v2 [nrhs][d2][2][k2] -> v1 [nrhs][d][2k]."""
    R = rows(P2, cdims, block2, k)
    agg = aggregate_of(cdims, block2)
    nrhs = v2.shape[0]
    vv = v2.reshape(nrhs, v2.shape[1], -1)
    return np.einsum("jab,rjb->rja", R, vv[:, agg])


def restrict(P2, v1, cdims, block2, k):
    """v2 = P2^dag v1: v1 [nrhs][d][2k] -> v2 [nrhs][d2][2][k2]."""
    R = rows(P2, cdims, block2, k)
    agg = aggregate_of(cdims, block2)
    d2 = int(agg.max()) + 1
    k2 = P2.shape[-1]
    nrhs = v1.shape[0]
    contrib = np.einsum("jab,rja->rjb", np.conj(R), v1.reshape(nrhs, R.shape[0], -1))
    out = np.zeros((nrhs, d2, 2 * k2), dtype=np.complex128)
    for r in range(nrhs):
        np.add.at(out[r], agg, contrib[r])
    return out.reshape(nrhs, d2, 2, k2)


def galerkin(Y, P2, cdims, block2, k):
    """Y2 [d2][9][2k2][2k2] = P2^dag D_c P2 in stencil form (see the module text)."""
    check_block(cdims, block2)
    R = rows(P2, cdims, block2, k)
    agg = aggregate_of(cdims, block2)
    d2 = int(agg.max()) + 1
    k2 = P2.shape[-1]
    cnb = neighbor_table(cdims)
    X = coords(cdims)
    Y2 = np.zeros((d2, 9, 2 * k2, 2 * k2), dtype=np.complex128)
    d = volume(cdims)
    for j in range(d):
        Y2[agg[j], 0] += np.conj(R[j]).T @ Y[j, 0] @ R[j]
        for dd in range(8):
            mu, fwd = dd % 4, dd < 4
            t = cnb[j, dd]
            face = (X[j, mu] % block2[mu] == block2[mu] - 1) if fwd else (X[j, mu] % block2[mu] == 0)
            Y2[agg[j], 1 + dd if face else 0] += np.conj(R[j]).T @ Y[j, 1 + dd] @ R[t]
    return Y2


class Level:
    pass


def setup(Y, cdims, block2, n_test, batch, rank, n_setup_iter=16, seed=0, level=1, restart=8,
          test_vectors=None):
    """Algorithm 4 with Algorithm 3 on the coarse stencil Y (coarse extents cdims)."""
    if n_test % batch:
        raise ValueError("n_test must be a multiple of the stream batch r")
    d, m = Y.shape[0], Y.shape[-1]
    k = m // 2
    n_s = n_test // batch

    def A(v):
        return coarse.coarse_apply(Y, v[None], cdims)[0]

    def smooth(phi):
        if n_setup_iter == 0:
            psi = phi.copy()
        else:
            dpsi, _, _ = krylov.gmres(A, -A(phi), None, restart=restart, max_iter=n_setup_iter, tol=0.0)
            psi = phi + dpsi
        return psi / np.linalg.norm(psi.ravel())

    def guess(v):
        if test_vectors is not None:
            return test_vectors[v].reshape(d, m).copy()
        return gaussian_coarse_vector(seed, v, d, m, level)

    d2 = volume(coarse_dims(cdims, block2))
    Phi = [[None, None] for _ in range(d2)]   # Phi_{-1} is empty
    sigma_hist = []
    for s in range(n_s):
        psi = np.stack([smooth(guess(s * batch + i)) for i in range(batch)])
        B = chiral_block(psi, cdims, block2, k)       # [d2][2][N2][r]
        U = np.empty((d2, 2, B.shape[2], min(rank, B.shape[3] + (0 if Phi[0][0] is None else Phi[0][0].shape[1]))),
                     dtype=np.complex128)
        S = np.empty((d2, 2, U.shape[-1]))
        for J in range(d2):
            for a in range(2):
                U[J, a], S[J, a] = ic.icsvd_update(Phi[J][a], B[J, a], rank)
                Phi[J][a] = U[J, a] * S[J, a][None, :]
        sigma_hist.append(S)
    lv = Level()
    lv.Y, lv.cdims, lv.block2, lv.k, lv.k2 = Y, tuple(cdims), tuple(block2), k, rank
    lv.cdims2 = coarse_dims(cdims, block2)
    lv.P, lv.sigma, lv.sigma_hist = U, S, sigma_hist
    lv.Y2 = galerkin(Y, U, cdims, block2, k)
    return lv


def solve_levels(h, lvs, b, tol=1e-10, max_iter=1000, restart=16, coarse_tol=0.03, coarse_restart=32,
                 coarse_max=500, n_post=8):
    """K-cycle preconditioned flexible GCR in FP64 over the fine level, the first coarse level
    (h from oracle.mg.setup) and the further levels lvs (each from setup() on the stencil of the
    level above).  Returns (x, stats) with stats["iters"][l] the Krylov iterations on level l
    (l = 0 outer) and stats["smooth"][l] the post-smoothing iterations on level l."""
    L = 2 + len(lvs)
    stats = {"iters": [0] * L, "smooth": [0] * L}
    ops = [None, (h.Y, h.cdims)] + [(lv.Y2, lv.cdims2) for lv in lvs]

    def A(l):
        Y, cd = ops[l]
        return lambda v: coarse.coarse_apply(Y, v[None], cd)[0]

    def cycle(l, r):  # K-cycle of level l >= 1: solve level l + 1, prolong, post-smooth on level l
        lv = lvs[l - 1]
        d, m = ops[l][0].shape[0], ops[l][0].shape[-1]
        r2 = restrict(lv.P, r.reshape(1, d, m), ops[l][1], lv.block2, lv.k)[0]
        if l + 1 == L - 1:
            e2, it, _ = krylov.gmres(A(l + 1), r2, None, restart=coarse_restart, max_iter=coarse_max, tol=coarse_tol)
        else:
            e2, it, _ = krylov.fgcr(A(l + 1), lambda q: cycle(l + 1, q), r2, None, tol=coarse_tol,
                                    restart=coarse_restart, max_iter=coarse_max)
        stats["iters"][l + 1] += it
        e = prolong(lv.P, e2[None], ops[l][1], lv.block2, lv.k)[0].reshape(r.shape)
        e, its, _ = krylov.gmres(A(l), r, e, restart=n_post, max_iter=n_post, tol=0.0)
        stats["smooth"][l] += its
        return e

    def k0(r):  # K-cycle of the fine level
        rc = mg.restrict(h, r[None])[0]
        if L == 2:
            ec, it, _ = krylov.gmres(A(1), rc, None, restart=coarse_restart, max_iter=coarse_max, tol=coarse_tol)
        else:
            ec, it, _ = krylov.fgcr(A(1), lambda q: cycle(1, q), rc, None, tol=coarse_tol, restart=coarse_restart,
                                    max_iter=coarse_max)
        stats["iters"][1] += it
        e = mg.prolong(h, ec[None])[0]
        e, its, _ = krylov.gmres(h.lat.D, r, e, restart=n_post, max_iter=n_post, tol=0.0)
        stats["smooth"][0] += its
        return e

    x, it, _ = krylov.fgcr(h.lat.D, k0, b, None, tol=tol, restart=restart, max_iter=max_iter)
    stats["iters"][0] = it
    stats["true_rel_res"] = float(np.linalg.norm((b - h.lat.D(x)).ravel()) / np.linalg.norm(b.ravel()))
    return x, stats


def solve3(h, lv, b, tol=1e-10, **kw):
    """Three levels: solve_levels with one further level.  Returns (x, stats) with stats["coarse"],
    stats["coarse2"] (iterations on levels 1 and 2) and stats["smoother1"] (post-smoothing on D_c)."""
    x, st = solve_levels(h, [lv], b, tol=tol, **kw)
    st.update(outer=st["iters"][0], coarse=st["iters"][1], coarse2=st["iters"][2], smoother=st["smooth"][0],
              smoother1=st["smooth"][1])
    return x, st
