"""Galerkin coarse operator D_c = R D P (Eq. (5)) as a nine-block coarse stencil.

For aggregate j the coarse operator couples j to itself and to its eight
neighbours on the coarse lattice:

  (D_c v)(j) = Y_0(j) v(j) + sum_{d=0..7} Y_{1+d}(j) v(j + dir_d)

Y_{1+d}(j) collects the fine hops in direction d that leave Lambda_j through its
face (x_mu mod b_mu = b_mu - 1 for +mu, = 0 for -mu); every other hop, and the
diagonal term, goes into Y_0(j).  The eight directional blocks are kept separate
even when a coarse extent is 2 or 1 (then several directions reach the same
aggregate) and are summed when the operator is applied.  Each block is (2k) x (2k)
in the coarse dof order (alpha, i).  The boundary sign of the fine hops is
included, so the coarse operator needs no separate boundary condition.
"""
import numpy as np

from .gamma import GAMMA, ID4
from .geometry import aggregate_map, coords, neighbor_table, hop_sign, coarse_dims, volume
from .wilson import hop_weights, diag_term


def fine_rows(U, dims, block):
    """[V][12][2k]: the rows of P at every fine site (zero outside the site's chirality)."""
    agg, inb = aggregate_map(dims, block)
    k = U.shape[-1]
    V = volume(dims)
    Pf = np.zeros((V, 12, 2 * k), dtype=np.complex128)
    for a in range(2):
        for sp in range(2):
            for c in range(3):
                Pf[:, 3 * (2 * a + sp) + c, a * k:(a + 1) * k] = U[agg, a, 6 * inb + 3 * sp + c, :]
    return Pf


def build_coarse(G, U, mass, xi, bc_t, dims, block, chunk=4096, T=None):
    """Y [d][9][2k][2k] from gauge links G [4][V][3][3] and prolongator blocks U [d][2][N][k].

    T: optional clover term [V][12][12] (clover.py), added to the diagonal term (it is site
    local, so it only enters Y_0)."""
    agg, _ = aggregate_map(dims, block)
    cd = coarse_dims(dims, block)
    d = volume(cd)
    k = U.shape[-1]
    Pf = fine_rows(U, dims, block)
    nb = neighbor_table(dims)
    sg = hop_sign(dims, bc_t)
    c = hop_weights(xi)
    X = coords(dims)
    Y = np.zeros((d, 9, 2 * k, 2 * k), dtype=np.complex128)
    V = volume(dims)
    # diagonal term
    diag = diag_term(mass, xi) * np.einsum("xsi,xsl->xil", np.conj(Pf), Pf)
    if T is not None:
        diag = diag + np.einsum("xsi,xst,xtl->xil", np.conj(Pf), T, Pf)
    np.add.at(Y, (agg, 0), diag)
    for dd in range(8):
        mu = dd % 4
        fwd = dd < 4
        proj = (ID4 - GAMMA[mu]) if fwd else (ID4 + GAMMA[mu])
        for s0 in range(0, V, chunk):
            xs = np.arange(s0, min(V, s0 + chunk))
            ys = nb[xs, dd]
            link = G[mu, xs] if fwd else np.conj(np.swapaxes(G[mu, ys], -1, -2))
            # H = -1/2 c_mu s (proj x link), a 12x12 matrix per site
            H = np.einsum("st,xab->xsatb", proj, link).reshape(len(xs), 12, 12)
            H = H * (-0.5 * c[mu] * sg[xs, dd])[:, None, None]
            contrib = np.einsum("xsi,xst,xtl->xil", np.conj(Pf[xs]), H, Pf[ys])
            face = (X[xs, mu] % block[mu] == block[mu] - 1) if fwd else (X[xs, mu] % block[mu] == 0)
            slot = np.where(face, 1 + dd, 0)
            np.add.at(Y, (agg[xs], slot), contrib)
    return Y


def coarse_apply(Y, v, cdims):
    """y = D_c v for v [nrhs][d][2][k] (or [nrhs][d][2k])."""
    shp = v.shape
    nrhs, d = shp[0], shp[1]
    vv = v.reshape(nrhs, d, -1)
    cnb = neighbor_table(cdims)
    y = np.einsum("jab,rjb->rja", Y[:, 0], vv)
    for dd in range(8):
        y += np.einsum("jab,rjb->rja", Y[:, 1 + dd], vv[:, cnb[:, dd]])
    return y.reshape(shp)


def dense_coarse(Y, cdims):
    """Dense matrix of the coarse stencil (small lattices)."""
    d, _, m, _ = Y.shape
    cnb = neighbor_table(cdims)
    Dc = np.zeros((d * m, d * m), dtype=np.complex128)
    for j in range(d):
        Dc[j * m:(j + 1) * m, j * m:(j + 1) * m] += Y[j, 0]
        for dd in range(8):
            t = cnb[j, dd]
            Dc[j * m:(j + 1) * m, t * m:(t + 1) * m] += Y[j, 1 + dd]
    return Dc
