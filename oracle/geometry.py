"""Lattice geometry: sites, neighbours, boundary signs, aggregates.

Site index is lexicographic, x fastest: s = x + Lx*(y + Ly*(z + Lz*t)).
Direction d = 0..3 is the forward hop +mu (mu = d), d = 4..7 the backward hop
-mu (mu = d-4).  The aggregates Lambda_j (Section 2.1 and Section 3: a uniform
domain decomposition into d blocks of n_d sites) are hyper-rectangular blocks
of extent b_mu; block j is the lexicographic index of (x_mu div b_mu) on the
coarse lattice of extent L_mu/b_mu, and a site's index inside its block is the
lexicographic index of (x_mu mod b_mu).
"""
import numpy as np


def volume(dims):
    return int(np.prod(dims))


def coords(dims):
    """[V][4] integer coordinates (x, y, z, t) of every site."""
    V = volume(dims)
    s = np.arange(V)
    out = np.empty((V, 4), dtype=np.int64)
    for mu in range(4):
        out[:, mu] = s % dims[mu]
        s = s // dims[mu]
    return out


def lex(c, dims):
    """Lexicographic index of coordinate array c[..., 4]."""
    c = np.asarray(c)
    return c[..., 0] + dims[0] * (c[..., 1] + dims[1] * (c[..., 2] + dims[2] * c[..., 3]))


def neighbor_table(dims):
    """[V][8] int32: site index of x+mu (d<4) and x-mu (d>=4), periodic wrap."""
    c = coords(dims)
    V = volume(dims)
    nb = np.empty((V, 8), dtype=np.int32)
    for d in range(8):
        mu, step = (d, 1) if d < 4 else (d - 4, -1)
        cc = c.copy()
        cc[:, mu] = (cc[:, mu] + step) % dims[mu]
        nb[:, d] = lex(cc, dims)
    return nb


def hop_sign(dims, bc_t):
    """[V][8] +/-1: the boundary factor of each hop.

    Periodic in x, y, z.  In t the factor bc_t (= -1 antiperiodic) multiplies every
    hop that crosses the t = Lt-1 <-> 0 boundary: forward from t = Lt-1 and
    backward from t = 0.
    """
    c = coords(dims)
    sg = np.ones((volume(dims), 8), dtype=np.int32)
    if bc_t == -1:
        sg[c[:, 3] == dims[3] - 1, 3] = -1
        sg[c[:, 3] == 0, 7] = -1
    return sg


def check_block(dims, block):
    for mu in range(4):
        if block[mu] < 1 or dims[mu] % block[mu] != 0:
            raise ValueError(f"block {block} does not divide lattice {dims}")


def coarse_dims(dims, block):
    check_block(dims, block)
    return tuple(dims[mu] // block[mu] for mu in range(4))


def aggregate_map(dims, block):
    """(agg[V], inblock[V]): aggregate j of each site and its index inside Lambda_j."""
    cd = coarse_dims(dims, block)
    c = coords(dims)
    blk = np.asarray(block)
    agg = lex(c // blk, cd).astype(np.int32)
    inb = lex(c % blk, block).astype(np.int32)
    return agg, inb


def block_sites(dims, block):
    """[d][n_d] fine site of (aggregate j, in-block index i)."""
    agg, inb = aggregate_map(dims, block)
    d = volume(coarse_dims(dims, block))
    nd = volume(block)
    out = np.empty((d, nd), dtype=np.int32)
    out[agg, inb] = np.arange(volume(dims), dtype=np.int32)
    return out


def coarse_neighbor_table(cdims):
    """Neighbour table of the coarse lattice (same direction convention)."""
    return neighbor_table(cdims)
