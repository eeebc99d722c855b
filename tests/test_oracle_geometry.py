"""Pins of oracle.geometry: brute-force coordinate loops and counting invariants."""
import itertools

import numpy as np
import pytest

from oracle import geometry as geo


def brute_index(x, y, z, t, dims):
    return x + dims[0] * (y + dims[1] * (z + dims[2] * t))


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 2, 6, 4), (3, 5, 2, 2)])
def test_neighbour_table_brute_force(dims):
    nb = geo.neighbor_table(dims)
    for t, z, y, x in itertools.product(*[range(L) for L in dims[::-1]]):
        s = brute_index(x, y, z, t, dims)
        c = [x, y, z, t]
        for d in range(8):
            mu, step = (d, 1) if d < 4 else (d - 4, -1)
            cc = list(c)
            cc[mu] = (cc[mu] + step) % dims[mu]
            assert nb[s, d] == brute_index(*cc, dims)


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 4, 2, 6)])
def test_every_site_is_neighbour_eight_times(dims):
    nb = geo.neighbor_table(dims)
    cnt = np.bincount(nb.ravel(), minlength=geo.volume(dims))
    assert np.all(cnt == 8)
    # forward and backward are inverse permutations per direction
    for mu in range(4):
        assert np.array_equal(nb[nb[:, mu], 4 + mu], np.arange(geo.volume(dims)))


def test_hop_sign_antiperiodic():
    dims = (2, 2, 2, 4)
    sg = geo.hop_sign(dims, -1)
    c = geo.coords(dims)
    for s in range(geo.volume(dims)):
        for d in range(8):
            expect = -1 if (d == 3 and c[s, 3] == 3) or (d == 7 and c[s, 3] == 0) else 1
            assert sg[s, d] == expect
    assert np.all(geo.hop_sign(dims, 1) == 1)


@pytest.mark.parametrize("dims,block", [((4, 4, 4, 4), (2, 2, 2, 2)), ((4, 6, 2, 4), (2, 3, 1, 4)),
                                        ((4, 4, 4, 4), (1, 1, 1, 1))])
def test_aggregates_brute_force(dims, block):
    agg, inb = geo.aggregate_map(dims, block)
    cd = geo.coarse_dims(dims, block)
    nd = int(np.prod(block))
    for t, z, y, x in itertools.product(*[range(L) for L in dims[::-1]]):
        s = brute_index(x, y, z, t, dims)
        c = [x, y, z, t]
        j = brute_index(*[c[m] // block[m] for m in range(4)], cd)
        i = brute_index(*[c[m] % block[m] for m in range(4)], block)
        assert agg[s] == j and inb[s] == i
    counts = np.bincount(agg)
    assert np.all(counts == nd)
    bs = geo.block_sites(dims, block)
    assert np.array_equal(agg[bs], np.repeat(np.arange(len(counts))[:, None], nd, axis=1))
    assert np.array_equal(inb[bs], np.repeat(np.arange(nd)[None, :], len(counts), axis=0))


def test_block_must_divide():
    with pytest.raises(ValueError):
        geo.aggregate_map((4, 4, 4, 4), (3, 2, 2, 2))


def test_coarse_neighbours_bijective():
    cnb = geo.coarse_neighbor_table((3, 2, 4, 2))
    for d in range(8):
        assert len(set(cnb[:, d].tolist())) == cnb.shape[0]
