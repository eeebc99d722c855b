"""Philox4x32-10 counter-based RNG and Box-Muller, for the random initial guesses phi_i.

The paper draws the starting vectors of the test-vector smoother at random
(Section 2.1, Eq. (2)) without fixing a distribution or generator.  Reading:
complex Gaussian entries (Re, Im ~ N(0,1)) from Philox4x32-10 as published by
Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as easy as 1, 2, 3",
SC'11): 10 rounds of the 4x32 Philox S-box with multipliers 0xD2511F53 and
0xCD9E8D57 and Weyl key increments 0x9E3779B9 and 0xBB67AE85.

Stream layout (shared definition, implemented independently on each side):
  key     = (seed mod 2^32, seed div 2^32)
  counter = (site, g, v, 0) for g = 0..5, v = global test-vector index
  u_i     = (x_i + 1/2) * 2^-32 in (0, 1)
  (u0,u1) -> z0 + i z1 and (u2,u3) -> z2 + i z3 by Box-Muller
            (r = sqrt(-2 ln u_a), theta = 2 pi u_b, z = r cos theta + i r sin theta)
  these are spin-colour components 2g and 2g+1 (component = 3*spin + colour).
"""
import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: uint array [..., 4]; key: (k0, k1) ints.  Returns uint32 array [..., 4]."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return np.stack(c, axis=-1).astype(np.uint32)


def gaussian_test_vector(seed, v, V):
    """phi_v: [V][4][3] complex128 for global test-vector index v."""
    site = np.arange(V, dtype=np.uint64)
    out = np.empty((V, 12), dtype=np.complex128)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    for g in range(6):
        ctr = np.zeros((V, 4), dtype=np.uint64)
        ctr[:, 0] = site
        ctr[:, 1] = g
        ctr[:, 2] = v
        x = philox4x32_10(ctr, key).astype(np.float64)
        u = (x + 0.5) * 2.0 ** -32
        r0 = np.sqrt(-2.0 * np.log(u[:, 0]))
        r1 = np.sqrt(-2.0 * np.log(u[:, 2]))
        out[:, 2 * g] = r0 * np.cos(2 * np.pi * u[:, 1]) + 1j * r0 * np.sin(2 * np.pi * u[:, 1])
        out[:, 2 * g + 1] = r1 * np.cos(2 * np.pi * u[:, 3]) + 1j * r1 * np.sin(2 * np.pi * u[:, 3])
    return out.reshape(V, 4, 3)
