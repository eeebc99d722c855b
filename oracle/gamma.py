"""Gamma matrices in the chiral basis.

The paper needs a basis in which gamma_5 is diagonal, so that the chiral
projectors of Eq. (3) select spin components 1,2 (alpha = 0) and 3,4
(alpha = 1).  It never writes the matrices; the reading used here:

  gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]  (k = 1,2,3 = x,y,z)
  gamma_4 = [[0, 1], [1, 0]]                  (t)
  gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1)
"""
import numpy as np

SIGMA = [np.array([[0, 1], [1, 0]], dtype=np.complex128),
         np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
         np.array([[1, 0], [0, -1]], dtype=np.complex128)]


def _chiral(a):
    z = np.zeros((2, 2), dtype=np.complex128)
    return np.block([[z, a], [np.conj(a).T, z]])


GAMMA = [_chiral(-1j * SIGMA[0]), _chiral(-1j * SIGMA[1]), _chiral(-1j * SIGMA[2]),
         _chiral(np.eye(2, dtype=np.complex128))]
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)

# chirality projectors (1 +/- gamma_5)/2 -- Eq. (3) with the factor 1/2 made explicit
PROJ = [(ID4 + GAMMA5) / 2, (ID4 - GAMMA5) / 2]
# spins carried by each chirality, Eq. (3): alpha=0 <-> beta=1,2 ; alpha=1 <-> beta=3,4
CHIRAL_SPINS = [(0, 1), (2, 3)]
