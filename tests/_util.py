"""Helpers shared by the GPU parity tests (conversion only; no arithmetic of the method)."""
import numpy as np
import torch


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    """||a - b|| / ||b|| over all entries."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def projector_dist(Ua, Ub):
    """Relative Frobenius distance of the projectors U U^dag (column phases and rotations
    inside degenerate subspaces are free): ||Pa - Pb||_F / ||Pb||_F, ||Pb||_F = sqrt(k)."""
    Pb = Ub @ np.conj(Ub.T)
    return float(np.linalg.norm(Ua @ np.conj(Ua.T) - Pb) / np.linalg.norm(Pb))


def canonical_rows_to_oracle(P):
    """GPU canonical prolongator blocks [d][2][N][k] use the oracle's row order already."""
    return P


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
