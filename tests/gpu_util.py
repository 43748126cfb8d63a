"""Helpers shared by the GPU tests: device transfers and oracle calls in the
paper's index order (oracle arrays are indexed [i, j, k]; device arrays are
(nz, ny, nx) with x fastest, so one is the other's transpose)."""

import numpy as np

import oracle


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def oracle_solve(eta, bcs):
    """Converged minimum-norm solution for a device-layout array."""
    return oracle.solve(eta.T, bcs).u.T


def oracle_laplacian(p, bcs):
    return oracle.apply_minus_laplacian(p.T, bcs).T


def oracle_pinv(r, bcs):
    V, lam, G = oracle.pinv_init(r.T.shape, bcs)
    return oracle.pinv_apply(r.T, V, G).T


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def grid_dims(shape):
    """(nx, ny, nz) of a device-layout shape (nz, ny, nx) or (ny, nx)."""
    if len(shape) == 3:
        return shape[2], shape[1], shape[0]
    return shape[1], shape[0], 1
