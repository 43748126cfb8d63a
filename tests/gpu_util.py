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
    """The minimum-norm solution L^+ eta for a device-layout array (the
    oracle's eigen-expansion; zero-mean for a singular set)."""
    return oracle.min_norm_solution(eta.T, bcs)[0].T


def oracle_laplacian(p, bcs):
    return oracle.apply_minus_laplacian(p.T, bcs).T


def oracle_pinv(r, bcs):
    V, lam, G = oracle.pinv_init(r.T.shape, bcs)
    return oracle.pinv_apply(r.T, V, G).T


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_max(a, b):
    """max |a - b| / max |b|: the element-wise counterpart of rel."""
    nb = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (nb if nb > 0 else 1.0)) if a.size else 0.0


def assert_close(u, ref, tol, what=""):
    """The solution parity bar: relative error at most tol both norm-wise,
    ||u - ref||_2 <= tol ||ref||_2, and element by element,
    max|u - ref| <= tol max|ref|."""
    e2, einf = rel(u, ref), rel_max(u, ref)
    assert e2 <= tol and einf <= tol, (what, e2, einf, tol)
    return e2, einf


def grid_dims(shape):
    """(nx, ny, nz) of a device-layout shape (nz, ny, nx) or (ny, nx)."""
    if len(shape) == 3:
        return shape[2], shape[1], shape[0]
    return shape[1], shape[0], 1
