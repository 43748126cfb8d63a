"""Seeded synthetic inputs shared by the GPU tests, the benchmark and the oracle.

This module only draws random numbers and lays them out; it holds none of the
solver's arithmetic.  Arrays come back in the device layout: C-order
(nz, ny, nx) for 3D and (ny, nx) for 2D, x fastest.  In the paper's index
order U[i, j, k] (Sec. 2.1) the same array is `a.T`.

Workloads (the paper's own right-hand sides, fabricated by Ferrodo2, are not
available, so these stand in for them):
  * gaussian_blobs_2d: sum of Gaussian blobs, sigma in cells, centres uniform
    in the grid, amplitudes uniform in [-1, 1];
  * charge_field: unit point charges of random sign at uniformly drawn cells
    (with replacement; coincident charges add), plus N(0, noise_std) noise,
    minus its mean (the workload is defined as zero-mean);
  * serving_requests: a seeded stream of solve requests of mixed grid size,
    boundary conditions and tolerance.
"""

import numpy as np

BC_CODES = {"P": 0, "D": 1, "N": 2, "DN": 3, "ND": 4}


def gaussian_blobs_2d(nx=64, ny=64, nblobs=16, sigma=2.0, seed=1):
    """(ny, nx) field: sum_b a_b exp(-((i-cx_b)^2 + (j-cy_b)^2) / (2 sigma^2)).

    Draw order: centres (nblobs x 2, uniform in [0, nx) x [0, ny)), then
    amplitudes (uniform in [-1, 1]).  Cell (i, j) sits at coordinates (i, j).
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(nblobs, 2)) * np.array([nx, ny])
    amps = rng.uniform(-1.0, 1.0, size=nblobs)
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    out = np.zeros((ny, nx))
    for (cx, cy), a in zip(centres, amps):
        out += a * np.exp(-((i - cx) ** 2 + (j - cy) ** 2) / (2.0 * sigma * sigma))
    return out


def charge_field(shape, ncharges=10_000, noise_std=1e-3, seed=2, zero_mean=True):
    """Random-sign unit charges plus Gaussian noise on a grid of `shape`.

    `shape` is (nz, ny, nx) or (ny, nx).  Draw order: cells
    (integers in [0, N), with replacement), signs (+-1), noise (N values).
    """
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    cells = rng.integers(0, n, size=ncharges)
    signs = rng.choice(np.array([-1.0, 1.0]), size=ncharges)
    flat = np.zeros(n)
    np.add.at(flat, cells, signs)
    flat += rng.normal(0.0, noise_std, size=n)
    if zero_mean:
        flat -= flat.mean()
    return flat.reshape(shape)


SERVING_GRIDS = ((64, 64, 64), (96, 96, 48), (128, 128, 128), (192, 192, 96), (256, 256, 256))
SERVING_BCS = ("P", "D", "N", "DN")
SERVING_TOLS = (1e-8, 1e-10)


def serving_requests(count=2000, seed=4, grids=SERVING_GRIDS):
    """Seeded request stream.  Each request: grid (nx, ny, nz), one BC per
    axis, tol, a field seed, and an exponential inter-arrival gap of unit mean
    (scale it by 1/rate).  Draw order per request: gap, grid, 3 BCs, tol."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        gap = float(rng.exponential(1.0))
        grid = grids[int(rng.integers(0, len(grids)))]
        bcs = tuple(SERVING_BCS[int(rng.integers(0, len(SERVING_BCS)))] for _ in range(3))
        tol = SERVING_TOLS[int(rng.integers(0, len(SERVING_TOLS)))]
        reqs.append({"id": r, "gap": gap, "grid": grid, "bcs": bcs, "tol": tol,
                     "field_seed": 100_000 + r})
    return reqs
