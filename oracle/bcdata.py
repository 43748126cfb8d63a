"""Non-homogeneous boundary data and the electric field.

Test infrastructure (see the package docstring); never used by the product.

Sources in the paper:
  * Sec. 3.4.2 ("Dirichlet and Neumann BCs update"): a prescribed potential
    u_B at the beginning of a Dirichlet axis is the value of the node before
    the first unknown, so moving it to the right-hand side gives
    L_n u = h + i_1 u_B (and h + i_n u_E at the end).  A prescribed Neumann
    value e_B at the beginning defines the ghost node u_0 = u_1 + e_B, which
    gives the Neumann row of eq. (3.1) and the update h + i_1 e_B (and
    h + i_n e_E at the end, with ghost u_{n+1} = u_n + e_E).  Mixed axes
    (DN, ND) combine one of each.  In 2D and 3D a value is constant on a
    whole side or face, and every cell next to that face receives it.
  * Sec. 1: the electric field is recovered from the potential as minus its
    gradient.

Readings (the paper gives no formulas for these):
  * A Neumann value is the outward normal derivative of the potential at that
    face (ghost = boundary cell + value at both ends, as printed for the
    beginning and "similar" at the end).
  * The field is taken at the grid points by second-order central
    differences, epsilon_a = -(u_{+1} - u_{-1}) / 2 along axis a, with the
    neighbours outside the grid given by the same ghost values as the
    right-hand side update (periodic: wrap; Dirichlet: the prescribed
    potential; Neumann: the boundary cell plus the prescribed value).
    Unit grid spacing as eq. (3.1).

Face data `faces` is an array of shape (ndim, 2): faces[a][0] the value at
the beginning of axis a, faces[a][1] at its end; periodic axes must have 0.
Arrays are indexed in the paper's order U[i, j(, k)].
"""

import numpy as np

from .laplacian import bc_corners

# Kind of each end of an axis: 'P' periodic, 'D' Dirichlet node, 'N' ghost.
_ENDS = {"P": ("P", "P"), "D": ("D", "D"), "N": ("N", "N"), "DN": ("D", "N"), "ND": ("N", "D")}


def _check(shape, bcs, faces):
    faces = np.zeros((len(shape), 2)) if faces is None else np.asarray(faces, dtype=float)
    if faces.shape != (len(shape), 2):
        raise ValueError("faces must have shape (ndim, 2)")
    for a, bc in enumerate(bcs):
        bc_corners(bc)
        if bc == "P" and np.any(faces[a] != 0.0):
            raise ValueError("a periodic axis takes no boundary data")
    return faces


def assemble_rhs(eta, bcs, faces):
    """eta plus the Sec. 3.4.2 updates of every non-periodic face."""
    h = np.array(eta, dtype=np.float64)
    faces = _check(h.shape, bcs, faces)
    for a, bc in enumerate(bcs):
        if bc == "P":
            continue
        lo = [slice(None)] * h.ndim
        hi = [slice(None)] * h.ndim
        lo[a] = 0
        hi[a] = h.shape[a] - 1
        h[tuple(lo)] += faces[a][0]      # i_1 u_B or i_1 e_B
        h[tuple(hi)] += faces[a][1]      # i_n u_E or i_n e_E
    return h


def ghost_extend(u, bcs, faces):
    """u padded by one ghost layer on each side of every axis, filled by the
    ghost rule of each end (wrap, prescribed potential, or cell + value).
    Corner and edge ghosts are never used by the 7-point stencil or by
    central differences and are left at zero."""
    u = np.asarray(u, dtype=np.float64)
    faces = _check(u.shape, bcs, faces)
    ext = np.zeros(tuple(n + 2 for n in u.shape))
    inner = tuple(slice(1, n + 1) for n in u.shape)
    ext[inner] = u
    for a, bc in enumerate(bcs):
        n = u.shape[a]
        kinds = _ENDS[bc]
        for end, (gidx, cidx, widx) in enumerate(((0, 0, n - 1), (n + 1, n - 1, 0))):
            dst = list(inner)
            dst[a] = gidx
            src = [slice(None)] * u.ndim
            if kinds[end] == "P":
                src[a] = widx                      # wrap to the far end
                ext[tuple(dst)] = u[tuple(src)]
            elif kinds[end] == "D":
                ext[tuple(dst)] = faces[a][end]    # the prescribed node value
            else:
                src[a] = cidx                      # boundary cell + value
                ext[tuple(dst)] = u[tuple(src)] + faces[a][end]
    return ext


def minus_laplacian_with_ghosts(u, bcs, faces):
    """sum over axes of (2 u - u_{-1} - u_{+1}) with ghost values: the
    operator of the non-homogeneous problem applied to u."""
    ext = ghost_extend(u, bcs, faces)
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros(u.shape)
    inner = tuple(slice(1, n + 1) for n in u.shape)
    for a in range(u.ndim):
        lo = list(inner)
        hi = list(inner)
        lo[a] = slice(0, u.shape[a])
        hi[a] = slice(2, u.shape[a] + 2)
        out += 2.0 * u - ext[tuple(lo)] - ext[tuple(hi)]
    return out


def field(u, bcs, faces=None):
    """epsilon = -grad u by central differences with ghost values; returns an
    array of shape (ndim,) + u.shape, component a along axis a."""
    ext = ghost_extend(u, bcs, faces)
    u = np.asarray(u, dtype=np.float64)
    inner = tuple(slice(1, n + 1) for n in u.shape)
    eps = np.zeros((u.ndim,) + u.shape)
    for a in range(u.ndim):
        lo = list(inner)
        hi = list(inner)
        lo[a] = slice(0, u.shape[a])
        hi[a] = slice(2, u.shape[a] + 2)
        eps[a] = -(ext[tuple(hi)] - ext[tuple(lo)]) / 2.0
    return eps
