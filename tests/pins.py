"""Independent pins for the oracle: closed forms, brute force and invariants.

Each helper raises AssertionError when the oracle disagrees with what the
paper or the mathematics fixes.  The closed forms below are retyped from the
spectral lemmas of Sec. 3.2 (Lemmas 3.1-3.4) and are independent of the
oracle, which takes its eigenvectors from LAPACK.
"""

import itertools
import math

import numpy as np

import oracle


# ---------------------------------------------------------------- lemmas ----
def lemma_eigenpairs(n, bc):
    """Closed-form (unnormalised) eigenpairs of L_n for one BC, Lemmas 3.1-3.4.

    Returns a list of (lambda, v) with v indexed j = 1..n.
    Periodic, odd n: the pairs run k = 1..(n-1)/2 and there is no eigenvalue 4
    (the printed lemma is garbled there; this reading matches the trace).
    The mixed DN vector is printed as sin(j theta - k pi) = (-1)^k sin(j theta).
    """
    j = np.arange(1, n + 1, dtype=np.float64)
    pairs = []
    if bc == "P":
        pairs.append((0.0, np.ones(n)))
        for k in range(1, (n - 1) // 2 + 1):
            th = 2.0 * k * math.pi / n
            lam = 2.0 - 2.0 * math.cos(th)
            pairs.append((lam, np.cos(j * th)))
            pairs.append((lam, np.sin(j * th)))
        if n % 2 == 0:
            pairs.append((4.0, (-1.0) ** (j + 1)))
    elif bc == "D":
        for k in range(1, n + 1):
            th = k * math.pi / (n + 1)
            pairs.append((2.0 - 2.0 * math.cos(th), np.sin(j * th)))
    elif bc == "N":
        for k in range(1, n + 1):
            th = (k - 1) * math.pi / n
            pairs.append((2.0 - 2.0 * math.cos(th), np.cos((j - 0.5) * th)))
    elif bc in ("DN", "ND"):
        for k in range(1, n + 1):
            th = (2 * k - 1) * math.pi / (2 * n + 1)
            lam = 2.0 - 2.0 * math.cos(th)
            if bc == "DN":
                v = np.sin(j * th - k * math.pi)
            else:
                v = np.cos(j * th - th / 2.0)
            pairs.append((lam, v))
    else:
        raise ValueError(bc)
    return pairs


def lemma_basis(n, bc):
    """Normalised closed-form eigenvectors (columns) and eigenvalues."""
    pairs = lemma_eigenpairs(n, bc)
    lam = np.array([p[0] for p in pairs])
    Q = np.stack([p[1] / np.linalg.norm(p[1]) for p in pairs], axis=1)
    return Q, lam


def pin_spectrum(n, bc, tol=1e-13):
    """Oracle eigenvalues and eigenspaces equal the lemma's."""
    V, lam, _ = oracle.pinv_init((n,), (bc,))
    V, lam = V[0], lam[0]
    Qc, lc = lemma_basis(n, bc)
    assert len(lc) == n, "lemma must give n eigenpairs"
    assert np.allclose(np.sort(lc), lam, atol=tol, rtol=0), (bc, n, np.sort(lc) - lam)
    L = oracle.laplacian_1d(n, bc)
    # the closed-form vectors are eigenvectors of the assembled eq. (3.1) matrix
    assert np.max(np.abs(L @ Qc - Qc * lc)) < tol * 10, (bc, n)
    # orthonormal oracle basis with the same spectral projectors (eigenspaces
    # of repeated eigenvalues admit any orthonormal basis)
    assert np.max(np.abs(V.T @ V - np.eye(n))) < tol * 10
    for value in np.unique(np.round(lc, 10)):
        sel_c = np.abs(lc - value) < 1e-9
        sel_o = np.abs(lam - value) < 1e-9
        assert sel_c.sum() == sel_o.sum(), (bc, n, value)
        Pc = Qc[:, sel_c] @ Qc[:, sel_c].T
        Po = V[:, sel_o] @ V[:, sel_o].T
        assert np.max(np.abs(Pc - Po)) < 1e-11, (bc, n, value)


# --------------------------------------------------------------- stencil ----
def ghost_rule_stencil(U, bcs):
    """Pure-Python 3/5/7-point stencil from ghost values, independent of the
    matrix assembly: each axis contributes 2u - u_lo - u_hi, where outside the
    grid a periodic axis wraps, a Dirichlet end has ghost 0 and a Neumann end
    has ghost equal to the boundary cell (Sec. 3.4.2 with homogeneous data)."""
    U = np.asarray(U, dtype=np.float64)
    W = np.zeros_like(U)
    ends = {"P": ("wrap", "wrap"), "D": ("zero", "zero"), "N": ("copy", "copy"),
            "DN": ("zero", "copy"), "ND": ("copy", "zero")}
    for idx in itertools.product(*[range(s) for s in U.shape]):
        total = 0.0
        for axis, bc in enumerate(bcs):
            n = U.shape[axis]
            lo_rule, hi_rule = ends[bc]
            c = U[idx]

            def nb(step, rule):
                pos = idx[axis] + step
                if 0 <= pos < n:
                    t = list(idx); t[axis] = pos
                    return U[tuple(t)]
                if rule == "wrap":
                    t = list(idx); t[axis] = pos % n
                    return U[tuple(t)]
                if rule == "zero":
                    return 0.0
                return c
            total += 2.0 * c - nb(-1, lo_rule) - nb(+1, hi_rule)
        W[idx] = total
    return W


# ------------------------------------------------------------------ pinv ----
def pin_pinv_modes(shape, bcs, picks=6, seed=0, tol=1e-12):
    """Manufactured eigenmodes: for H = v_i (x) v_j (x) v_k built from the
    closed-form lemma vectors, M(H) = H / (lambda_i + lambda_j + lambda_k),
    or 0 for the null mode."""
    rng = np.random.default_rng(seed)
    V, lam, G = oracle.pinv_init(shape, bcs)
    bases = [lemma_basis(n, bc) for n, bc in zip(shape, bcs)]
    for _ in range(picks):
        idx = [int(rng.integers(0, n)) for n in shape]
        H = np.ones([1] * len(shape))
        s = 0.0
        for axis, (Q, lc) in enumerate(bases):
            v = Q[:, idx[axis]]
            bshape = [1] * len(shape)
            bshape[axis] = shape[axis]
            H = H * v.reshape(bshape)
            s += lc[idx[axis]]
        Z = oracle.pinv_apply(H, V, G)
        expect = np.zeros_like(H) if abs(s) < 1e-13 else H / s
        assert np.max(np.abs(Z - expect)) < tol * max(1.0, np.max(np.abs(expect))), (shape, bcs, idx)


def pin_pinv_dense(shape, bcs, seed=0, tol=1e-12):
    """pinv_apply equals the SVD pseudoinverse of the assembled eq. (3.3)."""
    rng = np.random.default_rng(seed)
    R = rng.standard_normal(shape)
    V, lam, G = oracle.pinv_init(shape, bcs)
    Z = oracle.pinv_apply(R, V, G)
    L = oracle.kronecker_sum(shape, bcs)
    Zd = (np.linalg.pinv(L, rcond=1e-12, hermitian=True) @ R.ravel(order="F")).reshape(shape, order="F")
    assert np.max(np.abs(Z - Zd)) < tol * np.max(np.abs(Zd)), (shape, bcs)


# ----------------------------------------------------------------- solve ----
def pin_solve_brute(shape, bcs, seed=0, tol=1e-12):
    """PCG answer equals the brute-force minimum-norm solution."""
    rng = np.random.default_rng(seed)
    H = rng.standard_normal(shape)
    res = oracle.solve(H, bcs)
    ref = oracle.dense_pinv_solve(H, bcs)
    err = np.linalg.norm(res.u - ref) / np.linalg.norm(ref)
    assert err < tol, (shape, bcs, err)
    return res
