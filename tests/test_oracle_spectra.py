"""Oracle pins: 1D operators of eq. (3.1) and their spectra (Lemmas 3.1-3.4)."""

import math

import numpy as np
import pytest

import oracle
from pins import lemma_eigenpairs, pin_spectrum

SIZES = [3, 4, 5, 7, 8, 16, 33, 64]


@pytest.mark.parametrize("bc", oracle.BCS)
@pytest.mark.parametrize("n", SIZES)
def test_spectrum_matches_lemmas(n, bc):
    pin_spectrum(n, bc)


@pytest.mark.parametrize("bc", oracle.BCS)
def test_spectrum_large(bc):
    pin_spectrum(257, bc, tol=1e-12)


@pytest.mark.parametrize("bc,trace", [("P", lambda n: 2 * n), ("D", lambda n: 2 * n),
                                      ("N", lambda n: 2 * n - 2), ("DN", lambda n: 2 * n - 1),
                                      ("ND", lambda n: 2 * n - 1)])
@pytest.mark.parametrize("n", [3, 6, 11])
def test_trace_identity(n, bc, trace):
    # sum of eigenvalues = alpha + beta + 2(n-2), read off eq. (3.1)
    _, lam, _ = oracle.pinv_init((n,), (bc,))
    assert abs(lam[0].sum() - trace(n)) < 1e-12


def test_tiny_worked_spectra():
    # exact spectra of the smallest operators, derived by hand from eq. (3.1)
    s2 = math.sqrt(2.0)
    cases = {
        ("D", 3): [2 - s2, 2.0, 2 + s2],
        ("N", 3): [0.0, 1.0, 3.0],
        ("P", 3): [0.0, 3.0, 3.0],
        ("P", 4): [0.0, 2.0, 2.0, 4.0],
    }
    for (bc, n), expect in cases.items():
        _, lam, _ = oracle.pinv_init((n,), (bc,))
        assert np.allclose(lam[0], expect, atol=1e-14), (bc, n)
    # L_DN(3) = [[2,-1,0],[-1,2,-1],[0,-1,1]]: characteristic polynomial
    # -x^3 + 5x^2 - 6x + 1, roots 4 sin^2((2k-1) pi / 14)
    _, lam, _ = oracle.pinv_init((3,), ("DN",))
    roots = np.sort(np.roots([1.0, -5.0, 6.0, -1.0]).real)
    assert np.allclose(lam[0], roots, atol=1e-14)
    assert np.allclose(roots, [4 * math.sin((2 * k - 1) * math.pi / 14) ** 2 for k in (1, 2, 3)])


@pytest.mark.parametrize("bc", oracle.BCS)
def test_assembled_matrix_structure(bc):
    n = 6
    L = oracle.laplacian_1d(n, bc)
    alpha, beta, gamma = oracle.bc_corners(bc)
    assert np.array_equal(L, L.T)
    assert L[0, 0] == alpha and L[-1, -1] == beta and L[0, -1] == gamma
    assert np.all(np.diag(L)[1:-1] == 2.0)
    assert np.all(np.diag(L, 1) == -1.0)
    with pytest.raises(ValueError):
        oracle.laplacian_1d(2, bc)


def test_singular_sets():
    # Lemmas 3.1-3.4: only L_P and L_N have a zero eigenvalue; Sec. 3.3: the
    # Kronecker sum is singular iff every factor is
    for bc in oracle.BCS:
        _, lam, _ = oracle.pinv_init((5,), (bc,))
        assert (abs(lam[0][0]) < 1e-14) == (bc in ("P", "N"))
    assert oracle.is_singular(("P", "N", "P"))
    assert not oracle.is_singular(("P", "N", "D"))
    assert oracle.is_singular(("N", "N"))


@pytest.mark.parametrize("bcs", [("P", "D", "N"), ("N", "N", "P"), ("DN", "ND", "P")])
def test_kronecker_sum_spectrum(bcs):
    # sigma(L_3D) = {lambda_i + lambda_j + lambda_k}, Sec. 3.3
    shape = (3, 4, 5)
    L = oracle.kronecker_sum(shape, bcs)
    ev = np.linalg.eigvalsh(L)
    sums = []
    for n, bc in zip(shape, bcs):
        sums.append(np.array([p[0] for p in lemma_eigenpairs(n, bc)]))
    allsums = (sums[0][:, None, None] + sums[1][None, :, None] + sums[2][None, None, :]).ravel()
    assert np.allclose(np.sort(ev), np.sort(allsums), atol=1e-12)
