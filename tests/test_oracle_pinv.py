"""Oracle pins: pseudoinverse preconditioner, Algs. 4-7 and eqs. (4.5)-(4.7)."""

import itertools

import numpy as np
import pytest

import oracle
from pins import pin_pinv_dense, pin_pinv_modes

ALL3 = list(itertools.product(oracle.BCS, repeat=3))
ALL2 = list(itertools.product(oracle.BCS, repeat=2))


@pytest.mark.parametrize("bcs", ALL3)
def test_pinv_equals_dense_pseudoinverse_3d(bcs):
    pin_pinv_dense((3, 4, 5), bcs)


@pytest.mark.parametrize("bcs", ALL2)
def test_pinv_equals_dense_pseudoinverse_2d(bcs):
    pin_pinv_dense((6, 5), bcs)


@pytest.mark.parametrize("bcs", [("P", "P", "DN"), ("N", "N", "N"), ("D", "ND", "P"), ("P", "P", "D")])
@pytest.mark.parametrize("shape", [(8, 6, 5), (7, 9, 4)])
def test_manufactured_eigenmodes(shape, bcs):
    pin_pinv_modes(shape, bcs)


@pytest.mark.parametrize("bcs", [("D", "D"), ("P", "N"), ("N", "DN")])
def test_manufactured_eigenmodes_2d(bcs):
    pin_pinv_modes((9, 6), bcs)


def test_threshold_zeroes_exactly_the_null_mode():
    for bcs in ALL3:
        _, _, G = oracle.pinv_init((4, 3, 5), bcs)
        zeros = int(np.sum(G == 0.0))
        assert zeros == (1 if oracle.is_singular(bcs) else 0), bcs
        assert np.all(G >= 0.0)


def test_null_mode_maps_to_zero():
    shape = (5, 6, 4)
    V, lam, G = oracle.pinv_init(shape, ("P", "N", "P"))
    Z = oracle.pinv_apply(np.full(shape, 3.0), V, G)
    assert np.max(np.abs(Z)) < 1e-13


def test_pinv_is_inverse_on_range():
    # L M L = L (Moore-Penrose property) checked through the stencil
    rng = np.random.default_rng(7)
    shape = (6, 5, 7)
    for bcs in [("P", "P", "DN"), ("N", "N", "N"), ("D", "D", "D")]:
        V, lam, G = oracle.pinv_init(shape, bcs)
        x = rng.standard_normal(shape)
        Lx = oracle.apply_minus_laplacian(x, bcs)
        LMLx = oracle.apply_minus_laplacian(oracle.pinv_apply(Lx, V, G), bcs)
        assert np.max(np.abs(LMLx - Lx)) < 1e-11 * np.max(np.abs(Lx))
