"""Planted mistakes in the oracle must trip at least one pin.

Each case patches the oracle on the CPU (never the GPU path) with a plausible
error and checks that the corresponding pin raises."""

import importlib

import numpy as np
import pytest

import oracle
import oracle.laplacian as olap
import oracle.pinv as opinv
from pins import pin_pinv_dense, pin_pinv_modes, pin_solve_brute, pin_spectrum


def test_wrong_neumann_corner_is_caught(monkeypatch):
    monkeypatch.setitem(olap._CORNERS, "N", (2.0, 1.0, 0.0))
    with pytest.raises(AssertionError):
        pin_spectrum(6, "N")


def test_missing_periodic_wrap_is_caught(monkeypatch):
    monkeypatch.setitem(olap._CORNERS, "P", (2.0, 2.0, 0.0))
    with pytest.raises(AssertionError):
        pin_spectrum(6, "P")


def test_transposed_forward_transform_is_caught(monkeypatch):
    def bad_apply(R, V, G):
        F = np.asarray(R, dtype=np.float64)
        for axis, Q in enumerate(V):
            F = olap._mode_product(Q, F, axis)          # should be Q.T
        F = F * G
        for axis, Q in enumerate(V):
            F = olap._mode_product(Q, F, axis)
        return F
    monkeypatch.setattr(oracle, "pinv_apply", bad_apply)
    with pytest.raises(AssertionError):
        pin_pinv_modes((6, 5, 4), ("DN", "P", "N"))


def test_unthresholded_sum_is_caught(monkeypatch):
    monkeypatch.setattr(opinv, "ZERO_THRESHOLD", -1.0)   # divides by the zero sum
    with np.errstate(divide="ignore", invalid="ignore"):
        with pytest.raises(AssertionError):
            pin_pinv_dense((3, 4, 5), ("P", "N", "P"))


def test_wrong_residual_sign_is_caught(monkeypatch):
    real = olap.apply_minus_laplacian

    def flipped(U, bcs, dense=False):
        return -real(U, bcs, dense)
    opcg = importlib.import_module("oracle.pcg")
    monkeypatch.setattr(opcg, "apply_minus_laplacian", flipped)
    with pytest.raises((AssertionError, FloatingPointError)):
        with np.errstate(all="raise"):
            pin_solve_brute((3, 4, 5), ("D", "N", "P"))


def test_dropped_axis_is_caught(monkeypatch):
    real = olap.apply_minus_laplacian

    def two_axes(U, bcs, dense=False):
        W = real(U, bcs, dense)
        n = U.shape[2]
        return W - olap._mode_product(olap.laplacian_1d(n, bcs[2]), U, 2)
    opcg = importlib.import_module("oracle.pcg")
    monkeypatch.setattr(opcg, "apply_minus_laplacian", two_axes)
    with pytest.raises(AssertionError):
        pin_solve_brute((3, 4, 5), ("D", "D", "D"))
