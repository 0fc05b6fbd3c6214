"""Pins of the oracle's 1D FR basis against closed forms.

Gauss-Legendre points (the solution points of the FR scheme of Huynh 2007,
which the paper's Section 1 names for its solver) and the g_DG (right Radau)
correction function g_R = (P_p + P_{p+1})/2, g_L(x) = g_R(-x).
"""
import math

import numpy as np
import pytest

from oracle.oracle import basis


def test_gauss_legendre_closed_forms():
    b = basis(1)
    assert np.allclose(b["xi"], [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-15)
    assert np.allclose(b["w"], [1.0, 1.0], atol=1e-15)
    b = basis(2)
    assert np.allclose(b["xi"], [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(b["w"], [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


@pytest.mark.parametrize("order", range(1, 7))
def test_quadrature_exactness(order):
    b = basis(order)
    assert abs(b["w"].sum() - 2.0) < 1e-14
    for k in range(2 * order + 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(b["w"], b["xi"] ** k) - exact) < 1e-14


@pytest.mark.parametrize("order", range(1, 7))
def test_derivative_and_interpolation_exact_on_monomials(order):
    b = basis(order)
    x = b["xi"]
    for k in range(order + 1):
        f = x ** k
        df = k * x ** (k - 1) if k else np.zeros_like(x)
        assert np.allclose(b["D"] @ f, df, atol=1e-12)
        assert abs(b["lp"] @ f - 1.0) < 1e-13
        assert abs(b["lm"] @ f - (-1.0) ** k) < 1e-13


def test_radau_derivative_closed_forms():
    # p = 1: g_R = (x + (3x^2 - 1)/2)/2  ->  g_R' = (1 + 3x)/2
    b = basis(1)
    assert np.allclose(b["gRd"], (1 + 3 * b["xi"]) / 2, atol=1e-15)
    # p = 2: g_R = ((3x^2-1)/2 + (5x^3-3x)/2)/2  ->  g_R' = (3x + (15x^2 - 3)/2)/2
    b = basis(2)
    x = b["xi"]
    assert np.allclose(b["gRd"], (3 * x + (15 * x ** 2 - 3) / 2) / 2, atol=1e-14)


@pytest.mark.parametrize("order", range(1, 7))
def test_radau_boundary_values_via_quadrature(order):
    # int_{-1}^{1} g_R' = g_R(1) - g_R(-1) = 1 and int g_L' = -1 (exact: degree p)
    b = basis(order)
    assert abs(b["w"] @ b["gRd"] - 1.0) < 1e-13
    assert abs(b["w"] @ b["gLd"] + 1.0) < 1e-13
    # symmetry g_L(x) = g_R(-x)  ->  g_L'(x_i) = -g_R'(-x_i) = -g_R'(x_{n-1-i})
    assert np.allclose(b["gLd"], -b["gRd"][::-1], atol=1e-13)
