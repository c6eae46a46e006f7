"""Pins of the oracle's 1D building blocks (paper Sec. 2) against closed forms
and exactness properties that do not depend on the oracle's own formulas."""

import math

import numpy as np
import pytest

import oracle


CLOSED_FORM = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("p", sorted(CLOSED_FORM))
def test_gll_closed_form(p):
    xi, w = oracle.gll(p)
    x_ref, w_ref = CLOSED_FORM[p]
    assert np.allclose(xi, x_ref, atol=1e-15, rtol=0)
    assert np.allclose(w, w_ref, atol=1e-15, rtol=0)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7, 8, 12, 16, 24, 32])
def test_gll_quadrature_exactness(p):
    xi, w = oracle.gll(p)
    assert abs(w.sum() - 2.0) < 1e-13
    assert np.all(np.diff(xi) > 0) and xi[0] == -1.0 and xi[-1] == 1.0
    assert np.allclose(xi, -xi[::-1], atol=1e-15)
    for k in range(2 * p):           # exact up to degree 2p - 1
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13, k
    # degree 2p is not integrated exactly (GLL is not Gauss)
    if p <= 8:
        assert abs(np.dot(w, xi ** (2 * p)) - 2.0 / (2 * p + 1)) > 1e-10


@pytest.mark.parametrize("p", [1, 2, 4, 7, 8, 16, 32])
def test_derivative_exact_on_polynomials(p):
    xi, _ = oracle.gll(p)
    D = oracle.diff_matrix(xi)
    for k in range(p + 1):
        dk = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        assert np.allclose(D @ xi ** k, dk, atol=1e-10 * max(1, k * k)), k
    # rows sum to zero (constants have zero derivative)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-11)


@pytest.mark.parametrize("pc,pf", [(1, 2), (2, 4), (4, 7), (4, 8), (8, 16), (16, 32)])
def test_interpolation_exact(pc, pf):
    xc, _ = oracle.gll(pc)
    xf, _ = oracle.gll(pf)
    J = oracle.interp_matrix(xc, xf)
    for k in range(pc + 1):
        assert np.allclose(J @ xc ** k, xf ** k, atol=1e-12), k
    assert np.allclose(J.sum(axis=1), 1.0, atol=1e-13)


def test_product_formula_matches_vandermonde_route():
    xi, _ = oracle.gll(6)
    x = np.linspace(-1, 1, 11)
    phi, dphi = oracle.lagrange_eval(xi, x)
    assert np.allclose(phi, oracle.interp_matrix(xi, x), atol=1e-12)
    _, dphi_nodes = oracle.lagrange_eval(xi, xi)
    assert np.allclose(dphi_nodes, oracle.diff_matrix(xi), atol=1e-11)


# ---- Gauss-Legendre rule (Sec. 2; the GL rows of Table 1) -----------------
GL_CLOSED_FORM = {
    0: ([0.0], [2.0]),
    1: ([-1 / math.sqrt(3), 1 / math.sqrt(3)], [1.0, 1.0]),
    2: ([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)], [5 / 9, 8 / 9, 5 / 9]),
    3: ([-math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5)), -math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)),
         math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)), math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))],
        [(18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36,
         (18 - math.sqrt(30)) / 36]),
}


@pytest.mark.parametrize("p", sorted(GL_CLOSED_FORM))
def test_gl_closed_form(p):
    xi, w = oracle.gl(p)
    x_ref, w_ref = GL_CLOSED_FORM[p]
    assert np.allclose(xi, x_ref, atol=1e-15, rtol=0)
    assert np.allclose(w, w_ref, atol=1e-14, rtol=0)


@pytest.mark.parametrize("p", [1, 2, 4, 7, 8, 16, 32])
def test_gl_quadrature_exactness(p):
    xi, w = oracle.gl(p)
    assert np.all(np.diff(xi) > 0) and -1.0 < xi[0] and xi[-1] < 1.0
    assert np.allclose(xi, -xi[::-1], atol=1e-15)
    for k in range(2 * p + 2):       # exact up to degree 2p + 1 (Gauss)
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13, k
    if p <= 8:                       # not beyond
        assert abs(np.dot(w, xi ** (2 * p + 2)) - 2.0 / (2 * p + 3)) > 1e-10


@pytest.mark.parametrize("basis,p", [("gl", 1), ("gl", 2), ("gl", 5), ("gl", 8), ("gll", 4)])
def test_end_values_exact_on_polynomials(basis, p):
    # traces phi_j(+-1) and end derivatives phi_j'(+-1) reproduce every
    # polynomial of degree <= p (and agree with the product formula)
    xi, _ = oracle.rule(basis, p)
    pm, pp, dm, dp = oracle.end_values(xi)
    for k in range(p + 1):
        f = xi ** k
        assert abs(pm @ f - (-1.0) ** k) < 1e-11 and abs(pp @ f - 1.0) < 1e-11, k
        dk = k * (-1.0) ** (k - 1) if k > 0 else 0.0
        assert abs(dm @ f - dk) < 1e-9 * max(1, k * k) and abs(dp @ f - k) < 1e-9 * max(1, k * k), k
    phi, dphi = oracle.lagrange_eval(xi, [-1.0, 1.0])
    assert np.allclose(phi, [pm, pp], atol=1e-12) and np.allclose(dphi, [dm, dp], atol=1e-9)
