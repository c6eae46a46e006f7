"""1D nodal building blocks (paper Sec. 2, eq. (u_h)): Gauss-Lobatto-Legendre
(GLL) and Gauss-Legendre (GL) points and weights, the Lagrange derivative
matrix, and interpolation between two node sets.

Test infrastructure only (see the package docstring).

Everything here goes through the Legendre basis of numpy.polynomial: the
nodes are the roots of P_p' polished by Newton steps, the derivative and
interpolation matrices come from Legendre Vandermonde matrices.  A second,
independent evaluation of the Lagrange polynomials by their product formula
(``lagrange_eval``) is used by the quadrature assembly in ``sipg``.
"""

import numpy as np
from numpy.polynomial import legendre as npleg


def _legendre_coeffs(p):
    c = np.zeros(p + 1)
    c[p] = 1.0
    return c


def gll(p):
    """Gauss-Lobatto-Legendre nodes xi_0 < ... < xi_p on [-1, 1] and weights.

    The interior nodes are the zeros of P_p'; the weights are
    w_i = 2 / (p (p+1) P_p(xi_i)^2).  p = 1 gives the two end points with
    unit weights.
    """
    if p < 1:
        raise ValueError("order p must be >= 1")
    if p == 1:
        return np.array([-1.0, 1.0]), np.array([1.0, 1.0])
    c = _legendre_coeffs(p)
    dc = npleg.legder(c)
    d2c = npleg.legder(dc)
    x = np.sort(npleg.legroots(dc).real)
    for _ in range(4):  # Newton polish on P_p'
        x = x - npleg.legval(x, dc) / npleg.legval(x, d2c)
    xi = np.concatenate(([-1.0], x, [1.0]))
    w = 2.0 / (p * (p + 1) * npleg.legval(xi, c) ** 2)
    return xi, w


def gl(p):
    """Gauss-Legendre nodes xi_0 < ... < xi_p on (-1, 1) and weights: the
    p + 1 zeros of P_{p+1}, w_i = 2 / ((1 - xi_i^2) P_{p+1}'(xi_i)^2); the
    rule integrates polynomials of degree up to 2p + 1 exactly.  Neither end
    point is a node, so element traces are combinations of all nodal values
    (Sec. 2, the GL basis of Table 1)."""
    if p < 0:
        raise ValueError("order p must be >= 0")
    c = _legendre_coeffs(p + 1)
    dc = npleg.legder(c)
    x = np.sort(npleg.legroots(c).real)
    for _ in range(4):  # Newton polish on P_{p+1}
        x = x - npleg.legval(x, c) / npleg.legval(x, dc)
    w = 2.0 / ((1.0 - x ** 2) * npleg.legval(x, dc) ** 2)
    return x, w


def rule(basis, p):
    """(nodes, weights) of the nodal basis 'gll' or 'gl' of order p."""
    if basis == "gll":
        return gll(p)
    if basis == "gl":
        return gl(p)
    raise ValueError(f"unknown basis {basis!r}")


def _vander_and_deriv(x, p):
    V = npleg.legvander(x, p)
    Vd = np.empty_like(V)
    for j in range(p + 1):
        Vd[:, j] = npleg.legval(x, npleg.legder(_legendre_coeffs(j)))
    return V, Vd


def diff_matrix(xi):
    """D[i, j] = phi_j'(xi_i) for the Lagrange basis on the nodes xi.

    With V[i, k] = P_k(xi_i) the Lagrange basis is phi_j = sum_k P_k C[k, j]
    where C = V^{-1}; hence D = V' V^{-1}.
    """
    p = len(xi) - 1
    V, Vd = _vander_and_deriv(xi, p)
    return np.linalg.solve(V.T, Vd.T).T


def end_values(xi):
    """Values phi_j(-1), phi_j(+1) and derivatives phi_j'(-1), phi_j'(+1) of
    the Lagrange basis on the nodes xi, through the Legendre Vandermonde
    route: returns (phi_m, phi_p, dphi_m, dphi_p)."""
    p = len(xi) - 1
    V = npleg.legvander(np.asarray(xi, dtype=float), p)
    E, Ed = _vander_and_deriv(np.array([-1.0, 1.0]), p)
    phi = np.linalg.solve(V.T, E.T).T
    dphi = np.linalg.solve(V.T, Ed.T).T
    return phi[0], phi[1], dphi[0], dphi[1]


def interp_matrix(xi_from, x_to):
    """J[i, j] = phi_j(x_to[i]) for the Lagrange basis on the nodes xi_from
    (the embedded interpolation of Sec. 3.2 when x_to are finer GLL nodes)."""
    p = len(xi_from) - 1
    V = npleg.legvander(xi_from, p)
    W = npleg.legvander(np.asarray(x_to, dtype=float), p)
    return np.linalg.solve(V.T, W.T).T


def lagrange_eval(xi, x):
    """Values and derivatives of every Lagrange polynomial on the nodes xi at
    the points x, by the product formula (independent of the Vandermonde
    route above).  Returns (phi, dphi) with shape (len(x), len(xi))."""
    xi = np.asarray(xi, dtype=float)
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = len(xi)
    phi = np.ones((len(x), n))
    dphi = np.zeros((len(x), n))
    for j in range(n):
        others = [k for k in range(n) if k != j]
        denom = np.prod([xi[j] - xi[k] for k in others])
        for q, xq in enumerate(x):
            factors = [xq - xi[k] for k in others]
            phi[q, j] = np.prod(factors) / denom
            s = 0.0
            for a in range(len(others)):
                s += np.prod([factors[b] for b in range(len(others)) if b != a])
            dphi[q, j] = s / denom
    return phi, dphi
