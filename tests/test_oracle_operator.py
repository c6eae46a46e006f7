"""Pins of the oracle's SIPG operator (paper Sec. 2, eq. (A)): structural
properties the paper states, the constant null space of the periodic
problem, the stability threshold of the penalty, and an independent direct
quadrature assembly of the interior penalty form."""

import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle.sipg import Discretization1D


@pytest.mark.parametrize("p,ne,length", [(1, 4, 1.0), (2, 3, 2.0), (4, 4, 1.0), (7, 5, 3.0), (8, 4, 1.0)])
def test_1d_matrices_properties(p, ne, length):
    d = Discretization1D(p, ne, length)
    assert np.all(d.M > 0)
    assert abs(d.M.sum() - length) < 1e-13          # mass integrates the constant
    assert np.allclose(d.L, d.L.T, atol=1e-12)
    assert np.allclose(d.L @ np.ones(d.N), 0.0, atol=1e-10 * np.abs(d.L).max())
    ev = np.linalg.eigvalsh(d.L)
    assert ev[0] > -1e-10 * ev[-1] and abs(ev[0]) < 1e-10 * ev[-1]
    assert ev[1] > 1e-6                              # a single zero eigenvalue
    # block-cyclic tridiagonal: no coupling between elements two apart
    n = d.n
    if ne >= 4:
        assert np.all(d.L[:n, 2 * n:3 * n] == 0)


def test_second_eigenvalue_approaches_continuum():
    # the smallest nonzero generalized eigenvalue approximates (2 pi / l)^2
    d = Discretization1D(4, 4, 1.0)
    lam = scipy.linalg.eigh(d.L, np.diag(d.M), eigvals_only=True)
    assert abs(lam[1] - 4 * math.pi ** 2) / (4 * math.pi ** 2) < 1e-4


@pytest.mark.parametrize("p", [1, 2, 4, 8, 16])
def test_penalty_stability_threshold(p):
    # L is positive semi-definite iff c_mu >= 1/2 (the threshold P(P+1)/(2h))
    def min_ev(cmu):
        d = Discretization1D(p, 4, 1.0, cmu=cmu)
        return np.linalg.eigvalsh(d.L)[0] / np.abs(d.L).max()
    assert min_ev(0.49) < -1e-8
    assert min_ev(0.51) > -1e-12


@pytest.mark.parametrize("ne,length,p", [((3, 3, 3), (1.0, 1.0, 1.0), 2),
                                         ((3, 4, 3), (2.0, 1.0, 0.5), 2),
                                         ((3, 3, 3), (1.0, 1.0, 1.0), 3)])
def test_kronecker_equals_direct_quadrature(ne, length, p):
    A_direct = oracle.assemble_ip_dense(ne, length, p)
    discs = tuple(Discretization1D(p, ne[d], length[d]) for d in range(3))
    N = A_direct.shape[0]
    # columns of the Kronecker operator from global unit vectors
    n = p + 1
    A_kron = np.empty_like(A_direct)
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        g = e.reshape(ne[2] * n, ne[1] * n, ne[0] * n)
        A_kron[:, c] = oracle.sipg.apply_A_global(g, *discs).reshape(-1)
    scale = np.abs(A_direct).max()
    assert np.abs(A_kron - A_direct).max() < 1e-12 * scale


def test_3d_operator_symmetric_with_single_constant_null_vector():
    ne, p = (3, 3, 3), 2
    A = oracle.assemble_ip_dense(ne, (1.0, 1.0, 1.0), p)
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
    one = np.ones(A.shape[0])
    assert np.abs(A @ one).max() < 1e-12 * np.abs(A).max()
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0]) < 1e-10 * ev[-1]
    assert ev[1] > 1e-6 * ev[-1]


def test_element_major_roundtrip():
    ne, n = (3, 4, 5), 3
    v = np.arange(np.prod(ne) * n ** 3, dtype=float)
    g = oracle.to_global(v, ne, n)
    assert g.shape == (ne[2] * n, ne[1] * n, ne[0] * n)
    # element (ex,ey,ez)=(1,2,3), node (i,j,k)=(2,0,1)
    e = (3 * ne[1] + 2) * ne[0] + 1
    assert g[3 * n + 1, 2 * n + 0, 1 * n + 2] == v[e * n ** 3 + (1 * n + 0) * n + 2]
    assert np.array_equal(oracle.to_element(g, ne, n), v)


# ---- the GL basis (Sec. 2; Table 1 rows 7-14) ------------------------------
@pytest.mark.parametrize("p,ne,length", [(1, 4, 1.0), (2, 3, 2.0), (4, 4, 1.0), (7, 5, 3.0)])
def test_1d_matrices_properties_gl(p, ne, length):
    d = Discretization1D(p, ne, length, basis="gl")
    assert np.all(d.M > 0) and abs(d.M.sum() - length) < 1e-13
    assert np.allclose(d.L, d.L.T, atol=1e-12)
    assert np.allclose(d.L @ np.ones(d.N), 0.0, atol=1e-10 * np.abs(d.L).max())
    ev = np.linalg.eigvalsh(d.L)
    assert abs(ev[0]) < 1e-10 * ev[-1] and ev[1] > 1e-6
    n = d.n
    # the face coupling blocks are full (traces of GL lines use every node)
    assert np.count_nonzero(np.abs(d.L[:n, n:2 * n]) > 1e-12) == n * n
    if ne >= 4:
        assert np.all(d.L[:n, 2 * n:3 * n] == 0)


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_penalty_stability_threshold_gl(p):
    def min_ev(cmu):
        d = Discretization1D(p, 4, 1.0, cmu=cmu, basis="gl")
        return np.linalg.eigvalsh(d.L)[0] / np.abs(d.L).max()
    assert min_ev(0.49) < -1e-8
    assert min_ev(0.51) > -1e-12


@pytest.mark.parametrize("ne,length,p", [((3, 3, 3), (1.0, 1.0, 1.0), 2), ((3, 4, 3), (2.0, 1.0, 0.5), 1)])
def test_kronecker_equals_direct_quadrature_gl(ne, length, p):
    A_direct = oracle.assemble_ip_dense(ne, length, p, basis="gl")
    discs = tuple(Discretization1D(p, ne[d], length[d], basis="gl") for d in range(3))
    N = A_direct.shape[0]
    n = p + 1
    A_kron = np.empty_like(A_direct)
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        g = e.reshape(ne[2] * n, ne[1] * n, ne[0] * n)
        A_kron[:, c] = oracle.sipg.apply_A_global(g, *discs).reshape(-1)
    assert np.abs(A_kron - A_direct).max() < 1e-12 * np.abs(A_direct).max()
