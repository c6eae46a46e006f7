"""Pins of the oracle's Schwarz smoother (paper Sec. 3.1): N_O against the
paper's Table 1, fast diagonalization against dense LU of R_s A R_s^T, the
weights' partition of unity, and the whole additive step against a brute
force sum over subdomains with dense solves."""

import os

import numpy as np
import pytest

import oracle
from oracle.sipg import Discretization1D
from oracle.schwarz import SubdomainTables, overlap_delta, overlap_layers, subdomain_solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_gll.txt")


def _table1_rows():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows[int(t[0])] = {"solver": t[1], "overlap": t[2],
                               "no": [int(v) for v in t[3:8]],
                               "rate": [float(v) for v in t[8:12]]}
    return rows


TABLE1 = _table1_rows()
OVERLAP_REL = {"no1": 0.0, "rel08": 0.08, "rel50": 0.50}


@pytest.mark.parametrize("row", [1, 3, 5])
def test_overlap_layers_match_table1(row):
    spec = TABLE1[row]
    got = [overlap_layers(oracle.gll(p)[0], OVERLAP_REL[spec["overlap"]]) for p in (2, 4, 8, 16, 32)]
    assert got == spec["no"]


def test_overlap_modes():
    h = (2.0, 0.125, 0.125)   # the 16:1:1 aspect-ratio mesh, 8 elements on [0,16]x[0,1]^2
    assert overlap_delta("min", 0.08, h, 0) == 0.0
    assert overlap_delta("rel", 0.08, h, 1) == 0.08
    assert abs(overlap_delta("max", 0.08, h, 0) - 0.08) < 1e-15
    assert overlap_delta("max", 0.08, h, 1) == 1.0
    xi16 = oracle.gll(16)[0]
    assert overlap_layers(xi16, overlap_delta("max", 0.08, h, 0)) == 3
    assert overlap_layers(xi16, overlap_delta("max", 0.08, h, 2)) == 17


def test_weights_closed_form_minimal_overlap():
    # P=4, N_O=1: the first excluded node is xi_1 = -sqrt(3/7), so the
    # transition ends exactly at the inner core nodes and the weights are
    # 1/2 on the four face nodes and 1 on the three interior core nodes.
    w = oracle.hat_weights(oracle.gll(4)[0], 1)
    assert np.allclose(w, [0.5, 0.5, 1, 1, 1, 0.5, 0.5], atol=1e-14)


@pytest.mark.parametrize("p,no", [(2, 1), (4, 1), (4, 2), (8, 2), (8, 5), (16, 3), (16, 17), (7, 2), (32, 6)])
def test_weights_partition_of_unity_1d(p, no):
    ne = 5
    d = Discretization1D(p, ne, 1.0)
    t = SubdomainTables(d, no)
    acc = np.zeros(d.N)
    for e in range(ne):
        np.add.at(acc, t.index(e), t.w)
    assert np.allclose(acc, 1.0, atol=1e-14)
    n = p + 1
    assert abs(t.w[no] - 0.5) < 1e-14 and abs(t.w[no + n - 1] - 0.5) < 1e-14
    assert np.all(t.w >= 0) and np.all(t.w <= 1.0 + 1e-15)


def _dense_A(discs):
    dx, dy, dz = discs
    Lx, Ly, Lz = dx.L, dy.L, dz.L
    Mx, My, Mz = np.diag(dx.M), np.diag(dy.M), np.diag(dz.M)
    return (np.kron(Mz, np.kron(My, Lx)) + np.kron(Mz, np.kron(Ly, Mx))
            + np.kron(Lz, np.kron(My, Mx)))


def _sub_index3(tabs, e3, Ns):
    Ix, Iy, Iz = (tabs[d].index(e3[d]) for d in range(3))
    return ((Iz[:, None, None] * Ns[1] + Iy[None, :, None]) * Ns[0] + Ix[None, None, :]).reshape(-1)


CASES = [
    # (ne, length, p, overlap mode, omega)
    ((4, 4, 4), (1.0, 1.0, 1.0), 2, "min", 0.0),
    ((4, 3, 4), (2.0, 1.0, 1.0), 3, "rel", 0.3),    # N_O = 2 at P=3
    ((4, 4, 4), (4.0, 1.0, 1.0), 2, "max", 0.3),    # full-neighbour overlap in y, z
]


@pytest.mark.parametrize("ne,length,p,mode,omega", CASES)
def test_fdm_equals_dense_lu(ne, length, p, mode, omega):
    discs = tuple(Discretization1D(p, ne[d], length[d]) for d in range(3))
    h = tuple(length[d] / ne[d] for d in range(3))
    nos = [overlap_layers(discs[d].xi, overlap_delta(mode, omega, h, d)) for d in range(3)]
    tabs = tuple(SubdomainTables(discs[d], nos[d]) for d in range(3))
    A = _dense_A(discs)
    Ns = [discs[d].N for d in range(3)]
    rng = np.random.default_rng(3)
    for e3 in [(0, 0, 0), (1, 2, 3 % ne[2])]:
        I = _sub_index3(tabs, e3, Ns)
        Ass = A[np.ix_(I, I)]
        r = rng.standard_normal(len(I))
        du_lu = np.linalg.solve(Ass, r)
        m = [tabs[d].m for d in range(3)]
        du_fdm = subdomain_solve(r.reshape(m[2], m[1], m[0]), tabs).reshape(-1)
        assert np.linalg.norm(du_fdm - du_lu) <= 1e-12 * np.linalg.norm(du_lu)


@pytest.mark.parametrize("ne,length,p,mode,omega", CASES)
def test_schwarz_step_equals_brute_force(ne, length, p, mode, omega):
    discs = tuple(Discretization1D(p, ne[d], length[d]) for d in range(3))
    h = tuple(length[d] / ne[d] for d in range(3))
    nos = [overlap_layers(discs[d].xi, overlap_delta(mode, omega, h, d)) for d in range(3)]
    tabs = tuple(SubdomainTables(discs[d], nos[d]) for d in range(3))
    A = _dense_A(discs)
    Ns = [discs[d].N for d in range(3)]
    rng = np.random.default_rng(4)
    r = rng.standard_normal(A.shape[0])
    du = np.zeros_like(r)
    for ez in range(ne[2]):
        for ey in range(ne[1]):
            for ex in range(ne[0]):
                I = _sub_index3(tabs, (ex, ey, ez), Ns)
                loc = np.linalg.solve(A[np.ix_(I, I)], r[I])
                W = np.kron(tabs[2].w, np.kron(tabs[1].w, tabs[0].w))
                np.add.at(du, I, W * loc)
    got = oracle.schwarz_correction(r.reshape(Ns[2], Ns[1], Ns[0]), tabs).reshape(-1)
    assert np.linalg.norm(got - du) <= 1e-12 * np.linalg.norm(du)


def test_schwarz_weights_partition_of_unity_3d():
    # sum_s R_s^T W_s 1 = 1 on the 3D mesh (checked through the scatter path)
    ne, p = (3, 4, 5), 4
    discs = tuple(Discretization1D(p, ne[d], 1.0) for d in range(3))
    tabs = tuple(SubdomainTables(discs[d], 2) for d in range(3))
    Ns = [d.N for d in discs]
    acc = np.zeros(Ns[0] * Ns[1] * Ns[2])
    for ez in range(ne[2]):
        for ey in range(ne[1]):
            for ex in range(ne[0]):
                I = _sub_index3(tabs, (ex, ey, ez), Ns)
                np.add.at(acc, I, np.kron(tabs[2].w, np.kron(tabs[1].w, tabs[0].w)))
    assert np.allclose(acc, 1.0, atol=1e-14)


# ---- the weight function of Fig. 2 on dense synthetic node sets ------------
# The caption fixes: a piecewise quintic transition, 0 at the subdomain
# boundary, 1 on the part of the core that no neighbour's subdomain overlaps;
# the global correction is a weighted average (partition of unity).  Node sets
# with hundreds of nodes sample the transition finely enough to see its
# polynomial degree and where it ends.  (The C^2 smoothstep among the
# quintics is the reading, pinned by the golden 1D values and Table 1.)
def _dense_nodes(n):
    # symmetric, strictly increasing, end points +-1 (Chebyshev-Lobatto)
    return -np.cos(np.pi * np.arange(n) / (n - 1))


def _xi_h(xi, no):
    n = len(xi)
    return np.concatenate((xi[n - no:] - 2.0, xi, xi[:no] + 2.0))


@pytest.mark.parametrize("n,no", [(201, 20), (201, 57), (301, 120), (101, 4)])
def test_weight_transition_is_quintic_and_ends_at_subdomain_boundary(n, no):
    xi = _dense_nodes(n)
    w = oracle.hat_weights(xi, no)
    xh = _xi_h(xi, no)
    assert len(w) == n + 2 * no
    # 0 at the subdomain boundary: the first neighbour node left out of the
    # subdomain (the discrete Dirichlet boundary of the local problem) ...
    b = xi[n - no - 1] - 2.0
    # ... while every node of the subdomain keeps a positive weight
    assert np.all(w > 0.0)
    # 1 exactly on the core nodes no neighbour subdomain reaches (index
    # no .. n-1-no of the core), below 1 on the overlapped ones
    core = w[no:no + n]
    assert np.all(core[no:n - no] == 1.0)
    assert np.all(core[:no] < 1.0) and np.all(core[n - no:] < 1.0)
    # the left transition: halo nodes plus overlapped core nodes, a single
    # polynomial in xi_H of degree exactly 5 that vanishes at the boundary
    sel = xh < xi[no]                        # every node left of the first non-overlapped core node
    xs, ws = xh[sel], w[sel]
    assert len(xs) >= 8
    fit = np.polynomial.Polynomial.fit          # least squares on the scaled interval
    p5, p4 = fit(xs, ws, 5), fit(xs, ws, 4)
    r5 = np.abs(p5(xs) - ws).max()
    r4 = np.abs(p4(xs) - ws).max()
    assert r5 <= 1e-10, r5                   # a quintic ...
    assert r4 >= 1e-4, r4                    # ... not of lower degree (a cubic step fails here)
    assert abs(p5(b)) <= 1e-9
    # it reaches 1 where the non-overlapped core starts
    assert abs(p5(xi[no]) - 1.0) <= 1e-9
    # mirror symmetry and the weighted average: 1/2 at the face
    assert abs(p5(-1.0) - 0.5) <= 1e-9


def test_weights_full_neighbour_overlap_reading():
    # N_O = n (a whole neighbour in the subdomain): the transition is read as
    # spanning one element width on each side of the face (delta = 1), so the
    # three overlapping subdomains of a node still average to one; the outer
    # half of the included neighbour gets weight 0.
    xi = oracle.gll(16)[0]
    w = oracle.hat_weights(xi, 17)
    xh = _xi_h(xi, 17)
    assert np.all(w[np.abs(xh) >= 2.0] == 0.0)
    assert np.all(w[np.abs(xh) < 2.0] > 0.0)
    assert np.allclose(w[np.abs(np.abs(xh) - 1.0) < 1e-14], 0.5, atol=1e-14)


# ---- GL basis: overlap layers and weights (Table 1 rows 7-14) -------------
GOLDEN_GL = os.path.join(os.path.dirname(__file__), "golden", "table1_gl.txt")


def _gl_rows():
    rows = {}
    with open(GOLDEN_GL) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t = line.split()
                rows[int(t[0])] = (t[2], [int(v) for v in t[3:8]])
    return rows


GL_OVERLAP = {"rel08": (0.08, 0), "rel50": (0.5, 0), "rel09f": (0.09, 1)}


@pytest.mark.parametrize("row", [9, 10, 11, 12, 13, 14])
def test_gl_overlap_layers_match_table1(row):
    # strict count (a node exactly at delta_O is not included: the middle
    # node at 0.5 dx, row 11), possibly zero (row 9 at P = 2), and the lower
    # bound of rows 13-14
    spec, want = _gl_rows()[row]
    omega, floor = GL_OVERLAP[spec]
    got = [overlap_layers(oracle.gl(p)[0], omega, "gl", floor) for p in (2, 4, 8, 16, 32)]
    assert got == want


@pytest.mark.parametrize("p,no", [(2, 0), (4, 1), (4, 2), (8, 1), (8, 4), (16, 3), (16, 17)])
def test_gl_weights_partition_of_unity(p, no):
    xi = oracle.gl(p)[0]
    n = len(xi)
    w = oracle.hat_weights(xi, no)
    assert len(w) == n + 2 * no
    # own weights plus the left and right neighbours' halo weights on the
    # element's nodes sum to one
    tot = w[no:no + n].copy()
    if no:
        tot[:no] += w[-no:]           # the left neighbour's right halo
        tot[n - no:] += w[:no]        # the right neighbour's left halo
    assert np.allclose(tot, 1.0, atol=1e-14)
    if no == 0:
        assert np.all(w == 1.0)
