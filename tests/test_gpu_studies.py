"""The paper's convergence studies on the GPU solver.

Parity: on small meshes the GPU residual histories of the Table 1 methods
and of the three anisotropy methods equal the oracle's from the same seeded
start (same algorithm, rounding only).  Measurement: at the paper's own
meshes the GPU reproduces Table 1 (GLL rows) and the qualitative findings
of the anisotropic study (Sec. 4); the measured values are listed in the
design notes."""

import os

import numpy as np
import pytest

import oracle
from paper_1612_04796_amd import studies
from paper_1612_04796_amd.workloads import fourier_modes, uniform_vector

from _gpu import announce

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_gll.txt")
GOLDEN_FIG5 = os.path.join(os.path.dirname(__file__), "golden", "fig5_rates.txt")


def _oracle_history(params, solver, ncyc, tol=1e-11):
    h = oracle.Hierarchy(params["ne"], params["length"], params["P"], overlap=params["overlap"],
                         omega=params["omega"], growth=params.get("smooth_growth", 1),
                         basis=params.get("basis", "gll"), overlap_floor=params.get("overlap_floor", 0))
    k, phi, amp = fourier_modes(0, 3)
    b = oracle.fourier_rhs(k, phi, amp, h)
    x0 = uniform_vector(7, b.size)
    if solver == "mg":
        _, _, _, hist = oracle.mg_solve(b, h, tol=tol, maxcyc=ncyc, x0=x0)
    else:
        _, _, _, hist = oracle.fcg_solve(b, h, tol=tol, maxit=ncyc, x0=x0)
    return np.array(hist)


def _compare(params, solver, ncyc, tol=1e-11):
    got = np.array(studies.measure(params, solver=solver, ncyc=ncyc, tol=tol)["history"])
    ref = _oracle_history(params, solver, ncyc, tol)
    n = min(len(got), len(ref))
    assert n >= 3 and abs(len(got) - len(ref)) <= 1, (len(got), len(ref))
    # each entry relative to the initial residual (later entries are tiny)
    err = np.abs(got[:n] - ref[:n]) / ref[0]
    assert err.max() <= 1e-9, (err, got, ref)


@pytest.mark.parametrize("row", sorted(studies.TABLE1_ROWS))
def test_table1_methods_match_oracle_small(row):
    solver, overlap, omega, basis, floor = studies.TABLE1_ROWS[row]
    announce(f"table1 row {row} small")
    _compare(studies.table1_params(4, overlap, omega, ne=4, basis=basis, overlap_floor=floor), solver, ncyc=6)


@pytest.mark.parametrize("solver", ["mg", "fcg"])
@pytest.mark.parametrize("method", sorted(studies.ANISO_METHODS))
@pytest.mark.parametrize("AR", [4, 8])
def test_aniso_methods_match_oracle_small(method, AR, solver):
    announce(f"aniso {method} AR={AR} {solver} small")
    params = studies.aniso_params(AR, method, ne=4, P=4)
    _compare(params, solver, ncyc=6)


def _table1_paper():
    rows = {}
    for path in (GOLDEN, GOLDEN.replace("table1_gll", "table1_gl")):
        with open(path) as fh:
            for line in fh:
                if line.startswith("#") or not line.strip():
                    continue
                t = line.split()
                rows[int(t[0])] = dict(zip((4, 8, 16, 32), (float(v) for v in t[8:12])))
    return rows


def test_table1_at_paper_meshes():
    """-lg rho of the GLL rows at (128/P)^3 elements against the paper's
    Table 1: within 0.2 for the minimal and 8 % overlaps (rows 1-4; 20 of
    the 24 cells are within 0.1), within 0.3 for the 50 % overlap (rows 5-6),
    where 3-5 cycles reach 1e-11 and the rate estimate is coarser."""
    announce("table1 at paper meshes")
    paper = _table1_paper()
    for rec in studies.run_table1(rows=(1, 2, 3, 4, 5, 6)):
        want = paper[rec["row"]][rec["P"]]
        tol = 0.2 if rec["row"] <= 4 else 0.3
        assert abs(rec["neg_lg_rho"] - want) <= tol, (rec["row"], rec["P"], rec["neg_lg_rho"], want)


def test_table1_gl_at_paper_meshes():
    """The GL rows (7-14) of Table 1 at (128/P)^3 elements: every cell within
    0.3 of the paper's, except row 7 at P = 4, whose printed 0.73 repeats row
    9's cell although rows 7 and 13 have the same overlap layers at P = 4
    (row 13 reads 1.36; both measure about 1.38 here)."""
    announce("table1 GL at paper meshes")
    paper = _table1_paper()
    bad = []
    for rec in studies.run_table1(rows=tuple(range(7, 15))):
        if rec["row"] == 7 and rec["P"] == 4:
            continue
        want = paper[rec["row"]][rec["P"]]
        if abs(rec["neg_lg_rho"] - want) > 0.3:
            bad.append((rec["row"], rec["P"], rec["neg_lg_rho"], want))
    assert not bad, bad


def test_aniso_study_trends():
    """The anisotropic study (8^3 elements, P = 16, AR up to 48, the three
    methods as preconditioners of flexible CG) against the paper's account
    (Sec. 4, Anisotropic Meshes): the "max" overlap with the variable
    V-cycle needs 4 cycles per ten decades on the isotropic mesh and at most
    13 at AR = 48, and it is the best of the three at every aspect ratio
    from 8 on; the fixed V-cycle with the relative overlap has slowed by
    about two orders of magnitude at AR = 16 (its rate rho here grows by a
    factor 30 to 300) but still converges; the variable V-cycle improves on
    the fixed one up to AR = 12.  Not reproduced, and not asserted: the
    relative overlap with the variable cycle keeping a nearly constant
    count to AR = 12 and staying ahead of the fixed cycle beyond (it
    stagnates from AR = 16 here); the design notes list the readings
    tried."""
    announce("aniso study")
    ars = (1, 8, 12, 16, 48)
    res = {(r["method"], r["AR"]): r for r in studies.run_aniso(ars=ars)}
    n10 = {m: [res[(m, ar)]["n10"] for ar in ars] for m in studies.ANISO_METHODS}
    mv = n10["max_var"]
    assert all(v is not None for v in mv), n10
    assert mv[0] <= 4 and mv[-1] <= 13, n10                       # 4 ... 13 in the paper
    assert mv == sorted(mv), n10                                    # grows with AR
    for i, ar in enumerate(ars):
        if ar >= 8:
            assert mv[i] < n10["rel_fix"][i] and mv[i] < n10["rel_var"][i], (ar, n10)
    slow = res[("rel_fix", 16)]["rho"] / res[("rel_fix", 1)]["rho"]
    assert 30 <= slow <= 300 and n10["rel_fix"][3] is not None, (slow, n10)
    for i, ar in enumerate(ars):
        if ar <= 12:
            assert n10["rel_var"][i] <= n10["rel_fix"][i], (ar, n10)


def test_fig5_mesh_independence_and_rates():
    """Fig. 5 as the paper's text states it (Sec. 4): with 8 % overlap the
    V(1,1) rate is mesh independent from about 12^3 elements for P <= 16,
    and reaches about 6.3e-3 at P = 16 and 1.6e-3 at P = 32.  Checked on a
    reduced sweep: the rates on meshes of 8^3 elements and more agree within
    a factor 1.5 for each P <= 16, and the rates on the finest meshes run
    are within a factor 2 of the stated values (a rate from 4-6 cycles to
    1e-11 varies by about that much with the mesh)."""
    announce("fig5 sweep")
    stated = {}
    with open(GOLDEN_FIG5) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                p, rho = line.split()
                stated[int(p)] = float(rho)
    meshes = {8: (4, 8, 16), 16: (4, 8, 12), 32: (4, 6, 8)}
    res = {}
    for rec in studies.run_fig5(orders=(8, 16, 32), meshes=meshes):
        res[(rec["P"], rec["ne"])] = rec["rho"]
    for P in (8, 16):
        fine = [res[(P, ne)] for ne in meshes[P] if ne >= 8]
        assert max(fine) <= 1.5 * min(fine), (P, fine)
    for P in (16, 32):
        got = res[(P, meshes[P][-1])]
        assert stated[P] / 2 <= got <= 2 * stated[P], (P, got, stated[P])
