"""Convergence studies of the paper run on the GPU solver.

* Table 1 (Sec. 4, isotropic meshes): V(1,1) multigrid ("MG") and the
  multigrid-preconditioned flexible CG ("MGCG") on (128/P)^3 elements, GLL
  basis (rows 1-6) and GL basis (rows 7-14), overlaps "minimal", 8 %, 9 %
  (with at least one layer) and 50 % of the element width; the measure is
  -lg rho with rho = (r_n / r_0)^(1/n) from a random start.
* The anisotropic study (Sec. 4, anisotropic meshes, the three methods of
  Table 2): 8^3 elements of order 16 on (0, 2 pi AR) x (0, 2 pi ceil(AR/2))
  x (0, 2 pi), overlap 8 % relative or 8 % of the largest element side
  (capped by the element width), fixed V(1,1) or the variable V-cycle with
  3^(L-l) smoothing steps on level l, each as the preconditioner of
  flexible CG: Table 2 names only overlap and smoothing, and the paper's
  conclusions (Sec. 5) credit its anisotropic result to Krylov
  acceleration, variable smoothing and the larger overlap together.
* The mesh sweep of Fig. 5 (Sec. 4, isotropic meshes): the rate of V(1,1)
  multigrid with 8 % overlap against the number of elements, for P = 4, 8,
  16 and 32 (the paper reports mesh independence from about 12^3 elements
  for P <= 16, and rho of about 6.3e-3 at P = 16 and 1.6e-3 at P = 32).

Every input is seeded and synthetic: the right-hand side is the seeded
Fourier load and the start vector U[-1, 1] (the paper's own test problem is
printed garbled).  Run as

    python -m paper_1612_04796_amd.studies table1 | aniso | aniso_mg | fig5

which prints one JSON object per case.
"""

import json
import math
import sys
import time

from .workloads import fourier_modes, uniform_vector

# Table 1 rows: (solver, overlap policy, omega, basis, overlap floor); rows
# 1-6 use the GLL basis, rows 7-14 the GL basis (rows 13-14 with N_O >= 1)
TABLE1_ROWS = {
    1: ("mg", "min", 0.0, "gll", 0), 2: ("fcg", "min", 0.0, "gll", 0),
    3: ("mg", "rel", 0.08, "gll", 0), 4: ("fcg", "rel", 0.08, "gll", 0),
    5: ("mg", "rel", 0.5, "gll", 0), 6: ("fcg", "rel", 0.5, "gll", 0),
    7: ("mg", "min", 0.0, "gl", 0), 8: ("fcg", "min", 0.0, "gl", 0),
    9: ("mg", "rel", 0.08, "gl", 0), 10: ("fcg", "rel", 0.08, "gl", 0),
    11: ("mg", "rel", 0.5, "gl", 0), 12: ("fcg", "rel", 0.5, "gl", 0),
    13: ("mg", "rel", 0.09, "gl", 1), 14: ("fcg", "rel", 0.09, "gl", 1),
}

# the three methods of Table 2: (overlap policy, smoothing growth per level)
ANISO_METHODS = {"rel_fix": ("rel", 1), "rel_var": ("rel", 3), "max_var": ("max", 3)}
# Krylov-accelerated (multigrid-preconditioned CG), see the module docstring
ANISO_SOLVER = "fcg"


def table1_params(P, overlap, omega, ne=None, basis="gll", overlap_floor=0):
    ne = ne if ne is not None else 128 // P
    return dict(ne=(ne,) * 3, length=(1.0, 1.0, 1.0), P=P, overlap=overlap, omega=omega, basis=basis,
                overlap_floor=overlap_floor)


def aniso_params(AR, method, ne=8, P=16):
    overlap, growth = ANISO_METHODS[method]
    two_pi = 2.0 * math.pi
    return dict(ne=(ne,) * 3, length=(two_pi * AR, two_pi * math.ceil(AR / 2), two_pi), P=P,
                overlap=overlap, omega=0.08, smooth_growth=growth)


def rate(hist):
    """rho = (r_n / r_0)^(1/n), -lg rho and n10 = ceil(10 / -lg rho)."""
    n = len(hist) - 1
    rho = (hist[-1] / hist[0]) ** (1.0 / n) if n >= 1 and hist[0] > 0 else 0.0
    nlg = -math.log10(rho) if rho > 0 else math.inf
    return {"rho": rho, "neg_lg_rho": nlg, "n10": math.ceil(10.0 / nlg) if 0 < nlg < math.inf else None,
            "cycles": n}


def measure(params, solver="mg", ncyc=12, tol=1e-11, seed_rhs=0, seed_x0=7, kmax=3, precond_bits=64):
    """Residual history of one solve from the seeded random start; returns
    the rate measures, the history and the wall time per cycle."""
    import torch
    from . import sipg

    s = sipg.Solver(precond_bits=precond_bits, **params)
    try:
        N = s.ndof()
        b = torch.zeros(N, dtype=torch.float64, device="cuda")
        k, phi, amp = fourier_modes(seed_rhs, kmax)
        s.rhs_fourier(k, phi, amp, b)
        x0 = torch.as_tensor(uniform_vector(seed_x0, N), dtype=torch.float64).cuda()
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if solver == "mg":
            s.mg_solve(x, b, tol, ncyc, raise_on_noconv=False)
        else:
            s.pcg_solve(x, b, tol, ncyc, raise_on_noconv=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        hist = s.residual_history()
    finally:
        s.close()
    out = rate(hist)
    out.update({"ndof": N, "history": hist, "s_per_cycle": el / max(1, out["cycles"]),
                "us_per_unknown_per_cycle": 1e6 * el / max(1, out["cycles"]) / N})
    return out


def run_table1(orders=(4, 8, 16, 32), rows=tuple(TABLE1_ROWS), ncyc=12):
    for row in rows:
        solver, overlap, omega, basis, floor = TABLE1_ROWS[row]
        for P in orders:
            ne = 128 // P
            r = measure(table1_params(P, overlap, omega, ne=ne, basis=basis, overlap_floor=floor), solver=solver,
                        ncyc=ncyc)
            r.pop("history")
            yield {"study": "table1", "row": row, "solver": solver, "overlap": overlap, "omega": omega,
                   "basis": basis, "P": P, "ne": ne, **r}


def run_aniso(ars=(1, 2, 4, 8, 12, 16, 24, 32, 48), methods=tuple(ANISO_METHODS), ncyc=150, solver=ANISO_SOLVER):
    for method in methods:
        for AR in ars:
            r = measure(aniso_params(AR, method), solver=solver, ncyc=ncyc, tol=1e-10)
            r.pop("history")
            yield {"study": "aniso", "method": method, "solver": solver, "AR": AR, **r}


# element counts per direction of the Fig. 5 sweep, per order (the largest
# mesh of each order has 1.4e7 to 1.5e8 unknowns)
FIG5_MESHES = {4: (4, 6, 8, 12, 16, 24, 32, 48), 8: (4, 6, 8, 12, 16, 24, 32), 16: (4, 6, 8, 12, 16, 24),
               32: (3, 4, 6, 8, 12, 16)}


def run_fig5(orders=(4, 8, 16, 32), meshes=None, ncyc=12):
    meshes = meshes or FIG5_MESHES
    for P in orders:
        for ne in meshes[P]:
            r = measure(table1_params(P, "rel", 0.08, ne=ne), solver="mg", ncyc=ncyc)
            r.pop("history")
            yield {"study": "fig5", "P": P, "ne": ne, **r}


def main(argv):
    which = argv[1] if len(argv) > 1 else "table1"
    if which == "aniso_mg":  # the same methods as plain V-cycle iterations
        gen = run_aniso(ncyc=40, solver="mg")
    else:
        gen = {"table1": run_table1, "aniso": run_aniso, "fig5": run_fig5}[which]()
    for rec in gen:
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main(sys.argv)
