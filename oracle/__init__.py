"""FP64 CPU oracle for the Cartesian SIPG Poisson multigrid method.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package.  The product (the HIP library and its Python binding) never
imports, calls or links anything here, and this package imports nothing from
the product: the two share no code, tables or helpers.

The oracle is written to be read against the paper (Stiller, "Robust
Multigrid for Cartesian Interior Penalty DG Formulations of the Poisson
Equation in 3D", arXiv 1612.04796).  Everything is plain NumPy/SciPy in
float64, with dense 1D matrices and Kronecker-structured 3D operators, and no
blocking or fusion beyond what the method's definitions state.

Modules
  basis      GLL and GL nodes and weights, Lagrange derivative, end values and
             interpolation (Sec. 2)
  sipg       1D mass/stiffness, 3D Kronecker operator eq. (A), and an
             independent element+face quadrature of the interior penalty form
  schwarz    overlap layers, restricted 1D eigenpairs, hat weights and the
             weighted additive Schwarz step (Sec. 3.1)
  multigrid  polynomial hierarchy, transfers, coarse pseudo-inverse,
             V-cycle (Algorithm 1), MG solve, flexible CG (Sec. 3.2)
  problem    Fourier right-hand side, manufactured solution, exact discrete
             solution by global fast diagonalization, rate metrics (Sec. 4)

Readings of the paper where it is silent or garbled are stated in the
docstrings of the functions that take them (penalty factor, weight function,
level sequence for P not a power of two, right-hand-side projection, flexible
CG details).
"""

from .basis import gll, gl, rule, end_values, diff_matrix, interp_matrix, lagrange_eval
from .sipg import Discretization1D, apply_A, to_global, to_element, assemble_ip_dense
from .schwarz import overlap_layers, SubdomainTables, hat_weights, schwarz_correction
from .multigrid import (Hierarchy, level_orders, vcycle, smoother, mg_solve, fcg_solve,
                        coarse_solve, apply_level, schwarz_step_correction, restrict, prolong)
from .problem import (fourier_rhs, manufactured, manufactured_rhs, exact_solution,
                      residual_norm, rate_metrics, node_coordinates)

__all__ = [
    "gll", "gl", "rule", "end_values", "diff_matrix", "interp_matrix", "lagrange_eval",
    "Discretization1D", "apply_A", "to_global", "to_element", "assemble_ip_dense",
    "overlap_layers", "SubdomainTables", "hat_weights", "schwarz_correction",
    "Hierarchy", "level_orders", "apply_level", "schwarz_step_correction",
    "restrict", "prolong", "vcycle", "smoother", "mg_solve", "fcg_solve", "coarse_solve",
    "fourier_rhs", "manufactured", "manufactured_rhs", "node_coordinates", "exact_solution", "residual_norm", "rate_metrics",
]
