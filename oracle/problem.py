"""Right-hand sides, the exact discrete solution and the paper's rate metrics
(paper Sec. 4).

Test infrastructure only (see the package docstring).

The paper's own test problem is printed in a garbled form (all variables read
x), so the workloads use a seeded sum of Fourier modes instead: a smooth,
periodic, mean-free load.  The mode parameters (wavenumbers, phases and
amplitudes) are drawn by the shared workload generator and passed in here.

The discrete right-hand side is the GLL quadrature of int v f, i.e.
b = (Mz x My x Mx) f(nodes), projected onto the range of the singular
periodic operator (Euclidean mean removed).
"""

import math

import numpy as np
import scipy.linalg

from .sipg import to_element, to_global, _along as _axis


def node_coordinates(disc):
    """Physical coordinates of the N = ne*n global nodes of one direction."""
    e = np.arange(disc.ne)[:, None]
    return (e * disc.h + (1.0 + disc.xi[None, :]) * disc.h / 2.0).reshape(-1)


def _mass3(hier):
    dx, dy, dz = hier.top.discs
    return dz.M[:, None, None] * dy.M[None, :, None] * dx.M[None, None, :]


def fourier_rhs(k, phi, amp, hier):
    """b for f(x) = sum_q amp_q prod_d sin(2 pi k_qd x_d / l_d + phi_qd).

    k: (Q, 3) integer wavenumbers, phi: (Q, 3) phases, amp: (Q,) amplitudes.
    Returns the element-major b with its Euclidean mean removed."""
    dx, dy, dz = hier.top.discs
    X = [node_coordinates(d) for d in (dx, dy, dz)]
    k = np.asarray(k, dtype=float)
    phi = np.asarray(phi, dtype=float)
    F = np.zeros((dz.N, dy.N, dx.N))
    for q in range(len(amp)):
        fx = np.sin(2 * math.pi * k[q, 0] * X[0] / hier.length[0] + phi[q, 0])
        fy = np.sin(2 * math.pi * k[q, 1] * X[1] / hier.length[1] + phi[q, 1])
        fz = np.sin(2 * math.pi * k[q, 2] * X[2] / hier.length[2] + phi[q, 2])
        F += amp[q] * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    B = _mass3(hier) * F
    B -= B.mean()
    return to_element(B, hier.ne, hier.top.n)


def manufactured(hier):
    """Manufactured solution u = prod_d sin(2 pi x_d / l_d) and its load
    f = -lap u; returns (b, u_nodes) element-major, b mean-free."""
    dx, dy, dz = hier.top.discs
    X = [node_coordinates(d) for d in (dx, dy, dz)]
    s = [np.sin(2 * math.pi * X[d] / hier.length[d]) for d in range(3)]
    U = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
    lapc = sum((2 * math.pi / hier.length[d]) ** 2 for d in range(3))
    B = _mass3(hier) * (lapc * U)
    B -= B.mean()
    n = hier.top.n
    return to_element(B, hier.ne, n), to_element(U, hier.ne, n)


def manufactured_rhs(hier):
    return manufactured(hier)[0]


def exact_solution(b, hier):
    """u* = A^+ b on the top level by global fast diagonalization with the
    generalized eigenpairs of the global periodic (L_d, M_d); minimum
    Euclidean norm gauge."""
    discs = hier.top.discs
    eig = [scipy.linalg.eigh(d.L, np.diag(d.M)) for d in discs]
    (lx, Sx), (ly, Sy), (lz, Sz) = eig
    n = hier.top.n
    f = to_global(b, hier.ne, n)
    f = f - f.mean()
    t = _axis(f, Sx.T, 2)
    t = _axis(t, Sy.T, 1)
    t = _axis(t, Sz.T, 0)
    lam = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]
    inv = 1.0 / np.where(lam == 0, 1.0, lam)
    inv[np.argmin(np.abs(lz)), np.argmin(np.abs(ly)), np.argmin(np.abs(lx))] = 0.0
    t = t * inv
    t = _axis(t, Sx, 2)
    t = _axis(t, Sy, 1)
    u = _axis(t, Sz, 0)
    return to_element(u - u.mean(), hier.ne, n)


def residual_norm(x, b, hier):
    from .sipg import apply_A
    return float(np.linalg.norm(b - apply_A(x, hier.top.discs)))


def rate_metrics(hist, t_cycle=None):
    """rho = (r_n / r_0)^(1/n), n10 = ceil(-10 / lg rho),
    tau10 = -10 t_c / lg rho  (Sec. 4)."""
    n = len(hist) - 1
    if n < 1:
        return {"rho": 0.0, "n10": 0, "tau10": None}
    rho = (hist[-1] / hist[0]) ** (1.0 / n)
    lg = math.log10(rho) if rho > 0 else -math.inf
    n10 = math.ceil(-10.0 / lg) if lg < 0 else None
    tau = (-10.0 * t_cycle / lg) if (t_cycle is not None and lg < 0) else None
    return {"rho": rho, "neg_lg_rho": -lg, "n10": n10, "tau10": tau}
