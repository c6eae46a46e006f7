"""Polynomial multigrid and Krylov acceleration (paper Sec. 3.2, Algorithm 1).

Test infrastructure only (see the package docstring).

Readings where the paper is silent or garbled:

* Level sequence.  The paper uses P_l = 2^l from 1 to P, which covers powers
  of two only.  For other P the oracle takes 1, 2, 4, ..., 2^k < P, P
  (for P = 7: 1, 2, 4, 7).  A_l is rediscretized at order P_l (not Galerkin).
* Transfers.  Prolongation is the embedded interpolation I_l (J x J x J per
  element with J[i, j] = phi^{l-1}_j(xi^l_i)); restriction is its transpose.
* Coarse solve.  u_0 = A_0^+ f_0 is the minimum Euclidean norm solution.  The
  right side is first projected onto the range of A_0, which is the Euclidean
  complement of the constants (the printed "null space" is read as the
  range), then solved by fast diagonalization with the global periodic 1D
  eigenpairs of level 0 (the single zero mode dropped), and the Euclidean mean
  of the result is removed.
* Smoother.  One step is r = f - A u followed by u += sum_s R_s^T W_s du_s.
* Inexact PCG.  The paper defers the algorithm to other work.  The oracle uses
  flexible CG with beta = z_new . (r_new - r_old) / (r_old . z_old) and one
  V-cycle started from zero as the preconditioner.  Convergence is declared
  when the recursively updated residual satisfies the tolerance and the
  recomputed residual b - A x confirms it.

Internally every level vector is a global lexicographic (Nz, Ny, Nx) array;
the public functions take and return element-major vectors.
"""

import numpy as np
import scipy.linalg

from .basis import interp_matrix
from .sipg import Discretization1D, apply_A_global, to_global, to_element, _along as _axis
from .schwarz import SubdomainTables, overlap_delta, overlap_layers, schwarz_correction


def level_orders(P):
    """1, 2, 4, ..., 2^k < P, P  (P_l = 2^l when P is a power of two)."""
    if P < 1:
        raise ValueError("P must be >= 1")
    orders = []
    q = 1
    while q < P:
        orders.append(q)
        q *= 2
    orders.append(P)
    return orders


class Level:
    def __init__(self, p, ne, length, cmu, overlap, omega, smoothed, basis="gll", overlap_floor=0):
        self.p = p
        self.n = p + 1
        self.discs = tuple(Discretization1D(p, ne[d], length[d], cmu, basis=basis) for d in range(3))
        h = tuple(length[d] / ne[d] for d in range(3))
        floor = overlap_floor if overlap != "min" else 0
        self.no = tuple(overlap_layers(self.discs[d].xi, overlap_delta(overlap, omega, h, d), basis, floor)
                        for d in range(3))
        if overlap == "min":  # one node layer from each neighbour, for either basis
            self.no = (1, 1, 1)
        self.tabs = None
        if smoothed:
            self.tabs = tuple(SubdomainTables(self.discs[d], self.no[d]) for d in range(3))

    def A(self, G):
        return apply_A_global(G, *self.discs)


class Hierarchy:
    """All levels of the p-multigrid method for one problem.

    ne, length: elements and domain length per direction (x, y, z)
    P: top order; cmu: penalty factor; overlap in {'min', 'rel', 'max'} with
    width omega; (ns_pre, ns_post) smoothing steps on the top level, scaled by
    growth^(L - l) on level l (growth = 3 gives the variable V-cycle of
    Table 2); basis 'gll' or 'gl' (Table 1); overlap_floor: lower bound of
    the overlap layers on every level (Table 1 rows 13-14 use 1).
    """

    def __init__(self, ne, length, P, cmu=1.0, overlap="min", omega=0.08,
                 ns_pre=1, ns_post=1, growth=1, basis="gll", overlap_floor=0):
        self.ne = tuple(int(v) for v in ne)
        self.length = tuple(float(v) for v in length)
        self.basis = basis
        self.orders = level_orders(P)
        self.L = len(self.orders) - 1
        self.levels = [Level(p, self.ne, self.length, cmu, overlap, omega, smoothed=(l > 0), basis=basis,
                             overlap_floor=overlap_floor)
                       for l, p in enumerate(self.orders)]
        self.ns1 = [ns_pre * growth ** (self.L - l) for l in range(self.L + 1)]
        self.ns2 = [ns_post * growth ** (self.L - l) for l in range(self.L + 1)]
        # interpolation from level l-1 to level l
        self.J = [None] + [interp_matrix(self.levels[l - 1].discs[0].xi, self.levels[l].discs[0].xi)
                           for l in range(1, self.L + 1)]
        # level-0 global eigenpairs for the coarse pseudo-inverse
        self.coarse = []
        for d in range(3):
            dd = self.levels[0].discs[d]
            lam, S = scipy.linalg.eigh(dd.L, np.diag(dd.M))
            self.coarse.append((lam, S))

    @property
    def top(self):
        return self.levels[self.L]

    def ndof(self, l=None):
        lev = self.levels[self.L if l is None else l]
        return int(np.prod(self.ne)) * lev.n ** 3

    # ---- transfers on global arrays -------------------------------------
    def _blockwise(self, G, J, nfrom, nto):
        nez, ney, nex = self.ne[2], self.ne[1], self.ne[0]
        a = G.reshape(nez, nfrom, ney, nfrom, nex, nfrom)
        a = np.einsum('zkyjxi,ai->zkyjxa', a, J)
        a = np.einsum('zkyjxa,bj->zkybxa', a, J)
        a = np.einsum('zkybxa,ck->zcybxa', a, J)
        return a.reshape(nez * nto, ney * nto, nex * nto)

    def prolong(self, l, Gc):
        """I_l: level l-1 -> level l."""
        return self._blockwise(Gc, self.J[l], self.levels[l - 1].n, self.levels[l].n)

    def restrict(self, l, Gf):
        """I_l^T: level l -> level l-1."""
        return self._blockwise(Gf, self.J[l].T, self.levels[l].n, self.levels[l - 1].n)


def coarse_solve_global(F, hier):
    """u_0 = A_0^+ f_0 (minimum Euclidean norm) by global fast diagonalization."""
    (lx, Sx), (ly, Sy), (lz, Sz) = hier.coarse
    f = F - F.mean()
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
    return u - u.mean()


def _smooth_global(l, G, F, ns, hier):
    lev = hier.levels[l]
    for _ in range(ns):
        R = F - lev.A(G)
        G = G + schwarz_correction(R, lev.tabs)
    return G


def _vcycle_global(U, F, hier):
    """Algorithm 1 on global arrays; U is the top-level start value."""
    L = hier.L
    u = [None] * (L + 1)
    f = [None] * (L + 1)
    u[L], f[L] = U, F
    for l in range(L, 0, -1):
        if l < L:
            u[l] = np.zeros_like(f[l])
        u[l] = _smooth_global(l, u[l], f[l], hier.ns1[l], hier)
        f[l - 1] = hier.restrict(l, f[l] - hier.levels[l].A(u[l]))
    u[0] = coarse_solve_global(f[0], hier)
    for l in range(1, L + 1):
        u[l] = u[l] + hier.prolong(l, u[l - 1])
        u[l] = _smooth_global(l, u[l], f[l], hier.ns2[l], hier)
    return u[L]


# ---- public element-major API -------------------------------------------
def _g(v, hier, l=None):
    return to_global(v, hier.ne, hier.levels[hier.L if l is None else l].n)


def _e(G, hier, l=None):
    return to_element(G, hier.ne, hier.levels[hier.L if l is None else l].n)


def apply_level(v, hier, l=None):
    l = hier.L if l is None else l
    return _e(hier.levels[l].A(_g(v, hier, l)), hier, l)


def smoother(u, f, hier, l=None, ns=1):
    l = hier.L if l is None else l
    return _e(_smooth_global(l, _g(u, hier, l), _g(f, hier, l), ns, hier), hier, l)


def schwarz_step_correction(r, hier, l=None):
    """sum_s R_s^T W_s A_ss^{-1} R_s r for an element-major residual."""
    l = hier.L if l is None else l
    return _e(schwarz_correction(_g(r, hier, l), hier.levels[l].tabs), hier, l)


def restrict(r, hier, l):
    return _e(hier.restrict(l, _g(r, hier, l)), hier, l - 1)


def prolong(uc, hier, l):
    return _e(hier.prolong(l, _g(uc, hier, l - 1)), hier, l)


def coarse_solve(f0, hier):
    return _e(coarse_solve_global(_g(f0, hier, 0), hier), hier, 0)


def vcycle(u, f, hier):
    """One V-cycle (Algorithm 1) from the top-level value u for the right side f."""
    return _e(_vcycle_global(_g(u, hier), _g(f, hier), hier), hier)


def _project(B):
    """b - mean(b): the Euclidean projection onto the range of the singular
    periodic operator (its null space is the constants, Sec. 3.2)."""
    return B - B.mean()


def mg_solve(b, hier, tol=1e-10, maxcyc=100, x0=None):
    """Repeated V-cycles until ||b - A x|| <= tol ||b - A x0|| for b projected
    onto the range of A.  Returns (x, cycles, relres, history of residual
    norms) with x of zero Euclidean mean (the minimum-norm solution, as the
    pseudo-inverse of Algorithm 1)."""
    B = _project(_g(b, hier))
    X = np.zeros_like(B) if x0 is None else _g(x0, hier)
    lev = hier.top
    hist = []
    r0 = None
    for c in range(maxcyc + 1):
        rn = float(np.linalg.norm(B - lev.A(X)))
        hist.append(rn)
        if r0 is None:
            r0 = rn
        if rn <= tol * r0 or c == maxcyc:
            return _e(X - X.mean(), hier), c, rn / r0, hist
        X = _vcycle_global(X, B, hier)


def fcg_solve(b, hier, tol=1e-10, maxit=200, x0=None):
    """Flexible (inexact preconditioned) CG with one V-cycle from zero as the
    preconditioner, for b projected onto the range of A.  Returns
    (x, iterations, relres, history); a converged x has zero Euclidean mean
    (the mean is removed before the recomputed residual confirms
    convergence)."""
    B = _project(_g(b, hier))
    X = np.zeros_like(B) if x0 is None else _g(x0, hier)
    lev = hier.top
    R = B - lev.A(X)
    r0 = float(np.linalg.norm(R))
    hist = [r0]
    if r0 == 0.0:
        return _e(X - X.mean(), hier), 0, 0.0, hist
    Z = _vcycle_global(np.zeros_like(B), R, hier)
    Pd = Z.copy()
    rz = float(np.vdot(R, Z))
    it = 0
    while it < maxit:
        Q = lev.A(Pd)
        alpha = rz / float(np.vdot(Pd, Q))
        X = X + alpha * Pd
        R = R - alpha * Q
        it += 1
        rn = float(np.linalg.norm(R))
        if rn <= tol * r0:
            X = X - X.mean()
            Rt = B - lev.A(X)
            rt = float(np.linalg.norm(Rt))
            if rt <= tol * r0:
                hist.append(rt)
                return _e(X, hier), it, rt / r0, hist
            R, rn = Rt, rt
        hist.append(rn)
        Z = _vcycle_global(np.zeros_like(B), R, hier)
        beta = -alpha * float(np.vdot(Z, Q)) / rz
        rz = float(np.vdot(R, Z))
        Pd = Z + beta * Pd
    return _e(X, hier), it, hist[-1] / r0, hist
