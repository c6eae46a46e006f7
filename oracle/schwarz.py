"""Weighted overlapping additive Schwarz smoother (paper Sec. 3.1).

Test infrastructure only (see the package docstring).

Each element e owns the element-centred subdomain made of its own n nodes per
direction plus N_O node layers taken from each face neighbour (Fig. 1).  The
local problem A_ss du_s = r_s (eq. (subproblem)) is solved by fast
diagonalization from the generalized eigenpairs of the restricted 1D pairs
(L_s, M_s), and the global correction is the weighted sum of eq.
(correction:global).

Readings where the paper is silent:

* N_O from a geometric overlap width delta_O: the number of neighbour nodes j
  whose distance from the shared face, (1 + xi_j)/2 in units of the element
  width, is at most delta_O / h for GLL nodes and below it for GL nodes
  (with a 1e-12 tolerance), optionally bounded below (Table 1 rows 13-14).
  This reproduces every N_O column of Table 1, GLL and GL rows.
* delta_O / h per direction: 0 for the minimal overlap (N_O = 1), omega for
  the relative overlap, and min(omega * max_k h_k, h_d) / h_d for the
  "max" overlap of Table 2.
* The weight function (its full definition is in a reference that is not
  reproduced in the paper; Fig. 2 shows a hat with a piecewise quintic
  transition): in the coordinate xi_H of Fig. 2 (xi - 2, xi, xi + 2 in the
  left neighbour, the core and the right neighbour),
      w(xi_H) = S5( clip((1 + delta - |xi_H|) / (2 delta), 0, 1) ),
      S5(t) = 10 t^3 - 15 t^4 + 6 t^5,
  with delta = min(1, 1 + xi_{N_O}) the reference distance from the face to
  the first neighbour node outside the subdomain (delta = 1 when the whole
  neighbour element is included).  Face nodes get 1/2 and the weights form a
  partition of unity.
* The weights are applied once, to the local correction, as in eq.
  (correction:global); there is no damping factor.
"""

import numpy as np
import scipy.linalg

OVERLAP_MODES = ("min", "rel", "max")


def overlap_delta(mode, omega, h, d):
    """delta_O / h_d for direction d; h = (hx, hy, hz)."""
    if mode == "min":
        return 0.0
    if mode == "rel":
        return float(omega)
    if mode == "max":
        return min(omega * max(h), h[d]) / h[d]
    raise ValueError(f"unknown overlap mode {mode!r}")


def overlap_layers(xi, delta_rel, basis="gll", floor=0):
    """N_O: neighbour nodes within delta_O of the shared face.  GLL counts
    the nodes at distance <= delta_O (a node exactly at the distance is
    included), GL those at distance < delta_O (excluded); both with a 1e-12
    tolerance.  Table 1 fixes the tie: at delta_O = 0.5 dx the middle node of
    an odd node count is counted for GLL (row 5: 2, 3, 5, 9, 17 layers for
    P = 2 .. 32) and not for GL (row 11: 1, 2, 4, 8, 16).  With the GL basis
    the count can be 0 (row 9 at P = 2); `floor` is the lower bound of rows
    13-14 (N_O >= 1)."""
    d = (1.0 + np.asarray(xi)) / 2.0
    if basis == "gll":
        no = int(np.count_nonzero(d <= delta_rel + 1e-12))
    else:
        no = int(np.count_nonzero(d < delta_rel - 1e-12))
    return max(no, int(floor))


def hat_weights(xi, no):
    """1D weights of the m = n + 2 N_O subdomain nodes (left halo, core,
    right halo).  N_O = 0 (possible with GL nodes) leaves the element alone,
    with weight 1 on every node."""
    n = len(xi)
    p = n - 1
    xi_h = np.concatenate((xi[n - no:] - 2.0, xi, xi[:no] + 2.0)) if no > 0 else np.asarray(xi, dtype=float)
    delta = min(1.0, 1.0 + xi[no]) if no <= p else 1.0
    t = np.clip((1.0 + delta - np.abs(xi_h)) / (2.0 * delta), 0.0, 1.0)
    return 10 * t ** 3 - 15 * t ** 4 + 6 * t ** 5


class SubdomainTables:
    """Restricted 1D pair (L_s, M_s) of one direction, its generalized
    eigenpairs L_s S = M_s S Lambda with S^T M_s S = I, and the 1D weights.

    ``index(e)`` gives the global 1D node indices of the subdomain of
    element e (periodic wrap)."""

    def __init__(self, disc, no):
        if not 0 <= no <= disc.n:
            raise ValueError("overlap layers must be in 0..n")
        self.disc, self.no = disc, no
        self.n = disc.n
        self.m = disc.n + 2 * no
        I0 = self.index(0)
        self.Ls = disc.L[np.ix_(I0, I0)]
        self.Ms = disc.M[I0]
        lam, S = scipy.linalg.eigh(self.Ls, np.diag(self.Ms))
        self.lam, self.S = lam, S
        self.w = hat_weights(disc.xi, no)

    def index(self, e):
        return (e * self.n - self.no + np.arange(self.m)) % self.disc.N


def _contract_last3(T, A, axis):
    """sum_a A[a, b] T[..., a, ...] along one of the last three axes (-3, -2, -1)."""
    return np.moveaxis(np.moveaxis(T, axis, -1) @ A, -1, axis)


def subdomain_solve(r_s, tabs):
    """Fast diagonalization solve of one subdomain problem A_ss du = r_s;
    r_s has shape (mz, my, mx); tabs = (tx, ty, tz)."""
    tx, ty, tz = tabs
    t = _contract_last3(r_s, tx.S, -1)
    t = _contract_last3(t, ty.S, -2)
    t = _contract_last3(t, tz.S, -3)
    t = t / (tz.lam[:, None, None] + ty.lam[None, :, None] + tx.lam[None, None, :])
    t = _contract_last3(t, tx.S.T, -1)
    t = _contract_last3(t, ty.S.T, -2)
    return _contract_last3(t, tz.S.T, -3)


def schwarz_correction(r_global, tabs):
    """du = sum_s R_s^T W_s A_ss^{-1} R_s r  for a global (Nz, Ny, Nx) residual.

    All subdomains are gathered at once (they are independent), solved by
    fast diagonalization, weighted, and summed back into the global array.
    """
    tx, ty, tz = tabs
    nex, ney, nez = tx.disc.ne, ty.disc.ne, tz.disc.ne
    Ix = np.stack([tx.index(e) for e in range(nex)])   # (nex, mx)
    Iy = np.stack([ty.index(e) for e in range(ney)])
    Iz = np.stack([tz.index(e) for e in range(nez)])
    Nx, Ny = tx.disc.N, ty.disc.N
    gz = Iz[:, None, None, :, None, None]
    gy = Iy[None, :, None, None, :, None]
    gx = Ix[None, None, :, None, None, :]
    R = r_global[gz, gy, gx]                             # (nez, ney, nex, mz, my, mx)
    du = subdomain_solve(R, tabs)
    du *= tz.w[:, None, None] * ty.w[None, :, None] * tx.w[None, None, :]
    flat = (gz * Ny + gy) * Nx + gx
    flat = np.broadcast_to(flat, du.shape)
    out = np.bincount(flat.reshape(-1), weights=du.reshape(-1),
                      minlength=r_global.size)
    return out.reshape(r_global.shape)
