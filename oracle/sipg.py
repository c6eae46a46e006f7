"""SIPG discretization on a periodic Cartesian mesh (paper Sec. 2).

Test infrastructure only (see the package docstring).

Reading of the interior penalty form.  The printed form (eq. (ip)) swaps the
jump and average operators in the face integral and carries the wrong sign:
as printed it is symmetric but inconsistent.  The oracle uses the standard
symmetric interior penalty form that the paper cites for it (Arnold et al.):

    a(v, u) = int grad v . grad u
              - int_Gamma ( {grad v} . [[u]] + [[v]] . {grad u} )
              + int_Gamma mu [[v]] . [[u]]

with the quadrature rule of the nodal basis (GLL or GL, Sec. 2 and Table 1).
This yields the properties the paper states after eq. (A): M diagonal
positive, L symmetric positive semi-definite and block tridiagonal (block
cyclic on the periodic mesh).  For the GL basis the element traces and
normal derivatives at a face are combinations of all nodes of the element
line (the end points are not nodes), so the face coupling blocks are full.

Reading of the penalty.  The paper sets mu = 2 mu_min with
mu_min,x = P(P+1)/dx and calls mu_min the stability threshold; for the
standard form the threshold is P(P+1)/(2 dx), so the two statements differ by
a factor of two.  The oracle takes mu_d = c_mu P_l (P_l+1) / dx_d with
c_mu = 1 (twice the actual threshold) and the level's own order P_l.

Array layouts.  Element-major vectors have shape (E * n^3,) ordered
[ez][ey][ex][k][j][i] (x fastest inside and across elements).  Global
lexicographic arrays have shape (Nz, Ny, Nx) with N_d = ne_d * n and
index (ez*n + k, ey*n + j, ex*n + i).
"""

import numpy as np

from .basis import rule, diff_matrix, end_values, lagrange_eval


class Discretization1D:
    """1D mass and SIPG stiffness of one direction on the periodic mesh of
    ``ne`` equal elements of width h = length/ne, order p (eq. (A) factors),
    nodal basis 'gll' (the default) or 'gl'.

    Attributes: xi, w (the rule), D (derivative matrix), h, mu, n = p+1,
    N = ne*n, M (global diagonal, length N), L (global dense N x N).  The
    mass matrix is diagonal for both bases: the n-point rule integrates the
    products of two basis functions exactly for GL (degree 2p <= 2p + 1) and
    is the collocated (lumped) mass for GLL, as in the paper.
    """

    def __init__(self, p, ne, length, cmu=1.0, basis="gll"):
        if ne < 2:
            raise ValueError("need at least two elements per direction")
        self.p, self.ne, self.length, self.cmu = p, ne, float(length), float(cmu)
        self.basis = basis
        self.n = p + 1
        self.N = ne * self.n
        self.h = self.length / ne
        self.mu = self.cmu * p * (p + 1) / self.h
        self.xi, self.w = rule(basis, p)
        self.D = diff_matrix(self.xi)
        n, h = self.n, self.h
        # element mass (diagonal) and volume stiffness
        self.M_elem = 0.5 * h * self.w
        self.K_elem = (2.0 / h) * self.D.T @ np.diag(self.w) @ self.D
        M = np.tile(self.M_elem, ne)
        L = np.zeros((self.N, self.N))
        for e in range(ne):
            s = slice(e * n, (e + 1) * n)
            L[s, s] += self.K_elem
        # face between element e (minus side, xi=+1) and e+1 (plus side,
        # xi=-1); the traces are phi(+1) of e and phi(-1) of e+1 (unit
        # vectors for GLL, full vectors for GL)
        if basis == "gll":  # the end points are the first and last nodes
            phi_m, phi_p = np.eye(n)[0], np.eye(n)[n - 1]
            dphi_m, dphi_p = self.D[0, :], self.D[n - 1, :]
        else:
            phi_m, phi_p, dphi_m, dphi_p = end_values(self.xi)
        self.trace_m, self.trace_p, self.dtrace_m, self.dtrace_p = phi_m, phi_p, dphi_m, dphi_p
        jump = np.concatenate((phi_p, -phi_m))   # [[v]] = v^- - v^+ (normal of the minus side is +x)
        avg = np.concatenate((0.5 * (2.0 / h) * dphi_p,
                              0.5 * (2.0 / h) * dphi_m))   # {v'}
        F = -np.outer(avg, jump) - np.outer(jump, avg) + self.mu * np.outer(jump, jump)
        for e in range(ne):
            e1 = (e + 1) % ne
            idx = np.concatenate((np.arange(e * n, (e + 1) * n),
                                  np.arange(e1 * n, (e1 + 1) * n)))
            L[np.ix_(idx, idx)] += F
        self.M = M
        self.L = L


def to_global(u, ne, n):
    """Element-major vector -> global lexicographic (Nz, Ny, Nx) array."""
    nex, ney, nez = ne
    a = np.asarray(u).reshape(nez, ney, nex, n, n, n)
    return a.transpose(0, 3, 1, 4, 2, 5).reshape(nez * n, ney * n, nex * n)


def to_element(g, ne, n):
    """Global lexicographic (Nz, Ny, Nx) array -> element-major vector."""
    nex, ney, nez = ne
    a = np.asarray(g).reshape(nez, n, ney, n, nex, n)
    return np.ascontiguousarray(a.transpose(0, 2, 4, 1, 3, 5)).reshape(-1)


def _along(G, A, axis):
    """Apply the matrix A along one axis of the 3D array G."""
    return np.moveaxis(np.tensordot(A, G, axes=([1], [axis])), 0, axis)


def apply_A_global(G, dx, dy, dz):
    """eq. (A): (Mz x My x Lx + Mz x Ly x Mx + Lz x My x Mx) on a global array."""
    Mx, My, Mz = dx.M, dy.M, dz.M
    Y = (Mz[:, None, None] * My[None, :, None]) * _along(G, dx.L, 2)
    Y += (Mz[:, None, None] * Mx[None, None, :]) * _along(G, dy.L, 1)
    Y += (My[None, :, None] * Mx[None, None, :]) * _along(G, dz.L, 0)
    return Y


def apply_A(u, discs):
    """y = A u on element-major vectors; discs = (dx, dy, dz)."""
    dx, dy, dz = discs
    ne = (dx.ne, dy.ne, dz.ne)
    G = to_global(u, ne, dx.n)
    return to_element(apply_A_global(G, dx, dy, dz), ne, dx.n)


def assemble_ip_dense(ne, length, p, cmu=1.0, basis="gll"):
    """Dense 3D system matrix by direct quadrature (the basis' own rule) of the interior penalty
    form, element by element and face by face, in global lexicographic DOF
    numbering.  Independent of the Kronecker form: it evaluates the Lagrange
    polynomials by their product formula and never forms 1D L or M.  For small
    meshes only (N^2 storage)."""
    nex, ney, nez = ne
    h = [length[0] / nex, length[1] / ney, length[2] / nez]
    n = p + 1
    Nx, Ny, Nz = nex * n, ney * n, nez * n
    N = Nx * Ny * Nz
    xi, w = rule(basis, p)
    phi, dphi = lagrange_eval(xi, xi)            # at the quadrature points
    phib, dphib = lagrange_eval(xi, [-1.0, 1.0])  # at the element ends
    mu = [cmu * p * (p + 1) / h[d] for d in range(3)]
    A = np.zeros((N, N))

    def dofs(ex, ey, ez):
        i = np.arange(n)
        gx = (ex % nex) * n + i
        gy = (ey % ney) * n + i
        gz = (ez % nez) * n + i
        return (gz[:, None, None] * Ny + gy[None, :, None]) * Nx + gx[None, None, :]

    # basis function a = (k, j, i) of an element, flattened as k*n*n + j*n + i
    # volume term: gradients at the 3D quadrature points (s, r, q)
    W3 = (np.einsum('s,r,q->srq', w, w, w) * (h[0] * h[1] * h[2] / 8.0)).reshape(-1)
    gx_ = np.einsum('qi,rj,sk->srqkji', dphi, phi, phi).reshape(n ** 3, n ** 3) * (2 / h[0])
    gy_ = np.einsum('qi,rj,sk->srqkji', phi, dphi, phi).reshape(n ** 3, n ** 3) * (2 / h[1])
    gz_ = np.einsum('qi,rj,sk->srqkji', phi, phi, dphi).reshape(n ** 3, n ** 3) * (2 / h[2])
    Kvol = sum(g.T @ (W3[:, None] * g) for g in (gx_, gy_, gz_))
    for ez in range(nez):
        for ey in range(ney):
            for ex in range(nex):
                d = dofs(ex, ey, ez).reshape(-1)
                A[np.ix_(d, d)] += Kvol

    # face terms; for a face normal to direction d the minus element sits at
    # xi_d = +1 and the plus element at xi_d = -1.
    def face_arrays(d):
        # returns (trace, normal derivative) of every basis function of an element
        # at the face points for side s in {0: xi_d=-1, 1: xi_d=+1}; face points
        # are the tensor GLL points of the two tangential directions.
        out = []
        for s in (0, 1):
            vals = []
            ders = []
            for (tq, tr) in np.ndindex(n, n):
                # tangential point indices tq, tr map to the two other axes in order
                val = np.zeros((n, n, n))   # [k][j][i]
                der = np.zeros((n, n, n))
                for k in range(n):
                    for j in range(n):
                        for i in range(n):
                            idx = (i, j, k)
                            f = [0.0, 0.0, 0.0]
                            g = [0.0, 0.0, 0.0]
                            tang = [a for a in range(3) if a != d]
                            pt = {tang[0]: tq, tang[1]: tr}
                            for a in range(3):
                                if a == d:
                                    f[a] = phib[s, idx[a]]
                                    g[a] = dphib[s, idx[a]] * (2 / h[a])
                                else:
                                    f[a] = phi[pt[a], idx[a]]
                                    g[a] = f[a]
                            val[k, j, i] = f[0] * f[1] * f[2]
                            der[k, j, i] = g[0] * g[1] * g[2]
                vals.append(val.reshape(-1))
                ders.append(der.reshape(-1))
            out.append((np.array(vals), np.array(ders)))
        tang = [a for a in range(3) if a != d]
        Wf = np.array([w[tq] * w[tr] for (tq, tr) in np.ndindex(n, n)])
        Wf *= (h[tang[0]] / 2) * (h[tang[1]] / 2)
        return out, Wf

    for d in range(3):
        sides, Wf = face_arrays(d)
        val_m, der_m = sides[1]   # minus element: its xi_d = +1 side
        val_p, der_p = sides[0]   # plus element:  its xi_d = -1 side
        T = np.concatenate((val_m, -val_p), axis=1)          # jump along +e_d
        G = 0.5 * np.concatenate((der_m, der_p), axis=1)     # average normal derivative
        F = -(G.T @ (Wf[:, None] * T) + T.T @ (Wf[:, None] * G)) + mu[d] * (T.T @ (Wf[:, None] * T))
        for ez in range(nez):
            for ey in range(ney):
                for ex in range(nex):
                    e0 = [ex, ey, ez]
                    e1 = list(e0)
                    e1[d] += 1
                    dd = np.concatenate((dofs(*e0).reshape(-1), dofs(*e1).reshape(-1)))
                    A[np.ix_(dd, dd)] += F
    return A
