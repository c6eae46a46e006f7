"""The GL (Gauss-Legendre) nodal basis on the GPU (Sec. 2; Table 1 rows
7-14): the operator with full face traces, the Schwarz step (including a
level with no overlap layers, N_O = 0), the transfers, the V-cycle and the
solvers, each against the oracle on the same inputs; order 32 exercises the
large-element operator passes."""

import numpy as np
import pytest

import oracle
from paper_1612_04796_amd import sipg
from paper_1612_04796_amd.workloads import fourier_modes, uniform_vector

from _gpu import announce, dev, host, rel, torch_cuda, zeros

pytestmark = pytest.mark.gpu

TOL_OP = 1e-12
TOL_FDM = 1e-11


def gl_pair(ne, length, P, overlap="min", omega=0.08, floor=0, precond_bits=64):
    torch_cuda()
    h = oracle.Hierarchy(ne, length, P, overlap=overlap, omega=omega, basis="gl", overlap_floor=floor)
    s = sipg.Solver(ne=ne, length=length, P=P, overlap=overlap, omega=omega, basis="gl", overlap_floor=floor,
                    precond_bits=precond_bits)
    return h, s


CASES = [
    # (ne, length, P, overlap, omega, floor)
    ((4, 4, 5), (1.0, 2.0, 1.0), 4, "rel", 0.08, 0),     # N_O = 0 on the P = 2 level
    ((4, 5, 4), (1.0, 1.0, 1.0), 8, "rel", 0.5, 0),      # the 0.5 dx tie, counted strictly
    ((5, 4, 4), (2.0, 1.0, 0.5), 7, "rel", 0.09, 1),     # N_O >= 1
    ((4, 4, 4), (1.0, 1.0, 1.0), 3, "min", 0.0, 0),
    ((4, 4, 4), (8.0, 1.0, 1.0), 16, "max", 0.08, 0),    # wide subdomains
]


@pytest.mark.parametrize("ne,length,P,overlap,omega,floor", CASES)
def test_gl_operator_schwarz_transfers(ne, length, P, overlap, omega, floor):
    announce("gl ops", ne, length, P, overlap, omega, floor)
    h, s = gl_pair(ne, length, P, overlap, omega, floor)
    for l in range(h.L + 1):
        n = h.ndof(l)
        u = uniform_vector(11 + l, n)
        f = uniform_vector(23 + l, n)
        y = zeros(n)
        s.apply_A(dev(u), y, level=l)
        ref = oracle.apply_level(u, h, l)
        assert rel(host(y), ref) <= TOL_OP, ("apply", l, rel(host(y), ref))
        r = zeros(n)
        s.residual(dev(u), dev(f), r, level=l)
        assert rel(host(r), f - ref) <= TOL_OP, ("residual", l)
        if l == 0:
            continue
        ud = dev(u)
        s.schwarz(dev(f), ud, level=l)
        sref = u + oracle.schwarz_step_correction(f, h, l)
        assert rel(host(ud), sref) <= TOL_FDM, ("schwarz", l, h.levels[l].no, rel(host(ud), sref))
        fc = zeros(h.ndof(l - 1))
        s.restrict(dev(f), fc, level=l)
        assert rel(host(fc), oracle.restrict(f, h, l)) <= TOL_OP, ("restrict", l)
        uc = uniform_vector(60 + l, h.ndof(l - 1))
        ud = dev(u)
        s.prolong_add(dev(uc), ud, level=l)
        assert rel(host(ud), u + oracle.prolong(uc, h, l)) <= TOL_OP, ("prolong", l)
    s.close()


@pytest.mark.parametrize("ne,length,P,overlap,omega,floor,solver", [
    ((4, 4, 4), (1.0, 1.0, 1.0), 4, "rel", 0.08, 0, "mg"),
    ((4, 4, 4), (1.0, 1.0, 1.0), 8, "rel", 0.09, 1, "fcg"),
    ((4, 5, 4), (2.0, 1.0, 1.0), 7, "min", 0.0, 0, "fcg"),
])
def test_gl_vcycle_and_solvers(ne, length, P, overlap, omega, floor, solver):
    announce("gl solve", ne, length, P, overlap, solver)
    h, s = gl_pair(ne, length, P, overlap, omega, floor)
    k, phi, amp = fourier_modes(3, 3)
    b = oracle.fourier_rhs(k, phi, amp, h)
    bd = zeros(h.ndof())
    s.rhs_fourier(k, phi, amp, bd)
    assert rel(host(bd), b) <= TOL_OP
    u = uniform_vector(5, h.ndof())
    ud = dev(u)
    s.vcycle(ud, dev(b))
    assert rel(host(ud), oracle.vcycle(u, b, h)) <= TOL_FDM
    x = zeros(h.ndof())
    if solver == "mg":
        it, rr = s.mg_solve(x, dev(b), rtol=1e-10, maxcyc=60)
        xo, ito, _, _ = oracle.mg_solve(b, h, tol=1e-10, maxcyc=60)
    else:
        it, rr = s.pcg_solve(x, dev(b), rtol=1e-10, maxit=60)
        xo, ito, _, _ = oracle.fcg_solve(b, h, tol=1e-10, maxit=60)
    assert it == ito and rr <= 1e-10
    assert rel(host(x), xo) <= 1e-10
    assert rel(host(x), oracle.exact_solution(b, h)) <= 1e-8
    s.close()


def test_gl_fp32_preconditioner():
    announce("gl fp32")
    h, s = gl_pair((4, 4, 4), (1.0, 1.0, 1.0), 8, "rel", 0.08, 0, precond_bits=32)
    k, phi, amp = fourier_modes(4, 3)
    f = oracle.fourier_rhs(k, phi, amp, h)
    z = zeros(h.ndof())
    s.precond(dev(f), z)
    assert rel(host(z), oracle.vcycle(np.zeros_like(f), f, h)) <= 1e-5
    x = zeros(h.ndof())
    it, rr = s.pcg_solve(x, dev(f), rtol=1e-10, maxit=60)
    assert rr <= 1e-10 and rel(host(x), oracle.exact_solution(f, h)) <= 1e-8
    s.close()


def test_gl_order32_large_elements():
    announce("gl order32")
    h, s = gl_pair((4, 4, 4), (1.0, 1.0, 1.0), 32, "rel", 0.08, 0)
    L = h.L
    n = h.ndof(L)
    u = uniform_vector(101, n)
    f = uniform_vector(102, n)
    y = zeros(n)
    s.apply_A(dev(u), y)
    ref = oracle.apply_level(u, h, L)
    assert rel(host(y), ref) <= TOL_OP
    ud = dev(u)
    s.schwarz(dev(f), ud, level=L)
    assert rel(host(ud), u + oracle.schwarz_step_correction(f, h, L)) <= TOL_FDM
    s.close()
