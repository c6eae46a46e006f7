"""The autotuner (sipg_autotune): it picks a launch shape per level among
the valid candidates, leaves every computed value unchanged (the V-cycle
and the preconditioner are bitwise the same before and after tuning, as
each element and subdomain is computed the same way), keeps the solves
converging, and later contexts of the same shape reuse its choices."""

import numpy as np
import pytest

import oracle
from paper_1612_04796_amd import sipg
from paper_1612_04796_amd.workloads import fourier_modes, uniform_vector

from _gpu import announce, dev, host, pair, zeros

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ne,P,overlap,bits", [((6, 5, 4), 8, "rel", 64), ((5, 6, 4), 4, "min", 32),
                                               ((4, 4, 5), 7, "rel", 16)])
def test_autotune_keeps_results(ne, P, overlap, bits):
    announce("autotune", ne, P, overlap, bits)
    h, s = pair(ne, (1.0, 1.0, 1.0), P, overlap=overlap, precond_bits=bits)
    k, phi, amp = fourier_modes(1, 3)
    f = dev(oracle.fourier_rhs(k, phi, amp, h))
    u0 = dev(uniform_vector(4, h.ndof()))

    def outputs():
        u = u0.clone()
        s.vcycle(u, f)
        z = zeros(h.ndof())
        s.precond(f, z)
        return host(u), host(z)

    before = outputs()
    s.autotune(reps=3)
    after = outputs()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    tb = 64 if bits == 64 else 32
    for lv in range(1, h.L + 1):
        n = h.levels[lv].n
        epb, spb = s.tuning(lv, tb)
        full = max(1, 256 // (n * n))
        assert (epb == 0 and full == 1) or 1 <= epb <= full
        assert spb >= 0
    x = zeros(h.ndof())
    it, rr = s.mg_solve(x, f, 1e-10, 60)
    assert rr <= 1e-10
    # a second context of the same shape takes the cached choices
    s2 = sipg.Solver(ne=ne, length=(1.0, 1.0, 1.0), P=P, overlap=overlap, precond_bits=bits)
    s2.autotune(reps=3)
    for lv in range(1, h.L + 1):
        assert s2.tuning(lv, tb) == s.tuning(lv, tb)
    s2.close()
    s.close()


def test_kernel_trace_counts_launches_and_keeps_results():
    """SIPG_OPT_TRACE_KERNEL brackets each top-level FP64 launch of the chosen
    kernel with events: one V(1,1) cycle from a nonzero iterate launches the
    local solve, the assembly and the residual twice each on the top level and
    the restriction and prolongation once; the traced cycle computes the same
    values as an untraced one."""
    announce("kernel trace")
    h, s = pair((5, 4, 6), (1.0, 1.0, 1.0), 8, overlap="rel")
    k, phi, amp = fourier_modes(2, 3)
    f = dev(oracle.fourier_rhs(k, phi, amp, h))
    u0 = dev(uniform_vector(6, h.ndof()))
    ref = u0.clone()
    s.vcycle(ref, f)
    for name, launches in (("schwarz_solve", 2), ("schwarz_assemble", 2), ("residual", 2), ("restrict", 1),
                           ("prolong", 1)):
        s.trace_kernel(name)
        u = u0.clone()
        s.vcycle(u, f)
        ms, n = s.traced_kernel_ms()
        assert n == launches, (name, n)
        assert 0.0 < ms < 1e3
        assert np.array_equal(host(u), host(ref))
        assert s.traced_kernel_ms() == (0.0, 0)
    s.trace_kernel(None)
    s.vcycle(u0.clone(), f)
    assert s.traced_kernel_ms()[1] == 0
    with pytest.raises(sipg.SipgError):
        s.set_option(1, 7)


@pytest.mark.parametrize("ne,P,bits", [((3, 4, 5), 7, 64), ((5, 3, 4), 7, 32), ((4, 3, 5), 8, 64), ((3, 5, 4), 4, 32)])
def test_every_launch_shape_gives_the_same_values(ne, P, bits):
    """sipg_set_tuning: every accepted number of subdomains per local-solve
    workgroup (up to several per workgroup and a ragged last workgroup on
    these meshes) and of elements per operator workgroup computes the same
    preconditioner, bitwise, as the defaults; values beyond the limits are
    refused."""
    announce("set_tuning", ne, P, bits)
    h, s = pair(ne, (1.0, 1.0, 1.0), P, overlap="rel", precond_bits=bits)
    k, phi, amp = fourier_modes(3, 3)
    f = dev(oracle.fourier_rhs(k, phi, amp, h))
    tb = 64 if bits == 64 else 32

    def z_of():
        z = zeros(h.ndof())
        s.precond(f, z)
        return host(z)

    ref = z_of()
    limits = {lv: s.tuning_limits(lv, tb) for lv in range(1, h.L + 1)}
    most = max(ms for _, ms in limits.values())
    assert most >= 1
    for spb in range(1, most + 1):
        for lv, (me, ms) in limits.items():
            s.set_tuning(lv, tb, min(me, 1 + spb % max(me, 1)) if me else 0, min(spb, ms))
        assert np.array_equal(z_of(), ref), spb
    for lv, (me, ms) in limits.items():
        assert s.tuning(lv, tb)[1] == min(most, ms)
        with pytest.raises(sipg.SipgError):
            s.set_tuning(lv, tb, me + 1, 0)
        with pytest.raises(sipg.SipgError):
            s.set_tuning(lv, tb, 0, ms + 1)
    s.close()
