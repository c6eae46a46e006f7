"""CPU tests of the C ABI library: it loads and exports every declared entry
point, its host-side set-up tables (computed by independent C++ code) agree
with the oracle's, and invalid parameters are rejected with SIPG_EINVAL.
No device is needed: only host-only entry points are called."""

import os
import re

import numpy as np
import pytest

import oracle
from oracle.schwarz import overlap_delta, overlap_layers
from paper_1612_04796_amd import sipg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_header_symbol():
    header = open(os.path.join(ROOT, "include", "sipg_mg.h")).read()
    declared = set(re.findall(r"\b(sipg_[a-z_0-9A-Z]+)\s*\(", header))
    lib = sipg.lib()
    missing = [name for name in sorted(declared) if not hasattr(lib, name)]
    assert not missing, missing
    assert declared == set(sipg.EXPORTS), declared ^ set(sipg.EXPORTS)


CASES = [
    dict(ne=(4, 4, 4), length=(1.0, 1.0, 1.0), P=4, overlap="min"),
    dict(ne=(16, 16, 16), length=(1.0, 1.0, 1.0), P=8, overlap="rel", omega=0.08),
    dict(ne=(8, 8, 8), length=(16.0, 1.0, 1.0), P=16, overlap="max", omega=0.08),
    dict(ne=(5, 3, 4), length=(2.0, 1.0, 0.5), P=7, overlap="rel", omega=0.08),
    # the GL basis: full face traces, N_O = 0 on the P = 2 level (0.08 dx),
    # the 0.5 dx tie counted strictly, the N_O >= 1 floor, minimal overlap
    dict(ne=(4, 4, 4), length=(1.0, 1.0, 1.0), P=8, overlap="rel", omega=0.08, basis="gl"),
    dict(ne=(4, 4, 5), length=(2.0, 1.0, 0.5), P=4, overlap="rel", omega=0.5, basis="gl"),
    dict(ne=(4, 4, 4), length=(1.0, 1.0, 1.0), P=16, overlap="rel", omega=0.09, basis="gl", overlap_floor=1),
    dict(ne=(4, 4, 4), length=(1.0, 1.0, 1.0), P=4, overlap="min", basis="gl"),
    dict(ne=(4, 4, 4), length=(8.0, 1.0, 1.0), P=7, overlap="max", omega=0.08, basis="gl"),
]


def _hier(kw):
    return oracle.Hierarchy(kw["ne"], kw["length"], kw["P"], overlap=kw["overlap"],
                            omega=kw.get("omega", 0.08), basis=kw.get("basis", "gll"),
                            overlap_floor=kw.get("overlap_floor", 0))


def _t(level, d, which, kw):
    return np.array(sipg.host_table(level, d, which, **kw))


@pytest.mark.parametrize("kw", CASES)
def test_host_tables_match_oracle(kw):
    h = _hier(kw)
    for l, lev in enumerate(h.levels):
        for d in range(3):
            disc = lev.discs[d]
            n = disc.n
            assert np.allclose(_t(l, d, "nodes", kw), disc.xi, atol=1e-15)
            assert np.allclose(_t(l, d, "weights", kw), disc.w, atol=1e-14)
            assert np.allclose(_t(l, d, "deriv", kw).reshape(n, n), disc.D, atol=1e-10 * max(1, n * n))
            assert np.allclose(_t(l, d, "mass", kw), disc.M[:n], rtol=1e-14)
            scale = np.abs(disc.L).max()
            Ld = _t(l, d, "ldiag", kw).reshape(n, n)
            U = _t(l, d, "lupper", kw).reshape(n, n)
            assert np.abs(Ld - disc.L[:n, :n]).max() <= 1e-12 * scale
            assert np.abs(U - disc.L[:n, n:2 * n]).max() <= 1e-12 * scale
            if l == 0:
                continue
            tab = lev.tabs[d]
            assert int(_t(l, d, "overlap", kw)[0]) == tab.no
            m = tab.m
            assert np.abs(_t(l, d, "sub_l", kw).reshape(m, m) - tab.Ls).max() <= 1e-12 * scale
            assert np.allclose(_t(l, d, "sub_m", kw), tab.Ms, rtol=1e-14)
            lam = _t(l, d, "sub_lam", kw)
            assert np.allclose(lam, tab.lam, rtol=1e-11, atol=1e-12 * lam.max())
            S = _t(l, d, "sub_s", kw).reshape(m, m)
            # eigenvectors are defined up to sign: compare the inverse operator
            inv_c = S @ np.diag(1 / lam) @ S.T
            inv_o = tab.S @ np.diag(1 / tab.lam) @ tab.S.T
            assert np.abs(inv_c - inv_o).max() <= 1e-10 * np.abs(inv_o).max()
            assert np.allclose(S.T @ np.diag(tab.Ms) @ S, np.eye(m), atol=1e-11)
            assert np.allclose(_t(l, d, "sub_w", kw), tab.w, atol=1e-14)
            assert np.allclose(_t(l, d, "interp", kw).reshape(n, -1), h.J[l], atol=1e-13)
    # level-0 global eigenpairs: pseudo-inverse of the coarse 1D pair
    for d in range(3):
        lam_o, S_o = h.coarse[d]
        lam = _t(0, d, "coarse_lam", kw)
        N = len(lam)
        S = _t(0, d, "coarse_s", kw).reshape(N, N)
        z = np.argmin(np.abs(lam))
        assert lam[z] == 0.0
        keep = np.arange(N) != z
        pinv_c = S[:, keep] @ np.diag(1 / lam[keep]) @ S[:, keep].T
        zo = np.argmin(np.abs(lam_o))
        ko = np.arange(N) != zo
        pinv_o = S_o[:, ko] @ np.diag(1 / lam_o[ko]) @ S_o[:, ko].T
        assert np.abs(pinv_c - pinv_o).max() <= 1e-10 * np.abs(pinv_o).max()


@pytest.mark.parametrize("omega,mode", [(0.0, "min"), (0.08, "rel"), (0.5, "rel")])
def test_host_overlap_layers_match_table1(omega, mode):
    for P, expect_l in [(32, None), (16, None)]:
        kw = dict(ne=(4, 4, 4), length=(1.0, 1.0, 1.0), P=min(P, 16), overlap=mode, omega=omega)
        h = _hier(kw)
        for l in range(1, h.L + 1):
            got = int(_t(l, 0, "overlap", kw)[0])
            xi = h.levels[l].discs[0].xi
            assert got == overlap_layers(xi, overlap_delta(mode, omega, (0.25,) * 3, 0))


BAD = [
    dict(ne=(2, 4, 4)),                 # too few elements
    dict(P=0),                          # order below 1
    dict(P=17),                         # order above the compiled range
    dict(penalty=0.5),                  # at the stability threshold
    dict(length=(0.0, 1.0, 1.0)),       # empty domain
    dict(length=(float("nan"), 1.0, 1.0)),
    dict(overlap="rel", omega=1.5),     # overlap wider than the neighbour
    dict(nsmooth_pre=0, nsmooth_post=0),
    dict(precond_bits=8),
    dict(ne=(1025, 4, 4)),              # beyond the coarse solve's level-0 lines (ne_d <= 1024)
    dict(ne=(3, 3, 3), length=(16.0, 1.0, 1.0), overlap="max", omega=0.08, P=4),  # whole-neighbour overlap needs ne >= 4
    dict(basis=2),                      # unknown basis
    dict(basis="gl", ne=(4, 3, 4)),     # GL: at least 4 elements per direction
    dict(overlap="rel", overlap_floor=3),
]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_parameters_rejected(bad):
    kw = dict(ne=(4, 4, 4), length=(1.0, 1.0, 1.0), P=4)
    kw.update(bad)
    with pytest.raises(sipg.SipgError) as ei:
        sipg.footprint(**kw)
    assert ei.value.code == sipg.EINVAL
    assert sipg.lib().sipg_last_error().decode()


def test_footprint_scales_with_problem():
    small = sipg.footprint(ne=(4, 4, 4), P=4)
    big = sipg.footprint(ne=(16, 16, 16), P=8, overlap="rel")
    assert 0 < small < big
    # the 16^3 P=8 context holds at least the FCG vectors and the Schwarz scratch
    assert big > 4 * 2985984 * 8 + 4096 * 13 ** 3 * 8


def test_workload_generator_is_seeded():
    from paper_1612_04796_amd.workloads import fourier_modes, serving_stream
    a = fourier_modes(3, 8)
    b = fourier_modes(3, 8)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert a[0].min() >= 1 and a[0].max() <= 8
    s1 = serving_stream(1, 20, 5.0)
    s2 = serving_stream(1, 20, 5.0)
    assert s1 == s2
    assert all(4 <= r["ne"][0] <= 24 and r["P"] in (2, 4, 8, 16, 32) for r in s1)


def test_single_hip_runtime_in_process():
    """The library shares torch's HIP runtime (one libamdhip64 mapped)."""
    sipg.lib()
    with open("/proc/self/maps") as f:
        runtimes = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert len(runtimes) == 1, runtimes


@pytest.mark.parametrize("kw", [CASES[1], CASES[2], CASES[3]])
def test_host_even_odd_eigenpairs(kw):
    """The even-odd eigenpairs the compile-time-shape Schwarz kernel uses,
    against the oracle's restricted pair (L_s, M_s): the pair is
    reversal-symmetric, every column is exactly even (the first m - m/2) or
    odd, the generalized eigen-equation and M-orthonormality hold, and the
    inverse operator S diag(1/lam) S^T is the oracle's."""
    h = _hier(kw)
    for l in range(1, len(h.levels)):
        for d in range(3):
            tab = h.levels[l].tabs[d]
            m = tab.m
            Ls, Ms = tab.Ls, tab.Ms
            lam = _t(l, d, "sub_lam_eo", kw)
            S = _t(l, d, "sub_s_eo", kw).reshape(m, m)
            R = np.eye(m)[::-1]
            ne = m - m // 2
            scale = np.abs(Ls).max()
            assert np.abs(R @ Ls @ R - Ls).max() <= 1e-14 * scale
            assert np.allclose(Ms[::-1], Ms, rtol=1e-15)
            assert np.array_equal(R @ S[:, :ne], S[:, :ne])
            assert np.array_equal(R @ S[:, ne:], -S[:, ne:])
            assert np.abs(Ls @ S - (Ms[:, None] * S) * lam[None, :]).max() <= 1e-12 * scale
            assert np.abs(S.T @ (Ms[:, None] * S) - np.eye(m)).max() <= 1e-12
            inv_c = S @ np.diag(1 / lam) @ S.T
            inv_o = tab.S @ np.diag(1 / tab.lam) @ tab.S.T
            assert np.abs(inv_c - inv_o).max() <= 1e-10 * np.abs(inv_o).max()
