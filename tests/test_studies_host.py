"""Host-side pieces of the convergence studies: the rate measures and the
study configurations (no device needed)."""

import math

import pytest

from paper_1612_04796_amd import studies


def test_rate_measures_closed_form():
    # r_n = r_0 * 10^(-2 n): rho = 1e-2, -lg rho = 2, n10 = 5
    hist = [3.0 * 10.0 ** (-2 * n) for n in range(6)]
    r = studies.rate(hist)
    assert r["cycles"] == 5
    assert math.isclose(r["rho"], 1e-2, rel_tol=1e-12)
    assert math.isclose(r["neg_lg_rho"], 2.0, rel_tol=1e-12)
    assert r["n10"] == 5
    # a divergent history has no n10
    assert studies.rate([1.0, 2.0, 4.0])["n10"] is None


def test_table1_meshes_are_the_papers():
    # (128 / P)^3 elements of order P on the unit cube
    for P in (4, 8, 16, 32):
        prm = studies.table1_params(P, "rel", 0.08)
        assert prm["ne"] == (128 // P,) * 3 and prm["P"] == P


@pytest.mark.parametrize("AR", [1, 3, 16, 48])
def test_aniso_domain(AR):
    # (0, 2 pi AR) x (0, 2 pi ceil(AR/2)) x (0, 2 pi) with 8^3 elements of order 16
    prm = studies.aniso_params(AR, "max_var")
    assert prm["ne"] == (8, 8, 8) and prm["P"] == 16
    assert prm["length"] == pytest.approx((2 * math.pi * AR, 2 * math.pi * math.ceil(AR / 2), 2 * math.pi))
    assert prm["overlap"] == "max" and prm["smooth_growth"] == 3
    assert studies.aniso_params(AR, "rel_fix")["smooth_growth"] == 1
