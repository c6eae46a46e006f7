"""Host logic of bench.py: the algorithmic work model behind the roofline
figures (no GPU)."""

import bench


class _Levels:
    """Level geometry of the 16^3, P = 8 workload with overlap 0.08 dx:
    orders 1, 2, 4, 8 with 0, 1, 1, 2 overlap layers."""
    L = 3

    def level_info(self, l):
        order = [1, 2, 4, 8][l]
        no = [0, 1, 1, 2][l]
        return {"order": order, "no": [no] * 3, "ndof": 4096 * (order + 1) ** 3}


def test_schwarz_flops_counts_six_contractions_and_a_scaling():
    # m = 13: three forward and three backward 13 x 13 contractions of 13^2
    # lines each (2 flops per multiply-add), plus one division per entry
    assert bench.schwarz_flops((13, 13, 13)) == 6 * 2 * 13 ** 4 + 13 ** 3
    assert bench.schwarz_flops((7, 9, 11)) == 4 * 693 * 27 + 693


def test_solve_roofline_top_level_terms():
    s = _Levels()
    r = bench.solve_roofline(s, 4096, 8, 2.5)
    # the top level alone, by hand: per cycle two residuals, two local
    # solves, two assemblies with u, one restriction and one prolongation
    N, Nc, E = 4096 * 729, 4096 * 125, 4096
    bw, pk = 8e12, 78.6e12
    t = lambda by, fl: max(by / bw, fl / pk)
    res = t(24 * N, (6 * 9 + 36) * N)
    fdm = t(8 * N + 8 * 2197 * E, bench.schwarz_flops((13, 13, 13)) * E)
    asm1 = t((2 + 2197 / 729) * 8 * N, 2197 * E)
    asm0 = t((1 + 2197 / 729) * 8 * N, 2197 * E)
    rst = t(16 * N + 8 * Nc, (6 * 9 + 36) * N + 2 * E * (729 * 5 + 81 * 25 + 9 * 125))
    pro = t(16 * N + 8 * Nc, 2 * E * (125 * 9 + 25 * 81 + 5 * 729))
    top = 8 * (2 * res + 2 * fdm + 2 * asm1 + rst + pro) + res - (asm1 - asm0)
    assert top < r["t_roofline_ms"] * 1e-3 < 1.5 * top   # the small levels add the rest
    assert r["frac"] == r["t_roofline_ms"] / 2.5
    # the local solves of the top level are bound by arithmetic, the residual by bytes
    assert fdm == bench.schwarz_flops((13, 13, 13)) * E / pk
    assert res == 24 * N / bw


def test_local_solve_roofline_work_per_launch():
    s = _Levels()
    # FP64: the plain sum-factorized flops of 4096 subdomains of 13^3 per
    # launch against the FP64 vector peak; 40 us per launch
    r = bench.local_solve_roofline(s, 0.040, 64)
    work = bench.schwarz_flops((13, 13, 13)) * 4096
    assert r["work_per_launch"] == work and r["unit"] == "TFLOP/s"
    assert abs(r["achieved"] - work / 40e-6 / 1e12) < 1e-9 and r["peak"] == 78.6
    assert abs(r["frac"] - r["achieved"] / 78.6) < 1e-12
    # FP32: the FP32 peak
    assert bench.local_solve_roofline(s, 0.040, 32)["peak"] == 157.3
    # FP16 matrix-core form: bytes of R_s r gathered and C stored (4 B each)
    r16 = bench.local_solve_roofline(s, 0.040, 16, mfma16=True)
    assert r16["bound"] == "hbm" and r16["work_per_launch"] == 8 * 2197 * 4096


def test_rate_of_history():
    r = bench.rate_of([1.0, 1e-2, 1e-4, 1e-6])
    assert abs(r["rho"] - 1e-2) < 1e-15 and r["n10"] == 5 and r["cycles"] == 3
    assert bench.rate_of([1.0])["n10"] is None
