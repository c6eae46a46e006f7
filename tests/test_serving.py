"""Serving loop (continuous batching).  CPU part: request validation and
server creation without a device.  GPU part: a mix of heterogeneous requests
(different meshes, orders, aspect ratios) admitted by memory footprint and run
concurrently; every result must equal, bitwise, the same solve run alone
with sipg_pcg_solve (the kernels are deterministic), and must match the
exact discrete solution of the oracle."""

import numpy as np
import pytest

import oracle
from paper_1612_04796_amd import sipg
from paper_1612_04796_amd.workloads import fourier_modes


def test_server_rejects_invalid_requests():
    with pytest.raises(sipg.SipgError):
        sipg.Server(0, 4)
    with sipg.Server(1 << 30, 4) as srv:
        k, phi, amp = fourier_modes(0, 3)
        with pytest.raises(sipg.SipgError) as ei:
            srv.submit(k, phi, amp, ne=(2, 4, 4), P=4)
        assert ei.value.code == sipg.EINVAL
        with pytest.raises(sipg.SipgError):
            srv.submit(k, phi, amp, rtol=0.0, ne=(4, 4, 4), P=4)
        with pytest.raises(sipg.SipgError):
            srv.submit(k, phi, amp, ne=(4, 4, 4), P=20)


MIX = [
    dict(ne=(4, 4, 4), length=(1.0, 1.0, 1.0), P=2, overlap="max", omega=0.08),
    dict(ne=(6, 6, 6), length=(3.0, 1.0, 1.0), P=8, overlap="max", omega=0.08),
    dict(ne=(5, 5, 5), length=(1.0, 1.0, 1.0), P=4, overlap="max", omega=0.08),
    dict(ne=(4, 4, 4), length=(8.0, 1.0, 1.0), P=16, overlap="max", omega=0.08),
    dict(ne=(8, 8, 8), length=(2.0, 1.0, 1.0), P=4, overlap="max", omega=0.08),
    dict(ne=(3, 3, 3), length=(1.0, 1.0, 1.0), P=32, overlap="max", omega=0.08),
]


@pytest.mark.gpu
@pytest.mark.parametrize("bits", [32, 64])
def test_results_alone_equal_results_in_the_mix(bits):
    from _gpu import announce, host, rel, torch_cuda, zeros
    torch = torch_cuda()
    announce("serving mix", bits)
    alone = []
    for i, prm in enumerate(MIX):
        k, phi, amp = fourier_modes(100 + i, 3)
        with sipg.Solver(precond_bits=bits, **prm) as s:
            b = zeros(s.ndof())
            s.rhs_fourier(k, phi, amp, b)
            x = zeros(s.ndof())
            it, rr = s.pcg_solve(x, b, rtol=1e-10, maxit=100)
            alone.append((host(x), it, rr))
    with sipg.Server(64 << 30, max_active=4) as srv:
        ids = []
        for i, prm in enumerate(MIX):
            k, phi, amp = fourier_modes(100 + i, 3)
            ids.append(srv.submit(k, phi, amp, rtol=1e-10, maxit=100, precond_bits=bits, **prm))
        seen_active = 0
        for _ in range(100000):
            a, q, _c = srv.progress(wait_ms=50)
            seen_active = max(seen_active, a)
            if a == 0 and q == 0:
                break
        assert seen_active >= 2          # requests really ran together
        for i, rid in enumerate(ids):
            st = srv.status(rid)
            assert st["state"] == sipg.REQ_DONE, st
            assert st["t_submit"] <= st["t_admit"] <= st["t_done"]
            u = zeros(st["ndof"])
            srv.fetch(rid, u)
            xs, it, rr = alone[i]
            assert st["iters"] == it
            assert np.array_equal(host(u), xs), i
            assert st["relres"] <= 1e-10


@pytest.mark.gpu
def test_served_solution_matches_oracle():
    from _gpu import announce, host, rel, torch_cuda, zeros
    torch_cuda()
    announce("serving oracle")
    prm = dict(ne=(4, 4, 4), length=(4.0, 1.0, 1.0), P=8, overlap="max", omega=0.08)
    k, phi, amp = fourier_modes(7, 3)
    h = oracle.Hierarchy(prm["ne"], prm["length"], prm["P"], overlap="max", omega=0.08)
    b = oracle.fourier_rhs(k, phi, amp, h)
    with sipg.Server(8 << 30, max_active=2) as srv:
        rid = srv.submit(k, phi, amp, precond_bits=32, **prm)
        while True:
            a, q, _ = srv.progress(wait_ms=50)
            if a == 0 and q == 0:
                break
        st = srv.status(rid)
        assert st["state"] == sipg.REQ_DONE
        u = zeros(st["ndof"])
        srv.fetch(rid, u)
    x = host(u)
    assert rel(x, oracle.exact_solution(b, h)) <= 1e-8


@pytest.mark.gpu
def test_memory_budget_limits_admission():
    from _gpu import announce, torch_cuda
    torch_cuda()
    announce("serving budget")
    prm = dict(ne=(4, 4, 4), P=4, overlap="min")
    one = sipg.footprint(**prm) + 2 * 8000 * 8
    with sipg.Server(int(one * 1.5), max_active=8) as srv:
        ids = [srv.submit(*fourier_modes(i, 3), **prm) for i in range(3)]
        while True:
            a, q, _ = srv.progress(wait_ms=20)
            if a == 0 and q == 0:
                break
        st = [srv.status(r) for r in ids]
        assert all(x["state"] == sipg.REQ_DONE for x in st)
        # the budget holds one request at a time: active intervals are disjoint
        spans = sorted((x["t_admit"], x["t_done"]) for x in st)
        assert all(spans[i][1] <= spans[i + 1][0] for i in range(len(spans) - 1)), spans


# same order, same launch shape and size class: their flexible-CG iterations
# are batched into one operator launch when they are ready together
SAME_ORDER = [
    dict(ne=(6, 6, 6), length=(1.0, 1.0, 1.0), P=4, overlap="max", omega=0.08),
    dict(ne=(6, 5, 7), length=(2.0, 1.0, 1.0), P=4, overlap="max", omega=0.08),
    dict(ne=(7, 6, 6), length=(1.0, 1.0, 1.0), P=4, overlap="rel", omega=0.08),
    dict(ne=(5, 6, 6), length=(1.0, 3.0, 1.0), P=4, overlap="max", omega=0.08),
]


@pytest.mark.gpu
@pytest.mark.parametrize("bits", [32, 64])
def test_batched_operator_launches_keep_results(bits):
    """Same-order requests served with batched operator launches give, bitwise,
    the results of the same solves run alone, and the batching happened."""
    from _gpu import announce, host, zeros
    announce("serving batched", bits)
    alone = []
    for i, prm in enumerate(SAME_ORDER):
        k, phi, amp = fourier_modes(200 + i, 3)
        with sipg.Solver(precond_bits=bits, **prm) as s:
            b = zeros(s.ndof())
            s.rhs_fourier(k, phi, amp, b)
            x = zeros(s.ndof())
            it, rr = s.pcg_solve(x, b, rtol=1e-10, maxit=100)
            alone.append((host(x), it))
    for fuse in (1, 0):
        with sipg.Server(64 << 30, max_active=4) as srv:
            srv.set_option(0, fuse)
            ids = []
            for i, prm in enumerate(SAME_ORDER):
                k, phi, amp = fourier_modes(200 + i, 3)
                ids.append(srv.submit(k, phi, amp, rtol=1e-10, maxit=100, precond_bits=bits, **prm))
            for _ in range(100000):
                a, q, _c = srv.progress(wait_ms=50)
                if a == 0 and q == 0:
                    break
            launches, served = srv.stats()
            if fuse:
                assert launches >= 1 and served >= 2 * launches, (launches, served)
            else:
                assert launches == 0 and served == 0
            for i, rid in enumerate(ids):
                st = srv.status(rid)
                assert st["state"] == sipg.REQ_DONE, st
                u = zeros(st["ndof"])
                srv.fetch(rid, u)
                xs, it = alone[i]
                assert st["iters"] == it
                assert np.array_equal(host(u), xs), (fuse, i)


@pytest.mark.gpu
def test_mixed_precision_requests_batch_apart():
    """Same-order requests with FP64 and single-precision preconditioners in
    one server: the FP32 ones keep their search direction in FP32 (an
    operator reading FP32) and the FP64 ones in FP64, so only requests of
    one kind share a batched operator launch; every result equals, bitwise,
    the same solve run alone."""
    from _gpu import announce, host, zeros
    announce("serving mixed precisions")
    cases = [(prm, bits) for prm in SAME_ORDER for bits in (64, 32)]
    alone = []
    for i, (prm, bits) in enumerate(cases):
        k, phi, amp = fourier_modes(300 + i, 3)
        with sipg.Solver(precond_bits=bits, **prm) as s:
            b = zeros(s.ndof())
            s.rhs_fourier(k, phi, amp, b)
            x = zeros(s.ndof())
            it, rr = s.pcg_solve(x, b, rtol=1e-10, maxit=100)
            alone.append((host(x), it))
    with sipg.Server(64 << 30, max_active=8) as srv:
        srv.set_option(0, 1)
        ids = []
        for i, (prm, bits) in enumerate(cases):
            k, phi, amp = fourier_modes(300 + i, 3)
            ids.append(srv.submit(k, phi, amp, rtol=1e-10, maxit=100, precond_bits=bits, **prm))
        for _ in range(100000):
            a, q, _c = srv.progress(wait_ms=50)
            if a == 0 and q == 0:
                break
        launches, served = srv.stats()
        assert launches >= 1 and served >= 2 * launches, (launches, served)
        for i, rid in enumerate(ids):
            st = srv.status(rid)
            assert st["state"] == sipg.REQ_DONE, st
            u = zeros(st["ndof"])
            srv.fetch(rid, u)
            xs, it = alone[i]
            assert st["iters"] == it
            assert np.array_equal(host(u), xs), (i, cases[i][1])


# one preconditioner signature (order 4, the 8 % overlap on isotropic
# meshes: subdomains of 7^3 and 5^3 nodes on levels 2 and 1) and one size
# class: their V-cycles run as cohorts when they are ready together
SAME_SIGNATURE = [
    dict(ne=(6, 6, 6), length=(1.0, 1.0, 1.0), P=4, overlap="rel", omega=0.08),
    dict(ne=(5, 6, 7), length=(1.0, 1.2, 1.4), P=4, overlap="rel", omega=0.08),
    dict(ne=(7, 6, 5), length=(1.0, 1.0, 1.0), P=4, overlap="max", omega=0.08),
    dict(ne=(6, 5, 6), length=(1.0, 1.0, 1.0), P=4, overlap="rel", omega=0.08),
]


@pytest.mark.gpu
@pytest.mark.parametrize("bits", [32, 64])
def test_cohort_vcycles_keep_results(bits):
    """Requests of one preconditioner signature served with cohort V-cycles
    (every V-cycle step of the cohort in one segmented launch, the cycles
    captured in graphs), with the built-in or autotuned launch shapes, give
    bitwise the results of the same solves run alone with the same shapes, and
    the cohorts happened; with SIPG_SERVER_FUSE_SMOOTH = 0 none is formed."""
    from _gpu import announce, host, zeros
    announce("serving cohorts", bits)

    def alone_runs(tuned):
        # tuned: the shapes the process-wide cache holds for these meshes
        # (the server's autotuning put them there); the partial sums of the
        # flexible-CG dot products follow the operator's launch shape
        out = []
        for i, prm in enumerate(SAME_SIGNATURE):
            k, phi, amp = fourier_modes(300 + i, 3)
            with sipg.Solver(precond_bits=bits, **prm) as s:
                if tuned:
                    s.autotune(reps=3)
                b = zeros(s.ndof())
                s.rhs_fourier(k, phi, amp, b)
                x = zeros(s.ndof())
                it, rr = s.pcg_solve(x, b, rtol=1e-10, maxit=100)
                out.append((host(x), it))
        return out

    alone = alone_runs(False)
    for smooth, tune in ((1, 0), (0, 0), (1, 2)):
        with sipg.Server(64 << 30, max_active=4) as srv:
            srv.set_option(sipg.SERVER_FUSE_SMOOTH, smooth)
            srv.set_option(sipg.SERVER_TUNE, tune)
            ids = []
            for i, prm in enumerate(SAME_SIGNATURE):
                k, phi, amp = fourier_modes(300 + i, 3)
                ids.append(srv.submit(k, phi, amp, rtol=1e-10, maxit=100, precond_bits=bits, **prm))
            for _ in range(100000):
                a, q, _c = srv.progress(wait_ms=50)
                if a == 0 and q == 0:
                    break
            cycles, served = srv.smooth_stats()
            if smooth:
                assert cycles >= 1 and served >= 2 * cycles, (cycles, served)
            else:
                assert (cycles, served) == (0, 0)
            if tune == 2:
                alone = alone_runs(True)
            for i, rid in enumerate(ids):
                st = srv.status(rid)
                assert st["state"] == sipg.REQ_DONE, st
                u = zeros(st["ndof"])
                srv.fetch(rid, u)
                xs, it = alone[i]
                assert st["iters"] == it
                assert np.array_equal(host(u), xs), (smooth, tune, i)


def test_tuning_cache_round_trip(tmp_path):
    """The launch-shape cache as JSON: entries written by hand are merged and
    saved back; malformed files are refused."""
    path = tmp_path / "cache.json"
    path.write_text('{"sipg_tuning_cache": 1, "entries": [\n'
                    ' {"bits": 64, "n": 9, "mx": 13, "my": 13, "mz": 13, "elements": 1000, "mfma": 0, '
                    '"apply_epb": 2, "schwarz_spb": 3},\n'
                    ' {"bits": 32, "n": 8, "mx": 12, "my": 12, "mz": 12, "elements": 777, "mfma": 1, '
                    '"apply_epb": 4, "schwarz_spb": 0}]}\n')
    assert sipg.tuning_cache_load(str(path)) == 2
    out = tmp_path / "saved.json"
    sipg.tuning_cache_save(str(out))
    text = out.read_text()
    assert '"elements": 1000' in text and '"schwarz_spb": 3' in text and '"elements": 777' in text
    assert sipg.tuning_cache_load(str(out)) >= 2
    bad = tmp_path / "bad.json"
    bad.write_text('{"sipg_tuning_cache": 1, "entries": [{"bits": 64, "n": 9}]}')
    with pytest.raises(sipg.SipgError):
        sipg.tuning_cache_load(str(bad))
    bad.write_text('{"entries": []}')
    with pytest.raises(sipg.SipgError):
        sipg.tuning_cache_load(str(bad))
    with pytest.raises(sipg.SipgError):
        sipg.tuning_cache_load(str(tmp_path / "missing.json"))


def test_submit_rejects_a_request_larger_than_the_budget():
    # a request whose footprint exceeds the whole budget could never be
    # admitted and would block the FIFO: it is refused at submit
    prm = dict(ne=(8, 8, 8), P=8, overlap="min")
    need = sipg.footprint(**prm) + 2 * 8 ** 3 * 9 ** 3 * 8
    with sipg.Server(need - 1, 4) as srv:
        k, phi, amp = fourier_modes(0, 3)
        with pytest.raises(sipg.SipgError) as ei:
            srv.submit(k, phi, amp, **prm)
        assert ei.value.code == sipg.ENOMEM
    with sipg.Server(need, 4) as srv:
        srv.submit(*fourier_modes(0, 3), **prm)


@pytest.mark.gpu
def test_oversized_request_does_not_block_the_queue():
    from _gpu import announce, torch_cuda
    torch_cuda()
    announce("serving oversized")
    small = dict(ne=(4, 4, 4), P=4, overlap="min")
    budget = sipg.footprint(**small) + 2 * 8000 * 8
    with sipg.Server(budget, max_active=4) as srv:
        with pytest.raises(sipg.SipgError) as ei:
            srv.submit(*fourier_modes(1, 3), ne=(8, 8, 8), P=8, overlap="min")
        assert ei.value.code == sipg.ENOMEM
        rid = srv.submit(*fourier_modes(2, 3), **small)
        for _ in range(100000):
            a, q, _c = srv.progress(wait_ms=50)
            if a == 0 and q == 0:
                break
        assert srv.status(rid)["state"] == sipg.REQ_DONE


def test_server_options_validated():
    with sipg.Server(1 << 30, 4) as srv:
        assert srv.stats() == (0, 0)
        assert srv.smooth_stats() == (0, 0)
        srv.set_option(sipg.SERVER_FUSE_APPLY, 0)
        srv.set_option(sipg.SERVER_FUSE_SMOOTH, 0)
        for mode in (0, 1, 2):
            srv.set_option(sipg.SERVER_TUNE, mode)
        with pytest.raises(sipg.SipgError):
            srv.set_option(sipg.SERVER_TUNE, 3)
        with pytest.raises(sipg.SipgError):
            srv.set_option(5, 1)
