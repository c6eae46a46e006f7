#!/usr/bin/env python3
"""Benchmark of the p-multigrid solve: unknowns solved per second to a
relative residual of 1e-10, on one MI355X.

A step is one complete solve from x0 = 0 of a seeded synthetic problem (the
right-hand side already resident in HBM): every kernel of the hot path runs in
it (residuals, Schwarz local solves and assembly, restriction, coarse
pseudo-inverse, prolongation, norms).  Default workload: the periodic unit
cube with 16^3 elements at P = 8 (2,985,984 unknowns, the paper's own P = 8
mesh of its isotropic study), overlap delta_O = 0.08 dx, V(1,1) multigrid,
FP64.  Prints one JSON line on stdout; progress goes to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "unknowns solved/s to rel. residual 1e-10 (FP64 vs mixed); p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 157.3


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


PMC_SUMMARY = os.path.join(ROOT, "profiles", "schwarz_fdm_fixed_cube16_p8_pmc_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1612_04796_amd", "csrc", f)
                  for f in ("kernels_schwarz.hip", "device_common.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when that summary was taken on
    another version of the kernel's source."""
    try:
        with open(PMC_SUMMARY) as f:
            fields = dict(l.split(":", 1) for l in f.read().splitlines() if l.startswith(("source_sha256", "traffic_bytes")))
    except OSError:
        return None
    if fields.get("source_sha256", "").strip() != kernel_source_hash():
        return None
    return float(fields["traffic_bytes_per_launch"].strip())


def schwarz_flops(m):
    """Algorithmic flops of one subdomain's fast-diagonalization solve:
    three forward and three backward 1D contractions (2 flops per
    multiply-add) and one division per entry."""
    mx, my, mz = m
    vol = mx * my * mz
    return 4 * vol * (mx + my + mz) + vol


def solve_roofline(s, E, cycles, ms_measured):
    """Roofline time of a whole FP64 MG solve (x0 = 0, `cycles` V(1,1) cycles
    plus one residual norm per cycle and a final one): every launch priced at
    max(algorithmic bytes / HBM peak, algorithmic flops / FP64 peak), summed,
    and divided by the measured solve time.  Per level l >= 1 (n nodes per
    direction, N_l unknowns, subdomain volume V): residual 24 B and 6n + 36
    flop per unknown; residual + restriction 16 B per unknown plus 8 B per
    coarse unknown; prolongation the same bytes; local solves 8 B per
    unknown read plus 8 V B per subdomain written and 4 V (m_x + m_y + m_z)
    + V flop per subdomain; assembly (1 + V/n^3) or (2 + V/n^3) x 8 B per
    unknown (without or with the read of u).  Below the top level every
    pre-smoothing step starts from zero.  Level 0: three plane passes of
    16 B per unknown."""
    bw, pk = HBM_PEAK_GBS * 1e9, FP64_VALU_PEAK_TFLOPS * 1e12
    t = lambda by, fl: max(by / bw, fl / pk)
    total = 0.0
    L = s.L
    for l in range(L, 0, -1):
        n, m, N = level_geometry(s, l)
        Nc = s.level_info(l - 1)["ndof"]
        V = m[0] * m[1] * m[2]
        nc = s.level_info(l - 1)["order"] + 1
        res = t(24 * N, (6 * n + 36) * N)
        rst = t(16 * N + 8 * Nc, (6 * n + 36) * N + 2 * E * (n ** 3 * nc + n ** 2 * nc ** 2 + n * nc ** 3))
        pro = t(16 * N + 8 * Nc, 2 * E * (nc ** 3 * n + nc ** 2 * n ** 2 + nc * n ** 3))
        fdm = t(8 * N + 8 * V * E, schwarz_flops(m) * E)
        asm0 = t((1 + V / n ** 3) * 8 * N, V * E)
        asm1 = t((2 + V / n ** 3) * 8 * N, V * E)
        if l == L:  # check residual + both smoothing steps on a nonzero iterate (the first pre-step excepted)
            per = res + fdm + asm1 + rst + pro + res + fdm + asm1
            total += cycles * per + res - (asm1 - asm0)
        else:
            total += cycles * (fdm + asm0 + rst + pro + res + fdm + asm1)
    N0 = s.level_info(0)["ndof"]
    total += cycles * 3 * t(16 * N0, 0)
    return {"t_roofline_ms": 1e3 * total, "t_measured_ms": ms_measured, "frac": 1e3 * total / ms_measured,
            "model": "sum over all launches of max(bytes / 8 TB/s, flop / 78.6 TFLOP/s)"}


def level_geometry(s, l):
    info = s.level_info(l)
    n = info["order"] + 1
    m = tuple(n + 2 * no for no in info["no"])
    return n, m, info["ndof"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        return 1


def oracle_cycle_time(wl, k, phi, amp, nsample):
    """Seconds per V-cycle (with its residual norm) of the FP64 oracle on the
    host for workload wl, from `nsample` cycles of the solve from x0 = 0
    (for a flexible-CG workload the iteration costs one such V-cycle plus an
    operator application, both timed), and the residual norms seen."""
    import numpy as np
    import oracle
    from oracle.multigrid import _vcycle_global
    from oracle.sipg import to_global
    h = oracle.Hierarchy(wl.ne, wl.length, wl.P, overlap=wl.overlap, omega=wl.omega, growth=wl.growth)
    b = oracle.fourier_rhs(k, phi, amp, h)
    B = to_global(b, h.ne, h.top.n)
    X = np.zeros_like(B)
    lev = h.top
    hist = []
    t0 = time.perf_counter()
    for _ in range(nsample):
        hist.append(float(np.linalg.norm(B - lev.A(X))))
        X = _vcycle_global(X, B, h)
        if wl.solver != "mg":
            lev.A(X)  # the flexible CG's operator application q = A p
    t_c = (time.perf_counter() - t0) / nsample
    return t_c, hist


def cpu_baseline(wl, cycles, k, phi, amp, nsample=5):
    """The FP64 oracle on the host: time a sample of V-cycles plus their
    residual norms of the same solve, scale to the solve's cycle count."""
    blas = blas_threads()
    t_pair, _ = oracle_cycle_time(wl, k, phi, amp, nsample)
    t_solve = cycles * t_pair + t_pair / 4  # the final residual norm (about a quarter of a cycle)
    return {
        "value": wl.ndof / t_solve,
        "unit": "unknowns/s",
        "cores": int(blas),
        "kind": "oracle",
        "sample": (f"{nsample} V-cycles (each with its residual norm) of the same {wl.name} solve in the "
                   f"FP64 NumPy oracle on {cpu_model()} "
                   f"({os.cpu_count()} logical CPUs, BLAS threads {blas}, elementwise work single-threaded), "
                   f"scaled to the solve's {cycles} cycles: {t_pair:.2f} s per cycle"),
    }


def cpu_per_config(gpu_rates, nsample):
    """The CPU side of every workload: the oracle's seconds per cycle
    t_c on the host (a bounded sample), with the rate rho and cycles n10 of
    the same algorithm (taken from the GPU solve of the workload, which
    matches the oracle's iteration by iteration), tau10 = -10 t_c / lg rho
    (Sec. 4), the solve time to 1e-10 and unknowns/s."""
    from paper_1612_04796_amd.workloads import WORKLOADS, fourier_modes
    out = {"cpu": cpu_model(), "logical_cpus": os.cpu_count(), "blas_threads": blas_threads()}
    for name, rate in gpu_rates.items():
        wl = WORKLOADS[name]
        k, phi, amp = fourier_modes(0, wl.kmax)
        t_c, _ = oracle_cycle_time(wl, k, phi, amp, nsample.get(name, 1))
        nlg = rate["neg_lg_rho"]
        out[name] = {"t_c_s": t_c, "rho": rate["rho"], "n10": rate["n10"], "cycles_to_1e-10": rate["cycles"],
                     "tau10_us_per_unknown": 1e6 * 10.0 * t_c / nlg / wl.ndof if nlg > 0 else None,
                     "solve_s": rate["cycles"] * t_c, "unknowns_per_s": wl.ndof / (rate["cycles"] * t_c),
                     "sample_cycles": nsample.get(name, 1)}
        log(f"cpu {name}: {t_c:.3f} s per cycle, {out[name]['unknowns_per_s']:.3g} unknowns/s")
    return out


def rate_of(hist):
    import math
    n = len(hist) - 1
    rho = (hist[-1] / hist[0]) ** (1.0 / n) if n >= 1 and hist[0] > 0 else 0.0
    nlg = -math.log10(rho) if rho > 0 else math.inf
    return {"rho": rho, "neg_lg_rho": nlg, "n10": math.ceil(10.0 / nlg) if 0 < nlg < math.inf else None,
            "cycles": n}


def local_solve_roofline(s, ms, bits, mfma16=False):
    """Roofline of the top-level local-solve kernel from its mean launch
    duration `ms`: algorithmic flops (plain sum factorization) against the
    FP64 or FP32 peak, or, for the FP16 matrix-core form (bound by its
    gather and stores), algorithmic bytes (R_s r gathered and the
    corrections stored, 4 B each) against HBM."""
    n, m, N = level_geometry(s, s.L)
    E = N // n ** 3
    V = m[0] * m[1] * m[2]
    if mfma16:
        work = 8 * V * E
        achieved = work / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "work_per_launch": work, "ms_per_launch": ms,
                "subdomain": list(m)}
    work = schwarz_flops(m) * E
    peak = FP64_VALU_PEAK_TFLOPS if bits == 64 else FP32_VALU_PEAK_TFLOPS
    achieved = work / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "work_per_launch": work, "ms_per_launch": ms,
            "subdomain": list(m)}


def fcg_timing(wl, bits, b, steps, warmup, keep=None, autotune=True, trace=True):
    """Flexible CG from x0 = 0 to 1e-10 on workload wl with the given
    preconditioner precision (16: FP32 with FP16 matrix-core local solves):
    mean wall time over `steps` solves; keep[bits] receives the solution.
    With trace, every top-level local-solve launch of the last timed solve
    is bracketed by HIP events (in the preconditioner's precision) and the
    kernel's roofline is reported."""
    import torch
    from paper_1612_04796_amd import sipg
    s = sipg.Solver(ne=wl.ne, length=wl.length, P=wl.P, overlap=wl.overlap, omega=wl.omega,
                    smooth_growth=wl.growth, precond_bits=bits)
    if autotune:
        s.autotune()
    x = torch.zeros_like(b)
    for _ in range(max(1, warmup)):
        x.zero_()
        s.pcg_solve(x, b, 1e-10, 200)
    if trace:
        s.trace_kernel("schwarz_solve")
        s.trace_kernel(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if trace and i == steps - 1:
            s.trace_kernel("schwarz_solve")
        x.zero_()
        it, rr = s.pcg_solve(x, b, 1e-10, 200)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"unknowns_per_s": wl.ndof * steps / el, "ms_per_solve": 1e3 * el / steps,
           "iterations": it, "final_relres": rr, "rate": rate_of(s.residual_history())}
    if trace:
        ms, cnt = s.traced_kernel_ms()
        s.trace_kernel(None)
        if cnt:
            roof = local_solve_roofline(s, ms, bits, mfma16=(bits == 16 and wl.P in (7, 8)))
            roof["launches_timed"] = cnt
            out["local_solve_roofline"] = roof
    s.close()
    if keep is not None:
        keep[bits] = x
    log(f"FCG {wl.name}, FP{bits} preconditioner: {1e3 * el / steps:.3f} ms/solve, {it} iterations")
    return out


def mg_timing(wl, b, steps, warmup):
    """V(1,1) multigrid solve from x0 = 0 to 1e-10 (FP64): mean wall time."""
    import torch
    from paper_1612_04796_amd import sipg
    s = sipg.Solver(ne=wl.ne, length=wl.length, P=wl.P, overlap=wl.overlap, omega=wl.omega,
                    smooth_growth=wl.growth)
    x = torch.zeros_like(b)
    for _ in range(max(1, warmup)):
        x.zero_()
        s.mg_solve(x, b, 1e-10, 200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        it, rr = s.mg_solve(x, b, 1e-10, 200)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"unknowns_per_s": wl.ndof * steps / el, "ms_per_solve": 1e3 * el / steps, "cycles": it,
           "final_relres": rr, "rate": rate_of(s.residual_history())}
    s.close()
    log(f"MG {wl.name}: {out['ms_per_solve']:.3f} ms/solve, {it} cycles")
    return out


def workload_rhs(wl):
    import torch
    from paper_1612_04796_amd import sipg
    from paper_1612_04796_amd.workloads import fourier_modes
    s = sipg.Solver(ne=wl.ne, length=wl.length, P=wl.P, overlap=wl.overlap, omega=wl.omega,
                    smooth_growth=wl.growth)
    b = torch.zeros(s.ndof(), dtype=torch.float64, device="cuda")
    k, phi, amp = fourier_modes(0, wl.kmax)
    s.rhs_fourier(k, phi, amp, b)
    s.close()
    return b, (k, phi, amp)


def _replay(reqs, arrivals, submit, budget, options):
    """Replays a request stream in real time into a server with 8 slots and
    the given options; latency = finish - arrival."""
    import numpy as np
    from paper_1612_04796_amd import sipg

    nreq = len(reqs)
    lat, ndof, iters = [], [], []
    with sipg.Server(budget, max_active=8) as srv:
        for opt, val in options.items():
            srv.set_option(opt, val)
        t0 = time.perf_counter()
        ids = [None] * nreq
        sub_wall = [0.0] * nreq
        nxt = 0
        finished = 0
        while finished < nreq:
            now = time.perf_counter() - t0
            while nxt < nreq and arrivals[nxt] <= now:
                ids[nxt] = submit(srv, reqs[nxt])
                sub_wall[nxt] = time.perf_counter() - t0
                nxt += 1
            wait = 1 if nxt < nreq else 50
            srv.progress(wait_ms=wait)
            finished = sum(1 for i in range(nxt) if srv.status(ids[i])["state"] in (sipg.REQ_DONE, sipg.REQ_FAILED))
        t_end = time.perf_counter() - t0
        fused_launches, fused_requests = srv.stats()
        cohort_cycles, cohort_requests = srv.smooth_stats()
        for i, rid in enumerate(ids):
            st = srv.status(rid)
            if st["state"] != sipg.REQ_DONE or st["relres"] > 1e-10:
                raise RuntimeError(f"request {i} did not converge: {st}")
            # server clock: submit -> done, plus the wait between arrival and submit
            lat.append(st["t_done"] - st["t_submit"] + (sub_wall[i] - arrivals[i]))
            ndof.append(st["ndof"])
            iters.append(st["iters"])
    lat = np.array(lat)
    return {
        "p50_latency_ms": float(1e3 * np.percentile(lat, 50)),
        "p99_latency_ms": float(1e3 * np.percentile(lat, 99)),
        "max_latency_ms": float(1e3 * lat.max()),
        "unknowns_per_s": float(sum(ndof) / t_end),
        "makespan_s": t_end,
        "total_unknowns": int(sum(ndof)),
        "iterations": iters,
        "batched_operator_launches": fused_launches,
        "requests_in_batched_launches": fused_requests,
        "cohort_vcycles": cohort_cycles,
        "requests_in_cohort_vcycles": cohort_requests,
    }


def serving_run(nreq, seed, stream="mixed", variants=None, burst=False):
    """Serving stream, FP32-preconditioned FP64 flexible CG to 1e-10.
    stream "mixed": heterogeneous requests (4^3..24^3 elements, P in
    {2,4,8,16,32}, aspect ratio 1..8, "max" overlap); "same_order": small
    order-8 requests (4..7 elements per direction, 8 % overlap) that all share
    one preconditioner signature.  Poisson arrivals at the rate that gives
    about 70 % utilisation: the mean service time is measured first by serving
    the same requests one at a time; then the stream is replayed in real time
    into a server with 8 slots, once per variant (name -> server options), at
    the same arrival times; with burst, also with every request submitted at
    once (the makespan then measures the saturated throughput)."""
    import numpy as np
    import torch
    from paper_1612_04796_amd import sipg
    from paper_1612_04796_amd.workloads import fourier_modes, serving_stream, serving_stream_same_order

    free, _total = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    if stream == "mixed":
        reqs = serving_stream(seed, nreq, 1.0)
        common = dict(overlap="max", omega=0.08, precond_bits=32)
    else:
        reqs = serving_stream_same_order(seed, nreq, 1.0)
        common = dict(overlap="rel", omega=0.08, precond_bits=32)
    variants = variants or {"default": {}}

    def submit(srv, r):
        k, phi, amp = fourier_modes(r["rhs_seed"], 3)
        return srv.submit(k, phi, amp, rtol=1e-10, maxit=200, ne=r["ne"], length=r["length"], P=r["P"], **common)

    # calibration: one request at a time
    service = []
    with sipg.Server(budget, max_active=1) as srv:
        ids = [submit(srv, r) for r in reqs]
        while True:
            a, q, _ = srv.progress(wait_ms=100)
            if a == 0 and q == 0:
                break
        for rid in ids:
            st = srv.status(rid)
            if st["state"] != sipg.REQ_DONE:
                raise RuntimeError(f"request failed: {st}")
            service.append(st["t_done"] - st["t_admit"])
    mean_s = float(np.mean(service))
    qps = 0.7 / mean_s
    # arrival times: the stream's exponential gaps rescaled to this rate
    arrivals = [r["t_arrival"] / qps for r in reqs]
    log(f"serving ({stream}): {nreq} requests, mean service {1e3 * mean_s:.2f} ms alone, replay at {qps:.1f} req/s")
    out = {
        "stream": stream,
        "requests": nreq,
        "qps": qps,
        "utilisation_target": 0.7,
        "mean_service_alone_ms": 1e3 * mean_s,
        "precision": "FP32 preconditioner, FP64 flexible CG",
    }
    for name, options in variants.items():
        res = _replay(reqs, arrivals, submit, budget, options)
        log(f"serving ({stream}, {name}): p50 {res['p50_latency_ms']:.2f} ms, p99 {res['p99_latency_ms']:.2f} ms, "
            f"{res['unknowns_per_s']:.4g} unknowns/s, {res['cohort_vcycles']} cohort V-cycles")
        if burst:
            # every request at once: the server's throughput when saturated
            res["burst"] = _replay(reqs, [0.0] * nreq, submit, budget, options)
            bu = res["burst"]
            log(f"serving ({stream}, {name}, all at once): makespan {1e3 * bu['makespan_s']:.2f} ms, "
                f"{bu['unknowns_per_s']:.4g} unknowns/s, {bu['cohort_vcycles']} cohort V-cycles")
        if len(variants) == 1:
            out.update(res)
        else:
            out[name] = res
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube16_p8_rel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 32^3, P=7 mixed-precision solves")
    ap.add_argument("--no-scale", action="store_true", help="skip the 64^3, P=7 (134M unknowns) solves")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 4^3 P=4 and the anisotropic 8^3 P=16 workloads")
    ap.add_argument("--reps", type=int, default=20, help="launches per kernel timing")
    ap.add_argument("--serving-requests", type=int, default=24,
                    help="requests of the serving stream run after the main measurement (0 = skip)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes (no sipg_autotune before the timed runs)")
    ap.add_argument("--fcg-only", type=int, default=0, metavar="BITS",
                    help="profiling run: only the flexible-CG timing of --workload with this "
                         "preconditioner precision (64, 32 or 16); prints its JSON and exits")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this solver's build runs on a single MI355X "
              "(the multi-GPU decomposition is described, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    from paper_1612_04796_amd import sipg
    from paper_1612_04796_amd.workloads import WORKLOADS, fourier_modes

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    wl = WORKLOADS[args.workload]
    if args.fcg_only:
        b, _ = workload_rhs(wl)
        print(json.dumps({"workload": wl.name, "precond_bits": args.fcg_only,
                          **fcg_timing(wl, args.fcg_only, b, args.steps, args.warmup,
                                       autotune=not args.no_autotune)}))
        return
    log(f"workload {wl.name}: ne={wl.ne} P={wl.P} overlap={wl.overlap} N={wl.ndof}")
    s = sipg.Solver(ne=wl.ne, length=wl.length, P=wl.P, overlap=wl.overlap, omega=wl.omega,
                    smooth_growth=wl.growth)
    if not args.no_autotune:
        s.autotune()
    tuning = {f"level{l}": list(s.tuning(l, 64)) for l in range(1, s.L + 1)}
    log(f"launch shapes (elements / subdomains per workgroup, 0 = default): {tuning}")
    N = s.ndof()
    k, phi, amp = fourier_modes(0, wl.kmax)
    b = torch.zeros(N, dtype=torch.float64, device="cuda")
    s.rhs_fourier(k, phi, amp, b)
    x = torch.zeros_like(b)
    solve = s.mg_solve if wl.solver == "mg" else s.pcg_solve

    def step():
        x.zero_()
        return solve(x, b, 1e-10, 200)

    for i in range(args.warmup):
        it, rr = step()
        log(f"warmup {i}: {it} iterations, rel. residual {rr:.2e}")
    # every top-level launch of the local-solve kernel inside the last timed
    # solve is bracketed by HIP events on the library's stream (each event
    # record costs a few microseconds, so the other solves run without them);
    # the events are created here, before the timed region
    s.trace_kernel("schwarz_solve")
    s.trace_kernel(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for i in range(args.steps):
        if i == args.steps - 1:
            s.trace_kernel("schwarz_solve")
        it, rr = step()
        iters.append(it)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    traced_ms, traced_n = s.traced_kernel_ms()
    s.trace_kernel(None)
    main_rate = rate_of(s.residual_history())
    log(f"local-solve kernel in the timed solves: {traced_n} launches, {1e3 * traced_ms:.2f} us mean")
    ms = 1e3 * elapsed / args.steps
    value = N * args.steps / elapsed
    log(f"timed {args.steps} solves: {ms:.3f} ms/solve, {value:.4g} unknowns/s, iterations {iters}, "
        f"rel. residual {rr:.2e}")

    # ---- per-kernel timings on the top level (HIP events on the library stream)
    L = s.L
    n, m, _ = level_geometry(s, L)
    E = wl.ne[0] * wl.ne[1] * wl.ne[2]
    kern = {}
    for name in ("residual", "schwarz_solve", "schwarz_assemble", "restrict", "prolong"):
        kern[name] = s.time_kernel(name, level=L, bits=64, reps=args.reps)
    cyc = iters[-1]
    # launches per solve of the top-level kernels (MG: the residual of each
    # convergence check feeds the first pre-smoothing step)
    per_solve = {"residual": 2 * cyc + 1, "schwarz_solve": 2 * cyc, "schwarz_assemble": 2 * cyc,
                 "restrict": cyc, "prolong": cyc}
    if wl.solver != "mg":
        per_solve = {"residual": 2 * cyc + 1, "schwarz_solve": 2 * cyc + 2,
                     "schwarz_assemble": 2 * cyc + 2, "restrict": cyc + 1, "prolong": cyc + 1}
    share = {kname: kern[kname] * per_solve[kname] for kname in kern}
    dominant = max(share, key=share.get)
    log("top-level kernel ms/launch: " + ", ".join(f"{kk}={vv:.4f}" for kk, vv in kern.items())
        + f"; dominant {dominant}")
    if dominant == "schwarz_solve":
        roof = local_solve_roofline(s, traced_ms, 64)
        roof.update({
            "traffic": pmc_traffic() if (n, m) == (9, (13, 13, 13)) else None,
            # a tuned subdomains-per-workgroup count exists only for the
            # compile-time-shape kernel
            "kernel": (f"schwarz_fdm_fixed<double, {n}, {m[0]}, {m[1]}, {m[2]}>" if tuning[f"level{L}"][1] > 0
                       else f"local solves (n = {n}, m = {m[0]} x {m[1]} x {m[2]})"),
            "launches_timed": traced_n,
            "timing": "HIP events around each launch of the kernel inside the last timed solve",
            "ms_per_launch_isolated": kern[dominant]})
    else:
        bytes_per = {"residual": 24, "schwarz_assemble": 24, "restrict": 16 + 8 / 8, "prolong": 16 + 8 / 8}
        work = bytes_per.get(dominant, 24) * N
        achieved = work / (kern[dominant] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dominant,
                "work_per_launch": work, "ms_per_launch": kern[dominant]}

    detail = {"kernels_ms_per_launch": kern, "launches_per_solve": per_solve,
              "iterations": cyc, "final_relres": rr, "rate": main_rate, "launch_shapes": tuning}
    if wl.solver == "mg":
        detail["solve_roofline"] = solve_roofline(s, E, cyc, ms)
        log(f"whole-solve roofline: {detail['solve_roofline']['t_roofline_ms']:.3f} ms of {ms:.3f} ms "
            f"({detail['solve_roofline']['frac']:.2f})")
    s.close()
    # ---- flexible CG on the same workload, FP64 and FP32 preconditioner
    for bits in (64, 32):
        detail[f"fcg_precond_fp{bits}"] = fcg_timing(wl, bits, b, args.steps, args.warmup,
                                                    autotune=not args.no_autotune)
    gpu_rates = {wl.name: main_rate}
    # ---- the other solver workloads: 4^3 at P = 4 (MG) and the anisotropic
    # 8^3 at P = 16 ([0,16] x [0,1]^2, "max" overlap, flexible CG)
    if not args.no_configs:
        configs = {}
        wl1 = WORKLOADS["cube4_p4_min"]
        b1, _ = workload_rhs(wl1)
        configs[wl1.name] = {"ndof": wl1.ndof, "mg_fp64": mg_timing(wl1, b1, 4 * args.steps, args.warmup)}
        gpu_rates[wl1.name] = configs[wl1.name]["mg_fp64"]["rate"]
        wl3 = WORKLOADS["aniso16_p16_max"]
        b3, _ = workload_rhs(wl3)
        c3 = {"ndof": wl3.ndof}
        for bits in (64, 32):
            c3[f"fcg_precond_fp{bits}"] = fcg_timing(wl3, bits, b3, args.steps, args.warmup,
                                                     autotune=not args.no_autotune)
        configs[wl3.name] = c3
        gpu_rates[wl3.name] = c3["fcg_precond_fp64"]["rate"]
        r3 = c3["fcg_precond_fp64"].get("local_solve_roofline")
        if r3:
            log(f"{wl3.name}: local solves {r3['achieved']:.1f} TFLOP/s ({r3['frac']:.2f} of FP64 peak)")
        detail["configs"] = configs
        del b1, b3
    # ---- mixed precision at the 32^3, P = 7 workload (16.8M unknowns)
    sols = {}
    if not args.no_mixed:
        wl4 = WORKLOADS["cube32_p7_rel"]
        b4, modes4 = workload_rhs(wl4)
        mixed = {"workload": wl4.name, "ndof": wl4.ndof}
        for bits in (64, 32, 16):
            mixed[f"fcg_precond_fp{bits}"] = fcg_timing(wl4, bits, b4, args.steps, args.warmup, sols,
                                                        autotune=not args.no_autotune)
        for bits in (32, 16):
            mm = mixed[f"fcg_precond_fp{bits}"]
            mm["speedup_over_fp64"] = mixed["fcg_precond_fp64"]["ms_per_solve"] / mm["ms_per_solve"]
        mixed["speedup_fp32_over_fp64"] = mixed["fcg_precond_fp32"]["speedup_over_fp64"]
        mixed["speedup_fp16_over_fp64"] = mixed["fcg_precond_fp16"]["speedup_over_fp64"]
        gpu_rates[wl4.name] = mixed["fcg_precond_fp64"]["rate"]
        detail["mixed_precision"] = mixed
        log(f"mixed precision at {wl4.name}: FP32 preconditioner {mixed['speedup_fp32_over_fp64']:.2f}x, "
            f"FP16 local solves {mixed['speedup_fp16_over_fp64']:.2f}x the FP64 one")
        sols = {bits: v.cpu().numpy() for bits, v in sols.items()}
        del b4

    # ---- one GPU's share of a large job: 64^3 elements, P = 7 (134M unknowns)
    if not args.no_scale:
        wl6 = WORKLOADS["cube64_p7_rel"]
        b6, _ = workload_rhs(wl6)
        scale = {"workload": wl6.name, "ndof": wl6.ndof}
        for bits in (64, 32):
            scale[f"fcg_precond_fp{bits}"] = fcg_timing(wl6, bits, b6, 2, 1, autotune=not args.no_autotune)
            sc = scale[f"fcg_precond_fp{bits}"]
            log(f"FCG {wl6.name}, FP{bits} preconditioner: {sc['ms_per_solve']:.2f} ms/solve, "
                f"{sc['unknowns_per_s']:.4g} unknowns/s, {sc['iterations']} iterations")
        scale["speedup_fp32_over_fp64"] = (scale["fcg_precond_fp64"]["ms_per_solve"]
                                           / scale["fcg_precond_fp32"]["ms_per_solve"])
        detail["scale"] = scale
        del b6

    if args.serving_requests > 0:
        from paper_1612_04796_amd import sipg as _s
        log("serving stream ...")
        detail["serving"] = serving_run(args.serving_requests, seed=5)
        sv = detail["serving"]
        log(f"serving: p50 {sv['p50_latency_ms']:.2f} ms, p99 {sv['p99_latency_ms']:.2f} ms, "
            f"{sv['unknowns_per_s']:.4g} unknowns/s over {sv['makespan_s']:.2f} s")
        # one order, one preconditioner signature: with and without the
        # cohort V-cycles (segmented local solves and assemblies)
        detail["serving_same_order"] = serving_run(
            args.serving_requests, seed=6, stream="same_order",
            variants={"cohort_vcycles": {_s.SERVER_FUSE_SMOOTH: 1},
                      "no_cohort_vcycles": {_s.SERVER_FUSE_SMOOTH: 0}}, burst=True)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: periodic box {wl.length}, {wl.ne[0]}x{wl.ne[1]}x{wl.ne[2]} "
                               f"elements, P={wl.P} GLL SIPG, overlap {wl.overlap} {wl.omega}, "
                               f"V(1,1) {'MG' if wl.solver == 'mg' else 'MG-preconditioned flexible CG'} "
                               f"from x0=0 to rel. residual 1e-10, seeded 20-mode Fourier load",
                   "ne": list(wl.ne), "P": wl.P, "ndof": N, "solver": wl.solver,
                   "overlap": wl.overlap, "omega": wl.omega},
        "roofline": roof,
        "detail": detail,
    }
    if rank == 0 and not args.no_cpu_baseline:
        log("cpu baseline: oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(wl, cyc, k, phi, amp)
        log(f"cpu baseline {out['cpu_baseline']['value']:.4g} unknowns/s")
        try:  # the same sample with one BLAS thread (the paper times one core)
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                one = cpu_baseline(wl, cyc, k, phi, amp, nsample=2)
            detail["cpu_baseline_one_thread"] = {"value": one["value"], "unit": one["unit"], "cores": 1,
                                                 "sample": one["sample"]}
            log(f"cpu baseline, one thread: {one['value']:.4g} unknowns/s")
        except ImportError:
            pass
        # per workload (BASELINE's plan): t_c, rho, n10, tau10, unknowns/s
        detail["cpu_per_workload"] = cpu_per_config(
            gpu_rates, {"cube4_p4_min": 10, "cube16_p8_rel": 2, "aniso16_p16_max": 1, "cube32_p7_rel": 1})
        # the mixed-precision results against the oracle's exact discrete
        # solution (global fast diagonalization of the FP64 operator)
        if sols:
            import numpy as np
            import oracle
            wl4 = WORKLOADS["cube32_p7_rel"]
            h4 = oracle.Hierarchy(wl4.ne, wl4.length, wl4.P, overlap=wl4.overlap, omega=wl4.omega)
            xs = oracle.exact_solution(oracle.fourier_rhs(*modes4, h4), h4)
            nx = np.linalg.norm(xs)
            for bits, xv in sols.items():
                err = float(np.linalg.norm(xv - xs) / nx)
                detail["mixed_precision"][f"fcg_precond_fp{bits}"]["rel_l2_vs_oracle"] = err
                log(f"FP{bits}-preconditioned solve vs the oracle's exact solution: {err:.2e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
