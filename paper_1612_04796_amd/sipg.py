"""ctypes binding of the C ABI in include/sipg_mg.h (argument marshalling only).

Every computation runs in the HIP library; this module checks tensor
arguments (FP64, contiguous, on the GPU, of the level's size), passes raw
device pointers and the current torch stream, and turns status codes into
``SipgError``.  Importing it does not load the library; the first call does,
and raises if the library has not been built.
"""

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libsipgmg.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, EBREAKDOWN, ENOTFINITE = 0, -1, -2, -3, -4, -5, -6
OVERLAP = {"min": 0, "rel": 1, "max": 2}
BASIS = {"gll": 0, "gl": 1}
TABLES = {
    "nodes": 0, "weights": 1, "deriv": 2, "mass": 3, "ldiag": 4, "lupper": 5, "overlap": 6,
    "sub_l": 7, "sub_m": 8, "sub_lam": 9, "sub_s": 10, "sub_w": 11, "interp": 12,
    "coarse_lam": 13, "coarse_s": 14, "sub_lam_eo": 15, "sub_s_eo": 16,
}

# every entry point the header declares
EXPORTS = (
    "sipg_default_params", "sipg_setup", "sipg_destroy", "sipg_footprint", "sipg_nlevels",
    "sipg_level_info", "sipg_rhs_fourier", "sipg_apply_A", "sipg_residual", "sipg_schwarz",
    "sipg_smooth", "sipg_restrict", "sipg_prolong_add", "sipg_coarse_solve", "sipg_vcycle",
    "sipg_precond", "sipg_mg_solve", "sipg_pcg_solve", "sipg_residual_history",
    "sipg_last_error", "sipg_host_table", "sipg_time_kernel", "sipg_autotune", "sipg_tuning", "sipg_set_tuning", "sipg_tuning_limits", "sipg_tuning_cache_save", "sipg_tuning_cache_load",
    "sipg_set_option", "sipg_traced_kernel_ms", "sipg_ndof", "sipg_rhs_mean", "sipg_device_bytes",
    "sipg_schwarz_noalloc",
    "sipg_server_create", "sipg_server_submit", "sipg_server_progress", "sipg_server_status",
    "sipg_server_fetch", "sipg_server_destroy", "sipg_server_set_option", "sipg_server_stats", "sipg_server_smooth_stats",
)
REQ_QUEUED, REQ_ACTIVE, REQ_DONE, REQ_FAILED = 0, 1, 2, 3
SERVER_FUSE_APPLY, SERVER_FUSE_SMOOTH, SERVER_TUNE = 0, 1, 2
KERNELS = {"residual": 0, "schwarz_solve": 1, "schwarz_assemble": 2, "restrict": 3, "prolong": 4}


class SipgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sipg error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("ne", ctypes.c_int32 * 3),
        ("len", ctypes.c_double * 3),
        ("P", ctypes.c_int32),
        ("penalty", ctypes.c_double),
        ("overlap_mode", ctypes.c_int32),
        ("overlap", ctypes.c_double),
        ("nsmooth_pre", ctypes.c_int32),
        ("nsmooth_post", ctypes.c_int32),
        ("smooth_growth", ctypes.c_int32),
        ("precond_bits", ctypes.c_int32),
        ("basis", ctypes.c_int32),
        ("overlap_floor", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built ({LIB_PATH}); run "
                               "python -m paper_1612_04796_amd.build")
        # The library receives torch's device pointers and streams, so it must
        # bind to the HIP runtime torch has loaded: load torch first, and the
        # library's libamdhip64 dependency resolves to that same runtime
        # instead of bringing a second one into the process.
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        P, c_int, c_double, vp = ctypes.POINTER, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        sig = {
            "sipg_default_params": (None, [P(Params)]),
            "sipg_setup": (c_int, [P(Params), vp, P(vp)]),
            "sipg_destroy": (c_int, [vp]),
            "sipg_footprint": (c_int, [P(Params), P(ctypes.c_size_t)]),
            "sipg_nlevels": (c_int, [vp, P(c_int)]),
            "sipg_level_info": (c_int, [vp, c_int, P(c_int), P(c_int), P(ctypes.c_int64)]),
            "sipg_ndof": (c_int, [vp, c_int, P(ctypes.c_int64)]),
            "sipg_rhs_mean": (c_int, [vp, P(c_double)]),
            "sipg_device_bytes": (c_int, [vp, P(ctypes.c_size_t)]),
            "sipg_rhs_fourier": (c_int, [vp, c_int, P(ctypes.c_int32), P(c_double), P(c_double), vp]),
            "sipg_apply_A": (c_int, [vp, c_int, vp, vp]),
            "sipg_residual": (c_int, [vp, c_int, vp, vp, vp]),
            "sipg_schwarz": (c_int, [vp, c_int, vp, vp]),
            "sipg_schwarz_noalloc": (c_int, [vp, c_int, vp, vp]),
            "sipg_smooth": (c_int, [vp, c_int, vp, vp, c_int]),
            "sipg_restrict": (c_int, [vp, c_int, vp, vp]),
            "sipg_prolong_add": (c_int, [vp, c_int, vp, vp]),
            "sipg_coarse_solve": (c_int, [vp, vp, vp]),
            "sipg_vcycle": (c_int, [vp, vp, vp]),
            "sipg_precond": (c_int, [vp, vp, vp]),
            "sipg_mg_solve": (c_int, [vp, vp, vp, c_double, c_int, P(c_int), P(c_double)]),
            "sipg_pcg_solve": (c_int, [vp, vp, vp, c_double, c_int, P(c_int), P(c_double)]),
            "sipg_residual_history": (c_int, [vp, P(c_double), c_int, P(c_int)]),
            "sipg_last_error": (ctypes.c_char_p, []),
            "sipg_host_table": (c_int, [P(Params), c_int, c_int, c_int, P(c_double), c_int, P(c_int)]),
            "sipg_time_kernel": (c_int, [vp, c_int, c_int, c_int, c_int, P(c_double)]),
            "sipg_autotune": (c_int, [vp, c_int]),
            "sipg_tuning": (c_int, [vp, c_int, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
            "sipg_set_tuning": (c_int, [vp, c_int, c_int, c_int, c_int]),
            "sipg_tuning_cache_save": (c_int, [ctypes.c_char_p]),
            "sipg_tuning_cache_load": (c_int, [ctypes.c_char_p, ctypes.POINTER(c_int)]),
            "sipg_tuning_limits": (c_int, [vp, c_int, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
            "sipg_set_option": (c_int, [vp, c_int, c_int]),
            "sipg_traced_kernel_ms": (c_int, [vp, P(c_double), P(c_int)]),
            "sipg_server_create": (c_int, [ctypes.c_size_t, c_int, P(vp)]),
            "sipg_server_submit": (c_int, [vp, P(Params), c_int, P(ctypes.c_int32), P(c_double), P(c_double),
                                           c_double, c_int, P(ctypes.c_int64)]),
            "sipg_server_progress": (c_int, [vp, c_int, P(c_int), P(c_int), P(c_int)]),
            "sipg_server_status": (c_int, [vp, ctypes.c_int64, P(c_int), P(c_int), P(c_double), P(c_double),
                                           P(ctypes.c_int64)]),
            "sipg_server_fetch": (c_int, [vp, ctypes.c_int64, vp, vp]),
            "sipg_server_destroy": (c_int, [vp]),
            "sipg_server_set_option": (c_int, [vp, c_int, c_int]),
            "sipg_server_stats": (c_int, [vp, P(ctypes.c_int64), P(ctypes.c_int64)]),
            "sipg_server_smooth_stats": (c_int, [vp, P(ctypes.c_int64), P(ctypes.c_int64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        msg = lib().sipg_last_error().decode(errors="replace")
        raise SipgError(rc, msg)
    return rc


def make_params(ne=(4, 4, 4), length=(1.0, 1.0, 1.0), P=4, penalty=1.0, overlap="min",
                omega=0.08, nsmooth_pre=1, nsmooth_post=1, smooth_growth=1, precond_bits=64,
                basis="gll", overlap_floor=0):
    p = Params()
    lib().sipg_default_params(ctypes.byref(p))
    for d in range(3):
        p.ne[d] = int(ne[d])
        p.len[d] = float(length[d])
    p.P = int(P)
    p.penalty = float(penalty)
    p.overlap_mode = OVERLAP[overlap] if isinstance(overlap, str) else int(overlap)
    p.overlap = float(omega)
    p.nsmooth_pre, p.nsmooth_post = int(nsmooth_pre), int(nsmooth_post)
    p.smooth_growth = int(smooth_growth)
    p.precond_bits = int(precond_bits)
    p.basis = BASIS[basis] if isinstance(basis, str) else int(basis)
    p.overlap_floor = int(overlap_floor)
    return p


def tuning_cache_save(path):
    """Save the process-wide launch-shape cache as JSON (sipg_tuning_cache_save)."""
    _check(lib().sipg_tuning_cache_save(os.fsencode(path)))


def tuning_cache_load(path):
    """Merge a saved launch-shape cache; returns the entries read."""
    n = ctypes.c_int()
    _check(lib().sipg_tuning_cache_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def footprint(**kw):
    out = ctypes.c_size_t()
    _check(lib().sipg_footprint(ctypes.byref(make_params(**kw)), ctypes.byref(out)))
    return out.value


def host_table(level, d, which, **kw):
    """Host-computed set-up table (no device needed) as a list of floats."""
    p = make_params(**kw)
    cnt = ctypes.c_int()
    _check(lib().sipg_host_table(ctypes.byref(p), level, d, TABLES[which], None, 0, ctypes.byref(cnt)))
    buf = (ctypes.c_double * max(1, cnt.value))()
    _check(lib().sipg_host_table(ctypes.byref(p), level, d, TABLES[which], buf, cnt.value, ctypes.byref(cnt)))
    return list(buf[:cnt.value])


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One problem set-up (sipg_setup) and the operations on it.

    Vectors are torch float64 tensors on the current GPU in element-major
    order (see include/sipg_mg.h); every call enqueues on the stream that was
    current at construction."""

    def __init__(self, stream=None, **kw):
        self.params = make_params(**kw)
        self.kw = dict(kw)
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib().sipg_setup(ctypes.byref(self.params), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int()
        _check(lib().sipg_nlevels(self._h, ctypes.byref(n)))
        self.nlevels = n.value
        self.L = n.value - 1

    def close(self):
        if getattr(self, "_h", None):
            lib().sipg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- queries ---------------------------------------------------------
    def level_info(self, level=-1):
        order = ctypes.c_int()
        no = (ctypes.c_int * 3)()
        nd = ctypes.c_int64()
        _check(lib().sipg_level_info(self._h, level, ctypes.byref(order), no, ctypes.byref(nd)))
        return {"order": order.value, "no": tuple(no), "ndof": nd.value}

    def ndof(self, level=-1):
        n = ctypes.c_int64()
        _check(lib().sipg_ndof(self._h, level, ctypes.byref(n)))
        return n.value

    def rhs_mean(self):
        """Euclidean mean of f removed by the last mg_solve / pcg_solve."""
        m = ctypes.c_double()
        _check(lib().sipg_rhs_mean(self._h, ctypes.byref(m)))
        return m.value

    def device_bytes(self):
        """Device bytes the context holds now."""
        b = ctypes.c_size_t()
        _check(lib().sipg_device_bytes(self._h, ctypes.byref(b)))
        return b.value

    def _vec(self, t, level, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != self.ndof(level):
            raise ValueError(f"{name} has {t.numel()} values, level {level} needs {self.ndof(level)}")
        return ctypes.c_void_p(t.data_ptr())

    # ---- operations (same names as the C ABI) ----------------------------
    def rhs_fourier(self, k, phi, amp, b):
        import numpy as np
        k = np.ascontiguousarray(k, dtype=np.int32).reshape(-1)
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        amp = np.ascontiguousarray(amp, dtype=np.float64).reshape(-1)
        _check(lib().sipg_rhs_fourier(
            self._h, len(amp), k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            amp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self._vec(b, -1, "b")))
        return b

    def apply_A(self, u, y, level=-1):
        _check(lib().sipg_apply_A(self._h, level, self._vec(u, level, "u"), self._vec(y, level, "y")))
        return y

    def residual(self, u, f, r, level=-1):
        _check(lib().sipg_residual(self._h, level, self._vec(u, level, "u"), self._vec(f, level, "f"),
                                   self._vec(r, level, "r")))
        return r

    def schwarz(self, r, u, level=-1):
        _check(lib().sipg_schwarz(self._h, level, self._vec(r, level, "r"), self._vec(u, level, "u")))
        return u

    def schwarz_noalloc(self, r, u, level=-1):
        _check(lib().sipg_schwarz_noalloc(self._h, level, self._vec(r, level, "r"), self._vec(u, level, "u")))
        return u

    def smooth(self, u, f, nsteps=1, level=-1):
        _check(lib().sipg_smooth(self._h, level, self._vec(u, level, "u"), self._vec(f, level, "f"), nsteps))
        return u

    def restrict(self, r_fine, f_coarse, level):
        lv = self.L if level == -1 else level
        _check(lib().sipg_restrict(self._h, lv, self._vec(r_fine, lv, "r_fine"),
                                   self._vec(f_coarse, lv - 1, "f_coarse")))
        return f_coarse

    def prolong_add(self, u_coarse, u_fine, level):
        lv = self.L if level == -1 else level
        _check(lib().sipg_prolong_add(self._h, lv, self._vec(u_coarse, lv - 1, "u_coarse"),
                                      self._vec(u_fine, lv, "u_fine")))
        return u_fine

    def coarse_solve(self, f0, u0):
        _check(lib().sipg_coarse_solve(self._h, self._vec(f0, 0, "f0"), self._vec(u0, 0, "u0")))
        return u0

    def vcycle(self, u, f):
        _check(lib().sipg_vcycle(self._h, self._vec(u, -1, "u"), self._vec(f, -1, "f")))
        return u

    def precond(self, r, z):
        _check(lib().sipg_precond(self._h, self._vec(r, -1, "r"), self._vec(z, -1, "z")))
        return z

    def mg_solve(self, u, f, rtol=1e-10, maxcyc=100, raise_on_noconv=True):
        n = ctypes.c_int()
        rr = ctypes.c_double()
        rc = lib().sipg_mg_solve(self._h, self._vec(u, -1, "u"), self._vec(f, -1, "f"), rtol, maxcyc,
                                 ctypes.byref(n), ctypes.byref(rr))
        if rc != OK and (raise_on_noconv or rc != ENOCONV):
            _check(rc)
        return n.value, rr.value

    def pcg_solve(self, u, f, rtol=1e-10, maxit=200, raise_on_noconv=True):
        n = ctypes.c_int()
        rr = ctypes.c_double()
        rc = lib().sipg_pcg_solve(self._h, self._vec(u, -1, "u"), self._vec(f, -1, "f"), rtol, maxit,
                                  ctypes.byref(n), ctypes.byref(rr))
        if rc != OK and (raise_on_noconv or rc != ENOCONV):
            _check(rc)
        return n.value, rr.value

    def time_kernel(self, kernel, level=-1, bits=64, reps=20):
        """Mean duration (ms) of one launch of a hot-path kernel, timed with
        HIP events on the library's stream (see sipg_time_kernel)."""
        ms = ctypes.c_double()
        _check(lib().sipg_time_kernel(self._h, KERNELS[kernel], level, bits, reps, ctypes.byref(ms)))
        return ms.value

    def autotune(self, reps=10):
        """Time the candidate launch shapes of every level and keep the
        fastest (see sipg_autotune)."""
        _check(lib().sipg_autotune(self._h, int(reps)))

    def tuning(self, level=-1, bits=64):
        """(elements per workgroup, subdomains per workgroup) in use; 0 = default."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().sipg_tuning(self._h, level, bits, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_tuning(self, level=-1, bits=64, apply_epb=0, schwarz_spb=0):
        """Set the launch shapes of one level (see sipg_set_tuning); 0 = default."""
        _check(lib().sipg_set_tuning(self._h, level, bits, int(apply_epb), int(schwarz_spb)))

    def tuning_limits(self, level=-1, bits=64):
        """(largest elements per operator workgroup, largest subdomains per
        local-solve workgroup) accepted by set_tuning; 0 = no choice."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().sipg_tuning_limits(self._h, level, bits, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_option(self, option, value):
        """SIPG_OPT_GRAPH (0): replay the flexible-CG preconditioner from a
        captured HIP graph (needs a non-default stream); SIPG_OPT_WIDE_PLANES
        (2): planes per wave / workgroup of the wide local solves (0 = auto)."""
        _check(lib().sipg_set_option(self._h, int(option), int(value)))

    def wide_planes(self, k):
        """Planes per wave (matrix-core) or workgroup (vector) of the local
        solves of subdomains too large for the LDS kernels; 0 = automatic."""
        self.set_option(2, k)

    def trace_kernel(self, kernel):
        """Bracket every later top-level FP64 launch of `kernel` (a KERNELS
        name, or None to stop) with HIP events on the library's stream
        (SIPG_OPT_TRACE_KERNEL)."""
        self.set_option(1, -1 if kernel is None else KERNELS[kernel])

    def traced_kernel_ms(self):
        """(mean launch duration in ms, number of launches) of the traced
        kernel since tracing started or since the last call."""
        ms, n = ctypes.c_double(), ctypes.c_int()
        _check(lib().sipg_traced_kernel_ms(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def residual_history(self):
        n = ctypes.c_int()
        _check(lib().sipg_residual_history(self._h, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_double * max(1, n.value))()
        _check(lib().sipg_residual_history(self._h, buf, n.value, ctypes.byref(n)))
        return list(buf[:n.value])


class Server:
    """Continuous-batching solve server (sipg_server_*): submit heterogeneous
    solves, drive it with progress(), read status, fetch results."""

    def __init__(self, memory_budget, max_active=8):
        h = ctypes.c_void_p()
        _check(lib().sipg_server_create(int(memory_budget), int(max_active), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().sipg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, k, phi, amp, rtol=1e-10, maxit=100, **params):
        import numpy as np
        p = make_params(**params)
        k = np.ascontiguousarray(k, dtype=np.int32).reshape(-1)
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        amp = np.ascontiguousarray(amp, dtype=np.float64).reshape(-1)
        rid = ctypes.c_int64()
        _check(lib().sipg_server_submit(
            self._h, ctypes.byref(p), len(amp), k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            amp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(rtol), int(maxit), ctypes.byref(rid)))
        return rid.value

    def progress(self, wait_ms=10):
        a, q, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().sipg_server_progress(self._h, int(wait_ms), ctypes.byref(a), ctypes.byref(q), ctypes.byref(c)))
        return a.value, q.value, c.value

    def status(self, rid):
        st, it = ctypes.c_int(), ctypes.c_int()
        rr = ctypes.c_double()
        t = (ctypes.c_double * 3)()
        nd = ctypes.c_int64()
        _check(lib().sipg_server_status(self._h, int(rid), ctypes.byref(st), ctypes.byref(it), ctypes.byref(rr),
                                        t, ctypes.byref(nd)))
        out = {"state": st.value, "iters": it.value, "relres": rr.value, "t_submit": t[0], "t_admit": t[1],
               "t_done": t[2], "ndof": nd.value}
        if st.value == REQ_FAILED:
            out["error"] = lib().sipg_last_error().decode(errors="replace")
        return out

    def set_option(self, option, value):
        """SIPG_SERVER_FUSE_APPLY (0): batch the operator launches of
        same-order requests (1, the default) or not (0);
        SIPG_SERVER_FUSE_SMOOTH (1): cohort V-cycles of same-signature
        requests (1, the default) or not (0); SIPG_SERVER_TUNE (2): launch
        shapes of admitted requests (0 built-in, 1 cached, 2 autotuned)."""
        _check(lib().sipg_server_set_option(self._h, int(option), int(value)))

    def stats(self):
        """(fused operator launches, requests they served) so far."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sipg_server_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def smooth_stats(self):
        """(cohort V-cycles, requests they served) so far."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sipg_server_smooth_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def fetch(self, rid, u):
        import torch
        if u.dtype != torch.float64 or not u.is_cuda or not u.is_contiguous():
            raise TypeError("u must be a contiguous float64 CUDA tensor")
        if u.numel() != self.status(rid)["ndof"]:
            raise ValueError("u has the wrong number of values")
        _check(lib().sipg_server_fetch(self._h, int(rid), ctypes.c_void_p(u.data_ptr()), _stream_handle()))
        return u
