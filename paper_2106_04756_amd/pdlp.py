"""Python binding of the gfx950 PDLP solver (argument marshalling only).

Every step of the solve runs in libpdlp_hip.so; this module converts arrays to pointers and
structs to dicts.  Inputs may be NumPy arrays (host) or torch tensors (host or device); the
library deep-copies them.  The solver's HIP stream defaults to torch's current stream when a
GPU is visible.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdlp_hip.so")

OPTIMAL, ITERATION_LIMIT, NUMERICAL_ERROR, NOT_SOLVED = 0, 1, 2, 3
ERR_INVALID_ARGUMENT, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_INVALID_STATE = -1, -2, -3, -4
STATUS_NAMES = {0: "OPTIMAL", 1: "ITERATION_LIMIT", 2: "NUMERICAL_ERROR", 3: "NOT_SOLVED",
                -1: "INVALID_ARGUMENT", -2: "OUT_OF_MEMORY", -3: "DEVICE", -4: "INVALID_STATE"}

EXPORTED = ["pdlp_default_options", "pdlp_create", "pdlp_solve", "pdlp_get", "pdlp_get_info",
            "pdlp_destroy", "pdlp_last_error", "pdlp_set_host_threads", "pdlp_get_state", "pdlp_set_state",
            "pdlp_get_scaling", "pdlp_get_iterate",
            "pdlp_get_trace", "pdlp_spmv", "pdlp_kernel_times", "pdlp_pass_times", "pdlp_set_kernel_timing",
            "pdlp_reset_kernel_times",
            "pdlp_build_schedule", "pdlp_build_panel_layout", "pdlp_batch_create", "pdlp_batch_solve", "pdlp_batch_get",
            "pdlp_batch_solve_seconds", "pdlp_batch_destroy", "pdlp_batch_last_error",
            "pdlp_batch_tune", "pdlp_batch_set_schedule", "pdlp_batch_schedule", "pdlp_batch_tune_seconds",
            "pdlp_unroll_forward", "pdlp_unroll_forward_noalloc", "pdlp_unroll_backward",
            "pdlp_unroll_get_info"]


class Options(ctypes.Structure):
    _fields_ = [("ruiz_iters", ctypes.c_int32), ("pock_chambolle", ctypes.c_int32),
                ("adaptive_restarts", ctypes.c_int32), ("primal_weight_update", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("max_retries", ctypes.c_int32),
                ("trace_iters", ctypes.c_int32), ("trace_capacity", ctypes.c_int32),
                ("time_kernels", ctypes.c_int32), ("xcd_panels", ctypes.c_int32),
                ("beta_sufficient", ctypes.c_double), ("beta_necessary", ctypes.c_double),
                ("beta_artificial", ctypes.c_double), ("theta", ctypes.c_double),
                ("primal_importance", ctypes.c_double), ("eps_zero", ctypes.c_double),
                ("step_policy", ctypes.c_int32), ("restart_to_current", ctypes.c_int32),
                ("power_iters", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("mp_breaking_factor", ctypes.c_double), ("mp_downscaling", ctypes.c_double),
                ("mp_interpolation", ctypes.c_double), ("column_order", ctypes.c_int32),
                ("pw_power_of_two", ctypes.c_int32), ("lds_gather", ctypes.c_int32),
                ("lds_entries", ctypes.c_int32), ("xcd_subpanels", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("output_is_average", ctypes.c_int32),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("n_eq", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("attempts", ctypes.c_int64), ("restarts", ctypes.c_int64),
                ("checks", ctypes.c_int64), ("spmv_K", ctypes.c_int64), ("spmv_KT", ctypes.c_int64),
                ("omega", ctypes.c_double), ("eta_hat", ctypes.c_double),
                ("kkt", ctypes.c_double * 4), ("create_seconds", ctypes.c_double),
                ("solve_seconds", ctypes.c_double), ("step_bytes", ctypes.c_double),
                ("layout_K", ctypes.c_int32), ("layout_KT", ctypes.c_int32),
                ("panels_K", ctypes.c_int32), ("panels_KT", ctypes.c_int32)]


class State(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("t", ctypes.c_int64), ("n_outer", ctypes.c_int64),
                ("eta_hat", ctypes.c_double), ("omega", ctypes.c_double), ("s_eta", ctypes.c_double),
                ("mu_prev", ctypes.c_double), ("mu_anchor", ctypes.c_double)]


class AttemptRec(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("eta", ctypes.c_double), ("eta_bar", ctypes.c_double),
                ("accepted", ctypes.c_int32), ("pad", ctypes.c_int32)]


class CheckRec(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("mu_cur", ctypes.c_double), ("mu_avg", ctypes.c_double),
                ("kkt", ctypes.c_double), ("omega_after", ctypes.c_double),
                ("mu_anchor", ctypes.c_double), ("use_avg", ctypes.c_int32),
                ("mask", ctypes.c_int32), ("terminated", ctypes.c_int32), ("pad", ctypes.c_int32)]


class UnrollInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("segment", ctypes.c_int64),
                ("checkpoints", ctypes.c_int64), ("recomputed_steps", ctypes.c_int64),
                ("eta", ctypes.c_double), ("omega", ctypes.c_double),
                ("forward_seconds", ctypes.c_double), ("backward_seconds", ctypes.c_double),
                ("device_bytes", ctypes.c_double), ("ready", ctypes.c_int32), ("pad", ctypes.c_int32)]


_lib = None
P = ctypes.c_void_p
I64 = ctypes.c_int64


def lib() -> ctypes.CDLL:
    """Load libpdlp_hip.so (built in place by paper_2106_04756_amd.build); fail loudly if absent."""
    global _lib
    if _lib is None:
        # Load torch's HIP runtime first so the library and torch share one runtime (the
        # library links libamdhip64.so.7 by soname and binds to the copy already loaded).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2106_04756_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.pdlp_default_options.argtypes = [ctypes.POINTER(Options)]
        L.pdlp_default_options.restype = None
        L.pdlp_create.argtypes = [ctypes.POINTER(P), I64, I64, I64, P, P, P, P, P, P, P,
                                  ctypes.POINTER(Options), P]
        L.pdlp_create.restype = ctypes.c_int
        L.pdlp_solve.argtypes = [P, ctypes.c_double, I64]
        L.pdlp_solve.restype = ctypes.c_int
        L.pdlp_get.argtypes = [P, P, P, P]
        L.pdlp_get.restype = ctypes.c_int
        L.pdlp_get_info.argtypes = [P, ctypes.POINTER(Info)]
        L.pdlp_get_info.restype = ctypes.c_int
        L.pdlp_destroy.argtypes = [P]
        L.pdlp_destroy.restype = None
        L.pdlp_last_error.argtypes = [P]
        L.pdlp_last_error.restype = ctypes.c_char_p
        L.pdlp_get_state.argtypes = [P, P, P, P, P, P, P, ctypes.POINTER(State)]
        L.pdlp_get_state.restype = ctypes.c_int
        L.pdlp_set_state.argtypes = [P, P, P, P, P, P, P, ctypes.POINTER(State)]
        L.pdlp_set_state.restype = ctypes.c_int
        L.pdlp_get_scaling.argtypes = [P, P, P]
        L.pdlp_get_scaling.restype = ctypes.c_int
        L.pdlp_get_iterate.argtypes = [P, P, P]
        L.pdlp_get_iterate.restype = ctypes.c_int
        L.pdlp_get_trace.argtypes = [P, P, I64, P, P, I64, P, P, P, P]
        L.pdlp_get_trace.restype = ctypes.c_int
        L.pdlp_spmv.argtypes = [P, ctypes.c_int, P, P]
        L.pdlp_spmv.restype = ctypes.c_int
        L.pdlp_kernel_times.argtypes = [P, P, P]
        L.pdlp_kernel_times.restype = ctypes.c_int
        L.pdlp_set_kernel_timing.argtypes = [P, ctypes.c_int]
        L.pdlp_set_kernel_timing.restype = ctypes.c_int
        L.pdlp_pass_times.argtypes = [P, P, P]
        L.pdlp_pass_times.restype = ctypes.c_int
        L.pdlp_reset_kernel_times.argtypes = [P]
        L.pdlp_reset_kernel_times.restype = ctypes.c_int
        L.pdlp_set_host_threads.argtypes = [ctypes.c_int]
        L.pdlp_set_host_threads.restype = ctypes.c_int
        L.pdlp_build_schedule.argtypes = [P, I64, P, I64, P, P, P]
        L.pdlp_build_schedule.restype = ctypes.c_int
        L.pdlp_build_panel_layout.argtypes = [P, P, P, I64, I64, ctypes.c_int32, P, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(PanelLayoutC)]
        L.pdlp_build_panel_layout.restype = ctypes.c_int
        L.pdlp_batch_create.argtypes = [ctypes.POINTER(P), I64, P, P, P, P, P, P, P, P, P, P,
                                        ctypes.POINTER(Options), P]
        L.pdlp_batch_create.restype = ctypes.c_int
        L.pdlp_batch_solve.argtypes = [P, ctypes.c_double, I64]
        L.pdlp_batch_solve.restype = ctypes.c_int
        L.pdlp_batch_get.argtypes = [P, P, P, P, P, P]
        L.pdlp_batch_get.restype = ctypes.c_int
        L.pdlp_batch_solve_seconds.argtypes = [P]
        L.pdlp_batch_solve_seconds.restype = ctypes.c_double
        L.pdlp_batch_tune.argtypes = [P, I64, P, P]
        L.pdlp_batch_tune.restype = ctypes.c_int
        L.pdlp_batch_set_schedule.argtypes = [P, P, P]
        L.pdlp_batch_set_schedule.restype = ctypes.c_int
        L.pdlp_batch_schedule.argtypes = [P, P, P, P]
        L.pdlp_batch_schedule.restype = ctypes.c_int
        L.pdlp_batch_tune_seconds.argtypes = [P]
        L.pdlp_batch_tune_seconds.restype = ctypes.c_double
        L.pdlp_batch_destroy.argtypes = [P]
        L.pdlp_batch_destroy.restype = None
        L.pdlp_batch_last_error.argtypes = [P]
        L.pdlp_batch_last_error.restype = ctypes.c_char_p
        L.pdlp_unroll_forward.argtypes = [P, P, P, I64, I64, ctypes.c_double, ctypes.c_double, P, P]
        L.pdlp_unroll_forward.restype = ctypes.c_int
        L.pdlp_unroll_forward_noalloc.argtypes = [P, P, P, I64, I64, ctypes.c_double, ctypes.c_double, P, P]
        L.pdlp_unroll_forward_noalloc.restype = ctypes.c_int
        L.pdlp_unroll_backward.argtypes = [P, P, P, P, P]
        L.pdlp_unroll_backward.restype = ctypes.c_int
        L.pdlp_unroll_get_info.argtypes = [P, ctypes.POINTER(UnrollInfo)]
        L.pdlp_unroll_get_info.restype = ctypes.c_int
        _lib = L
    return _lib


class PdlpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def default_options(**overrides) -> Options:
    o = Options()
    lib().pdlp_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _ptr(a, dtype):
    """(pointer, keep-alive) of a NumPy array or torch tensor of the given dtype."""
    if a is None:
        return None, None
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):          # torch tensor
        import torch
        tdt = {np.float64: torch.float64, np.int64: torch.int64, np.int32: torch.int32}[dtype]
        if a.dtype != tdt or not a.is_contiguous():
            a = a.to(tdt).contiguous()
        return ctypes.c_void_p(a.data_ptr()), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return ctypes.c_void_p(arr.ctypes.data), arr


def _out_ptr(a):
    """Pointer of a caller's float64 output buffer (NumPy array or torch tensor).  The library
    writes through this pointer, so a buffer it cannot write in place (another dtype, not
    contiguous, read-only) is refused instead of being replaced by a temporary copy."""
    if a is None:
        return None
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):          # torch tensor
        import torch
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise ValueError("output tensor must be contiguous torch.float64 "
                             f"(got {a.dtype}, contiguous={a.is_contiguous()})")
        return ctypes.c_void_p(a.data_ptr())
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous \
            or not a.flags.writeable:
        raise ValueError("output array must be a writeable C-contiguous numpy.float64 array")
    return ctypes.c_void_p(a.ctypes.data)


def _default_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def schedule(row_ptr):
    """Host-only: the SpMV schedule of a CSR matrix: (tasks as an (k, 4) int32 array of
    {a, b, kind | log2(lanes) << 8, split id}, number of split rows, row permutation)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    nd = ctypes.c_int64()
    ns = ctypes.c_int64()
    rc = lib().pdlp_build_schedule(rp.ctypes.data, rp.size - 1, None, 0, ctypes.byref(nd),
                                   ctypes.byref(ns), None)
    if rc != 0:
        raise PdlpError(rc, "pdlp_build_schedule failed")
    desc = np.zeros((nd.value, 4), dtype=np.int32)
    perm = np.full(max(rp.size - 1, 1), -1, dtype=np.int32)
    lib().pdlp_build_schedule(rp.ctypes.data, rp.size - 1, desc.ctypes.data, nd.value,
                              ctypes.byref(nd), ctypes.byref(ns), perm.ctypes.data)
    return desc, ns.value, perm[:rp.size - 1]


class PanelLayoutC(ctypes.Structure):
    _fields_ = [("nprow", ctypes.c_int64), ("nwave", ctypes.c_int64), ("nblock", ctypes.c_int64),
                ("nslots", ctypes.c_int64), ("nseg", ctypes.c_int64)] + \
               [(k, ctypes.c_void_p) for k in ("cut", "prow_ptr", "prow_row", "src", "slot_ptr", "slot_idx",
                                               "wave", "wave_begin", "task_off", "cis", "vs", "seg_ptr", "seg")]


def set_host_threads(n: int = 0) -> int:
    """Host threads of the preparation in the next solver creations (0 = the default); returns
    the count in effect (pdlp_set_host_threads)."""
    return int(lib().pdlp_set_host_threads(int(n)))


def panel_layout(row_ptr, col_idx, val, ncols, npanel, cuts=None, groups=256, aligned=False, emax=8):
    """Host-only: the column-panel layout of a CSR matrix as the products read it, its
    interleaved entries and the LDS workgroups' segments (pdlp_build_panel_layout), as a
    dict of NumPy arrays."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    nrows = rp.size - 1
    cu = None if cuts is None else np.ascontiguousarray(cuts, dtype=np.int32)
    args = (rp.ctypes.data, ci.ctypes.data, v.ctypes.data, nrows, int(ncols), int(npanel),
            None if cu is None else cu.ctypes.data, int(emax), int(groups), int(bool(aligned)))
    L = PanelLayoutC()
    if lib().pdlp_build_panel_layout(*args, ctypes.byref(L)) != 0:
        raise PdlpError(-1, "pdlp_build_panel_layout failed")
    shapes = {"cut": (npanel + 1, np.int32), "prow_ptr": (L.nprow + 1, np.int64), "prow_row": (L.nprow, np.int32),
              "src": (int(rp[-1]), np.int64), "slot_ptr": (nrows + 1, np.int64), "slot_idx": (L.nprow, np.int32),
              "wave": ((L.nwave, 4), np.int32), "wave_begin": (npanel + 1, np.int32),
              "task_off": (L.nwave + 1, np.int64), "cis": (L.nslots, np.int32), "vs": (L.nslots, np.float64),
              "seg_ptr": (groups + 1, np.int32), "seg": ((L.nseg, 4), np.int32)}
    out = {k: np.zeros(shp, dtype=dt) for k, (shp, dt) in shapes.items()}
    for k, a in out.items():
        setattr(L, k, a.ctypes.data if a.size else None)
    if lib().pdlp_build_panel_layout(*args, ctypes.byref(L)) != 0:
        raise PdlpError(-1, "pdlp_build_panel_layout failed")
    out["nblock"] = L.nblock
    return out


class Solver:
    """One LP on the GPU.  See include/pdlp.h for the semantics of every call."""

    def __init__(self, m, n, n_eq, c, row_ptr, col_idx, val, q, l, u, options: Options | None = None,
                 stream=None, **option_overrides):
        L = lib()
        if options is None:
            options = default_options(**option_overrides)
        elif option_overrides:
            for k, v in option_overrides.items():
                setattr(options, k, v)
        self.options = options
        self.m, self.n, self.n_eq = int(m), int(n), int(n_eq)
        keep = []
        ptrs = []
        for a, dt in ((c, np.float64), (row_ptr, np.int64), (col_idx, np.int32), (val, np.float64),
                      (q, np.float64), (l, np.float64), (u, np.float64)):
            p, k = _ptr(a, dt)
            keep.append(k)
            ptrs.append(p)
        self._stream = stream if stream is not None else _default_stream()
        h = ctypes.c_void_p()
        rc = L.pdlp_create(ctypes.byref(h), self.m, self.n, self.n_eq, *ptrs, ctypes.byref(options),
                           self._stream)
        if rc != 0:
            raise PdlpError(rc, L.pdlp_last_error(None).decode())
        self._h = h

    @classmethod
    def from_lp(cls, lp, **kw):
        return cls(lp.m, lp.n, lp.n_eq, lp.c, lp.row_ptr, lp.col_idx, lp.val, lp.q, lp.l, lp.u, **kw)

    def _check(self, rc):
        if rc < 0:
            raise PdlpError(rc, lib().pdlp_last_error(self._h).decode())
        return rc

    def solve(self, tol: float = 1e-8, iter_limit: int = 100000) -> int:
        return self._check(lib().pdlp_solve(self._h, float(tol), int(iter_limit)))

    def get(self):
        x = np.empty(self.n)
        y = np.empty(self.m)
        kkt = np.empty(4)
        self._check(lib().pdlp_get(self._h, x.ctypes.data, y.ctypes.data if self.m else None, kkt.ctypes.data))
        return x, y, kkt

    def get_into(self, x=None, y=None):
        """Write the returned point into caller tensors / arrays (host or device)."""
        self._check(lib().pdlp_get(self._h, _out_ptr(x), _out_ptr(y), None))

    def info(self) -> dict:
        inf = Info()
        self._check(lib().pdlp_get_info(self._h, ctypes.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in Info._fields_}
        d["kkt"] = list(inf.kkt)
        return d

    _STATE_KEYS = ("k", "t", "n_outer", "eta_hat", "omega", "s_eta", "mu_prev", "mu_anchor")

    def get_state(self) -> dict:
        """Checkpoint in the preconditioned variables (see pdlp_get_state)."""
        n, m = self.n, self.m
        v = {k: np.empty(n if k in ("x", "xa", "Sx") else m) for k in ("x", "y", "xa", "ya", "Sx", "Sy")}
        st = State()
        ptr = {k: (a.ctypes.data if a.size else None) for k, a in v.items()}
        self._check(lib().pdlp_get_state(self._h, ptr["x"], ptr["y"], ptr["xa"], ptr["ya"], ptr["Sx"],
                                         ptr["Sy"], ctypes.byref(st)))
        v.update({k: getattr(st, k) for k in self._STATE_KEYS})
        v["Seta"] = v.pop("s_eta")
        return v

    def set_state(self, state: dict):
        """Resume from a checkpoint with the keys of get_state (the oracle's state records
        use the same names)."""
        arrs = {k: np.ascontiguousarray(state[k], dtype=np.float64) for k in ("x", "y", "xa", "ya", "Sx", "Sy")}
        st = State(k=int(state["k"]), t=int(state["t"]), n_outer=int(state["n_outer"]),
                   eta_hat=float(state["eta_hat"]), omega=float(state["omega"]),
                   s_eta=float(state["Seta"]), mu_prev=float(state["mu_prev"]),
                   mu_anchor=float(state["mu_anchor"]))
        p = {k: (a.ctypes.data if a.size else None) for k, a in arrs.items()}
        self._check(lib().pdlp_set_state(self._h, p["x"], p["y"], p["xa"], p["ya"], p["Sx"], p["Sy"],
                                         ctypes.byref(st)))

    def scaling(self):
        D1 = np.empty(self.m)
        D2 = np.empty(self.n)
        self._check(lib().pdlp_get_scaling(self._h, D1.ctypes.data if self.m else None, D2.ctypes.data))
        return D1, D2

    def iterate(self):
        xs = np.empty(self.n)
        ys = np.empty(self.m)
        self._check(lib().pdlp_get_iterate(self._h, xs.ctypes.data, ys.ctypes.data if self.m else None))
        return xs, ys

    def trace(self) -> dict:
        cap = max(int(self.options.trace_capacity), 1)
        att = (AttemptRec * cap)()
        chk = (CheckRec * cap)()
        na, nc, ni = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        ti = int(self.options.trace_iters)
        xs = np.empty((max(ti, 1), self.n))
        ys = np.empty((max(ti, 1), max(self.m, 1)))
        self._check(lib().pdlp_get_trace(self._h, ctypes.cast(att, P), cap, ctypes.byref(na),
                                         ctypes.cast(chk, P), cap, ctypes.byref(nc),
                                         xs.ctypes.data if ti else None,
                                         ys.ctypes.data if (ti and self.m) else None,
                                         ctypes.byref(ni)))
        na_k = min(na.value, cap)
        nc_k = min(nc.value, cap)
        attempts = [(a.k, a.eta, a.eta_bar, bool(a.accepted)) for a in att[:na_k]]
        checks = [dict(k=r.k, mu_cur=r.mu_cur, mu_avg=r.mu_avg, kkt=r.kkt, omega_after=r.omega_after,
                       mu_anchor=r.mu_anchor, use_avg=bool(r.use_avg), mask=r.mask,
                       terminated=bool(r.terminated)) for r in chk[:nc_k]]
        return dict(attempts=attempts, n_attempts=na.value, checks=checks, n_checks=nc.value,
                    xs=xs[:ni.value], ys=ys[:ni.value, :self.m], n_iter=ni.value)

    def spmv(self, x, out, transpose=False):
        """out = K~ x (or K~^T x) on device tensors."""
        px, kx = _ptr(x, np.float64)
        self._check(lib().pdlp_spmv(self._h, 1 if transpose else 0, px, _out_ptr(out)))

    # ---- unrolled PDHG (frozen eta, omega, D1, D2) and its adjoint ----

    def unroll_forward(self, c=None, q=None, steps=500, segment=50, eta=0.0, omega=0.0,
                       x_out=None, y_out=None):
        """x_T, y_T after `steps` fixed PDHG steps with objective c and right-hand side q (user
        units; None = the LP's own).  Outputs go to x_out / y_out (NumPy or torch, host or
        device) when given, else to new NumPy arrays, which are returned."""
        pc, kc = _ptr(c, np.float64)
        pq, kq = _ptr(q, np.float64)
        xo = np.empty(self.n) if x_out is None else x_out
        yo = np.empty(self.m) if y_out is None else y_out
        px, py = _out_ptr(xo), _out_ptr(yo)
        self._check(lib().pdlp_unroll_forward(self._h, pc, pq, int(steps), int(segment), float(eta),
                                              float(omega), px, py if self.m else None))
        self.unroll_id = getattr(self, "unroll_id", 0) + 1
        return xo, yo

    def unroll_forward_noalloc(self, c=None, q=None, steps=500, segment=50, eta=0.0, omega=0.0,
                               x_out=None, y_out=None):
        """unroll_forward with the unroll's buffers in the library's per-GPU scratch array
        (pdlp_unroll_forward_noalloc: no device allocation)."""
        pc, kc = _ptr(c, np.float64)
        pq, kq = _ptr(q, np.float64)
        xo = np.empty(self.n) if x_out is None else x_out
        yo = np.empty(self.m) if y_out is None else y_out
        px, py = _out_ptr(xo), _out_ptr(yo)
        self._check(lib().pdlp_unroll_forward_noalloc(self._h, pc, pq, int(steps), int(segment), float(eta),
                                                      float(omega), px, py if self.m else None))
        self.unroll_id = getattr(self, "unroll_id", 0) + 1
        return xo, yo

    def unroll_backward(self, gx=None, gy=None, gc_out=None, gq_out=None):
        """(dL/dc, dL/dq) of the last unroll_forward given dL/dx_T, dL/dy_T (None = 0)."""
        pgx, kgx = _ptr(gx, np.float64)
        pgy, kgy = _ptr(gy, np.float64)
        gc = np.empty(self.n) if gc_out is None else gc_out
        gq = np.empty(self.m) if gq_out is None else gq_out
        pc, pq = _out_ptr(gc), _out_ptr(gq)
        self._check(lib().pdlp_unroll_backward(self._h, pgx, pgy if self.m else None, pc,
                                               pq if self.m else None))
        return gc, gq

    def unroll_info(self) -> dict:
        u = UnrollInfo()
        self._check(lib().pdlp_unroll_get_info(self._h, ctypes.byref(u)))
        return {k: getattr(u, k) for k, _ in UnrollInfo._fields_ if k != "pad"}

    def kernel_times(self):
        t = np.zeros(2)
        c = np.zeros(2, dtype=np.int64)
        self._check(lib().pdlp_kernel_times(self._h, t.ctypes.data, c.ctypes.data))
        return t, c

    def set_kernel_timing(self, on: bool):
        """Kernel timing (options.time_kernels) on or off for the next solves."""
        self._check(lib().pdlp_set_kernel_timing(self._h, 1 if on else 0))
        self.options.time_kernels = 1 if on else 0

    def pass_times(self):
        """(times_ms[4], counts[4]) of the primal first pass, primal combine, dual first pass
        and dual combine over the slots that ran (options.time_kernels)."""
        t = np.zeros(4)
        c = np.zeros(4, dtype=np.int64)
        self._check(lib().pdlp_pass_times(self._h, t.ctypes.data, c.ctypes.data))
        return t, c

    def reset_kernel_times(self):
        self._check(lib().pdlp_reset_kernel_times(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().pdlp_destroy(self._h)
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


class Batch:
    """Many independent LPs solved in one persistent launch (one workgroup per LP).
    See pdlp_batch_create in include/pdlp.h."""

    def __init__(self, lps, options: Options | None = None, stream=None, **option_overrides):
        L = lib()
        if options is None:
            options = default_options(**option_overrides)
        self.options = options
        self.count = len(lps)
        self.m = np.array([lp.m for lp in lps], dtype=np.int64)
        self.n = np.array([lp.n for lp in lps], dtype=np.int64)
        self.n_eq = np.array([lp.n_eq for lp in lps], dtype=np.int64)
        cat = lambda key, dt: np.ascontiguousarray(np.concatenate([np.asarray(getattr(lp, key)) for lp in lps]), dtype=dt)
        arrs = [self.m, self.n, self.n_eq, cat("c", np.float64), cat("row_ptr", np.int64),
                cat("col_idx", np.int32), cat("val", np.float64), cat("q", np.float64),
                cat("l", np.float64), cat("u", np.float64)]
        self._keep = arrs
        self._stream = stream if stream is not None else _default_stream()
        h = ctypes.c_void_p()
        rc = L.pdlp_batch_create(ctypes.byref(h), self.count, *[a.ctypes.data for a in arrs],
                                 ctypes.byref(options), self._stream)
        if rc != 0:
            raise PdlpError(rc, L.pdlp_batch_last_error(None).decode())
        self._h = h
        self.xoff = np.concatenate([[0], np.cumsum(self.n)])
        self.yoff = np.concatenate([[0], np.cumsum(self.m)])

    def _check(self, rc):
        if rc < 0:
            raise PdlpError(rc, lib().pdlp_batch_last_error(self._h).decode())
        return rc

    def solve(self, tol: float = 1e-8, iter_limit: int = 100000) -> float:
        """Solve every member; returns the wall time of the launch in seconds."""
        self._check(lib().pdlp_batch_solve(self._h, float(tol), int(iter_limit)))
        return lib().pdlp_batch_solve_seconds(self._h)

    BATCH_CLASSES = 4

    SCHEDULES = [(64, 1), (128, 1), (128, 2), (256, 1), (256, 2), (512, 1), (512, 2), (1024, 1)]

    def tune(self, steps: int = 200):
        """Pick each size class's schedule by timing every candidate (pdlp_batch_tune);
        returns [(threads, rows per thread)] per class."""
        th = np.zeros(self.BATCH_CLASSES, dtype=np.int32)
        rw = np.zeros(self.BATCH_CLASSES, dtype=np.int32)
        self._check(lib().pdlp_batch_tune(self._h, int(steps), th.ctypes.data, rw.ctypes.data))
        return [(int(a), int(b)) for a, b in zip(th, rw)]

    def set_schedule(self, schedule):
        """schedule: (threads, rows per thread) per class."""
        if len(schedule) != self.BATCH_CLASSES:
            raise ValueError(f"need {self.BATCH_CLASSES} schedules")
        th = np.ascontiguousarray([a for a, _ in schedule], dtype=np.int32)
        rw = np.ascontiguousarray([b for _, b in schedule], dtype=np.int32)
        self._check(lib().pdlp_batch_set_schedule(self._h, th.ctypes.data, rw.ctypes.data))

    def schedule(self):
        """([(threads, rows per thread)] per class, members per class)."""
        th = np.zeros(self.BATCH_CLASSES, dtype=np.int32)
        rw = np.zeros(self.BATCH_CLASSES, dtype=np.int32)
        mc = np.zeros(self.BATCH_CLASSES, dtype=np.int64)
        self._check(lib().pdlp_batch_schedule(self._h, th.ctypes.data, rw.ctypes.data, mc.ctypes.data))
        return [(int(a), int(b)) for a, b in zip(th, rw)], [int(v) for v in mc]

    def tune_seconds(self) -> float:
        return lib().pdlp_batch_tune_seconds(self._h)

    def get(self):
        """(list of x, list of y, status[count], iterations[count], kkt[count, 4])."""
        x = np.empty(int(self.xoff[-1]))
        y = np.empty(max(int(self.yoff[-1]), 1))
        st = np.empty(self.count, dtype=np.int32)
        it = np.empty(self.count, dtype=np.int64)
        kkt = np.empty((self.count, 4))
        self._check(lib().pdlp_batch_get(self._h, x.ctypes.data, y.ctypes.data, st.ctypes.data,
                                         it.ctypes.data, kkt.ctypes.data))
        xs = [x[self.xoff[k]:self.xoff[k + 1]] for k in range(self.count)]
        ys = [y[self.yoff[k]:self.yoff[k + 1]] for k in range(self.count)]
        return xs, ys, st, it, kkt

    def close(self):
        if getattr(self, "_h", None):
            lib().pdlp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
