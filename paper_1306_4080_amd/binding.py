"""ctypes binding of ``libpcdn.so`` (declared in ``include/pcdn.h``).

Argument marshalling only: every step of the method runs in the HIP library.
There is no fallback: if the library is missing or does not load, every entry
point raises.  The functions carry the C names; ``Solver`` is a small owner of
one context.

Device arrays may be passed as torch tensors (their ``data_ptr()`` is handed
over with ``ptr_kind = 1``); host arrays as numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcdn.so")

PCDN_LOSS_LOGISTIC = 0
PCDN_LOSS_L2SVM = 1
PCDN_OK = 0
PCDN_NOT_CONVERGED = 1
ERRORS = {-1: "PCDN_E_ARG", -2: "PCDN_E_CSC", -3: "PCDN_E_OOM", -4: "PCDN_E_DEVICE",
          -5: "PCDN_E_STATE", -6: "PCDN_E_NUMERIC"}
LOSSES = {"lr": PCDN_LOSS_LOGISTIC, "logistic": PCDN_LOSS_LOGISTIC,
          "svm": PCDN_LOSS_L2SVM, "l2svm": PCDN_LOSS_L2SVM}

# entry points declared in include/pcdn.h
SYMBOLS = ("pcdn_create", "pcdn_load_csc", "pcdn_load_csc_bias", "pcdn_solve", "pcdn_reset", "pcdn_step",
           "pcdn_iterate",
           "pcdn_solve_batch", "pcdn_solve_path", "pcdn_solve_path_lanes", "pcdn_autotune", "pcdn_iterate_batch",
           "pcdn_server_create", "pcdn_server_submit", "pcdn_server_step", "pcdn_server_status",
           "pcdn_server_take", "pcdn_server_last_error", "pcdn_server_destroy",
           "pcdn_permutation", "pcdn_get_w", "pcdn_get_cache", "pcdn_evaluate",
           "pcdn_profile", "pcdn_profile_read", "pcdn_last_error", "pcdn_destroy",
           "pcdn_solve_static")


class PcdnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class pcdn_opts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("max_outer", ctypes.c_int32),
                ("max_ls", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("nu", ctypes.c_double), ("w0", ctypes.c_void_p),
                ("schedule", ctypes.c_int32), ("shrink", ctypes.c_int32),
                ("penalty", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("l2", ctypes.c_double)]


class pcdn_info(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("bundles", ctypes.c_int64), ("ls_steps", ctypes.c_int64),
                ("ls_fail", ctypes.c_int64), ("nnz_swept", ctypes.c_int64),
                ("objective", ctypes.c_double), ("subgrad", ctypes.c_double),
                ("subgrad0", ctypes.c_double), ("alg_bytes", ctypes.c_double),
                ("seconds", ctypes.c_double), ("min_armijo_margin", ctypes.c_double),
                ("min_stop_margin", ctypes.c_double), ("schedule", ctypes.c_int32),
                ("chunk", ctypes.c_int32)]


class pcdn_step_info(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("delta", ctypes.c_double),
                ("dF", ctypes.c_double), ("q", ctypes.c_int32), ("pad", ctypes.c_int32)]


class pcdn_job(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("C", ctypes.c_double), ("P", ctypes.c_int64),
                ("eps", ctypes.c_double), ("loss", ctypes.c_int32), ("status", ctypes.c_int32),
                ("opts", ctypes.POINTER(pcdn_opts)), ("w_out", ctypes.c_void_p),
                ("info", ctypes.POINTER(pcdn_info))]


class pcdn_tune_point(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64), ("schedule", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("sec_per_outer", ctypes.c_double), ("rate", ctypes.c_double),
                ("predicted_seconds", ctypes.c_double), ("chunk", ctypes.c_int32),
                ("narrow", ctypes.c_int32)]


class pcdn_tune(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64), ("schedule", ctypes.c_int32), ("n_tried", ctypes.c_int32),
                ("predicted_seconds", ctypes.c_double), ("chunk", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("tried", pcdn_tune_point * 12)]


class pcdn_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("y", ctypes.c_void_p), ("C", ctypes.c_double),
                ("P", ctypes.c_int64), ("eps", ctypes.c_double), ("loss", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("opts", ctypes.POINTER(pcdn_opts))]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpcdn.so (after torch, if torch is importable, so that one HIP
    runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"PCDN HIP library not built: {path} is missing "
                           "(run `python -m paper_1306_4080_amd.build`)")
    if "torch" not in sys.modules:
        try:
            import torch  # noqa: F401  (shares its HIP runtime with the library)
        except Exception:
            pass
    L = ctypes.CDLL(path)
    vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                              ctypes.c_uint64, ctypes.c_double)
    L.pcdn_create.argtypes = [ctypes.POINTER(vp), i32, vp]
    L.pcdn_load_csc.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, i32]
    L.pcdn_load_csc_bias.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, i32, ctypes.c_float]
    L.pcdn_solve.argtypes = [vp, dbl, i64, dbl, i32, ctypes.POINTER(pcdn_opts), vp,
                             ctypes.POINTER(pcdn_info)]
    L.pcdn_reset.argtypes = [vp, i32, dbl, vp]
    L.pcdn_step.argtypes = [vp, vp, i64, ctypes.POINTER(pcdn_opts),
                            ctypes.POINTER(pcdn_step_info), vp, vp, vp, vp]
    L.pcdn_iterate.argtypes = [vp, i64, i64, i64, ctypes.POINTER(pcdn_opts), vp]
    L.pcdn_solve_batch.argtypes = [ctypes.POINTER(pcdn_job), ctypes.c_int32]
    L.pcdn_iterate_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.c_int32, i64,
                                     i64, ctypes.POINTER(pcdn_opts), ctypes.POINTER(dbl)]
    L.pcdn_autotune.argtypes = [vp, i32, dbl, dbl, ctypes.POINTER(pcdn_opts),
                                ctypes.POINTER(pcdn_tune)]
    L.pcdn_solve_path.argtypes = [vp, ctypes.POINTER(dbl), ctypes.c_int32, i64, dbl, i32,
                                  ctypes.POINTER(pcdn_opts), vp, ctypes.POINTER(pcdn_info)]
    L.pcdn_solve_path_lanes.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(dbl),
                                        ctypes.c_int32, i64, dbl, i32, ctypes.POINTER(pcdn_opts),
                                        vp, ctypes.POINTER(pcdn_info)]
    L.pcdn_permutation.argtypes = [vp, u64, i64, vp]
    L.pcdn_get_w.argtypes = [vp, vp]
    L.pcdn_get_cache.argtypes = [vp, vp]
    L.pcdn_evaluate.argtypes = [vp, vp, vp]
    L.pcdn_profile.argtypes = [vp, i32]
    L.pcdn_profile_read.argtypes = [vp, i32, vp, vp, vp]
    L.pcdn_last_error.argtypes = [vp]
    L.pcdn_last_error.restype = ctypes.c_char_p
    L.pcdn_server_create.argtypes = [ctypes.POINTER(vp), i32, i64]
    L.pcdn_server_submit.argtypes = [vp, ctypes.POINTER(pcdn_request), ctypes.POINTER(i64)]
    L.pcdn_server_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.pcdn_server_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(i64)]
    L.pcdn_server_take.argtypes = [vp, i64, vp, ctypes.POINTER(pcdn_info),
                                   ctypes.POINTER(ctypes.c_int32)]
    L.pcdn_server_last_error.argtypes = [vp]
    L.pcdn_server_last_error.restype = ctypes.c_char_p
    L.pcdn_server_destroy.argtypes = [vp]
    L.pcdn_destroy.argtypes = [vp]
    L.pcdn_solve_static.argtypes = [i32, vp, i64, i64, i64, vp, vp, vp, vp, dbl, i64, dbl, i32,
                                    ctypes.POINTER(pcdn_opts), vp, ctypes.POINTER(pcdn_info)]
    for s in SYMBOLS:
        if s not in ("pcdn_last_error", "pcdn_server_last_error"):
            getattr(L, s).restype = ctypes.c_int
    _lib = L
    return L


def _ptr(a) -> int:
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _check(ctx, rc, allow=(PCDN_OK,)):
    if rc in allow:
        return rc
    msg = load_library().pcdn_last_error(ctx)
    raise PcdnError(rc, msg.decode() if msg else "")


SCHEDULES = {"auto": 0, "wide": 1, "narrow": 2}
PENALTIES = {"l1": 0, "elastic": 1, "l2": 2}


def _opts(seed=0, max_outer=0, max_ls=0, sigma=0.0, beta=0.0, gamma=0.0, nu=0.0, w0=None,
          schedule="auto", shrink=False, penalty="l1", l2=0.0, chunk=0):
    schedule = SCHEDULES.get(schedule, schedule)
    penalty = PENALTIES.get(penalty, penalty)
    o = pcdn_opts(seed, max_outer, max_ls, sigma, beta, gamma, nu, None, int(schedule),
                  int(bool(shrink)), int(penalty), int(chunk), float(l2))
    keep = None
    if w0 is not None:
        keep = np.ascontiguousarray(w0, dtype=np.float64)
        o.w0 = keep.ctypes.data
    return o, keep


# --------------------------------------------------------------------------
# entry points with the C names
# --------------------------------------------------------------------------
def pcdn_create(device: int = 0, hip_stream: int | None = None):
    L = load_library()
    h = ctypes.c_void_p()
    rc = L.pcdn_create(ctypes.byref(h), int(device), hip_stream)
    _check(None, rc)
    return h


def pcdn_destroy(ctx) -> None:
    load_library().pcdn_destroy(ctx)


def pcdn_last_error(ctx) -> str:
    m = load_library().pcdn_last_error(ctx)
    return m.decode() if m else ""


def pcdn_load_csc(ctx, n, p, col_ptr, row_idx, val, y) -> None:
    """Load X (CSC) and y; numpy arrays (host) or torch CUDA tensors (device)."""
    on_device = hasattr(col_ptr, "is_cuda") and col_ptr.is_cuda
    if not on_device:
        col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int64)
        row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.int8)
    nnz = int(col_ptr[-1])
    rc = load_library().pcdn_load_csc(ctx, int(n), int(p), nnz, _ptr(col_ptr), _ptr(row_idx),
                                      _ptr(val), _ptr(y), 1 if on_device else 0)
    _check(ctx, rc)


def pcdn_load_csc_bias(ctx, n, p, col_ptr, row_idx, val, y, bias: float) -> None:
    """pcdn_load_csc with a constant feature of value `bias` appended."""
    on_device = hasattr(col_ptr, "is_cuda") and col_ptr.is_cuda
    if not on_device:
        col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int64)
        row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.int8)
    nnz = int(col_ptr[-1])
    rc = load_library().pcdn_load_csc_bias(ctx, int(n), int(p), nnz, _ptr(col_ptr), _ptr(row_idx),
                                           _ptr(val), _ptr(y), 1 if on_device else 0, float(bias))
    _check(ctx, rc)


def pcdn_solve(ctx, C, P, eps, loss, p, **opts):
    """Returns (status, w, info dict)."""
    loss = LOSSES.get(loss, loss)
    o, keep = _opts(**opts)
    w = np.empty(int(p), dtype=np.float64)
    info = pcdn_info()
    rc = load_library().pcdn_solve(ctx, float(C), int(P), float(eps), int(loss),
                                   ctypes.byref(o), w.ctypes.data, ctypes.byref(info))
    _check(ctx, rc, (PCDN_OK, PCDN_NOT_CONVERGED))
    return rc, w, _info_dict(info)


def pcdn_solve_static(device, n, p, col_ptr, row_idx, val, y, C, P, eps, loss, w_out,
                      hip_stream=None, **opts):
    """The allocation-free solve: X (CSC), y and w_out are torch CUDA tensors
    (int64, int32, float32, int8, float64) on `device`.  Returns (status,
    info dict); w_out holds the solution."""
    for t, dt in ((col_ptr, "int64"), (row_idx, "int32"), (val, "float32"), (y, "int8"),
                  (w_out, "float64")):
        if not (hasattr(t, "is_cuda") and t.is_cuda and str(t.dtype).endswith(dt)
                and t.is_contiguous()):
            raise TypeError(f"pcdn_solve_static takes contiguous device tensors ({dt})")
    if w_out.numel() != int(p):
        raise ValueError("w_out must hold p entries")
    loss = LOSSES.get(loss, loss)
    o, keep = _opts(**opts)
    info = pcdn_info()
    nnz = int(row_idx.numel())
    rc = load_library().pcdn_solve_static(int(device), hip_stream, int(n), int(p), nnz,
                                          _ptr(col_ptr), _ptr(row_idx), _ptr(val), _ptr(y),
                                          float(C), int(P), float(eps), int(loss), ctypes.byref(o),
                                          _ptr(w_out), ctypes.byref(info))
    _check(None, rc, (PCDN_OK, PCDN_NOT_CONVERGED))
    return rc, _info_dict(info)


def _info_dict(info) -> dict:
    return {f: getattr(info, f) for f, _ in pcdn_info._fields_}


def pcdn_solve_batch(specs):
    """specs: list of dicts with keys ctx, C, P, eps, loss, p and optional
    opts (a dict of option keywords).  Returns a list of (status, w, info)."""
    n = len(specs)
    jobs = (pcdn_job * max(n, 1))()
    infos = [pcdn_info() for _ in range(n)]
    ws, keep = [], []
    for i, sp in enumerate(specs):
        o, k = _opts(**sp.get("opts", {}))
        keep.append((o, k))
        w = np.empty(int(sp["p"]), dtype=np.float64)
        ws.append(w)
        jobs[i].ctx = sp["ctx"]
        jobs[i].C = float(sp["C"])
        jobs[i].P = int(sp["P"])
        jobs[i].eps = float(sp["eps"])
        jobs[i].loss = int(LOSSES.get(sp["loss"], sp["loss"]))
        jobs[i].opts = ctypes.pointer(o)
        jobs[i].w_out = w.ctypes.data
        jobs[i].info = ctypes.pointer(infos[i])
    rc = load_library().pcdn_solve_batch(jobs, n)
    if rc != PCDN_OK:
        bad = next((sp["ctx"] for i, sp in enumerate(specs) if jobs[i].status == rc),
                   specs[0]["ctx"] if specs else None)
        _check(bad, rc)
    out = []
    for i in range(n):
        info = _info_dict(infos[i])
        info["P"] = jobs[i].P          # the autotuner's choice where P was 0
        out.append((jobs[i].status, ws[i], info))
    return out


def pcdn_autotune(ctx, C, eps, loss, **opts) -> dict:
    """Pilot-based bundle-size choice; returns the choice and every pilot."""
    loss = LOSSES.get(loss, loss)
    o, keep = _opts(**opts)
    t = pcdn_tune()
    _check(ctx, load_library().pcdn_autotune(ctx, int(loss), float(C), float(eps),
                                             ctypes.byref(o), ctypes.byref(t)))
    tried = [{f: getattr(t.tried[k], f) for f, _ in pcdn_tune_point._fields_}
             for k in range(t.n_tried)]
    return {"P": t.P, "schedule": t.schedule, "chunk": t.chunk,
            "predicted_seconds": t.predicted_seconds, "tried": tried}


def pcdn_iterate_batch(ctxs, Ps, k_first, iters, **opts):
    """Outer iterations of several contexts' current states together;
    returns each one's stopping norm after the last iteration."""
    n = len(ctxs)
    arr = (ctypes.c_void_p * max(n, 1))(*[c.value if hasattr(c, "value") else c for c in ctxs])
    P = (ctypes.c_int64 * max(n, 1))(*[int(x) for x in Ps])
    G = (ctypes.c_double * max(n, 1))()
    o, keep = _opts(**opts)
    rc = load_library().pcdn_iterate_batch(arr, P, n, int(k_first), int(iters), ctypes.byref(o), G)
    if rc != PCDN_OK:
        _check(ctxs[0] if n else None, rc)
    return [G[k] for k in range(n)]


def iterate_batch(solvers, Ps, k_first, iters, **opts):
    """pcdn_iterate_batch over Solver objects."""
    return pcdn_iterate_batch([s.ctx for s in solvers], Ps, k_first, iters, **opts)


def pcdn_solve_path(ctx, Cs, P, eps, loss, p, **opts):
    """Returns (status, W (len(Cs) x p), list of info dicts)."""
    loss = LOSSES.get(loss, loss)
    Cs = np.ascontiguousarray(Cs, dtype=np.float64)
    o, keep = _opts(**opts)
    W = np.empty((len(Cs), int(p)), dtype=np.float64)
    infos = (pcdn_info * max(len(Cs), 1))()
    rc = load_library().pcdn_solve_path(ctx, Cs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        len(Cs), int(P), float(eps), int(loss), ctypes.byref(o),
                                        W.ctypes.data, infos)
    _check(ctx, rc, (PCDN_OK, PCDN_NOT_CONVERGED))
    return rc, W, [_info_dict(infos[k]) for k in range(len(Cs))]


def pcdn_solve_path_lanes(ctxs, Cs, P, eps, loss, p, **opts):
    """The path over len(ctxs) contexts holding the same data (contiguous runs
    of Cs advanced together); returns (status, W, list of info dicts)."""
    loss = LOSSES.get(loss, loss)
    Cs = np.ascontiguousarray(Cs, dtype=np.float64)
    o, keep = _opts(**opts)
    W = np.empty((len(Cs), int(p)), dtype=np.float64)
    infos = (pcdn_info * max(len(Cs), 1))()
    arr = (ctypes.c_void_p * len(ctxs))(*ctxs)
    rc = load_library().pcdn_solve_path_lanes(arr, len(ctxs),
                                              Cs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              len(Cs), int(P), float(eps), int(loss),
                                              ctypes.byref(o), W.ctypes.data, infos)
    _check(ctxs[0], rc, (PCDN_OK, PCDN_NOT_CONVERGED))
    return rc, W, [_info_dict(infos[k]) for k in range(len(Cs))]


def pcdn_reset(ctx, loss, C, w=None) -> None:
    loss = LOSSES.get(loss, loss)
    keep = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    rc = load_library().pcdn_reset(ctx, int(loss), float(C),
                                   None if keep is None else keep.ctypes.data)
    _check(ctx, rc)


def pcdn_step(ctx, bundle, n, want=("g", "h", "d", "dtx"), **opts):
    bundle = np.ascontiguousarray(bundle, dtype=np.int32)
    P = len(bundle)
    o, _ = _opts(**opts)
    out = {k: np.empty(P if k != "dtx" else int(n)) for k in want}
    si = pcdn_step_info()
    rc = load_library().pcdn_step(ctx, bundle.ctypes.data, P, ctypes.byref(o), ctypes.byref(si),
                                  *[(_ptr(out[k]) if k in out else None)
                                    for k in ("g", "h", "d", "dtx")])
    _check(ctx, rc)
    out.update(alpha=si.alpha, delta=si.delta, dF=si.dF, q=si.q)
    return out


def pcdn_iterate(ctx, P, k_first, count, want_subgrad=True, **opts):
    """Run outer iterations from the current device state; returns the
    stopping norm after the last one (or None)."""
    o, _ = _opts(**opts)
    G = ctypes.c_double()
    rc = load_library().pcdn_iterate(ctx, int(P), int(k_first), int(count), ctypes.byref(o),
                                     ctypes.byref(G) if want_subgrad else None)
    _check(ctx, rc)
    return G.value if want_subgrad else None


def pcdn_permutation(ctx, seed, k, p) -> np.ndarray:
    out = np.empty(int(p), dtype=np.int32)
    _check(ctx, load_library().pcdn_permutation(ctx, int(seed), int(k), out.ctypes.data))
    return out


def pcdn_get_w(ctx, p) -> np.ndarray:
    out = np.empty(int(p))
    _check(ctx, load_library().pcdn_get_w(ctx, out.ctypes.data))
    return out


def pcdn_get_cache(ctx, n) -> np.ndarray:
    out = np.empty(int(n))
    _check(ctx, load_library().pcdn_get_cache(ctx, out.ctypes.data))
    return out


def pcdn_evaluate(ctx):
    F = ctypes.c_double()
    G = ctypes.c_double()
    _check(ctx, load_library().pcdn_evaluate(ctx, ctypes.byref(F), ctypes.byref(G)))
    return F.value, G.value


def pcdn_profile(ctx, mask: int) -> None:
    """mask: bit k brackets kernel class k with HIP events (0: off)."""
    _check(ctx, load_library().pcdn_profile(ctx, int(mask)))


def pcdn_profile_read(ctx, which: int):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    b = ctypes.c_double()
    _check(ctx, load_library().pcdn_profile_read(ctx, int(which), ctypes.byref(ms),
                                                 ctypes.byref(n), ctypes.byref(b)))
    return ms.value, n.value, b.value


# --------------------------------------------------------------------------
# convenience owner
# --------------------------------------------------------------------------
@dataclass
class Solver:
    """One library context holding one loaded problem."""
    device: int = 0
    hip_stream: int | None = None

    def __post_init__(self):
        self.ctx = pcdn_create(self.device, self.hip_stream)
        self.n = self.p = None

    def load(self, n, p, col_ptr, row_idx, val, y):
        pcdn_load_csc(self.ctx, n, p, col_ptr, row_idx, val, y)
        self.n, self.p = int(n), int(p)
        return self

    def load_data(self, d, bias=None):
        """Load a synth.Data; bias (a number): append the constant feature."""
        if bias is None:
            return self.load(d.n, d.p, d.col_ptr, d.row_idx, d.val, d.y)
        pcdn_load_csc_bias(self.ctx, d.n, d.p, d.col_ptr, d.row_idx, d.val, d.y, bias)
        self.n, self.p = int(d.n), int(d.p) + 1
        return self

    def solve(self, C, P, eps, loss, **opts):
        return pcdn_solve(self.ctx, C, P, eps, loss, self.p, **opts)

    def autotune(self, C, eps, loss, **opts):
        return pcdn_autotune(self.ctx, C, eps, loss, **opts)

    def solve_path(self, Cs, P, eps, loss, **opts):
        return pcdn_solve_path(self.ctx, Cs, P, eps, loss, self.p, **opts)

    def job(self, C, P, eps, loss, **opts) -> dict:
        """A job description for solve_batch()."""
        return {"ctx": self.ctx, "C": C, "P": P, "eps": eps, "loss": loss, "p": self.p,
                "opts": opts}

    def reset(self, loss, C, w=None):
        pcdn_reset(self.ctx, loss, C, w)

    def step(self, bundle, **opts):
        return pcdn_step(self.ctx, bundle, self.n, **opts)

    def iterate(self, P, k_first, count, want_subgrad=True, **opts):
        return pcdn_iterate(self.ctx, P, k_first, count, want_subgrad, **opts)

    def permutation(self, seed, k):
        return pcdn_permutation(self.ctx, seed, k, self.p)

    def w(self):
        return pcdn_get_w(self.ctx, self.p)

    def cache(self):
        return pcdn_get_cache(self.ctx, self.n)

    def evaluate(self):
        return pcdn_evaluate(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            pcdn_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(jobs):
    """Solve the jobs (from Solver.job) together; list of (status, w, info)."""
    return pcdn_solve_batch(jobs)


class Server:
    """Solve server with continuous batching (pcdn_server_*): submit()
    queues a problem, step() admits what fits the device-memory budget and
    runs one outer iteration of every admitted solve, take() returns a
    finished result.  The submitted arrays are kept referenced until taken."""

    def __init__(self, device: int = 0, budget_bytes: int = 64 << 30):
        L = load_library()
        h = ctypes.c_void_p()
        rc = L.pcdn_server_create(ctypes.byref(h), int(device), int(budget_bytes))
        if rc != PCDN_OK:
            raise PcdnError(rc, "pcdn_server_create failed")
        self.h = h
        self._keep = {}
        self._p = {}

    def _check(self, rc, allow=(PCDN_OK,)):
        if rc in allow:
            return rc
        m = load_library().pcdn_server_last_error(self.h)
        raise PcdnError(rc, m.decode() if m else "")

    def last_error(self) -> str:
        m = load_library().pcdn_server_last_error(self.h)
        return m.decode() if m else ""

    def submit(self, d, C, P, eps, loss, **opts) -> int:
        col_ptr = np.ascontiguousarray(d.col_ptr, dtype=np.int64)
        row_idx = np.ascontiguousarray(d.row_idx, dtype=np.int32)
        val = np.ascontiguousarray(d.val, dtype=np.float32)
        y = np.ascontiguousarray(d.y, dtype=np.int8)
        o, w0 = _opts(**opts)
        r = pcdn_request(int(d.n), int(d.p), int(col_ptr[-1]), col_ptr.ctypes.data,
                         row_idx.ctypes.data, val.ctypes.data, y.ctypes.data, float(C), int(P),
                         float(eps), int(LOSSES.get(loss, loss)), 0, ctypes.pointer(o))
        rid = ctypes.c_int64()
        self._check(load_library().pcdn_server_submit(self.h, ctypes.byref(r), ctypes.byref(rid)))
        self._keep[rid.value] = (col_ptr, row_idx, val, y, o, w0)
        self._p[rid.value] = int(d.p)
        return rid.value

    def step(self) -> int:
        fin = ctypes.c_int32()
        self._check(load_library().pcdn_server_step(self.h, ctypes.byref(fin)))
        return fin.value

    def status(self):
        w, r, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        self._check(load_library().pcdn_server_status(self.h, ctypes.byref(w), ctypes.byref(r),
                                                      ctypes.byref(b)))
        return w.value, r.value, b.value

    def take(self, rid):
        """(status, w, info) of a finished request, or None if it has not
        finished yet."""
        p = self._p.get(rid)
        w = np.empty(p) if p is not None else None
        info = pcdn_info()
        st = ctypes.c_int32()
        rc = load_library().pcdn_server_take(self.h, int(rid), None if w is None else w.ctypes.data,
                                             ctypes.byref(info), ctypes.byref(st))
        if rc == -5:
            return None
        self._check(rc)
        self._keep.pop(rid, None)
        self._p.pop(rid, None)
        return st.value, w, _info_dict(info)

    def close(self):
        if getattr(self, "h", None) is not None:
            load_library().pcdn_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
