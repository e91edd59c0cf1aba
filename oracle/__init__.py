"""FP64 CPU oracle of PCDN -- test infrastructure only.

Thin ctypes wrapper over ``pcdn_oracle.c`` (plain C, single-threaded, FP64).
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the GPU library never does, and the two
share no code.  See ``pcdn_oracle.c`` for the paper passages each routine
follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcdn_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
# the same source built with OpenMP: the multicore CPU timing baseline only
# (its reductions over samples run in another order, so parity uses _SO)
_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")

LOGISTIC = 0
L2SVM = 1
_LOSS = {"lr": LOGISTIC, "logistic": LOGISTIC, "svm": L2SVM, "l2svm": L2SVM}
PENALTIES = {"l1": 0, "elastic": 1, "l2": 2}


def build(omp: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math);
    omp=True: the multicore timing build (-fopenmp)."""
    out = _SO_OMP if omp else _SO
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math"] + (["-fopenmp"] if omp else []) + ["-o", out, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _X(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_int64),
                ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class _Par(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_int32), ("max_ls", ctypes.c_int32),
                ("C", ctypes.c_double), ("sigma", ctypes.c_double),
                ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("nu", ctypes.c_double), ("shrink", ctypes.c_int32), ("penalty", ctypes.c_int32),
                ("l2", ctypes.c_double)]


class _StepInfo(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("delta", ctypes.c_double),
                ("dF", ctypes.c_double), ("q", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("margin", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("bundles", ctypes.c_int64), ("ls_steps", ctypes.c_int64),
                ("ls_fail", ctypes.c_int64), ("nnz_swept", ctypes.c_int64),
                ("objective", ctypes.c_double), ("subgrad", ctypes.c_double),
                ("subgrad0", ctypes.c_double), ("min_armijo_margin", ctypes.c_double),
                ("min_stop_margin", ctypes.c_double)]


_libs = {}


def threads_available(threads: int) -> int:
    """How many threads the multicore build runs with when asked for `threads`."""
    return int(lib(omp=True).orc_set_threads(int(threads)))


def lib(omp: bool = False):
    if omp in _libs:
        return _libs[omp]
    so = _SO_OMP if omp else _SO
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(_SRC):
        build(omp)
    L = ctypes.CDLL(so)
    vp, i64, i32, u64, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_uint64, ctypes.c_double)
    L.orc_splitmix64.argtypes = [u64, u64]
    L.orc_splitmix64.restype = u64
    L.orc_permutation.argtypes = [u64, i64, i64, vp]
    L.orc_permutation.restype = None
    L.orc_permutation_active.argtypes = [u64, i64, i64, vp, vp]
    L.orc_permutation_active.restype = i64
    L.orc_margins.argtypes = [vp, vp, vp]
    L.orc_cache_from_w.argtypes = [vp, i32, vp, vp]
    L.orc_grad_hess.argtypes = [vp, vp, vp, vp, i64, vp, vp]
    L.orc_newton_direction.argtypes = [dbl, dbl, dbl]
    L.orc_newton_direction.restype = dbl
    L.orc_newton_direction_reg.argtypes = [dbl, dbl, dbl, dbl, dbl]
    L.orc_newton_direction_reg.restype = dbl
    L.orc_subgrad_l1.argtypes = [vp, vp, vp, vp, vp]
    L.orc_subgrad_l1.restype = dbl
    L.orc_loss_change.argtypes = [i32, dbl, i32, dbl]
    L.orc_loss_change.restype = dbl
    L.orc_objective_cache.argtypes = [vp, vp, vp, vp]
    L.orc_objective_cache.restype = dbl
    L.orc_objective_direct.argtypes = [vp, vp, vp]
    L.orc_objective_direct.restype = dbl
    L.orc_step.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp]
    L.orc_step.restype = i32
    L.orc_solve.argtypes = [vp, vp, i64, dbl, u64, i32, vp, vp, vp]
    L.orc_solve.restype = i32
    L.orc_set_threads.argtypes = [i32]
    L.orc_set_threads.restype = i32
    _libs[omp] = L
    return L


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Problem:
    """A CSC design matrix with labels, held as contiguous numpy arrays."""
    n: int
    p: int
    col_ptr: np.ndarray  # int64[p+1]
    row_idx: np.ndarray  # int32[nnz]
    val: np.ndarray      # float32[nnz]
    y: np.ndarray        # int8[n]

    def __post_init__(self):
        self.col_ptr = np.ascontiguousarray(self.col_ptr, dtype=np.int64)
        self.row_idx = np.ascontiguousarray(self.row_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(self.val, dtype=np.float32)
        self.y = np.ascontiguousarray(self.y, dtype=np.int8)
        self._x = _X(self.n, self.p, _ptr(self.col_ptr), _ptr(self.row_idx),
                     _ptr(self.val), _ptr(self.y))

    @classmethod
    def from_data(cls, d) -> "Problem":
        return cls(int(d.n), int(d.p), d.col_ptr, d.row_idx, d.val, d.y)

    @property
    def ref(self):
        return ctypes.byref(self._x)

    @property
    def nnz(self) -> int:
        return int(self.col_ptr[-1])


@dataclass
class Params:
    loss: int = LOGISTIC
    C: float = 1.0
    sigma: float = 0.01
    beta: float = 0.5
    gamma: float = 0.0
    nu: float = 1e-12
    max_ls: int = 30
    shrink: bool = False
    penalty: int = 0     # "l1" (eq. (1)), "elastic" (|w| + l2/2 w^2) or "l2" (l2/2 w^2)
    l2: float = 0.0

    def __post_init__(self):
        if isinstance(self.loss, str):
            self.loss = _LOSS[self.loss]
        if isinstance(self.penalty, str):
            self.penalty = PENALTIES[self.penalty]

    def reg_ab(self) -> tuple:
        """(a, b) of the regulariser sum_j a |w_j| + (b/2) w_j^2."""
        return (0.0 if self.penalty == 2 else 1.0, 0.0 if self.penalty == 0 else float(self.l2))

    def c(self):
        return _Par(int(self.loss), int(self.max_ls), float(self.C), float(self.sigma),
                    float(self.beta), float(self.gamma), float(self.nu), int(bool(self.shrink)),
                    int(self.penalty), float(self.l2))


def splitmix64(seed: int, i: int) -> int:
    return int(lib().orc_splitmix64(seed, i))


def permutation(seed: int, k: int, p: int) -> np.ndarray:
    out = np.empty(p, dtype=np.int32)
    lib().orc_permutation(seed, k, p, _ptr(out))
    return out


def permutation_active(seed: int, k: int, active) -> tuple:
    """The partition restricted to the active features (shrinking): returns
    (permutation of all features, number of active ones leading it)."""
    active = np.ascontiguousarray(active, dtype=np.int8)
    out = np.empty(len(active), dtype=np.int32)
    n_act = lib().orc_permutation_active(seed, k, len(active), _ptr(active), _ptr(out))
    return out, int(n_act)


def margins(prob: Problem, w: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    z = np.empty(prob.n, dtype=np.float64)
    lib().orc_margins(prob.ref, _ptr(w), _ptr(z))
    return z


def cache_from_w(prob: Problem, loss, w: np.ndarray) -> np.ndarray:
    loss = _LOSS[loss] if isinstance(loss, str) else int(loss)
    w = np.ascontiguousarray(w, dtype=np.float64)
    c = np.empty(prob.n, dtype=np.float64)
    lib().orc_cache_from_w(prob.ref, loss, _ptr(w), _ptr(c))
    return c


def grad_hess(prob: Problem, par: Params, cache: np.ndarray, feats) -> tuple:
    feats = np.ascontiguousarray(feats, dtype=np.int32)
    cache = np.ascontiguousarray(cache, dtype=np.float64)
    g = np.empty(len(feats)); h = np.empty(len(feats))
    pc = par.c()
    lib().orc_grad_hess(prob.ref, ctypes.byref(pc), _ptr(cache), _ptr(feats),
                        len(feats), _ptr(g), _ptr(h))
    return g, h


def newton_direction(g: float, h: float, w: float, a: float = None, b: float = None) -> float:
    """Minimiser of g d + h d^2/2 + a|w+d| + (b/2)(w+d)^2; eq. (5) without a, b."""
    if a is None and b is None:
        return float(lib().orc_newton_direction(g, h, w))
    return float(lib().orc_newton_direction_reg(g, h, w, 1.0 if a is None else a,
                                                0.0 if b is None else b))


def subgrad_l1(prob: Problem, par: Params, w, cache, return_grad=False):
    w = np.ascontiguousarray(w, dtype=np.float64)
    cache = np.ascontiguousarray(cache, dtype=np.float64)
    g = np.empty(prob.p)
    pc = par.c()
    G = lib().orc_subgrad_l1(prob.ref, ctypes.byref(pc), _ptr(w), _ptr(cache), _ptr(g))
    return (G, g) if return_grad else G


def loss_change(loss, cache: float, y: int, a: float) -> float:
    """Per-sample loss change of the descent condition (see pcdn_oracle.c)."""
    loss = _LOSS[loss] if isinstance(loss, str) else int(loss)
    return float(lib().orc_loss_change(loss, float(cache), int(y), float(a)))


def objective_cache(prob: Problem, par: Params, w, cache) -> float:
    w = np.ascontiguousarray(w, dtype=np.float64)
    cache = np.ascontiguousarray(cache, dtype=np.float64)
    pc = par.c()
    return float(lib().orc_objective_cache(prob.ref, ctypes.byref(pc), _ptr(w), _ptr(cache)))


def objective_direct(prob: Problem, par: Params, w) -> float:
    w = np.ascontiguousarray(w, dtype=np.float64)
    pc = par.c()
    return float(lib().orc_objective_direct(prob.ref, ctypes.byref(pc), _ptr(w)))


def step(prob: Problem, par: Params, w: np.ndarray, cache: np.ndarray, bundle) -> dict:
    """One inner iteration; updates ``w`` and ``cache`` in place."""
    assert w.dtype == np.float64 and w.flags.c_contiguous
    assert cache.dtype == np.float64 and cache.flags.c_contiguous
    bundle = np.ascontiguousarray(bundle, dtype=np.int32)
    P = len(bundle)
    g = np.empty(P); h = np.empty(P); d = np.empty(P); dtx = np.empty(prob.n)
    si = _StepInfo()
    pc = par.c()
    q = lib().orc_step(prob.ref, ctypes.byref(pc), _ptr(w), _ptr(cache), _ptr(bundle), P,
                       _ptr(g), _ptr(h), _ptr(d), _ptr(dtx), ctypes.byref(si))
    return dict(q=int(q), alpha=si.alpha, delta=si.delta, dF=si.dF, margin=si.margin,
                g=g, h=h, d=d, dtx=dtx)


def solve(prob: Problem, par: Params, P: int, eps: float, seed: int = 0,
          max_outer: int = 1000, w0=None, threads: int = 0) -> tuple:
    """Algorithm 3 to the relative subgradient stopping rule; returns (w, info, F_trace).
    threads > 0 runs the multicore timing build on that many threads (its
    sums over samples run in another order: not the parity oracle)."""
    if not (1 <= P <= prob.p):
        raise ValueError("bundle size P must lie in [1, p]")
    w = np.zeros(prob.p) if w0 is None else np.array(w0, dtype=np.float64, copy=True)
    trace = np.zeros(max(max_outer, 1))
    info = _Info()
    pc = par.c()
    L = lib(omp=threads > 0)
    if threads > 0:
        L.orc_set_threads(int(threads))
    status = L.orc_solve(prob.ref, ctypes.byref(pc), int(P), float(eps), int(seed),
                             int(max_outer), _ptr(w), ctypes.byref(info), _ptr(trace))
    d = {f: getattr(info, f) for f, _ in _Info._fields_}
    d["status"] = int(status)
    return w, d, trace[: info.outer_iters].copy()
