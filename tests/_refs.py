"""Independent references used to pin the oracle.

Everything here is written from the paper's problem statement (eqs. (1)-(3),
Algorithm 1) in dense numpy or in mpmath multiprecision; nothing is shared with
``oracle/`` or with the GPU library.  These are deliberately different
computations: dense products instead of CSC sweeps, multiprecision instead of
FP64, direct objective evaluation instead of retained quantities, sign-pattern
enumeration instead of coordinate descent.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import mpmath
import numpy as np


# --------------------------------------------------------------------------
# objective in FP64 (dense) and in multiprecision
# --------------------------------------------------------------------------
def loss_vec(z, y, loss):
    m = y * z
    if loss == "lr":
        return np.logaddexp(0.0, -m)
    b = 1.0 - m
    return np.where(b > 0, b * b, 0.0)


def F_dense(X, y, w, C, loss, a=1.0, b=0.0):
    """a ||w||_1 + (b/2) ||w||^2 + C sum_i phi_i (eq. (1) for a = 1, b = 0)."""
    return float(a * np.abs(w).sum() + 0.5 * b * np.dot(w, w) + C * loss_vec(X @ w, y, loss).sum())


def _mp_loss(zm, yi, loss):
    if loss == "lr":
        return mpmath.log1p(mpmath.exp(-yi * zm))
    b = 1 - yi * zm
    return b * b if b > 0 else mpmath.mpf(0)


def F_mp(X, y, w, C, loss, dps=50, a=1, b=0):
    """F(w) in multiprecision from the dense matrix (entries taken exactly),
    with the regulariser a ||w||_1 + (b/2) ||w||^2."""
    with mpmath.workdps(dps):
        W = [mpmath.mpf(float(v)) for v in w]
        s = mpmath.mpf(0)
        for i in range(X.shape[0]):
            zi = mpmath.fsum(mpmath.mpf(float(X[i, j])) * W[j]
                             for j in range(X.shape[1]) if X[i, j] != 0)
            s += _mp_loss(zi, int(y[i]), loss)
        reg = mpmath.mpf(a) * mpmath.fsum(abs(v) for v in W)
        if b:
            reg += mpmath.mpf(b) / 2 * mpmath.fsum(v * v for v in W)
        return reg + mpmath.mpf(C) * s


def L_mp_shift(X, y, w, C, loss, j, eps, dps=60):
    """L(w + eps e_j) in multiprecision (eps may be an mpf)."""
    with mpmath.workdps(dps):
        W = [mpmath.mpf(float(v)) for v in w]
        W[j] += eps
        s = mpmath.mpf(0)
        for i in range(X.shape[0]):
            zi = mpmath.fsum(mpmath.mpf(float(X[i, k])) * W[k]
                             for k in range(X.shape[1]) if X[i, k] != 0)
            s += _mp_loss(zi, int(y[i]), loss)
        return mpmath.mpf(C) * s


def grad_hess_fd(X, y, w, C, loss, j, dps=60):
    """Central finite differences of L in multiprecision: (g_j, h_j)."""
    with mpmath.workdps(dps):
        e = mpmath.mpf("1e-15")
        Lp = L_mp_shift(X, y, w, C, loss, j, e, dps)
        L0 = L_mp_shift(X, y, w, C, loss, j, mpmath.mpf(0), dps)
        Lm = L_mp_shift(X, y, w, C, loss, j, -e, dps)
        g = (Lp - Lm) / (2 * e)
        h = (Lp - 2 * L0 + Lm) / (e * e)
        return float(g), float(h)


def loss_change_mp(loss, E, y, a, dps=60):
    """phi(z + a) - phi(z) with z = log E (LR) or b = cache (SVM), multiprecision."""
    with mpmath.workdps(dps):
        if loss == "lr":
            z = mpmath.log(mpmath.mpf(E))
            a = mpmath.mpf(a)
            return (mpmath.log1p(mpmath.exp(-y * (z + a)))
                    - mpmath.log1p(mpmath.exp(-y * z)))
        b = mpmath.mpf(E)
        bn = b - y * mpmath.mpf(a)
        return (bn * bn if bn > 0 else 0) - (b * b if b > 0 else 0)


# --------------------------------------------------------------------------
# the one-dimensional subproblem, eq. (4), minimised numerically
# --------------------------------------------------------------------------
def subproblem_value(g, h, w, d, a=1.0, b=0.0):
    """Eq. (4) with the regulariser a|u| + (b/2)u^2 in place of |u| (the
    constant R(w) dropped)."""
    return g * d + 0.5 * h * d * d + a * abs(w + d) + 0.5 * b * (w + d) ** 2


def golden_section_min(f, lo, hi, iters=400):
    invphi = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    c = b - invphi * (b - a)
    d = a + invphi * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(iters):
        if fc <= fd:
            b, d, fd = d, c, fc
            c = b - invphi * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + invphi * (b - a)
            fd = f(d)
        if b - a <= 1e-15 * (abs(a) + abs(b)):
            break
    return (a + b) / 2.0


# --------------------------------------------------------------------------
# Lemma 1(a): E[max_{j in B} lambda_j] over uniform P-subsets, closed form
# --------------------------------------------------------------------------
def lemma1a_expected_max(lams, P):
    lam = sorted(Fraction(x) for x in lams)
    p = len(lam)
    tot = Fraction(0)
    for k in range(P, p + 1):  # k-th smallest, 1-based
        tot += lam[k - 1] * math.comb(k - 1, P - 1)
    return float(tot / math.comb(p, P))


# --------------------------------------------------------------------------
# Algorithm 1 (CDN), with the 1-D Armijo search by direct multiprecision
# evaluation of F (no retained quantities)
# --------------------------------------------------------------------------
def cdn(X, y, C, loss, orders, sigma=0.01, beta=0.5, gamma=0.0, nu=1e-12, max_ls=30,
        a=1.0, b=0.0):
    n, p = X.shape
    w = np.zeros(p)
    for order in orders:
        for j in order:
            z = X @ w
            x = X[:, j]
            if loss == "lr":
                m = y * z
                err = 1.0 / (1.0 + np.exp(m))        # 1 - tau(y z)
                g = -C * np.sum(err * y * x)
                h = C * np.sum(err * (1.0 - err) * x * x)
            else:
                bz = 1.0 - y * z
                act = bz > 0
                g = -2.0 * C * np.sum((y * x * bz)[act])
                h = 2.0 * C * np.sum((x * x)[act])
            if h <= 0:
                h += nu
            # 1-D subproblem by numerical minimisation, then the kink if lower
            R = (abs(g) + a) / h + (1.0 + b / h) * abs(w[j]) + 1.0
            f = lambda dd: subproblem_value(g, h, w[j], dd, a, b)
            d = golden_section_min(f, -R, R)
            if f(-w[j]) <= f(d):
                d = -w[j]
            reg = lambda u: a * abs(u) + 0.5 * b * u * u
            delta = g * d + gamma * h * d * d + reg(w[j] + d) - reg(w[j])
            F0 = F_mp(X, y, w, C, loss, a=a, b=b)
            alpha = 1.0
            for _ in range(max_ls):
                wn = w.copy()
                wn[j] += alpha * d
                if F_mp(X, y, wn, C, loss, a=a, b=b) - F0 <= sigma * alpha * delta:
                    w = wn
                    break
                alpha *= beta
    return w


# --------------------------------------------------------------------------
# exact optimum of tiny problems by enumerating sign patterns
# --------------------------------------------------------------------------
def _smooth_min(Xs, y, C, loss, s, b=0.0):
    """argmin_v C sum phi(X_s v) + s.v + (b/2)||v||^2 by damped Newton; None if
    unbounded."""
    m = Xs.shape[1]
    v = np.zeros(m)

    def f(v):
        return C * loss_vec(Xs @ v, y, loss).sum() + s @ v + 0.5 * b * (v @ v)

    scale = 1.0 + C * np.abs(Xs).sum()
    for _ in range(500):
        z = Xs @ v
        if loss == "lr":
            err = 1.0 / (1.0 + np.exp(y * z))
            grad = -C * Xs.T @ (y * err) + s + b * v
            D = C * err * (1.0 - err)
        else:
            bb = 1.0 - y * z
            act = (bb > 0).astype(float)
            grad = -2.0 * C * Xs.T @ (y * bb * act) + s + b * v
            D = 2.0 * C * act
        if np.max(np.abs(grad)) <= 1e-13 * scale:
            return v
        H = Xs.T @ (D[:, None] * Xs) + b * np.eye(m)
        step = np.linalg.lstsq(H, -grad, rcond=1e-14)[0]
        if not np.all(np.isfinite(step)) or grad @ step >= 0:
            step = -grad
        fv, t = f(v), 1.0
        while t > 1e-20 and f(v + t * step) > fv + 1e-4 * t * (grad @ step):
            t *= 0.5
        if t <= 1e-20:
            return v
        v = v + t * step
        if np.max(np.abs(v)) > 1e7:
            return None
    return v


def brute_force_optimum(X, y, C, loss, a=1.0, b=0.0):
    """min F over w by enumerating sign patterns {-,0,+}^p (p <= 5); F with the
    regulariser a ||w||_1 + (b/2) ||w||^2."""
    n, p = X.shape
    best = F_dense(X, y, np.zeros(p), C, loss, a, b)
    best_w = np.zeros(p)
    for s in itertools.product((-1, 0, 1), repeat=p):
        s = np.array(s, dtype=float)
        S = np.flatnonzero(s)
        if len(S) == 0:
            continue
        v = _smooth_min(X[:, S], y, C, loss, a * s[S], b)
        if v is None or np.any(s[S] * v < -1e-12):
            continue
        w = np.zeros(p)
        w[S] = v
        Fw = F_dense(X, y, w, C, loss, a, b)
        if Fw < best:
            best, best_w = Fw, w
    return best, best_w


def ridge_optimum(X, y, C, loss, b):
    """min (b/2)||w||^2 + C sum phi (smooth and strongly convex): damped Newton
    over every feature at once."""
    w = _smooth_min(X, y, C, loss, np.zeros(X.shape[1]), b)
    return F_dense(X, y, w, C, loss, 0.0, b), w
