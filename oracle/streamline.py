"""Streamlines of an LR-spline vector field by explicit Runge-Kutta methods,
FP64 (Sec. 5).

A streamline with seed x0 solves dx/dt = f(x), x(0) = x0 (Eq. 5).  One step of
an explicit RK method with tableau (A, b, c) is
    k_i = f(x_n + h sum_{j<i} a_ij k_j),   x_{n+1} = x_n + h sum_i b_i k_i   (Eq. 6).
Step sizes
  'heuristic'  h = base * 2^-d * (min side of the element holding x_n): the
               sampling distance of Eq. 4 used as the time step (Sec. 5.2); the
               element is found at x_n rounded to FP32, like the GPU's look-up.
  'constant'   h = base.
  'embedded'   error control with the embedded pair of HE, BS or RKF45: the
               higher-order solution is kept, err = |x_high - x_low|_2, the step
               is accepted when err <= tol (or h has reached H_MIN, or after
               MAX_REJECT rejections), and the next h is
               h * min(5, max(0.2, 0.9 (tol/err)^(1/q))), q the propagated
               order; the first h is the heuristic step at the seed.
Stage positions are clamped to [0,1]^3 before f is evaluated.  A line ends
when t reaches t_end (the last step is shortened to land on it), when a step
would leave [0,1]^3 (that step is not taken), or after max_samples points
(the seed included).

The error metric Eq. 7, E = max_j sum_i dt_i |x_j(t_i) - y_j(t_i)|_2, takes
x_j from a reference solution: RKF5 with a small constant step, evaluated at
the approximation's times by cubic Hermite interpolation of the reference
points and their derivatives.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np

H_MIN = 1e-14
MAX_REJECT = 64


def _tab(c, a, b, b_low=None, order=None):
    to = lambda v: np.array([float(Fr(x)) for x in v])
    A = np.zeros((len(c), len(c)))
    for i, row in enumerate(a):
        A[i + 1, :len(row)] = [float(Fr(x)) for x in row]
    return dict(c=to(c), A=A, b=to(b), b_low=None if b_low is None else to(b_low), order=order)


# Butcher tableaus of the methods compared in Sec. 5.4 (published coefficients).
TABLEAUS = {
    "rk1": _tab(["0"], [], ["1"], order=1),                                           # explicit Euler
    "rk2": _tab(["0", "1/2"], [["1/2"]], ["0", "1"], order=2),                        # midpoint
    "rk3": _tab(["0", "1/2", "1"], [["1/2"], ["-1", "2"]], ["1/6", "2/3", "1/6"], order=3),   # Kutta
    "rk4": _tab(["0", "1/2", "1/2", "1"], [["1/2"], ["0", "1/2"], ["0", "0", "1"]],
                ["1/6", "1/3", "1/3", "1/6"], order=4),
    "rk4_38": _tab(["0", "1/3", "2/3", "1"], [["1/3"], ["-1/3", "1"], ["1", "-1", "1"]],
                   ["1/8", "3/8", "3/8", "1/8"], order=4),
    # Fehlberg's 4(5) pair; 'rkf5' steps with its fifth-order weights
    "rkf5": _tab(["0", "1/4", "3/8", "12/13", "1", "1/2"],
                 [["1/4"], ["3/32", "9/32"], ["1932/2197", "-7200/2197", "7296/2197"],
                  ["439/216", "-8", "3680/513", "-845/4104"],
                  ["-8/27", "2", "-3544/2565", "1859/4104", "-11/40"]],
                 ["16/135", "0", "6656/12825", "28561/56430", "-9/50", "2/55"], order=5),
    "he": _tab(["0", "1"], [["1"]], ["1/2", "1/2"], b_low=["1", "0"], order=2),       # Heun-Euler 2(1)
    "bs": _tab(["0", "1/2", "3/4", "1"], [["1/2"], ["0", "3/4"], ["2/9", "1/3", "4/9"]],
               ["2/9", "1/3", "4/9", "0"], b_low=["7/24", "1/4", "1/3", "1/8"], order=3),   # Bogacki-Shampine 3(2)
}
TABLEAUS["rkf45"] = dict(TABLEAUS["rkf5"], b_low=np.array([float(Fr(x)) for x in
                                                           ["25/216", "0", "1408/2565", "2197/4104", "-1/5", "0"]]))
EMBEDDED = ("he", "bs", "rkf45")


def rk_step(f, x, h, tab):
    """One step of Eq. 6 for a batch x [m, 3] with steps h [m]; returns
    (x_high, x_low or None, k_1)."""
    s = tab["c"].shape[0]
    A = tab["A"]
    k = []
    for i in range(s):
        y = x.copy()
        for j in range(i):
            if A[i, j] != 0.0:
                y = y + (h * A[i, j])[:, None] * k[j]
        k.append(f(np.clip(y, 0.0, 1.0)))
    hi = x + h[:, None] * sum(tab["b"][i] * k[i] for i in range(s))
    lo = None
    if tab["b_low"] is not None:
        lo = x + h[:, None] * sum(tab["b_low"][i] * k[i] for i in range(s))
    return hi, lo, k[0]


def heuristic_ds(elem_box, eidx, x, p_max):
    """Eq. 4 sampling distance at x (element found at x rounded to FP32)."""
    x32 = np.clip(x, 0.0, 1.0).astype(np.float32)
    e = eidx.find(x32.astype(np.float64))
    b = elem_box[e].astype(np.float32)
    side = np.minimum(np.minimum(b[:, 3] - b[:, 0], b[:, 4] - b[:, 1]), b[:, 5] - b[:, 2])
    return (side * np.float32(2.0 ** -p_max)).astype(np.float64)


def _inside(x):
    return np.all((x >= 0.0) & (x <= 1.0), axis=1)


def integrate(f, seeds, method, step, base, t_end, max_samples, elem_box=None, eidx=None, p_max=2, tol=1e-6):
    """Streamlines of all seeds [m, 3] (FP64).  Returns (x [m, max_samples, 3],
    t [m, max_samples], count [m])."""
    tab = TABLEAUS[method]
    m = seeds.shape[0]
    X = np.zeros((m, max_samples, 3))
    T = np.zeros((m, max_samples))
    X[:, 0] = seeds
    cnt = np.ones(m, dtype=np.int64)
    x = np.asarray(seeds, dtype=np.float64).copy()
    t = np.zeros(m)
    active = np.ones(m, dtype=bool) & (max_samples > 1)
    h_next = None
    if step == "embedded":
        h_next = base * heuristic_ds(elem_box, eidx, x, p_max)
    while np.any(active):
        idx = np.nonzero(active & (t < t_end))[0]
        active[active & ~(t < t_end)] = False
        if idx.size == 0:
            break
        xi = x[idx]
        rem = t_end - t[idx]
        if step == "heuristic":
            h = np.minimum(base * heuristic_ds(elem_box, eidx, xi, p_max), rem)
            xn, _, _ = rk_step(f, xi, h, tab)
        elif step == "constant":
            h = np.minimum(np.full(idx.size, float(base)), rem)
            xn, _, _ = rk_step(f, xi, h, tab)
        else:
            h = np.minimum(h_next[idx], rem)
            xn = np.zeros_like(xi)
            done = np.zeros(idx.size, dtype=bool)
            rej = np.zeros(idx.size, dtype=np.int64)
            hn = np.zeros(idx.size)
            q = tab["order"]
            while not done.all():
                w = np.nonzero(~done)[0]
                hi, lo, _ = rk_step(f, xi[w], h[w], tab)
                err = np.sqrt(((hi - lo) ** 2).sum(axis=1))
                ok = (err <= tol) | (h[w] <= H_MIN) | (rej[w] >= MAX_REJECT)
                fac = np.where(err > 0, 0.9 * (tol / np.maximum(err, 1e-300)) ** (1.0 / q), 5.0)
                a = w[ok]
                xn[a] = hi[ok]
                hn[a] = h[a] * np.minimum(5.0, np.maximum(0.2, fac[ok]))
                done[a] = True
                r = w[~ok]
                h[r] = np.maximum(h[r] * np.maximum(0.2, fac[~ok]), H_MIN)
                rej[r] += 1
            h_next[idx] = hn
        inside = _inside(xn)
        active[idx[~inside]] = False
        g = idx[inside]
        x[g] = xn[inside]
        t[g] = t[g] + h[inside]
        X[g, cnt[g]] = x[g]
        T[g, cnt[g]] = t[g]
        cnt[g] += 1
        active[g[cnt[g] >= max_samples]] = False
    return X, T, cnt


def reference(f, seeds, t_end, h_ref):
    """RKF5 with the constant step h_ref from every seed (no domain stop):
    grid times, positions and velocities for Hermite interpolation."""
    n = int(np.ceil(t_end / h_ref))
    tab = TABLEAUS["rkf5"]
    m = seeds.shape[0]
    xs = np.zeros((n + 1, m, 3))
    ks = np.zeros((n + 1, m, 3))
    x = np.asarray(seeds, dtype=np.float64).copy()
    for i in range(n):
        xs[i] = x
        x, _, k1 = rk_step(f, x, np.full(m, h_ref), tab)
        ks[i] = k1
    xs[n] = x
    ks[n] = f(np.clip(x, 0.0, 1.0))
    return h_ref, xs, ks


def interpolate(ref, j, t):
    """Reference position of seed j at times t (cubic Hermite on the grid)."""
    h, xs, ks = ref
    i = np.minimum((t / h).astype(np.int64), xs.shape[0] - 2)
    s = (t - i * h) / h
    h00 = 2 * s ** 3 - 3 * s ** 2 + 1
    h10 = s ** 3 - 2 * s ** 2 + s
    h01 = -2 * s ** 3 + 3 * s ** 2
    h11 = s ** 3 - s ** 2
    return (h00[:, None] * xs[i, j] + (h10 * h)[:, None] * ks[i, j] + h01[:, None] * xs[i + 1, j]
            + (h11 * h)[:, None] * ks[i + 1, j])


def error_metric(ref, X, T, cnt):
    """Eq. 7 over the streamlines (X, T, cnt) of the seeds of `ref`."""
    worst = 0.0
    for j in range(X.shape[0]):
        n = int(cnt[j])
        if n < 2:
            continue
        t = T[j, 1:n]
        dt = np.diff(T[j, :n])
        d = np.sqrt(((X[j, 1:n] - interpolate(ref, j, t)) ** 2).sum(axis=1))
        worst = max(worst, float((dt * d).sum()))
    return worst
