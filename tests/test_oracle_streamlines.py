"""Pins of the streamline oracle (Sec. 5): the Runge-Kutta tableaus against
exact solutions of linear ODEs, the step rules, the stopping rules and the
error metric Eq. 7 against closed forms."""
import numpy as np
import pytest
from scipy.linalg import expm

import lrgen
from oracle import streamline as ost
from oracle.bspline import LREvaluator
from oracle.lookup import ElementIndex, find_element_scan

M = np.array([[-0.3, -1.0, 0.0], [1.0, -0.3, 0.0], [0.0, 0.0, 0.2]])
X0 = np.array([0.5, 0.5, 0.5])


def _affine(x):
    return (x - X0) @ M.T + np.array([0.0, 0.0, 0.05])


def _exact(seed, t):
    """x(t) of dx/dt = M (x - X0) + v (closed form through the matrix exponential)."""
    v = np.array([0.0, 0.0, 0.05])
    z0 = seed - X0 + np.linalg.solve(M, v)
    return X0 - np.linalg.solve(M, v) + expm(M * t) @ z0


@pytest.mark.parametrize("method", list(ost.TABLEAUS))
def test_tableau_consistency(method):
    tab = ost.TABLEAUS[method]
    assert np.allclose(tab["A"].sum(axis=1), tab["c"], atol=1e-15)
    assert abs(tab["b"].sum() - 1.0) < 1e-15
    if tab["b_low"] is not None:
        assert abs(tab["b_low"].sum() - 1.0) < 1e-15


@pytest.mark.parametrize("method,order", [("rk1", 1), ("rk2", 2), ("rk3", 3), ("rk4", 4), ("rk4_38", 4),
                                          ("rkf5", 5), ("he", 2), ("bs", 3), ("rkf45", 5)])
def test_convergence_order(method, order):
    """Global error at t = 1 on a linear ODE against expm: halving h divides it
    by 2^order (Eq. 6 with the published tableau)."""
    seed = np.array([[0.7, 0.45, 0.3]])
    ref = _exact(seed[0], 1.0)
    errs = []
    for h in (1 / 16, 1 / 32):
        X, T, cnt = ost.integrate(_affine, seed, method, "constant", h, 1.0, 10000)
        assert abs(T[0, cnt[0] - 1] - 1.0) < 1e-14
        errs.append(np.linalg.norm(X[0, cnt[0] - 1] - ref))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - order) < 0.35, rate


def test_embedded_low_order_is_one_less():
    for method, order in (("he", 1), ("bs", 2), ("rkf45", 4)):
        tab = dict(ost.TABLEAUS[method])
        tab["b"], tab["b_low"] = tab["b_low"], None
        seed = np.array([[0.7, 0.45, 0.3]])
        errs = []
        for h in (1 / 16, 1 / 32):
            x = seed.copy()
            for _ in range(int(round(1 / h))):
                x, _, _ = ost.rk_step(_affine, x, np.array([h]), tab)
            errs.append(np.linalg.norm(x[0] - _exact(seed[0], 1.0)))
        assert abs(np.log2(errs[0] / errs[1]) - order) < 0.35


def _linear_lr(ncomp=3):
    """An LR-spline reproducing the affine field exactly (degree 2 reproduces
    polynomials of degree 1: coefficients = field at the Greville points)."""
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=40, seed=25)
    return s.with_coef(_affine(s.greville()))


def test_lr_streamline_converges_to_exact():
    """Heuristic steps (Eq. 4 as h) through an LR-spline that reproduces the
    affine field: RK4 error against the closed form falls like base^4."""
    s = _linear_lr()
    ev = LREvaluator(s)
    ei = ElementIndex(s.elem_box)
    f = lambda x: ev.evaluate(x)
    seeds = np.array([[0.6, 0.5, 0.3], [0.55, 0.35, 0.2], [0.4, 0.6, 0.5]])
    errs = []
    for base in (4.0, 2.0):
        X, T, cnt = ost.integrate(f, seeds, "rk4", "heuristic", base, 0.5, 4000, elem_box=s.elem_box, eidx=ei)
        e = max(np.linalg.norm(X[j, cnt[j] - 1] - _exact(seeds[j], T[j, cnt[j] - 1])) for j in range(3))
        errs.append(e)
        # every step is base * 2^-2 * min side of the element at the start (or the final clip)
        d = np.diff(T[0, :cnt[0]])
        e = find_element_scan(s.elem_box, X[0, :cnt[0] - 1].astype(np.float32).astype(np.float64))
        hs = base * (s.elem_box[e, 3:] - s.elem_box[e, :3]).min(axis=1) / 4.0     # Eq. 4, d = 2
        assert np.all((d == hs) | ((d < hs) & (np.arange(d.size) == d.size - 1)))
    assert errs[1] < errs[0] / 8


def test_stopping_rules():
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=20, seed=26)
    const = np.tile([0.8, 0.0, 0.1], (s.n_bspl, 1))
    s = s.with_coef(const)
    ev = LREvaluator(s)
    ei = ElementIndex(s.elem_box)
    f = lambda x: ev.evaluate(x)
    seeds = np.array([[0.5, 0.5, 0.5], [0.1, 0.2, 0.3]])
    X, T, cnt = ost.integrate(f, seeds, "rk2", "heuristic", 1.0, 10.0, 100000, elem_box=s.elem_box, eidx=ei)
    for j in range(2):                       # the domain exit ends the line, inside [0,1]^3
        n = cnt[j]
        assert np.all((X[j, :n] >= 0) & (X[j, :n] <= 1))
        assert 1.0 - X[j, n - 1, 0] < 1.0001 * 0.8 * base_step(s, ei, X[j, n - 1])
        assert np.allclose(X[j, n - 1] - seeds[j], [0.8 * T[j, n - 1], 0, 0.1 * T[j, n - 1]], atol=1e-12)
    X, T, cnt = ost.integrate(f, seeds, "rk2", "heuristic", 1.0, 0.05, 100000, elem_box=s.elem_box, eidx=ei)
    assert np.all(T[np.arange(2), cnt - 1] == 0.05)          # the time limit is landed on
    X, T, cnt = ost.integrate(f, seeds, "rk2", "heuristic", 1.0, 10.0, 7, elem_box=s.elem_box, eidx=ei)
    assert np.all(cnt == 7)                                  # the sample cap (seed included)


def base_step(s, ei, x):
    e = find_element_scan(s.elem_box, x[None].astype(np.float32).astype(np.float64))[0]
    return (s.elem_box[e, 3:] - s.elem_box[e, :3]).min() / 4.0


def test_embedded_tolerance_controls_error():
    s = _linear_lr()
    ev = LREvaluator(s)
    ei = ElementIndex(s.elem_box)
    f = lambda x: ev.evaluate(x)
    seeds = np.array([[0.6, 0.5, 0.3], [0.55, 0.35, 0.2]])
    errs = []
    for tol in (1e-5, 1e-8):
        X, T, cnt = ost.integrate(f, seeds, "rkf45", "embedded", 1.0, 0.5, 4000, elem_box=s.elem_box, eidx=ei,
                                  tol=tol)
        errs.append(max(np.linalg.norm(X[j, cnt[j] - 1] - _exact(seeds[j], T[j, cnt[j] - 1])) for j in range(2)))
    assert errs[1] < errs[0] / 20 and errs[1] < 1e-7


def test_error_metric_closed_form():
    """Eq. 7 against a trajectory offset by a known constant: E = |offset| t_end;
    the exact trajectory scores ~0 through the Hermite-interpolated reference."""
    seeds = np.array([[0.7, 0.45, 0.3], [0.4, 0.6, 0.5]])
    ref = ost.reference(_affine, seeds, 1.0, 1e-3)
    t = np.linspace(0, 1.0, 41)
    X = np.stack([np.stack([_exact(sd, ti) for ti in t]) for sd in seeds])
    T = np.tile(t, (2, 1))
    cnt = np.array([41, 41])
    assert ost.error_metric(ref, X, T, cnt) < 1e-12
    off = np.array([3e-3, -4e-3, 0.0])
    X2 = X + off
    X2[1] = X[1]
    assert abs(ost.error_metric(ref, X2, T, cnt) - 5e-3 * 1.0) < 1e-12
