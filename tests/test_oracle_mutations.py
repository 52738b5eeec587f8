"""The pins are sensitive: a plausible mistake planted in the oracle (on the
CPU) makes the corresponding pin fail."""
import numpy as np
import pytest

import oracle.bezier as obez
import oracle.bspline as obs
import oracle.camera as ocam
import oracle.render as orr
import test_oracle_pins as pins


def _fails(fn, *a):
    with pytest.raises(AssertionError):
        fn(*a)


def test_cox_de_boor_wrong_denominator(monkeypatch):
    good = obs.cox_de_boor

    def bad(x, t, p):                      # second weight uses t_{j+k} instead of t_{j+k+1}
        x = np.asarray(x, dtype=np.float64)
        t = np.asarray(t, dtype=np.float64)
        m = x.shape[0]
        N = np.zeros((m, p + 1))
        for j in range(p + 1):
            N[:, j] = (t[:, j] <= x) & (x < t[:, j + 1])
        for k in range(1, p + 1):
            Nn = np.zeros((m, p + 1 - k))
            for j in range(p + 1 - k):
                d1 = t[:, j + k] - t[:, j]
                d2 = t[:, j + k] - t[:, j + 1]
                w1 = np.divide(x - t[:, j], d1, out=np.zeros(m), where=d1 != 0)
                w2 = np.divide(t[:, j + k + 1] - x, d2, out=np.zeros(m), where=d2 != 0)
                Nn[:, j] = w1 * N[:, j] + w2 * N[:, j + 1]
            N = Nn
        return N[:, 0]

    monkeypatch.setattr(obs, "cox_de_boor", bad)
    _fails(pins.test_tensor_matches_scipy, (2, 2, 2), (4, 3, 5))
    monkeypatch.setattr(obs, "cox_de_boor", good)
    pins.test_tensor_matches_scipy((2, 2, 2), (4, 3, 5))


def test_missing_gamma_weight(monkeypatch):
    orig = obs.LREvaluator.partition_of_unity

    def no_gamma(self, x):
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        pt, bs, val = self.basis(x)
        return np.bincount(pt, weights=val, minlength=x.shape[0])

    monkeypatch.setattr(obs.LREvaluator, "partition_of_unity", no_gamma)
    _fails(pins.test_partition_of_unity, lambda: pins.lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=40, seed=8))
    monkeypatch.setattr(obs.LREvaluator, "partition_of_unity", orig)


def test_compositing_without_transmittance(monkeypatch):
    def bad(C, A, csrc, asrc, ds, xi):          # drops the (1 - alpha_dst) factor
        T = (1.0 - asrc) ** (ds / xi)
        C += (1.0 - T)[:, None] * csrc
        A += (1.0 - T)
        return T

    monkeypatch.setattr(orr, "composite", bad)
    _fails(pins.test_constant_field_closed_form, "adaptive")
    _fails(pins.test_over_operator)


def test_opacity_correction_exponent_inverted(monkeypatch):
    def bad(C, A, csrc, asrc, ds, xi):          # xi / ds instead of ds / xi
        T = (1.0 - asrc) ** (xi / ds)
        C += ((1.0 - T) * (1.0 - A))[:, None] * csrc
        A += (1.0 - T) * (1.0 - A)
        return T

    monkeypatch.setattr(orr, "composite", bad)
    _fails(pins.test_constant_field_closed_form, "fixed")


def test_bernstein_order_reversed(monkeypatch):
    good = obez.bernstein

    def bad(p, u):
        return good(p, u)[..., ::-1]

    monkeypatch.setattr(obez, "bernstein", bad)
    _fails(pins.test_bernstein_basis)


def test_extraction_axes_swapped(monkeypatch):
    good = obez.extract

    def bad(spline, ev, elems=None):
        C = good(spline, ev, elems)
        q = [v + 1 for v in spline.p]
        return C.reshape(C.shape[0], C.shape[1], q[2], q[1], q[0]).transpose(0, 1, 4, 3, 2).reshape(C.shape)

    monkeypatch.setattr(obez, "extract", bad)
    _fails(pins.test_extraction_closed_form, (2, 2, 2), (3, 3, 3), 40, "uniform")


def test_transfer_off_by_one(monkeypatch):
    good = orr.transfer

    def bad(v, lut, vmin, vmax):
        rgba, st = good(np.asarray(v) + 1.0 / 255.0 * (vmax - vmin), lut, vmin, vmax)
        return rgba, st

    monkeypatch.setattr(orr, "transfer", bad)
    _fails(pins.test_transfer_function)


def test_camera_axes_swapped(monkeypatch):
    good = ocam.primary_rays

    def bad(view, ii, jj):
        return good(view, jj % view.width, ii % view.height)

    monkeypatch.setattr(ocam, "primary_rays", bad)
    _fails(pins.test_perspective_rays_geometry)


def test_hue_sign_flipped(monkeypatch):
    good = orr.hue

    def bad(fx, fy):
        return good(fx, -fy)

    monkeypatch.setattr(orr, "hue", bad)
    _fails(pins.test_hsv_matches_colorsys)


def test_extraction_adjoint_untransposed(monkeypatch):
    """The adjoint must apply the transposed inverse collocation matrices."""
    def bad(spline, ev, G):
        p = tuple(int(v) for v in spline.p)
        n, nq = spline.elem_box.shape[0], spline.coef.shape[1]
        nodes = [obez.collocation_nodes(p[d]) for d in range(3)]
        Minv = [np.linalg.inv(obez.bernstein(p[d], nodes[d])) for d in range(3)]
        H = np.asarray(G).reshape(n, nq, p[2] + 1, p[1] + 1, p[0] + 1)
        H = np.einsum("kj,nqzyj->nqzyk", Minv[0], H)          # not transposed
        H = np.einsum("kj,nqzjx->nqzkx", Minv[1], H)
        H = np.einsum("kj,nqjyx->nqkyx", Minv[2], H)
        H = H.reshape(n, nq, -1).transpose(0, 2, 1).reshape(-1, nq)
        uz, uy, ux = np.meshgrid(nodes[2], nodes[1], nodes[0], indexing="ij")
        u = np.stack([ux.ravel(), uy.ravel(), uz.ravel()], axis=1)
        box = spline.elem_box
        x = (box[:, None, :3] + u[None] * (box[:, None, 3:] - box[:, None, :3])).reshape(-1, 3)
        pt, bs, val = ev.basis(x)
        out = np.zeros((spline.coef.shape[0], nq))
        for q in range(nq):
            out[:, q] = np.bincount(bs, weights=val * H[pt, q], minlength=out.shape[0])
        return out * spline.gamma[:, None]

    monkeypatch.setattr(obez, "extract_adjoint", bad)
    _fails(pins.test_extraction_adjoint_brute_force)
    _fails(pins.test_extraction_adjoint_of_point_evaluation, lambda: pins.workload("scalar_ortho64").spline)


def test_extraction_adjoint_without_gamma(monkeypatch):
    good = obez.extract_adjoint

    def bad(spline, ev, G):
        return good(spline, ev, G) / spline.gamma[:, None]

    monkeypatch.setattr(obez, "extract_adjoint", bad)
    _fails(pins.test_extraction_adjoint_of_point_evaluation, lambda: pins.lrgen.small_random(p=(2, 2, 2), n=(3, 3, 3), n_ref=40, seed=11))


def test_derivative_factor_wrong(monkeypatch):
    good = obs.cox_de_boor_derivative

    def bad(x, t, p):                      # factor p - 1 instead of p
        return good(x, t, p) * (p - 1) / p

    monkeypatch.setattr(obs, "cox_de_boor_derivative", bad)
    _fails(pins.test_gradient_of_reproduced_polynomial, (2, 2, 2), (3, 3, 3), 40, "uniform")


def test_illumination_unnormalised(monkeypatch):
    def bad(f, grad, ldir):                 # forgets to normalise the gradient
        n = grad[:, 0, :] if f.shape[1] == 1 else (f[:, :, None] * grad).sum(axis=1)
        return np.maximum(0.4, np.abs((n * ldir).sum(axis=1)))

    monkeypatch.setattr(orr, "illumination", bad)
    _fails(pins.test_illumination_of_linear_field, "lut")


def test_rk4_weight_misprinted(monkeypatch):
    import oracle.streamline as ost
    import test_oracle_streamlines as sp
    bad = dict(ost.TABLEAUS["rk4"])
    bad["b"] = np.array([1 / 6, 1 / 6, 1 / 2, 1 / 6])          # sums to 1, wrong order
    monkeypatch.setitem(ost.TABLEAUS, "rk4", bad)
    _fails(sp.test_convergence_order, "rk4", 4)


def test_heuristic_step_wrong_degree(monkeypatch):
    import oracle.streamline as ost
    import test_oracle_streamlines as sp
    good = ost.heuristic_ds

    def bad(elem_box, eidx, x, p_max):
        return good(elem_box, eidx, x, p_max - 1)

    monkeypatch.setattr(ost, "heuristic_ds", bad)
    _fails(sp.test_lr_streamline_converges_to_exact)


def test_positions_in_fp64(monkeypatch):
    """Sample positions computed in FP64 instead of the FP32 replay (R11)."""
    def bad(o, d, t):
        return np.clip(o.astype(np.float64) + t[:, None].astype(np.float64) * d.astype(np.float64), 0.0, 1.0)

    monkeypatch.setattr(orr, "positions", bad)
    _fails(pins.test_sample_positions_on_ray, "adaptive")


def test_positions_fused(monkeypatch):
    """o + t d rounded once (a fused multiply-add) instead of twice."""
    def bad(o, d, t):
        p = (o.astype(np.float64) + t[:, None].astype(np.float64) * d.astype(np.float64)).astype(np.float32)
        return np.clip(p, np.float32(0.0), np.float32(1.0))

    monkeypatch.setattr(orr, "positions", bad)
    _fails(pins.test_sample_positions_on_ray, "fixed")


def test_fixed_samples_at_segment_starts(monkeypatch):
    """Fixed steps sampled at the start of each segment instead of its midpoint."""
    def bad(t0, dsf, k):
        return t0 + np.float32(k) * dsf

    monkeypatch.setattr(orr, "fixed_sample_t", bad)
    _fails(pins.test_fixed_schedule_midpoints)


def test_fixed_samples_off_by_one(monkeypatch):
    """Fixed-step sample index shifted by one segment."""
    def bad(t0, dsf, k):
        return t0 + np.float32(k + 1.5) * dsf

    monkeypatch.setattr(orr, "fixed_sample_t", bad)
    _fails(pins.test_fixed_schedule_midpoints)


def test_ray_direction_normalised_in_fp64(monkeypatch):
    """Ray directions normalised in FP64 and rounded once instead of the FP32
    operation sequence."""
    good = ocam.primary_rays

    def bad(view, ii, jj):
        o, d, t0, t1, hit = good(view, ii, jj)
        if view.proj == "persp":
            sx = ((2 * np.asarray(ii) + 1) / view.width - 1.0) * float(view.tx)
            sy = (1.0 - (2 * np.asarray(jj) + 1) / view.height) * float(view.ty)
            dp = (view.fwd.astype(float) + sx[:, None] * view.right.astype(float)
                  + sy[:, None] * view.up.astype(float))
            d = (dp / np.linalg.norm(dp, axis=1, keepdims=True)).astype(np.float32)
        return o, d, t0, t1, hit

    monkeypatch.setattr(ocam, "primary_rays", bad)
    _fails(pins.test_ray_setup_exact_replay)


def test_fine_mode_too_coarse(monkeypatch):
    """Mode F with a step 16x coarser no longer is the limit of fine fixed steps."""
    monkeypatch.setattr(orr, "FINE_STEP", 2.0 ** -8)
    _fails(pins.test_fixed_steps_converge_to_fine_mode)
