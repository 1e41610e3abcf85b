"""Pins of the FP64 oracle to things other than itself: library routines,
closed forms, invariants and brute force on tiny inputs.  CPU only.

Each test names the passage of the paper (arXiv 2206.05047) it pins and what
a plausible mistake in the oracle would make it fail.
"""
import itertools

import numpy as np
import pytest
from scipy import ndimage, optimize

import oracle
from helpers import motion_kernel

TINY = dict(U=3, V=3, sy=6, sx=7, zeta=2, kb=5, sigma_b=1.0, lambda1=1.0, lambda2=1.0, win=3,
            sigma_s=1.0, sigma_e=1.0, theta=1.0, n_iter=5, cg_iter=5)


def _o(**kw):
    c = dict(TINY)
    c.update(kw)
    return oracle.Oracle(c)


def _rng(seed=0):
    return np.random.default_rng(seed)


def _disp_smooth(o, rng, amp=1.3):
    H, W = o.hr_shape
    yy, xx = np.mgrid[0:H, 0:W]
    return amp * np.sin(0.37 * yy + 0.21 * xx + rng.uniform(0, 6))


def _disp_steps(o, rng):
    H, W = o.hr_shape
    d = np.full((H, W), rng.uniform(-1.7, 1.7))
    d[H // 3:, W // 2:] = rng.uniform(-1.7, 1.7)
    d[: H // 2, : W // 3] = rng.uniform(-1.7, 1.7)
    return d


# ---------------------------------------------------------------- blur (sec 4.1)

def test_blur_kernel_is_normalised_separable_gaussian():
    o = _o(kb=7, sigma_b=1.3)
    h = o.blur_kernel()
    a = np.arange(-3, 4)
    g = np.exp(-a ** 2 / (2 * 1.3 ** 2))
    g /= g.sum()
    np.testing.assert_allclose(h, np.outer(g, g), rtol=0, atol=1e-15)
    assert abs(h.sum() - 1) < 1e-14


def test_blur_equals_scipy_correlate_zero_padding():
    o = _o(kb=5, sigma_b=1.1)
    x = _rng(1).standard_normal(o.hr_shape)
    ref = ndimage.correlate(x, o.blur_kernel(), mode="constant", cval=0.0)
    np.testing.assert_allclose(o.blur(x), ref, rtol=0, atol=1e-14)


def test_blur_delta_response_is_kernel():
    o = _o(sy=9, sx=9, kb=5)
    x = np.zeros(o.hr_shape)
    x[9, 9] = 1.0
    out = o.blur(x)
    np.testing.assert_allclose(out[7:12, 7:12], o.blur_kernel()[::-1, ::-1], atol=1e-15)
    assert abs(out.sum() - 1) < 1e-14


def test_blur_adjoint():
    o = _o(kb=7, sigma_b=1.5)
    rng = _rng(2)
    x, y = rng.standard_normal(o.hr_shape), rng.standard_normal(o.hr_shape)
    lhs, rhs = np.vdot(o.blur(x), y), np.vdot(x, o.blur_t(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ---------------------------------------------------------------- D (sec 4.1)

def test_down_is_top_left_of_block_and_up_is_its_transpose():
    o = _o(zeta=3)
    rng = _rng(3)
    x = rng.standard_normal(o.hr_shape)
    np.testing.assert_array_equal(o.down(x), x[::3, ::3])
    lr = rng.standard_normal((o.pb.sy, o.pb.sx))
    np.testing.assert_array_equal(o.down(o.up(lr)), lr)          # D D^T = I
    mask = np.zeros(o.hr_shape)
    mask[::3, ::3] = 1
    np.testing.assert_array_equal(o.up(o.down(x)), mask * x)    # D^T D = lattice mask


# ---------------------------------------------------------------- W_k (sec 4.1)

@pytest.mark.parametrize("k", range(9))
def test_warp_integer_disparity_is_zero_filled_shift(k):
    o = _o(sy=8, sx=9)
    x = _rng(4).standard_normal(o.hr_shape)
    disp = np.full(o.hr_shape, 2.0)
    tau, rho = o.view_offset(k)
    sy, sx = int(2 * tau), int(2 * rho)
    H, W = o.hr_shape
    ref = np.zeros_like(x)
    ys = slice(max(0, -sy), min(H, H - sy))
    xs = slice(max(0, -sx), min(W, W - sx))
    ref[ys, xs] = x[ys.start + sy: ys.stop + sy, xs.start + sx: xs.stop + sx]
    np.testing.assert_array_equal(o.warp(x, disp, k), ref)


def test_view_offsets_centre_is_reference():
    o = _o(U=5, V=3)
    offs = [o.view_offset(k) for k in range(15)]
    assert offs[7] == (0, 0)
    assert offs[0] == (-2, -1) and offs[14] == (2, 1)
    assert offs[1] == (-2, 0)  # row-major: column index moves fastest


@pytest.mark.parametrize("kind", ["smooth", "steps"])
def test_warp_equals_scipy_map_coordinates(kind):
    o = _o(U=3, V=5, sy=7, sx=8)
    rng = _rng(5)
    x = rng.standard_normal(o.hr_shape)
    disp = _disp_smooth(o, rng) if kind == "smooth" else _disp_steps(o, rng)
    H, W = o.hr_shape
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    for k in range(o.pb.sk):
        tau, rho = o.view_offset(k)
        ref = ndimage.map_coordinates(x, [yy + tau * disp, xx + rho * disp], order=1,
                                      mode="grid-constant", cval=0.0)
        np.testing.assert_allclose(o.warp(x, disp, k), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind", ["smooth", "steps"])
def test_warp_adjoint(kind):
    o = _o(U=5, V=5, sy=9, sx=8)
    rng = _rng(6)
    disp = _disp_smooth(o, rng, 1.7) if kind == "smooth" else _disp_steps(o, rng)
    for k in (0, 7, 12, 24):
        x, u = rng.standard_normal(o.hr_shape), rng.standard_normal(o.hr_shape)
        lhs, rhs = np.vdot(o.warp(x, disp, k), u), np.vdot(x, o.warp_t(u, disp, k))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_warp_transpose_matches_dense_matrix():
    o = _o(U=3, V=3, sy=4, sx=5)
    rng = _rng(7)
    disp = _disp_steps(o, rng)
    n = o.pb.H * o.pb.W
    eye = np.eye(n)
    k = 2
    Wd = np.stack([o.warp(eye[i].reshape(o.hr_shape), disp, k).ravel() for i in range(n)], axis=1)
    WTd = np.stack([o.warp_t(eye[i].reshape(o.hr_shape), disp, k).ravel() for i in range(n)], axis=1)
    np.testing.assert_allclose(WTd, Wd.T, atol=1e-15)


# ---------------------------------------------------------------- A_k = D B W_k (sec 3.1)

def test_forward_is_composition_down_blur_warp():
    o = _o(U=3, V=3, sy=6, sx=5, zeta=3, kb=7, sigma_b=1.5)
    rng = _rng(8)
    x = rng.standard_normal(o.hr_shape)
    disp = _disp_smooth(o, rng)
    t = o.forward(x, disp)
    for k in range(9):
        np.testing.assert_allclose(t[k], o.down(o.blur(o.warp(x, disp, k))), atol=1e-14)


@pytest.mark.parametrize("zeta,kb", [(2, 5), (3, 9), (4, 7)])
def test_forward_adjoint_all_views(zeta, kb):
    o = _o(U=3, V=5, sy=5, sx=6, zeta=zeta, kb=kb, sigma_b=1.2)
    rng = _rng(9 + zeta)
    disp = _disp_steps(o, rng)
    x = rng.standard_normal(o.hr_shape)
    e = rng.standard_normal(o.lr_shape)
    lhs, rhs = np.vdot(o.forward(x, disp), e), np.vdot(x, o.adjoint(e, disp))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_forward_per_view_disparity_maps():
    o = _o(U=3, V=3, n_disp=9)
    rng = _rng(10)
    disps = np.stack([_disp_smooth(o, rng) for _ in range(9)])
    x = rng.standard_normal(o.hr_shape)
    t = o.forward(x, disps)
    o1 = _o(U=3, V=3)
    for k in (0, 4, 8):
        np.testing.assert_allclose(t[k], o1.forward(x, disps[k])[k], atol=1e-14)
    e = rng.standard_normal(o.lr_shape)
    lhs, rhs = np.vdot(t, e), np.vdot(x, o.adjoint(e, disps))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ---------------------------------------------------------------- weights (sec 3.4)

def test_spatial_weight_decreases_with_distance():
    o = _o(sigma_s=2.5)
    assert o.spatial_weight(0, 1) == pytest.approx(np.exp(-1 / 2.5), rel=1e-15)
    assert o.spatial_weight(2, -1) == pytest.approx(np.exp(-5 / 2.5), rel=1e-15)
    assert o.spatial_weight(1, 1) < o.spatial_weight(0, 1)


def test_edge_weight_on_linear_ramp():
    o = _o(sigma_e=0.7)
    H, W = o.hr_shape
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    a, b = 0.3, -0.2
    x = a * xx + b * yy
    occ = _rng(11).uniform(0.2, 1.0, size=(H, W))
    m = o.edge_weight(x, occ)
    exp_int = np.exp(-(a * a + b * b) / 0.7)
    np.testing.assert_allclose(m[:-1, :-1], exp_int * occ[:-1, :-1], rtol=1e-14)
    np.testing.assert_allclose(m[:-1, -1], np.exp(-(b * b) / 0.7) * occ[:-1, -1], rtol=1e-14)
    np.testing.assert_allclose(m[-1, :-1], np.exp(-(a * a) / 0.7) * occ[-1, :-1], rtol=1e-14)
    assert m[-1, -1] == pytest.approx(occ[-1, -1], rel=1e-15)


def test_edge_weight_off_when_sigma_inf():
    o = _o(sigma_e=float("inf"))
    x = _rng(12).standard_normal(o.hr_shape)
    np.testing.assert_array_equal(o.edge_weight(x), np.ones(o.hr_shape))


# ---------------------------------------------------------------- S, S^T (sec 3.4, 4.1)

def test_nltv_offsets_full_window_without_centre():
    o = _o(win=5)
    offs = [o.offset(d) for d in range(24)]
    assert len(set(offs)) == 24 and (0, 0) not in offs
    assert offs[0] == (-2, -2) and offs[23] == (2, 2) and offs[12] == (0, 1)


def test_regulariser_equals_pairwise_definition_brute_force():
    """sec 3.4: R(x) = sum_u sum_{v in N(u)} w(u,v) |x_u - x_v| with
    w(u,v) = w_d(u-v...) * m(u): brute force over all pixel pairs."""
    o = _o(sy=4, sx=5, win=5, sigma_s=1.7)
    rng = _rng(13)
    x = rng.standard_normal(o.hr_shape)
    m = rng.uniform(0.1, 1.0, size=o.hr_shape)
    H, W = o.hr_shape
    R = 0.0
    for (Y, X), (Y2, X2) in itertools.product(itertools.product(range(H), range(W)), repeat=2):
        dy, dx = Y2 - Y, X2 - X
        if (dy, dx) == (0, 0) or abs(dy) > 2 or abs(dx) > 2:
            continue
        R += np.exp(-(dy * dy + dx * dx) / 1.7) * m[Y, X] * abs(x[Y, X] - x[Y2, X2])
    assert np.abs(o.nltv_grad(x, m)).sum() == pytest.approx(R, rel=1e-13)


def test_nltv_adjoint_and_constant_kernel():
    o = _o(sy=7, sx=6, win=5)
    rng = _rng(14)
    m = rng.uniform(0.1, 1.0, size=o.hr_shape)
    x = rng.standard_normal(o.hr_shape)
    g = rng.standard_normal((o.pb.sd,) + o.hr_shape)
    lhs, rhs = np.vdot(o.nltv_grad(x, m), g), np.vdot(x, o.nltv_div(g, m))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    np.testing.assert_array_equal(o.nltv_grad(np.full(o.hr_shape, 3.25), m), 0.0)
    # 1^T S^T g = 0 for every g (the divergence has zero mean)
    assert abs(o.nltv_div(g, m).sum()) < 1e-11


# ---------------------------------------------------------------- prox (sec 4)

def test_soft_threshold_closed_form_and_clip_identity():
    o = _o()
    t = 0.7
    for u in [-2.0, -0.7, -0.3, 0.0, 0.2, 0.7, 1.9]:
        s = o.soft(u, t)
        assert s == pytest.approx(np.sign(u) * max(abs(u) - t, 0.0), abs=0)
        assert u - s == pytest.approx(np.clip(u, -t, t), abs=1e-15)


@pytest.mark.parametrize("u,theta", [(1.3, 2.0), (-0.2, 2.0), (0.45, 2.0), (-3.0, 0.5)])
def test_soft_threshold_minimises_prox_objective_brute_force(u, theta):
    """sec 4: z = argmin |z| + (theta/2)(z-u)^2, found on a fine grid."""
    o = _o()
    grid = np.linspace(-5, 5, 2000001)
    z_bf = grid[np.argmin(np.abs(grid) + 0.5 * theta * (grid - u) ** 2)]
    assert o.soft(u, 1.0 / theta) == pytest.approx(z_bf, abs=1e-5)


# ---------------------------------------------------------------- x0 (sec 5)

def test_bicubic_interpolates_and_reproduces_quadratics():
    """Keys' a=-1/2 cubic convolution passes through the samples and is exact
    for polynomials of degree <= 2 (away from the clamped border)."""
    o = _o(sy=10, sx=12, zeta=3)
    rng = _rng(15)
    lr = rng.standard_normal((10, 12))
    x0 = o.bicubic(lr)
    np.testing.assert_allclose(x0[::3, ::3], lr, atol=1e-14)
    ii, jj = np.mgrid[0:10, 0:12].astype(float)
    q = 0.3 + 0.2 * ii - 0.1 * jj + 0.05 * ii * ii - 0.03 * ii * jj + 0.02 * jj * jj
    x0 = o.bicubic(q)
    Y, X = np.mgrid[0:30, 0:36].astype(float) / 3.0
    qhr = 0.3 + 0.2 * Y - 0.1 * X + 0.05 * Y * Y - 0.03 * Y * X + 0.02 * X * X
    np.testing.assert_allclose(x0[3:25, 3:31], qhr[3:25, 3:31], atol=1e-12)


# ---------------------------------------------------------------- x-step (sec 5, Alg. 2)

def _dense(fn, n, shape):
    eye = np.eye(n)
    return np.stack([np.asarray(fn(eye[i].reshape(shape))).ravel() for i in range(n)], axis=1)


def test_normal_operator_matches_dense_composition():
    """sec 5: G^T G = (lambda2 + vartheta lambda1^2/2) A^T A + (vartheta/2) S^T S."""
    o = _o(sy=3, sx=4, lambda1=0.8, lambda2=1.7, theta=1.3)
    rng = _rng(16)
    disp = _disp_smooth(o, rng)
    m = rng.uniform(0.2, 1.0, size=o.hr_shape)
    n = o.pb.H * o.pb.W
    A = _dense(lambda v: o.forward(v, disp), n, o.hr_shape)
    S = _dense(lambda v: o.nltv_grad(v, m), n, o.hr_shape)
    Hd = (1.7 + 0.5 * 1.3 * 0.8 ** 2) * A.T @ A + 0.5 * 1.3 * S.T @ S
    Hn = _dense(lambda v: o.normal_apply(disp, m, v), n, o.hr_shape)
    np.testing.assert_allclose(Hn, Hd, atol=1e-12)


def test_cg_full_steps_solves_dense_system():
    o = _o(sy=3, sx=3, cg_iter=200, lambda2=2.0, lambda1=0.5)
    rng = _rng(17)
    disp = _disp_smooth(o, rng)
    m = rng.uniform(0.5, 1.0, size=o.hr_shape)
    n = o.pb.H * o.pb.W
    Hd = _dense(lambda v: o.normal_apply(disp, m, v), n, o.hr_shape)
    v = rng.standard_normal(o.hr_shape)
    delta, pi, steps = o.cg(disp, m, v)
    ref = np.linalg.solve(Hd, -v.ravel())
    np.testing.assert_allclose(delta.ravel(), ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    assert steps <= 200 and pi < 1e-20


def test_cg_energy_error_decreases():
    o = _o(sy=4, sx=4, cg_iter=1)
    rng = _rng(18)
    disp = _disp_smooth(o, rng)
    m = rng.uniform(0.5, 1.0, size=o.hr_shape)
    n = o.pb.H * o.pb.W
    Hd = _dense(lambda v: o.normal_apply(disp, m, v), n, o.hr_shape)
    v = rng.standard_normal(o.hr_shape)
    ref = np.linalg.solve(Hd, -v.ravel())
    errs = []
    for K in range(0, 8):
        oK = _o(sy=4, sx=4, cg_iter=K)
        d, _, _ = oK.cg(disp, m, v)
        e = d.ravel() - ref
        errs.append(e @ Hd @ e)
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_cg_zero_rhs_takes_no_step():
    o = _o()
    delta, pi, steps = o.cg(np.zeros(o.hr_shape), np.ones(o.hr_shape), np.zeros(o.hr_shape))
    assert steps == 0 and pi == 0.0 and not delta.any()


# ---------------------------------------------------------------- ADMM (sec 5, Alg. 1)

def _problem(o, seed, noise=0.05):
    rng = _rng(seed)
    x_gt = rng.uniform(0, 1, size=o.hr_shape)
    disp = _disp_smooth(o, rng, 0.9)
    y = o.forward(x_gt, disp) + noise * rng.standard_normal(o.lr_shape)
    return y, disp


def test_admm_l2_only_no_tv_reaches_min_norm_least_squares():
    """lambda1 = 0 and no regulariser: each x-step is an exact least-squares
    solve, so the iterate is x0 + pinv(A)(y - A x0)."""
    o = _o(sy=8, sx=8, zeta=2, lambda1=0.0, lambda2=1.0, win=1, cg_iter=400, theta=1.0)
    y, disp = _problem(o, 19)
    x, stats = o.solve(y, disp, n_iter=20)
    n = o.pb.H * o.pb.W
    A = _dense(lambda v: o.forward(v, disp), n, o.hr_shape)
    x0 = o.x0(y).ravel()
    ref = x0 + np.linalg.lstsq(A, y.ravel() - A @ x0, rcond=None)[0]
    np.testing.assert_allclose(x.ravel(), ref, rtol=0, atol=1e-8)


def _linprog_optimum(o, y, disp, m):
    """min lambda1 |A x - y|_1 + |S x|_1 as a linear program (HiGHS)."""
    n = o.pb.H * o.pb.W
    A = _dense(lambda v: o.forward(v, disp), n, o.hr_shape)
    S = _dense(lambda v: o.nltv_grad(v, m), n, o.hr_shape)
    na, ns = A.shape[0], S.shape[0]
    # variables [x, s, t]; s >= |Ax - y|, t >= |Sx|
    c = np.concatenate([np.zeros(n), o.pb.lambda1 * np.ones(na), np.ones(ns)])
    I_a, I_s = np.eye(na), np.eye(ns)
    Z_as, Z_sa = np.zeros((na, ns)), np.zeros((ns, na))
    A_ub = np.block([[A, -I_a, Z_as], [-A, -I_a, Z_as], [S, Z_sa, -I_s], [-S, Z_sa, -I_s]])
    b_ub = np.concatenate([y.ravel(), -y.ravel(), np.zeros(ns), np.zeros(ns)])
    res = optimize.linprog(c, A_ub=A_ub, b_ub=b_ub, bounds=[(None, None)] * (n + na + ns),
                           method="highs")
    assert res.status == 0
    return res.fun


def test_admm_l1_only_fixed_weights_reaches_lp_optimum():
    """lambda2 = 0 with fixed weights: the cost is a linear program; ADMM's
    objective must approach the LP optimum."""
    o = _o(sy=3, sx=3, zeta=2, lambda1=1.0, lambda2=0.0, win=3, theta=8.0, cg_iter=30,
           reweight=0, sigma_e=float("inf"))
    y, disp = _problem(o, 20, noise=0.1)
    x, stats = o.solve(y, disp, n_iter=1600)
    m = np.ones(o.hr_shape)
    jstar = _linprog_optimum(o, y, disp, m)
    j = o.objective(y, disp, m, x)
    assert j >= jstar * (1 - 1e-9)
    assert (j - jstar) / jstar < 1e-6


def _dense_admm_other_splitting(o, y, disp, m, rho=16.0, iters=4000):
    """Independent solver for the full convex cost with fixed weights: textbook
    scaled ADMM on dense matrices with a *different* splitting from the
    paper's (z1 = A x - y carries both data norms through their joint prox,
    z2 = S x the l1 prox, and the x-step is an exact dense solve)."""
    n = o.pb.H * o.pb.W
    A = _dense(lambda v: o.forward(v, disp), n, o.hr_shape)
    S = _dense(lambda v: o.nltv_grad(v, m), n, o.hr_shape)
    l1, l2 = o.pb.lambda1, o.pb.lambda2
    yv = y.ravel()
    Minv = np.linalg.inv(A.T @ A + S.T @ S)
    x = np.zeros(n)
    z1, u1 = np.zeros(len(yv)), np.zeros(len(yv))
    z2, u2 = np.zeros(S.shape[0]), np.zeros(S.shape[0])
    for _ in range(iters):
        x = Minv @ (A.T @ (yv + z1 - u1) + S.T @ (z2 - u2))
        d = A @ x - yv + u1
        # argmin_z l1|z| + l2 z^2 + (rho/2)(z - d)^2
        z1 = np.sign(d) * np.maximum(np.abs(d) - l1 / rho, 0) / (1 + 2 * l2 / rho)
        s2 = S @ x + u2
        z2 = np.sign(s2) * np.maximum(np.abs(s2) - 1 / rho, 0)
        u1 += A @ x - yv - z1
        u2 += S @ x - z2
    return x


def test_admm_full_cost_fixed_weights_matches_independent_solver():
    """Full convex cost (both data norms + weighted NLTV, fixed weights): the
    oracle's iterate must reach the optimum an independent solver finds."""
    o = _o(sy=4, sx=4, zeta=2, lambda1=3.0, lambda2=10.0, win=3, theta=16.0, cg_iter=60,
           reweight=0, sigma_e=float("inf"))
    y, disp = _problem(o, 21, noise=0.1)
    x, stats = o.solve(y, disp, n_iter=800)
    m = np.ones(o.hr_shape)
    x_ref = _dense_admm_other_splitting(o, y, disp, m)
    j, j_ref = o.objective(y, disp, m, x), o.objective(y, disp, m, x_ref)
    assert abs(j - j_ref) / j_ref < 1e-8
    np.testing.assert_allclose(x, x_ref.reshape(x.shape), atol=1e-5)
    # J_n from the statistics is the cost at x^(n-1)
    assert stats[-1, 0] == pytest.approx(j, rel=1e-8)


def test_admm_stats_objective_is_cost_of_previous_iterate():
    o = _o(sy=5, sx=5, win=3)
    y, disp = _problem(o, 22)
    st = o.init_state(y)
    x_prev = st["x"].copy()
    s1 = o.iterate(st, y, disp, count=1)
    assert s1[0, 0] == pytest.approx(o.objective(y, disp, st["m"], x_prev), rel=1e-12)
    assert s1[0, 3] == 5


def test_admm_residual_decays_and_cost_drops_fixed_weights():
    o = _o(sy=8, sx=8, win=3, lambda1=1.0, lambda2=1.0, theta=16.0, cg_iter=10, reweight=0)
    y, disp = _problem(o, 23)
    x, stats = o.solve(y, disp, n_iter=300)
    assert stats[-1, 1] <= 1e-2 * stats[0, 1]
    assert stats[-1, 0] < stats[0, 0]


def test_admm_resume_equals_uninterrupted():
    o = _o(sy=6, sx=6, win=3)
    y, disp = _problem(o, 24)
    a = o.init_state(y)
    o.iterate(a, y, disp, count=6)
    b = o.init_state(y)
    o.iterate(b, y, disp, count=2)
    o.iterate(b, y, disp, count=4)
    for key in ("x", "wD", "wS", "m"):
        np.testing.assert_array_equal(a[key], b[key])


def _edge_weight_closed_form(x, sigma_e, occ):
    """sec 3.4 edge weight read with a decreasing exponent: forward differences,
    zero at the last row / column, times the occlusion map."""
    gx = np.zeros_like(x)
    gy = np.zeros_like(x)
    gx[:, :-1] = x[:, 1:] - x[:, :-1]
    gy[:-1, :] = x[1:, :] - x[:-1, :]
    return np.exp(-(gx ** 2 + gy ** 2) / sigma_e) * occ


def test_reweighted_schedule_recomputes_weights_from_previous_iterate():
    """sec 7.1: with reweighting the edge weight is recomputed at every ADMM
    iteration.  The reading is that iteration n takes m = w_e(x^(n-1)) * w_o
    and holds it through its z/w-steps and its CG x-step.  The pin replays
    the six iterations one at a time with reweighting switched off, setting m
    each time from the closed form of the weight at the current iterate.  The
    one-call reweighted run must match it at every step.  Its J_n must also be
    the cost at x^(n-1) under that m.  If the oracle froze m after the first
    iteration, or took it from the wrong iterate, this fails from n = 2 on."""
    kw = dict(sy=6, sx=6, win=3, sigma_e=0.05, lambda1=2.0, lambda2=1.0, theta=4.0)
    o_rw = _o(reweight=1, **kw)
    o_fix = _o(reweight=0, **kw)
    y, disp = _problem(o_rw, 31, noise=0.1)
    occ = _rng(32).uniform(0.2, 1.0, size=o_rw.hr_shape)

    a = o_rw.init_state(y)
    stats_a = o_rw.iterate(a, y, disp, occ=occ, count=6)

    b = o_fix.init_state(y)
    xs, ms = [], []
    stats_b = np.zeros_like(stats_a)
    for n in range(1, 7):
        xs.append(b["x"].copy())
        b["m"][...] = _edge_weight_closed_form(b["x"], o_fix.pb.sigma_e, occ)
        ms.append(b["m"].copy())
        b["n"] = n - 1
        stats_b[n - 1] = o_fix.iterate(b, y, disp, occ=occ, count=1)[0]
        # the replay must not have touched m for n >= 2 (reweighting is off)
        if n >= 2:
            np.testing.assert_array_equal(b["m"], ms[-1])

    np.testing.assert_allclose(a["x"], b["x"], rtol=0, atol=1e-11 * np.abs(b["x"]).max())
    np.testing.assert_allclose(stats_a[:, :2], stats_b[:, :2], rtol=1e-10)
    np.testing.assert_allclose(a["m"], ms[-1], rtol=1e-12, atol=0)
    for n in range(1, 7):
        j_ref = o_fix.objective(y, disp, ms[n - 1], xs[n - 1])
        assert stats_a[n - 1, 0] == pytest.approx(j_ref, rel=1e-10), n
    # the weights really change over the iterations (otherwise the pin is void)
    assert np.abs(ms[-1] - ms[0]).max() > 1e-3


def test_fixed_weights_keep_the_first_iterations_map():
    """reweight = 0: m = w_e(x^0) * w_o is computed at n = 1 only and kept."""
    kw = dict(sy=6, sx=6, win=3, sigma_e=0.05, lambda1=2.0, lambda2=1.0, theta=4.0, reweight=0)
    o = _o(**kw)
    y, disp = _problem(o, 33, noise=0.1)
    occ = _rng(34).uniform(0.2, 1.0, size=o.hr_shape)
    st = o.init_state(y)
    m0 = _edge_weight_closed_form(st["x"], o.pb.sigma_e, occ)
    x0 = st["x"].copy()
    stats = o.iterate(st, y, disp, occ=occ, count=6)
    np.testing.assert_allclose(st["m"], m0, rtol=1e-12, atol=0)
    assert np.abs(st["x"] - x0).max() > 1e-3
    assert stats[5, 0] != stats[0, 0]


# ---------------------------------------------------------------- occlusion weight (sec 3.4, eq. weight_occ)

def test_occlusion_weight_step_disparity_closed_form():
    """Constant views (no projection error): w_o = exp(-b^2/(2 s1^2)) where b
    is the negative part of the forward-difference divergence of the map.  A
    drop of D at column c gives b = -D on column c-1; a drop of E at row r
    gives b = -E on row r-1; where both meet, b = -(D+E); a rise gives 1.
    Fails for backward differences, a dropped sign clip, or a wrong axis."""
    o = _o(zeta=1, sy=9, sx=11)
    H, W = o.hr_shape
    y = np.full(o.lr_shape, 0.4)
    s1 = 0.7
    D, E = 0.9, 0.5
    d = np.full((H, W), 1.2)
    d[:, 6:] -= D
    d[5:, :] -= E
    b = np.zeros((H, W))
    b[:, 5] -= D
    b[4, :] -= E
    ref = np.exp(-b ** 2 / (2 * s1 ** 2))
    np.testing.assert_allclose(o.occlusion_weight(y, d, s1, np.inf), ref, rtol=0, atol=1e-14)
    rise = np.full((H, W), -0.3)
    rise[:, 6:] += D
    rise[5:, :] += E
    np.testing.assert_allclose(o.occlusion_weight(y, rise, s1, 0.3), 1.0, rtol=0, atol=1e-14)


def test_occlusion_weight_intensity_offsets_closed_form():
    """Zero disparity, views = one LR image + a constant c_k per view: the
    bicubic up-sampling is linear and keeps constants, so the projection error
    of view k is c_ref - c_k everywhere and w_o = exp(-mean_k (c_ref - c_k)^2
    / (2 s2^2)) with the mean over the views other than the reference."""
    o = _o(U=3, V=5, zeta=3)
    rng = _rng(41)
    base = rng.uniform(0, 1, (o.pb.sy, o.pb.sx))
    c = rng.uniform(-0.3, 0.3, o.pb.sk)
    y = base[None] + c[:, None, None]
    kref = (o.pb.U // 2) * o.pb.V + o.pb.V // 2
    p2 = np.mean([(c[kref] - c[k]) ** 2 for k in range(o.pb.sk) if k != kref])
    s2 = 0.25
    got = o.occlusion_weight(y, np.zeros(o.hr_shape), np.inf, s2)
    np.testing.assert_allclose(got, np.exp(-p2 / (2 * s2 ** 2)), rtol=1e-12, atol=0)


def test_occlusion_weight_consistent_scene_is_one_in_the_interior():
    """Scale 1, constant integer disparity, views made as exact shifts of one
    image by the forward model's convention (view k at u shows the reference
    at u + theta_k w): every view brought back to the reference matches it
    wherever the shifted position stays in the image, so w_o = 1 there.
    Fails for the forward instead of the inverse warp (a doubled shift)."""
    o = _o(U=3, V=3, zeta=1, sy=12, sx=13)
    H, W = o.hr_shape
    rng = _rng(42)
    x = ndimage.gaussian_filter(rng.uniform(0, 1, (H, W)), 1.0)
    w = 1
    y = np.zeros(o.lr_shape)
    for k in range(o.pb.sk):
        tau, rho = o.view_offset(k)
        xp = np.pad(x, 2, mode="edge")
        y[k] = xp[2 + tau * w:2 + tau * w + H, 2 + rho * w:2 + rho * w + W]
    got = o.occlusion_weight(y, np.full((H, W), float(w)), np.inf, 0.05)
    np.testing.assert_allclose(got[1:-1, 1:-1], 1.0, rtol=0, atol=1e-13)
    assert got.min() < 0.99  # the border rows/columns do see the edge padding


def test_occlusion_weight_sampling_equals_scipy_map_coordinates():
    """The projection error's sampling step against scipy: view k's bicubic
    up-sampling read with map_coordinates(order=1, mode='nearest') (linear
    interpolation, clamp-to-edge) at z - theta_k w(z), on a smooth map at
    scale 2 (the bicubic step itself is pinned above)."""
    o = _o(U=3, V=3, zeta=2, sy=8, sx=9)
    rng = _rng(43)
    y = rng.uniform(0, 1, o.lr_shape)
    d = _disp_smooth(o, rng, amp=1.6)
    H, W = o.hr_shape
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    kref = (o.pb.U // 2) * o.pb.V + o.pb.V // 2
    l0 = o.bicubic(y[kref])
    acc = np.zeros((H, W))
    for k in range(o.pb.sk):
        if k == kref:
            continue
        tau, rho = o.view_offset(k)
        s = ndimage.map_coordinates(o.bicubic(y[k]), [yy - tau * d, xx - rho * d], order=1, mode="nearest")
        acc += (l0 - s) ** 2
    p2 = acc / (o.pb.sk - 1)
    s2 = 0.2
    got = o.occlusion_weight(y, d, np.inf, s2)
    np.testing.assert_allclose(got, np.exp(-p2 / (2 * s2 ** 2)), rtol=1e-11, atol=1e-14)


# ---------------------------------------------------------------- multi-image workload (sec 7.3)

def test_btv_spatial_weight_closed_form():
    """BTV weights (sec 7.3 configures the non-local weights to match BTV):
    alpha^(|dy|+|dx|) with alpha = sigma_s; the Gaussian form otherwise."""
    o = _o(win=5, sigma_s=0.7, weight_kind=1)
    for dy, dx in [(0, 1), (-1, 0), (1, 1), (-2, 1), (2, -2)]:
        assert abs(o.spatial_weight(dy, dx) - 0.7 ** (abs(dy) + abs(dx))) < 1e-15
    g = _o(win=5, sigma_s=0.7)
    assert abs(g.spatial_weight(1, 1) - np.exp(-2 / 0.7)) < 1e-15


def test_btv_regulariser_is_twice_the_half_window_pair_sum():
    """With m = 1 (no edge weight) and BTV weights, the full-window NLTV term
    sum_d sum_z c_d |x(z) - x(z+d)| counts every unordered pixel pair twice
    (c_d = c_-d): it equals 2 x the half-window form of BTV (offsets with
    dy > 0, or dy = 0 and dx > 0), brute-forced here over pixel pairs."""
    o = _o(win=5, sigma_s=0.6, weight_kind=1, sigma_e=np.inf, zeta=1, sy=9, sx=8)
    x = _rng(61).uniform(0, 1, o.hr_shape)
    m = np.ones(o.hr_shape)
    full = np.abs(o.nltv_grad(x, m)).sum()
    H, W = o.hr_shape
    half = 0.0
    for dy in range(0, 3):
        for dx in range(-2, 3):
            if dy == 0 and dx <= 0:
                continue
            c = 0.6 ** (abs(dy) + abs(dx))
            for Y in range(H):
                for X in range(W):
                    if 0 <= Y + dy < H and 0 <= X + dx < W:
                        half += c * abs(x[Y, X] - x[Y + dy, X + dx])
    assert abs(full - 2 * half) < 1e-12 * full


def test_even_grid_offsets_and_reference_view():
    """A 2 x 2 set of images (the x2 multi-image workload): offsets {0,1}^2
    from view 0, which is the reference (x0 is its bicubic up-sampling); with
    a constant map of 1/2 the views are the reference shifted by half a pixel
    (the warp against scipy's linear interpolation)."""
    o = _o(U=2, V=2, zeta=1, sy=10, sx=11)
    assert [o.view_offset(k) for k in range(4)] == [(0, 0), (0, 1), (1, 0), (1, 1)]
    assert o.ref_view() == 0
    y = _rng(62).uniform(0, 1, o.lr_shape)
    np.testing.assert_array_equal(o.x0(y), o.bicubic(y[0]))
    x = _rng(63).uniform(0, 1, o.hr_shape)
    H, W = o.hr_shape
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    for k in range(4):
        tau, rho = o.view_offset(k)
        ref = ndimage.map_coordinates(x, [yy + 0.5 * tau, xx + 0.5 * rho], order=1, mode="grid-constant", cval=0.0)
        np.testing.assert_allclose(o.warp(x, np.full((H, W), 0.5), k), ref, rtol=0, atol=1e-14)
    assert _o(U=3, V=5).ref_view() == 7


# ---------------------------------------------------------------- gradient-descent baselines (sec 7.1)

def test_cost_subgradient_matches_finite_differences():
    """At a generic point (no residual or pixel difference at zero) J is
    differentiable and the subgradient A^T q + S^T sgn(g) is its gradient:
    central differences along random directions agree.  Fails for a dropped
    factor 2 on the l2 part, a sign error or a transposed operator."""
    o = _o(win=3, sigma_e=np.inf, reweight=0)
    rng = _rng(81)
    d = _disp_smooth(o, rng)
    y = rng.uniform(0, 1, o.lr_shape)
    x = rng.uniform(0, 1, o.hr_shape)
    m = rng.uniform(0.3, 1.0, o.hr_shape)
    J, q, t = o.cost_parts(y, d, m, x)
    assert abs(J - o.objective(y, d, m, x)) < 1e-10 * J
    grad = o.adjoint(q, d) + t
    for _ in range(4):
        v = rng.standard_normal(o.hr_shape)
        eps = 1e-6
        fd = (o.cost_parts(y, d, m, x + eps * v)[0] - o.cost_parts(y, d, m, x - eps * v)[0]) / (2 * eps)
        assert abs(fd - np.vdot(grad, v)) < 1e-6 * abs(fd)


def test_gd_l2_only_equals_dense_iteration():
    """lambda1 = 0 and no regulariser: gd is x <- x - step 2 lambda2 A^T (A x - y),
    reproduced with a dense matrix of A built column by column from the
    forward operator alone."""
    o = _o(sy=4, sx=5, lambda1=0.0, lambda2=1.5, win=1, sigma_e=np.inf, reweight=0)
    rng = _rng(82)
    d = _disp_smooth(o, rng)
    y = rng.uniform(0, 1, o.lr_shape)
    n = o.hr_shape[0] * o.hr_shape[1]
    A = np.stack([o.forward(np.eye(n)[i].reshape(o.hr_shape), d).ravel() for i in range(n)], axis=1)
    x, hist = o.gd(y, d, 5, 0.05)
    xr = o.x0(y).ravel()
    for _ in range(5):
        xr = xr - 0.05 * 2 * 1.5 * A.T @ (A @ xr - y.ravel())
    np.testing.assert_allclose(x.ravel(), xr, rtol=0, atol=1e-12)
    assert list(hist[:, 1]) == [2, 4, 6, 8, 10, 12]


def test_gd_line_search_is_monotone_with_armijo_steps():
    o = _o(reweight=0)
    rng = _rng(83)
    d = _disp_smooth(o, rng)
    y = rng.uniform(0, 1, o.lr_shape)
    x, hist = o.gd(y, d, 12, 0.05, line_search=True)
    J, cu = hist[:, 0], hist[:, 1]
    assert np.all(np.diff(J) <= 0) and J[-1] < J[0]
    assert np.all(np.diff(cu) >= 2)  # at least one trial and one adjoint per step


# ---------------------------------------------------------------- general blur kernel (sec 7.1: motion blur)

def test_explicit_blur_kernel_equals_scipy_correlate_and_is_not_symmetric():
    h = motion_kernel(7)
    assert np.abs(h - h[::-1, ::-1]).max() > 1e-3
    o = _o(kb=7, blur_taps=h)
    np.testing.assert_array_equal(o.blur_kernel(), h)
    x = _rng(91).standard_normal(o.hr_shape)
    ref = ndimage.correlate(x, h, mode="constant", cval=0.0)
    np.testing.assert_allclose(o.blur(x), ref, rtol=0, atol=1e-14)


def test_explicit_blur_adjoint_and_forward_composition():
    """B^T of a non-symmetric kernel is its transpose (not B again), and
    A_k = D B W_k with it; the adjoint of the whole forward model holds."""
    h = motion_kernel(9, angle_deg=30.0)
    o = _o(kb=9, zeta=2, blur_taps=h)
    rng = _rng(92)
    u, v = rng.standard_normal(o.hr_shape), rng.standard_normal(o.hr_shape)
    assert abs(np.vdot(o.blur(u), v) - np.vdot(u, o.blur_t(v))) < 1e-12 * np.abs(u).sum() * np.abs(v).sum()
    assert np.abs(o.blur_t(v) - o.blur(v)).max() > 1e-3
    d = _disp_smooth(o, rng)
    x = rng.standard_normal(o.hr_shape)
    t = o.forward(x, d)
    for k in (0, 4, 8):
        np.testing.assert_allclose(t[k], o.down(o.blur(o.warp(x, d, k))), rtol=0, atol=1e-13)
    e = rng.standard_normal(o.lr_shape)
    lhs, rhs = np.vdot(t, e), np.vdot(x, o.adjoint(e, d))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
