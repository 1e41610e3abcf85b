"""GPU parity with an explicit, non-symmetric blur kernel (sec 7.1 models
motion blur as another convolution kernel for B): the tiled forward and
adjoint apply it as a 2-D correlation and its transpose.  Kernels: a 45
degree motion line at x2 with 5 x 5 views (the paper's motion-blur setting),
a 30 degree line at x3, a random non-symmetric 5 x 5 kernel.  Operators 2e-5
max-abs relative, whole solves 1e-4 relative L2 against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import CASES, disp_bound, make_case, motion_kernel, rel_err  # noqa: E402

from paper_2206_05047_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu
OP_TOL = 2e-5

KERNELS = {
    "motion45_x2_5x5": (dict(CASES["c1"], U=5, V=5, n_iter=10), motion_kernel(7, 45.0)),
    "motion30_x3": (CASES["ragged"], motion_kernel(9, 30.0)),
    "random5_x2": (CASES["c1"], None),
}


@pytest.fixture(scope="module")
def lfsr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05047_amd import lfsr as mod
    mod.load()
    return mod


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module", params=list(KERNELS))
def bcase(request):
    print(f"[blur case {request.param}]", flush=True)
    cfg, h = KERNELS[request.param]
    if h is None:
        h = np.random.default_rng(93).uniform(0, 1, (5, 5))
        h /= h.sum()
    h = h.astype(np.float32)  # the device reads float32 taps; the oracle gets the same values
    cfg = dict(cfg, kb=h.shape[0], blur_taps=h.astype(np.float64))
    return make_case(cfg)


def _solver(lfsr, case):
    cfg = case["cfg"]
    return lfsr.Solver(lfsr.make_params(cfg, disp_bound=disp_bound(cfg), blur_taps=cfg["blur_taps"]))


def test_explicit_blur_operators_match_oracle(lfsr, bcase):
    s = _solver(lfsr, bcase)
    o, d = bcase["oracle"], bcase["disp"]
    rng = np.random.default_rng(94)
    x = rng.uniform(0, 1, o.hr_shape).astype(np.float32)
    t = _n(s.lfsr_forward(_t(x), _t(d)))
    assert rel_err(t, o.forward(x, d)) < OP_TOL
    e = rng.standard_normal(o.lr_shape).astype(np.float32)
    a = _n(s.lfsr_adjoint(_t(e), _t(d)))
    assert rel_err(a, o.adjoint(e, d)) < OP_TOL
    lhs, rhs = np.vdot(t, e), np.vdot(x, a)
    assert abs(lhs - rhs) <= 1e-5 * np.sqrt(np.vdot(t, t) * np.vdot(e, e))
    m = rng.uniform(0.2, 1.0, o.hr_shape).astype(np.float32)
    assert rel_err(_n(s.lfsr_normal(_t(x), _t(d), _t(m))), o.normal_apply(d, m, x)) < OP_TOL


def test_explicit_blur_solve_matches_oracle(lfsr, bcase):
    s = _solver(lfsr, bcase)
    o = bcase["oracle"]
    x, st = s.lfsr_solve(_t(bcase["y"]), _t(bcase["disp"]))
    xr, sr = o.solve(bcase["y"], bcase["disp"])
    x = _n(x)
    err = synth.rel_l2(x, xr)
    x0 = o.x0(bcase["y"])
    print(f"{bcase['cfg']['name']} kb={bcase['cfg']['kb']}: rel_l2={err:.3e} PSNR bicubic "
          f"{synth.psnr(x0, bcase['x_gt']):.2f} -> {synth.psnr(x, bcase['x_gt']):.2f} dB", flush=True)
    assert err < 1e-4
    np.testing.assert_allclose(st["hist"][:, 0], sr[:, 0], rtol=1e-4)
