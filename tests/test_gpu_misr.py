"""GPU parity on the multi-image workload (sec 7.3): 2 x 2 images at
half-pixel shifts for x2 and 3 x 3 at third-pixel shifts for x3, the l2 term
off, BTV weights, no edge weight.

* Small variants: operators (2e-5 max-abs relative) and whole solves (1e-4
  relative L2) against the FP64 oracle.
* Full size (HR 5760 x 5760): the forward and adjoint operators on sampled
  blocks against the oracle run on a crop (both operators are local: with a
  constant shift an output depends only on inputs within the blur and warp
  reach, so the crop's interior is exact), and the whole solve through
  properties that hold at any size: J ends below its start and at its
  minimum over the run (ADMM is not a descent method, though the oracle's J
  decreases at every step on the small and 512^2 variants), the primal
  residual falls below a fifth of its first value, and the result beats
  bicubic up-sampling.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import rel_err  # noqa: E402

import oracle  # noqa: E402
from paper_2206_05047_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

OP_TOL = 2e-5
SMALL = {"misr2": dict(sy=32, sx=36, n_iter=20), "misr3": dict(sy=24, sx=26, n_iter=20)}


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


def _solver(lfsr, cfg):
    return lfsr.Solver(lfsr.make_params(cfg, disp_bound=max(cfg["shift"], 1e-3)))


@pytest.fixture(scope="module", params=list(SMALL))
def small(request):
    print(f"[misr small {request.param}]", flush=True)
    cfg = synth.config(request.param, **SMALL[request.param])
    o = oracle.Oracle(cfg)
    sc = synth.make_scene(cfg)
    y = synth.degrade(o.forward(sc["x_gt"], sc["disp"]), synth.make_noise(cfg))
    return dict(cfg=cfg, o=o, sc=sc, y=y)


def test_misr_small_operators(lfsr, small):
    s = _solver(lfsr, small["cfg"])
    o, d = small["o"], small["sc"]["disp"]
    rng = np.random.default_rng(71)
    x = rng.uniform(0, 1, o.hr_shape).astype(np.float32)
    assert rel_err(_n(s.lfsr_forward(_t(x), _t(d))), o.forward(x, d)) < OP_TOL
    e = rng.standard_normal(o.lr_shape).astype(np.float32)
    assert rel_err(_n(s.lfsr_adjoint(_t(e), _t(d))), o.adjoint(e, d)) < OP_TOL
    m = np.ones(o.hr_shape, np.float32)
    assert rel_err(_n(s.lfsr_normal(_t(x), _t(d), _t(m))), o.normal_apply(d, m, x)) < OP_TOL


def test_misr_small_solve(lfsr, small):
    s = _solver(lfsr, small["cfg"])
    o = small["o"]
    x, st = s.lfsr_solve(_t(small["y"]), _t(small["sc"]["disp"]))
    xr, sr = o.solve(small["y"], small["sc"]["disp"])
    err = synth.rel_l2(_n(x), xr)
    print(f"{small['cfg']['name']} small: rel_l2={err:.3e} psnr={synth.psnr(_n(x), small['sc']['x_gt']):.2f}",
          flush=True)
    assert err < 1e-4
    np.testing.assert_allclose(st["hist"][:, 0], sr[:, 0], rtol=1e-4)


@pytest.fixture(scope="module", params=["misr2", "misr3"])
def full(request, lfsr):
    print(f"[misr full {request.param}]", flush=True)
    cfg = synth.config(request.param)
    sc = synth.make_scene(cfg)
    s = _solver(lfsr, cfg)
    d = _t(sc["disp"])
    y = _t(synth.degrade(_n(s.lfsr_forward(_t(sc["x_gt"]), d)), synth.make_noise(cfg)))
    return dict(cfg=cfg, sc=sc, s=s, d=d, y=y)


def test_misr_full_operators_on_sampled_blocks(full):
    """Forward and adjoint at 5760^2 against the oracle on 48 x 48 HR crops at
    six seeded places (interior of each crop compared: 8 HR / 4 LR pixels of
    margin cover the blur and warp reach)."""
    cfg, s = full["cfg"], full["s"]
    z = cfg["zeta"]
    H, W = z * cfg["sy"], z * cfg["sx"]
    rng = np.random.default_rng(72)
    x = rng.uniform(0, 1, (H, W)).astype(np.float32)
    e = rng.standard_normal((cfg["U"] * cfg["V"], cfg["sy"], cfg["sx"])).astype(np.float32)
    t_gpu = _n(s.lfsr_forward(_t(x), full["d"]))
    a_gpu = _n(s.lfsr_adjoint(_t(e), full["d"]))
    cl = 48 // z  # crop size in LR pixels
    oc = oracle.Oracle(dict(cfg, sy=cl, sx=cl))
    dc = np.full((cl * z, cl * z), cfg["shift"])
    mg = 4  # LR margin
    for _ in range(6):
        i0 = int(rng.integers(0, cfg["sy"] - cl)) if rng.random() < 0.8 else 0
        j0 = int(rng.integers(0, cfg["sx"] - cl))
        xs = x[i0 * z:(i0 + cl) * z, j0 * z:(j0 + cl) * z]
        tr = oc.forward(xs, dc)
        tg = t_gpu[:, i0:i0 + cl, j0:j0 + cl]
        lo = 0 if i0 == 0 else mg
        assert rel_err(tg[:, lo:cl - mg, mg:cl - mg], tr[:, lo:cl - mg, mg:cl - mg]) < OP_TOL
        ar = oc.adjoint(e[:, i0:i0 + cl, j0:j0 + cl], dc)
        ag = a_gpu[i0 * z:(i0 + cl) * z, j0 * z:(j0 + cl) * z]
        lh = 0 if i0 == 0 else mg * z
        assert rel_err(ag[lh:(cl - mg) * z, mg * z:(cl - mg) * z], ar[lh:(cl - mg) * z, mg * z:(cl - mg) * z]) < OP_TOL


def test_misr_full_solve_properties(full, lfsr):
    cfg, s = full["cfg"], full["s"]
    x, st = s.lfsr_solve(full["y"], full["d"])
    J = st["hist"][:, 0]
    x = _n(x)
    kref = ((cfg["U"] - 1) // 2) * cfg["V"] + (cfg["V"] - 1) // 2
    x0 = _n(s.lfsr_bicubic(full["y"][kref]))
    p, p0 = synth.psnr(x, full["sc"]["x_gt"]), synth.psnr(x0, full["sc"]["x_gt"])
    print(f"{cfg['name']} full: PSNR {p:.2f} dB (bicubic {p0:.2f}), J {J[0]:.6g} -> {J[-1]:.6g}", flush=True)
    res = st["hist"][:, 1]
    print(f"  J steps up: {int(np.sum(np.diff(J) > 0))}, residual {res[0]:.4g} -> {res[-1]:.4g}", flush=True)
    assert st["iters_run"] == cfg["n_iter"]
    assert J[-1] < J[0] and J[-1] <= (1 + 1e-5) * J.min()
    assert res[-1] <= 0.2 * res[0]
    assert p > p0 + 0.25  # 5760^2 1/f scenes are smooth per pixel: bicubic is already ~35 dB there
