"""Shared test helpers: seeded problem cases built from the synthetic generator
and the oracle's forward model (never from the HIP path)."""
import numpy as np

import oracle
from paper_2206_05047_amd import synth

# A ragged case: several forward/adjoint tiles with partial tails in both
# directions, a non-square angular grid, scale 3 and smooth + stepped disparity.
RAGGED = dict(synth.CONFIGS["c1"], name="ragged", U=3, V=5, sy=37, sx=29, zeta=3, kb=7, sigma_b=1.3, win=5,
              n_iter=6, seed=11, noise_sigma=0.03, impulse_frac=0.1, impulse="salt_pepper", scene="layers",
              n_layers=5, disp_max=1.5)

# Degenerate shapes: one view, no blur, no regulariser, scale 1.
SINGLE = dict(synth.CONFIGS["c1"], name="single", U=1, V=1, sy=21, sx=19, zeta=1, kb=1, sigma_b=1.0, win=1,
              n_iter=4, seed=12, scene="layers", n_layers=3, disp_max=1.0)

CASES = {"c1": synth.CONFIGS["c1"], "ragged": RAGGED, "single": SINGLE}


def disp_bound(cfg):
    return float(cfg.get("disp_max", 2.0))


def make_case(cfg, seed=None):
    """Seeded scene -> LR views through the oracle's forward model -> noise."""
    o = oracle.Oracle(cfg)
    sc = synth.make_scene(cfg, seed)
    nz = synth.make_noise(cfg, seed)
    y = synth.degrade(o.forward(sc["x_gt"], sc["disp"]), nz)
    return {"cfg": cfg, "oracle": o, "x_gt": sc["x_gt"], "disp": sc["disp"], "y": y}


def rel_err(a, ref):
    """max |a - ref| / max |ref| (elementwise parity measure)."""
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.abs(ref).max()
    return float(np.abs(a - ref).max() / (den if den > 0 else 1.0))


def occ_exponent_err(got, ref, s1, s2):
    """Occlusion weight parity on its exponent E = -log w_o = b^2 c1 + p^2 c2
    (c = 1/(2 sigma^2)): returns max |E_got - E_ref| / bound.  FP32 bicubic
    values are within 2.5e-6 of exact (16 Keys taps, sum |weight| < 1.3, on
    [0,1] data, two of them per difference), so a squared projection error
    moves by at most 2 |d| 2.5e-6 <= 5e-6 and p^2 (a mean of them) too; b is a
    difference of two disparity values (relative 1.2e-7, |b| <= 8).  Where
    the exact weight is below FP32's normal range (E >= 80) the FP32 result
    may underflow: there it must only be below 1e-34."""
    c1 = 0.0 if np.isinf(s1) else 0.5 / s1 ** 2
    c2 = 0.0 if np.isinf(s2) else 0.5 / s2 ** 2
    bound = 5e-6 * c2 + 2e-6 * 8.0 * c1 + 1e-6
    got = np.asarray(got, np.float64)
    er = -np.log(np.asarray(ref, np.float64))
    deep = er >= 80.0
    if np.any(got[deep] >= 1e-34):
        return float("inf")
    eg = -np.log(np.maximum(got[~deep], 1e-300))
    return float(np.max(np.abs(eg - er[~deep]), initial=0.0) / bound)


def motion_kernel(kb, angle_deg=45.0, length=None):
    """A line (motion-blur) kernel on a kb x kb grid: samples along a segment
    through the centre at the given angle, bilinearly splatted, normalised
    to 1; off-centre weighting makes it non-symmetric."""
    L = (kb - 1) if length is None else length
    r = kb // 2
    h = np.zeros((kb, kb))
    t = np.linspace(-L / 2, L / 2, 8 * kb)
    w = 1.0 + 0.8 * (t - t.min()) / (t.max() - t.min())  # heavier at one end: not symmetric
    ang = np.deg2rad(angle_deg)
    for tt, ww in zip(t, w):
        yy, xx = r - tt * np.sin(ang), r + tt * np.cos(ang)
        i0, j0 = int(np.floor(yy)), int(np.floor(xx))
        fy, fx = yy - i0, xx - j0
        for di, dj, c in ((0, 0, (1 - fy) * (1 - fx)), (0, 1, (1 - fy) * fx), (1, 0, fy * (1 - fx)), (1, 1, fy * fx)):
            if 0 <= i0 + di < kb and 0 <= j0 + dj < kb:
                h[i0 + di, j0 + dj] += ww * c
    return h / h.sum()
