"""GPU parity at the kernel shapes of the serving workload: angular grids 3x3,
5x5 and 9x9 with (scale, blur) = (2, 7x7 s=1.2) and (3, 9x9 s=1.5), NLTV 7x7,
planar-ramp-and-patches disparity in [-2, 2], FP32 and FP16 storage, each
solved through lfsr_solve and compared with the FP64 oracle.

The serving job types run these shapes at HR 256^2 to 1152^2; the images here
are reduced so that the oracle finishes in seconds, with ragged LR sizes that
span several forward and adjoint tiles in both directions.  The operator
kernels (column-per-lane forms, quad cells when there are eight views or more,
view groups of the adjoint) are chosen from the view count, scale, blur and
disparity bound, so these cases run the same specialisations as the serving
sizes.  Tolerances as elsewhere: FP32 whole solves 1e-4 relative L2 and the
objective history to 1e-4; FP16 storage 2e-3 relative L2 (u = 2^-11 per
stored value, carried through the iteration).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import disp_bound, make_case  # noqa: E402

from paper_2206_05047_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

SOLVE_TOL = {"f32": 1e-4, "f16": 2e-3}
# (scale, blur size, blur sigma, LR rows, LR columns) per serving scale
SCALES = {2: (7, 1.2, 37, 41), 3: (9, 1.5, 29, 27)}


def _cfg(U, z):
    kb, sb, sy, sx = SCALES[z]
    return dict(synth.CONFIGS["c3"], name=f"serve{U}x{U}_x{z}", U=U, V=U, sy=sy, sx=sx, zeta=z, kb=kb,
                sigma_b=sb, win=7, n_iter=4, seed=100 + 10 * U + z)


@pytest.fixture(scope="module")
def lfsr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05047_amd import lfsr as mod
    mod.load()
    return mod


_cases = {}


def _case(U, z):
    key = (U, z)
    if key not in _cases:
        print(f"[serving shape {U}x{U} x{z}]", flush=True)
        c = make_case(_cfg(U, z))
        c["ref_x"], c["ref_stats"] = c["oracle"].solve(c["y"], c["disp"])
        _cases[key] = c
    return _cases[key]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


@pytest.mark.parametrize("st", ["f32", "f16"])
@pytest.mark.parametrize("z", [2, 3])
@pytest.mark.parametrize("U", [3, 5, 9])
def test_serving_shape_solve_matches_oracle(lfsr, U, z, st):
    c = _case(U, z)
    storage = {"f32": lfsr.LFSR_F32, "f16": lfsr.LFSR_F16}[st]
    s = lfsr.Solver(lfsr.make_params(c["cfg"], disp_bound=disp_bound(c["cfg"]), storage=storage))
    x, stats = s.lfsr_solve(_t(c["y"]), _t(c["disp"]))
    torch.cuda.synchronize()
    x = x.cpu().numpy().astype(np.float64)
    err = synth.rel_l2(x, c["ref_x"])
    print(f"{c['cfg']['name']} {st}: rel_l2={err:.3e}", flush=True)
    assert np.all(np.isfinite(x))
    assert err < SOLVE_TOL[st]
    if st == "f32":
        np.testing.assert_allclose(stats["hist"][:, 0], c["ref_stats"][:, 0], rtol=1e-4)
