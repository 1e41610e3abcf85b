"""GPU parity of the gradient-descent baselines (sec 7.1: gd, gd-ls) against
the FP64 oracle: the cost history and the iterate of fixed-step gd, and the
accepted steps and costs of gd-ls, on the c1 and ragged workloads with the
weights fixed at x0.  Cost values 1e-5 relative per evaluation (FP64 sums of
FP32 terms), iterates 1e-4 relative L2 (the solver bar)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import CASES, disp_bound, make_case  # noqa: E402

import oracle  # noqa: E402
from paper_2206_05047_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lfsr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05047_amd import lfsr as mod
    mod.load()
    return mod


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


@pytest.fixture(scope="module", params=["c1", "ragged"])
def case(request):
    print(f"[gd case {request.param}]", flush=True)
    c = make_case(dict(CASES[request.param], reweight=0))
    c["oracle"] = oracle.Oracle(c["cfg"])
    return c


def _solver(lfsr, case):
    s = lfsr.Solver(lfsr.make_params(case["cfg"], disp_bound=disp_bound(case["cfg"])))
    s.lfsr_init(_t(case["y"]), _t(case["disp"]))
    return s


def test_gd_fixed_step_matches_oracle(lfsr, case):
    s = _solver(lfsr, case)
    hist = s.lfsr_gd(10, 2e-3)
    x = s.lfsr_read_state()["x"].cpu().numpy()
    xr, hr = case["oracle"].gd(case["y"], case["disp"], 10, 2e-3)
    np.testing.assert_array_equal(hist[:, 1], hr[:, 1])
    np.testing.assert_allclose(hist[:, 0], hr[:, 0], rtol=1e-5)
    assert synth.rel_l2(x, xr) < 1e-4


def test_gd_line_search_matches_oracle(lfsr, case):
    s = _solver(lfsr, case)
    hist = s.lfsr_gd(8, 1e-2, line_search=True)
    xr, hr = case["oracle"].gd(case["y"], case["disp"], 8, 1e-2, line_search=True)
    print("gd-ls steps", hist[:, 2], "oracle", hr[:, 2], flush=True)
    assert np.all(np.diff(hist[:, 0]) <= 0)
    np.testing.assert_array_equal(hist[:, 1], hr[:, 1])  # same trials accepted
    np.testing.assert_allclose(hist[:, 2], hr[:, 2], rtol=1e-6)  # the GPU starts from the float32 step
    np.testing.assert_allclose(hist[:, 0], hr[:, 0], rtol=1e-5)
