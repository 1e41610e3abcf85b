"""lfsr_solve_noalloc (the solve over the library's static per-GPU scratch,
for callers that cannot allocate device memory) against lfsr_solve with a
caller workspace, through the C ABI: two calls in a row on one GPU, the second
with a smaller problem, each bit-identical to its workspace solve (same
kernels, same launch sequence); the first also within the solver's 1e-4
relative-L2 bar of the FP64 oracle.  Problems above the scratch size are
rejected before any work is enqueued."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import CASES, disp_bound, make_case  # noqa: E402

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


def _solve_both(lfsr, case, storage="f32"):
    cfg = case["cfg"]
    prm = lfsr.make_params(cfg, disp_bound=disp_bound(cfg), storage=storage)
    y, d = _t(case["y"]), _t(case["disp"])
    ref_solver = lfsr.Solver(prm)
    ref, ref_st = ref_solver.lfsr_solve(y, d)
    got, got_st = lfsr.solve_noalloc(prm, y, d, stats=True)
    torch.cuda.synchronize()
    ref_solver.close()
    return got.cpu().numpy(), ref.cpu().numpy(), got_st, ref_st


def test_noalloc_matches_workspace_solve_twice_shrinking(lfsr):
    small_cfg = dict(CASES["c1"], name="small", sy=20, sx=24, n_iter=5, seed=13)
    big, small = make_case(CASES["c1"]), make_case(small_cfg)
    assert big["y"].size > small["y"].size
    for case in (big, small):
        print(f"[noalloc {case['cfg']['name']}]", flush=True)
        got, ref, gst, rst = _solve_both(lfsr, case)
        assert np.array_equal(got, ref), np.abs(got - ref).max()
        assert gst["iters_run"] == rst["iters_run"] == case["cfg"]["n_iter"]
        assert np.array_equal(gst["hist"], rst["hist"])
    # the first problem again after the smaller one: no state carries over
    got, ref, _, _ = _solve_both(lfsr, big)
    assert np.array_equal(got, ref)
    xr, _ = big["oracle"].solve(big["y"], big["disp"])
    assert synth.rel_l2(got, xr) < 1e-4


def test_noalloc_16bit_storage_matches(lfsr):
    case = make_case(CASES["ragged"])
    got, ref, _, _ = _solve_both(lfsr, case, storage="f16")
    assert np.array_equal(got, ref)


def test_noalloc_rejects_problems_above_the_scratch(lfsr):
    prm = lfsr.make_params(synth.config("c3"), disp_bound=2.0)
    assert lfsr.workspace_bytes(prm) > lfsr.NOALLOC_MAX_BYTES
    y = torch.zeros(1, device="cuda")
    with pytest.raises(lfsr.LfsrError) as ei:
        lfsr.solve_noalloc(prm, y, y, out=y)
    assert ei.value.code == lfsr.LFSR_ENOMEM
    assert "static scratch" in str(ei.value)
