"""GPU parity of the 16-bit storage forms (FP16, BF16) against the FP64 oracle.

With 16-bit storage the stencils read x, w_D, w_S and the LR stack rounded to
nearest even at unit roundoff u (2^-11 for FP16, 2^-8 for BF16) while every
sum stays FP32, so the error of one operator application or of one dual
update is a small multiple of u relative to the largest value (bound: the
taps and bilinear weights are non-negative and sum to at most one, so a sum
of rounded inputs is off by at most u times the largest input).  Whole solves
carry the perturbation through the iteration; they are checked by relative
L2 against the oracle (bound stated per form below) and by the PSNR against
the ground truth, which must stay within 0.05 dB of the oracle's.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import CASES, disp_bound, make_case, rel_err  # noqa: E402

from paper_2206_05047_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

U = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
# whole-solve relative L2 bounds (c1: 20 iterations, ragged: 6)
SOLVE_TOL = {"f16": 2e-3, "bf16": 1.5e-2}
PSNR_TOL_DB = 0.05


@pytest.fixture(scope="module")
def lfsr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05047_amd import lfsr as mod
    mod.load()
    return mod


def _storage(lfsr, name):
    return {"f16": lfsr.LFSR_F16, "bf16": lfsr.LFSR_BF16}[name]


def _solver(lfsr, cfg, st, **over):
    return lfsr.Solver(lfsr.make_params(cfg, disp_bound=disp_bound(cfg), storage=_storage(lfsr, st), **over))


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


_cases = {}


def _case(name):
    if name not in _cases:
        print(f"[case {name}]", flush=True)
        _cases[name] = make_case(CASES[name])
        c = _cases[name]
        c["ref_x"], c["ref_stats"] = c["oracle"].solve(c["y"], c["disp"])
    return _cases[name]


@pytest.mark.parametrize("st", ["f16", "bf16"])
@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_normal_operator_16bit(lfsr, name, st):
    """t = A p is stored in 16 bits between the two halves of G^T G."""
    c = _case(name)
    o = c["oracle"]
    rng = np.random.default_rng(3)
    pv = rng.standard_normal(o.hr_shape).astype(np.float32)
    m = rng.uniform(0.2, 1.0, o.hr_shape).astype(np.float32)
    got = _n(_solver(lfsr, c["cfg"], st).lfsr_normal(_t(pv), _t(c["disp"]), _t(m)))
    assert rel_err(got, o.normal_apply(c["disp"], m, pv)) < 4 * U[st]


@pytest.mark.parametrize("st", ["f16", "bf16"])
@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_one_iteration_16bit(lfsr, name, st):
    c = _case(name)
    o = c["oracle"]
    s = _solver(lfsr, c["cfg"], st)
    s.lfsr_init(_t(c["y"]), _t(c["disp"]))
    s.lfsr_iterate(1)
    got = s.lfsr_read_state()
    ref = o.init_state(c["y"])
    o.iterate(ref, c["y"], c["disp"], count=1)
    tol = 8 * U[st]
    assert rel_err(_n(got["m"]), ref["m"]) < tol
    assert rel_err(_n(got["wD"]), ref["wD"]) < tol
    assert rel_err(_n(got["wS"]), ref["wS"]) < tol
    assert synth.rel_l2(_n(got["x"]), ref["x"]) < tol


@pytest.mark.parametrize("st", ["f16", "bf16"])
@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_full_solve_16bit(lfsr, name, st):
    c = _case(name)
    s = _solver(lfsr, c["cfg"], st)
    x, stats = s.lfsr_solve(_t(c["y"]), _t(c["disp"]))
    x = _n(x)
    err = synth.rel_l2(x, c["ref_x"])
    p16, pref = synth.psnr(x, c["x_gt"]), synth.psnr(c["ref_x"], c["x_gt"])
    print(f"{name} {st}: rel_l2={err:.3e} psnr={p16:.3f} oracle={pref:.3f}", flush=True)
    assert err < SOLVE_TOL[st]
    assert abs(p16 - pref) <= PSNR_TOL_DB
    assert stats["iters_run"] == c["cfg"]["n_iter"]
    np.testing.assert_allclose(stats["hist"][:, 0], c["ref_stats"][:, 0], rtol=SOLVE_TOL[st])


@pytest.mark.parametrize("st", ["f16", "bf16"])
def test_resume_16bit_bitwise(lfsr, st):
    """read_state -> write_state loses nothing: x splits exactly, the duals
    come back in the storage type they were read from."""
    c = _case("ragged")
    y, d = _t(c["y"]), _t(c["disp"])
    a = _solver(lfsr, c["cfg"], st)
    a.lfsr_init(y, d)
    a.lfsr_iterate(5)
    sa = a.lfsr_read_state()
    b = _solver(lfsr, c["cfg"], st)
    b.lfsr_init(y, d)
    b.lfsr_iterate(2)
    sb = b.lfsr_read_state()
    r = _solver(lfsr, c["cfg"], st)
    r.lfsr_init(y, d)
    r.lfsr_write_state(sb["x"], sb["wD"], sb["wS"], sb["m"], 2)
    r.lfsr_iterate(3)
    sr = r.lfsr_read_state()
    for key in ("x", "wD", "wS", "m"):
        np.testing.assert_array_equal(_n(sa[key]), _n(sr[key]))


@pytest.mark.parametrize("st", ["f16", "bf16"])
def test_deterministic_bits_16bit(lfsr, st):
    c = _case("ragged")
    s = _solver(lfsr, c["cfg"], st)
    y, d = _t(c["y"]), _t(c["disp"])
    x1, _ = s.lfsr_solve(y, d)
    x1 = _n(x1)
    x2, _ = s.lfsr_solve(y, d)
    np.testing.assert_array_equal(x1, _n(x2))
