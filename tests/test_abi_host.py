"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, validates parameters and sizes the workspace.  No call here
touches a GPU."""
import ctypes
import os
import re

import pytest

from paper_2206_05047_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lfsr():
    from paper_2206_05047_amd import lfsr as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_2206_05047_amd import build
        build.build()
    mod.load()
    return mod


def _declared():
    src = open(os.path.join(ROOT, "include", "lfsr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lfsr_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_names(lfsr):
    assert _declared() == sorted(lfsr.EXPORTS)


def test_library_exports_every_declared_symbol(lfsr):
    lib = ctypes.CDLL(lfsr.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def _params(lfsr, name="c1", **over):
    return lfsr.make_params(synth.config(name), **over)


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_workspace_covers_the_state(lfsr, name):
    c = synth.config(name)
    p = _params(lfsr, name)
    n = lfsr.workspace_bytes(p)
    H, W = c["zeta"] * c["sy"], c["zeta"] * c["sx"]
    sk, sd = c["U"] * c["V"], c["win"] ** 2 - 1
    state = 4 * (H * W * 6 + 2 * sk * c["sy"] * c["sx"] + 2 * sd * H * W)
    assert state <= n <= state * 1.5 + (1 << 20)


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_16bit_storage_halves_the_stored_fields(lfsr, name):
    """With F16/BF16 storage x, w_D, w_S and the LR stack take 2 bytes per
    element; an FP32 remainder of x is added (the CG accumulator)."""
    c = synth.config(name)
    H, W = c["zeta"] * c["sy"], c["zeta"] * c["sx"]
    sk, sd, q = c["U"] * c["V"], c["win"] ** 2 - 1, c["sy"] * c["sx"]
    n32 = lfsr.workspace_bytes(_params(lfsr, name))
    saved = 2 * (H * W + 2 * sk * q + 2 * sd * H * W) - 4 * H * W
    for st in (lfsr.LFSR_F16, lfsr.LFSR_BF16):
        p = _params(lfsr, name)
        p.storage = st
        n16 = lfsr.workspace_bytes(p)
        assert abs((n32 - n16) - saved) <= 256 * 8


@pytest.mark.parametrize("field,value", [
    ("ang_rows", 64), ("ang_cols", 0), ("lr_h", 0), ("scale", 0), ("scale", 9), ("n_disp", 2), ("n_disp", 8),
    ("blur_size", 4), ("blur_size", 33), ("lambda1", -1.0), ("nltv_window", 4), ("nltv_window", 17),
    ("sigma_s", 0.0), ("sigma_e", 0.0), ("admm_penalty", 0.0), ("admm_iters", 0), ("cg_iters", -1),
    ("cg_tol", -1.0), ("stop_tol", float("nan")), ("disp_bound", 0.0), ("disp_bound", float("inf")),
    ("reweight", 2), ("storage", 7), ("spatial_weight", 2),
])
def test_invalid_params_rejected(lfsr, field, value):
    p = _params(lfsr)
    setattr(p, field, value)
    assert lfsr.load().lfsr_workspace_bytes(ctypes.byref(p)) == 0
    assert lfsr.last_error() != "no error"
    h = ctypes.c_void_p()
    code = lfsr.load().lfsr_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), 1 << 40, ctypes.byref(h))
    assert code == lfsr.LFSR_EINVAL and not h.value


def test_both_lambdas_zero_rejected(lfsr):
    p = _params(lfsr, lambda1=0.0, lambda2=0.0)
    assert lfsr.load().lfsr_workspace_bytes(ctypes.byref(p)) == 0
    assert "lambda" in lfsr.last_error()


def test_paper_default_blur_accepted(lfsr):
    p = _params(lfsr, blur_size=0, blur_sigma=0.0)
    assert lfsr.workspace_bytes(p) > 0


def test_disparity_bound_too_large_rejected(lfsr):
    p = _params(lfsr, "c3", disp_bound=60.0)
    assert lfsr.load().lfsr_workspace_bytes(ctypes.byref(p)) == 0
    assert "disp_bound" in lfsr.last_error()


def test_create_checks_workspace(lfsr):
    lib = lfsr.load()
    p = _params(lfsr)
    need = lfsr.workspace_bytes(p)
    h = ctypes.c_void_p()
    assert lib.lfsr_create(ctypes.byref(p), None, need, ctypes.byref(h)) == lfsr.LFSR_ENOMEM
    assert lib.lfsr_create(ctypes.byref(p), ctypes.c_void_p(4096 + 8), need, ctypes.byref(h)) == lfsr.LFSR_EINVAL
    assert lib.lfsr_create(ctypes.byref(p), ctypes.c_void_p(4096), need - 1, ctypes.byref(h)) == lfsr.LFSR_ENOMEM
    assert "too small" in lfsr.last_error()
    # creation is host-only: a fake (never dereferenced) aligned address is fine
    assert lib.lfsr_create(ctypes.byref(p), ctypes.c_void_p(1 << 32), need, ctypes.byref(h)) == lfsr.LFSR_OK
    assert h.value
    assert lib.lfsr_last_error(h) == b"no error"
    lib.lfsr_destroy(h)
    lib.lfsr_destroy(None)


def test_null_handle_calls_fail_cleanly(lfsr):
    lib = lfsr.load()
    assert lib.lfsr_iterate(None, 1, None) == lfsr.LFSR_EINVAL
    assert lib.lfsr_init(None, None, None, None, None, None) == lfsr.LFSR_EINVAL
    assert lib.lfsr_forward(None, None, None, None, None) == lfsr.LFSR_EINVAL
    assert "NULL" in lfsr.last_error()


def test_iterate_before_init_is_a_state_error(lfsr):
    lib = lfsr.load()
    p = _params(lfsr)
    h = ctypes.c_void_p()
    assert lib.lfsr_create(ctypes.byref(p), ctypes.c_void_p(1 << 32), lfsr.workspace_bytes(p), ctypes.byref(h)) == 0
    assert lib.lfsr_iterate(h, 1, None) == lfsr.LFSR_ESTATE
    assert lib.lfsr_init(h, None, None, None, None, None) == lfsr.LFSR_EINVAL
    lib.lfsr_destroy(h)


def test_pool_argument_errors(lfsr):
    """Pool creation checks its arguments before touching the device."""
    lib = lfsr.load()
    h = ctypes.c_void_p()
    assert lib.lfsr_pool_create(None, 1 << 20, 4, ctypes.byref(h)) == lfsr.LFSR_ENOMEM and not h.value
    assert lib.lfsr_pool_create(ctypes.c_void_p(1 << 20), 0, 4, ctypes.byref(h)) == lfsr.LFSR_ENOMEM
    assert lib.lfsr_pool_create(ctypes.c_void_p((1 << 20) + 8), 1 << 20, 4, ctypes.byref(h)) == lfsr.LFSR_EINVAL
    for slots in (0, 65):
        assert lib.lfsr_pool_create(ctypes.c_void_p(1 << 20), 1 << 20, slots, ctypes.byref(h)) == lfsr.LFSR_EINVAL
    assert lib.lfsr_pool_last_error(None).decode() != "no error"
    n = ctypes.c_int32()
    assert lib.lfsr_pool_tick(None, None, ctypes.byref(n)) == lfsr.LFSR_EINVAL
    assert lib.lfsr_pool_poll(None, None, None, None, 0, ctypes.byref(n)) == lfsr.LFSR_EINVAL
    assert lib.lfsr_pool_info(None, None, None, None, None) == lfsr.LFSR_EINVAL
    jid = ctypes.c_int64()
    p = _params(lfsr)
    assert lib.lfsr_pool_submit(None, ctypes.byref(p), None, None, None, None, None, None,
                                ctypes.byref(jid)) == lfsr.LFSR_EINVAL
    lib.lfsr_pool_destroy(None)


def test_per_view_maps_accepted(lfsr):
    """n_disp = 1 (one map) or ang_rows*ang_cols (one map per view); the maps
    are inputs, so the workspace holds the same state either way (its size
    differs only by the tiling's partial images)."""
    one = lfsr.workspace_bytes(_params(lfsr, "c1"))
    per = lfsr.workspace_bytes(_params(lfsr, "c1", n_disp=9))
    assert per > 0 and abs(per - one) < 0.2 * one


def test_btv_weight_needs_alpha_at_most_one(lfsr):
    assert lfsr.workspace_bytes(_params(lfsr, weight_kind=1, sigma_s=0.7)) > 0
    p = _params(lfsr, weight_kind=1, sigma_s=1.5)
    assert lfsr.load().lfsr_workspace_bytes(ctypes.byref(p)) == 0
    assert "BTV" in lfsr.last_error()


def test_even_angular_grid_accepted(lfsr):
    """The 2 x 2 images of the x2 multi-image workload: offsets 0..1."""
    assert lfsr.workspace_bytes(_params(lfsr, U=2, V=2)) > 0
