"""Python binding of the C ABI in include/lfsr.h (ctypes).

Argument marshalling only: torch tensors provide device memory and streams,
every step of the solver runs in the HIP library.  There is no fallback: if
the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch  # imported before the library so both share torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblfsr.so")
_lib = None

LFSR_OK, LFSR_EINVAL, LFSR_ENOMEM, LFSR_EDEVICE, LFSR_ESTATE, LFSR_ENONFINITE, LFSR_EBUSY = 0, -1, -2, -3, -4, -5, -6
LFSR_F32, LFSR_F16, LFSR_BF16 = 0, 1, 2
LFSR_NSTAT = 6

EXPORTS = [
    "lfsr_workspace_bytes", "lfsr_create", "lfsr_destroy", "lfsr_last_error", "lfsr_solve", "lfsr_init",
    "lfsr_iterate", "lfsr_read_state", "lfsr_write_state", "lfsr_get_stats", "lfsr_forward", "lfsr_adjoint",
    "lfsr_normal", "lfsr_edge_weight", "lfsr_bicubic", "lfsr_profile_begin", "lfsr_profile_end",
    "lfsr_pool_create", "lfsr_pool_destroy", "lfsr_pool_last_error", "lfsr_pool_submit", "lfsr_pool_tick",
    "lfsr_pool_poll", "lfsr_pool_info", "lfsr_solve_noalloc",
    "lfsr_occlusion_weight", "lfsr_gd",
]
LFSR_K_FORWARD, LFSR_K_ADJOINT, LFSR_K_NLTV, LFSR_K_NORMAL, LFSR_K_CG, LFSR_K_OTHER, LFSR_K_COUNT = range(7)
KERNEL_KINDS = ["forward", "adjoint", "nltv", "normal", "cg", "other"]


class lfsr_params(ctypes.Structure):
    _fields_ = [
        ("ang_rows", ctypes.c_int32), ("ang_cols", ctypes.c_int32),
        ("lr_h", ctypes.c_int32), ("lr_w", ctypes.c_int32),
        ("scale", ctypes.c_int32), ("n_disp", ctypes.c_int32),
        ("blur_size", ctypes.c_int32), ("blur_sigma", ctypes.c_float),
        ("lambda1", ctypes.c_float), ("lambda2", ctypes.c_float),
        ("nltv_window", ctypes.c_int32),
        ("sigma_s", ctypes.c_float), ("sigma_e", ctypes.c_float),
        ("reweight", ctypes.c_int32),
        ("admm_penalty", ctypes.c_float),
        ("admm_iters", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
        ("cg_tol", ctypes.c_float), ("stop_tol", ctypes.c_float),
        ("disp_bound", ctypes.c_float),
        ("storage", ctypes.c_int32),
        ("spatial_weight", ctypes.c_int32),
        ("blur_taps", ctypes.POINTER(ctypes.c_float)),
    ]


class lfsr_stats(ctypes.Structure):
    _fields_ = [
        ("iters_run", ctypes.c_int32), ("cg_steps", ctypes.c_int32),
        ("objective", ctypes.c_double), ("primal_res", ctypes.c_double), ("cg_pi", ctypes.c_double),
        ("h_hist", ctypes.POINTER(ctypes.c_double)),
    ]


class LfsrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lfsr error {code}: {msg}")
        self.code = code


def load():
    """Load liblfsr.so (built by paper_2206_05047_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, V, F, I = ctypes.POINTER(lfsr_params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32
    H = ctypes.c_void_p
    lib.lfsr_workspace_bytes.argtypes = [P]
    lib.lfsr_workspace_bytes.restype = ctypes.c_size_t
    lib.lfsr_create.argtypes = [P, V, ctypes.c_size_t, ctypes.POINTER(H)]
    lib.lfsr_create.restype = I
    lib.lfsr_destroy.argtypes = [H]
    lib.lfsr_destroy.restype = None
    lib.lfsr_last_error.argtypes = [H]
    lib.lfsr_last_error.restype = ctypes.c_char_p
    lib.lfsr_solve.argtypes = [H, F, F, F, F, F, ctypes.POINTER(lfsr_stats), V]
    lib.lfsr_solve.restype = I
    lib.lfsr_solve_noalloc.argtypes = [P, F, F, F, F, F, ctypes.POINTER(lfsr_stats), V]
    lib.lfsr_solve_noalloc.restype = I
    lib.lfsr_init.argtypes = [H, F, F, F, F, V]
    lib.lfsr_init.restype = I
    lib.lfsr_iterate.argtypes = [H, I, V]
    lib.lfsr_iterate.restype = I
    lib.lfsr_read_state.argtypes = [H, F, F, F, F, V]
    lib.lfsr_read_state.restype = I
    lib.lfsr_write_state.argtypes = [H, F, F, F, F, I, V]
    lib.lfsr_write_state.restype = I
    lib.lfsr_get_stats.argtypes = [H, ctypes.POINTER(lfsr_stats), V]
    lib.lfsr_get_stats.restype = I
    for name in ("lfsr_forward", "lfsr_adjoint"):
        getattr(lib, name).argtypes = [H, F, F, F, V]
        getattr(lib, name).restype = I
    lib.lfsr_normal.argtypes = [H, F, F, F, F, V]
    lib.lfsr_normal.restype = I
    lib.lfsr_edge_weight.argtypes = [H, F, F, F, V]
    lib.lfsr_edge_weight.restype = I
    lib.lfsr_occlusion_weight.argtypes = [H, F, F, ctypes.c_float, ctypes.c_float, F, V]
    lib.lfsr_occlusion_weight.restype = I
    lib.lfsr_gd.argtypes = [H, I, ctypes.c_float, I, ctypes.POINTER(ctypes.c_double), V]
    lib.lfsr_gd.restype = I
    lib.lfsr_bicubic.argtypes = [H, F, F, V]
    lib.lfsr_bicubic.restype = I
    lib.lfsr_profile_begin.argtypes = [H, ctypes.c_uint32, I]
    lib.lfsr_profile_begin.restype = I
    lib.lfsr_profile_end.argtypes = [H, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    lib.lfsr_profile_end.restype = I
    PL = ctypes.c_void_p
    lib.lfsr_pool_create.argtypes = [V, ctypes.c_size_t, I, ctypes.POINTER(PL)]
    lib.lfsr_pool_create.restype = I
    lib.lfsr_pool_destroy.argtypes = [PL]
    lib.lfsr_pool_destroy.restype = None
    lib.lfsr_pool_last_error.argtypes = [PL]
    lib.lfsr_pool_last_error.restype = ctypes.c_char_p
    lib.lfsr_pool_submit.argtypes = [PL, P, F, F, F, F, F, V, ctypes.POINTER(ctypes.c_int64)]
    lib.lfsr_pool_submit.restype = I
    lib.lfsr_pool_tick.argtypes = [PL, V, ctypes.POINTER(I)]
    lib.lfsr_pool_tick.restype = I
    lib.lfsr_pool_poll.argtypes = [PL, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(I), ctypes.POINTER(I), I,
                                   ctypes.POINTER(I)]
    lib.lfsr_pool_poll.restype = I
    lib.lfsr_pool_info.argtypes = [PL, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_size_t)]
    lib.lfsr_pool_info.restype = I
    _lib = lib
    return lib


def last_error(handle=None) -> str:
    return load().lfsr_last_error(handle).decode()


STORAGE = {"f32": LFSR_F32, "f16": LFSR_F16, "bf16": LFSR_BF16}


def make_params(cfg: dict, **over) -> lfsr_params:
    """lfsr_params from a workload dict (keys as in synth.CONFIGS); `storage`
    may be an lfsr_storage value or one of "f32", "f16", "bf16"."""
    c = dict(cfg)
    c.update(over)
    if isinstance(c.get("storage"), str):
        c["storage"] = STORAGE[c["storage"]]
    taps = c.get("blur_taps")
    if taps is not None:  # explicit kernel: kept alive on the struct (lfsr_create copies it)
        import numpy as np
        taps = np.ascontiguousarray(np.asarray(taps, dtype=np.float32))
        c["kb"] = int(taps.shape[0])
    prm = lfsr_params(
        ang_rows=c["U"], ang_cols=c["V"], lr_h=c["sy"], lr_w=c["sx"], scale=c["zeta"],
        n_disp=c.get("n_disp", 1), blur_size=c["kb"], blur_sigma=c["sigma_b"],
        lambda1=c["lambda1"], lambda2=c["lambda2"], nltv_window=c["win"],
        sigma_s=c["sigma_s"], sigma_e=c["sigma_e"], reweight=c.get("reweight", 1),
        admm_penalty=c["theta"], admm_iters=c["n_iter"], cg_iters=c["cg_iter"],
        cg_tol=c.get("cg_tol", 0.0), stop_tol=c.get("stop_tol", 0.0),
        disp_bound=c.get("disp_bound", 2.0), storage=c.get("storage", LFSR_F32),
        spatial_weight=c.get("weight_kind", 0),
        blur_taps=taps.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if taps is not None else None,
    )
    prm._taps = taps
    return prm


def workspace_bytes(params: lfsr_params) -> int:
    n = load().lfsr_workspace_bytes(ctypes.byref(params))
    if n == 0:
        raise LfsrError(LFSR_EINVAL, last_error())
    return int(n)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float32, (t.device, t.dtype)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One lfsr_handle over a torch-allocated workspace."""

    def __init__(self, params: lfsr_params, device="cuda"):
        self.lib = load()
        self.params = params
        self.device = torch.device(device)
        self.bytes = workspace_bytes(params)
        self.workspace = torch.empty(self.bytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        self._check(self.lib.lfsr_create(ctypes.byref(params), ctypes.c_void_p(self.workspace.data_ptr()),
                                         self.bytes, ctypes.byref(h)), None)
        self.handle = h
        p = params
        self.H, self.W = p.scale * p.lr_h, p.scale * p.lr_w
        self.sk = p.ang_rows * p.ang_cols
        self.sd = p.nltv_window * p.nltv_window - 1

    def _check(self, code, h):
        if code != LFSR_OK:
            raise LfsrError(code, self.lib.lfsr_last_error(h).decode())

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.lfsr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tensor helpers
    def _empty(self, *shape):
        return torch.empty(shape, dtype=torch.float32, device=self.device)

    # -- C ABI, one method per entry point
    def lfsr_solve(self, y, disp, occ=None, x0=None, out=None, stats=True, stream=None):
        out = self._empty(self.H, self.W) if out is None else out
        st, hist = self._stats_buf() if stats else (None, None)
        self._check(self.lib.lfsr_solve(self.handle, _ptr(y), _ptr(disp), _ptr(occ), _ptr(x0), _ptr(out),
                                        ctypes.byref(st) if st is not None else None, _stream(stream)), self.handle)
        return out, (self._stats_dict(st, hist) if stats else None)

    def lfsr_init(self, y, disp, occ=None, x0=None, stream=None):
        self._bound = (y, disp, occ, x0)  # keep the inputs alive while bound
        self._check(self.lib.lfsr_init(self.handle, _ptr(y), _ptr(disp), _ptr(occ), _ptr(x0), _stream(stream)),
                    self.handle)

    def lfsr_iterate(self, count=1, stream=None):
        self._check(self.lib.lfsr_iterate(self.handle, int(count), _stream(stream)), self.handle)

    def lfsr_read_state(self, stream=None):
        p = self.params
        x = self._empty(self.H, self.W)
        wd = self._empty(self.sk, p.lr_h, p.lr_w)
        ws = self._empty(max(self.sd, 0), self.H, self.W)
        m = self._empty(self.H, self.W)
        self._check(self.lib.lfsr_read_state(self.handle, _ptr(x), _ptr(wd), _ptr(ws) if self.sd > 0 else None,
                                             _ptr(m), _stream(stream)), self.handle)
        return {"x": x, "wD": wd, "wS": ws, "m": m}

    def lfsr_write_state(self, x, wd, ws, m, n_done, stream=None):
        self._check(self.lib.lfsr_write_state(self.handle, _ptr(x), _ptr(wd), _ptr(ws) if self.sd > 0 else None,
                                              _ptr(m), int(n_done), _stream(stream)), self.handle)

    def _stats_buf(self):
        hist = (ctypes.c_double * (self.params.admm_iters * LFSR_NSTAT))()
        st = lfsr_stats()
        st.h_hist = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        return st, hist

    def _stats_dict(self, st, hist):
        import numpy as np
        n = min(st.iters_run, self.params.admm_iters)
        h = np.frombuffer(hist, dtype=np.float64).reshape(self.params.admm_iters, LFSR_NSTAT)[:n].copy()
        return {"iters_run": st.iters_run, "cg_steps": st.cg_steps, "objective": st.objective,
                "primal_res": st.primal_res, "cg_pi": st.cg_pi, "hist": h}

    def lfsr_get_stats(self, stream=None):
        st, hist = self._stats_buf()
        self._check(self.lib.lfsr_get_stats(self.handle, ctypes.byref(st), _stream(stream)), self.handle)
        return self._stats_dict(st, hist)

    def lfsr_forward(self, x, disp, out=None, stream=None):
        p = self.params
        out = self._empty(self.sk, p.lr_h, p.lr_w) if out is None else out
        self._check(self.lib.lfsr_forward(self.handle, _ptr(x), _ptr(disp), _ptr(out), _stream(stream)), self.handle)
        return out

    def lfsr_adjoint(self, lr, disp, out=None, stream=None):
        out = self._empty(self.H, self.W) if out is None else out
        self._check(self.lib.lfsr_adjoint(self.handle, _ptr(lr), _ptr(disp), _ptr(out), _stream(stream)), self.handle)
        return out

    def lfsr_normal(self, pvec, disp, m, out=None, stream=None):
        out = self._empty(self.H, self.W) if out is None else out
        self._check(self.lib.lfsr_normal(self.handle, _ptr(pvec), _ptr(disp), _ptr(m), _ptr(out), _stream(stream)),
                    self.handle)
        return out

    def lfsr_edge_weight(self, x, occ=None, out=None, stream=None):
        out = self._empty(self.H, self.W) if out is None else out
        self._check(self.lib.lfsr_edge_weight(self.handle, _ptr(x), _ptr(occ), _ptr(out), _stream(stream)),
                    self.handle)
        return out

    def lfsr_occlusion_weight(self, lr, disp, sigma_o1, sigma_o2, out=None, stream=None):
        out = self._empty(self.H, self.W) if out is None else out
        self._check(self.lib.lfsr_occlusion_weight(self.handle, _ptr(lr), _ptr(disp), float(sigma_o1),
                                                   float(sigma_o2), _ptr(out), _stream(stream)), self.handle)
        return out

    def lfsr_gd(self, iters, step, line_search=False, stream=None):
        """Gradient-descent baseline on the bound inputs; returns the
        [iters + 1][3] history (J, computation units, step)."""
        import numpy as np
        hist = (ctypes.c_double * (3 * (int(iters) + 1)))()
        self._check(self.lib.lfsr_gd(self.handle, int(iters), float(step), int(bool(line_search)),
                                     ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), _stream(stream)),
                    self.handle)
        return np.frombuffer(hist, dtype=np.float64).reshape(int(iters) + 1, 3).copy()

    def lfsr_bicubic(self, lr_view, out=None, stream=None):
        out = self._empty(self.H, self.W) if out is None else out
        self._check(self.lib.lfsr_bicubic(self.handle, _ptr(lr_view), _ptr(out), _stream(stream)), self.handle)
        return out


    def lfsr_profile_begin(self, kinds=None, capacity=8192):
        mask = 0
        for k in (kinds if kinds is not None else range(LFSR_K_COUNT)):
            mask |= 1 << k
        self._check(self.lib.lfsr_profile_begin(self.handle, mask, int(capacity)), self.handle)

    def lfsr_profile_end(self):
        """{kind name: (total ms, timed launches)}"""
        tot = (ctypes.c_double * LFSR_K_COUNT)()
        cnt = (ctypes.c_int32 * LFSR_K_COUNT)()
        self._check(self.lib.lfsr_profile_end(self.handle, tot, cnt), self.handle)
        return {KERNEL_KINDS[k]: (tot[k], cnt[k]) for k in range(LFSR_K_COUNT)}


NOALLOC_MAX_BYTES = 64 << 20  # LFSR_NOALLOC_MAX_BYTES


def solve_noalloc(params: lfsr_params, y, disp, occ=None, x0=None, out=None, stats=False, stream=None):
    """lfsr_solve_noalloc: a complete solve over the library's static per-GPU
    scratch (no workspace allocation).  Returns (x, stats dict or None)."""
    lib = load()
    H, W = params.scale * params.lr_h, params.scale * params.lr_w
    out = torch.empty((H, W), dtype=torch.float32, device=y.device) if out is None else out
    st = hist = None
    if stats:
        hist = (ctypes.c_double * (params.admm_iters * LFSR_NSTAT))()
        st = lfsr_stats()
        st.h_hist = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    code = lib.lfsr_solve_noalloc(ctypes.byref(params), _ptr(y), _ptr(disp), _ptr(occ), _ptr(x0), _ptr(out),
                                  ctypes.byref(st) if st is not None else None, _stream(stream))
    if code != LFSR_OK:
        raise LfsrError(code, last_error())
    if not stats:
        return out, None
    import numpy as np
    n = min(st.iters_run, params.admm_iters)
    h = np.frombuffer(hist, dtype=np.float64).reshape(params.admm_iters, LFSR_NSTAT)[:n].copy()
    return out, {"iters_run": st.iters_run, "cg_steps": st.cg_steps, "objective": st.objective,
                 "primal_res": st.primal_res, "cg_pi": st.cg_pi, "hist": h}


def disp_bound_for(disp, margin=1.0) -> float:
    """A disp_bound covering a disparity map (host-side helper)."""
    import numpy as np
    m = float(np.max(np.abs(np.asarray(disp)))) if np.asarray(disp).size else 0.0
    return max(m * margin, 1e-3) if math.isfinite(m) else float("nan")


class Pool:
    """lfsr_pool over a torch-allocated device arena.  Each submitted job's
    tensors are kept alive until the job is harvested by lfsr_pool_poll."""

    def __init__(self, arena_bytes: int, max_slots: int = 16, device="cuda"):
        self.lib = load()
        self.device = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        self._check(self.lib.lfsr_pool_create(ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                              int(max_slots), ctypes.byref(h)), None)
        self.handle = h
        self.max_slots = int(max_slots)
        self.jobs = {}

    def _check(self, code, h):
        if code != LFSR_OK:
            raise LfsrError(code, self.lib.lfsr_pool_last_error(h).decode())

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.lfsr_pool_destroy(self.handle)
            self.handle = None
            self.jobs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lfsr_pool_submit(self, params: lfsr_params, y, disp, occ=None, x0=None, out=None, stream=None):
        """Job id, or None when the pool is full right now (LFSR_EBUSY)."""
        H, W = params.scale * params.lr_h, params.scale * params.lr_w
        out = torch.empty((H, W), dtype=torch.float32, device=self.device) if out is None else out
        jid = ctypes.c_int64()
        code = self.lib.lfsr_pool_submit(self.handle, ctypes.byref(params), _ptr(y), _ptr(disp), _ptr(occ),
                                         _ptr(x0), _ptr(out), _stream(stream), ctypes.byref(jid))
        if code == LFSR_EBUSY:
            return None
        self._check(code, self.handle)
        self.jobs[jid.value] = (params, y, disp, occ, x0, out)
        return jid.value

    def lfsr_pool_tick(self, stream=None) -> int:
        n = ctypes.c_int32()
        self._check(self.lib.lfsr_pool_tick(self.handle, _stream(stream), ctypes.byref(n)), self.handle)
        return n.value

    def lfsr_pool_poll(self, cap: int = 64):
        """[(job id, output tensor, status, iterations run)] of harvested jobs."""
        ids = (ctypes.c_int64 * cap)()
        st = (ctypes.c_int32 * cap)()
        it = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32()
        self._check(self.lib.lfsr_pool_poll(self.handle, ids, st, it, cap, ctypes.byref(n)), self.handle)
        res = []
        for i in range(n.value):
            job = self.jobs.pop(ids[i])
            res.append((ids[i], job[5], st[i], it[i]))
        return res

    def lfsr_pool_info(self):
        a, r = ctypes.c_int32(), ctypes.c_int32()
        f, big = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self.lib.lfsr_pool_info(self.handle, ctypes.byref(a), ctypes.byref(r), ctypes.byref(f),
                                            ctypes.byref(big)), self.handle)
        return {"active": a.value, "retiring": r.value, "free": f.value, "largest_free": big.value}
