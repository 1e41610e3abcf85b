"""FP64 CPU oracle for the ADMM light-field super-resolution method of
arXiv 2206.05047 ("GPU-accelerated light-field super-resolution").

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke entry and the CPU-baseline
leg of the benchmark are the only callers.  The product path never imports
this package.  It shares no code with the HIP library; the two meet only at
the seeded input generator, which holds none of the method's arithmetic.

The numerical work lives in ``lfsr_oracle.c`` (plain double-precision loops);
this module is argument marshalling over ctypes plus ``solve``, which strings
the C steps together exactly as the paper's Algorithm 1 does (sec 5).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblfsr_oracle.so")
_lib = None

NSTAT = 6  # per-iteration statistics, see orc_admm_iterate


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("U", ctypes.c_int32),
        ("V", ctypes.c_int32),
        ("sy", ctypes.c_int32),
        ("sx", ctypes.c_int32),
        ("zeta", ctypes.c_int32),
        ("n_disp", ctypes.c_int32),
        ("kb", ctypes.c_int32),
        ("sigma_b", ctypes.c_double),
        ("lambda1", ctypes.c_double),
        ("lambda2", ctypes.c_double),
        ("win", ctypes.c_int32),
        ("sigma_s", ctypes.c_double),
        ("sigma_e", ctypes.c_double),
        ("reweight", ctypes.c_int32),
        ("theta", ctypes.c_double),
        ("cg_iter", ctypes.c_int32),
        ("cg_tol", ctypes.c_double),
        ("weight_kind", ctypes.c_int32),
        ("blur_taps", ctypes.POINTER(ctypes.c_double)),
    ]


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE arithmetic, OpenMP)."""
    from .buildlib import build_oracle

    return build_oracle(verbose=verbose)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(OrcParams)
    D = ctypes.POINTER(ctypes.c_double)
    I = ctypes.c_int
    sigs = {
        "orc_num_threads": ([], I),
        "orc_ref_view": ([P], I),
        "orc_blur_kernel": ([P, D], None),
        "orc_warp": ([P, D, D, I, D], None),
        "orc_warp_t_acc": ([P, D, D, I, D], None),
        "orc_blur": ([P, D, D], None),
        "orc_blur_t": ([P, D, D], None),
        "orc_down": ([P, D, D], None),
        "orc_up": ([P, D, D], None),
        "orc_forward": ([P, D, D, D], None),
        "orc_adjoint": ([P, D, D, D], None),
        "orc_spatial_weight": ([P, I, I], ctypes.c_double),
        "orc_edge_weight": ([P, D, D, D], None),
        "orc_nltv_grad": ([P, D, D, D], None),
        "orc_nltv_div": ([P, D, D, D], None),
        "orc_bicubic": ([P, D, D], None),
        "orc_normal_apply": ([P, D, D, D, D], None),
        "orc_cg": ([P, D, D, D, D, D], I),
        "orc_soft_threshold": ([ctypes.c_double, ctypes.c_double], ctypes.c_double),
        "orc_admm_iterate": ([P, D, D, D, D, D, D, D, I, I, D], None),
        "orc_objective": ([P, D, D, D, D], ctypes.c_double),
        "orc_occlusion_weight": ([P, D, D, ctypes.c_double, ctypes.c_double, D], None),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    lib.orc_view_offset.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.orc_view_offset.restype = None
    lib.orc_offset.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.orc_offset.restype = None
    _lib = lib
    return lib


@dataclass
class Problem:
    """Shape and parameters of one solve (the paper's problem statement)."""

    U: int
    V: int
    sy: int
    sx: int
    zeta: int
    kb: int
    sigma_b: float
    lambda1: float
    lambda2: float
    win: int
    sigma_s: float
    sigma_e: float
    theta: float
    n_iter: int
    cg_iter: int
    cg_tol: float = 0.0
    reweight: int = 1
    n_disp: int = 1
    weight_kind: int = 0
    blur_taps: object = None  # None: Gaussian; else a [kb][kb] correlation kernel

    @classmethod
    def from_any(cls, cfg) -> "Problem":
        if isinstance(cfg, Problem):
            return cfg
        get = (lambda k: cfg[k]) if isinstance(cfg, dict) else (lambda k: getattr(cfg, k))
        kw = {}
        for f in cls.__dataclass_fields__:
            try:
                kw[f] = get(f)
            except (KeyError, AttributeError):
                pass
        return cls(**kw)

    @property
    def H(self) -> int:
        return self.zeta * self.sy

    @property
    def W(self) -> int:
        return self.zeta * self.sx

    @property
    def sk(self) -> int:
        return self.U * self.V

    @property
    def sd(self) -> int:
        return self.win * self.win - 1

    def c(self) -> OrcParams:
        return OrcParams(
            self.U, self.V, self.sy, self.sx, self.zeta, self.n_disp, self.kb, float(self.sigma_b),
            float(self.lambda1), float(self.lambda2), self.win, float(self.sigma_s),
            float(self.sigma_e), int(self.reweight), float(self.theta), self.cg_iter,
            float(self.cg_tol), int(self.weight_kind),
            _d(self._taps) if self._taps is not None else None,
        )

    def __post_init__(self):
        self._taps = None
        if self.blur_taps is not None:
            t = np.ascontiguousarray(np.asarray(self.blur_taps, dtype=np.float64))
            assert t.shape == (self.kb, self.kb), (t.shape, self.kb)
            self._taps = t


def _d(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """Typed access to the FP64 oracle for one problem shape."""

    def __init__(self, cfg):
        self.pb = Problem.from_any(cfg)
        self.lib = _load()
        self._p = self.pb.c()
        self._pp = ctypes.byref(self._p)

    # -- shapes
    @property
    def hr_shape(self):
        return (self.pb.H, self.pb.W)

    @property
    def lr_shape(self):
        return (self.pb.sk, self.pb.sy, self.pb.sx)

    def _disp(self, disp):
        pb = self.pb
        shape = (pb.H, pb.W) if pb.n_disp == 1 else (pb.sk, pb.H, pb.W)
        return _f64(disp, shape)

    # -- geometry
    def view_offset(self, k):
        t, r = ctypes.c_int(), ctypes.c_int()
        self.lib.orc_view_offset(self._pp, k, ctypes.byref(t), ctypes.byref(r))
        return t.value, r.value

    def offset(self, d):
        a, b = ctypes.c_int(), ctypes.c_int()
        self.lib.orc_offset(self._pp, d, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def spatial_weight(self, dy, dx):
        return self.lib.orc_spatial_weight(self._pp, dy, dx)

    def blur_kernel(self):
        h = np.zeros((self.pb.kb, self.pb.kb))
        self.lib.orc_blur_kernel(self._pp, _d(h))
        return h

    # -- single operators (sec 4.1)
    def warp(self, x, disp, k):
        x = _f64(x, self.hr_shape)
        out = np.zeros(self.hr_shape)
        self.lib.orc_warp(self._pp, _d(x), _d(self._disp(disp)), k, _d(out))
        return out

    def warp_t(self, u, disp, k):
        u = _f64(u, self.hr_shape)
        out = np.zeros(self.hr_shape)
        self.lib.orc_warp_t_acc(self._pp, _d(u), _d(self._disp(disp)), k, _d(out))
        return out

    def blur(self, u):
        u = _f64(u, self.hr_shape)
        out = np.zeros(self.hr_shape)
        self.lib.orc_blur(self._pp, _d(u), _d(out))
        return out

    def blur_t(self, u):
        u = _f64(u, self.hr_shape)
        out = np.zeros(self.hr_shape)
        self.lib.orc_blur_t(self._pp, _d(u), _d(out))
        return out

    def down(self, u):
        u = _f64(u, self.hr_shape)
        out = np.zeros((self.pb.sy, self.pb.sx))
        self.lib.orc_down(self._pp, _d(u), _d(out))
        return out

    def up(self, lr):
        lr = _f64(lr, (self.pb.sy, self.pb.sx))
        out = np.zeros(self.hr_shape)
        self.lib.orc_up(self._pp, _d(lr), _d(out))
        return out

    def forward(self, x, disp):
        """A_k x for every view -> [sk][sy][sx]."""
        x = _f64(x, self.hr_shape)
        out = np.zeros(self.lr_shape)
        self.lib.orc_forward(self._pp, _d(x), _d(self._disp(disp)), _d(out))
        return out

    def adjoint(self, e, disp):
        """sum_k A_k^T e_k -> [H][W]."""
        e = _f64(e, self.lr_shape)
        out = np.zeros(self.hr_shape)
        self.lib.orc_adjoint(self._pp, _d(e), _d(self._disp(disp)), _d(out))
        return out

    def edge_weight(self, x, occ=None):
        x = _f64(x, self.hr_shape)
        m = np.zeros(self.hr_shape)
        o = _f64(occ, self.hr_shape) if occ is not None else None
        self.lib.orc_edge_weight(self._pp, _d(x), _d(o) if o is not None else None, _d(m))
        return m

    def nltv_grad(self, x, m):
        x = _f64(x, self.hr_shape)
        m = _f64(m, self.hr_shape)
        g = np.zeros((max(self.pb.sd, 0),) + self.hr_shape)
        if self.pb.sd > 0:
            self.lib.orc_nltv_grad(self._pp, _d(x), _d(m), _d(g))
        return g

    def nltv_div(self, g, m):
        g = _f64(g, (self.pb.sd,) + self.hr_shape)
        m = _f64(m, self.hr_shape)
        out = np.zeros(self.hr_shape)
        self.lib.orc_nltv_div(self._pp, _d(g), _d(m), _d(out))
        return out

    def bicubic(self, lr_ref):
        lr = _f64(lr_ref, (self.pb.sy, self.pb.sx))
        out = np.zeros(self.hr_shape)
        self.lib.orc_bicubic(self._pp, _d(lr), _d(out))
        return out

    def occlusion_weight(self, y, disp, sigma_o1, sigma_o2):
        """Occlusion weight w_o [H][W] (sec 3.4, eq. weight_occ) from the LR
        views and the reference view's disparity map."""
        y = _f64(y, self.lr_shape)
        out = np.zeros(self.hr_shape)
        self.lib.orc_occlusion_weight(self._pp, _d(y), _d(self._disp(disp)), ctypes.c_double(sigma_o1),
                                      ctypes.c_double(sigma_o2), _d(out))
        return out

    def x0(self, y):
        """Bicubic up-sampling of the reference view."""
        y = _f64(y, self.lr_shape)
        return self.bicubic(y[self.ref_view()])

    def ref_view(self):
        """Index of the reference view (angular offset (0, 0))."""
        return self.lib.orc_ref_view(self._pp)

    def normal_apply(self, disp, m, x):
        x = _f64(x, self.hr_shape)
        out = np.zeros(self.hr_shape)
        self.lib.orc_normal_apply(self._pp, _d(self._disp(disp)), _d(_f64(m, self.hr_shape)), _d(x), _d(out))
        return out

    def cg(self, disp, m, v):
        v = _f64(v, self.hr_shape)
        delta = np.zeros(self.hr_shape)
        pi = np.zeros(1)
        steps = self.lib.orc_cg(self._pp, _d(self._disp(disp)), _d(_f64(m, self.hr_shape)), _d(v), _d(delta), _d(pi))
        return delta, float(pi[0]), int(steps)

    def objective(self, y, disp, m, x):
        return self.lib.orc_objective(
            self._pp, _d(_f64(y, self.lr_shape)), _d(self._disp(disp)), _d(_f64(m, self.hr_shape)),
            _d(_f64(x, self.hr_shape)))

    # -- ADMM (sec 5, Algorithm 1)
    def init_state(self, y, x0=None):
        pb = self.pb
        x = self.x0(y) if x0 is None else _f64(x0, self.hr_shape).copy()
        return {
            "x": x,
            "wD": np.zeros(self.lr_shape),
            "wS": np.zeros((pb.sd,) + self.hr_shape),
            "m": np.ones(self.hr_shape),
            "n": 0,
        }

    def iterate(self, state, y, disp, occ=None, count=1):
        """Advance `state` (dict from init_state) by `count` ADMM iterations in
        place; returns the [count][NSTAT] statistics."""
        y = _f64(y, self.lr_shape)
        o = _f64(occ, self.hr_shape) if occ is not None else None
        stats = np.zeros((count, NSTAT))
        for key in ("x", "wD", "wS", "m"):
            assert state[key].flags["C_CONTIGUOUS"] and state[key].dtype == np.float64
        self.lib.orc_admm_iterate(
            self._pp, _d(y), _d(self._disp(disp)), _d(o) if o is not None else None,
            _d(state["x"]), _d(state["wD"]), _d(state["wS"]) if self.pb.sd > 0 else _d(np.zeros(1)),
            _d(state["m"]), int(state["n"]) + 1, int(count), _d(stats))
        state["n"] += count
        return stats

    def solve(self, y, disp, occ=None, x0=None, n_iter=None):
        """Full solve: x0 (bicubic of the reference view unless given), w = 0,
        then N ADMM iterations.  Returns (x, stats)."""
        st = self.init_state(y, x0)
        n = self.pb.n_iter if n_iter is None else n_iter
        stats = self.iterate(st, y, disp, occ, count=n)
        return st["x"], stats

    # -- gradient descent baselines (sec 7.1: gd and gd-ls against ADMM)
    def cost_parts(self, y, disp, m, x):
        """J(x) (sec 4, cost J), and the two factors of a subgradient: q =
        lambda1 sgn(r) + 2 lambda2 r on the LR views (r = A x - y) and
        S^T sgn(V (I - S) x) on the HR grid (sgn(0) = 0)."""
        pb = self.pb
        r = self.forward(x, disp) - _f64(y, self.lr_shape)
        g = self.nltv_grad(x, m)
        J = pb.lambda1 * np.abs(r).sum() + pb.lambda2 * (r * r).sum() + np.abs(g).sum()
        q = pb.lambda1 * np.sign(r) + 2.0 * pb.lambda2 * r
        t = self.nltv_div(np.sign(g), m) if pb.sd > 0 else np.zeros(self.hr_shape)
        return J, q, t

    def gd(self, y, disp, iters, step, line_search=False, x0=None, occ=None):
        """Subgradient descent on J with the weights fixed at m = w_e(x0) w_o
        (the comparison of sec 7.1).  Each step costs computation units (CU)
        as the paper counts them: one CU is A with S (the cost), or A^T with
        S^T (the gradient).  Fixed step (gd): x <- x - step g, 2 CU.  With
        line search (gd-ls): backtracking from twice the last accepted step
        (the first from `step`), halving until the Armijo condition
        J(x - eta g) <= J(x) - 1e-4 eta |g|^2 holds (one CU per trial, at most
        30 trials, else the step is skipped), then A^T for the new gradient.
        Returns (x, hist) with hist[n] = (J(x_n), CU spent after step n,
        eta) for n = 0 (x0) .. iters."""
        x = self.x0(y) if x0 is None else _f64(x0, self.hr_shape).copy()
        m = self.edge_weight(x, occ)
        J, q, t = self.cost_parts(y, disp, m, x)
        g = self.adjoint(q, disp) + t
        cu = 2
        hist = [(J, cu, 0.0)]
        eta = step
        for _ in range(iters):
            if not line_search:
                x = x - step * g
                J, q, t = self.cost_parts(y, disp, m, x)
                g = self.adjoint(q, disp) + t
                cu += 2
                hist.append((J, cu, step))
                continue
            gg = float((g * g).sum())
            eta = 2.0 * eta if len(hist) > 1 else step
            for _trial in range(30):
                xc = x - eta * g
                Jc, qc, tc = self.cost_parts(y, disp, m, xc)
                cu += 1
                if Jc <= J - 1e-4 * eta * gg:
                    x, J, q, t = xc, Jc, qc, tc
                    g = self.adjoint(q, disp) + t
                    cu += 1
                    break
                eta *= 0.5
            hist.append((J, cu, eta))
        return x, np.array(hist)

    def soft(self, u, t):
        return self.lib.orc_soft_threshold(float(u), float(t))

    @staticmethod
    def num_threads():
        return _load().orc_num_threads()
