"""Benchmark of the ADMM light-field super-resolution solve on one MI355X.

One step = one complete solve (lfsr_solve: x0, w = 0, N ADMM iterations of K
CG steps each, output copy) of the 9x9-view, 1152x1152, x3 workload with the
inputs resident in HBM.  Prints one JSON line: throughput in HR
Mpixel-views x ADMM iterations per second, the roofline of the dominant kernel
(its average launch duration measured with HIP events on its launch stream
over the timed region) and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HR Mpixel-views x ADMM iters/s + achieved HBM GB/s; p50/p99 job latency"
UNIT = "HR Mpixel-views x ADMM iters/s"
PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0      # MI355X published HBM3E bandwidth


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_flops_per_launch(kind, cfg):
    """Algorithmic FLOPs of one launch of a kernel kind:
    forward: per view-pixel 9 (bilinear as three lerps) + 2 kb/zeta
             (horizontal blur at lattice columns) + 2 kb/zeta^2 (vertical),
    adjoint: per view-pixel 2 kb/zeta + 2 kb/zeta^2 (polyphase B^T D^T)
             + 10 (bilinear-transpose weights and accumulation),
    normal:  per pixel 4 flops per NLTV offset."""
    H, W = cfg["zeta"] * cfg["sy"], cfg["zeta"] * cfg["sx"]
    sk, kb, z = cfg["U"] * cfg["V"], cfg["kb"], cfg["zeta"]
    vp = H * W * sk
    if kind == "forward":
        return vp * (9 + 2 * kb / z + 2 * kb / z ** 2)
    if kind == "adjoint":
        return vp * (2 * kb / z + 2 * kb / z ** 2 + 10)
    if kind == "normal":
        return H * W * 4 * (cfg["win"] ** 2 - 1)
    return None


def bytes_per_iteration(cfg, es=4):
    """Algorithmic HBM bytes of one ADMM iteration: the state and operator
    streams each iteration must move at least once (x, disparity, weight map,
    LR views, both duals read+written, e written and read, v; per CG step
    p, t = A p written and read, and ten HR-vector passes)."""
    H, W = cfg["zeta"] * cfg["sy"], cfg["zeta"] * cfg["sx"]
    p, q = H * W, cfg["sy"] * cfg["sx"]
    sk, sd, K = cfg["U"] * cfg["V"], cfg["win"] ** 2 - 1, cfg["cg_iter"]
    wz = p * es + 2 * p * 4 + sk * q * 4 + 2 * (sk * q + sd * p) * es + 2 * sk * q * es + p * 4
    cg = K * (2 * p * 4 + 2 * sk * q * es + 10 * p * 4)
    return wz + cg


def traffic_from_profiles(kind):
    """HBM bytes per launch of `kind` from the committed rocprofv3 counter
    summary, or None if it is absent or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_2206_05047_amd", "csrc", "lfsr_kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kind)
    if not k or rec.get("kernel_source_sha256") != sha:
        return None
    return k.get("hbm_bytes_per_launch")


def counter_bytes_per_solve(n_iter):
    """HBM bytes of one solve from the committed FETCH_SIZE / WRITE_SIZE
    record (copy-calibrated, per kernel): the per-iteration kernels times
    their launches per iteration, times N, plus the once-per-solve set-up;
    None if the record is absent or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_2206_05047_amd", "csrc", "lfsr_kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    per = rec.get("per_solve")
    if not per or rec.get("kernel_source_sha256") != sha:
        return None
    return per["bytes_per_iteration"] * n_iter + per["bytes_setup"]


def oracle_one_thread(name, iters):
    """CPU-only child: the oracle's ADMM iterations on one thread (OMP_NUM_THREADS=1),
    inputs from the oracle's own forward model; prints seconds per iteration."""
    import oracle
    from paper_2206_05047_amd import synth

    cfg = synth.config(name)
    o = oracle.Oracle(cfg)
    sc = synth.make_scene(cfg)
    y = synth.degrade(o.forward(sc["x_gt"], sc["disp"]), synth.make_noise(cfg))
    st = o.init_state(y)
    t0 = time.perf_counter()
    o.iterate(st, y, sc["disp"], count=iters)
    dt = time.perf_counter() - t0
    print(json.dumps({"threads": oracle.Oracle.num_threads(), "s_per_iter": dt / iters, "iters": iters}), flush=True)


def convergence(name, budget):
    """Loss against computation units (CU) for the four solvers the paper
    compares (sec 7.1) on one workload with the weights fixed at x0: gd (fixed
    step, the best of a small sweep at 80 CU), gd-ls (backtracking), admm-5
    and admm-10 (K = 5 / 10 CG steps, early stop at |r|^2 <= tau).  A CU is A
    with S (a cost) or A^T with S^T (a gradient); an ADMM iteration costs
    2 + 2 K_n (K_n CG steps taken).  Prints one JSON line."""
    import numpy as np
    import torch

    from paper_2206_05047_amd import lfsr, synth

    torch.cuda.set_device(0)
    cfg = synth.config(name, reweight=0)
    sc = synth.make_scene(cfg)
    bound = max(float(np.abs(sc["disp"]).max()), 1e-3)
    disp = torch.from_numpy(sc["disp"]).cuda()
    base = lfsr.Solver(lfsr.make_params(cfg, disp_bound=bound))
    clean = base.lfsr_forward(torch.from_numpy(sc["x_gt"].astype(np.float32)).cuda(), disp)
    y = torch.from_numpy(synth.degrade(clean.cpu().numpy(), synth.make_noise(cfg))).cuda()
    curves, info = {}, {}

    def run_gd(step, ls, iters):
        base.lfsr_init(y, disp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = base.lfsr_gd(iters, step, line_search=ls)
        dt = time.perf_counter() - t0
        return h, dt

    sweep = {}
    for step in (5e-4, 1e-3, 2e-3, 4e-3, 8e-3):
        h, _ = run_gd(step, False, 39)
        sweep[step] = float(h[-1, 0])
    best = min(sweep, key=sweep.get)
    h, dt = run_gd(best, False, budget // 2 - 1)
    curves["gd"] = [(float(c), float(j)) for j, c, _ in h]
    info["gd"] = {"step": best, "sweep_J_at_80cu": sweep, "ms_per_cu": dt * 1e3 / h[-1, 1]}
    h, dt = run_gd(10 * best, True, budget)
    keep = h[:, 1] <= budget
    curves["gd-ls"] = [(float(c), float(j)) for j, c, _ in h[keep]]
    info["gd-ls"] = {"first_step": 10 * best, "ms_per_cu": dt * 1e3 / h[-1, 1]}
    for K in (5, 10):
        tau = 1.0
        s = lfsr.Solver(lfsr.make_params(dict(cfg, cg_iter=K, cg_tol=tau, n_iter=budget // 4), disp_bound=bound))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = s.lfsr_solve(y, disp)
        dt = time.perf_counter() - t0
        hist = st["hist"]
        cu_before = np.concatenate([[0.0], np.cumsum(2 + 2 * hist[:, 3])])
        # J_n is the cost at x^(n-1), evaluated by the first CU of iteration n
        pts = [(float(cu_before[n] + 1), float(hist[n, 0])) for n in range(len(hist)) if cu_before[n] + 1 <= budget]
        curves[f"admm-{K}"] = pts
        info[f"admm-{K}"] = {"cg_tol": tau, "cg_steps": [int(k) for k in hist[:, 3]],
                             "ms_per_cu": dt * 1e3 / cu_before[-1]}
        s.close()
    marks = [20, 40, 80, 160, 320, budget]
    table = {k: {m: min([j for c, j in v if c <= m], default=None) for m in marks} for k, v in curves.items()}
    print(json.dumps({"experiment": "loss vs computation units", "workload": synth.WORKLOAD_TEXT.get(name, name),
                      "weights": "fixed at x0 (reweight = 0)", "budget_cu": budget, "best_J_within_cu": table,
                      "info": info, "curves": curves}), flush=True)


def probe_ops(name, reps, which):
    """Counter-run driver: the forward, adjoint and normal operators of a
    workload on seeded random inputs, `reps` launches of each selected kind."""
    import numpy as np
    import torch

    from paper_2206_05047_amd import lfsr, synth

    cfg = synth.config(name)
    sc = synth.make_scene(cfg)
    s = lfsr.Solver(lfsr.make_params(cfg, disp_bound=float(np.abs(sc["disp"]).max())))
    g = torch.Generator(device="cuda").manual_seed(7)
    d = torch.from_numpy(sc["disp"]).cuda()
    x = torch.rand(s.H, s.W, device="cuda", generator=g)
    m = torch.rand(s.H, s.W, device="cuda", generator=g)
    e = torch.randn(s.sk, cfg["sy"], cfg["sx"], device="cuda", generator=g)
    out = torch.empty(s.H, s.W, device="cuda")
    lr = torch.empty_like(e)
    for _ in range(reps):
        if which in ("all", "adj"):
            s.lfsr_adjoint(e, d, out=out)
        if which in ("all", "fwd"):
            s.lfsr_forward(x, d, out=lr)
        if which in ("all", "hp"):
            s.lfsr_normal(x, d, m, out=out)
    torch.cuda.synchronize()
    log(f"[probe] ops {name} x{reps} {which} done")


def probe_copy(nbytes, reps):
    """Counter calibration: `reps` plain device copies of `nbytes` bytes.  The
    FETCH_SIZE / WRITE_SIZE readings of one copy, against its known 2 x nbytes
    of traffic, turn the counters of any other kernel into HBM bytes."""
    import torch

    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[probe] copy {n * 4} bytes x{reps} done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--probe", choices=["ops", "copy"], default=None,
                    help="counter-run drivers instead of the benchmark: 'ops' launches operators of --config "
                         "(--probe-which fwd|adj|hp|all), 'copy' the plain-copy calibration (--probe-bytes)")
    ap.add_argument("--probe-which", default="all")
    ap.add_argument("--probe-reps", type=int, default=3)
    ap.add_argument("--probe-bytes", type=int, default=1 << 30)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--cpu-iters", type=int, default=8, help="ADMM iterations of the oracle CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iters", type=int, default=0, help="override the ADMM iteration count (profiling only)")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP16/BF16 storage runs")
    ap.add_argument("--serve-jobs", type=int, default=0,
                    help="jobs in a serving stream run in a child process (0: skip; the serving run is "
                         "currently disabled and reports an error)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="serving arrival rate, jobs/s")
    ap.add_argument("--oracle-1thread", type=int, default=1,
                    help="ADMM iterations of the one-thread oracle sample (0: skip)")
    ap.add_argument("--no-other-workloads", action="store_true", help="skip the c1 / c2 throughput lines")
    ap.add_argument("--oracle-1thread-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--convergence", default=None, metavar="WORKLOAD",
                    help="instead of the benchmark: loss vs computation units of gd, gd-ls, admm-5, admm-10")
    ap.add_argument("--budget", type=int, default=400, help="computation units of the convergence experiment")
    args = ap.parse_args()
    if args.convergence:
        return convergence(args.convergence, args.budget)
    if args.oracle_1thread_child:
        return oracle_one_thread(args.oracle_1thread_child, args.oracle_1thread)
    if args.probe == "ops":
        return probe_ops(args.config, args.probe_reps, args.probe_which)
    if args.probe == "copy":
        return probe_copy(args.probe_bytes, args.probe_reps)
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU split into HR row bands is not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2206_05047_amd import lfsr, synth

    torch.cuda.set_device(0)
    cfg = synth.config(args.config)
    if args.iters > 0:
        cfg["n_iter"] = args.iters
    sc = synth.make_scene(cfg)
    noise = synth.make_noise(cfg)
    bound = float(np.abs(sc["disp"]).max())
    params = lfsr.make_params(cfg, disp_bound=max(bound, 1e-3))
    solver = lfsr.Solver(params)
    disp = torch.from_numpy(sc["disp"]).cuda()
    # LR views from the library's own forward model (inputs only; not timed)
    clean = solver.lfsr_forward(torch.from_numpy(sc["x_gt"].astype(np.float32)).cuda(), disp)
    y = torch.from_numpy(synth.degrade(clean.cpu().numpy(), noise)).cuda()
    out = torch.empty((solver.H, solver.W), dtype=torch.float32, device="cuda")
    N, K = cfg["n_iter"], cfg["cg_iter"]
    launches_per_solve = N * (K + 1)

    # warm-up; the first warm-up solve is timed per kernel kind to find the dominant kernel
    breakdown = None
    for i in range(max(args.warmup, 1)):
        if i == 0:
            # every launch of a solve: per iteration 8 + 7 K kernels at most
            solver.lfsr_profile_begin(capacity=N * (8 + 7 * K) + 64)
        solver.lfsr_solve(y, disp, out=out, stats=False)
        if i == 0:
            breakdown = solver.lfsr_profile_end()
    torch.cuda.synchronize()
    dom = max((k for k in breakdown if k in ("forward", "adjoint", "normal", "nltv")),
              key=lambda k: breakdown[k][0])
    dom_kind = lfsr.KERNEL_KINDS.index(dom)

    # timed region: K solves; the dominant kernel kind is bracketed by events
    solver.lfsr_profile_begin(kinds=[dom_kind], capacity=launches_per_solve * 2 * args.steps + 64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.lfsr_solve(y, disp, out=out, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = solver.lfsr_profile_end()
    stats = solver.lfsr_get_stats()
    ms = (t1 - t0) * 1e3 / max(args.steps, 1)
    H, W, sk = solver.H, solver.W, solver.sk
    value = H * W * sk * N * args.steps / (t1 - t0) / 1e6
    x = out.cpu().numpy()
    log(f"[bench] {args.config}: {ms:.2f} ms/solve, PSNR {synth.psnr(x, sc['x_gt']):.2f} dB, "
        f"J_N={stats['objective']:.6g}, iters={stats['iters_run']}")
    log("[bench] warm-up kernel time per solve (ms): " +
        ", ".join(f"{k}={v[0]:.1f} ({v[1]})" for k, v in breakdown.items()))

    tot_ms, n_launch = prof[dom]
    avg_s = tot_ms / max(n_launch, 1) / 1e3
    flops = kernel_flops_per_launch(dom, cfg)
    traffic = traffic_from_profiles(dom)
    if dom == "nltv":
        bpl = 2 * (cfg["win"] ** 2 - 1) * H * W * 4 + 3 * H * W * 4
        roof = {"bound": "hbm", "achieved": bpl / avg_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic
    roof["kernel"] = dom
    roof["avg_launch_us"] = avg_s * 1e6
    roof["launches_timed"] = n_launch

    hbm_gbs = bytes_per_iteration(cfg) * N * args.steps / (t1 - t0) / 1e9
    cb = counter_bytes_per_solve(N)
    hbm_gbs_counters = cb * args.steps / (t1 - t0) / 1e9 if cb else None
    line = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": synth.WORKLOAD_TEXT[args.config], "name": args.config, "views": sk,
                   "hr": [H, W], "scale": cfg["zeta"], "admm_iters": N, "cg_iters": K},
        "hbm_gbs_algorithmic": hbm_gbs,
        "hbm_frac_algorithmic": hbm_gbs / PEAK_HBM_GBS,
        "hbm_gbs_counters": hbm_gbs_counters,
        "hbm_frac_counters": hbm_gbs_counters / PEAK_HBM_GBS if hbm_gbs_counters else None,
        "roofline": roof,
        "kernel_ms_per_solve": {k: v[0] for k, v in breakdown.items()},
    }

    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", f"solve_{args.config}.npz")
    if os.path.exists(gpath) and args.iters == 0:
        g = np.load(gpath, allow_pickle=False)
        if "x" in g:
            golden = (g["x"].astype(np.float64), float(g["psnr_gt"]))

    def vs_oracle(xr):
        """rel-L2 and PSNR difference against the stored FP64 oracle solve of
        this workload (its LR views come from the oracle's forward model,
        which the library's matches to FP32 rounding)."""
        if golden is None:
            return {}
        return {"rel_l2_vs_oracle": synth.rel_l2(xr, golden[0]),
                "psnr_delta_vs_oracle": synth.psnr(xr, sc["x_gt"]) - golden[1]}

    line["accuracy"] = dict(vs_oracle(x.astype(np.float64)), psnr_gt=synth.psnr(x, sc["x_gt"]))

    if not args.no_precision:
        # the same workload with the state stored in 16 bits (FP32 stencil arithmetic)
        ref = out.cpu().numpy().astype(np.float64)
        prec = {}
        for st in ("f16", "bf16"):
            s16 = lfsr.Solver(lfsr.make_params(cfg, disp_bound=max(bound, 1e-3), storage=st))
            o16 = torch.empty_like(out)
            s16.lfsr_profile_begin(capacity=N * (8 + 7 * K) + 64)  # the warm-up solve, timed per kernel kind
            s16.lfsr_solve(y, disp, out=o16, stats=False)
            bd16 = s16.lfsr_profile_end()
            torch.cuda.synchronize()
            n16 = max(1, min(args.steps, 3))
            ta = time.perf_counter()
            for _ in range(n16):
                s16.lfsr_solve(y, disp, out=o16, stats=False)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            x16 = o16.cpu().numpy().astype(np.float64)
            prec[st] = {
                "value": H * W * sk * N * n16 / (tb - ta) / 1e6,
                "ms_per_step": (tb - ta) * 1e3 / n16,
                "speedup_vs_f32": ms / ((tb - ta) * 1e3 / n16),
                "rel_l2_vs_f32": synth.rel_l2(x16, ref),
                "psnr_gt": synth.psnr(x16, sc["x_gt"]),
                "psnr_f32": synth.psnr(ref, sc["x_gt"]),
                "workspace_bytes": s16.bytes,
                "steps": n16,
                "kernel_ms_per_solve": {k: v[0] for k, v in bd16.items()},
                "kernel_time_ratio_vs_f32": {k: bd16[k][0] / breakdown[k][0] for k in bd16 if breakdown[k][0] > 0},
                **vs_oracle(x16),
            }
            s16.close()
            log(f"[bench] {st}: {prec[st]['ms_per_step']:.2f} ms/solve, rel_l2 vs f32 {prec[st]['rel_l2_vs_f32']:.2e}")
        prec["target_speedup"] = 1.6
        prec["target_met"] = all(prec[k]["speedup_vs_f32"] >= 1.6 for k in ("f16", "bf16"))
        line["precision"] = prec

    if args.serve_jobs > 0:
        # in a child process: a failure there must not lose the line above
        import subprocess

        res = subprocess.run([sys.executable, "-m", "paper_2206_05047_amd.serve", str(args.serve_jobs),
                              str(args.serve_rate)], cwd=ROOT, capture_output=True, text=True, timeout=600)
        serving = None
        for ln in res.stdout.splitlines():
            if ln.startswith("{"):
                serving = json.loads(ln)
        if res.returncode != 0 or serving is None:
            serving = {"error": f"serving run exited with status {res.returncode}"}
        log(f"[bench] serving: {serving}")
        line["serving"] = serving

    if not args.no_other_workloads and args.config == "c3" and args.iters == 0:
        # the other two plain-method workloads and the multi-image workload at 5760^2
        # (throughput only; parity is in the tests)
        others = {}
        for name in ("c1", "c2", "misr2", "misr3"):
            c2 = synth.config(name)
            sc2 = synth.make_scene(c2)
            sv = lfsr.Solver(lfsr.make_params(c2, disp_bound=max(float(np.abs(sc2["disp"]).max()), 1e-3)))
            d2 = torch.from_numpy(sc2["disp"]).cuda()
            cl = sv.lfsr_forward(torch.from_numpy(sc2["x_gt"].astype(np.float32)).cuda(), d2)
            y2 = torch.from_numpy(synth.degrade(cl.cpu().numpy(), synth.make_noise(c2))).cuda()
            o2 = torch.empty((sv.H, sv.W), dtype=torch.float32, device="cuda")
            sv.lfsr_solve(y2, d2, out=o2, stats=False)
            torch.cuda.synchronize()
            reps = {"c1": 20, "c2": 5}.get(name, 2)
            ta = time.perf_counter()
            for _ in range(reps):
                sv.lfsr_solve(y2, d2, out=o2, stats=False)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            others[name] = {"workload": synth.WORKLOAD_TEXT[name], "ms_per_step": (tb - ta) * 1e3 / reps,
                            "value": sv.H * sv.W * sv.sk * c2["n_iter"] * reps / (tb - ta) / 1e6, "unit": UNIT,
                            "steps": reps}
            sv.close()
            log(f"[bench] {name}: {others[name]['ms_per_step']:.2f} ms/solve")
        # the c3 workload with one disparity map per view (sec 4.1): the scene's
        # map plus a smooth per-view perturbation of amplitude 0.4, clipped to [-2, 2]
        c2 = dict(synth.config("c3"), n_disp=81)
        sc2 = synth.make_scene(c2)
        H2, W2 = sc2["disp"].shape
        yy, xx = np.mgrid[0:H2, 0:W2]
        ph = np.random.default_rng(33).uniform(0, 6, 81)
        maps = np.stack([np.clip(sc2["disp"] + 0.4 * np.sin(0.21 * yy + 0.13 * xx + ph[k]), -2.0, 2.0)
                         for k in range(81)]).astype(np.float32)
        sv = lfsr.Solver(lfsr.make_params(c2, disp_bound=2.0))
        d2 = torch.from_numpy(maps).cuda()
        cl = sv.lfsr_forward(torch.from_numpy(sc2["x_gt"].astype(np.float32)).cuda(), d2)
        y2 = torch.from_numpy(synth.degrade(cl.cpu().numpy(), synth.make_noise(c2))).cuda()
        o2 = torch.empty((sv.H, sv.W), dtype=torch.float32, device="cuda")
        sv.lfsr_solve(y2, d2, out=o2, stats=False)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(2):
            sv.lfsr_solve(y2, d2, out=o2, stats=False)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        others["c3_per_view_maps"] = {
            "workload": synth.WORKLOAD_TEXT["c3"] + "; one disparity map per view (81 maps)",
            "ms_per_step": (tb - ta) * 1e3 / 2, "value": sv.H * sv.W * sv.sk * c2["n_iter"] * 2 / (tb - ta) / 1e6,
            "unit": UNIT, "steps": 2}
        sv.close()
        log(f"[bench] c3 per-view maps: {others['c3_per_view_maps']['ms_per_step']:.2f} ms/solve")
        line["other_workloads"] = others

    if not args.no_cpu_baseline:
        import oracle

        o = oracle.Oracle(cfg)
        yy = y.cpu().numpy()
        st = o.init_state(yy)
        tc0 = time.perf_counter()
        o.iterate(st, yy, sc["disp"], count=args.cpu_iters)
        tc1 = time.perf_counter()
        line["cpu_baseline"] = {
            "value": H * W * sk * args.cpu_iters / (tc1 - tc0) / 1e6,
            "unit": UNIT,
            "cores": oracle.Oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{args.cpu_iters} ADMM iterations (K={K}) of the same workload from x0, FP64, "
                      f"{tc1 - tc0:.1f} s",
        }
        if args.oracle_1thread > 0:
            # one thread, in a CPU-only child process (OpenMP's thread count is fixed per process)
            import subprocess

            env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
            res = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-1thread-child", args.config,
                                  "--oracle-1thread", str(args.oracle_1thread)], cwd=ROOT, env=env,
                                 capture_output=True, text=True, timeout=600)
            one = None
            for ln in res.stdout.splitlines():
                if ln.startswith("{"):
                    one = json.loads(ln)
            if one:
                line["cpu_baseline"]["one_thread"] = {
                    "value": H * W * sk / one["s_per_iter"] / 1e6, "unit": UNIT, "cores": one["threads"],
                    "s_per_admm_iteration": one["s_per_iter"],
                    "sample": f"{one['iters']} ADMM iteration(s) of the same workload (oracle's own LR views)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
