"""Benchmark of the ADMM light-field super-resolution solve on one MI355X.

One step = one complete solve (lfsr_solve: x0, w = 0, N ADMM iterations of
K CG steps each, output copy) of the 9x9-view, 1152x1152, x3 workload, with
the inputs resident in HBM.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--cpu-iters", type=int, default=2, help="ADMM iterations of the oracle CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iters", type=int, default=0, help="override the ADMM iteration count (profiling only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU row-band design is described in DESIGN.md, not built).", file=sys.stderr)
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
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        solver.lfsr_solve(y, disp, out=out, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.lfsr_solve(y, disp, out=out, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = solver.lfsr_get_stats()
    ms = (t1 - t0) * 1e3 / max(args.steps, 1)
    H, W, sk, N = solver.H, solver.W, solver.sk, cfg["n_iter"]
    pv_iters = H * W * sk * N
    value = pv_iters * args.steps / (t1 - t0) / 1e6
    x = out.cpu().numpy()
    log(f"[bench] {args.config}: {ms:.2f} ms/solve, PSNR {synth.psnr(x, sc['x_gt']):.2f} dB, "
        f"J_N={stats['objective']:.6g}, iters={stats['iters_run']}")

    line = {
        "metric": "HR Mpixel-views x ADMM iters/s",
        "value": value,
        "unit": "Mpixel-view-iter/s",
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
                   "hr": [H, W], "scale": cfg["zeta"], "admm_iters": N, "cg_iters": cfg["cg_iter"]},
    }

    if not args.no_cpu_baseline:
        import oracle

        o = oracle.Oracle(cfg)
        st = o.init_state(y.cpu().numpy())
        yy = y.cpu().numpy()
        dd = sc["disp"]
        tc0 = time.perf_counter()
        o.iterate(st, yy, dd, count=args.cpu_iters)
        tc1 = time.perf_counter()
        line["cpu_baseline"] = {
            "value": H * W * sk * args.cpu_iters / (tc1 - tc0) / 1e6,
            "unit": "Mpixel-view-iter/s",
            "cores": oracle.Oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{args.cpu_iters} ADMM iterations (K={cfg['cg_iter']}) of the same workload from x0, FP64",
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
