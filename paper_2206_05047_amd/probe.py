"""Launch drivers for hardware-counter runs.

  python paper_2206_05047_amd/probe.py ops c3 3 [fwd|adj|hp|all]
      launches the forward, adjoint and normal operators of a workload a few
      times on random inputs (one kernel of each kind per repetition);
  python paper_2206_05047_amd/probe.py copy 1073741824 4
      copies a buffer of that many bytes a few times (one plain copy kernel
      per repetition): the calibration that turns FETCH_SIZE / WRITE_SIZE
      counter readings into HBM bytes.

Run under `rocprofv3 --pmc ...` or `--kernel-trace --stats`, from any
working directory.
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def ops(name, reps, which):
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
    print(f"probe ops {name} x{reps} {which} done", flush=True)


def copy(nbytes, reps):
    import torch

    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"probe copy {n * 4} bytes x{reps} done", flush=True)


def main(argv):
    if not argv or argv[0] not in ("ops", "copy"):
        print(__doc__, file=sys.stderr)
        return 2
    if argv[0] == "ops":
        ops(argv[1] if len(argv) > 1 else "c3", int(argv[2]) if len(argv) > 2 else 3,
            argv[3] if len(argv) > 3 else "all")
    else:
        copy(int(argv[1]) if len(argv) > 1 else 1 << 30, int(argv[2]) if len(argv) > 2 else 4)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
