"""Write the stored expected values of the full-size parity tests.

Calls only the FP64 oracle (and the seeded input generator): for each workload
the LR views are made with the oracle's forward model, the oracle runs the
full solve, and the result is stored with a hash of the inputs so that a test
can tell whether it regenerated the same inputs.

  python tests/golden/make_golden.py c2 c3

Each record keeps the whole HR result (rounded to float32, far below the
1e-4 relative-L2 bar), its L2 norm and the per-iteration statistics
(objective, primal residual, CG pi).
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2206_05047_amd import synth  # noqa: E402


def inputs(name):
    cfg = synth.config(name)
    o = oracle.Oracle(cfg)
    sc = synth.make_scene(cfg)
    y = synth.degrade(o.forward(sc["x_gt"], sc["disp"]), synth.make_noise(cfg))
    return cfg, o, sc, y


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(names):
    for name in names:
        t0 = time.time()
        cfg, o, sc, y = inputs(name)
        x, stats = o.solve(y, sc["disp"])
        rec = dict(y_sha256=sha(y), disp_sha256=sha(sc["disp"]), hist=stats, norm=np.linalg.norm(x),
                   psnr_gt=synth.psnr(x, sc["x_gt"]), threads=oracle.Oracle.num_threads())
        rec["x"] = x.astype(np.float32)
        np.savez_compressed(os.path.join(HERE, f"solve_{name}.npz"), **rec)
        print(f"{name}: {time.time() - t0:.0f} s, PSNR {rec['psnr_gt']:.3f} dB, J_N {stats[-1, 0]:.8g}",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c3"])
