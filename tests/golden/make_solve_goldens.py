"""Write the stored expected values of the long solve parity tests.

Calls only the FP64 oracle (``oracle/``) on the seeded workloads; nothing here
comes from the GPU path.  Run from the repository root:
    python tests/golden/make_solve_goldens.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import torch  # noqa: E402

import workloads as W  # noqa: E402
from oracle import svgd  # noqa: E402

CASES = {
    # name: (cfg_id, iters, lr)
    "cfg2_solve_lr1e-3_it100": (2, 100, 1e-3),
    "cfg2_solve_lr1e-2_it10": (2, 10, 1e-2),
}


def main(names=None):
    torch.set_num_threads(os.cpu_count() or 1)
    for name, (cfg, iters, lr) in CASES.items():
        if names and name not in names:
            continue
        scene, w, th = W.config_problem(cfg)
        t = time.time()
        out = svgd.solve(scene, w, th, iters, lr=lr, history=True)
        np.savez_compressed(os.path.join(HERE, name + ".npz"), theta=out["theta"], cost=out["cost"],
                            modes=out["modes"], h=out["h"], iters=iters, lr=lr, cfg=cfg,
                            mean_cost=np.array([h["mean_cost"] for h in out["hist"]]))
        print(name, "done in %.0f s, final mean cost %.4f" % (time.time() - t, out["cost"].mean()), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
