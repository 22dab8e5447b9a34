"""Learning-rate selection for the two minibatch configurations, the paper's
way (Sec. 5, hyper-parameters: the rate with the smallest angular error summed
over the run), with the float64 oracle only.

For each configuration and each eta0 of the grid {1, 1e-1, 1e-2, 1e-3}, the
oracle's priming runs the configuration's own number of minibatch steps, with
its batch and schedule, over a 50,000-row sample of the same generator (rows
cycled); after every tenth of the run the angles between the top-k columns and
the true eigenvectors are summed.  Writes eta_selection.json beside this file.

    python tests/golden/select_eta.py
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ppca_oracle as O            # noqa: E402
from synthdata import gaussian_block, make_problem   # noqa: E402

SAMPLE_ROWS = 50_000
GRID = (1.0, 1e-1, 1e-2, 1e-3)
SNAPSHOTS = 10
# Oja on 1M x 1024 float32 data and EigenGame on 8M x 2048 fp8 data (its
# fp8 storage is not emulated: the sample is used in float64)
CONFIGS = {
    "oja-f32": dict(n=1_000_000, d=1024, spectrum="pow1.2+1e-4", k=32, l=32, batch=1024,
                    epochs=1.0, t0=1000.0, seed=1002, rule="oja"),
    "eigengame-fp8": dict(n=8_000_000, d=2048, spectrum="exp0.97+1e-5", k=32, l=32,
                          batch=4096, epochs=3.0, t0=0.0, seed=1004, rule="eigengame"),
}


def top_k_angles(v, q, k):
    vk = v[:, :k] / np.linalg.norm(v[:, :k], axis=0)
    return np.arccos(np.clip(np.abs(np.sum(vk * q[:, :k], axis=0)), 0.0, 1.0))


def summed_angle(x, q, c, eta0):
    fn = O.prime_oja if c["rule"] == "oja" else O.prime_eigengame
    steps = int(math.ceil(c["epochs"] * c["n"] / c["batch"]))
    v = gaussian_block(c["d"], c["k"] + c["l"], c["seed"] + 1000, np.float64)
    buf, done, tot = None, 0, 0.0
    for i in range(SNAPSHOTS):
        ns = steps * (i + 1) // SNAPSHOTS - done
        v, buf = fn(x, v, batch=c["batch"], steps=ns, eta0=eta0, t0=c["t0"], start_step=done,
                    mom_buf=buf, orthonormalise_start=(i == 0))
        done += ns
        a = top_k_angles(v, q, c["k"])
        if not np.all(np.isfinite(a)):
            return float("inf"), steps
        tot += float(a.sum())
    return tot, steps


def main():
    out = {"sample_rows": SAMPLE_ROWS, "grid": list(GRID), "snapshots": SNAPSHOTS, "configs": {}}
    for name, c in CONFIGS.items():
        p = make_problem(SAMPLE_ROWS, c["d"], c["spectrum"], seed=c["seed"], mode="gaussian",
                         dtype=np.float64)
        x = p.x - p.x.mean(axis=0, keepdims=True)
        scores = {}
        for eta in GRID:
            s, steps = summed_angle(x, p.q, c, eta)
            scores[str(eta)] = s
            print(f"{name} eta0 {eta}: summed angle {s:.4f} over {steps} steps", flush=True)
        best = min(GRID, key=lambda e: scores[str(e)])
        out["configs"][name] = {"steps": steps, "batch": c["batch"], "t0": c["t0"],
                                "summed_angle": scores, "eta0": best}
    with open(os.path.join(HERE, "eta_selection.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
