"""Writes the FP64 oracle's reference values for the full-size image-stack workloads.

Calls only the seeded generator (synth/) and the oracle (oracle/): the stored values never come
from the GPU path.  Usage (from the repository root; minutes of CPU time):

    python tests/golden/make_stack_oracle.py stack1080
    python tests/golden/make_stack_oracle.py stack2160

Output: tests/golden/<name>_oracle.json with the fit after the T-HOSVD start and after every
sweep, the final core norm, ||X||^2, and per mode the Gram eigenvalues at the rank boundary
and the gap factor (the quantities the rotation-invariant comparisons need).
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import STACK_CONFIGS, make_stereo_stack  # noqa: E402


def main(name):
    c = STACK_CONFIGS[name]
    x = make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"]).astype(np.float64)
    t = time.time()
    r = oracle.hooi(x, c["ranks"], c["sweeps"])
    modes = []
    for n, rank in enumerate(c["ranks"]):
        lam = r.spectra[n]
        modes.append({"rank": rank, "lam_1": float(lam[0]),
                      "lam_R": float(lam[rank - 1]) if rank <= len(lam) else None,
                      "lam_R1": float(lam[rank]) if rank < len(lam) else None,
                      "lam_sum": float(np.sum(lam)), "gap_factor": float(r.gap_factor(n, rank))})
    out = {"workload": name, "dims": list(x.shape), "ranks": list(c["ranks"]), "sweeps": c["sweeps"],
           "seed": c["seed"], "fits": [float(f) for f in r.fits], "core_norm": float(np.linalg.norm(r.core)),
           "x_norm2": float(np.sum(x * x)), "modes": modes, "oracle_seconds": round(time.time() - t, 1)}
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("workload", "oracle_seconds", "core_norm")}))


if __name__ == "__main__":
    main(sys.argv[1])
