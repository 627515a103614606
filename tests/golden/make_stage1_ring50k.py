"""Writes stage1_ring-50k-256px.json: the oracle's Stage-1 trajectory on the
50K-Gaussian ring workload (SH degree 1, four 256 x 256 views on a ring,
held-out view at 45 degrees), float32 NTC parameters from seed 0, 150
iterations of Sec. 4.1 (Eq. 5-6, Adam lr 0.002), views from the seeded
schedule of reading C10 (seed 0); then the same loop MEMBERS more times with
the image and gradients of every iteration perturbed by float32-sized
relative noise (1e-6; oracle/stage1.py), whose held-out PSNR curves show how
far rounding alone moves the trajectory.  Calls only the oracle and the
seeded input generator.  Run from the repository root (about 40 minutes):

    python tests/golden/make_stage1_ring50k.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ntc as ontc  # noqa: E402
from oracle import raster as orc  # noqa: E402
from oracle import stage1  # noqa: E402
from paper_2403_01444_amd import synth  # noqa: E402

ITERS, SEED, PARAM_SEED, VIEW_SEED = 150, 0, 0, 0
MEMBERS, REL = 8, 1e-6


def inputs():
    g, cams, held, nxt = synth.workload("ring-50k-256px", seed=SEED)
    targets = [orc.render(nxt, c)["image"].astype(np.float32) for c in cams]
    held_t = orc.render(nxt, held[0])["image"].astype(np.float32)
    cfg = synth.NTCConfig()
    return g, cams, held[0], targets, held_t, cfg, synth.ntc_init_params(cfg, PARAM_SEED)


def main():
    g, cams, held, targets, held_t, cfg, p0 = inputs()
    views = synth.view_schedule(len(cams), ITERS, VIEW_SEED)
    t0 = time.time()
    r = stage1.ntc_stage1(ontc.NTCSpec(cfg), p0, g, cams, targets, views, held_cam=held, held_target=held_t,
                          log_every=10)
    secs = round(time.time() - t0, 1)
    members = []
    for k in range(1, MEMBERS + 1):
        rk = stage1.ntc_stage1(ontc.NTCSpec(cfg), p0, g, cams, targets, views, held_cam=held, held_target=held_t,
                               log_every=10, perturb=(k, REL))
        members.append([float(p) for _, p in rk["psnr"]])
        print(f"member {k}: {members[-1]}", flush=True)
    out = {"workload": "ring-50k-256px", "seed": SEED, "param_seed": PARAM_SEED, "view_seed": VIEW_SEED,
           "iters": ITERS, "lambda": 0.2, "lr": 0.002, "betas": [0.9, 0.99], "eps": 1e-15, "views": views,
           "loss": [float(x) for x in r["loss"]], "psnr": [[int(i), float(p)] for i, p in r["psnr"]],
           "oracle_seconds": secs, "perturbation": {"rel": REL, "seeds": list(range(1, MEMBERS + 1))},
           "member_psnr": members}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stage1_ring-50k-256px.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["psnr"])


if __name__ == "__main__":
    main()
