"""Write the algorithmic work model of the benchmark workload.

Runs only oracle code (FP64, CPU) on a seeded receiver sample of the
64-segment scene (box + 64 segments, 256x256 receivers, order <= 2) and of
the 3D scene (room + 32 rectangles, 256x256 receivers, order <= 2) and writes
per-path-evaluation counts to bench_work_model.json at the repository root.
bench.py turns them into algorithmic FLOPs with the per-operation weights
stored alongside.

Usage: python -m oracle.count_work [--sample 256]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import tracer as T  # noqa: E402
from oracle import tracer3d as T3  # noqa: E402
from paper_2401_11882_amd import workloads as WL  # noqa: E402

# FLOPs per operation (FMA = 2, add/mul/compare = 1, exp2/rcp = 1), credited
# by one rule: only an active pair's work counts (oracle.tracer.work_counts:
# valid, interaction factor nonzero in FP32, bound F / max(d^2, d_min^2) of
# its contribution above 2^-24 P(r) / C, P the receiver's full power and C the
# scene's candidate count), and of its obstruction tests only the unsaturated
# ones (a saturated factor is 1.0f in FP32).  Work an implementation spends
# to prove a pair or a test away (screens, back-traces of pairs whose factor
# is 0, band checks) is not credited.  An active pair's tests are all
# credited, also those a kernel skips once the pair's running product has
# fallen below the cut, so this is the method's work on the pairs that can
# contribute, not a count of what a kernel executes: it is reported beside
# the executed-FLOP counters as context.
WEIGHTS = {
    "fwd_per_active_pair": 13,          # |r - I_k|^2, floor, divide, compensated sum
    "fwd_per_active_interaction": 40,   # back-trace step (20) + in(t) in(u): 4 exp, reciprocal, products (20)
    "fwd_per_unsaturated": 44,          # den, tau/ups (18) + reciprocal, 4 exp, stable 1 - in*in (26)
    "bwd_per_active_pair": 12,          # dL/dc, |r - I_k|^2 adjoint
    "bwd_per_active_interaction": 80,   # back-trace + mirror adjoint, in(t) in(u) and its derivative
    "bwd_per_unsaturated": 94,          # the test's values (44) + dlog q/d(tau, ups) and the chain (50)
}


# The same accounting for panels in 3D (dot products of three, one more
# panel coordinate and one more smoothed comparison per test).
WEIGHTS_3D = {
    "fwd_per_active_pair": 14,          # |r - I_k|^2, floor, divide, compensated sum
    "fwd_per_active_interaction": 64,   # back-trace to the plane, panel coordinates (36) + 3 factors (28)
    "fwd_per_unsaturated": 76,          # plane crossing and band tests (42), three n_x and the factor (34)
    "bwd_per_active_pair": 14,          # dL/dc, |r - I_k|^2 adjoint
    "bwd_per_active_interaction": 141,  # derivatives of the three factors, back-trace and mirror adjoint
    "bwd_per_unsaturated": 176,         # the test's values (72) + three log-derivatives and the chain (104)
}


def n_candidates(n: int, max_order: int) -> int:
    """Interaction sequences of length <= max_order over n surfaces, no surface twice in a row."""
    return 1 + sum(n * (n - 1) ** (k - 1) for k in range(1, max_order + 1))


def model(counts: dict, W: dict) -> dict:
    n = counts["path_evals"]
    per = {k: v / n for k, v in counts.items()}
    fwd = (W["fwd_per_active_pair"] * per["active"] + W["fwd_per_active_interaction"] * per["active_interactions"] +
           W["fwd_per_unsaturated"] * per["unsaturated"])
    bwd = (W["bwd_per_active_pair"] * per["active"] + W["bwd_per_active_interaction"] * per["active_interactions"] +
           W["bwd_per_unsaturated"] * per["unsaturated"])
    return {"counts": counts, "per_path_eval": per, "fwd_flops_per_path_eval": fwd, "bwd_flops_per_path_eval": bwd}


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--sample", type=int, default=256)
    ap.add_argument("--alphas", default="10,100,1000")
    ap.add_argument("--cut-total", type=float, default=2.0 ** -24,
                    help="contribution cut: pairs that can change P(r) by at most cut_total P(r) / C count "
                         "nothing (the kernels drop only what lies below that times a lower bound of P)")
    args = ap.parse_args()
    out = {"workload": "box + 64 segments, 256x256 receivers, order <= 2 (4,625 candidates)",
           "sample_receivers": args.sample, "cut_total": args.cut_total, "weights": WEIGHTS, "per_alpha": {}}
    for a in [float(x) for x in args.alphas.split(",")]:
        s = WL.scene_64(alpha=a)
        idx = np.random.default_rng(11882).choice(s.n_rx, size=args.sample, replace=False)
        c = T.work_counts(s.walls, s.tx, s.rx[idx], s.max_order, a,
                          cut=args.cut_total / n_candidates(s.walls.shape[0], s.max_order))
        out["per_alpha"][str(int(a))] = model(c, WEIGHTS)
        print(a, json.dumps(out["per_alpha"][str(int(a))]), flush=True)
    s3 = WL.scene3d_32()
    idx = np.random.default_rng(11882).choice(s3.n_rx, size=args.sample, replace=False)
    c3 = T3.work_counts(s3.panels, s3.tx, s3.rx[idx], s3.max_order, s3.alpha,
                        cut=args.cut_total / n_candidates(s3.panels.shape[0], s3.max_order))
    out["scene3d"] = {"workload": "room + 32 rectangles (38 panels), 256x256 receivers, order <= 2 (1,445 candidates)",
                      "weights": WEIGHTS_3D, "per_alpha": {str(int(s3.alpha)): model(c3, WEIGHTS_3D)}}
    print("3d", json.dumps(out["scene3d"]["per_alpha"]), flush=True)
    with open(os.path.join(ROOT, "bench_work_model.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
