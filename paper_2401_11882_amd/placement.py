"""Transmitter placement with an annealed sharpness (Sec. VII).

The paper places one transmitter to serve several receivers by maximising
Eq. 8, F(tx) = min_i P_Rx_i(tx), by gradient steps, raising alpha after every
iteration along a geometric progression from 1 to 100 over the iterations;
started inside the zero-gradient region of the unsmoothed objective, plain
gradient steps do not move while the annealed ones do.  It then reports how
often repeated optimisations on random scenes reach the optimum, with and
without the approximation.

Here many independent problems (one transmitter, 1..64 receivers each) run
as the scenes of one batched launch per iteration: the schedule kernel writes
every problem's alpha from the device step counter, the batched tracer forms
L = -F and its gradient w.r.t. each transmitter, and one Adam launch moves all
transmitters.  The iteration is captured once in a HIP graph and replayed.

``study`` measures success rates on seeded random problems.  The unsmoothed
objective is the sigmoid at alpha = 1e6 (its transition is narrower than
1e-5 of a segment, so FP32 gives exact zeros in shadows, as the step does);
the reference optimum of a problem is the best value of that objective on a
grid of transmitter positions, evaluated from the receivers' side: with line
of sight only, P(a -> b) = P(b -> a).
"""
from __future__ import annotations

import numpy as np
import torch

from . import tracer as tr
from . import workloads as WL
from .batched import BatchPlan

HARD_ALPHA = 1e6


def optimize(problems, steps: int = 100, lr: float = 1e-2, a_first: float = 1.0, a_last: float = 100.0,
             fixed_alpha: float | None = None, max_order: int = 0, use_graph: bool = True, device="cuda"):
    """Annealed (or fixed-alpha) Adam on the transmitters of all problems at once.

    ``problems``: objects with ``walls`` [W,4], ``rx`` [1..64, 2] and the start
    ``tx`` [2] (numpy float32).  Returns dict with device tensors tx [S,2],
    tx_hist [steps+1, S, 2] and loss_hist [steps, S] (loss_hist[i] = -F at
    tx_hist[i], with alpha of iteration i).
    """
    S = len(problems)
    scenes = [WL.Scene(p.walls, p.tx, p.rx, 0, max_order, 1.0) for p in problems]
    plan = BatchPlan(scenes, max_order, device=device)
    dev = plan.device
    if fixed_alpha is not None:
        plan.alpha.fill_(float(fixed_alpha))
    m = torch.zeros(S, 2, device=dev)
    v = torch.zeros(S, 2, device=dev)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    tx_hist = torch.zeros(steps + 1, S, 2, device=dev)
    loss_hist = torch.zeros(steps, S, device=dev)
    tx_hist[0] = plan.tx

    def one_step():
        if fixed_alpha is None:
            tr.alpha_schedule(step, steps, a_first, a_last, plan.alpha)
        _, L, gtx, _ = plan.run(loss="neg_min")
        idx = step.long()
        loss_hist.index_copy_(0, idx, L.view(1, S))
        tr.adam_points(plan.tx, gtx, m, v, step, lr=lr)
        tx_hist.index_copy_(0, idx + 1, plan.tx.view(1, S, 2))

    if use_graph:
        # warm the launch outside the capture on a copy of the state
        saved = plan.tx.clone()
        plan.run(loss="neg_min")
        torch.cuda.synchronize()
        plan.tx.copy_(saved)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                one_step()
        torch.cuda.current_stream().wait_stream(side)
        for _ in range(steps):
            g.replay()
    else:
        for _ in range(steps):
            one_step()
    torch.cuda.synchronize()
    out = {"tx": plan.tx.clone(), "tx_hist": tx_hist, "loss_hist": loss_hist}
    plan.close()
    return out


def objective(problems, tx: torch.Tensor, alpha: float = HARD_ALPHA, max_order: int = 0) -> torch.Tensor:
    """F = min_i P_Rx_i at the given transmitters [S,2] (one batched forward)."""
    scenes = [WL.Scene(p.walls, tx[i].detach().cpu().numpy(), p.rx, 0, max_order, alpha)
              for i, p in enumerate(problems)]
    plan = BatchPlan(scenes, max_order, device=tx.device)
    _, L, _, _ = plan.run(loss="neg_min")
    F = -L.clone()
    plan.close()
    return F


def grid_optimum(problems, grid_n: int = 128, alpha: float = HARD_ALPHA) -> torch.Tensor:
    """Best F over the cell centres of a grid_n x grid_n grid of transmitter
    positions, per problem: every receiver is used as the source of a power
    map over the grid (line-of-sight reciprocity), then min over receivers,
    max over the grid."""
    grid = WL.rx_grid(grid_n)
    scenes, owner = [], []
    for k, p in enumerate(problems):
        for r in p.rx:
            scenes.append(WL.Scene(p.walls, np.asarray(r, np.float32), grid, grid_n, 0, alpha))
            owner.append(k)
    plan = BatchPlan(scenes, 0)
    P = plan.run(loss="none")[0].view(len(scenes), grid_n * grid_n)
    counts = [len(p.rx) for p in problems]
    if len(set(counts)) == 1:
        best = P.view(len(problems), counts[0], -1).min(1).values.max(1).values.clone()
    else:
        best = torch.empty(len(problems), device=P.device)
        owner = np.asarray(owner)
        for k in range(len(problems)):
            idx = np.nonzero(owner == k)[0]
            best[k] = P[int(idx[0]):int(idx[-1]) + 1].min(0).values.max()
    plan.close()
    return best


def study(n_per_count: int = 256, rx_counts=(2, 3, 4), steps: int = 100, lr: float = 1e-2,
          grid_n: int = 128, threshold: float = 0.9):
    """Success rate of annealed versus unsmoothed optimisation on seeded problems.

    A run succeeds when the unsmoothed objective at its final transmitter is at
    least ``threshold`` times the grid optimum.  Returns a dict per receiver
    count with both rates, their ratio and the share of the unsmoothed
    successes that the annealed run also reaches.
    """
    out = {}
    for n_rx in rx_counts:
        probs = [WL.placement_problem(k, n_rx) for k in range(n_per_count)]
        ref = grid_optimum(probs, grid_n)
        ann = optimize(probs, steps=steps, lr=lr)
        hard = optimize(probs, steps=steps, lr=lr, fixed_alpha=HARD_ALPHA)
        fa = objective(probs, ann["tx"]) / ref
        fh = objective(probs, hard["tx"]) / ref
        sa, sh = (fa >= threshold).cpu().numpy(), (fh >= threshold).cpu().numpy()
        out[n_rx] = {
            "problems": n_per_count,
            "annealed_success": float(sa.mean()),
            "unsmoothed_success": float(sh.mean()),
            "ratio": float(sa.mean() / sh.mean()) if sh.any() else None,
            "annealed_given_unsmoothed": float(sa[sh].mean()) if sh.any() else None,
        }
    return out
