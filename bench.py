"""Benchmark: smoothed path-evaluations per second, forward + adjoint, one GPU.

Workload: box + 64 seeded segments (68 walls), 256 x 256 receiver grid,
order <= 2 (4,625 wall sequences), alpha = 100, loss = -mean log(P + 1e-6).
One step = the forward pass (power map, loss, seed dL/dP) followed by the
adjoint pass (gradients w.r.t. the transmitter and all 272 wall coordinates)
starting from the contributions the forward recorded -- the same kernels
drt_forward_backward enqueues, issued as two calls so that HIP events can
bracket each kernel.  path-evals per step =
receivers x candidates = 65,536 x 4,625.

Prints one JSON line (see the fields below).  Inputs are resident in device
memory before timing starts.  --gpus N > 1 is refused: the benchmark runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3        # MI355X vector FP32 (datasheet, counts packed issue)
UNPACKED_FP32_TFLOPS = 78.6     # the same without packed FP32: 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz


# The sources the single-scene 2D tracer kernels (k_forward, k_backward) are
# built from: counter figures are valid only while these are unchanged.
TRACER_SOURCES = ("dev.h", "path.h", "screen.h", "trace.h", "trace.hip", "view.h")
TRACER3D_SOURCES = ("dev.h", "path3d.h", "screen3.h", "trace3d.h", "trace3d.hip")
BATCHED_SOURCES = ("dev.h", "path.h", "screen.h", "batched.h", "batched.hip")
FERMAT_SOURCES = ("dev.h", "path.h", "trace.h", "view.h", "fermat.h", "fermat.hip")


def source_hash(names=TRACER_SOURCES) -> str:
    """sha256 over the tracer kernels' HIP sources; counter figures are valid for this hash only."""
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2401_11882_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_counters(tag: str, kernel: str, sources=TRACER_SOURCES):
    """The committed rocprofv3 PMC summary of one kernel (HBM bytes per launch,
    executed FP32 FLOPs per launch, ...), or None when the kernels changed
    since those counters were taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{tag}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_sha256") != source_hash(sources):
        return None
    return t["kernels"].get(kernel)


def measured_traffic(tag: str, kernel: str, sources=TRACER_SOURCES):
    """HBM bytes per launch, or None (see measured_counters)."""
    k = measured_counters(tag, kernel, sources)
    return None if k is None else int(k["hbm_bytes"])


def work_model(section: str = "2d", alpha: float = 100.0):
    """Per-path-evaluation figures of the oracle's work model (bench_work_model.json), or None."""
    p = os.path.join(ROOT, "bench_work_model.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        wm = json.load(f)
    sec = wm["per_alpha"] if section == "2d" else wm.get(section, {}).get("per_alpha", {})
    return sec.get(str(int(alpha)))


def alu_roofline(tag: str, kernel: str, kernel_ms: float, sources=TRACER_SOURCES, model_flops=None,
                 time_basis: str = "HIP events around the launch, averaged over the timed steps"):
    """Roofline of an FP32-VALU-bound kernel: the FP32 FLOPs it executes per
    launch (64 lanes x (ADD + MUL + TRANS + 2 FMA) from the committed
    rocprofv3 counters profiles/traffic_<tag>.json, valid while the kernel
    sources are unchanged) over its average launch time.  The oracle's work
    model (algorithmic FLOPs of the pairs that can contribute) rides along as
    context."""
    r = {"bound": "alu", "achieved": None, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": None,
         "traffic": None, "kernel": kernel, "kernel_ms": round(kernel_ms, 4), "time_basis": time_basis}
    ctr = measured_counters(tag, kernel, sources)
    if ctr is None or not ctr.get("executed_fp32_flops"):
        r["basis"] = f"no counters for these kernel sources in profiles/traffic_{tag}.json"
    else:
        ex = float(ctr["executed_fp32_flops"])
        ach = ex / (kernel_ms * 1e-3) / 1e12
        r.update(achieved=round(ach, 3), frac=round(ach / PEAK_FP32_TFLOPS, 4),
                 traffic=int(ctr["hbm_bytes"]) if ctr.get("hbm_bytes") is not None else None,
                 basis=f"executed FP32 FLOPs per launch from profiles/traffic_{tag}.json",
                 executed_flops_per_launch=ex, frac_of_unpacked_peak=round(ach / UNPACKED_FP32_TFLOPS, 4))
        if ctr.get("avg_us"):
            r["profiled_kernel_ms"] = round(ctr["avg_us"] / 1e3, 4)
            r["frac_at_profiled_time"] = round(ex / (ctr["avg_us"] * 1e-6) / 1e12 / PEAK_FP32_TFLOPS, 4)
        if ctr.get("sq_insts_valu"):
            r["valu_wave_instructions_per_launch"] = ctr["sq_insts_valu"]
    if model_flops is not None:
        r["model_flops_per_launch"] = model_flops
        r["model_tflops"] = round(model_flops / (kernel_ms * 1e-3) / 1e12, 3)
    return r


def copy_calibration(dev, mib: int) -> None:
    """One plain device copy of mib MiB, the reference the HBM counters are scaled by."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(alpha: float, n_rx: int, n_rx_single: int, repeats: int = 3):
    """The FP64 oracle (as it stands) on bounded receiver samples, fwd + VJP:
    the median of `repeats` runs with all host threads, and the median of
    `repeats` single-thread runs on a smaller sample."""
    import numpy as np
    import torch

    from oracle import tracer as T
    from paper_2401_11882_amd import workloads as WL

    s = WL.scene_64(alpha=alpha)
    n_cand = WL.n_candidates(s.n_walls, s.max_order)

    def rate(n, seed):
        idx = np.random.default_rng(seed).choice(s.n_rx, size=n, replace=False)
        rx = s.rx[idx]
        t0 = time.perf_counter()
        P = T.power(s.walls, s.tx, rx, s.max_order, alpha)
        g = T.loss_seed(P, "neg_mean_log") * (n / s.n_rx)
        T.vjp(s.walls, s.tx, rx, s.max_order, alpha, g)
        dt = time.perf_counter() - t0
        return n * n_cand / dt, dt

    threads = torch.get_num_threads()
    multi = [rate(n_rx, 7 + i) for i in range(repeats)]
    torch.set_num_threads(1)
    try:
        single = [rate(n_rx_single, 17 + i) for i in range(repeats)]
    finally:
        torch.set_num_threads(threads)
    med = float(np.median([r for r, _ in multi]))
    med1 = float(np.median([r for r, _ in single]))
    total = sum(dt for _, dt in multi + single)
    return {"value": med, "unit": "path-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"median of {repeats} runs of {n_rx} random receivers of the 256x256 grid x {n_cand} candidates "
                      f"(fwd + VJP, FP64, torch CPU, {threads} threads); {total:.1f} s of CPU work in all",
            "runs": [round(r, 1) for r, _ in multi],
            "single_thread": {"value": med1, "unit": "path-evals/s", "cores": 1,
                              "sample": f"median of {repeats} runs of {n_rx_single} random receivers",
                              "runs": [round(r, 1) for r, _ in single]},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def extra_batched(dev):
    """512 scenes (8..128 interior segments, 64^2..256^2 receivers, order <= 2,
    alpha 100): forward + per-scene loss + adjoint in one persistent launch."""
    import torch

    from paper_2401_11882_amd import batched
    from paper_2401_11882_amd import workloads as WL
    scenes = WL.batch_scenes(512)
    plan = batched.BatchPlan(scenes, 2, tune_cache=os.path.join(ROOT, "paper_2401_11882_amd", "tune_cache.txt"))
    info = plan.info()
    plan.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        plan.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    out = {"workload": "512 scenes, 8..128 segments + box, 64^2/128^2/256^2 rx, order<=2, alpha=100, fwd+adjoint",
           "path_evals": info["path_evals"], "ms": round(ms, 3),
           "value": info["path_evals"] / (ms * 1e-3), "unit": "path-evals/s", "launch": plan.config(),
           "roofline": alu_roofline("batched512_alpha100", "k_batched", ms, BATCHED_SOURCES,
                                    time_basis="HIP events around the whole batched call (k_batched and its "
                                               "two small setup/reduction kernels), averaged over 3 calls")}
    plan.close()
    return out


def extra_order3_loop(dev):
    """Box + 32 segments, 512^2 receivers, order <= 3: 200 graph-replayed Adam steps."""
    import torch

    from paper_2401_11882_amd import workloads as WL
    from paper_2401_11882_amd.optimize import optimize_tx
    s = WL.scene_32_order3()
    walls, tx, rx = (torch.tensor(a, device=dev) for a in (s.walls, s.tx, s.rx))
    optimize_tx(walls, tx, rx, 3, 100.0, steps=2, grid_nx=512)   # warm-up (workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = optimize_tx(walls, tx, rx, 3, 100.0, steps=200, grid_nx=512)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pe = s.n_rx * 45397
    L = res["loss_hist"].cpu().numpy()
    out = {"workload": "box + 32 segments, 512^2 rx, order<=3 (45397 candidates), alpha=100, 200 Adam steps",
           "s_total": round(dt, 3), "ms_per_step": round(1e3 * dt / 200, 3),
           "value": pe * 200 / dt, "unit": "path-evals/s", "loss_first": float(L[0]), "loss_last": float(L[-1])}
    # the steps replay one captured graph, so the kernel's own time comes from its kernel trace
    ctr = measured_counters("order3_loop_alpha100", "k_forward")
    if ctr is not None and ctr.get("avg_us"):
        out["roofline"] = alu_roofline("order3_loop_alpha100", "k_forward", ctr["avg_us"] / 1e3,
                                       time_basis="rocprofv3 kernel trace of the graph-replayed loop")
    return out


def extra_hard_sigmoid(dev, steps: int = 10):
    """Sec. IV-B says the hard sigmoid is much cheaper to evaluate than the
    sigmoid: the same fwd + adjoint step on the 64-segment scene with each."""
    import torch

    from paper_2401_11882_amd import tracer as tr
    from paper_2401_11882_amd import workloads as WL
    out = {"workload": "box + 64 segments, 256^2 rx, order<=2, fwd + adjoint"}
    for alpha in (50.0, 100.0):
        s = WL.scene_64(alpha=alpha)
        walls, tx, rx = (torch.tensor(a, device=dev) for a in (s.walls, s.tx, s.rx))
        row = {}
        for mode in ("sigmoid", "hard_sigmoid"):
            sc = tr.Scene(walls, tx, rx, 2, alpha, grid_nx=s.grid_n, smoothing=mode)
            for _ in range(2):
                tr.forward_backward(sc, loss="neg_mean_log")
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                tr.forward_backward(sc, loss="neg_mean_log")
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            row[mode] = {"ms": round(ms, 4), "value": s.n_rx * 4625 / (ms * 1e-3)}
        row["hard_over_sigmoid_speed"] = round(row["sigmoid"]["ms"] / row["hard_sigmoid"]["ms"], 3)
        out[f"alpha_{int(alpha)}"] = row
    return out


def extra_alpha_sweep(dev, steps: int = 10):
    """The benchmark step at the other sharpness values of the 64-segment
    workload (alpha = 10 and 1000; 100 is the main line)."""
    import numpy as np
    import torch

    from paper_2401_11882_amd import tracer as tr
    from paper_2401_11882_amd import workloads as WL
    out = {"workload": "box + 64 segments, 256^2 rx, order<=2 (4625 candidates), fwd + adjoint from the cache"}
    for alpha in (10.0, 1000.0):
        s = WL.scene_64(alpha=alpha)
        walls, tx, rx = (torch.tensor(a, device=dev) for a in (s.walls, s.tx, s.rx))
        sc = tr.Scene(walls, tx, rx, 2, alpha, grid_nx=s.grid_n)

        def step():
            P, L, seed = tr.forward(sc, loss="neg_mean_log", want_seed=True)
            mid = torch.cuda.Event(enable_timing=True)
            mid.record()
            tr.backward(sc, seed, reuse_forward=True)
            return mid

        for _ in range(2):
            step()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        mids = []
        for e0, e1 in ev:
            e0.record()
            mids.append(step())
            e1.record()
        torch.cuda.synchronize()
        fwd = float(np.mean([e0.elapsed_time(m) for (e0, _), m in zip(ev, mids)]))
        bwd = float(np.mean([m.elapsed_time(e1) for (_, e1), m in zip(ev, mids)]))
        row = {"ms_per_step": round(fwd + bwd, 4), "fwd_ms": round(fwd, 4),
               "bwd_ms": round(bwd, 4), "value": s.n_rx * 4625 / ((fwd + bwd) * 1e-3)}
        name, kms, key = (("k_backward", bwd, "bwd_flops_per_path_eval") if bwd >= fwd
                          else ("k_forward", fwd, "fwd_flops_per_path_eval"))
        pa = work_model("2d", alpha)
        row["roofline"] = alu_roofline(f"scene64_alpha{int(alpha)}", name, kms,
                                       model_flops=None if pa is None else pa[key] * s.n_rx * 4625)
        out[f"alpha_{int(alpha)}"] = row
    return out


def extra_fermat(dev, steps: int = 5):
    """Sec. V-B's second path finder on the benchmark scene: the forward pass
    with Fermat path tracing (Newton on the path length per lane, smoothed
    convergence check) next to the image-method forward."""
    import torch

    from paper_2401_11882_amd import tracer as tr
    from paper_2401_11882_amd import workloads as WL
    s = WL.scene_64(alpha=100.0)
    walls, tx, rx = (torch.tensor(a, device=dev) for a in (s.walls, s.tx, s.rx))
    sc = tr.Scene(walls, tx, rx, 2, 100.0, grid_nx=s.grid_n)
    out = {"workload": "box + 64 segments, 256^2 rx, order<=2 (4625 candidates), alpha=100, forward only"}
    for name, fn in (("fermat", lambda: tr.forward_fermat(sc, loss="neg_mean_log")),
                     ("image_method", lambda: tr.forward(sc, loss="neg_mean_log"))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[name] = {"ms": round(ms, 4), "value": s.n_rx * 4625 / (ms * 1e-3), "unit": "path-evals/s"}
    Pf, _ = tr.forward_fermat(sc)
    Pi, _, _ = tr.forward(sc)
    r = (Pf.double() - Pi.double()).abs() / Pi.double()
    out["power_rel_diff_to_image_method"] = {"median": float(r.median()), "frac_below_1e-5": float((r < 1e-5).double().mean())}
    out["roofline"] = alu_roofline("fermat_scene64", "k_forward_fermat", out["fermat"]["ms"], sources=FERMAT_SOURCES,
                                   time_basis="HIP events around the whole Fermat forward call (k_forward_fermat "
                                              "and its small setup and loss kernels), averaged over the calls")
    return out


PEAK_BF16_TFLOPS = 2500.0      # MI355X dense BF16 MFMA (datasheet, without sparsity)
MLP_FWD_FLOPS = 2 * (128 * 256 + 4 * 256 * 256 + 256)   # per row: 5 hidden layers + head
# training adds the weight gradients of every layer, the input gradients of
# hidden layers 1..4 (layer 0's inputs are fixed features) and the head's
MLP_TRAIN_FLOPS = MLP_FWD_FLOPS + 2 * (128 * 256 + 4 * 256 * 256) + 2 * (4 * 256 * 256) + 2 * 256


def extra_mlp(dev, steps: int = 20):
    """The surrogate's BF16-MFMA kernels alone: the fused forward on 2^20 rows,
    the transmitter scan of the search (128^2 tx x 64^2 rx) and one training
    step (16,384 rows: forward, MSE, backward, Adam), against the dense BF16
    peak.  FLOPs are the network's multiply-adds (2 per MAC)."""
    import torch

    from paper_2401_11882_amd import surrogate as S
    from paper_2401_11882_amd import workloads as WL
    net = S.Surrogate(WL.fourier_matrix(0), S.init_params(0), max_batch=65536)
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    out = {"workload": "6-layer MLP, width 256, 64 Fourier features, BF16 MFMA / FP32 accumulation"}

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    v = torch.rand(1 << 20, 4, device=dev, generator=g)
    ms = timed(lambda: net.forward(v), steps)
    tf = (1 << 20) * MLP_FWD_FLOPS / (ms * 1e-3) / 1e12
    out["forward_2p20_rows"] = {"ms": round(ms, 4), "tflops": round(tf, 1), "frac": round(tf / PEAK_BF16_TFLOPS, 4)}
    txg = torch.tensor(WL.rx_grid(128), device=dev)
    rxs = torch.tensor(WL.rx_grid(64), device=dev)
    ms = timed(lambda: net.scan(txg, rxs), 3)
    rows = 128 * 128 * 64 * 64
    tf = rows * MLP_FWD_FLOPS / (ms * 1e-3) / 1e12
    out["scan_128sq_tx_64sq_rx"] = {"ms": round(ms, 3), "tflops": round(tf, 1), "frac": round(tf / PEAK_BF16_TFLOPS, 4)}
    vb = torch.rand(16384, 4, device=dev, generator=g)
    yb = torch.randn(16384, device=dev, generator=g)
    ms = timed(lambda: net.train_step(vb, yb, 1e-4), steps)
    tf = 16384 * MLP_TRAIN_FLOPS / (ms * 1e-3) / 1e12
    out["train_step_16384_rows"] = {"ms": round(ms, 4), "tflops": round(tf, 1),
                                    "frac": round(tf / PEAK_BF16_TFLOPS, 4)}
    net.close()
    out["roofline"] = {"bound": "mfma", "achieved": out["scan_128sq_tx_64sq_rx"]["tflops"], "peak": PEAK_BF16_TFLOPS,
                       "unit": "TFLOP/s", "frac": out["scan_128sq_tx_64sq_rx"]["frac"], "traffic": None,
                       "kernel": "k_mlp_fused (scan)",
                       "time_basis": "HIP events around the whole scan (fused forward launches and per-transmitter means)"}
    return out


def extra_placement():
    """Sec. VII: success rate of annealed versus unsmoothed transmitter placement."""
    import torch

    from paper_2401_11882_amd import placement
    t0 = time.perf_counter()
    res = placement.study(n_per_count=1024, rx_counts=(2, 3, 4), grid_n=128)
    torch.cuda.synchronize()
    return {"workload": "1024 seeded problems per receiver count (2, 3, 4), LOS, 100 Adam iterations, "
                        "alpha 1 -> 100 geometric vs alpha 1e6; success = unsmoothed F >= 0.9 x best of a 128^2 grid",
            "s_total": round(time.perf_counter() - t0, 3),
            "by_rx_count": {str(k): v for k, v in res.items()}}


def extra_surrogate():
    from paper_2401_11882_amd import surrogate
    r = surrogate.experiment(seed=0)
    sur = r["surrogate"]
    return {"workload": "64-segment scene, 1e7 tracer samples, 6-layer BF16 MLP, 128^2 tx scan, exact refinement",
            "speedup_at_1pct": None if r["speedup"] is None else round(r["speedup"], 3),
            "speedup_lower_bound": None if r["speedup_lower_bound"] is None else round(r["speedup_lower_bound"], 3),
            "speedup_basis": "search time only (scan + exact refinement vs exact Adam from random starts); "
                             "data generation and training reported separately",
            "exact_step_ratio": round(r["exact_step_ratio"], 3),
            "plain_s": [round(p["t_total"], 3) for p in r["plain"]],
            "plain_starts_tried": [int(p["starts_tried"]) for p in r["plain"]],
            "surrogate_s": round(sur["t_total"], 3), "surrogate_scan_s": round(sur["t_scan"], 3),
            "surrogate_exact_steps": sur.get("exact_steps"),
            "surrogate_reached": sur["reached"], "plain_reached": [p["reached"] for p in r["plain"]],
            "F_star": r["F_star"], "F_surrogate": sur["F"], "F_plain": [p["F"] for p in r["plain"]],
            "datagen_s": round(r["datagen_s"], 3), "train_s": round(r["train_s"], 3),
            "surrogate_end_to_end_s": round(r["surrogate_end_to_end_s"], 3),
            "break_even_searches": r["break_even_searches"],
            "heldout_rmse": round(r["heldout_rmse"], 4), "heldout_max_abs": round(r["heldout_max_abs"], 4),
            "target_std": round(r["target_std"], 4),
            "objective_error_log_power": {"at_top_scan_start": round(sur["abs_err_top"], 4),
                                          "Fhat_top": round(sur["Fhat_top"], 4), "F_top": round(sur["F_top"], 4),
                                          "at_refined_tx": round(sur["abs_err_best"], 4),
                                          "Fhat_refined": round(sur["Fhat_best"], 4)}}


def extra_3d(dev, steps: int = 10, smoothing: str = "sigmoid"):
    """Sec. VI: the method in three dimensions.  Room (6 panels) + 32 random
    rectangles, 256^2 receivers at mid-height, order <= 2 (1,445 panel
    sequences), alpha = 100: forward, then the adjoint from the recorded
    contributions, as in the main step."""
    import numpy as np
    import torch

    from paper_2401_11882_amd import tracer3d as tr3
    from paper_2401_11882_amd import workloads as WL
    s = WL.scene3d_32()
    pan, tx, rx = (torch.tensor(a, device=dev) for a in (s.panels, s.tx, s.rx))
    sc = tr3.Scene3(pan, tx, rx, s.max_order, s.alpha, grid_nx=s.grid_n, smoothing=smoothing)
    n_cand = 1 + s.n_panels + s.n_panels * (s.n_panels - 1)

    def step():
        P, L, seed = tr3.forward(sc, loss="neg_mean_log", want_seed=True)
        mid = torch.cuda.Event(enable_timing=True)
        mid.record()
        tr3.backward(sc, seed, reuse_forward=True)
        return mid

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    mids = []
    for e0, e1 in ev:
        e0.record()
        mids.append(step())
        e1.record()
    torch.cuda.synchronize()
    fwd = float(np.mean([e0.elapsed_time(m) for (e0, _), m in zip(ev, mids)]))
    bwd = float(np.mean([m.elapsed_time(e1) for (_, e1), m in zip(ev, mids)]))
    ms = fwd + bwd
    out = {"workload": "room + 32 rectangles (38 panels), 256^2 rx, order<=2 (1445 candidates), alpha=100, "
                       "fwd + adjoint w.r.t. tx and all panel corners",
           "ms_per_step": round(ms, 4), "fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4),
           "value": s.n_rx * n_cand / (ms * 1e-3), "unit": "path-evals/s"}
    if smoothing != "sigmoid":
        return out
    out["hard_sigmoid"] = extra_3d(dev, steps, smoothing="hard_sigmoid")
    out["hard_over_sigmoid_speed"] = round(out["ms_per_step"] / out["hard_sigmoid"]["ms_per_step"], 3)
    pa = work_model("scene3d", s.alpha)
    name, kms, key = (("k_backward3", bwd, "bwd_flops_per_path_eval") if bwd >= fwd
                      else ("k_forward3", fwd, "fwd_flops_per_path_eval"))
    out["roofline"] = alu_roofline("scene3d_32_alpha100", name, kms, TRACER3D_SOURCES,
                                   model_flops=None if pa is None else pa[key] * s.n_rx * n_cand)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--alpha", type=float, default=100.0)
    ap.add_argument("--cpu-sample", type=int, default=192, help="receivers per CPU oracle baseline run")
    ap.add_argument("--cpu-sample-single", type=int, default=16,
                    help="receivers per single-thread CPU oracle baseline run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, order-3 loop and surrogate measurements")
    ap.add_argument("--extra", default=None,
                    help="run only the named extra measurement (scene3d, alpha_sweep, hard_sigmoid, ...) "
                         "and print its JSON")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="after timing, copy a buffer of this many MiB once (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding over several GPUs is "
              "described, not implemented.", file=sys.stderr)
        return 2
    rank = int(os.environ.get("RANK", "0"))
    if args.extra is not None:
        import torch
        dev = torch.device("cuda:0")
        fns = {"scene3d": lambda: extra_3d(dev), "alpha_sweep": lambda: extra_alpha_sweep(dev),
               "hard_sigmoid": lambda: extra_hard_sigmoid(dev), "batched": lambda: extra_batched(dev),
               "order3_loop": lambda: extra_order3_loop(dev), "placement": extra_placement,
               "fermat": lambda: extra_fermat(dev), "mlp": lambda: extra_mlp(dev),
               "surrogate": extra_surrogate}
        if args.extra not in fns:
            print(f"unknown extra {args.extra!r}; choose from {sorted(fns)}", file=sys.stderr)
            return 2
        print(json.dumps({args.extra: fns[args.extra]()}), flush=True)
        if args.copy_calib_mb > 0:
            copy_calibration(dev, args.copy_calib_mb)
        return 0

    import numpy as np
    import torch

    from paper_2401_11882_amd import tracer as tr
    from paper_2401_11882_amd import workloads as WL

    dev = torch.device("cuda:0")
    s = WL.scene_64(alpha=args.alpha)
    walls = torch.tensor(s.walls, device=dev)
    tx = torch.tensor(s.tx, device=dev)
    rx = torch.tensor(s.rx, device=dev)
    scene = tr.Scene(walls, tx, rx, s.max_order, args.alpha, grid_nx=s.grid_n)
    n_cand = tr.num_candidates(s.n_walls, s.max_order)
    pe_per_step = s.n_rx * n_cand

    def step():
        P, L, seed = tr.forward(scene, loss="neg_mean_log", want_seed=True)
        ev_mid = torch.cuda.Event(enable_timing=True)
        ev_mid.record()
        gtx, gw, _ = tr.backward(scene, seed, reuse_forward=True)
        return ev_mid, L, gtx

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    mids = []
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for i in range(args.steps):
        starts[i].record()
        ev_mid, L, gtx = step()
        mids.append(ev_mid)
        ends[i].record()
    ev1 = torch.cuda.Event(enable_timing=True)
    ev1.record()
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    fwd_ms = float(np.mean([starts[i].elapsed_time(mids[i]) for i in range(args.steps)]))
    bwd_ms = float(np.mean([mids[i].elapsed_time(ends[i]) for i in range(args.steps)]))
    total_s = max(wall_s, gpu_ms / 1e3)
    ms_per_step = 1e3 * total_s / args.steps
    value = pe_per_step * args.steps / total_s

    if args.copy_calib_mb > 0:
        copy_calibration(dev, args.copy_calib_mb)

    # dominant kernel: executed FP32 FLOPs (committed counters) over its live time
    name, kms, key = (("k_backward", bwd_ms, "bwd_flops_per_path_eval") if bwd_ms >= fwd_ms
                      else ("k_forward", fwd_ms, "fwd_flops_per_path_eval"))
    pa = work_model("2d", args.alpha)
    roofline = alu_roofline(f"scene64_alpha{int(args.alpha)}", name, kms,
                            model_flops=None if pa is None else pa[key] * pe_per_step)
    if pa is not None:
        roofline["model_flops_per_path_eval"] = round(pa[key], 3)
    try:
        fma_peak, exp_rate = tr.valu_peak()
        roofline["sustained_fma_tflops"] = round(fma_peak, 2)
        roofline["sustained_exp_tlanes"] = round(exp_rate, 2)
        if roofline["achieved"] is not None:
            roofline["frac_of_sustained_fma"] = round(roofline["achieved"] / fma_peak, 4)
    except Exception as exc:  # diagnostic only; the line is valid without it
        roofline["sustained_fma_tflops"] = f"unavailable: {exc}"

    out = {
        "metric": "smoothed path-evals/s fwd+bwd (rx x candidates)",
        "value": value, "unit": "path-evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "box + 64 segments, 256x256 rx grid, order<=2 (4625 candidates), alpha=100, "
                               "fwd + adjoint w.r.t. tx and all wall endpoints",
                   "receivers": s.n_rx, "candidates": n_cand, "alpha": args.alpha,
                   "path_evals_per_step": pe_per_step},
        "fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4),
        "roofline": roofline,
    }
    if rank == 0 and not args.no_extras:
        out["extras"] = {"batched_512_scenes": extra_batched(dev), "order3_adam_loop": extra_order3_loop(dev),
                         "hard_sigmoid": extra_hard_sigmoid(dev), "scene3d": extra_3d(dev),
                         "alpha_sweep": extra_alpha_sweep(dev), "fermat": extra_fermat(dev),
                         "mlp_kernels": extra_mlp(dev),
                         "placement_study": extra_placement(),
                         "surrogate": extra_surrogate()}
        out["surrogate_speedup_at_1pct"] = out["extras"]["surrogate"]["speedup_at_1pct"]
        out["surrogate_speedup_lower_bound"] = out["extras"]["surrogate"]["speedup_lower_bound"]
    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.alpha, args.cpu_sample, args.cpu_sample_single)
    if rank == 0:
        print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
