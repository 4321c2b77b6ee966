"""Throughput benchmark of the sampler's hot path on one MI355X.

One step = the whole hot path over one batch of the 42-node, 48-edge,
4-objective workload (20 000 Dirichlet weight vectors x 256 replicas x 2 000
steps): ballistic and discrete SB sampling with fused exact cut evaluation
(FP32), non-dominated filtering of the pooled 10.24 M cut vectors, and the
exact hypervolume of the resulting front.  Inputs are seeded synthetic
stand-ins for the paper's 42-node instances and are resident on the GPU before
the timed region.

Prints one JSON line.  The optional CPU baseline runs the oracle (test
infrastructure) on a bounded slice of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "replica-steps/s & time-to-ref-hypervolume: chosen form vs plain FP32, 1 GPU"
WORKLOAD = "c2_n42_m4"
# FP32 FMA on the vector ALUs with packed FP32 disabled (the build turns it
# off): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s (the
# datasheet's 157.3 counts packed FMA).
PEAK_FP32_FMA_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def fma_flops_per_replica_step(n: int, E: int) -> int:
    """Algorithmic flops of one replica-step of the sparse kernel: 2|E| field
    FMAs plus, per spin, one FMA for -(a0 - a_t) x and one for x += dt a0 y,
    two flops each.  The wall's compare/select/clamp (and dSB's sign) are
    integer-like selects, not flops."""
    return 2 * (2 * E + 2 * n)


def cpu_baseline(inst, weights, R, T, budget_s=12.0):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    probe = weights[:4]
    t0 = time.perf_counter()
    oracle.sb_sample(inst, probe, R, T, "bsb", dt=0.5, seed=7, nthreads=threads)
    dt_probe = time.perf_counter() - t0
    rate = probe.shape[0] * R * T / max(dt_probe, 1e-9)
    nw = int(max(4, min(weights.shape[0], budget_s * rate / (R * T))))
    t0 = time.perf_counter()
    spins = oracle.sb_sample(inst, weights[:nw], R, T, "bsb", dt=0.5, seed=7, nthreads=threads)
    oracle.cut_values(inst, spins)
    el = time.perf_counter() - t0
    return {"value": nw * R * T / el, "unit": "replica-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"bSB on the first {nw} of {weights.shape[0]} weight vectors x {R} replicas x "
                      f"{T} steps, fp64 dynamics + exact cuts ({el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--path", default="auto")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sampler's work shards over weight vectors "
              "with one front merge, which this build does not implement (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_26477_amd as q
    import workloads as wl

    cfg = wl.WORKLOADS[WORKLOAD]
    inst = wl.workload_instance(WORKLOAD)
    c_host = wl.workload_weights(WORKLOAD)
    W, R, T = cfg["W"], cfg["R"], cfg["T"]
    dev = torch.device("cuda", 0)
    prob = q.problem_from_instance(inst, 0)
    c = torch.from_numpy(c_host).to(dev)
    variants = ("bsb", "dsb")
    scheds = {v: q.make_schedule(v, steps=T, dt=0.5, seed=cfg["seed"] + 3 + i, path=args.path)
              for i, v in enumerate(variants)}
    rows = W * R
    spins = torch.empty((2 * rows, prob.words), dtype=torch.int64, device=dev)
    obj = torch.empty((2 * rows, inst.m), dtype=torch.int64, device=dev)
    ws_s = torch.empty(max(q.qaia_sample_workspace_bytes(prob, W, R, s) for s in scheds.values()),
                       dtype=torch.uint8, device=dev)
    keep = torch.empty(2 * rows, dtype=torch.int64, device=dev)
    nkeep = torch.empty(1, dtype=torch.int64, device=dev)
    ws_f = torch.empty(q.qaia_pareto_filter_workspace_bytes(2 * rows, inst.m), dtype=torch.uint8,
                       device=dev)
    stream = torch.cuda.current_stream()
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("bsb", "dsb", "filter")}
    ref = np.zeros(inst.m, np.int64)

    def step(record):
        times = {}
        for i, v in enumerate(variants):
            if record:
                ev[v][0].record(stream)
            q.qaia_sample(prob, c, R, scheds[v], spins=spins[i * rows:(i + 1) * rows],
                          obj=obj[i * rows:(i + 1) * rows], workspace=ws_s, stream=stream)
            if record:
                ev[v][1].record(stream)
        if record:
            ev["filter"][0].record(stream)
        q.qaia_pareto_filter(obj, keep_idx=keep, num_keep=nkeep, workspace=ws_f, stream=stream)
        if record:
            ev["filter"][1].record(stream)
        P = int(nkeep.item())  # synchronises the stream
        front = obj[keep[:P]].cpu().numpy()
        t0 = time.perf_counter()
        hv = q.qaia_hypervolume(front, ref)
        times["hv_ms"] = (time.perf_counter() - t0) * 1e3
        if record:
            for k in ev:
                times[f"{k}_ms"] = ev[k][0].elapsed_time(ev[k][1])
        return P, hv, times

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P, hv, times = step(True)
        per.append(times)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    total_rs = 2 * rows * T
    stage = {k: float(np.mean([p[k] for p in per])) for k in per[0]}

    # roofline of the dominant kernel: the generated sparse SB kernel, whose
    # launches (one bSB, one dSB per step) do the same flops each
    flops_per_launch = fma_flops_per_replica_step(inst.n, inst.num_edges) * rows * T
    avg_launch_ms = float(np.mean([stage[f"{v}_ms"] for v in variants]))
    achieved = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    result = {
        "metric": METRIC, "value": total_rs / (ms_per_step * 1e-3), "unit": "replica-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "42-node degree<=3 graph, 48 edges, m=4 N(0,1) int32 fixed-point "
                               "weights; 20000 Dirichlet(1,1,1,1) weight vectors x 256 replicas x "
                               "2000 steps, dt=0.5; bSB and dSB FP32 sampling + exact cuts, "
                               "filter of the 10.24M-vector pool, exact hypervolume (origin)",
                   "W": W, "R": R, "T": T, "n": inst.n, "m": inst.m, "edges": inst.num_edges,
                   "path": args.path},
        "roofline": {"bound": "alu", "kernel": "qaia_sb_reg (bSB and dSB launches)",
                     "achieved": achieved, "peak": PEAK_FP32_FMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_FMA_TFLOPS, "traffic": None,
                     "avg_launch_ms": avg_launch_ms, "flops_per_launch": flops_per_launch},
        "stages_ms": stage,
        "sampling_replica_steps_per_s": {v: rows * T / (stage[f"{v}_ms"] * 1e-3) for v in variants},
        "front_size": P, "hypervolume": str(hv),
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(inst, c_host, R, T)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
