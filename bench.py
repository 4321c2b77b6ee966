"""Throughput benchmark of the sampler's hot path on one MI355X.

One step = the whole hot path over one batch of the 42-node, 48-edge,
4-objective workload (20 000 Dirichlet weight vectors x 256 replicas x 2 000
steps): ballistic and discrete SB sampling with fused exact cut evaluation
(FP32), non-dominated filtering of the pooled 10.24 M cut vectors, and the
exact hypervolume of the resulting front.  Inputs are seeded synthetic
stand-ins for the paper's 42-node instances and are resident on the GPU before
the timed region.

Consecutive steps are pipelined: the exact hypervolume of step k runs on a
host thread while the GPU samples step k + 1; every step's hypervolume
completes inside the timed region.

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
# Datasheet FP32 vector peak of the MI355X (256 CUs x 2.4 GHz, counting packed
# FP32 FMA): the denominator of the sparse kernel's algorithmic roofline.
PEAK_FP32_VECTOR_TFLOPS = 157.3
# Single-issue rate of non-packed FP32 FMAs (256 CUs x 4 SIMDs x 16 lanes x 2
# flop x 2.4 GHz; the library is compiled with packed FP32 disabled).  Two
# waves' 32-bit-encoded FMAs (v_fmac_f32) can issue in the same slot, which is
# how non-packed code goes past it toward the datasheet figure.
PEAK_FP32_FMA_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
SIMDS, CLOCK_HZ = 256 * 4, 2.4e9

# HBM bytes of one qaia_sb_reg launch on this workload, from two rocprofv3
# --pmc passes over `bench.py --traffic-probe` (FETCH_SIZE, then WRITE_SIZE,
# KiB per dispatch), each scaled by the same counter's reading for a plain
# 1 GiB device copy in the same process (nine copy dispatches: read 524322.4375
# KiB, written 1048579.46875 KiB).  Set to None whenever the generated kernel
# changes, until the counters are taken again.
_KIB = 1024.0
_FETCH_SCALE = 1048576.0 / 524322.4375
_WRITE_SCALE = 1048576.0 / 1048579.46875
SB_REG_TRAFFIC_BYTES = (5243.5 * _FETCH_SCALE + 203296.25 * _WRITE_SCALE) * _KIB


def algorithmic_flops_per_replica_step(n: int, E: int) -> int:
    """Algorithmic work of one sparse replica-step in the combined-weight form:
    2|E| field FMAs plus three per spin (the stiffness term, the coupling scale
    and the x update), two flops each."""
    return 2 * (2 * E + 3 * n)


def fma_flops_per_replica_step(n: int, E: int) -> int:
    """Flops the generated kernel performs per replica-step: 2|E| field FMAs
    (c0 folded into the coefficients) plus one FMA for -(a0 - a_t) x and one
    for x += dt a0 y per spin."""
    return 2 * (2 * E + 2 * n)


def valu_instructions_per_replica_step(inst, variant: str) -> int:
    """VALU instructions of the generated kernel's step loop per replica (one
    replica per lane): 2|E| + 2n FMAs, three wall operations per spin
    (compare, select, clamp) and, for discrete SB, one copysign per spin that
    feeds a neighbour.  For the 42-node, 48-edge graph: 306 (bSB), 347 (dSB);
    the compiled loop, two steps per iteration, adds one register move per
    step (the step coefficient into a VGPR)."""
    n, E = inst.n, inst.num_edges
    base = 2 * E + 5 * n
    if variant == "dsb":
        deg = np.bincount(np.concatenate([inst.edge_u, inst.edge_v]), minlength=n)
        base += int((deg > 0).sum())
    return base


def cpu_baseline(inst, weights, R, T, budget_s=12.0):
    """The oracle on the host cores, on bounded slices of the same workload: bSB
    and dSB sampling (fp64 dynamics + exact cuts) on the first weight vectors,
    the non-dominated filter on the oracle's own sample pool (at most 200 000
    rows) and the exact hypervolume of its front.  value: replica-steps/s of
    the whole step (both variants, filter and hypervolume) extrapolated from
    the per-row and per-replica-step costs of the slices."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    probe = weights[:4]
    t0 = time.perf_counter()
    oracle.sb_sample(inst, probe, R, T, "bsb", dt=0.5, seed=7, nthreads=threads)
    dt_probe = time.perf_counter() - t0
    rate = probe.shape[0] * R * T / max(dt_probe, 1e-9)
    nw = int(max(4, min(weights.shape[0], budget_s * 0.6 * rate / (R * T))))
    t0 = time.perf_counter()
    spins = oracle.sb_sample(inst, weights[:nw], R, T, "bsb", dt=0.5, seed=7, nthreads=threads)
    obj_b = oracle.cut_values(inst, spins)
    el_b = time.perf_counter() - t0
    rate_b = nw * R * T / el_b
    nwd = int(max(4, min(weights.shape[0], budget_s * 0.25 * rate / (R * T))))
    t0 = time.perf_counter()
    spins = oracle.sb_sample(inst, weights[:nwd], R, T, "dsb", dt=0.5, seed=8, nthreads=threads)
    obj_d = oracle.cut_values(inst, spins)
    el_d = time.perf_counter() - t0
    rate_d = nwd * R * T / el_d
    pool = np.concatenate([obj_b, obj_d])[:200000]
    t0 = time.perf_counter()
    keep = oracle.pareto_filter(pool)
    el_f = time.perf_counter() - t0
    front = pool[keep]
    t0 = time.perf_counter()
    oracle.hypervolume(front, np.zeros(inst.m, np.int64))
    el_hv = time.perf_counter() - t0
    rows = weights.shape[0] * R
    # one step on the CPU at these rates: both variants, the filter at the
    # slice's cost per row (a lower bound: the oracle's filter grows faster
    # than linearly), one hypervolume
    step_s = rows * T / rate_b + rows * T / rate_d + 2 * rows * el_f / pool.shape[0] + el_hv
    value = 2 * rows * T / step_s
    # the bSB sampler on one core, on about 3 s of work
    n1 = int(max(1, min(weights.shape[0], 3.0 * rate_b / threads / (R * T))))
    t0 = time.perf_counter()
    spins = oracle.sb_sample(inst, weights[:n1], R, T, "bsb", dt=0.5, seed=7, nthreads=1)
    oracle.cut_values(inst, spins)
    el1 = time.perf_counter() - t0
    return {"value": value, "unit": "replica-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"bSB on the first {nw} and dSB on the first {nwd} of {weights.shape[0]} weight vectors "
                      f"x {R} replicas x {T} steps (fp64 dynamics + exact cuts, {el_b:.1f} s + {el_d:.1f} s); "
                      f"filter of {pool.shape[0]} of those cut vectors ({el_f:.2f} s, front {front.shape[0]}); "
                      f"exact hypervolume of that front ({el_hv:.2f} s); whole-step rate extrapolated to "
                      f"{2 * rows} rows",
            "stages": {"bsb_replica_steps_per_s": rate_b, "dsb_replica_steps_per_s": rate_d,
                       "filter_rows": int(pool.shape[0]), "filter_s": el_f, "filter_rows_per_s": pool.shape[0] / el_f,
                       "front": int(front.shape[0]), "hypervolume_s": el_hv},
            "one_core": {"value": n1 * R * T / el1, "unit": "replica-steps/s",
                         "sample": f"bSB on the first {n1} weight vectors, 1 thread ({el1:.1f} s)"}}


def precision_form(q, wl, torch, T=1000):
    """Precision workload: dSB on a complete 2048-node, 3-objective graph, 512
    Dirichlet weight vectors x 8 replicas (4096 matrix columns), 1000 steps,
    FP32 vs BF16 vs FP8 coupling products (exact integer cut evaluation)."""
    N, m, W, R = 2048, 3, 512, 8
    inst = wl.random_instance(N, m, "complete", seed=3000)
    prob = q.problem_from_instance(inst, 0)
    c = torch.from_numpy(wl.dirichlet_weights(W, m, 3002)).cuda()
    out = {"workload": f"complete N={N}, m={m}, {W} weight vectors x {R} replicas, T={T}, dSB dense, "
                       "LDS-staged matrix-core tiles (128 x 256 for BF16 and FP8, 128 x 128 for FP32)"}
    flops = 2 * m * N * N * W * R * T
    for prec in ("fp32", "bf16", "fp8"):
        s = q.make_schedule("dsb", precision=prec, steps=T, dt=0.5, seed=3003, path="dense_staged")
        spins, obj, ws = q.qaia_sample(prob, c, R, s)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        q.qaia_sample(prob, c, R, s, spins=spins, obj=obj, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out[prec] = {"ms": ms, "replica_steps_per_s": W * R * T / (ms * 1e-3),
                     "matrix_TFLOPs": flops / (ms * 1e-3) / 1e12}
    return out


def measured_peaks(q, torch, reps=3):
    """This GPU's own ceilings, from the library's measurement kernels (best
    of `reps` timed launches after one untimed): fp32 FMA issue (eight
    independent chains per lane, 16 waves per CU), the matrix-core rate per
    operand format (four independent 32x32 accumulators per wave, 16 waves
    per CU) and an HBM-to-HBM copy of 1 GiB."""
    dev = torch.device("cuda", 0)

    def best_ms(fn):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return min(times)

    out = torch.empty(4096 * 256, dtype=torch.float32, device=dev)
    fma_iters = 1 << 15
    ms = best_ms(lambda: q.qaia_peak_fma(4096, fma_iters, 1.0, 1.0, out=out))
    res = {"fp32_fma_TFLOPs": 4096 * 256 * fma_iters * 16 / (ms * 1e-3) / 1e12}
    mix_iters = 1 << 13
    ms = best_ms(lambda: q.qaia_peak_valu(4096, mix_iters, 0.0, out=out))
    res["valu_mix_Tinstr_per_s"] = 4096 * 256 * mix_iters * 102 / (ms * 1e-3) / 1e12
    for prec, K, iters in (("fp32", 2, 8192), ("bf16", 16, 16384), ("fp8", 64, 16384)):
        ms = best_ms(lambda: q.qaia_peak_mfma(prec, 1024, iters, out=out))
        res[f"{prec}_mfma_TFLOPs"] = 1024 * 4 * iters * 4 * 2 * 32 * 32 * K / (ms * 1e-3) / 1e12
    src = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(3)
    dst = torch.empty_like(src)
    ms = best_ms(lambda: q.qaia_peak_copy(src, dst))
    res["hbm_copy_GBps"] = 2 * src.numel() * 4 / (ms * 1e-3) / 1e9
    del src, dst
    res["method"] = ("library measurement kernels: 4096 x 256 lanes of 8 FMA chains; 4096 x 256 lanes of the "
                     "sparse SB instruction mix (60 FMAs + 42 compare/select/clamp per iteration); 1024 x 4 waves "
                     "of 4 independent 32x32 MFMAs (operands 1.0); 1 GiB device copy; best of 3")
    return res


def _race(q, prob, base, ref_rounds, contenders, seeds, cap=1.6):
    """One time-to-reference race: the reference hypervolume is the final
    archive of the plain FP32 loop (uniform Dirichlet vectors, seed 777) after
    ref_rounds rounds (10x the budget); every contender runs, per seed, until
    its archive reaches it or cap x the reference's rounds / seconds pass,
    and is judged afterwards (learned.time_to_hypervolume)."""
    from paper_2604_26477_amd.learned import ProposerLoop, reference_run, time_to_hypervolume
    ProposerLoop(prob, learned=False, seed=5, judge="record", **base).round()  # warm-up
    ref_hv, ref_s, ref_front = reference_run(prob, ref_rounds, 777, **base)
    out = {"reference": {"rounds": ref_rounds, "seconds": ref_s, "front": ref_front, "hv": str(ref_hv)},
           "seeds": list(seeds), "contenders": {}}
    for name, extra in contenders:
        kw = dict(base)
        kw.update(extra)
        ProposerLoop(prob, seed=5, judge="record", **kw).round()  # kernels built on first use, caches
        runs = []
        for sd in seeds:
            loop = ProposerLoop(prob, seed=sd, judge="record", **kw)
            runs.append(time_to_hypervolume(loop, ref_hv, int(ref_rounds * cap) + 1, max_seconds=ref_s * cap))
        secs = [r["seconds"] for r in runs if r["reached"]]
        rnds = [r["rounds"] for r in runs if r["reached"]]
        out["contenders"][name] = {
            "reached": f"{len(secs)}/{len(runs)}",
            "seconds_median": float(np.median(secs)) if len(secs) == len(runs) else None,
            "seconds_min": min(secs) if secs else None, "seconds_max": max(secs) if secs else None,
            "rounds_median": float(np.median(rnds)) if len(rnds) == len(runs) else None,
            "seconds_per_round": float(np.median([r["seconds_run"] / r["rounds_run"] for r in runs])),
            "runs": runs}
    return out


def learned_form(q, wl, torch, seeds=(11, 12, 13)):
    """Time to a reference hypervolume (the learned form's measurement and the
    metric's time-to-reference part).  Both workloads run rounds of 1024 weight
    vectors, each sampled, filtered against the loop's archive and labelled;
    the reference is the plain FP32 loop at 10x its budget.
      42-node m = 4 (sparse, 256 replicas, 2000 steps): plain FP32 bSB, the
        learned proposer with the same sampler, and noise-injected bSB with the
        paper's short schedule (50 steps, dt 1, alpha 0.1, Eq. 10) as its own
        contender;
      complete N = 512 m = 4 (dense, 8 replicas, 1000 steps): plain FP32 bSB on
        the matrix cores, discrete SB on the BF16 path with uniform vectors, and
        the combined form: the learned proposer with discrete SB on the BF16
        path (each round one batched launch of all its weight vectors x
        replicas)."""
    out = {}
    inst = wl.instance_42_node(4, seed=2000)
    prob = q.problem_from_instance(inst, 0)
    out["n42_m4"] = _race(q, prob, dict(R=256, steps=2000, n_cand=65536, n_sel=1024), 400,
                          (("plain_fp32_bsb", dict(learned=False)),
                           ("learned_fp32_bsb", dict(learned=True)),
                           ("ni_bsb_short", dict(learned=False, steps=50, dt=1.0, noise_alpha=0.1))), seeds)
    inst = wl.random_instance(512, 4, "complete", seed=5000)
    prob = q.problem_from_instance(inst, 0)
    out["complete512_m4"] = _race(q, prob, dict(R=8, steps=1000, n_cand=65536, n_sel=1024, variant="bsb",
                                                precision="fp32"), 20,
                                  (("plain_fp32_bsb", dict(learned=False)),
                                   ("uniform_dsb_bf16", dict(learned=False, variant="dsb", precision="bf16")),
                                   ("learned_dsb_bf16", dict(learned=True, variant="dsb", precision="bf16"))), seeds)
    return out


def batch_form(q, wl, torch):
    """Batching workload: 64 ragged instances, each 1024 Dirichlet weight
    vectors x 32 replicas x 1500 steps; one autotuned batched graph launch vs
    64 per-instance qaia_sample calls on the same paths.  The same instances
    with 32 weight vectors each show the regime batching is for: every
    instance alone leaves most of the GPU idle."""
    return {"full": batch_run(q, wl, torch, W=1024), "small_instances": batch_run(q, wl, torch, W=32)}


def batch_run(q, wl, torch, variant="bsb", precision="fp32", T=1500, W=1024, R=32, count=64):
    specs = wl.ragged_batch(count)
    items, probs = [], []
    for n, m, kind, sd in specs:
        inst = wl.random_instance(n, m, kind, seed=sd)
        p = q.problem_from_instance(inst, 0)
        c = torch.from_numpy(wl.dirichlet_weights(W, m, sd + 2)).cuda()
        probs.append((p, c))
        items.append(q.BatchItem(p, c, R, "auto"))
    s = q.make_schedule(variant, precision=precision, steps=T, dt=0.5, seed=4444)
    t0 = time.perf_counter()
    est = q.qaia_plan_autotune(items, s, probe_steps=10)
    tune_s = time.perf_counter() - t0
    ws = torch.empty(q.qaia_sample_batch_workspace_bytes(items, s), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q.qaia_sample_batch(items, s, workspace=ws)
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t0
    del ws
    t0 = time.perf_counter()
    for (p, c), it in zip(probs, items):
        # per-instance calls on the autotuned family (at its default tile)
        s1 = q.make_schedule(variant, precision=precision, steps=T, dt=0.5, seed=4444, path=it.path)
        q.qaia_sample(p, c, R, s1, spins=it.spins, obj=it.obj)
    torch.cuda.synchronize()
    single_s = time.perf_counter() - t0
    paths = {}
    dense_flops = sparse_flops = 0
    for (n, m, kind, sd), it in zip(specs, items):
        key = it.path if not it.tile else f"{it.path}/tile{it.tile}"
        paths[key] = paths.get(key, 0) + 1
        if it.path.startswith("dense"):
            dense_flops += 2 * m * n * n * W * R * T  # the stacked product, unpadded
        else:
            inst = wl.random_instance(n, m, kind, seed=sd)
            sparse_flops += fma_flops_per_replica_step(n, inst.num_edges) * W * R * T
    total = count * W * R * T
    return {"workload": f"{count} instances, N~U[42,1024], m~U{{3,4}}, class~U{{deg3,10%,50%}}, "
                        f"{W} weight vectors x {R} replicas x {T} steps, {variant} {precision}",
            "autotune_s": tune_s, "paths": paths, "estimated_s": float(est.sum()),
            "batched_graph_s": batch_s, "per_instance_s": single_s,
            "batched_replica_steps_per_s": total / batch_s, "per_instance_replica_steps_per_s": total / single_s,
            "algorithmic_flops": {"dense_matrix": dense_flops, "sparse_fma": sparse_flops},
            "batched_TFLOPs": (dense_flops + sparse_flops) / batch_s / 1e12,
            # the dense items' matrix work alone, against the FP32 matrix peak: a
            # lower bound on matrix-core use (the sparse items take part of the time)
            "dense_matrix_frac_of_fp32_mfma_peak": dense_flops / batch_s / 1e12 / 157.3}


def noise_form(q, wl, torch, recovery_budget_s=15.0):
    """Synthetic analogues of the paper's noise studies on 25-node instances
    whose exact fronts come from GPU enumeration (2^24 cuts): an Appendix-E
    three-objective instance (190 Das-Dennis vectors, the paper's alpha 0.15)
    and a four-objective instance with N(0,1) weights (220 vectors, alpha
    0.1).  Recovery (Fig. 3 analogue): batches of the vectors x 3000 replicas,
    each filtered into the archive, until every exact front vector has been
    sampled; plain SB (1000 steps, dt 0.5) against noise-injected SB (50
    steps, dt 1, Eq. 10) and uniform random spins, reporting the samples and
    seconds to full recall (or the recall at the budget).  Noise sweep
    (Appendix C analogue): one batch of the short schedule per noise
    amplitude, reporting recall and the hypervolume ratio to the exact front
    (reference point: the per-objective minimum cut)."""
    from paper_2604_26477_amd.protocols import run_budget
    cases = (("appendix_e_n25_m3", wl.appendix_e_instance(25, 0.5, seed=7000), wl.das_dennis_interior(3, 21), 0.15),
             ("gauss_n25_m4_p0.5", wl.random_instance(25, 4, "p0.5", seed=7001), wl.das_dennis_interior(4, 13), 0.1))
    out = {"workload": "25-node instances with exact fronts; batches of Das-Dennis vectors x 3000 replicas",
           "instances": []}
    for ci, (name, inst, weights, alpha) in enumerate(cases):
        prob = q.problem_from_instance(inst, 0)
        _, front, lo = q.exact_front(prob, with_min=True)
        hv_ref = q.qaia_hypervolume(front, lo)
        rec = {"name": name, "m": inst.m, "weight_vectors": len(weights), "paper_alpha": alpha,
               "front_size": int(front.shape[0]), "recovery": {}, "noise_sweep": []}
        # the paper's protocol samples in half precision: the noise-injected
        # runs again in binary16 (the generated kernel, two replicas per lane)
        runs = (("random", "random", 50, 1.0, 0.0, "fp32"), ("bsb_plain_T1000", "bsb", 1000, 0.5, 0.0, "fp32"),
                ("dsb_plain_T1000", "dsb", 1000, 0.5, 0.0, "fp32"), ("bsb_noise_T50", "bsb", 50, 1.0, alpha, "fp32"),
                ("dsb_noise_T50", "dsb", 50, 1.0, alpha, "fp32"),
                ("bsb_noise_T50_fp16", "bsb", 50, 1.0, alpha, "fp16"),
                ("dsb_noise_T50_fp16", "dsb", 50, 1.0, alpha, "fp16"))
        for ri, (label, method, steps, dt, a, prec) in enumerate(runs):
            r = run_budget(prob, method, recovery_budget_s, weights=weights, R=3000, steps=steps, dt=dt, alpha=a,
                           seed=7100 + 10 * ci + ri, target=front, precision=prec)
            h = r["history"]
            full = h[-1]["recall"] == 1.0
            rec["recovery"][label] = {"full_recall": full, "samples": h[-1]["samples"], "seconds": h[-1]["seconds"],
                                      "recall": h[-1]["recall"], "batches": r["batches"],
                                      "recall_after_first_batch": h[0]["recall"]}
            print(json.dumps({"noise_recovery": [name, label, rec["recovery"][label]]}), file=sys.stderr, flush=True)
        for ai, a in enumerate((0.0, 0.05, 0.1, 0.15, 0.2, 0.3, 0.5, 1.0)):
            for method in ("bsb", "dsb"):
                r = run_budget(prob, method, float("inf"), weights=weights, R=3000, steps=50, dt=1.0, alpha=a,
                               seed=7300 + 10 * ci + ai, max_batches=1, target=front)
                rec["noise_sweep"].append({"method": method, "alpha": a, "recall": r["history"][-1]["recall"],
                                           "hv_ratio": q.qaia_hypervolume(r["front"], lo) / hv_ref})
        out["instances"].append(rec)
        print(json.dumps({"noise_instance": rec}), file=sys.stderr, flush=True)
    return out


def table2_form(q, wl, torch, sizes=((25, 0.5), (25, 1.0), (100, 0.5), (100, 1.0), (200, 0.5), (200, 1.0))):
    """Budgeted protocol on correlated three-objective instances shaped like
    Appendix E: 190 Das-Dennis weight vectors x 3000 replicas per batch
    (570 000 candidates), noise amplitude 0.1, 50 steps (n = 25) or 1000 steps,
    5 s (n = 25) or 10 s budgets; random uniform spins as the sanity baseline.
    n = 25 is scored against the exact front by GPU enumeration (reference
    point: per-objective minimum cut); larger n against the composite front of
    all methods (reference point: minimum over all samples)."""
    from paper_2604_26477_amd.protocols import run_budget
    weights = wl.das_dennis_interior(3, 21)
    out = {"workload": "Appendix-E-shaped instances (A, B in [-25, 25], J1 = A + B, J2 = 0.2 A - 5 B, J3 "
                       "independent, Bernoulli mask); 190 Das-Dennis vectors x 3000 replicas per batch, "
                       "alpha 0.1, dt 1.0", "instances": []}
    # construction includes compiling the generated bSB and dSB kernels when
    # the graph qualifies for them (sparse enough: here n = 25 at density 0.5)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # release memory cached by earlier forms
    for idx, (n, d) in enumerate(sizes):
        inst = wl.appendix_e_instance(n, d, seed=5000 + idx)
        torch.cuda.synchronize()  # earlier work must not land in the construction time
        t0 = time.perf_counter()
        prob = q.problem_from_instance(inst, 0)
        torch.cuda.synchronize()
        create_s = time.perf_counter() - t0
        budget, T = (5.0, 50) if n <= 42 else (10.0, 1000)
        rec = {"n": n, "density": d, "edges": inst.num_edges, "budget_s": budget, "steps": T,
               "problem_create_s": create_s}
        runs = {}
        for mi, method in enumerate(("random", "bsb", "dsb")):
            runs[method] = run_budget(prob, method, budget, weights=weights, R=3000, steps=T, dt=1.0,
                                      alpha=0.1, seed=6000 + 10 * idx + mi)
        if n <= 30:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, ref_front, lo = q.exact_front(prob, with_min=True)
            rec["exact_front_seconds"] = time.perf_counter() - t0
            rec["reference"] = "exact front by enumeration of 2^%d cuts" % (n - 1)
        else:
            allf = np.concatenate([r["front"] for r in runs.values()])
            keep = q.pareto_front(torch.from_numpy(allf).cuda()).cpu().numpy()
            ref_front = allf[keep]
            lo = np.min(np.stack([r["min"] for r in runs.values()]), axis=0)
            rec["reference"] = "composite front of the three methods"
        ref_set = {tuple(v) for v in ref_front}
        hv_ref = q.qaia_hypervolume(ref_front, lo)
        rec["reference_front_size"] = len(ref_set)
        for method, r in runs.items():
            got = {tuple(v) for v in r["front"]}
            rec[method] = {"front_points": len(got & ref_set), "archive": len(got),
                           "hv_ratio": q.qaia_hypervolume(r["front"], lo) / hv_ref if hv_ref else None,
                           "batches": r["batches"], "samples": r["samples"], "seconds": r["seconds"]}
        out["instances"].append(rec)
        print(json.dumps({"table2_row": rec}), file=sys.stderr, flush=True)
    return out


def traffic_probe(q, wl, torch, kind="sparse"):
    """For counter collection.  sparse (sparse-dsb): one bSB (dSB) sampling
    launch of the benchmark workload.  dense: one 20-step dSB call of the precision workload
    per operand format (FP32, BF16, FP8).  Then, as the counters' calibration,
    one plain device copy of 1 GiB (1 GiB read, 1 GiB written)."""
    if kind == "dense":
        N, m, W, R = 2048, 3, 512, 8
        inst = wl.random_instance(N, m, "complete", seed=3000)
        prob = q.problem_from_instance(inst, 0)
        c = torch.from_numpy(wl.dirichlet_weights(W, m, 3002)).cuda()
        for prec in ("fp32", "bf16", "fp8"):
            s = q.make_schedule("dsb", precision=prec, steps=20, dt=0.5, seed=3003, path="dense_staged")
            spins, obj, ws = q.qaia_sample(prob, c, R, s)
            torch.cuda.synchronize()
    else:
        cfg = wl.WORKLOADS[WORKLOAD]
        inst = wl.workload_instance(WORKLOAD)
        prob = q.problem_from_instance(inst, 0)
        c = torch.from_numpy(wl.workload_weights(WORKLOAD)).cuda()
        variant = "dsb" if kind == "sparse-dsb" else "bsb"
        s = q.make_schedule(variant, steps=cfg["T"], dt=0.5, seed=cfg["seed"] + 3)
        spins, obj, ws = q.qaia_sample(prob, c, cfg["R"], s)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "traffic", "sample_rows": int(obj.shape[0]), "copy_bytes": 1 << 30}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--path", default="auto")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision and learned form measurements")
    ap.add_argument("--batch-form", action="store_true",
                    help="also measure the 64-instance ragged batch (takes minutes in FP32)")
    ap.add_argument("--only-form", choices=["precision", "learned", "batching", "table2", "peaks", "noise"],
                    help="run one form measurement alone and print its JSON (for profiling)")
    ap.add_argument("--precision-steps", type=int, default=1000,
                    help="SB steps of the precision form (shorter runs for counter collection)")
    ap.add_argument("--traffic-probe", nargs="?", const="sparse", choices=["sparse", "sparse-dsb", "dense"],
                    help="run one bSB (sparse) or dSB (sparse-dsb) sampling launch of the workload or 20 dSB steps of the "
                         "precision workload per operand format (dense), then one 1 GiB device copy, for "
                         "counter collection (rocprofv3 --pmc), then exit")
    ap.add_argument("--noise-form", action="store_true",
                    help="also run the noise studies (front recovery, noise sweep) on 25-node exact fronts")
    ap.add_argument("--table2-form", action="store_true",
                    help="also run the budgeted protocol on Appendix-E-shaped instances (about 2 minutes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sampler's work shards over weight vectors "
              "with one front merge, which is not implemented here (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_26477_amd as q
    import workloads as wl

    if args.traffic_probe:
        traffic_probe(q, wl, torch, args.traffic_probe)
        return
    if args.only_form:
        if args.only_form == "precision":
            res = precision_form(q, wl, torch, T=args.precision_steps)
        elif args.only_form == "peaks":
            res = measured_peaks(q, torch)
        elif args.only_form == "noise":
            res = noise_form(q, wl, torch)
        else:
            res = {"learned": learned_form, "batching": batch_form, "table2": table2_form}[args.only_form](q, wl, torch)
        print(json.dumps({"form": args.only_form, "result": res}), flush=True)
        return
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
    ref = np.zeros(inst.m, np.int64)

    from concurrent.futures import ThreadPoolExecutor
    host = ThreadPoolExecutor(max_workers=1)

    def hypervolume(front):
        t0 = time.perf_counter()
        hv = q.qaia_hypervolume(front, ref)  # the ctypes call releases the GIL
        return hv, (time.perf_counter() - t0) * 1e3

    # The front of step k is gathered on the device (qaia_gather_rows reads the
    # kept count from device memory) and copied to pinned host memory on a
    # second stream, so step k + 1's sampling is queued without a host round
    # trip; step k + 1's filter waits until those copies have read keep/nkeep.
    front_dev = torch.empty((2 * rows, inst.m), dtype=torch.int64, device=dev)
    host_cap = 1 << 16
    front_host = [torch.empty((host_cap, inst.m), dtype=torch.int64, pin_memory=True) for _ in range(2)]
    nkeep_host = [torch.empty(1, dtype=torch.int64, pin_memory=True) for _ in range(2)]
    copy_stream = torch.cuda.Stream()

    def step(record, slot, prev):
        """Queue sampling, filtering and the front copy of one batch (no host
        wait).  `prev` is the previous step's record, whose copies this
        step's filter must not overtake."""
        ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for k in ("bsb", "dsb", "filter")}
        for i, v in enumerate(variants):
            if record:
                ev[v][0].record(stream)
            q.qaia_sample(prob, c, R, scheds[v], spins=spins[i * rows:(i + 1) * rows],
                          obj=obj[i * rows:(i + 1) * rows], workspace=ws_s, stream=stream)
            if record:
                ev[v][1].record(stream)
        if prev is not None:
            stream.wait_event(prev["copied"])
        if record:
            ev["filter"][0].record(stream)
        q.qaia_pareto_filter(obj, keep_idx=keep, num_keep=nkeep, workspace=ws_f, stream=stream)
        if record:
            ev["filter"][1].record(stream)
        q.qaia_gather_rows(obj, keep, nkeep, front_dev, 2 * rows, stream=stream)
        filtered = torch.cuda.Event()
        filtered.record(stream)
        copy_stream.wait_event(filtered)
        with torch.cuda.stream(copy_stream):
            nkeep_host[slot].copy_(nkeep, non_blocking=True)
            front_host[slot].copy_(front_dev[:host_cap], non_blocking=True)
            copied = torch.cuda.Event()
            copied.record(copy_stream)
        return {"copied": copied, "slot": slot, "record": record, "ev": ev}

    def finish(rec):
        """Host side of a queued step: wait for its copies, hand the front to
        the hypervolume worker.  Returns (front size, hv future, times)."""
        rec["copied"].synchronize()
        P = int(nkeep_host[rec["slot"]][0])
        if P <= host_cap:
            front = front_host[rec["slot"]][:P].numpy().copy()
        else:
            front = front_dev[:P].cpu().numpy()
        fut = host.submit(hypervolume, front)
        times = {}
        if rec["record"]:
            for k, (e0, e1) in rec["ev"].items():
                times[f"{k}_ms"] = e0.elapsed_time(e1)
        return P, fut, times

    for i in range(args.warmup):
        finish(step(False, i & 1, None))[1].result()
    torch.cuda.synchronize()
    per, futs = [], []
    t0 = time.perf_counter()
    pending = None
    for k in range(args.steps):
        rec = step(True, k & 1, pending)
        if pending is not None:
            P, fut, times = finish(pending)
            futs.append(fut)
            per.append(times)
        pending = rec
    P, fut, times = finish(pending)
    futs.append(fut)
    per.append(times)
    hvs = [f.result() for f in futs]  # every step's hypervolume is inside the timed region
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    total_rs = 2 * rows * T
    hv = hvs[-1][0]
    for p_, (_, hv_ms) in zip(per, hvs):
        p_["hv_ms"] = hv_ms
    stage = {k: float(np.mean([p[k] for p in per])) for k in per[0]}

    # roofline of the dominant kernel: the generated sparse SB kernel, whose
    # launches (one bSB, one dSB per step) do the same algorithmic work each
    algo_flops_per_launch = algorithmic_flops_per_replica_step(inst.n, inst.num_edges) * rows * T
    performed_flops_per_launch = fma_flops_per_replica_step(inst.n, inst.num_edges) * rows * T
    # algorithmic HBM bytes of one launch: spins + cut vectors out, folded
    # coefficients, c0 and the step table in
    algo_bytes = rows * 8 * (prob.words + inst.m) + W * (4 * inst.num_edges + 8) + 4 * T
    avg_launch_ms = float(np.mean([stage[f"{v}_ms"] for v in variants]))
    achieved = algo_flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    instr = {v: valu_instructions_per_replica_step(inst, v) for v in variants}
    issue_rate = sum(instr[v] * rows * T for v in variants) / (sum(stage[f"{v}_ms"] for v in variants) * 1e-3) / 1e12
    fma_per_rs = fma_flops_per_replica_step(inst.n, inst.num_edges) // 2
    # every issue slot filled with two instructions (one each from two waves)
    dual_ceiling = {v: SIMDS * CLOCK_HZ / 4 * 2 * 64 / instr[v] for v in variants}
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
                   "path": args.path,
                   "pipelining": "step k+1 is queued before step k's front is read back (device-side gather, copy stream); the host hypervolume of step k overlaps the device work of step k+1"},
        "roofline": {"bound": "alu", "kernel": "qaia_sb_reg (bSB and dSB launches)",
                     "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": SB_REG_TRAFFIC_BYTES,
                     "traffic_unit": "bytes per launch (HBM, counters)", "algorithmic_bytes_per_launch": algo_bytes,
                     "avg_launch_ms": avg_launch_ms,
                     "algorithmic_flops_per_replica_step": algorithmic_flops_per_replica_step(inst.n, inst.num_edges),
                     "flops_per_launch": algo_flops_per_launch,
                     "performed_fma_flops": {
                         "per_replica_step": fma_flops_per_replica_step(inst.n, inst.num_edges),
                         "TFLOPs": performed_flops_per_launch / (avg_launch_ms * 1e-3) / 1e12,
                         "frac_of_datasheet_peak": performed_flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
                         / PEAK_FP32_VECTOR_TFLOPS,
                         "single_issue_fma_TFLOPs": PEAK_FP32_FMA_TFLOPS},
                     "issue": {"valu_instructions_per_replica_step": instr,
                               "fma_instructions_per_replica_step": fma_per_rs,
                               "achieved_Tinstr_per_s": issue_rate,
                               "dual_issue_ceiling_replica_steps_per_s": dual_ceiling,
                               "frac": {v: rows * T / (stage[f"{v}_ms"] * 1e-3) / dual_ceiling[v] for v in variants},
                               "model": "a SIMD issues one wave64 VALU instruction per 4 cycles, or two from "
                                        "two waves; the loop's 32-bit-encoded instructions (v_fmac_f32, "
                                        "v_cndmask_b32, bSB's wall compare) co-issue, its VOP3 ones (med3, "
                                        "copysign, dSB's |x| compare) mostly issue alone (SQ_ACTIVE_INST_VALU2); "
                                        "ceiling = two instructions "
                                        "in every slot: 1024 SIMDs x 2.4 GHz / 4 x 2 x 64 lanes / VALU "
                                        "instructions per replica-step"}},
        "stages_ms": stage,
        "sampling_replica_steps_per_s": {v: rows * T / (stage[f"{v}_ms"] * 1e-3) for v in variants},
        "front_size": P, "hypervolume": str(hv),
    }
    peaks = measured_peaks(q, torch)
    result["measured_peaks"] = peaks
    result["roofline"]["issue"]["measured_mix_Tinstr_per_s"] = peaks["valu_mix_Tinstr_per_s"]
    result["roofline"]["performed_fma_flops"]["measured_vop3_fma_loop_TFLOPs"] = peaks["fp32_fma_TFLOPs"]
    if not args.no_forms:
        result["forms"] = {"precision": precision_form(q, wl, torch)}
        for prec in ("fp32", "bf16", "fp8"):
            pf = result["forms"]["precision"][prec]
            pf["frac_of_measured_peak"] = pf["matrix_TFLOPs"] / peaks[f"{prec}_mfma_TFLOPs"]
        lf = learned_form(q, wl, torch)
        result["forms"]["learned"] = lf
        # the ragged 64-instance batch at a tenth of its 1500 steps (same
        # instances, plans, launch structure and per-step work), so the
        # default run reports the batched / per-instance ratio
        bs = batch_run(q, wl, torch, T=150)
        bs["speedup_batched_over_per_instance"] = bs["per_instance_s"] / bs["batched_graph_s"]
        result["forms"]["batching_t150"] = bs
        if args.batch_form:
            result["forms"]["batching"] = batch_form(q, wl, torch)
        if args.table2_form:
            result["forms"]["table2"] = table2_form(q, wl, torch)
        if args.noise_form:
            result["forms"]["noise"] = noise_form(q, wl, torch)
        dense = lf["complete512_m4"]["contenders"]
        sparse = lf["n42_m4"]["contenders"]
        result["time_to_ref_hypervolume"] = {
            "reference": "hypervolume of the plain FP32 uniform-Dirichlet loop at 10x its budget (seed 777); "
                         "medians over seeds 11, 12, 13",
            "chosen_form": "learned proposer + discrete SB on the BF16 matrix-core path (complete N=512, m=4)",
            "chosen_form_s": dense["learned_dsb_bf16"]["seconds_median"],
            "plain_fp32_s": dense["plain_fp32_bsb"]["seconds_median"],
            "speedup": (dense["plain_fp32_bsb"]["seconds_median"] / dense["learned_dsb_bf16"]["seconds_median"]
                        if dense["plain_fp32_bsb"]["seconds_median"] and dense["learned_dsb_bf16"]["seconds_median"]
                        else None),
            "complete512_m4_s": {k: v["seconds_median"] for k, v in dense.items()},
            "n42_m4_s": {k: v["seconds_median"] for k, v in sparse.items()},
            "n42_m4_rounds": {k: v["rounds_median"] for k, v in sparse.items()},
        }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(inst, c_host, R, T)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
