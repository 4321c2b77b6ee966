"""Sampling-filtering under a wall-clock budget (section "Comparison to
evolutionary algorithm-based heuristics"): a sampler is called repeatedly on a
fixed set of weight vectors, every batch is filtered together with the running
non-dominated archive, and the archive is returned when the budget is spent.

Samplers: noise-injected ballistic or discrete SB (Eq. 10) through qaia_sample,
and the random-sampling sanity baseline (uniform spins through
qaia_random_spins + qaia_evaluate).  The archive holds objective vectors only.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import (make_schedule, qaia_evaluate, qaia_gather_rows, qaia_objective_min, qaia_pareto_filter,
               qaia_pareto_filter_workspace_bytes, qaia_random_spins, qaia_sample, qaia_sample_workspace_bytes)


def run_budget(prob, method: str, budget_s: float, weights=None, R: int = 3000, steps: int = 50,
               dt: float = 1.0, alpha: float = 0.1, seed: int = 0, path: str = "auto",
               precision: str = "fp32", archive_cap: int = 1 << 20, max_batches: int | None = None,
               target=None):
    """Sampling-filtering rounds until budget_s seconds of wall time have passed.

    method: "random", "bsb" or "dsb".  SB methods sample every weight vector
    (float32 [W, m], host or device) with R replicas per batch; the random
    baseline draws W * R uniform configurations per batch.  Returns a dict
    with the archive (host int64 [P, m]), the per-objective minimum over all
    samples, the batch and sample counts and the elapsed seconds.

    max_batches stops after that many batches.  target (host int64 [F, m], a
    known Pareto front) adds the recall after every batch (the fraction of
    target vectors in the archive; a front vector, once sampled, is never
    dominated, so it stays) to "history", and stops at full recall."""
    dev = prob.torch_device
    m = prob.m
    if weights is None:
        raise ValueError("weights are required (they also size the random baseline's batches)")
    c = torch.as_tensor(np.ascontiguousarray(weights, np.float32)).to(dev)
    rows = c.shape[0] * R
    pool = torch.empty((archive_cap + rows, m), dtype=torch.int64, device=dev)
    front = torch.empty((archive_cap + rows, m), dtype=torch.int64, device=dev)
    spins = torch.empty((rows, prob.words), dtype=torch.int64, device=dev)
    keep = torch.empty(archive_cap + rows, dtype=torch.int64, device=dev)
    nkeep = torch.empty(1, dtype=torch.int64, device=dev)
    ws_f = torch.empty(qaia_pareto_filter_workspace_bytes(archive_cap + rows, m), dtype=torch.uint8, device=dev)
    ws_s = None
    if method in ("bsb", "dsb"):
        s0 = make_schedule(method, precision=precision, steps=steps, dt=dt, noise_alpha=alpha, seed=seed,
                           path=path)
        ws_s = torch.empty(qaia_sample_workspace_bytes(prob, c.shape[0], R, s0), dtype=torch.uint8, device=dev)
    elif method != "random":
        raise ValueError(method)
    A = 0
    lo = torch.empty(m, dtype=torch.int64, device=dev)
    batches = 0
    tset = {tuple(int(v) for v in r) for r in np.asarray(target)} if target is not None else None
    history = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        new = pool[A:A + rows]
        if method == "random":
            qaia_random_spins(prob.n, rows, seed, offset=batches * rows, spins=spins, device=dev)
            qaia_evaluate(prob, spins, obj=new)
        else:
            s = make_schedule(method, precision=precision, steps=steps, dt=dt, noise_alpha=alpha, seed=seed,
                              replica_offset=batches * rows, path=path)
            qaia_sample(prob, c, R, s, spins=spins, obj=new, workspace=ws_s)
        qaia_objective_min(new, out=lo, accumulate=batches > 0)
        qaia_pareto_filter(pool[:A + rows], keep_idx=keep, num_keep=nkeep, workspace=ws_f)
        P = int(nkeep.item())
        if P > archive_cap:
            raise RuntimeError("archive capacity exceeded")
        qaia_gather_rows(pool, keep, nkeep, front, P)
        pool[:P] = front[:P]
        A = P
        batches += 1
        if tset is not None:
            found = sum(1 for r in pool[:A].cpu().tolist() if tuple(r) in tset)
            history.append({"samples": batches * rows, "seconds": time.perf_counter() - t0,
                            "recall": found / max(len(tset), 1)})
            if found == len(tset):
                break
        if max_batches is not None and batches >= max_batches:
            break
        if time.perf_counter() - t0 >= budget_s:
            break
    elapsed = time.perf_counter() - t0
    out = {"front": pool[:A].cpu().numpy(), "min": lo.cpu().numpy(), "batches": batches,
           "samples": batches * rows, "seconds": elapsed}
    if tset is not None:
        out["history"] = history
    return out
