"""Online loop of the learned weight proposer (form F3) and its uniform baseline.

Each round:
  1. draw candidate weight vectors c ~ Dirichlet(1, ..., 1) (device, seeded);
  2. learned: score them with the MLP on (c, eight front-gap features) and
     draw a share of n_sel of them without replacement with probabilities
     proportional to exp(score / temperature) (Gumbel top-k), and take the
     rest as fresh uniform draws; the network's share is (1 - explore) unless
     its picks have found new points significantly less often than the
     uniform picks over the last rounds, or the labels carry no contrast
     (network_trusted), and explore otherwise (the uniform Dirichlet
     fallback, which keeps measuring the network); baseline: n_sel uniform
     candidates;
  3. sample every kept vector with R replicas (qaia_sample);
  4. filter [archive ; new samples] (qaia_pareto_filter) and label each kept
     vector 1 iff it produced a vector that enters the front and was not in
     the archive (qaia_new_point_labels);
  5. learned: the (input row, label) pairs join a ring buffer of the last
     rounds, and a few Adam steps on minibatches (windows of random
     permutations of the buffer) minimise the mean binary cross-entropy;
  6. the new archive is the filtered set; its exact hypervolume (host) judges
     progress.
The driver only orchestrates library calls; tensors are device memory.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import (make_schedule, qaia_dirichlet_weights, qaia_front_features, qaia_gather_rows, qaia_hypervolume,
               qaia_mlp_forward, qaia_mlp_param_count, qaia_mlp_train, qaia_new_point_labels,
               qaia_pareto_filter, qaia_pareto_filter_workspace_bytes, qaia_sample,
               qaia_sample_workspace_bytes, qaia_topk)

HIDDEN = 128


def _init_params(D: int, rng: np.random.Generator) -> np.ndarray:
    """He-style initialisation, flat layout W1, b1, W2, b2, w3, b3."""
    parts = [rng.standard_normal(HIDDEN * D) * np.sqrt(2.0 / D), np.zeros(HIDDEN),
             rng.standard_normal(HIDDEN * HIDDEN) * np.sqrt(2.0 / HIDDEN), np.zeros(HIDDEN),
             rng.standard_normal(HIDDEN) * np.sqrt(1.0 / HIDDEN), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def _to_bf16_bits(a: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


class ProposerLoop:
    def __init__(self, prob, R=256, steps=2000, variant="bsb", n_cand=65536, n_sel=1024,
                 explore=0.1, lr=1e-3, learned=True, seed=0, archive_cap=1 << 20, ref=None,
                 precision="fp32", path="auto", temperature=1.0, replay_rounds=8, train_steps=16,
                 batch=1024, dt=0.5, noise_alpha=0.0, judge="each", feature_front=2048):
        if judge not in ("each", "record"):
            raise ValueError("judge must be 'each' (exact hypervolume every round) or 'record' (archive kept "
                             "per round, judged afterwards)")
        self.judge = judge
        self.feature_front = feature_front
        self.train_ws = None
        self.archives = []
        self.prob, self.m, self.R = prob, prob.m, R
        self.n_cand, self.n_sel, self.explore, self.lr = n_cand, n_sel, explore, lr
        self.learned = learned
        self.rng = np.random.Generator(np.random.PCG64(seed))
        self.sched_args = dict(variant=variant, precision=precision, steps=steps, dt=dt, noise_alpha=noise_alpha,
                               path=path)
        self.seed = seed
        self.dev = prob.torch_device
        self.ref = np.zeros(self.m, np.int64) if ref is None else np.asarray(ref, np.int64)
        self.D = self.m + 8
        dev = self.dev
        self.rows_new = n_sel * R
        self.cap = archive_cap
        self.pool_obj = torch.empty((archive_cap + self.rows_new, self.m), dtype=torch.int64, device=dev)
        self.pool_spins = torch.empty((archive_cap + self.rows_new, prob.words), dtype=torch.int64, device=dev)
        self.tmp_obj = torch.empty((archive_cap, self.m), dtype=torch.int64, device=dev)
        self.tmp_spins = torch.empty((archive_cap, prob.words), dtype=torch.int64, device=dev)
        self.A = 0
        self.keep = torch.empty(archive_cap + self.rows_new, dtype=torch.int64, device=dev)
        self.nkeep = torch.empty(1, dtype=torch.int64, device=dev)
        self.ws_filter = torch.empty(qaia_pareto_filter_workspace_bytes(archive_cap + self.rows_new, self.m),
                                     dtype=torch.uint8, device=dev)
        s0 = make_schedule(seed=0, **self.sched_args)
        self.ws_sample = torch.empty(qaia_sample_workspace_bytes(prob, n_sel, R, s0), dtype=torch.uint8,
                                     device=dev)
        npar = qaia_mlp_param_count(self.D)
        theta = _init_params(self.D, np.random.Generator(np.random.PCG64(seed + 17)))
        self.master = torch.from_numpy(theta).to(dev)
        self.params = torch.from_numpy(_to_bf16_bits(theta).view(np.int16)).to(dev)
        self.m1 = torch.zeros(npar, dtype=torch.float32, device=dev)
        self.m2 = torch.zeros(npar, dtype=torch.float32, device=dev)
        self.adam_step = 0
        self.temperature, self.train_steps, self.batch = temperature, train_steps, batch
        self.replay_cap = replay_rounds * n_sel
        self.replay_X = torch.zeros((self.replay_cap, self.D), dtype=torch.float32, device=dev)
        self.replay_y = torch.zeros(self.replay_cap, dtype=torch.float32, device=dev)
        self.replay_n = 0
        self.replay_slot = 0
        self.replay_zero = torch.zeros(self.replay_cap, dtype=torch.float32, device=dev)
        self.iota_sel = torch.arange(n_sel, dtype=torch.int64, device=dev)
        self.explore_idx = torch.arange(n_cand, n_cand + n_sel, dtype=torch.int64, device=dev)
        self.hits = torch.zeros((0, self.m), dtype=torch.float32, device=dev)
        self.misses = torch.zeros((0, self.m), dtype=torch.float32, device=dev)
        # per round: (network picks, their hits, uniform picks, their hits)
        self.arm_window = 8
        self.arms = []
        self.n_top_last = 0
        self.round_no = 0
        self.replica_offset = 0
        self.history = []

    # -------------------------------------------------------------- selection
    def _select(self):
        """Candidate weight vectors (device), the picked rows and the MLP inputs.

        Candidates are drawn on the device (uniform on the simplex).  Learned:
        n_cand candidates are scored and (1 - explore) n_sel of them drawn by
        Gumbel top-k; the exploration share are n_explore further fresh uniform
        draws (i.i.d. candidates, so equivalent to uniform picks among the rest).
        Uniform: n_sel fresh draws."""
        key = self.seed * 1000003 + self.round_no
        if not self.learned:
            cands = qaia_dirichlet_weights(self.m, self.n_sel, seed=key, device=self.dev)
            return cands, self.iota_sel, None
        minority = int(round(self.explore * self.n_sel))
        n_top = self.n_sel - minority if self.network_trusted() else minority
        n_exp = self.n_sel - n_top
        self.n_top_last = n_top
        cands = qaia_dirichlet_weights(self.m, self.n_cand + n_exp, seed=key, device=self.dev)
        front = self.pool_obj[: self.A]
        if self.A > self.feature_front:
            # the features see an evenly strided subset of at most feature_front
            # archive points (their cost grows with the archive)
            front = front[:: -(-self.A // self.feature_front)].contiguous()
        X = qaia_front_features(front, cands, self.hits, self.misses)
        scores = qaia_mlp_forward(self.params, self.D, X[: self.n_cand])
        top = qaia_topk(scores, n_top, temperature=self.temperature, seed=key)
        pick = torch.cat([top, self.explore_idx[:n_exp]])
        return cands, pick, X

    def network_trusted(self) -> bool:
        """Whether the network takes the larger share of the picks.  It does
        unless, over the last rounds, its picks found new non-dominated points
        significantly less often than the uniform picks (one-sided
        two-proportion z-test, z < -2), or the labels are saturated (more than
        98 % positive: nothing to learn when almost every weight vector finds
        a new point), in which case the uniform Dirichlet fallback takes the
        larger share and the network keeps the smaller one (which keeps
        measuring it).  Rare positives are not a reason to fall back: finding
        them is what the network is for."""
        n1 = sum(a[0] for a in self.arms)
        h1 = sum(a[1] for a in self.arms)
        n2 = sum(a[2] for a in self.arms)
        h2 = sum(a[3] for a in self.arms)
        if n1 == 0 or n2 == 0:
            return True
        p = (h1 + h2) / (n1 + n2)
        if p == 0.0:
            return True
        if p > 0.98:
            return False
        se = (p * (1.0 - p) * (1.0 / n1 + 1.0 / n2)) ** 0.5
        return (h1 / n1 - h2 / n2) >= -2.0 * se

    # -------------------------------------------------------------- one round
    def round(self):
        t0 = time.perf_counter()
        m, R, dev = self.m, self.R, self.dev
        cands, pick, X = self._select()
        count = torch.tensor([self.n_sel], dtype=torch.int64, device=dev)
        w_sel = torch.empty((self.n_sel, m), dtype=torch.float32, device=dev)
        qaia_gather_rows(cands, pick, count, w_sel, self.n_sel)
        s = make_schedule(seed=self.seed, replica_offset=self.replica_offset, **self.sched_args)
        self.replica_offset += self.rows_new
        A = self.A
        qaia_sample(self.prob, w_sel, R, s, spins=self.pool_spins[A:A + self.rows_new],
                    obj=self.pool_obj[A:A + self.rows_new], workspace=self.ws_sample)
        M = A + self.rows_new
        qaia_pareto_filter(self.pool_obj[:M], keep_idx=self.keep, num_keep=self.nkeep, workspace=self.ws_filter)
        labels = qaia_new_point_labels(self.keep, self.nkeep, A, R, self.n_sel)
        qaia_gather_rows(self.pool_obj, self.keep, self.nkeep, self.tmp_obj, self.cap)
        qaia_gather_rows(self.pool_spins, self.keep, self.nkeep, self.tmp_spins, self.cap)
        P = int(self.nkeep.item())  # the round's one wait for the device
        if P > self.cap:
            raise RuntimeError("archive capacity exceeded")
        lab = labels.cpu().numpy() > 0.5  # ready: the wait above covered the labels
        self.pool_obj[:P].copy_(self.tmp_obj[:P])
        self.pool_spins[:P].copy_(self.tmp_spins[:P])
        front = self.pool_obj[:P].cpu().numpy()
        self.A = P
        if self.learned:
            nt = self.n_top_last
            self.arms.append((nt, int(lab[:nt].sum()), self.n_sel - nt, int(lab[nt:].sum())))
            self.arms = self.arms[-self.arm_window:]
            w_h = w_sel.cpu().numpy()
            self.hits = torch.from_numpy(np.ascontiguousarray(w_h[lab])).to(dev)
            self.misses = torch.from_numpy(np.ascontiguousarray(w_h[~lab])).to(dev)
            # this round's rows and labels enter the ring buffer
            lo = self.replay_slot * self.n_sel
            qaia_gather_rows(X, pick, count, self.replay_X[lo:lo + self.n_sel], self.n_sel)
            self.replay_y[lo:lo + self.n_sel].copy_(labels)
            self.replay_slot = (self.replay_slot + 1) % (self.replay_cap // self.n_sel)
            self.replay_n = min(self.replay_n + self.n_sel, self.replay_cap)
            # Adam steps on minibatches: consecutive windows of random
            # permutations of the ring buffer, one permutation per pass (a
            # single library call queues the whole loop; the host goes on)
            Rn = self.replay_n
            self.train_ws = qaia_mlp_train(self.master, self.params, self.m1, self.m2, self.D,
                                           self.replay_X[:Rn], self.replay_y[:Rn], self.batch, self.train_steps,
                                           self.adam_step + 1, lr=self.lr, seed=self.seed * 7919,
                                           workspace=self.train_ws)
            self.adam_step += self.train_steps
        new_points = int(lab.sum())
        if self.judge == "each":
            hv = qaia_hypervolume(front, self.ref)
        else:
            hv = None
            self.archives.append(front)
        self.round_no += 1
        rec = {"round": self.round_no, "front": P, "hv": hv, "hit_vectors": new_points,
               "seconds": time.perf_counter() - t0}
        self.history.append(rec)
        return rec

    def front(self):
        return self.pool_obj[: self.A].cpu().numpy()


def reference_run(prob, rounds: int, seed: int, **loop_kw):
    """The reference of a time-to-hypervolume race: the plain loop (uniform
    Dirichlet weight vectors) for `rounds` rounds; its final archive is the
    union of its rounds' fronts.  Returns (exact hypervolume, seconds)."""
    loop = ProposerLoop(prob, learned=False, seed=seed, judge="record", **loop_kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(rounds):
        loop.round()
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    return qaia_hypervolume(loop.archives[-1], loop.ref), seconds, loop.archives[-1].shape[0]


def time_to_hypervolume(loop: ProposerLoop, target_hv: int, max_rounds: int, max_seconds: float = float("inf")):
    """Rounds of `loop` (built with judge="record"), each round's end time and
    archive recorded, until max_rounds or max_seconds; then the judge: the
    first round whose archive's exact hypervolume reaches target_hv, found by
    bisection (the archive only grows in dominance, so its hypervolume never
    decreases).  The time to the target is that round's end plus the time of
    one exact hypervolume evaluation of its archive (the judge confirming it).
    To end early, the archive is also judged after rounds 1, 2, 4, 8, ...;
    those pauses are taken out of the recorded round times."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    paused = 0.0
    ends = []
    hv_at = {}

    def hv(k):
        if k not in hv_at:
            t1 = time.perf_counter()
            hv_at[k] = (qaia_hypervolume(loop.archives[k], loop.ref), time.perf_counter() - t1)
        return hv_at[k][0]
    for r in range(max_rounds):
        loop.round()
        ends.append(time.perf_counter() - t0 - paused)
        if ends[-1] >= max_seconds:
            break
        if (r + 1) & r == 0:  # r + 1 is a power of two
            t1 = time.perf_counter()
            reached = hv(r) >= target_hv
            paused += time.perf_counter() - t1
            if reached:
                break
    last = len(ends) - 1
    out = {"rounds_run": len(ends), "seconds_run": ends[-1], "final_hv": str(hv(last)),
           "final_front": int(loop.archives[last].shape[0])}
    if hv(last) < target_hv:
        out.update(reached=False, rounds=None, seconds=None)
        return out
    lo, hi = -1, last  # hv(lo) < target <= hv(hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if hv(mid) >= target_hv:
            hi = mid
        else:
            lo = mid
    out.update(reached=True, rounds=hi + 1, seconds=ends[hi] + hv_at[hi][1], judge_seconds=hv_at[hi][1])
    return out


def run_until(loop: ProposerLoop, target_hv: int, max_rounds: int, max_seconds: float = float("inf")):
    """Rounds until the archive's hypervolume reaches target_hv, or max_rounds
    rounds or max_seconds have passed; returns (rounds, seconds, reached)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(max_rounds):
        rec = loop.round()
        if rec["hv"] >= target_hv:
            return r + 1, time.perf_counter() - t0, True
        if time.perf_counter() - t0 >= max_seconds:
            return r + 1, time.perf_counter() - t0, False
    return max_rounds, time.perf_counter() - t0, False
