"""CPU checks of the FP32 trajectory bound (tests/fp32_bounds.py) that the GPU
trajectory tests use as their tolerance.

An FP32 emulation of the sparse kernels' update order (fused multiply-adds,
coefficients rounded once, the device's Gaussian draw moved by up to its error
bound with random signs) must stay inside the bound on every seed, while the
bound stays small enough to catch a misplaced or mis-scaled noise term.
"""
import numpy as np
import pytest

import fp32_bounds as fb
import noise_model as nm
import oracle
import workloads as wl

NOISE_SEEDS = range(43, 60)


def _worst_case_eta(seed):
    rng = np.random.default_rng(seed)

    def perturb(eta, r, th):
        return eta + rng.choice([-1.0, 1.0], size=eta.shape) * fb.eta_error_bound(r, th)
    return perturb


def _noise_case():
    inst = wl.random_instance(12, 3, "deg3", seed=41, num_edges=16)
    c = wl.dirichlet_weights(6, 3, 42)
    return inst, c, 8, 1000, 50, 0.15


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_bound_contains_fp32_emulation_on_every_seed(variant):
    """Noise-injected SB (Eq. 10), the instance and schedule of the GPU trace
    test, every SB seed 43..59: the emulated FP32 run stays within the bound
    wherever the bound is defined, the bound is defined on nearly every step,
    and it stays far below the trajectory's scale (x is O(0.1 .. 1))."""
    inst, c, R, T, steps, alpha = _noise_case()
    checked, finals = [], []
    for seed in NOISE_SEEDS:
        b = fb.Bound(inst, c, R, T, variant, alpha=alpha, seed=seed, steps=steps)
        _, ref = oracle.sb_sample(inst, c, R, T, variant, dt=0.5, seed=seed, alpha=alpha, trace_steps=steps)
        emu = fb.emulate_fp32(inst, c, R, T, variant, alpha=alpha, seed=seed, steps=steps,
                              eta_perturb=_worst_case_eta(seed))
        ok, ratio, frac = b.check(emu, ref)
        assert ok, (seed, ratio)
        checked.append(frac)
        finals.append(np.median(b.err_x[:, -1].max(axis=1)))
    assert np.mean(checked) >= 0.95 and min(checked) >= 0.9, checked
    assert np.median(finals) <= 1e-3, finals


def test_bound_contains_fp32_emulation_degenerate_graphs():
    """A lone spin (c0 = 0) and two spins on one edge (c0 J(c) = 1, whose
    antisymmetric mode starts at zero stiffness and amplifies the rounding of
    the step coefficient), ballistic SB, 100 steps."""
    c = wl.dirichlet_weights(5, 2, 81)
    lone = wl.Instance(1, 2, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((2, 0), np.int32))
    w = (np.array([[5], [3]], np.int64) << 16).astype(np.int32)
    pair = wl.Instance(2, 2, np.array([0], np.int32), np.array([1], np.int32), w)
    for inst, R, seed in ((lone, 4, 82), (pair, 32, 84)):
        b = fb.Bound(inst, c, R, 1000, "bsb", seed=seed, steps=100)
        _, ref = oracle.sb_sample(inst, c, R, 1000, "bsb", dt=0.5, seed=seed, trace_steps=100)
        emu = fb.emulate_fp32(inst, c, R, 1000, "bsb", seed=seed, steps=100)
        ok, ratio, frac = b.check(emu, ref)
        assert ok and frac >= 0.9, (inst.n, ratio, frac)


@pytest.mark.parametrize("mistake", ["noise_twice", "noise_on_x", "eta_index"])
def test_bound_rejects_planted_mistakes(mistake):
    """The bound is a test, not a blanket: an FP32 run with the noise term
    mis-scaled (dt dropped, i.e. doubled at dt = 0.5), added to x, or drawn
    for the wrong spin leaves it within a few steps on every seed tried."""
    inst, c, R, T, steps, alpha = _noise_case()
    for seed in (43, 50, 59):
        b = fb.Bound(inst, c, R, T, "bsb", alpha=alpha, seed=seed, steps=steps)
        _, ref = oracle.sb_sample(inst, c, R, T, "bsb", dt=0.5, seed=seed, alpha=alpha, trace_steps=steps)
        if mistake == "noise_twice":
            emu = fb.emulate_fp32(inst, c, R, T, "bsb", alpha=2 * alpha, seed=seed, steps=steps)
        elif mistake == "eta_index":
            emu = fb.emulate_fp32(inst, c, R, T, "bsb", alpha=alpha, seed=seed, steps=steps,
                                  eta_perturb=lambda e, r, th: e[:, :, ::-1].copy())
        else:
            # noise in x: y without noise, then x += dt alpha eta on top of the update
            plain = fb.emulate_fp32(inst, c, R, T, "bsb", alpha=0.0, seed=seed, steps=1)
            emu = plain.copy()
            eta = np.array([[nm.noise(seed, nm.noise_counter(g, T, 0, inst.n, i))[0] for i in range(inst.n)]
                            for g in range(c.shape[0] * R)])
            emu[:, 0] = np.clip(plain[:, 0] + np.float32(0.5 * alpha) * eta, -1, 1)
            ok, _, _ = b.check(np.concatenate([emu, ref[:, 1:]], axis=1), ref)
            assert not ok
            continue
        ok, ratio, _ = b.check(emu, ref)
        assert not ok, (seed, ratio)
        first_bad = np.argmax(((np.abs(emu - ref) > b.err_x * 1.000001 + 1e-12).any(axis=2)
                               & b.valid).any(axis=0))
        assert first_bad <= 3, first_bad


def test_eta_bound_covers_float32_box_muller():
    """The device draw in float32 (numpy's log, sqrt and cos, each correctly
    rounded or within an ulp) stays inside eta_error_bound on 20 000 draws."""
    worst = 0.0
    for idx in range(20000):
        bits = nm.splitmix64(7 ^ nm.NOISE_KEY, idx)
        eta, r, th = nm.box_muller(bits)
        u1 = np.float32(((bits >> 40) + 1) * 2.0 ** -24)
        u2 = np.float32((bits & 0xFFFFFF) * 2.0 ** -24)
        rf = np.sqrt(np.float32(-2.0) * np.log(u1))
        cf = np.cos(np.float32(6.2831853071795864769) * u2)
        ef = float(np.float32(rf * cf))
        bound = fb.eta_error_bound(r, th)
        assert abs(ef - eta) <= bound, (idx, ef, eta, bound)
        if r > 0:
            worst = max(worst, abs(ef - eta) / bound)
    assert worst > 0.05  # the bound is not loose by orders of magnitude


@pytest.mark.parametrize("variant,alpha", [("bsb", 0.0), ("dsb", 0.0), ("bsb", 0.15)])
def test_bound_contains_fp16_emulation(variant, alpha):
    """The same bound at the binary16 unit roundoff (u = 2^-11, rounded
    start) contains the binary16 emulation of the half-precision form on
    seeds 43..49 over 30 steps; where it is defined the ratio stays well
    below 1."""
    inst = wl.random_instance(12, 3, "deg3", seed=41, num_edges=16)
    c = wl.dirichlet_weights(6, 3, 42)
    worst, checked = 0.0, []
    for seed in range(43, 50):
        b = fb.Bound(inst, c, 8, 1000, variant, alpha=alpha, seed=seed, steps=30, u=fb.U16, rounded_start=True)
        _, ref = oracle.sb_sample(inst, c, 8, 1000, variant, dt=0.5, seed=seed, alpha=alpha, trace_steps=30)
        emu = fb.emulate_fp16(inst, c, 8, 1000, variant, alpha=alpha, seed=seed, steps=30)
        ok, ratio, frac = b.check(emu.astype(np.float64), ref)
        assert ok, (seed, ratio)
        worst = max(worst, ratio)
        checked.append(frac)
    assert worst < 0.8 and np.mean(checked) > 0.1, (worst, checked)
