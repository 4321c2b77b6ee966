"""First-order bounds on how far an FP32 simulated-bifurcation trajectory can
drift from the float64 one, and a plain FP32 emulation of the update to check
those bounds on the CPU.

Why a bound instead of one tolerance: once spins start to bifurcate, SB
amplifies every rounding difference (the trajectory is chaotic), so how far
an FP32 run strays from float64 after k steps depends on the seed.  The bound
below follows the float64 trajectory and carries, spin by spin, the largest
absolute difference that FP32 arithmetic in any evaluation order could have
produced so far, to first order in the unit roundoff u = 2^-24:

* local errors of one step, in y:  K_i u S_i  +  dt alpha B_eta, where
  S_i = |y_i| + |k_t x_i| + sum_j sum_k |dt c0 c_k W_k,ij phi_j| + |dt alpha eta_i|
  bounds every partial sum of the force (any order, per-objective or folded
  coefficients), K_i = deg_i + m + 6 counts the roundings that can touch it
  (each coupling term, the per-objective reduction, the step coefficient, the
  folded coefficient roundings, the noise term, the final add), and B_eta is
  the error of the device's float32 Gaussian draw (eta_error_bound);
  in x:  u (|x_new| + |dt a0 y_new|);
* propagation: an error made at step s reaches step t through the product
  of the update's Jacobians (y' = y + (k_t I - dt c0 J(c) Dphi) x,
  x' = x + dt a0 y'; Dphi = I for ballistic SB, 0 for discrete SB, whose
  coupling sees exact +-1); the bound at step t is sum_s |P(t, s)| l_s, the
  absolute value taken elementwise after the product, so the linearised
  dynamics keep their oscillation and only the rounding signs are unknown;
* the wall and the sign are decisions: where the float64 value is farther
  from the threshold than the bound, both sides decide alike (a clamped spin
  then carries no error: x = +-1 and y = 0 on both sides); where it is not,
  the two runs may part for good, and the comparison of that replica stops
  there (through that step for the wall, which moves x continuously; before
  it for the discrete sign, which decides the step's force).

The float64 recursion here restates Eq. (9)/(10) only to evaluate the bound
along the trajectory; the tests compare the device trace with the oracle's
trace, and assert that this recursion reproduces the oracle to 1e-12.
"""
from __future__ import annotations

import math

import numpy as np

import noise_model as nm

U32 = 2.0 ** -24
U16 = 2.0 ** -11  # IEEE binary16 (the half-precision form)


def eta_error_bound(r: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Largest |eta_f32 - eta| of the device draw sqrtf(-2 logf u1) * cosf(2pi_f u2)
    against the exact r cos(theta), first order in u:

      r:     logf within 1 ulp (relative 2^-23), -2x exact, sqrtf correctly
             rounded: |dr| <= r 2^-23;
      theta: 2pi rounded to float32 and one product rounding: |dtheta| <= theta 2^-23;
      cos:   within 2 ulp of the result (absolute 2^-23), plus |dtheta|;
      product rounding: |eta| 2^-24 <= r 2^-24;
    total r 2^-24 (2 + 2 + 2 theta + 1).  One more unit of margin for the
    library routines' ulp claims gives r 2^-24 (6 + 2 theta)."""
    return U32 * r * (6.0 + 2.0 * theta)


def _csr(inst):
    n = inst.n
    nbr = [[] for _ in range(n)]
    for e in range(inst.num_edges):
        u, v = int(inst.edge_u[e]), int(inst.edge_v[e])
        nbr[u].append((v, e))
        nbr[v].append((u, e))
    return [sorted(a) for a in nbr]


def _draws(seed, g0, rows, T, steps, n):
    """eta, r, theta [rows, steps, n] of the noise stream."""
    eta = np.empty((rows, steps, n))
    r = np.empty_like(eta)
    th = np.empty_like(eta)
    for row in range(rows):
        g = g0 + row
        for t in range(steps):
            for i in range(n):
                eta[row, t, i], r[row, t, i], th[row, t, i] = nm.noise(seed, nm.noise_counter(g, T, t, n, i))
    return eta, r, th


def _init(seed, g0, rows, n, amp):
    """x0, y0 [rows, n]: float32(amp * (2u - 1)), u the top 24 bits of the draw."""
    out = np.empty((2, rows, n))
    a32 = np.float32(amp)
    for row in range(rows):
        g = g0 + row
        for i in range(n):
            for comp in (0, 1):
                bits = nm.splitmix64(seed, ((g * n + i) << 1) | comp)
                v = np.float32(2.0 * ((bits >> 40) * 2.0 ** -24) - 1.0)
                out[comp, row, i] = float(np.float32(a32 * v))
    return out[0], out[1]


def _scalarise(inst, c):
    """J(c)_e = sum_k c_k W_k,e 2^-frac (float64), c0 per the row-sum rule and
    the per-edge sum_k |c_k W_k,e| 2^-frac."""
    scale = 2.0 ** -inst.frac_bits
    W = inst.weights.astype(np.float64) * scale
    cd = c.astype(np.float64)
    jc = cd @ W                                   # [nw, E]
    jabs = np.abs(cd) @ np.abs(W)                 # [nw, E]
    n = inst.n
    row = np.zeros((c.shape[0], n))
    rowabs = np.zeros((c.shape[0], n))
    for e in range(inst.num_edges):
        for node in (inst.edge_u[e], inst.edge_v[e]):
            row[:, node] += jc[:, e]
            rowabs[:, node] += np.abs(jc[:, e])
    mx = np.abs(row).max(axis=1) if n else np.zeros(c.shape[0])
    mxa = rowabs.max(axis=1) if n else np.zeros(c.shape[0])
    c0 = np.where(mx > 0, 1.0 / np.where(mx > 0, mx, 1), np.where(mxa > 0, 1.0 / np.where(mxa > 0, mxa, 1), 0.0))
    return jc, jabs, c0


class Bound:
    """The float64 trajectory and its first-order FP32 error bound.

    x_ref  [rows, steps, n]  float64 x after each step
    err_x  [rows, steps, n]  bound on |x_fp32 - x_ref|
    valid  [rows, steps]     True where the comparison is defined

    The bound is sum_s |P(t, s)| l_s: l_s holds the local error bounds of
    step s (x and y), P(t, s) is the tangent propagator that carries an
    error made at step s to step t (the product of the update's Jacobians,
    the wall zeroing clamped rows), and |.| is taken elementwise only at the
    end, so the oscillation of the linearised dynamics is kept and only the
    unknown signs of the roundings are bounded.
    """

    def __init__(self, inst, c, R, T, variant="bsb", dt=0.5, a0=1.0, amp=0.1, alpha=0.0, seed=0,
                 steps=100, replica_offset=0, u=U32, rounded_start=False):
        """u: the unit roundoff of the arithmetic (U32, or U16 for the binary16
        form, whose values also take the float32 coefficients rounded once
        more, within the same K u S term); rounded_start: x0 and y0 are the
        float32 draws rounded to that precision (an initial error u |x0|,
        u |y0| carried like the others)."""
        n, m = inst.n, inst.m
        nw = c.shape[0]
        rows = nw * R
        nbr = _csr(inst)
        jc, jabs, c0 = _scalarise(inst, np.asarray(c, np.float32))
        x, y = _init(seed, replica_offset, rows, n, amp)
        if alpha != 0.0:
            eta, r, th = _draws(seed, replica_offset, rows, T, steps, n)
            beta = eta_error_bound(r, th)
        self.x_ref = np.zeros((rows, steps, n))
        self.err_x = np.zeros((rows, steps, n))
        self.valid = np.zeros((rows, steps), bool)
        alive = np.ones(rows, bool)
        wrow = np.arange(rows) // R
        dtc0 = dt * c0[wrow]                       # [rows]
        deg = np.array([len(a) for a in nbr])
        K = deg + m + 6
        # dense coupling c0 J(c) per row, for the Jacobian
        Jd = np.zeros((rows, n, n))
        for i in range(n):
            for j, e in nbr[i]:
                Jd[:, i, j] = c0[wrow] * jc[wrow, e]
        eye = np.eye(n)
        # propagators of the local errors made so far: [rows, s, 2n, 2n]
        P = np.zeros((rows, 0, 2 * n, 2 * n))
        L = np.zeros((rows, 0, 2 * n))
        if rounded_start:
            P = np.broadcast_to(np.eye(2 * n), (rows, 1, 2 * n, 2 * n)).copy()
            L = (u * np.concatenate([np.abs(x), np.abs(y)], axis=1))[:, None, :]
        ex_post = np.matmul(np.abs(P), L[..., None])[..., 0].sum(axis=1)[:, :n] if rounded_start \
            else np.zeros((rows, n))
        for t in range(steps):
            at = a0 * t / (T - 1) if T > 1 else 0.0
            kt = -dt * (a0 - at)
            if variant == "dsb":
                phi = np.where(x >= 0, 1.0, -1.0)
                # a spin whose x is within its bound of 0 may take the other sign
                alive &= ~(np.abs(x) <= ex_post).any(axis=1)
                dphi = np.zeros((rows, n, n))
            else:
                phi = x
                dphi = Jd
            f = np.einsum("rij,rj->ri", Jd, phi)
            fa = np.zeros((rows, n))
            for i in range(n):
                for j, e in nbr[i]:
                    fa[:, i] += jabs[wrow, e] * np.abs(phi[:, j])
            S = np.abs(y) + np.abs(kt * x) + dtc0[:, None] * fa
            ly = K[None, :] * u * S
            force = -(a0 - at) * x - f
            if alpha != 0.0:
                force = force + alpha * eta[:, t, :]
                ly = ly + dt * alpha * (beta[:, t, :] + u * np.abs(eta[:, t, :]))
            y = y + dt * force
            xn = x + dt * a0 * y
            lx = u * (np.abs(xn) + np.abs(dt * a0 * y))
            # Jacobian of the step before the wall: y' = y + (kt I - dt J Dphi) x,
            # x' = x + dt a0 y'
            dydx = kt * eye[None] - dt * dphi
            A = np.zeros((rows, 2 * n, 2 * n))
            A[:, n:, :n] = dydx
            A[:, n:, n:] = eye
            A[:, :n, :n] = eye + dt * a0 * dydx
            A[:, :n, n:] = dt * a0 * eye
            # injection of this step's local errors: (dx, dy) -> (dx + dt a0 dy, dy)
            B = np.zeros((rows, 1, 2 * n, 2 * n))
            B[:, 0, :n, :n] = eye
            B[:, 0, :n, n:] = dt * a0 * eye
            B[:, 0, n:, n:] = eye
            P = np.concatenate([np.matmul(A[:, None], P), B], axis=1)
            L = np.concatenate([L, np.concatenate([lx, ly], axis=1)[:, None, :]], axis=1)
            e_pre = np.matmul(np.abs(P), L[..., None])[..., 0].sum(axis=1)
            ex_pre = e_pre[:, :n]
            ax = np.abs(xn)
            clamp = ax > 1.0
            unsure_wall = np.abs(ax - 1.0) <= ex_pre
            sure = clamp & ~unsure_wall
            keep = np.concatenate([~sure, ~sure], axis=1).astype(np.float64)   # rows of x and y
            P = P * keep[:, None, :, None]
            x = np.where(clamp, np.sign(xn), xn)
            y = np.where(clamp, 0.0, y)
            ex_post = np.matmul(np.abs(P), L[..., None])[..., 0].sum(axis=1)[:, :n]
            self.x_ref[:, t] = x
            self.err_x[:, t] = np.maximum(ex_post, np.where(unsure_wall, ex_pre, 0.0))
            self.valid[:, t] = alive
            alive &= ~unsure_wall.any(axis=1)

    def check(self, x_dev: np.ndarray, x_oracle: np.ndarray, slack: float = 1e-12):
        """(ok, worst ratio |x_dev - x_oracle| / bound over valid entries, checked fraction)."""
        assert np.abs(self.x_ref - x_oracle).max() <= 1e-12, "bound recursion departs from the oracle"
        d = np.abs(x_dev.astype(np.float64) - x_oracle)
        lim = self.err_x * (1.0 + 1e-6) + slack
        v = self.valid[:, :, None]
        ok = bool(((d <= lim) | ~v).all())
        ratio = float(np.where(v, d / lim, 0.0).max())
        return ok, ratio, float(self.valid.mean())


def fma32(a, b, c):
    """float32 fused multiply-add: a*b is exact in float64, one rounding of the
    sum to float64 and one to float32 (double rounding is rarer than 2^-28 and
    moves the result by one float32 ulp at most)."""
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(np.float32)


def emulate_fp32(inst, c, R, T, variant="bsb", dt=0.5, a0=1.0, amp=0.1, alpha=0.0, seed=0, steps=100,
                 replica_offset=0, eta_perturb=None):
    """The sparse kernels' FP32 update order: y_i <- fma(k_t, x_i, y_i), then
    fma(-dt c0 J(c)_e, phi_j, y_i) per neighbour in increasing order, then
    fma(fl(dt alpha), eta_i, y_i); x_i <- fma(dt a0, y_i, x_i); the wall.  k_t
    and the folded coefficients are rounded once from float64.  eta is the
    float64 draw rounded to float32, moved by eta_perturb(eta, r, theta) if
    given (to model the device's draw).  Returns the x trace [rows, steps, n]."""
    n = inst.n
    nw = c.shape[0]
    rows = nw * R
    nbr = _csr(inst)
    jc, _, c0 = _scalarise(inst, np.asarray(c, np.float32))
    x0, y0 = _init(seed, replica_offset, rows, n, amp)
    X = x0.astype(np.float32) + np.float32(0.0)
    Y = y0.astype(np.float32)
    wrow = np.arange(rows) // R
    jf = (-dt * c0[:, None] * jc).astype(np.float32)     # [nw, E]
    dta0 = np.float32(dt * a0)
    dtal = np.float32(np.float32(dt) * np.float32(alpha))
    if alpha != 0.0:
        eta, r, th = _draws(seed, replica_offset, rows, T, steps, n)
        e64 = eta if eta_perturb is None else eta_perturb(eta, r, th)
        eta32 = e64.astype(np.float32)
    out = np.zeros((rows, steps, n), np.float32)
    for t in range(steps):
        at = a0 * t / (T - 1) if T > 1 else 0.0
        kt = np.float32(-dt * (a0 - at))
        phi = np.where(X >= 0, np.float32(1), np.float32(-1)) if variant == "dsb" else X
        Yn = Y.copy()
        for i in range(n):
            acc = fma32(kt, X[:, i], Y[:, i])
            for j, e in nbr[i]:
                acc = fma32(jf[wrow, e], phi[:, j], acc)
            if alpha != 0.0:
                acc = fma32(dtal, eta32[:, t, i], acc)
            Yn[:, i] = acc
        Y = Yn
        X = fma32(dta0, Y, X)
        clamp = np.abs(X) > 1
        Y = np.where(clamp, np.float32(0), Y)
        X = np.clip(X, -1, 1).astype(np.float32)
        out[:, t] = X
    return out


def fma16(a, b, c):
    """binary16 fused multiply-add: a*b + c formed exactly in float64 (the
    product of two binary16 values has at most 22 significant bits and the
    exponents of binary16 span 40 binary places, so the sum is exact), then
    rounded once to binary16."""
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(np.float16)


def emulate_fp16(inst, c, R, T, variant="bsb", dt=0.5, a0=1.0, amp=0.1, alpha=0.0, seed=0, steps=100,
                 replica_offset=0):
    """The binary16 form's update order (QAIA_FP16): the FP32 form's values
    (x0, y0, k_t, the folded coefficients, dt a0, dt alpha, the noise draw)
    rounded to binary16, every update a binary16 fused multiply-add in the
    FP32 form's order, the wall on binary16 values.  Returns the x trace."""
    n = inst.n
    nw = c.shape[0]
    rows = nw * R
    nbr = _csr(inst)
    jc, _, c0 = _scalarise(inst, np.asarray(c, np.float32))
    x0, y0 = _init(seed, replica_offset, rows, n, amp)
    X = x0.astype(np.float16) + np.float16(0.0)
    Y = y0.astype(np.float16)
    wrow = np.arange(rows) // R
    jf = (-dt * c0[:, None] * jc).astype(np.float32).astype(np.float16)
    dta0 = np.float16(np.float32(dt * a0))
    dtal = np.float16(np.float32(np.float32(dt) * np.float32(alpha)))
    if alpha != 0.0:
        eta, _, _ = _draws(seed, replica_offset, rows, T, steps, n)
        eta16 = eta.astype(np.float32).astype(np.float16)
    out = np.zeros((rows, steps, n), np.float16)
    for t in range(steps):
        at = a0 * t / (T - 1) if T > 1 else 0.0
        kt = np.float16(np.float32(-dt * (a0 - at)))
        phi = np.where(X >= 0, np.float16(1), np.float16(-1)) if variant == "dsb" else X
        Yn = Y.copy()
        for i in range(n):
            acc = fma16(kt, X[:, i], Y[:, i])
            for j, e in nbr[i]:
                acc = fma16(jf[wrow, e], phi[:, j], acc)
            if alpha != 0.0:
                acc = fma16(dtal, eta16[:, t, i], acc)
            Yn[:, i] = acc
        Y = Yn
        X = fma16(dta0, Y, X)
        clamp = np.abs(X) > 1
        Y = np.where(clamp, np.float16(0), Y)
        X = np.clip(X, -1, 1).astype(np.float16)
        out[:, t] = X
    return out
