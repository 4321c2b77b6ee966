"""Float64 oracle of the learned weight proposer.  TEST INFRASTRUCTURE ONLY.

The paper has no learned component; this oracle states, as plainly as
possible, what the library's proposer kernels compute so that their
gradients and features can be checked:

* a multilayer perceptron D -> 128 -> 128 -> 1 with the exact-erf GELU
  activation, trained with the mean binary cross-entropy on logits and the
  Adam update (Kingma and Ba, 2015);
* eight "front-gap" features of a candidate weight vector w against the
  current non-dominated archive.

Parameter layout (a flat float vector, in this order): W1 [H][D], b1 [H],
W2 [H][H], b2 [H], w3 [H], b3 [1], with H = 128 and D = m + 8 (the weight
vector followed by the eight features).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

H = 128


def n_params(D: int, Hh: int = H) -> int:
    return Hh * D + Hh + Hh * Hh + Hh + Hh + 1


def unpack(theta: np.ndarray, D: int, Hh: int = H):
    o = 0
    W1 = theta[o:o + Hh * D].reshape(Hh, D); o += Hh * D
    b1 = theta[o:o + Hh]; o += Hh
    W2 = theta[o:o + Hh * Hh].reshape(Hh, Hh); o += Hh * Hh
    b2 = theta[o:o + Hh]; o += Hh
    w3 = theta[o:o + Hh]; o += Hh
    b3 = theta[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X, D):
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(theta, np.float64), D)
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    a1 = gelu(z1)
    z2 = a1 @ W2.T + b2
    a2 = gelu(z2)
    z3 = a2 @ w3 + b3[0]
    return z3, (X, z1, a1, z2, a2)


def bce_with_logits(z, y):
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(theta, X, y, D):
    """Gradient of the mean BCE loss with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(theta, np.float64), D)
    z3, (X, z1, a1, z2, a2) = forward(theta, X, D)
    B = X.shape[0]
    dz3 = (1.0 / (1.0 + np.exp(-z3)) - np.asarray(y, np.float64)) / B
    gw3 = a2.T @ dz3
    gb3 = np.array([dz3.sum()])
    dz2 = np.outer(dz3, w3) * gelu_grad(z2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, gb3])


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def _angle(a, b):
    na, nb = np.linalg.norm(a), np.linalg.norm(b)
    c = float(np.dot(a, b) / (na * nb))
    return math.acos(max(-1.0, min(1.0, c)))


def features(front: np.ndarray, cands: np.ndarray, hits: np.ndarray, misses: np.ndarray) -> np.ndarray:
    """Eight front-gap features per candidate (float64 [N, 8]).

    The archive front is normalised per objective to [0, 1] by its nadir
    (minimum) and ideal (maximum) point; an objective with zero range maps to
    1.  With v_j = w . y^_j over the front points j:
      f1 = max_j v_j, f2 = max - second largest, f3 = max - eighth largest
      (the smallest when fewer than eight points), f4 = Euclidean distance from
      the maximising point y^* (first index on ties) to its nearest other front
      point, f5 = fraction of front points within distance 0.05 of y^*
      (itself included), f6 / f7 = smallest angle between w and the previous
      round's weight vectors that did / did not find a new non-dominated point
      (pi/2 when there are none), f8 = max_k |w_k - 1/m|.
    An empty front gives f1..f5 = 0.
    """
    front = np.asarray(front, np.float64)
    cands = np.asarray(cands, np.float64)
    N, m = cands.shape
    out = np.zeros((N, 8))
    P = front.shape[0]
    if P:
        lo, hi = front.min(axis=0), front.max(axis=0)
        rng = hi - lo
        yh = np.where(rng > 0, (front - lo) / np.where(rng > 0, rng, 1.0), 1.0)
    for c in range(N):
        w = cands[c]
        if P:
            v = yh @ w
            order = np.argsort(-v, kind="stable")
            jstar = int(order[0])
            vmax = v[jstar]
            out[c, 0] = vmax
            out[c, 1] = vmax - v[order[1]] if P > 1 else 0.0
            out[c, 2] = vmax - v[order[min(7, P - 1)]]
            d = np.linalg.norm(yh - yh[jstar], axis=1)
            out[c, 3] = np.min(np.delete(d, jstar)) if P > 1 else 0.0
            out[c, 4] = np.count_nonzero(d <= 0.05) / P
        out[c, 5] = min((_angle(w, h) for h in hits), default=math.pi / 2)
        out[c, 6] = min((_angle(w, h) for h in misses), default=math.pi / 2)
        out[c, 7] = np.max(np.abs(w - 1.0 / m))
    return out
