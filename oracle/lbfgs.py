"""L-BFGS search direction (paper Algorithm 1; H0 = I, or a given H0).

Test infrastructure only (see the package docstring).
"""

from __future__ import annotations

import numpy as np


def _dot(a, b):
    return float(np.sum(a * b))


def two_loop(G: np.ndarray, pairs, h0=None) -> np.ndarray:
    """Direction from the gradient G and the stored pairs (s_t, y_t), oldest first.

    Starts from D = -G; the first loop runs from the newest pair to the oldest,
    alpha_t = beta_t <s_t, D>, D -= alpha_t y_t; then D <- H0 D (Algorithm 1 has
    H0 = I; `h0` is a callable applying another H0); the second loop runs from
    the oldest to the newest, D += (alpha_t - beta_t <y_t, D>) s_t, with
    beta_t = 1/<y_t, s_t>.
    """
    D = -G.copy()
    alpha = [0.0] * len(pairs)
    beta = [1.0 / _dot(yt, st) for (st, yt) in pairs]
    for t in range(len(pairs) - 1, -1, -1):
        st, yt = pairs[t]
        alpha[t] = beta[t] * _dot(st, D)
        D = D - alpha[t] * yt
    if h0 is not None:
        D = h0(D)
    for t in range(len(pairs)):
        st, yt = pairs[t]
        D = D + (alpha[t] - beta[t] * _dot(yt, D)) * st
    return D


def accept_pair(s: np.ndarray, yv: np.ndarray) -> bool:
    """Curvature guard: keep the pair only if <y, s> > 1e-12 ||y|| ||s||."""
    ys = _dot(yv, s)
    return ys > 1e-12 * np.sqrt(_dot(yv, yv) * _dot(s, s))
