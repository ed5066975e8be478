"""Warm-start model: per-node features and a 16-64-64-2 tanh MLP, in float64.

Test infrastructure only (see the package docstring).  The paper has no warm
start; this is the reference for the project's own extension: a per-node MLP
that predicts the MaxCut multipliers y0 (through t_i = -4 y_i / sum_j |w_ij|)
and a log-scale for the initial penalty.  Every piece is the plain definition:
features from explicit per-node neighbour loops over the weighted graph, the
forward pass as matrix products, the backward pass by the chain rule, Adam as
published (Kingma & Ba, 2015).
"""

from __future__ import annotations

import numpy as np

NF, H, NO = 16, 64, 2
SHAPES = [("W1", (H, NF)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (NO, H)), ("b3", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[k:k + size].reshape(shape)
        k += size
    return out


def init_params(seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = 1.0 / np.sqrt(shape[1])
            parts.append(rng.uniform(-lim, lim, shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts)


def features(n: int, u, v, w=None) -> np.ndarray:
    """16 features per node of the weighted graph (edges u-v with weights w).

    With d_i the degree, s_i = sum_j w_ij, a_i = sum_j |w_ij|, l_i = log(1 + d_i),
    b_i = s_i / max(a_i, 1) and dbar = 2|E|/n:
      0 l_i              1 b_i                 2 log(1 + a_i)
      3 mean_j l_j       4 std_j l_j           5 mean_j w_ij b_j
      6 mean_j 1/(1+d_j) 7 log(1 + d_i/dbar)   8 1/(1 + d_i)
      9 a_i/max(d_i,1)  10 mean_j w_ij         11 log(n)/20
     12 log(1 + dbar)   13 max_j l_j - l_i     14 mean_j d_j/(d_i+d_j)   15 1
    (neighbour statistics are 0 for isolated nodes).
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.ones(len(u)) if w is None else np.asarray(w, dtype=np.float64)
    nbrs = [[] for _ in range(n)]
    for a, b, ww in zip(u.tolist(), v.tolist(), w.tolist()):
        nbrs[a].append((b, ww))
        nbrs[b].append((a, ww))
    d = np.array([len(x) for x in nbrs], dtype=np.float64)
    s = np.array([sum(ww for _, ww in x) for x in nbrs])
    a = np.array([sum(abs(ww) for _, ww in x) for x in nbrs])
    l = np.log1p(d)
    bal = s / np.maximum(a, 1.0)
    dbar = 2.0 * len(u) / n
    F = np.zeros((n, NF))
    for i in range(n):
        F[i, 0] = l[i]
        F[i, 1] = bal[i]
        F[i, 2] = np.log1p(a[i])
        F[i, 7] = np.log1p(d[i] / dbar) if dbar > 0 else 0.0
        F[i, 8] = 1.0 / (1.0 + d[i])
        F[i, 9] = a[i] / max(d[i], 1.0)
        F[i, 11] = np.log(n) / 20.0
        F[i, 12] = np.log1p(dbar)
        F[i, 15] = 1.0
        if nbrs[i]:
            js = np.array([j for j, _ in nbrs[i]])
            ws = np.array([ww for _, ww in nbrs[i]])
            F[i, 3] = l[js].mean()
            F[i, 4] = np.sqrt(max(np.mean(l[js] ** 2) - F[i, 3] ** 2, 0.0))
            F[i, 5] = np.mean(ws * bal[js])
            F[i, 6] = np.mean(1.0 / (1.0 + d[js]))
            F[i, 10] = ws.mean()
            F[i, 13] = l[js].max() - l[i]
            F[i, 14] = np.mean(d[js] / (d[i] + d[js]))
    return F


def forward(theta: np.ndarray, X: np.ndarray):
    P = unpack(theta)
    h1 = np.tanh(X @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    out = h2 @ P["W3"].T + P["b3"]
    return out, (h1, h2)


def loss(theta, X, T):
    """Mean over nodes of the squared error of both outputs."""
    out, _ = forward(theta, X)
    return float(np.sum((out - T) ** 2) / X.shape[0])


def backward(theta: np.ndarray, X: np.ndarray, G_out: np.ndarray) -> np.ndarray:
    """Gradient of sum_i <G_out_i, out_i> with respect to the parameters."""
    P = unpack(theta)
    _, (h1, h2) = forward(theta, X)
    dW3 = G_out.T @ h2
    db3 = G_out.sum(axis=0)
    gz2 = (G_out @ P["W3"]) * (1.0 - h2 * h2)
    dW2 = gz2.T @ h1
    db2 = gz2.sum(axis=0)
    gz1 = (gz2 @ P["W2"]) * (1.0 - h1 * h1)
    dW1 = gz1.T @ X
    db1 = gz1.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])


def loss_grad(theta, X, T):
    out, _ = forward(theta, X)
    G = 2.0 * (out - T) / X.shape[0]
    return backward(theta, X, G)


def adam(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def multipliers_from_output(out: np.ndarray, absdeg: np.ndarray) -> np.ndarray:
    """y0_i = -t_i sum_j |w_ij| / 4 from the first output, t_i = out_i0 limited to
    [-2, 2]: at an optimum y*_i = -sum_j w_ij (1 - X*_ij) / 4 with |X*_ij| <= 1, so
    |t_i| <= 2 for every exact label."""
    return -0.25 * np.clip(out[:, 0], -2.0, 2.0) * absdeg


def initial_penalty(out: np.ndarray, sigma_default: float, log_lo: float, log_hi: float) -> float:
    """sigma0 = sigma_default exp(s / 2) with s the mean second output limited to
    [log_lo, log_hi] (the range of the training labels): the output predicts
    log(final penalty / default) of a cold solve, and the warm start begins at
    the geometric mean of the default and that final penalty."""
    return sigma_default * float(np.exp(0.5 * np.clip(out[:, 1].mean(), log_lo, log_hi)))


def sigma_label(sigma_final: float, sigma_default: float) -> float:
    """Penalty label of a cold solve: log(sigma_final / sigma_default)."""
    return float(np.log(sigma_final / sigma_default))


def to_bfloat16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even) and
    return them widened back to float64: keep the top 16 bits of the float32
    pattern after adding 0x7fff plus the lowest kept bit."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def targets_from_solution(y: np.ndarray, absdeg: np.ndarray) -> np.ndarray:
    """t_i = -4 y_i / sum_j |w_ij| (0 for isolated nodes)."""
    return np.where(absdeg > 0, -4.0 * y / np.maximum(absdeg, 1e-300), 0.0)
