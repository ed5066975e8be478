"""Pins of the oracle's L-BFGS direction (Algorithm 1).

* On a strictly convex quadratic with exact line search, L-BFGS with H0 = I and
  any memory T >= 1 produces the conjugate-gradient iterates (Nocedal & Wright,
  Thm. on L-BFGS/CG equivalence for quadratics).
* The two-loop matrix H satisfies the secant condition H y_k = s_k for the newest
  pair, and H is symmetric positive definite when every <y_t, s_t> > 0.
"""

import numpy as np
import pytest

from oracle.lbfgs import two_loop


def spd(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(np.linspace(1.0, 30.0, n)) @ Q.T, rng.standard_normal(n)


def cg_iterates(A, b, x0, k):
    x = x0.copy()
    r = b - A @ x
    p = r.copy()
    out = [x.copy()]
    for _ in range(k):
        Ap = A @ p
        alpha = (r @ r) / (p @ Ap)
        x = x + alpha * p
        rn = r - alpha * Ap
        p = rn + (rn @ rn) / (r @ r) * p
        r = rn
        out.append(x.copy())
    return out


@pytest.mark.parametrize("T", [1, 2, 4])
def test_lbfgs_equals_cg_on_quadratic(T):
    A, b = spd(30, 11)
    x = np.zeros(30)
    grad = lambda z: A @ z - b
    ref = cg_iterates(A, b, x, 12)
    pairs = []
    g = grad(x)
    for k in range(12):
        d = two_loop(g, pairs)
        tau = -(g @ d) / (d @ A @ d)           # exact step on the quadratic
        xn = x + tau * d
        gn = grad(xn)
        pairs.append((tau * d, gn - g))
        if len(pairs) > T:
            pairs.pop(0)
        x, g = xn, gn
        assert np.allclose(x, ref[k + 1], rtol=1e-9, atol=1e-9)


def test_secant_condition_and_spd():
    rng = np.random.default_rng(3)
    n = 15
    A, _ = spd(n, 4)
    pairs = []
    for _ in range(4):
        s = rng.standard_normal(n)
        pairs.append((s, A @ s))
    s_new, y_new = pairs[-1]
    # two_loop returns -H g; the secant condition gives H y_new = s_new
    assert np.allclose(-two_loop(y_new, pairs), s_new, rtol=1e-10, atol=1e-10)
    H = np.stack([-two_loop(e, pairs) for e in np.eye(n)], axis=1)
    assert np.allclose(H, H.T, atol=1e-10)
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0


def test_empty_memory_is_steepest_descent():
    g = np.arange(6.0)
    assert np.array_equal(two_loop(g, []), -g)
