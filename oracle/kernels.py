"""Per-iteration quantities of the Burer-Monteiro augmented Lagrangian method.

Test infrastructure only (see the package docstring).  Convention (appendix,
exact line search):

    L(R; y, sigma) = <C, RR^T> + y^T (b - A(RR^T)) + sigma/2 ||b - A(RR^T)||^2

Each function is the plain definition written out with numpy / scipy.
"""

from __future__ import annotations

import numpy as np

from .problem import SDPProblem


# ---------------------------------------------------------------------------
# Linear algebra of the map (Section 3.3-3.4)
# ---------------------------------------------------------------------------

def spmm(prob: SDPProblem, ytil: np.ndarray | None, V: np.ndarray) -> np.ndarray:
    """(C - A*(ytil)) V, the sparse-times-tall-skinny product of eq. At.

    With ytil = None the product is C V.
    """
    S = prob.C if ytil is None else (prob.C - prob.A_adj(ytil)).tocsr()
    return S @ V


def constraint_map(prob: SDPProblem, U: np.ndarray, V: np.ndarray | None = None) -> np.ndarray:
    """A(U V^T) through the compressed outer product (Section 3.4)."""
    return prob.A_of(U, V)


# ---------------------------------------------------------------------------
# Lagrangian, gradient, multiplier estimate
# ---------------------------------------------------------------------------

def lagrangian(prob: SDPProblem, R: np.ndarray, y: np.ndarray, sigma: float) -> float:
    q0 = prob.b - prob.A_of(R)
    return prob.objective(R) + float(y @ q0) + 0.5 * sigma * float(q0 @ q0)


def multiplier_estimate(prob: SDPProblem, R: np.ndarray, y: np.ndarray, sigma: float) -> np.ndarray:
    """ytil = y + sigma (b - A(RR^T)): the first-order multiplier estimate, which is
    also the ALM dual update of Section 2.1 in this sign convention."""
    return y + sigma * (prob.b - prob.A_of(R))


def gradient(prob: SDPProblem, R: np.ndarray, y: np.ndarray, sigma: float) -> np.ndarray:
    """grad_R L = 2 C R - 2 A*(y) R + 2 sigma A*(A(RR^T) - b) R  (Section 2.1,
    in the appendix sign convention).  With per-block ranks, the gradient with
    respect to the free entries only (the others are held at zero)."""
    res = prob.A_of(R) - prob.b
    G = (2.0 * (prob.C @ R) - 2.0 * (prob.A_adj(y) @ R)
         + 2.0 * sigma * (prob.A_adj(res) @ R))
    mask = prob.rank_mask(R.shape[1])
    return G if mask is None else G * mask


# ---------------------------------------------------------------------------
# Exact line search (appendix A.2)
# ---------------------------------------------------------------------------

def linesearch_coeffs(prob: SDPProblem, R, D, y, sigma) -> dict:
    """Coefficients of  L(R + tau D) - L(R) = a1 tau^4 + a2 tau^3 + a3 tau^2 + a4 tau."""
    p1 = prob.objective(R, D) + prob.objective(D, R)          # <C, R D^T + D R^T>
    p2 = prob.objective(D, D)                                  # <C, D D^T>
    q0 = prob.b - prob.A_of(R)                                 # b - A(RR^T)
    q1 = prob.A_of(R, D) + prob.A_of(D, R)                     # A(R D^T + D R^T)
    q2 = prob.A_of(D, D)                                       # A(D D^T)
    lam_eff = y + sigma * q0                                   # lambda + rho q0
    a1 = 0.5 * sigma * float(q2 @ q2)
    a2 = sigma * float(q1 @ q2)
    a3 = p2 - float(lam_eff @ q2) + 0.5 * sigma * float(q1 @ q1)
    a4 = p1 - float(lam_eff @ q1)
    return dict(p1=p1, p2=p2, q0=q0, q1=q1, q2=q2, a1=a1, a2=a2, a3=a3, a4=a4)


def quartic(a, tau):
    a1, a2, a3, a4 = a
    return ((a1 * tau + a2) * tau + a3) * tau * tau + a4 * tau


def exact_step(a1: float, a2: float, a3: float, a4: float) -> float:
    """Step tau minimising the quartic over tau > 0.

    The stationary points solve 4 a1 t^3 + 3 a2 t^2 + 2 a3 t + a4 = 0.  All real
    roots are taken (numpy.roots, then two Newton polishing steps on the cubic);
    among the positive ones the one with the smallest quartic value is returned,
    the smaller tau on an exact tie.  Returns 0.0 when no positive root lowers
    the quartic (the direction is not a descent direction).
    """
    a = (a1, a2, a3, a4)
    coeffs = np.array([4.0 * a1, 3.0 * a2, 2.0 * a3, a4])
    nz = np.nonzero(coeffs)[0]
    if nz.size == 0 or nz[0] == 3:
        return 0.0
    roots = np.roots(coeffs[nz[0]:])
    cand = []
    for z in roots:
        if abs(z.imag) <= 1e-7 * max(1.0, abs(z.real)):
            t = float(z.real)
            for _ in range(2):
                f1 = ((4.0 * a1 * t + 3.0 * a2) * t + 2.0 * a3) * t + a4
                f2 = (12.0 * a1 * t + 6.0 * a2) * t + 2.0 * a3
                if f2 != 0.0:
                    t = t - f1 / f2
            if t > 0.0:
                cand.append(t)
    best, fbest = 0.0, 0.0
    for t in sorted(cand):
        ft = quartic(a, t)
        if ft < fbest:
            best, fbest = t, ft
    return best


# ---------------------------------------------------------------------------
# ALM measures (paper, experimental setting: err1, err2, err3)
# ---------------------------------------------------------------------------

def alm_measures(prob: SDPProblem, R: np.ndarray, y: np.ndarray) -> dict:
    """Objective, dual objective and the primal infeasibility / gap errors."""
    obj = prob.objective(R)
    res = prob.A_of(R) - prob.b
    res_norm = float(np.sqrt(res @ res))
    dual = float(prob.b @ y)
    err1 = res_norm / (1.0 + float(np.abs(prob.b).sum()))
    err1_inf = res_norm / (1.0 + float(np.abs(prob.b).max()))
    err3 = (obj - dual) / (1.0 + abs(obj) + abs(dual))
    return dict(obj=obj, dual=dual, res_norm=res_norm, err1=err1,
                err1_inf=err1_inf, err3=err3)
