"""Burer-Monteiro ALM solve with L-BFGS and exact line search (paper Sections 2.1-2.2,
Algorithm 1, appendix A.2), and the splitting (ADMM) phase (Section 2.2, eqs. 2.2-2.3,
Algorithm 2).

Test infrastructure only (see the package docstring).

Where the paper defers to LoRADS/SDPLR for schedule details (initial multiplier,
penalty schedule, inner tolerance, memory length), the numbers below are this
project's own reading; the GPU library takes the same numbers from its own
options struct (the two share numbers, not code):

* y0 = 0; sigma0 = 4 ||vec(C)||_1 / m unless given;
* after each inner solve: y <- y + sigma (b - A(RR^T));
  sigma <- min(sigma_factor * sigma, sigma_max_ratio * sigma0) (sigma_factor = 4) when err1 did not
  fall below feas_decrease * (previous err1);
* inner L-BFGS stops when ||grad||_F <= eta_k * max(1, ||grad at its start||_F),
  eta_0 = eta0, eta_{k+1} = max(eta_factor * eta_k, eta_min);
* L-BFGS memory T = lbfgs_mem (default 1) pairs from consecutive iterations; a pair failing
  the curvature guard, or a direction that is not a descent direction, clears
  the memory (the next direction is -grad);
* stop when err1 <= tol and |err3| <= tol (the paper's mild re-opt criterion);
  with ``reopt`` >= 1 the paper's re-optimisation instead (Section 4.1, see
  ``reopt_solve``).
"""

from __future__ import annotations

import dataclasses
import time
from dataclasses import dataclass, field

import numpy as np

from . import kernels as K
from .certify import lambda_min
from .lbfgs import accept_pair, two_loop
from .problem import SDPProblem


@dataclass
class Options:
    tol: float = 1e-5
    lbfgs_mem: int = 1
    max_outer: int = 300
    max_inner: int = 1000
    max_iter_total: int = 200000
    sigma0: float = 0.0            # 0 selects 4 ||vec(C)||_1 / m
    sigma_factor: float = 4.0
    sigma_max_ratio: float = 1e8
    feas_decrease: float = 0.25
    eta0: float = 1e-1
    eta_factor: float = 0.25
    eta_min: float = 1e-9
    time_limit: float = 1e30
    phase2: bool = False           # switch to the splitting phase (Section 2.2)
    rank_max: int = 0              # dynamic rank (appendix A.1); 0 or <= rank: off
    rank_trigger: int = 1000       # L-BFGS iterations of a subproblem that trigger growth
    rank_scale: float = 1e-2       # standard deviation of the new entries
    rank_seed: int = 15049
    precond: int = 0               # MaxCut: row-block H0 for the L-BFGS direction (not in the paper):
                                   # 1 static h, 2 h from the diagonal of C - Diag(ytil)
    switch_err1: float = 1e-3      # ... once err1 <= switch_err1 after an ALM step
    admm_check: int = 10
    max_admm: int = 5000
    reopt: int = 0                 # re-optimisation (Section 4.1): 0 off, 1 mild, 2 strict
    reopt_factor: float = 0.1      # objective scale applied per round
    max_reopt: int = 10            # rounds after the first at most


@dataclass
class SolveResult:
    R: np.ndarray
    y: np.ndarray
    sigma: float
    obj: float
    dual: float
    err1: float
    err1_inf: float
    err3: float
    outer: int
    inner: int
    converged: bool
    seconds: float
    history: list = field(default_factory=list)
    admm_iters: int = 0
    admm_fallbacks: int = 0
    rank_final: int = 0
    reopt_rounds: int = 0
    err2: float = float("nan")
    eta: float = 0.0               # inner tolerance factor of the last subproblem


def default_sigma0(prob: SDPProblem) -> float:
    return max(4.0 * prob.c_l1 / prob.m, 1e-8)


_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64_at(seed: int, j: np.ndarray) -> np.ndarray:
    """Output j (from 0) of the SplitMix64 sequence seeded with `seed` (Steele,
    Lea and Flood, 2014): mix(seed + (j+1) gamma), arithmetic modulo 2^64."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(j, dtype=np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def new_columns(n: int, c0: int, c1: int, seed: int) -> np.ndarray:
    """N(0, 1) entries for columns c0..c1-1 of an n-row factor: entry (i, c) takes
    outputs 2k and 2k+1, k = 65536 i + c, as uniforms ((x >> 11) + 0.5) 2^-53,
    then Box-Muller sqrt(-2 ln u0) cos(2 pi u1)."""
    i = np.arange(n, dtype=np.uint64)[:, None]
    c = np.arange(c0, c1, dtype=np.uint64)[None, :]
    k = i * np.uint64(65536) + c
    u0 = ((splitmix64_at(seed, np.uint64(2) * k) >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    u1 = ((splitmix64_at(seed, np.uint64(2) * k + np.uint64(1)) >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)


def row_block_h0(prob: SDPProblem, R: np.ndarray, sigma: float, y=None, mode: int = 1):
    """H0 = P^{-1} with P block diagonal over rows, P_i = h_i I + 4 sigma R_i R_i^T,
    h_i = 2 max(sum_j |C_ij|, 1e-3 ||vec(C)||_1 / n) (mode 1), or (mode 2, with
    the multipliers y) h_i = 2 max(C_ii - ytil_i, 0.005 h_i of mode 1) where
    ytil = y + sigma (1 - ||R_i||^2) is the multiplier estimate at R.

    An extension, not in the paper (Algorithm 1 uses H0 = I).  For MaxCut the
    Hessian of the Lagrangian in row i has the penalty block 4 sigma R_i R_i^T
    (constraint i involves row i only) next to a part of the size of row i of
    C; P models both.  Applied per row by Sherman-Morrison:
    P_i^{-1} q = (q - kappa_i (R_i . q) R_i) / h_i, kappa_i = 4 sigma / (h_i + 4 sigma ||R_i||^2).
    """
    rowabs = np.asarray(abs(prob.C).sum(axis=1)).ravel()
    h = 2.0 * np.maximum(rowabs, 1e-3 * prob.c_l1 / prob.n)
    rr = np.sum(R * R, axis=1)
    if mode == 2:
        ytil = y + sigma * (1.0 - rr)
        h = 2.0 * np.maximum(np.asarray(prob.C.diagonal()).ravel() - ytil, 0.005 * h)
    kappa = 4.0 * sigma / (h + 4.0 * sigma * rr)

    def apply(Q):
        return (Q - (kappa * np.sum(R * Q, axis=1))[:, None] * R) / h[:, None]
    return apply


def lbfgs_minimize(prob: SDPProblem, R, y, sigma, eta, opts: Options, budget: int, floor: float = 1.0):
    """Minimise L(.; y, sigma) from R with Algorithm 1 and the exact step, until
    ||grad||_F <= eta max(floor, ||grad at R||_F) (floor: the objective's scale)."""
    G = K.gradient(prob, R, y, sigma)
    gnorm = float(np.sqrt(np.sum(G * G)))
    target = eta * max(floor, gnorm)
    pairs = []
    it = 0
    while it < min(opts.max_inner, budget):
        if gnorm <= target:
            break
        h0 = row_block_h0(prob, R, sigma, y, int(opts.precond)) if opts.precond else None
        D = two_loop(G, pairs, h0)
        c = K.linesearch_coeffs(prob, R, D, y, sigma)
        if not c["a4"] < 0.0:
            pairs = []
            D = -G if h0 is None else -h0(G)
            c = K.linesearch_coeffs(prob, R, D, y, sigma)
        tau = K.exact_step(c["a1"], c["a2"], c["a3"], c["a4"])
        it += 1
        if tau <= 0.0:
            break
        Rn = R + tau * D
        Gn = K.gradient(prob, Rn, y, sigma)
        s = tau * D
        yv = Gn - G
        if accept_pair(s, yv):
            pairs.append((s, yv))
            if len(pairs) > opts.lbfgs_mem:
                pairs.pop(0)
        else:
            pairs = []
        R, G = Rn, Gn
        gnorm = float(np.sqrt(np.sum(G * G)))
    return R, it, gnorm


def alm_solve(prob: SDPProblem, R0: np.ndarray, y0=None, opts: Options | None = None,
              log=None) -> SolveResult:
    opts = opts or Options()
    if opts.reopt:
        return reopt_solve(prob, R0, y0, opts, log)
    return _alm_run(prob, R0, y0, opts, log)


def _alm_run(prob: SDPProblem, R0: np.ndarray, y0, opts: Options, log=None, sigma=None, sigma_cap=None,
             err1_only=False, floor=1.0, eta=None) -> SolveResult:
    """One ALM run.  sigma / sigma_cap / eta: starting penalty, its cap and the
    starting inner tolerance factor (defaults from the options); floor: the
    inner stop's floor; err1_only: stop as soon as err1 <= tol (a
    re-optimisation round), otherwise when err1 <= tol and |err3| <= tol."""
    t0 = time.perf_counter()
    R = np.array(R0, dtype=np.float64, copy=True)
    mask = prob.rank_mask(R.shape[1])
    if mask is not None:      # per-block ranks: the entries past a block's rank start (and stay) at zero
        R *= mask
    y = np.zeros(prob.m) if y0 is None else np.array(y0, dtype=np.float64, copy=True)
    if sigma is None:
        sigma = opts.sigma0 if opts.sigma0 > 0 else default_sigma0(prob)
    if sigma_cap is None:
        sigma_cap = sigma * opts.sigma_max_ratio
    eta = opts.eta0 if eta is None else eta
    err1_prev = np.inf
    total = 0
    hist = []
    converged = False
    meas = K.alm_measures(prob, R, y)
    outer = 0
    phase2_on = opts.phase2
    admm_total = fallbacks = 0
    rank_cur = R.shape[1]
    rank_cap = min(max(opts.rank_max, rank_cur), int(np.floor(np.sqrt(2.0 * prob.m))))
    for outer in range(1, opts.max_outer + 1):
        R, it, gnorm = lbfgs_minimize(prob, R, y, sigma, eta, opts, opts.max_iter_total - total, floor)
        total += it
        y = K.multiplier_estimate(prob, R, y, sigma)
        meas = K.alm_measures(prob, R, y)
        rec = dict(outer=outer, inner=it, sigma=sigma, gnorm=gnorm, **meas)
        hist.append(rec)
        if log is not None:
            log(rec)
        if meas["err1"] <= opts.tol and (err1_only or abs(meas["err3"]) <= opts.tol):
            converged = True
            break
        # penalty and inner-tolerance schedule, from the measures after the
        # multiplier step
        sigma_sub = sigma
        if meas["err1"] > opts.feas_decrease * err1_prev:
            sigma = min(sigma * opts.sigma_factor, sigma_cap)
        err1_prev = meas["err1"]
        eta = max(eta * opts.eta_factor, opts.eta_min)
        if rank_cur < rank_cap and it >= opts.rank_trigger:
            # dynamic rank (appendix A.1): rank <- min(ceil(1.5 rank), cap), new
            # columns rank_scale * N(0, 1) from the seeded generator; the new
            # columns move err1, so the penalty rule restarts its reference
            r_new = min(rank_cap, (3 * rank_cur + 1) // 2)
            R = np.hstack([R, opts.rank_scale * new_columns(prob.n, rank_cur, r_new, opts.rank_seed)])
            mask = prob.rank_mask(r_new)
            if mask is not None:
                R *= mask
            rank_cur = r_new
            meas = K.alm_measures(prob, R, y)
            hist.append(dict(outer=outer, rank=rank_cur, **meas))
            err1_prev = np.inf
        if phase2_on and meas["err1"] <= opts.switch_err1:
            # Splitting phase with the penalty of the subproblem just solved.  If it
            # diverges or stops at max_admm unconverged, the ALM goes on from the
            # point of the switch with the splitting phase off (the paper leaves
            # this case open).
            Rm, _, _, y2, meas2, it2, diverged = admm_phase(
                prob, R, y, sigma_sub, tol=opts.tol, max_iter=opts.max_admm, check_every=opts.admm_check,
                diverge_factor=10.0, err1_only=err1_only)
            admm_total += it2
            hist.append(dict(outer=outer, admm=it2, sigma=sigma_sub, diverged=diverged, **meas2))
            if not diverged and meas2["err1"] <= opts.tol and (err1_only or abs(meas2["err3"]) <= opts.tol):
                R, y, meas = Rm, y2, meas2
                converged = True
                break
            phase2_on = False
            fallbacks += 1
        if total >= opts.max_iter_total or time.perf_counter() - t0 > opts.time_limit:
            break
    return SolveResult(R=R, y=y, sigma=sigma, obj=meas["obj"], dual=meas["dual"],
                       err1=meas["err1"], err1_inf=meas["err1_inf"], err3=meas["err3"],
                       outer=outer, inner=total, converged=converged,
                       seconds=time.perf_counter() - t0, history=hist,
                       admm_iters=admm_total, admm_fallbacks=fallbacks, rank_final=R.shape[1], eta=eta)


def scaled_objective(prob: SDPProblem, alpha: float) -> SDPProblem:
    """The same constraints with the objective matrix alpha C."""
    return dataclasses.replace(prob, C=(alpha * prob.C).tocsr())


def reopt_solve(prob: SDPProblem, R0: np.ndarray, y0=None, opts: Options | None = None,
                log=None) -> SolveResult:
    """Re-optimisation (Section 4.1).  A round stops once the primal
    infeasibility tolerance holds (err1 <= tol).  The final criteria are then
    evaluated on the original problem: |err3| <= tol (level 1), and also
    err2 <= tol (level 2).  While they fail, the next round solves the problem
    with the objective matrix scaled down by reopt_factor once more (factor^k C
    in round k), warm from the previous round's output: its R, its multipliers
    times reopt_factor (the multipliers of the scaled problem), its penalty, and
    its inner tolerance factor taken one schedule step further.  The floor of
    the inner stop is in the objective's units, so it scales with C (alpha in
    round k); the penalty rule's err1 reference restarts each round; the
    penalty cap stays that of the first round; only the first round may enter
    the splitting phase.  max_outer and max_iter_total bound all rounds
    together.  The result is stated for the original problem: objective,
    multipliers and penalty of the last round divided by its scale (the
    Lagrangian of alpha C with y and sigma is alpha times that of C with y/alpha
    and sigma/alpha)."""
    opts = opts or Options()
    t0 = time.perf_counter()
    sigma0 = opts.sigma0 if opts.sigma0 > 0 else default_sigma0(prob)
    sigma_cap = sigma0 * opts.sigma_max_ratio
    alpha = 1.0
    rounds = 0
    outer = inner = admm = fallbacks = 0
    hist = []
    err2 = float("nan")
    R, y, sigma, eta = R0, y0, sigma0, opts.eta0
    converged = False
    while True:
        ro = dataclasses.replace(opts, reopt=0, max_outer=opts.max_outer - outer,
                                 max_iter_total=opts.max_iter_total - inner,
                                 phase2=opts.phase2 and rounds == 0)
        res = _alm_run(scaled_objective(prob, alpha), R, y, ro, log, sigma=sigma, sigma_cap=sigma_cap,
                       err1_only=True, floor=alpha, eta=eta)
        outer += res.outer
        inner += res.inner
        admm += res.admm_iters
        fallbacks += res.admm_fallbacks
        hist.extend(dict(round=rounds, alpha=alpha, **h) for h in res.history)
        R, y, sigma = res.R, res.y, res.sigma
        eta = max(res.eta * opts.eta_factor, opts.eta_min)
        if not res.converged:
            break
        obj, dual = res.obj / alpha, res.dual / alpha
        err3 = (obj - dual) / (1.0 + abs(obj) + abs(dual))
        ok = abs(err3) <= opts.tol
        if ok and opts.reopt == 2:
            err2 = max(0.0, -lambda_min(prob, y / alpha)) / (1.0 + prob.c_l1)
            ok = err2 <= opts.tol
        hist.append(dict(round=rounds, alpha=alpha, err3_original=err3, err2=err2, met=ok))
        if ok:
            converged = True
            break
        if rounds >= opts.max_reopt or inner >= opts.max_iter_total or outer >= opts.max_outer:
            break
        rounds += 1
        alpha *= opts.reopt_factor
        y = opts.reopt_factor * y
    meas = K.alm_measures(prob, R, y / alpha)
    return SolveResult(R=R, y=y / alpha, sigma=sigma / alpha, obj=meas["obj"], dual=meas["dual"],
                       err1=meas["err1"], err1_inf=meas["err1_inf"], err3=meas["err3"],
                       outer=outer, inner=inner, converged=converged,
                       seconds=time.perf_counter() - t0, history=hist,
                       admm_iters=admm, admm_fallbacks=fallbacks, rank_final=R.shape[1],
                       reopt_rounds=rounds, err2=err2, eta=eta)


# ---------------------------------------------------------------------------
# Splitting (ADMM) phase, Section 2.2 (LoRADS): X = U V^T with the penalty
# sigma/2 ||U - V||^2, in the appendix sign convention
#   L(U, V, y) = <C, U V^T> + y^T (b - A(U V^T)) + sigma/2 ||b - A(U V^T)||^2
#                + sigma/2 ||U - V||^2.
# ---------------------------------------------------------------------------

def split_operator(prob: SDPProblem, V: np.ndarray, sigma: float):
    """The positive definite map of eq. 2.2 for the U-step: U -> sigma A*(A(U V^T)) V + sigma U."""
    def apply(U):
        return sigma * (prob.A_adj(prob.A_of(U, V)) @ V) + sigma * U
    return apply


def split_rhs(prob: SDPProblem, V: np.ndarray, y: np.ndarray, sigma: float) -> np.ndarray:
    """Right-hand side of eq. 2.2 for the U-step: -C V + A*(y) V + sigma A*(b) V + sigma V."""
    return -(prob.C @ V) + prob.A_adj(y) @ V + sigma * (prob.A_adj(prob.b) @ V) + sigma * V


def cg(apply, B, X0, eps, K):
    """Conjugate gradients (Algorithm 2, no preconditioner) for apply(X) = B."""
    X = X0.copy()
    r = B - apply(X)
    if np.sqrt(np.sum(r * r)) <= eps:
        return X, 0
    p = r.copy()
    rr = float(np.sum(r * r))
    for k in range(K):
        Q = apply(p)
        alpha = rr / float(np.sum(p * Q))
        X = X + alpha * p
        r = r - alpha * Q
        rr_new = float(np.sum(r * r))
        if np.sqrt(rr_new) <= eps:
            return X, k + 1
        p = r + (rr_new / rr) * p
        rr = rr_new
    return X, K


def admm_step(prob: SDPProblem, U, V, y, sigma, cg_tol=1e-12, cg_iters=1000):
    """One splitting iteration: U-step and V-step by CG on eq. 2.2, then the
    multiplier step y <- y + sigma (b - A(U V^T))."""
    B = split_rhs(prob, V, y, sigma)
    U, _ = cg(split_operator(prob, V, sigma), B, U, cg_tol * max(1.0, np.linalg.norm(B)), cg_iters)
    B = split_rhs(prob, U, y, sigma)
    V, _ = cg(split_operator(prob, U, sigma), B, V, cg_tol * max(1.0, np.linalg.norm(B)), cg_iters)
    y = y + sigma * (prob.b - prob.A_of(U, V))
    return U, V, y


def admm_phase(prob: SDPProblem, R, y, sigma, tol=1e-5, max_iter=2000, check_every=10, log=None,
               diverge_factor=None, err1_only=False):
    """Run splitting iterations from U = V = R until err1 and |err3| at
    R = (U + V)/2 are below tol (checked every `check_every` iterations; err1
    alone with err1_only).
    With diverge_factor, stop early (diverged = True) when a check finds a
    non-finite value or err1 above diverge_factor times its value at R."""
    U, V = R.copy(), R.copy()
    meas = K.alm_measures(prob, R, y)
    err1_0 = meas["err1"]
    it = 0
    diverged = False
    with np.errstate(all="ignore"):
        for it in range(1, max_iter + 1):
            U, V, y = admm_step(prob, U, V, y, sigma)
            if it % check_every == 0 or it == max_iter:
                Rm = 0.5 * (U + V)
                meas = K.alm_measures(prob, Rm, y)
                if log is not None:
                    log(dict(it=it, **meas))
                if diverge_factor is not None and (not np.isfinite(meas["obj"]) or not np.isfinite(meas["err1"])
                                                   or meas["err1"] > diverge_factor * err1_0):
                    diverged = True
                    break
                if meas["err1"] <= tol and (err1_only or abs(meas["err3"]) <= tol):
                    break
    if diverge_factor is None:
        return 0.5 * (U + V), U, V, y, meas, it
    return 0.5 * (U + V), U, V, y, meas, it, diverged
