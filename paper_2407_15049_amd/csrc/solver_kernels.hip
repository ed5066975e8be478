// Streaming and single-workgroup kernels of the device-resident ALM/L-BFGS loop.
//
// The L-BFGS memory (Algorithm 1) is kept as two rings of n x ld arrays: the
// last T+1 gradients G and the last T directions D.  Pair t of Algorithm 1 is
// s_t = tau_t D_t and y_t = G_{t+1} - G_t.  The Gram matrix of the ring slots
// is maintained incrementally (each sweep that writes a new G or D also takes
// its dot products with every slot), so the two-loop recursion of Algorithm 1
// runs on (2T+1)-vectors of coefficients in one thread; the new direction is
// then formed by one streaming pass D = sum_j coef_j basis_j.  This is the same
// recursion as Algorithm 1 (identical up to rounding) with two passes over the
// history per iteration instead of 2T dependent passes.
#include "device.h"
#include "kernels.h"

namespace lrsdp {

// ---------------------------------------------------------------------------
// Exact step of the quartic line search (appendix A.2), float64, one thread.
//
// f(t) = a1 t^4 + a2 t^3 + a3 t^2 + a4 t with a1 >= 0.  Local minima of f on
// t > 0 are the roots where f' = 4a1 t^3 + 3a2 t^2 + 2a3 t + a4 crosses from
// negative to positive, i.e. lie where f' is increasing: split (0, inf) at the
// roots of f'' (a quadratic), bracket each sign change of f' on an increasing
// piece and refine by safeguarded Newton/bisection.  Returns the minimiser with
// the smallest f (smaller t on a tie) if f < 0 there, else 0.
// ---------------------------------------------------------------------------
namespace {

struct Quartic {
    double a1, a2, a3, a4;
    __host__ __device__ double f(double t) const { return (((a1 * t + a2) * t + a3) * t + a4) * t; }
    __host__ __device__ double d1(double t) const { return ((4.0 * a1 * t + 3.0 * a2) * t + 2.0 * a3) * t + a4; }
    __host__ __device__ double d2(double t) const { return (12.0 * a1 * t + 6.0 * a2) * t + 2.0 * a3; }
};

// Root of f' in (lo, hi) with f'(lo) < 0 < f'(hi), f' increasing there.
__host__ __device__ double refine_root(const Quartic &q, double lo, double hi) {
    double t = 0.5 * (lo + hi);
    for (int it = 0; it < 300; ++it) {
        double v = q.d1(t);
        if (v == 0.0) return t;
        if (v < 0.0) lo = t; else hi = t;
        double d = q.d2(t);
        double tn = (d > 0.0) ? t - v / d : 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (hi - lo <= 4e-16 * fabs(hi)) return tn;
        if (tn == t) return t;
        t = tn;
    }
    return t;
}

// Smallest hi > lo with f'(hi) > 0 (f' -> +inf since a1 > 0 or a quadratic
// with positive leading term); doubling from a scale guess.
__host__ __device__ double bracket_up(const Quartic &q, double lo, double guess) {
    double hi = fmax(guess, lo > 0.0 ? 2.0 * lo : 1e-300);
    for (int it = 0; it < 2200 && !(q.d1(hi) > 0.0); ++it) hi *= 2.0;
    return hi;
}

__host__ __device__ double exact_step(double a1, double a2, double a3, double a4) {
    Quartic q{a1, a2, a3, a4};
    double cand[2];
    int nc = 0;
    double scale = 1.0;
    if (a3 != 0.0 && a4 != 0.0) scale = fabs(a4 / a3);
    if (a1 > 0.0 || (a1 == 0.0 && a2 > 0.0)) {
        // f' -> +inf.  Increasing pieces of f': where f'' >= 0.
        // f'' = 12 a1 t^2 + 6 a2 t + 2 a3 (or 6 a2 t + 2 a3 when a1 = 0)
        double tm = 0.0, tn = 0.0;  // f' increasing on (-inf, tm] and [tn, inf)
        bool two = false;
        if (a1 > 0.0) {
            double A = 12.0 * a1, B = 6.0 * a2, C = 2.0 * a3;
            double disc = B * B - 4.0 * A * C;
            if (disc > 0.0) {
                double sq = sqrt(disc);
                double qq = -0.5 * (B + (B >= 0.0 ? sq : -sq));
                double r1 = qq / A, r2 = (qq != 0.0) ? C / qq : -B / A;
                tm = fmin(r1, r2);
                tn = fmax(r1, r2);
                two = true;
            }
        } else {
            // f' = 3a2 t^2 + 2a3 t + a4 (a2 > 0): increasing on [-a3/(3a2), inf)
            tn = -a3 / (3.0 * a2);
            tm = -INFINITY;
            two = true;
        }
        if (!two) {
            if (q.d1(0.0) < 0.0) {
                double hi = bracket_up(q, 0.0, scale);
                cand[nc++] = refine_root(q, 0.0, hi);
            }
        } else {
            if (tm > 0.0 && q.d1(0.0) < 0.0 && q.d1(tm) > 0.0) cand[nc++] = refine_root(q, 0.0, tm);
            double s0 = fmax(0.0, tn);
            if (q.d1(s0) < 0.0) {
                double hi = bracket_up(q, s0, fmax(scale, 2.0 * s0));
                cand[nc++] = refine_root(q, s0, hi);
            }
        }
    } else if (a1 == 0.0 && a2 == 0.0) {
        if (a3 > 0.0 && a4 < 0.0) cand[nc++] = -a4 / (2.0 * a3);
    } else if (a1 == 0.0 && a2 < 0.0) {
        // f' = 3a2 t^2 + 2a3 t + a4 opens downward: increasing on (-inf, -a3/(3a2)]
        double tm = -a3 / (3.0 * a2);
        if (tm > 0.0 && q.d1(0.0) < 0.0 && q.d1(tm) > 0.0) cand[nc++] = refine_root(q, 0.0, tm);
    }
    double best = 0.0, fbest = 0.0;
    for (int c = 0; c < nc; ++c) {
        double t = cand[c];
        double ft = q.f(t);
        if (t > 0.0 && (ft < fbest || (ft == fbest && t < best && ft < 0.0))) {
            best = t;
            fbest = ft;
        }
    }
    return best;
}

// ---------------------------------------------------------------------------
// Two-loop recursion of Algorithm 1 on coefficient vectors (one thread, on the
// state copy in LDS).  Basis index of G slot g is g (0..T), of D slot d is
// T+1+d.  The current gradient is G slot gk; pair it (k-nmem <= it < k) has
// s_it = tau_it D_it with D_it in slot (dk - (k-it)) mod T, and
// y_it = G_{it+1} - G_it with G_it in slot (gk - (k-it)) mod (T+1).  Each s_t
// and y_t has one or two nonzero coefficients, so every inner product is a
// row (or a difference of two rows) of the Gram matrix times q.
// ---------------------------------------------------------------------------
__device__ double grow(const double *M, int i, int NB, const double *q) {
    double t = 0.0;
    for (int j = 0; j < NB; ++j) t += M[i * kMaxBasis + j] * q[j];
    return t;
}

__device__ void two_loop_coef(SolverState &st) {
    const int T = st.T, NB = 2 * T + 1, nmem = st.nmem, gk = st.gk, dk = st.dk;
    const double *M = st.gram;
    // work arrays in LDS: indexed at run time, they would otherwise live in
    // scratch memory (one thread of the workgroup runs this)
    __shared__ double q[kMaxBasis], alpha[kMaxMem], beta[kMaxMem];
    __shared__ int ds[kMaxMem], g0[kMaxMem], g1[kMaxMem];
    __shared__ double tau[kMaxMem];
    for (int j = 0; j < NB; ++j) q[j] = 0.0;
    q[gk] = -1.0;
    for (int t = 0; t < nmem; ++t) {  // t = 0 oldest
        const int back = nmem - t;
        ds[t] = T + 1 + ((dk - back) % T + T) % T;
        g0[t] = ((gk - back) % (T + 1) + (T + 1)) % (T + 1);
        g1[t] = (g0[t] + 1) % (T + 1);
        tau[t] = st.taus[ds[t] - T - 1];
        beta[t] = 1.0 / (tau[t] * (M[g1[t] * kMaxBasis + ds[t]] - M[g0[t] * kMaxBasis + ds[t]]));
    }
    for (int t = nmem - 1; t >= 0; --t) {
        alpha[t] = beta[t] * tau[t] * grow(M, ds[t], NB, q);
        q[g1[t]] -= alpha[t];
        q[g0[t]] += alpha[t];
    }
    for (int t = 0; t < nmem; ++t) {
        const double yq = grow(M, g1[t], NB, q) - grow(M, g0[t], NB, q);
        q[ds[t]] += (alpha[t] - beta[t] * yq) * tau[t];
    }
    // descent safeguard: <G_k, D> must be negative
    if (!(grow(M, gk, NB, q) < 0.0)) {
        st.nmem = 0;
        for (int j = 0; j < NB; ++j) q[j] = 0.0;
        q[gk] = -1.0;
    }
    for (int j = 0; j < kMaxBasis; ++j) st.coef[j] = j < NB ? q[j] : 0.0;
}

// The same recursion with H0 = P^{-1} (row-block H0, see PcBufs).  The first
// loop keeps q in the span of the G slots (coefficients qa); the middle step
// r = P^{-1} q is kept symbolic; the second loop needs y_t^T P^{-1} q, which
// is a combination of entries of the P^{-1}-weighted Gram matrix of the G
// slots (wgram, recomputed every iteration because P moves with R), and
// y_t^T s_t', entries of the plain Gram matrix.  Output: coefficients qa on the
// G slots (the combine pass applies P^{-1} to that part) and on the D slots.
__device__ void two_loop_coef_pc(SolverState &st) {
    const int T = st.T, NB = 2 * T + 1, nmem = st.nmem, gk = st.gk, dk = st.dk;
    const double *M = st.gram;
    const double *W = st.wgram;
    constexpr int WS = kMaxMem + 1;
    // work arrays in LDS (see two_loop_coef)
    __shared__ double qa[kMaxMem + 1], alpha[kMaxMem], beta[kMaxMem], fd[kMaxMem], tau[kMaxMem];
    __shared__ int ds[kMaxMem], g0[kMaxMem], g1[kMaxMem];
    for (int j = 0; j <= T; ++j) qa[j] = 0.0;
    qa[gk] = -1.0;
    for (int t = 0; t < nmem; ++t) {  // t = 0 oldest
        const int back = nmem - t;
        ds[t] = T + 1 + ((dk - back) % T + T) % T;
        g0[t] = ((gk - back) % (T + 1) + (T + 1)) % (T + 1);
        g1[t] = (g0[t] + 1) % (T + 1);
        tau[t] = st.taus[ds[t] - T - 1];
        beta[t] = 1.0 / (tau[t] * (M[g1[t] * kMaxBasis + ds[t]] - M[g0[t] * kMaxBasis + ds[t]]));
        fd[t] = 0.0;
    }
    for (int t = nmem - 1; t >= 0; --t) {
        double sq = 0.0;
        for (int j = 0; j <= T; ++j) sq += M[ds[t] * kMaxBasis + j] * qa[j];
        alpha[t] = beta[t] * tau[t] * sq;
        qa[g1[t]] -= alpha[t];
        qa[g0[t]] += alpha[t];
    }
    for (int t = 0; t < nmem; ++t) {
        double yr = 0.0;
        for (int j = 0; j <= T; ++j) yr += (W[g1[t] * WS + j] - W[g0[t] * WS + j]) * qa[j];
        for (int u = 0; u < t; ++u) yr += (M[g1[t] * kMaxBasis + ds[u]] - M[g0[t] * kMaxBasis + ds[u]]) * fd[u];
        fd[t] = (alpha[t] - beta[t] * yr) * tau[t];
    }
    // descent safeguard: <G_k, D> < 0, else D = -P^{-1} G_k (always a descent direction)
    double gd = 0.0;
    for (int j = 0; j <= T; ++j) gd += W[gk * WS + j] * qa[j];
    for (int t = 0; t < nmem; ++t) gd += M[gk * kMaxBasis + ds[t]] * fd[t];
    if (!(gd < 0.0)) {
        st.nmem = 0;
        for (int j = 0; j <= T; ++j) qa[j] = 0.0;
        qa[gk] = -1.0;
        for (int t = 0; t < nmem; ++t) fd[t] = 0.0;
    }
    for (int j = 0; j < kMaxBasis; ++j) st.coef[j] = 0.0;
    for (int j = 0; j <= T; ++j) st.coef[j] = qa[j];
    if (st.nmem > 0)
        for (int t = 0; t < nmem; ++t) st.coef[ds[t]] = fd[t];
    (void)NB;
}

}  // namespace

// ---------------------------------------------------------------------------
// Single-workgroup kernels.  Each stages the 3 KB state in LDS, reduces the
// partial sums of the preceding grid kernel, runs its scalar logic in one
// thread and writes the state back.
// ---------------------------------------------------------------------------

// Line-search stage: fold the previous combine pass's dots into the Gram
// matrix, form a1..a4 and take the exact step.
// kind: LRSDP_MAXCUT (p2 summed by the SpMM epilogue) or LRSDP_COMPLETION
// (C = cs I, so p2 = <C, D D^T> = cs ||D||_F^2, from a Gram entry).
__global__ __launch_bounds__(kBlock) void k_ls_finalize(SolverState *gst, const double *ls_part, int n_ls,
                                                        const double *cb_part, int n_cb, int kind, double cs) {
    __shared__ SolverState st;
    __shared__ double ls[kLsSums];
    __shared__ double cb[kMaxBasis + 1];
    block_copy(&st, gst);
    __syncthreads();
    if (st.done) return;
    reduce_rows<kLsSums>(ls_part, n_ls, ls);
    reduce_rows<kMaxBasis + 1>(cb_part, n_cb, cb);
    if (threadIdx.x == 0) {
        const int T = st.T, NB = 2 * T + 1, dcol = T + 1 + st.dk;
        double *M = st.gram;
        for (int j = 0; j < NB; ++j) {
            if (j == dcol) continue;
            M[dcol * kMaxBasis + j] = cb[j];
            M[j * kMaxBasis + dcol] = cb[j];
        }
        M[dcol * kMaxBasis + dcol] = cb[kMaxBasis];
        const double sigma = st.sigma;
        const double a1 = 0.5 * sigma * ls[3];
        const double a2 = sigma * ls[4];
        const double p2 = kind == LRSDP_COMPLETION ? cs * M[dcol * kMaxBasis + dcol] : ls[0];
        const double a3 = p2 - ls[1] + 0.5 * sigma * ls[5];
        const double a4 = M[st.gk * kMaxBasis + dcol];
        st.a[0] = a1;
        st.a[1] = a2;
        st.a[2] = a3;
        st.a[3] = a4;
        const bool finite = isfinite(a1) && isfinite(a2) && isfinite(a3) && isfinite(a4);
        const double tau = finite ? exact_step(a1, a2, a3, a4) : 0.0;
        if (!finite) st.numeric = 1;
        st.tau = tau;
        st.taus[st.dk] = tau;
        if (!(tau > 0.0)) {
            st.done = 3;
            st.k += 1;
            st.inner_total += 1;
        }
    }
    __syncthreads();
    block_copy(gst, &st);
}

// L-BFGS stage: fold the update pass's dots (new gradient) into the Gram
// matrix, apply the curvature guard to the new pair, advance the rings and
// compute the next direction's coefficients.
__global__ __launch_bounds__(kBlock) void k_lbfgs_finalize(SolverState *gst, const double *up_part, int n_up) {
    __shared__ SolverState st;
    __shared__ double raw[kMaxSums];
    block_copy(&st, gst);
    __syncthreads();
    if (st.done) return;
    if (st.precond) reduce_rows<kMaxSums>(up_part, n_up, raw);
    else reduce_rows<kMaxBasis>(up_part, n_up, raw);
    if (threadIdx.x == 0) {
        const int T = st.T, NB = 2 * T + 1;
        const int gk = st.gk, gk1 = (gk + 1) % (T + 1), ds = T + 1 + st.dk;
        double *M = st.gram;
        for (int j = 0; j < NB; ++j) {
            const double v = j <= T ? raw[j] : raw[kMaxMem + 1 + (j - T - 1)];
            M[gk1 * kMaxBasis + j] = v;
            M[j * kMaxBasis + gk1] = v;
        }
        if (st.precond) {
            for (int j = 0; j <= T; ++j)
                for (int l = j; l <= T; ++l) {
                    const double v = raw[kPcOff + pc_pair(j, l)];
                    st.wgram[j * (kMaxMem + 1) + l] = v;
                    st.wgram[l * (kMaxMem + 1) + j] = v;
                }
        }
        const double tau = st.tau;
        const double ys = tau * (M[gk1 * kMaxBasis + ds] - M[gk * kMaxBasis + ds]);
        const double yy = M[gk1 * kMaxBasis + gk1] - 2.0 * M[gk1 * kMaxBasis + gk] + M[gk * kMaxBasis + gk];
        const double ss = tau * tau * M[ds * kMaxBasis + ds];
        if (ys > 1e-12 * sqrt(fabs(yy * ss))) st.nmem = min(st.nmem + 1, T);
        else st.nmem = 0;
        st.k += 1;
        st.inner_total += 1;
        st.gk = gk1;
        st.dk = (st.dk + 1) % T;
        const double g2 = M[gk1 * kMaxBasis + gk1];
        st.gnorm = sqrt(fmax(g2, 0.0));
        if (!isfinite(g2)) {
            st.numeric = 1;
            st.done = 3;
        } else if (st.gnorm <= st.target) {
            st.done = 1;
        } else if (st.k >= st.max_inner) {
            st.done = 2;
        } else if (st.precond) {
            two_loop_coef_pc(st);
        } else {
            two_loop_coef(st);
        }
    }
    __syncthreads();
    block_copy(gst, &st);
}

// Start of a subproblem: gradient norm known, empty memory, D = -G.
// k_limit < 0: restart inside a subproblem after an exact gradient refresh
// (iteration count, limit and target kept).
__global__ __launch_bounds__(kBlock) void k_init_finalize(SolverState *gst, const double *part, int n_part,
                                                          int k_limit) {
    __shared__ SolverState st;
    __shared__ double g2[1];
    block_copy(&st, gst);
    reduce_rows<1>(part, n_part, g2);
    if (threadIdx.x == 0) {
        const bool restart = k_limit < 0;
        for (int j = 0; j < kMaxBasis * kMaxBasis; ++j) st.gram[j] = 0.0;
        st.gram[0] = g2[0];
        st.gk = 0;
        st.dk = 0;
        st.nmem = 0;
        st.gnorm = sqrt(fmax(g2[0], 0.0));
        if (!restart) {
            st.k = 0;
            st.max_inner = k_limit;
            st.target = st.eta * fmax(st.gfloor, st.gnorm);
        }
        k_limit = st.max_inner - st.k;
        for (int j = 0; j < kMaxBasis; ++j) st.coef[j] = 0.0;
        st.coef[0] = -1.0;
        st.done = 0;
        if (!isfinite(g2[0])) {
            st.numeric = 1;
            st.done = 3;
        } else if (st.gnorm <= st.target) {
            st.done = 1;
        } else if (k_limit <= 0) {
            st.done = 2;
        }
    }
    __syncthreads();
    block_copy(gst, &st);
}

// ALM step: measures after the multiplier update, stop test, penalty and
// inner-tolerance schedules.  mode 0: initial point (no schedule update).
// obj_scale multiplies the first sum: the objective of a completion problem
// with C = cs I arrives as ||R||_F^2 (MaxCut's SpMM already applies cs).
__global__ __launch_bounds__(kBlock) void k_alm_finalize(SolverState *gst, const double *part, int n_part,
                                                         int mode, double obj_scale) {
    __shared__ SolverState st;
    __shared__ double rs[3];
    block_copy(&st, gst);
    reduce_rows<3>(part, n_part, rs);
    if (threadIdx.x == 0) {
        const double obj = obj_scale * rs[0], dual = rs[1];
        const double res_norm = sqrt(fmax(rs[2], 0.0));
        st.obj = obj;
        st.dual = dual;
        st.res_norm = res_norm;
        st.err1 = res_norm / (1.0 + st.b_l1);
        st.err1_inf = res_norm / (1.0 + st.b_inf);
        st.err3 = (obj - dual) / (1.0 + fabs(obj) + fabs(dual));
        if (!isfinite(obj) || !isfinite(dual) || !isfinite(res_norm)) st.numeric = 1;
        st.refreshes += 1;
        if (mode != 0) {
            st.converged = (st.err1 <= st.tol && (st.stop_rule == 1 || fabs(st.err3) <= st.tol)) ? 1 : 0;
            if (!st.converged) {
                if (st.err1 > st.feas_decrease * st.err1_prev)
                    st.sigma = fmin(st.sigma * st.sigma_factor, st.sigma_cap);
                st.err1_prev = st.err1;
                st.eta = fmax(st.eta * st.eta_factor, st.eta_min);
            }
        }
    }
    __syncthreads();
    block_copy(gst, &st);
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_reduce(const double *part, int n_part, double *out) {
    __shared__ double r[K];
    reduce_rows<K>(part, n_part, r);
    if (threadIdx.x < K) out[threadIdx.x] = r[threadIdx.x];
}

__global__ void k_cubic(const double *a, double *tau) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *tau = exact_step(a[0], a[1], a[2], a[3]);
}

// ---------------------------------------------------------------------------
// Streaming kernels
// ---------------------------------------------------------------------------

template <typename S>
struct UpdateArgs {
    SolverState *st;
    S *R;
    const S *CD;
    const double *y;
    const double *rn;        // ||R_i||^2 of the current R (SpMM epilogue)
    const double *q1;        // 2 R_i . D_i
    const double *q2;        // ||D_i||^2
    const double *ytil_in;   // multiplier estimate used for the current G
    double *ytil_out;        // multiplier estimate of the new R
    Rings<S> rings;
    int64_t nchunks;         // n * chunks per row
    int cpr;                 // 16-byte chunks per row
    double *partials;
};

// MaxCut update sweep for step tau along D_k (one thread per 16-byte chunk):
//   R <- R + tau D,
//   ||R_new,i||^2 = ||R_i||^2 + tau q1_i + tau^2 q2_i,
//   ytil_i <- y_i + sigma (1 - ||R_new,i||^2),
//   G_{k+1} = 2 (C R_new - ytil_new o R_new) with C R_new = C R + tau C D and
//   C R = G_k/2 + ytil_old o R_old (so C R need not be stored),
// and the dot products of G_{k+1} with every ring slot.  TM is the largest
// memory the instance handles (T <= TM); each workgroup stores one compact row
// of 2 TM + 1 sums (G slots 0..TM, then D slots 0..TM-1) at a.partials.
template <typename S, int TM>
__global__ __launch_bounds__(kBlock) void k_update_maxcut(UpdateArgs<S> a) {
    using CV = typename Chunk<S>::V;
    constexpr int KS = 2 * TM + 1;
    SolverState *st = a.st;
    if (st->done) return;
    const double tau = st->tau, sigma = st->sigma;
    const int T = st->T, gk = st->gk, gk1 = (gk + 1) % (T + 1), dk = st->dk;
    double s[KS];
#pragma unroll
    for (int j = 0; j < KS; ++j) s[j] = 0.0;
    const CV *D = nullptr;
    const CV *Go = nullptr;
    CV *Gn = nullptr;
#pragma unroll
    for (int g = 0; g <= TM; ++g) {
        if (g == gk) Go = reinterpret_cast<const CV *>(a.rings.g[g]);
        if (g == gk1) Gn = reinterpret_cast<CV *>(a.rings.g[g]);
    }
#pragma unroll
    for (int d = 0; d < TM; ++d)
        if (d == dk) D = reinterpret_cast<const CV *>(a.rings.d[d]);
    CV *R = reinterpret_cast<CV *>(a.R);
    const CV *CD = reinterpret_cast<const CV *>(a.CD);
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < a.nchunks; c += (int64_t)gridDim.x * kBlock) {
        const int64_t row = c / a.cpr;
        const CV r = R[c], d = D[c], cd = CD[c], go = Go[c];
        const double yold = a.ytil_in[row];
        const double rnn = a.rn[row] + tau * (a.q1[row] + tau * a.q2[row]);
        const double ynew = a.y[row] + sigma * (1.0 - rnn);
        const D4 R0 = widen(r), Dd = widen(d), CDd = widen(cd), G0 = widen(go);
        D4 Rn;
#pragma unroll
        for (int e = 0; e < 4; ++e) Rn.v[e] = fma(tau, Dd.v[e], R0.v[e]);
        CV rn_s;
        narrow(Rn, rn_s);
        Rn = widen(rn_s);
        D4 Gv;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            Gv.v[e] = G0.v[e] + 2.0 * tau * CDd.v[e] + 2.0 * yold * R0.v[e] - 2.0 * ynew * Rn.v[e];
        CV gn_s;
        narrow(Gv, gn_s);
        R[c] = rn_s;
        Gn[c] = gn_s;
        if (c - row * a.cpr == 0) a.ytil_out[row] = ynew;
#pragma unroll
        for (int g = 0; g <= TM; ++g) {
            if (g <= T) {
                CV b;
                if (g == gk1) b = gn_s;
                else if (g == gk) b = go;
                else b = reinterpret_cast<const CV *>(a.rings.g[g])[c];
                s[g] += vdot(gn_s, b);
            }
        }
#pragma unroll
        for (int dd = 0; dd < TM; ++dd) {
            if (dd < T) {
                const CV b = (dd == dk) ? d : reinterpret_cast<const CV *>(a.rings.d[dd])[c];
                s[TM + 1 + dd] += vdot(gn_s, b);
            }
        }
    }
    block_sums_store<KS>(s, a.partials + (size_t)blockIdx.x * KS);
}

// Second level of the flat sweeps' sums: workgroup b adds the compact rows
// [b kL1PerL2, (b+1) kL1PerL2) of `in` (K doubles each, rows < nrows) in a
// fixed tree order and writes row b of `out` at stride kMaxSums, every column
// of it: compact sum j goes to column j for j < split, to column
// kMaxMem + 1 + (j - split) past it (the update's D slots; split = K keeps
// them in place) and, with last_col >= 0, the final sum to column last_col
// (the combine's ||out||^2).  Other columns are zero.
template <int K>
__global__ __launch_bounds__(kL1PerL2) void k_sum_l1(const SolverState *st, const double *in, int nrows, int split,
                                                     int last_col, double *out) {
    if (st && st->done) return;
    __shared__ double sh[kL1PerL2 / 64][K];
    const int r = blockIdx.x * kL1PerL2 + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double v = wave_sum(r < nrows ? in[(size_t)r * K + k] : 0.0);
        if (lane == 0) sh[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kMaxSums) {
        const int col = threadIdx.x;
        int j = -1;
        const int body = last_col >= 0 ? K - 1 : K;   // sums placed by `split`
        if (col < split && col < body) j = col;
        else if (col >= kMaxMem + 1 && split + (col - kMaxMem - 1) < body) j = split + (col - kMaxMem - 1);
        if (last_col >= 0 && col == last_col) j = K - 1;
        double t = 0.0;
        if (j >= 0) {
#pragma unroll
            for (int w = 0; w < kL1PerL2 / 64; ++w) t += sh[w][j];
        }
        out[(size_t)blockIdx.x * kMaxSums + col] = t;
    }
}

// The update sweep with the row-block H0 (solve option precond): one lane
// group of GS lanes per row (row dots need the whole row).  Besides everything
// k_update_maxcut computes it stores, for the new R, rho_g = R_i . G_{g,i} for
// every G slot and kap_i, and sums the P^{-1}-weighted Gram matrix of the G
// slots, sum_i [G_j,i . G_l,i - kap_i rho_j rho_l] / h_i, at partial indices
// kPcOff + pc_pair(j, l).  T <= kPcMem.
template <typename S, int GS>
__global__ __launch_bounds__(kBlock) void k_update_maxcut_pc(UpdateArgs<S> a, PcBufs pc, int ld) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    SolverState *st = a.st;
    if (st->done) return;
    const double tau = st->tau, sigma = st->sigma;
    const int T = st->T, gk = st->gk, gk1 = (gk + 1) % (T + 1), dk = st->dk;
    const int lane = threadIdx.x % GS, grp = threadIdx.x / GS;
    const bool active = lane * NV < ld;
    const int cpr = ld / NV;
    const CV zero = vzero(CV{});
    // sums: G slots [0, kPcMem], D slots [kPcMem + 1, 2 kPcMem], weighted pairs after
    constexpr int NS = 2 * kPcMem + 1 + kPcPairs;
    double s[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) s[j] = 0.0;
    const CV *D = nullptr;
    const CV *Go = nullptr;
    CV *Gn = nullptr;
#pragma unroll
    for (int g = 0; g <= kPcMem; ++g) {
        if (g == gk) Go = reinterpret_cast<const CV *>(a.rings.g[g]);
        if (g == gk1) Gn = reinterpret_cast<CV *>(a.rings.g[g]);
    }
#pragma unroll
    for (int d = 0; d < kPcMem; ++d)
        if (d == dk) D = reinterpret_cast<const CV *>(a.rings.d[d]);
    CV *R = reinterpret_cast<CV *>(a.R);
    const CV *CD = reinterpret_cast<const CV *>(a.CD);
    for (int64_t row = (int64_t)blockIdx.x * GPB + grp; row < pc.n; row += (int64_t)gridDim.x * GPB) {
        const int64_t c0 = row * cpr, c = c0 + lane;
        const CV r = vchunk_or_zero(R + c0, lane, active), d = vchunk_or_zero(D + c0, lane, active);
        const CV cd = vchunk_or_zero(CD + c0, lane, active), go = vchunk_or_zero(Go + c0, lane, active);
        const double yold = a.ytil_in[row];
        const double rnn = a.rn[row] + tau * (a.q1[row] + tau * a.q2[row]);
        const double ynew = a.y[row] + sigma * (1.0 - rnn);
        const D4 R0 = widen(r), Dd = widen(d), CDd = widen(cd), G0 = widen(go);
        D4 Rn;
#pragma unroll
        for (int e = 0; e < 4; ++e) Rn.v[e] = fma(tau, Dd.v[e], R0.v[e]);
        CV rn_s;
        narrow(Rn, rn_s);
        Rn = widen(rn_s);
        D4 Gv;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            Gv.v[e] = G0.v[e] + 2.0 * tau * CDd.v[e] + 2.0 * yold * R0.v[e] - 2.0 * ynew * Rn.v[e];
        CV gn_s;
        narrow(Gv, gn_s);
        if (active) {
            R[c] = rn_s;
            Gn[c] = gn_s;
        }
        // the G slots of this chunk (new gradient in slot gk1), held as named
        // values: kPcMem = 2, so three slots and six pairs, written out
        static_assert(kPcMem == 2, "the preconditioned sweep is written for three G slots");
        const CV *gp0 = reinterpret_cast<const CV *>(a.rings.g[0]);
        const CV *gp1 = reinterpret_cast<const CV *>(a.rings.g[1]);
        const CV *gp2 = reinterpret_cast<const CV *>(a.rings.g[2]);
        const CV b0 = gk1 == 0 ? gn_s : (gk == 0 ? go : (T >= 0 ? vchunk_or_zero(gp0 + c0, lane, active) : zero));
        const CV b1 = gk1 == 1 ? gn_s : (gk == 1 ? go : (T >= 1 ? vchunk_or_zero(gp1 + c0, lane, active) : zero));
        const CV b2 = gk1 == 2 ? gn_s : (gk == 2 ? go : (T >= 2 ? vchunk_or_zero(gp2 + c0, lane, active) : zero));
        s[0] += vdot(gn_s, b0);
        s[1] += vdot(gn_s, b1);
        if (T >= 2) s[2] += vdot(gn_s, b2);
        {
            const CV *dp0 = reinterpret_cast<const CV *>(a.rings.d[0]);
            const CV *dp1 = reinterpret_cast<const CV *>(a.rings.d[1]);
            const CV bd0 = dk == 0 ? d : vchunk_or_zero(dp0 + c0, lane, active);
            s[kPcMem + 1] += vdot(gn_s, bd0);
            if (T >= 2) {
                const CV bd1 = dk == 1 ? d : vchunk_or_zero(dp1 + c0, lane, active);
                s[kPcMem + 2] += vdot(gn_s, bd1);
            }
        }
        const double rho0 = group_sum<GS>(vdot(rn_s, b0));
        const double rho1 = group_sum<GS>(vdot(rn_s, b1));
        const double rho2 = T >= 2 ? group_sum<GS>(vdot(rn_s, b2)) : 0.0;
        const double hs = pc.cs * pc.hrow[row];
        const double h = pc.mode == 2 ? 2.0 * fmax(pc.cs * pc.diag[row] - ynew, 0.005 * hs) : hs;
        const double w = 1.0 / h;
        const double kap = 4.0 * sigma / (h + 4.0 * sigma * rnn);
        const double wk = lane == 0 ? w * kap : 0.0;
        constexpr int P0 = 2 * kPcMem + 1;
        s[P0 + pc_pair(0, 0)] += w * vdot(b0, b0) - wk * rho0 * rho0;
        s[P0 + pc_pair(0, 1)] += w * vdot(b0, b1) - wk * rho0 * rho1;
        s[P0 + pc_pair(1, 1)] += w * vdot(b1, b1) - wk * rho1 * rho1;
        if (T >= 2) {
            s[P0 + pc_pair(0, 2)] += w * vdot(b0, b2) - wk * rho0 * rho2;
            s[P0 + pc_pair(1, 2)] += w * vdot(b1, b2) - wk * rho1 * rho2;
            s[P0 + pc_pair(2, 2)] += w * vdot(b2, b2) - wk * rho2 * rho2;
        }
        if (lane == 0) {
            a.ytil_out[row] = ynew;
            pc.kap[row] = kap;
            if (pc.mode == 2) pc.hdyn[row] = h;
            pc.rho[row] = rho0;
            pc.rho[pc.n + row] = rho1;
            if (T >= 2) pc.rho[2 * pc.n + row] = rho2;
        }
    }
    // partial row in the layout of the flat sweep (G slot g at g, D slot d at
    // kMaxMem + 1 + d) plus the weighted pairs at kPcOff
    double out[kMaxSums];
#pragma unroll
    for (int j = 0; j < kMaxSums; ++j) out[j] = 0.0;
#pragma unroll
    for (int g = 0; g <= kPcMem; ++g) out[g] = s[g];
#pragma unroll
    for (int d = 0; d < kPcMem; ++d) out[kMaxMem + 1 + d] = s[kPcMem + 1 + d];
#pragma unroll
    for (int q = 0; q < kPcPairs; ++q) out[kPcOff + q] = s[2 * kPcMem + 1 + q];
    block_sums_store<kMaxSums>(out, a.partials + (size_t)blockIdx.x * kMaxSums);
}

template <typename S>
struct CombineArgs {
    SolverState *st;        // coefficients (solver) or nullptr
    const double *coef;     // used when st == nullptr
    const S *basis[kMaxBasis];
    int nb;                 // basis size when st == nullptr
    S *out;                 // used when st == nullptr
    int64_t nchunks;        // n * ld / chunk
    double *partials;       // dots of out with each basis entry, then ||out||^2
    uint16_t *shadow;       // float32 only: bfloat16 copy of out (row stride ldb), or nullptr
    int64_t ld, ldb;
    const S *R;             // precond: current R
    PcBufs pc;              // precond: rho, kap, h
};

// out = sum_j coef_j basis_j, and <out, basis_j> (pre-update values) for all j
// plus <out, out>.  In the solver the output is D slot dk, itself basis entry
// T+1+dk (read before written by the same thread).  The instance handles up to
// KB = 2 TM + 1 basis entries; each workgroup stores one compact row of KB + 1
// sums (the basis dots, then <out, out>) at a.partials.
template <typename S, bool PC, int TM>
__global__ __launch_bounds__(kBlock) void k_combine(CombineArgs<S> a) {
    constexpr int KB = 2 * TM + 1;
    using CV = typename Chunk<S>::V;
    const SolverState *st = a.st;
    if (st && st->done) return;
    const int NB = st ? 2 * st->T + 1 : a.nb;
    const double *coef = st ? st->coef : a.coef;
    S *out = a.out;
    if (st) {
        const int oj = st->T + 1 + st->dk;
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (j == oj) out = const_cast<S *>(a.basis[j]);
    }
    double cf[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) cf[j] = j < NB ? coef[j] : 0.0;
    double s[KB + 1];
#pragma unroll
    for (int j = 0; j <= KB; ++j) s[j] = 0.0;
    constexpr bool pcon = PC;   // row-block H0: the solver's state has precond set
    const int TG = PC ? st->T : -1;                              // G slots 0..TG
    const int64_t cpr = PC ? a.nchunks / (a.pc.n > 0 ? a.pc.n : 1) : 1;  // chunks per row
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < a.nchunks; c += (int64_t)gridDim.x * kBlock) {
        CV b[KB];
        D4 acc{{0.0, 0.0, 0.0, 0.0}};
        if constexpr (pcon) {
            // D = P^{-1} (sum over G slots) + sum over D slots, row by row
            D4 accg{{0.0, 0.0, 0.0, 0.0}};
            const int64_t row = c / cpr;
            double ra = 0.0;
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                if (j < NB) {
                    b[j] = reinterpret_cast<const CV *>(a.basis[j])[c];
                    D4 w = widen(b[j]);
                    if (j <= TG) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) accg.v[e] = fma(cf[j], w.v[e], accg.v[e]);
                        ra = fma(cf[j], a.pc.rho[j * a.pc.n + row], ra);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc.v[e] = fma(cf[j], w.v[e], acc.v[e]);
                    }
                }
            }
            const D4 r = widen(reinterpret_cast<const CV *>(a.R)[c]);
            const double hi = 1.0 / (a.pc.mode == 2 ? a.pc.hdyn[row] : a.pc.cs * a.pc.hrow[row]), kr = a.pc.kap[row] * ra;
#pragma unroll
            for (int e = 0; e < 4; ++e) acc.v[e] = fma(hi, accg.v[e] - kr * r.v[e], acc.v[e]);
        } else {
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                if (j < NB) {
                    b[j] = reinterpret_cast<const CV *>(a.basis[j])[c];
                    D4 w = widen(b[j]);
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc.v[e] = fma(cf[j], w.v[e], acc.v[e]);
                }
            }
        }
        CV o;
        narrow(acc, o);
        reinterpret_cast<CV *>(out)[c] = o;
        if constexpr (sizeof(S) == 4) {
            if (a.shadow) {
                const int64_t e = c * 4, row = e / a.ld, col = e - row * a.ld;
                const D4 w = widen(o);
                uint2 pk;
                pk.x = (uint32_t)bf16_rne((float)w.v[0]) | ((uint32_t)bf16_rne((float)w.v[1]) << 16);
                pk.y = (uint32_t)bf16_rne((float)w.v[2]) | ((uint32_t)bf16_rne((float)w.v[3]) << 16);
                *reinterpret_cast<uint2 *>(a.shadow + row * a.ldb + col) = pk;
            }
        }
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (j < NB) s[j] += vdot(o, b[j]);
        s[KB] += vdot(o, o);
    }
    block_sums_store<KB + 1>(s, a.partials + (size_t)blockIdx.x * (KB + 1));
}

template <typename S>
struct GradInitArgs {
    SolverState *st;
    const S *R;
    const S *CR;
    const double *y;
    const double *rn;   // ||R_i||^2
    double *ytil;
    S *G;
    int64_t n, ld;
    double *partials;
    PcBufs pc;          // precond: rho of G slot 0 and kap (rho == nullptr: off)
};

// Start of a subproblem (MaxCut): ytil = y + sigma (1 - ||R_i||^2),
// G = 2 (C R - ytil o R), and ||G||^2.
template <typename S, int GS>
__global__ __launch_bounds__(kBlock) void k_grad_init_maxcut(GradInitArgs<S> a) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    const double sigma = a.st->sigma;
    const int lane = threadIdx.x % GS, grp = threadIdx.x / GS;
    const bool active = lane * NV < a.ld;
    double s[1] = {0.0};
    for (int64_t row = (int64_t)blockIdx.x * GPB + grp; row < a.n; row += (int64_t)gridDim.x * GPB) {
        const int64_t rb = row * a.ld, off = rb + lane * NV;
        const double yt = a.y[row] + sigma * (1.0 - a.rn[row]);
        if (lane == 0) a.ytil[row] = yt;
        const CV rs = chunk_or_zero(a.R + rb, lane, active);
        D4 r = widen(rs);
        D4 cr = widen(chunk_or_zero(a.CR + rb, lane, active));
        D4 g;
#pragma unroll
        for (int c = 0; c < 4; ++c) g.v[c] = 2.0 * (cr.v[c] - yt * r.v[c]);
        CV gs;
        narrow(g, gs);
        if (active) *reinterpret_cast<CV *>(a.G + off) = gs;
        s[0] += vdot(gs, gs);
        if (a.pc.rho) {
            // row-block H0: R_i . G_i for G slot 0 and kap_i at the current R
            const double rho = group_sum<GS>(vdot(rs, gs));
            if (lane == 0) {
                const double hs = a.pc.cs * a.pc.hrow[row];
                const double h = a.pc.mode == 2 ? 2.0 * fmax(a.pc.cs * a.pc.diag[row] - yt, 0.005 * hs) : hs;
                if (a.pc.mode == 2) a.pc.hdyn[row] = h;
                a.pc.rho[row] = rho;
                a.pc.kap[row] = 4.0 * sigma / (h + 4.0 * sigma * a.rn[row]);
            }
        }
    }
    block_sums_store<1>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

// Dynamic rank (appendix A.1): new columns [c0, c1) of R get scale * N(0, 1)
// values from a counter-based generator.  Entry (i, c) takes outputs 2k and
// 2k+1, k = 65536 i + c, of the SplitMix64 sequence seeded with `seed` (output
// j is mix(seed + (j+1) gamma), Steele, Lea and Flood 2014) as uniforms
// u = ((x >> 11) + 0.5) 2^-53 in (0, 1), then Box-Muller:
// z = sqrt(-2 ln u0) cos(2 pi u1).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
    uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_rank_grow(S *R, int64_t n, int64_t ld, int c0, int c1, uint64_t seed,
                                                      double scale, const int32_t *label) {
    const int w = c1 - c0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * w; e += (int64_t)gridDim.x * kBlock) {
        const int64_t i = e / w;
        const int c = c0 + (int)(e - i * w);
        // the draw belongs to the caller's node: a relabelled problem grows the same columns
        const uint64_t li = label ? (uint64_t)label[i] : (uint64_t)i;
        const uint64_t k = li * 65536ull + (uint64_t)c;
        const uint64_t x0 = splitmix64_at(seed, 2 * k), x1 = splitmix64_at(seed, 2 * k + 1);
        const double u0 = ((double)(x0 >> 11) + 0.5) * 0x1.0p-53;
        const double u1 = ((double)(x1 >> 11) + 0.5) * 0x1.0p-53;
        const double z = sqrt(-2.0 * log(u0)) * cos(6.283185307179586 * u1);
        R[i * ld + c] = (S)(scale * z);
    }
}

// x <- a x elementwise (float64 vectors)
__global__ __launch_bounds__(kBlock) void k_dscale(double *x, double a, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        x[i] *= a;
}

// out = (a + b) / 2 elementwise
template <typename S>
__global__ __launch_bounds__(kBlock) void k_avg(const S *a, const S *b, S *out, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        out[i] = (S)(0.5 * ((double)a[i] + (double)b[i]));
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_fill(S *p, int64_t count, S v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) p[i] = v;
}

template <typename S>
struct DotsArgs {
    const S *x;
    const S *basis[kMaxBasis];
    int nb;
    int64_t nchunks;
    double *partials;
};

// <x, basis_j> for j < nb (float64 sums)
template <typename S>
__global__ __launch_bounds__(kBlock) void k_dots(DotsArgs<S> a) {
    using CV = typename Chunk<S>::V;
    double s[kMaxBasis];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j) s[j] = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < a.nchunks; c += (int64_t)gridDim.x * kBlock) {
        CV x = reinterpret_cast<const CV *>(a.x)[c];
#pragma unroll
        for (int j = 0; j < kMaxBasis; ++j)
            if (j < a.nb) s[j] += vdot(x, reinterpret_cast<const CV *>(a.basis[j])[c]);
    }
    block_sums_store<kMaxBasis>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static int grid_for(int64_t work_items, int per_block) {
    int64_t need = (work_items + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, kMaxBlocks));
}

static int chunks_per_row(int prec, int64_t ld) { return (int)(ld * (prec == LRSDP_F64 ? 8 : 4) / 16); }

int launch_ls_finalize(hipStream_t s, SolverState *st, const double *ls, int nls, const double *cb, int ncb,
                       int kind, double cs) {
    hipLaunchKernelGGL(k_ls_finalize, dim3(1), dim3(kBlock), 0, s, st, ls, nls, cb, ncb, kind, cs);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_lbfgs_finalize(hipStream_t s, SolverState *st, const double *up, int nup) {
    hipLaunchKernelGGL(k_lbfgs_finalize, dim3(1), dim3(kBlock), 0, s, st, up, nup);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_init_finalize(hipStream_t s, SolverState *st, const double *part, int np, int k_limit) {
    hipLaunchKernelGGL(k_init_finalize, dim3(1), dim3(kBlock), 0, s, st, part, np, k_limit);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_alm_finalize(hipStream_t s, SolverState *st, const double *part, int np, int mode, double obj_scale) {
    hipLaunchKernelGGL(k_alm_finalize, dim3(1), dim3(kBlock), 0, s, st, part, np, mode, obj_scale);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_reduce(hipStream_t s, const double *part, int np, int K, double *out) {
    switch (K) {
#define LRSDP_RED(k) \
    case k: hipLaunchKernelGGL(k_reduce<k>, dim3(1), dim3(kBlock), 0, s, part, np, out); break;
        LRSDP_RED(1) LRSDP_RED(2) LRSDP_RED(3) LRSDP_RED(4) LRSDP_RED(5) LRSDP_RED(6) LRSDP_RED(7)
        LRSDP_RED(8) LRSDP_RED(9) LRSDP_RED(10) LRSDP_RED(11) LRSDP_RED(12) LRSDP_RED(13) LRSDP_RED(14)
        LRSDP_RED(15) LRSDP_RED(16) LRSDP_RED(17) LRSDP_RED(18)
#undef LRSDP_RED
        default: return set_error(LRSDP_EINVAL, "reduction width %d unsupported", K);
    }
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_cubic(hipStream_t s, const double *a, double *tau) {
    hipLaunchKernelGGL(k_cubic, dim3(1), dim3(64), 0, s, a, tau);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

template <typename S>
static int update_pc(hipStream_t s, const UpdateArgs<S> &a, const PcBufs &pc, int64_t ld, int cpr, int *nb) {
    const int gs = cpr <= 4 ? 4 : (cpr <= 8 ? 8 : 16);
    *nb = grid_for(pc.n, kBlock / gs);
    if (gs == 4) hipLaunchKernelGGL((k_update_maxcut_pc<S, 4>), dim3(*nb), dim3(kBlock), 0, s, a, pc, (int)ld);
    else if (gs == 8) hipLaunchKernelGGL((k_update_maxcut_pc<S, 8>), dim3(*nb), dim3(kBlock), 0, s, a, pc, (int)ld);
    else hipLaunchKernelGGL((k_update_maxcut_pc<S, 16>), dim3(*nb), dim3(kBlock), 0, s, a, pc, (int)ld);
    return LRSDP_OK;
}

// Smallest build of the flat sweeps that holds an L-BFGS memory of T (2T + 1 ring slots).
static int mem_build(int T) { return T <= 1 ? 1 : (T <= 2 ? 2 : (T <= 4 ? 4 : 8)); }

// Workgroups of a flat sweep over nch chunks whose compact sum rows hold K doubles.
static int flat_grid(int64_t nch, int K) {
    const int64_t need = (nch + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)(kL1Bytes / (sizeof(double) * (size_t)K)) / kL1PerL2 * kL1PerL2;
    return (int)std::max<int64_t>(1, std::min(need, cap));
}

// Second level of a flat sweep's sums into `partials`; returns the row count.
template <int K>
static int sum_l1(hipStream_t s, const SolverState *st, const double *l1, int rows1, int split, int last_col,
                  double *partials) {
    const int rows2 = (rows1 + kL1PerL2 - 1) / kL1PerL2;
    hipLaunchKernelGGL(k_sum_l1<K>, dim3(rows2), dim3(kL1PerL2), 0, s, st, l1, rows1, split, last_col, partials);
    return rows2;
}

template <typename S, int TM>
static int update_flat(hipStream_t s, UpdateArgs<S> a, double *partials, double *l1) {
    constexpr int KS = 2 * TM + 1;
    const int g = flat_grid(a.nchunks, KS);
    a.partials = l1;
    hipLaunchKernelGGL((k_update_maxcut<S, TM>), dim3(g), dim3(kBlock), 0, s, a);
    return sum_l1<KS>(s, a.st, l1, g, TM + 1, -1, partials);
}

template <typename S>
static int update_flat_t(hipStream_t s, const UpdateArgs<S> &a, int T, double *partials, double *l1) {
    switch (mem_build(T)) {
        case 1: return update_flat<S, 1>(s, a, partials, l1);
        case 2: return update_flat<S, 2>(s, a, partials, l1);
        case 4: return update_flat<S, 4>(s, a, partials, l1);
        default: return update_flat<S, 8>(s, a, partials, l1);
    }
}

int launch_update_maxcut(hipStream_t s, int prec, SolverState *st, void *R, const void *CD, const double *y,
                         const double *rn, const double *q1, const double *q2, const double *ytil_in,
                         double *ytil_out, void *const *gring, void *const *dring, int T, int64_t n, int64_t ld,
                         double *partials, double *l1, int *nb, const PcBufs *pc) {
    if (T < 1 || T > kMaxMem) return set_error(LRSDP_EINVAL, "L-BFGS memory %d outside [1, %d]", T, kMaxMem);
    const int cpr = chunks_per_row(prec, ld);
    const int64_t nch = n * cpr;
    if (prec == LRSDP_F64) {
        UpdateArgs<double> a{st, (double *)R, (const double *)CD, y, rn, q1, q2, ytil_in, ytil_out, {}, nch, cpr,
                             partials};
        for (int g = 0; g <= T; ++g) a.rings.g[g] = (double *)gring[g];
        for (int d = 0; d < T; ++d) a.rings.d[d] = (double *)dring[d];
        if (pc) update_pc<double>(s, a, *pc, ld, cpr, nb);
        else *nb = update_flat_t<double>(s, a, T, partials, l1);
    } else {
        UpdateArgs<float> a{st, (float *)R, (const float *)CD, y, rn, q1, q2, ytil_in, ytil_out, {}, nch, cpr,
                            partials};
        for (int g = 0; g <= T; ++g) a.rings.g[g] = (float *)gring[g];
        for (int d = 0; d < T; ++d) a.rings.d[d] = (float *)dring[d];
        if (pc) update_pc<float>(s, a, *pc, ld, cpr, nb);
        else *nb = update_flat_t<float>(s, a, T, partials, l1);
    }
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

template <typename S, bool PC, int TM>
static int combine_flat(hipStream_t s, CombineArgs<S> a, double *partials, double *l1) {
    constexpr int K = 2 * TM + 2;
    const int g = flat_grid(a.nchunks, K);
    a.partials = l1;
    hipLaunchKernelGGL((k_combine<S, PC, TM>), dim3(g), dim3(kBlock), 0, s, a);
    return sum_l1<K>(s, a.st, l1, g, K, kMaxBasis, partials);
}

// nb basis entries need a build with 2 TM + 1 >= nb; the row-block H0 only
// comes with memories up to kPcMem = 2.
template <typename S, bool PC>
static int combine_flat_t(hipStream_t s, const CombineArgs<S> &a, int nb, double *partials, double *l1) {
    const int tm = mem_build(nb / 2);
    if constexpr (PC) {
        if (tm == 1) return combine_flat<S, true, 1>(s, a, partials, l1);
        return combine_flat<S, true, 2>(s, a, partials, l1);
    } else {
        switch (tm) {
            case 1: return combine_flat<S, false, 1>(s, a, partials, l1);
            case 2: return combine_flat<S, false, 2>(s, a, partials, l1);
            case 4: return combine_flat<S, false, 4>(s, a, partials, l1);
            default: return combine_flat<S, false, 8>(s, a, partials, l1);
        }
    }
}

// basis: nb device arrays of n*ld elements; out = sum coef_j basis_j.
int launch_combine(hipStream_t s, int prec, SolverState *st, const double *coef, const void *const *basis, int nb,
                   void *out, int64_t n, int64_t ld, double *partials, double *l1, int *nblk, uint16_t *shadow,
                   const void *R, const PcBufs *pc) {
    if (nb < 1 || nb > kMaxBasis) return set_error(LRSDP_EINVAL, "basis of %d vectors outside [1, %d]", nb, kMaxBasis);
    if (pc && nb > 2 * kPcMem + 1)
        return set_error(LRSDP_EINVAL, "row-block H0 takes an L-BFGS memory of at most %d", kPcMem);
    const int64_t nch = n * ld * (prec == LRSDP_F64 ? 8 : 4) / 16;
    const PcBufs p = pc ? *pc : PcBufs{nullptr, nullptr, nullptr, n, 0, nullptr, nullptr, 1.0};
    if (prec == LRSDP_F64) {
        CombineArgs<double> a{st, coef, {}, nb, (double *)out, nch, partials, nullptr, ld, ld, (const double *)R, p};
        for (int j = 0; j < nb; ++j) a.basis[j] = (const double *)basis[j];
        if (pc) *nblk = combine_flat_t<double, true>(s, a, nb, partials, l1);
        else *nblk = combine_flat_t<double, false>(s, a, nb, partials, l1);
    } else {
        CombineArgs<float> a{st, coef, {}, nb, (float *)out, nch, partials, shadow, ld, bf16_ld(ld), (const float *)R,
                             p};
        for (int j = 0; j < nb; ++j) a.basis[j] = (const float *)basis[j];
        if (pc) *nblk = combine_flat_t<float, true>(s, a, nb, partials, l1);
        else *nblk = combine_flat_t<float, false>(s, a, nb, partials, l1);
    }
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_grad_init_maxcut(hipStream_t s, int prec, SolverState *st, const void *R, const void *CR,
                            const double *y, const double *rn, double *ytil, void *G, int64_t n, int64_t ld,
                            double *partials, int *nblk, const PcBufs *pc) {
    const int cpr = chunks_per_row(prec, ld);
    const int gs = cpr <= 4 ? 4 : (cpr <= 8 ? 8 : 16);
    *nblk = grid_for(n, kBlock / gs);
    const PcBufs p = pc ? *pc : PcBufs{nullptr, nullptr, nullptr, n, 0, nullptr, nullptr, 1.0};
    if (prec == LRSDP_F64) {
        GradInitArgs<double> a{st, (const double *)R, (const double *)CR, y, rn, ytil, (double *)G, n, ld, partials,
                               p};
        if (gs == 4) hipLaunchKernelGGL((k_grad_init_maxcut<double, 4>), dim3(*nblk), dim3(kBlock), 0, s, a);
        else if (gs == 8) hipLaunchKernelGGL((k_grad_init_maxcut<double, 8>), dim3(*nblk), dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_grad_init_maxcut<double, 16>), dim3(*nblk), dim3(kBlock), 0, s, a);
    } else {
        GradInitArgs<float> a{st, (const float *)R, (const float *)CR, y, rn, ytil, (float *)G, n, ld, partials, p};
        if (gs == 4) hipLaunchKernelGGL((k_grad_init_maxcut<float, 4>), dim3(*nblk), dim3(kBlock), 0, s, a);
        else if (gs == 8) hipLaunchKernelGGL((k_grad_init_maxcut<float, 8>), dim3(*nblk), dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_grad_init_maxcut<float, 16>), dim3(*nblk), dim3(kBlock), 0, s, a);
    }
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_rank_grow(hipStream_t s, int prec, void *R, int64_t n, int64_t ld, int c0, int c1, uint64_t seed,
                     double scale, const int32_t *label) {
    if (c1 <= c0) return LRSDP_OK;
    const int nb = grid_for(n * (c1 - c0), kBlock);
    if (prec == LRSDP_F64)
        hipLaunchKernelGGL(k_rank_grow<double>, dim3(nb), dim3(kBlock), 0, s, (double *)R, n, ld, c0, c1, seed, scale,
                           label);
    else
        hipLaunchKernelGGL(k_rank_grow<float>, dim3(nb), dim3(kBlock), 0, s, (float *)R, n, ld, c0, c1, seed, scale,
                           label);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

// Node-order moves (declared in internal.h).
__global__ __launch_bounds__(kBlock) void k_permute_rows(const int4 *src, int4 *dst, const int32_t *perm, int64_t n,
                                                         int64_t cpr, int scatter) {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * cpr; e += (int64_t)gridDim.x * kBlock) {
        const int64_t k = e / cpr, q = e - k * cpr, j = perm[k];
        if (scatter) dst[j * cpr + q] = src[e];
        else dst[e] = src[j * cpr + q];
    }
}

__global__ __launch_bounds__(kBlock) void k_permute_vec(const double *src, double *dst, const int32_t *perm,
                                                        int64_t n, int scatter) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock) {
        if (scatter) dst[perm[k]] = src[k];
        else dst[k] = src[perm[k]];
    }
}

int launch_permute_rows(hipStream_t s, const void *src, void *dst, const int32_t *perm, int64_t n, int64_t row_bytes,
                        int scatter) {
    if (row_bytes % 16 != 0) return set_error(LRSDP_EINVAL, "row of %lld bytes is not a multiple of 16",
                                              (long long)row_bytes);
    if (n <= 0) return LRSDP_OK;
    const int64_t cpr = row_bytes / 16;
    hipLaunchKernelGGL(k_permute_rows, dim3(grid_for(n * cpr, kBlock)), dim3(kBlock), 0, s, (const int4 *)src,
                       (int4 *)dst, perm, n, cpr, scatter);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_permute_vec(hipStream_t s, const double *src, double *dst, const int32_t *perm, int64_t n, int scatter) {
    if (n <= 0) return LRSDP_OK;
    hipLaunchKernelGGL(k_permute_vec, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, src, dst, perm, n, scatter);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_dscale(hipStream_t s, double *x, double a, int64_t count) {
    if (count <= 0) return LRSDP_OK;
    hipLaunchKernelGGL(k_dscale, dim3(grid_for(count, kBlock)), dim3(kBlock), 0, s, x, a, count);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_fill(hipStream_t s, int prec, void *p, int64_t count) {
    int nb = grid_for(count, kBlock);
    if (prec == LRSDP_F64) hipLaunchKernelGGL(k_fill<double>, dim3(nb), dim3(kBlock), 0, s, (double *)p, count, 0.0);
    else hipLaunchKernelGGL(k_fill<float>, dim3(nb), dim3(kBlock), 0, s, (float *)p, count, 0.0f);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_avg(hipStream_t s, int prec, const void *a, const void *b, void *out, int64_t count) {
    int nb = grid_for(count, kBlock);
    if (prec == LRSDP_F64)
        hipLaunchKernelGGL(k_avg<double>, dim3(nb), dim3(kBlock), 0, s, (const double *)a, (const double *)b,
                           (double *)out, count);
    else
        hipLaunchKernelGGL(k_avg<float>, dim3(nb), dim3(kBlock), 0, s, (const float *)a, (const float *)b,
                           (float *)out, count);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_fill_f64(hipStream_t s, double *p, int64_t count, double v) {
    int nb = grid_for(count, kBlock);
    hipLaunchKernelGGL(k_fill<double>, dim3(nb), dim3(kBlock), 0, s, p, count, v);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_dots(hipStream_t s, int prec, const void *x, const void *const *basis, int nb, int64_t n, int64_t ld,
                double *partials, int *nblk) {
    const int64_t nch = n * ld * (prec == LRSDP_F64 ? 8 : 4) / 16;
    *nblk = grid_for(nch, kBlock);
    if (prec == LRSDP_F64) {
        DotsArgs<double> a{(const double *)x, {}, nb, nch, partials};
        for (int j = 0; j < nb; ++j) a.basis[j] = (const double *)basis[j];
        hipLaunchKernelGGL(k_dots<double>, dim3(*nblk), dim3(kBlock), 0, s, a);
    } else {
        DotsArgs<float> a{(const float *)x, {}, nb, nch, partials};
        for (int j = 0; j < nb; ++j) a.basis[j] = (const float *)basis[j];
        hipLaunchKernelGGL(k_dots<float>, dim3(*nblk), dim3(kBlock), 0, s, a);
    }
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

// host copy of the step rule for kernels that need it on the host side
double exact_step_host(double a1, double a2, double a3, double a4) { return exact_step(a1, a2, a3, a4); }

}  // namespace lrsdp
