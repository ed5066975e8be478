// Kernel launchers and the device-resident solver state.
#pragma once

#include "internal.h"

namespace lrsdp {

// Solver state kept in device memory: the host only enqueues kernels and reads
// this block back every few iterations.
struct SolverState {
    // current L-BFGS subproblem
    double tau;                          // last step
    double sigma;                        // penalty
    double sigma_cap;                    // sigma_max_ratio * sigma0
    double eta;                          // inner tolerance factor
    double target;                       // inner stop: ||G||_F <= target
    double gfloor;                       // target = eta max(gfloor, ||G_0||_F); gfloor = objective scale
    double gnorm;                        // ||G_k||_F
    double a[4];                         // quartic coefficients a1..a4
    double taus[kMaxMem];                // step of the direction in each D slot
    double gram[kMaxBasis * kMaxBasis];  // Gram matrix of the G/D ring slots
    double coef[kMaxBasis];              // next direction = sum coef_j basis_j (precond: the
                                         // G-slot part is multiplied by P^{-1} row by row)
    double wgram[(kMaxMem + 1) * (kMaxMem + 1)];  // precond: G slots' Gram in the P^{-1} metric
    // ALM measures after the last multiplier step
    double obj, dual, res_norm, err1, err1_inf, err3, err1_prev;
    // options copied at solve start
    double tol, sigma_factor, feas_decrease, eta_factor, eta_min, b_l1, b_inf;
    int64_t inner_total;
    int max_inner;
    int T;          // L-BFGS memory
    int k;          // iteration within the subproblem
    int nmem;       // valid pairs
    int gk;         // G ring slot of the current gradient (0..T)
    int dk;         // D ring slot of the current direction (0..T-1)
    int done;       // 0 running; 1 gradient small; 2 max_inner; 3 no descent step
    int converged;  // ALM stop test met
    int numeric;    // NaN/Inf met
    int refreshes;  // exact C R recomputations
    int precond;    // 1: row-block H0 = P^{-1} in the two-loop (MaxCut)
    int stop_rule;  // 0: err1 <= tol and |err3| <= tol; 1: err1 <= tol (a re-optimisation round)
};

// Row-block H0 of the L-BFGS direction (solve option precond, MaxCut):
// P_i = h_i I + 4 sigma R_i R_i^T (h_i static, or from the diagonal of
// C - Diag(ytil) at the current iterate), applied as
// P_i^{-1} q = (q - kap_i (R_i . q) R_i) / h_i with kap_i = 4 sigma / (h_i + 4 sigma ||R_i||^2).
// rho[g * n + i] = R_i . G_{g,i} (row dots of the current R with G ring slot g).
constexpr int kPcMem = 2;              // largest L-BFGS memory with precond
constexpr int kPcPairs = (kPcMem + 1) * (kPcMem + 2) / 2;
constexpr int kPcOff = 17;             // partial-sum index of the first weighted Gram pair
struct PcBufs {
    double *rho;         // (T + 1) x n
    double *kap;         // n
    const double *hrow;  // n: static h_i = 2 max(sum_j |C_ij|, 1e-3 ||vec(C)||_1 / n)
    int64_t n;
    int mode;            // 1: h = hrow; 2: h_i = 2 max(C_ii - ytil_i, 0.01 hrow_i), moves with ytil
    const double *diag;  // mode 2: C_ii
    double *hdyn;        // mode 2: h of the current iterate (n)
    double cs;           // objective scale: h from cs C
};

// index of the unordered G-slot pair (j, l), j <= l <= kPcMem
__host__ __device__ inline int pc_pair(int j, int l) {
    return j * (kPcMem + 1) - j * (j - 1) / 2 + (l - j);
}

// Pointers of the L-BFGS rings: G slots 0..T, D slots 0..T-1.  Basis index of
// G slot g is g, of D slot d is T + 1 + d.
template <typename S>
struct Rings {
    S *g[kMaxMem + 1];
    S *d[kMaxMem];
};

enum EpiKind { kEpiPlain = 0, kEpiLS = 1, kEpiRefresh = 2, kEpiSplit = 3 };

// Arguments of one SpMM Y = C V (+ epilogue).  See spmm_maxcut.hip.
struct SpmmArgs {
    int epi = kEpiPlain;
    const void *V = nullptr;        // gathered operand (bfloat16 for LRSDP_F32_BF16IN)
    const void *Vown = nullptr;     // kEpiLS with bfloat16 input: float32 copy of V
    int64_t ldv = 0;                // row stride of V (set by spmm_maxcut)
    void *Y = nullptr;              // output rows (C V, shifted for kEpiPlain)
    const void *R = nullptr;        // kEpiLS: R rows
    const void *aux = nullptr;      // kEpiLS: C R rows for p1 (nullable)
    const double *ytil = nullptr;   // kEpiPlain: shift (nullable); kEpiLS: ytil
    double *y = nullptr;            // kEpiRefresh: multipliers
    double *rn = nullptr;           // kEpiRefresh / kEpiLS: ||R_i||^2 out (nullable)
    double sigma = 0.0;             // kEpiRefresh: y <- y - sigma (rn - 1) if > 0; kEpiSplit: penalty
    double cs = 1.0;                // objective scale: the operator is cs C (re-optimisation)
    double *q1 = nullptr;           // kEpiLS: optional per-constraint outputs
    double *q2 = nullptr;
    int64_t ld = 0;
    double *partials = nullptr;     // per-block sums (kMaxSums stride)
    const SolverState *st = nullptr;  // if set, skip when st->done != 0
};

// MaxCut SpMM; returns status, *nparts = rows written in partials.
int spmm_maxcut(hipStream_t s, const DevCsr &P, int prec, const SpmmArgs &a, int *nparts);

// Completion SpMM Y = (I - A*(ytil)) V and SDDMMs.
int spmm_completion(hipStream_t s, const DevCompletion &P, int prec, const void *V, int64_t ld,
                    const double *ytil, void *Y);

// Row stride (elements) of the bfloat16 copy of an n x ld float32 array:
// ld rounded up to a multiple of 8 (16-byte rows).
inline int64_t bf16_ld(int64_t ld) { return (ld + 7) / 8 * 8; }

// number of sums per partial row of each stage
constexpr int kLsSums = 8;
constexpr int kRefSums = 4;

}  // namespace lrsdp
