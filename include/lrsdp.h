/*
 * lrsdp.h - C ABI of the MI355X (gfx950) low-rank SDP library.
 *
 * The library solves the linear SDP
 *
 *     min <C, X>   s.t.   A(X) = b,   X psd,   X = R R^T,  R in R^{n x r}
 *
 * (the problem statement of the paper's introduction, eq. prob:sdp, with the
 * Burer-Monteiro factorisation of Section 2.1) for two constraint families:
 *
 *   MaxCut      C = -L(G,w)/4, A(X) = diag(X), b = 1   (paper, MaxCut section)
 *   completion  C = I, A_k = E_{i,n1+j} + E_{n1+j,i}, b_k = 2 M_ij
 *               (paper, matrix-completion section)
 *
 * Multiplier convention (the paper's appendix A.2 and its error measures):
 *
 *     L(R; y, sigma) = <C,RR^T> + y^T (b - A(RR^T)) + sigma/2 ||b - A(RR^T)||^2
 *     ytil           = y + sigma (b - A(RR^T))
 *     grad_R L       = 2 (C - A*(ytil)) R,      multiplier update  y <- ytil
 *
 * (the introduction's  lambda <- lambda + rho (A(RR^T) - b)  is the same method
 * with lambda = -y and rho = sigma).
 *
 * Conventions for every call:
 *   - Return value: LRSDP_OK (0) or a negative LRSDP_E* code; lrsdp_last_error()
 *     returns a thread-local message for the last failing call.  No C++
 *     exception crosses the ABI.
 *   - "host" pointers are read (or written) during the call only and stay owned
 *     by the caller.  "device" pointers are caller-owned HIP device memory on
 *     the context's device; the library never frees them.
 *   - Device work is enqueued on the stream given to lrsdp_ctx_create.  Calls
 *     returning host results synchronise that stream; kernel entry points
 *     (lrsdp_k_*) only enqueue.
 *   - Factor matrices are row-major n x ld with ld >= r; element type is double
 *     (LRSDP_F64) or float (LRSDP_F32, LRSDP_F32_BF16IN).  Pad columns r..ld-1
 *     must hold zeros and are kept at zero.  ld * sizeof(element) must be a
 *     multiple of 16 bytes.
 *   - Handles are not thread-safe: use one context per host thread / stream.
 */
#ifndef LRSDP_H
#define LRSDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
#define LRSDP_OK              0
#define LRSDP_NOT_CONVERGED   1   /* solve stopped at a limit; result is valid   */
#define LRSDP_EINVAL         -1   /* invalid argument or malformed input data    */
#define LRSDP_ENOMEM         -2   /* caller buffer too small (message has size)  */
#define LRSDP_EHIP           -3   /* HIP runtime error                           */
#define LRSDP_ENUMERIC       -4   /* NaN/Inf met in a reduction                  */
#define LRSDP_EUNSUPPORTED   -5   /* valid request not supported by this build   */

/* ---- precisions (storage of R and the n x r work arrays) ------------------- */
#define LRSDP_F64          0   /* everything in float64                          */
#define LRSDP_F32          1   /* n x r arrays in float32, reductions in float64  */
#define LRSDP_F32_BF16IN   2   /* as F32, plus a bfloat16 shadow of the gathered
                                  SpMM operand (round-to-nearest-even)            */

/* ---- problem kinds --------------------------------------------------------- */
#define LRSDP_MAXCUT       1
#define LRSDP_COMPLETION   2
#define LRSDP_GENERAL      3

typedef struct lrsdp_ctx lrsdp_ctx;
typedef struct lrsdp_problem lrsdp_problem;

/* Last error message of the calling thread ("" if none). */
const char *lrsdp_last_error(void);

/* Library version string. */
const char *lrsdp_version(void);

/* ---- context ----------------------------------------------------------------
 * Binds a HIP device and a stream (hipStream_t passed as void*, NULL = the
 * default stream).  Allocates, once, a small device scratch area for reduction
 * partials and solver state, and a pinned host block for status read-back.
 * Errors: EINVAL (bad device), EHIP.
 */
int  lrsdp_ctx_create(int device, void *hip_stream, lrsdp_ctx **out);
void lrsdp_ctx_destroy(lrsdp_ctx *ctx);

/* ---- problems (host-side build) -------------------------------------------
 * MaxCut on an undirected graph with n nodes and n_edges edges (u[e], v[e]),
 * host int32 arrays; w = host float64 weights or NULL for unit weights.  Builds
 * the CSR of C = -L/4 (off-diagonal C_ij = w_ij/4, diagonal kept separately as
 * C_ii = -sum_j w_ij/4), b = 1.  Rejects (EINVAL) endpoints outside [0,n), self
 * loops, repeated edges and non-finite weights.  When every weight is +1 or -1
 * the values are stored implicitly in the column index.
 */
int lrsdp_problem_maxcut(int64_t n, int64_t n_edges, const int32_t *u,
                         const int32_t *v, const double *w,
                         lrsdp_problem **out);

/* Node order of a MaxCut problem (an implementation choice; the paper leaves
 * the order to the input).  LRSDP_ORDER_INPUT keeps the caller's labels
 * (lrsdp_problem_maxcut).  LRSDP_ORDER_DEGREE relabels the nodes inside the
 * library by decreasing degree, ties by increasing label: the rows of the factor
 * that the SpMM gathers most often then share cache lines.  The problem is the
 * same up to a symmetric permutation, so results agree with the input order up
 * to rounding.  lrsdp_solve, lrsdp_certify, lrsdp_warmstart, lrsdp_ws_features
 * and lrsdp_ws_targets take and return every per-node array (R, y, y0, features)
 * in the caller's labels; the per-kernel entry points (lrsdp_k_*) work in the
 * library's order and return EUNSUPPORTED for such a problem.  Arguments and
 * errors otherwise as lrsdp_problem_maxcut (EINVAL for another node_order). */
#define LRSDP_ORDER_INPUT  0
#define LRSDP_ORDER_DEGREE 1
int lrsdp_problem_maxcut_ex(int64_t n, int64_t n_edges, const int32_t *u, const int32_t *v,
                            const double *w, int node_order, lrsdp_problem **out);

/* Matrix completion: n1 x n2 matrix, m observed entries (i[k], j[k]) with values
 * Mij[k] (host arrays).  X has order n1 + n2, C = I, b_k = 2 Mij[k].  Rejects
 * (EINVAL) out-of-range or repeated (i, j) and non-finite values.
 */
int lrsdp_problem_completion(int64_t n1, int64_t n2, int64_t m,
                             const int32_t *i, const int32_t *j,
                             const double *Mij, lrsdp_problem **out);

/* General single-block problem: min <C, X> s.t. <A_k, X> = b_k (k < m), X psd
 * of order n, with sparse symmetric C and A_k given as triplets (host arrays).
 * C: c_nnz entries (c_row[t], c_col[t], c_val[t]); A: a_nnz entries
 * (a_con[t], a_row[t], a_col[t], a_val[t]) of constraint a_con[t].  Each
 * off-diagonal entry is given once, in either triangle, and stands for both
 * (r, c) and (c, r); repeated positions are summed.  The build compresses the
 * stacked constraint matrix to its nonzero columns (positions of the upper
 * triangle) and keeps the union Omega of those positions with the nonzeros of
 * C (Section 3.4): <A_k, X> = sum over a < b of A_k,ab (X_ab + X_ba) plus
 * sum_a A_k,aa X_aa, and the solve applies C - A*(y) as one sparse matrix on
 * Omega.  Rejects (EINVAL) indices out of range, non-finite values, and
 * n or |Omega| beyond int32.  The row-block H0 and the warm start are not
 * available for this kind (EUNSUPPORTED); the certificate's dual bound is NaN
 * (no bound on trace X is stated).
 */
int lrsdp_problem_general(int64_t n, int64_t c_nnz, const int32_t *c_row, const int32_t *c_col,
                          const double *c_val, int64_t m, int64_t a_nnz, const int32_t *a_con,
                          const int32_t *a_row, const int32_t *a_col, const double *a_val,
                          const double *b, lrsdp_problem **out);

/* Storage of C for general problems (Section 3.5, last paragraph: a small C
 * with many nonzeros is stored densely and applied with dense operators).
 * LRSDP_C_DENSE keeps C as an n x n float64 matrix (n <= 16384; n^2 * 8 bytes
 * of device memory): C V is a dense product (float64 matrix cores), Omega
 * holds only the nonzero columns of the stacked constraint matrix, and the
 * objective and line-search terms <C, U V^T> come from the rows of C V.
 * LRSDP_C_SPARSE keeps C on Omega.  LRSDP_C_AUTO (lrsdp_problem_general)
 * takes dense storage when n <= 8192 and at least 10% of the upper-triangle
 * positions of C are nonzero.  lrsdp_problem_info.c_dense reports the choice. */
#define LRSDP_C_AUTO   0
#define LRSDP_C_SPARSE 1
#define LRSDP_C_DENSE  2
int lrsdp_problem_general_ex(int64_t n, int64_t c_nnz, const int32_t *c_row, const int32_t *c_col,
                             const double *c_val, int64_t m, int64_t a_nnz, const int32_t *a_con,
                             const int32_t *a_row, const int32_t *a_col, const double *a_val,
                             const double *b, int c_storage, lrsdp_problem **out);

/* Several PSD blocks: min sum_j <C_j, X_j> s.t. sum_j <A_kj, X_j> = b_k, every
 * X_j psd of order block_n[j] (a block of order 1 is a nonnegative scalar).
 * Triplets as in lrsdp_problem_general with block-local indices and a block id
 * per triplet (c_blk, a_blk).  The blocks are laid out one after another in a
 * single factor R of order sum_j block_n[j] and one rank: the data touches no
 * position between two blocks, so the entries of RR^T outside the diagonal
 * blocks enter neither the objective nor the constraints, and RR^T psd makes
 * every block psd.  Row offset of block j = sum_{i<j} block_n[i].  EINVAL for
 * a bad block id or a local index outside its block.
 */
int lrsdp_problem_general_blocks(int64_t nblocks, const int64_t *block_n, int64_t c_nnz, const int32_t *c_blk,
                                 const int32_t *c_row, const int32_t *c_col, const double *c_val, int64_t m,
                                 int64_t a_nnz, const int32_t *a_con, const int32_t *a_blk, const int32_t *a_row,
                                 const int32_t *a_col, const double *a_val, const double *b,
                                 lrsdp_problem **out);

/* Rank of each block's factor in the multi-block case (appendix A.2: the exact
 * line search carries over to several blocks, X_j = R_j R_j^T, each R_j of its
 * own width block_rank[j]).  block_rank: host array of one entry per block of
 * lrsdp_problem_general_blocks (one entry for a problem from
 * lrsdp_problem_general), each >= 1.  In the stacked factor R of
 * a solve, the rows of block j keep columns < min(block_rank[j], rank) and hold
 * zeros in the others: lrsdp_solve sets those entries of the caller's R to zero
 * at its start, the gradient leaves them at zero, and dynamic rank growth adds
 * columns to a block's rows only up to its rank.  Call before the upload.
 * Errors: EINVAL (NULL, a rank < 1, already uploaded), EUNSUPPORTED (not a
 * general problem).
 */
int lrsdp_problem_block_ranks(lrsdp_problem *prob, const int32_t *block_rank);

void lrsdp_problem_destroy(lrsdp_problem *prob);

typedef struct {
    int     kind;        /* LRSDP_MAXCUT, LRSDP_COMPLETION or LRSDP_GENERAL      */
    int64_t n;           /* order of X                                           */
    int64_t m;           /* number of constraints                                */
    int64_t nnz;         /* stored off-diagonal nonzeros of the SpMM operator    */
    int64_t n1, n2;      /* completion block sizes (0 for MaxCut)                */
    int     weights;     /* MaxCut: 0 unit, 1 sign (+-1), 2 general               */
    int64_t max_row_nnz; /* longest row of the SpMM operator                     */
    double  c_l1;        /* ||vec(C)||_1                                         */
    double  b_l1;        /* ||b||_1                                              */
    double  b_inf;       /* ||b||_inf                                            */
    int     c_dense;     /* general problems: 1 when C is stored densely         */
    int     node_order;  /* MaxCut: LRSDP_ORDER_INPUT or LRSDP_ORDER_DEGREE      */
} lrsdp_problem_info;

int lrsdp_problem_get_info(const lrsdp_problem *prob, lrsdp_problem_info *out);

/* Bytes of device memory the problem occupies once uploaded. */
int lrsdp_problem_device_bytes(const lrsdp_problem *prob, size_t *bytes);

/* Copy the problem into caller-owned device memory `dev` of `bytes` bytes
 * (ENOMEM if smaller than lrsdp_problem_device_bytes; the message states the
 * size).  Synchronises the context stream.  `dev` must stay alive while the
 * problem is used.  A problem is uploaded to one context at a time.
 */
int lrsdp_problem_upload(lrsdp_ctx *ctx, lrsdp_problem *prob, void *dev,
                         size_t bytes);

/* ---- solver options ---------------------------------------------------------
 * Defaults (lrsdp_options_default): F64, T = 1 L-BFGS pair, tol = 1e-5,
 * sigma0 = 0 (selects 4 ||vec(C)||_1 / m), sigma_factor = 4, sigma_max_ratio =
 * 1e8, feas_decrease = 0.25, eta0 = 0.1, eta_factor = 0.25, eta_min = 1e-9,
 * max_outer = 300, max_inner = 1000, max_iter_total = 200000,
 * check_every = 8, time_limit_s = 1e30, refresh_every = 0 (off), phase2 = 0,
 * switch_err1 = 1e-3, admm_check = 10, max_admm = 5000, precond = 0,
 * rank_max = 0 (off), rank_trigger = 1000, rank_scale = 1e-2, rank_seed = 15049,
 * reopt = 0, reopt_factor = 0.1, max_reopt = 10, cert_iters = 300.
 * With re-optimisation the results (obj, dual, err3, sigma, y) are those of
 * the original problem: the last round's divided by its objective scale.
 */
typedef struct {
    int     prec;             /* LRSDP_F64 / LRSDP_F32 / LRSDP_F32_BF16IN      */
    int     rank;             /* r (columns of R actually used)                */
    int     ld;               /* row stride of R and work arrays (>= rank)     */
    int     lbfgs_mem;        /* T, 1..8                                       */
    double  tol;              /* stop when err1 <= tol and |err3| <= tol       */
    int     max_outer;
    int     max_inner;        /* L-BFGS iterations per ALM subproblem          */
    int64_t max_iter_total;
    double  time_limit_s;
    double  sigma0;           /* <= 0: 4 ||vec(C)||_1 / m                      */
    double  sigma_factor;     /* sigma growth when err1 stalls                 */
    double  sigma_max_ratio;  /* sigma <= sigma_max_ratio * sigma0             */
    double  feas_decrease;    /* stall test: err1 > feas_decrease * err1_prev  */
    double  eta0;             /* inner tolerance factor of the first subproblem*/
    double  eta_factor;
    double  eta_min;
    int     check_every;      /* L-BFGS iterations enqueued between host checks*/
    int     refresh_every;    /* recompute C R exactly every k inner iterations
                                 (0 = only at each ALM step)                   */
    int     profile;          /* 1: time SpMM launches with HIP events         */
    int     verbose;          /* 1: print one line per ALM step to stderr      */
    int     phase2;           /* 1: switch to the splitting (ADMM) phase of
                                 Section 2.2 once err1 <= switch_err1         */
    double  switch_err1;      /* ALM -> splitting threshold on err1            */
    int     admm_check;       /* splitting iterations between measure checks   */
    int     max_admm;         /* splitting iterations at most                  */
    int     precond;          /* 1: MaxCut L-BFGS with the row-block H0
                                 P^{-1}, P_i = h_i I + 4 sigma R_i R_i^T and
                                 h_i = 2 max(sum_j |C_ij|, 1e-3 ||vec(C)||_1 / n),
                                 in place of Algorithm 1's H0 = I (an extension;
                                 lbfgs_mem <= 2; EUNSUPPORTED for completion);
                                 2: the same with h_i = 2 max(C_ii - ytil_i,
                                 0.005 h_i of mode 1) at the current iterate    */
    int     rank_max;         /* dynamic rank (appendix A.1): after an ALM step
                                 whose L-BFGS run took >= rank_trigger
                                 iterations, rank <- min(ceil(1.5 rank),
                                 rank_max, ld, floor(sqrt(2m))); the new columns
                                 of R get rank_scale * N(0, 1) values; 0 or
                                 <= rank: off                                  */
    int     rank_trigger;     /* L-BFGS iterations of one subproblem that
                                 trigger a rank increase                       */
    double  rank_scale;       /* standard deviation of the new entries         */
    int64_t rank_seed;        /* seed of the new entries: entry (i, c) takes
                                 outputs 2k and 2k+1 (k = 65536 i + c) of the
                                 SplitMix64 sequence seeded with rank_seed, as
                                 uniforms u = ((x >> 11) + 0.5) 2^-53, through
                                 Box-Muller: sqrt(-2 ln u0) cos(2 pi u1)        */
    int     reopt;            /* re-optimisation level (Section 4.1).  0: off,
                                 the ALM runs until err1 <= tol and
                                 |err3| <= tol.  1 (mild): each round stops
                                 when err1 <= tol; if |err3| > tol on the
                                 original problem, a new round solves the
                                 problem with reopt_factor times the previous
                                 round's C, warm from its R, its y times
                                 reopt_factor and its penalty (inner tolerance
                                 restarted, no splitting phase after the first
                                 round).  2 (strict): as 1, and the final test
                                 also needs err2 <= tol, err2 from the
                                 estimated lower bound lambda_min - resid of a
                                 block Lanczos run (lrsdp_certify, at most
                                 cert_iters steps, residual target
                                 0.1 tol (1 + ||vec(C)||_1)) on C - A*(y)    */
    double  reopt_factor;     /* objective scale per round, 0 < f < 1          */
    int     max_reopt;        /* rounds after the first at most                */
    int     cert_iters;       /* reopt = 2: Lanczos steps per certificate      */
} lrsdp_options;

void lrsdp_options_default(lrsdp_options *opts);

typedef struct {
    double  obj;          /* <C, RR^T>                                         */
    double  dual;         /* b^T y                                             */
    double  err1;         /* ||A(X) - b||_2 / (1 + ||b||_1)                    */
    double  err1_inf;     /* ||A(X) - b||_2 / (1 + ||b||_inf)                  */
    double  err3;         /* (obj - dual) / (1 + |obj| + |dual|)               */
    double  sigma;        /* final penalty                                     */
    double  seconds;      /* wall time of the solve (host clock)               */
    int64_t outer;        /* ALM steps                                         */
    int64_t inner;        /* total L-BFGS iterations                           */
    int     status;       /* LRSDP_OK or LRSDP_NOT_CONVERGED                   */
    int     spmm_launches;/* profiled SpMM launches (profile = 1)              */
    double  spmm_ms;      /* summed duration of those launches (HIP events)    */
    double  spmm_bytes;   /* algorithmic bytes of one SpMM launch              */
    int64_t admm_iters;   /* splitting-phase iterations (phase2 = 1)           */
    int64_t admm_fallbacks; /* splitting phases abandoned (diverged: not finite
                               or err1 above 10x its value at the switch; or
                               max_admm reached): R, y and the ALM state of the
                               switch were restored and the ALM went on alone */
    int64_t rank_final;   /* rank at the end (differs from opts->rank when the
                             dynamic rank grew it)                             */
    int64_t reopt_rounds; /* re-optimisation rounds after the first (reopt >= 1)*/
    double  err2;         /* reopt = 2: err2 of the last certificate (from
                             lambda_lb); NaN when none was run                 */
} lrsdp_result;

/* Device workspace the solve needs for this problem and these options. */
int lrsdp_workspace_bytes(const lrsdp_problem *prob, const lrsdp_options *opts,
                          size_t *bytes);

/* Solve from the starting factor R (device, n x ld, element type of
 * opts->prec; overwritten with the final factor) and multipliers y (device,
 * m float64; in: y0, out: final y).  `ws` is caller-owned device memory of at
 * least lrsdp_workspace_bytes.  Blocking.  Returns LRSDP_OK when converged,
 * LRSDP_NOT_CONVERGED at a limit (res still filled), or an error code.
 * The algorithm: ALM (Section 2.1) whose subproblem is minimised by L-BFGS
 * (Algorithm 1, H0 = I; the row-block H0 with precond = 1) with the exact
 * quartic line search of appendix A.2.
 */
int lrsdp_solve(lrsdp_ctx *ctx, lrsdp_problem *prob, const lrsdp_options *opts,
                void *ws, size_t ws_bytes, void *R, double *y,
                lrsdp_result *res);

/* ---- kernel entry points (enqueue only; all pointers device) ----------------
 * `prec` selects the element type of the n x ld arrays as above.
 */

/* Y = (C - A*(ytil)) V  (eq. At of Section 3.4); ytil (m float64) may be NULL
 * (then Y = C V).  Y must not alias V.  With prec = LRSDP_F32_BF16IN (MaxCut
 * only) V is bfloat16 with row stride ld rounded up to a multiple of 8 and Y
 * is float32 with row stride ld; products accumulate in float32. */
int lrsdp_k_spmm(lrsdp_ctx *ctx, const lrsdp_problem *prob, int prec,
                 const void *V, int64_t ld, const double *ytil, void *Y);

/* out[k] = <A_k, U V^T> (m float64): the compressed outer product of Section
 * 3.4 (MaxCut: row dot U_i.V_i; completion: 2 U_i . V_{n1+j}; general: the
 * stacked constraint matrix times the outer products at the positions of
 * Omega).  V may be NULL (then V = U).  General problems use scratch inside
 * the problem's device memory: calls on one problem must not overlap. */
int lrsdp_k_constraint(lrsdp_ctx *ctx, const lrsdp_problem *prob, int prec,
                       const void *U, const void *V, int64_t ld, double *out);

/* Exact line-search coefficients of appendix A.2 for direction D at R with
 * multipliers y and penalty sigma.  out (device, 8 float64) receives
 * {a1, a2, a3, a4, p1, p2, ||q1||^2, ||q2||^2}; q1, q2 (device, m float64) may
 * be NULL or receive A(RD^T + DR^T) and A(DD^T).  `work` is device scratch of
 * at least 2*n*ld*(element bytes) + 16*m bytes. */
int lrsdp_k_ls_coeffs(lrsdp_ctx *ctx, const lrsdp_problem *prob, int prec,
                      const void *R, const void *D, int64_t ld,
                      const double *y, double sigma, void *work,
                      double *out, double *q1, double *q2);

/* Step tau >= 0 minimising a1 t^4 + a2 t^3 + a3 t^2 + a4 t over t > 0 (roots of
 * 4 a1 t^3 + 3 a2 t^2 + 2 a3 t + a4; the real root with the smallest quartic
 * value, smaller t on ties; 0 when no positive step decreases it).  a: device
 * 4 float64, tau: device 1 float64. */
int lrsdp_k_cubic(lrsdp_ctx *ctx, const double *a, double *tau);

/* ALM multiplier step and measures at R (Section 2.1; error measures of the
 * experimental setting): y <- y + sigma (b - A(RR^T)) when sigma > 0 (y left
 * unchanged when sigma == 0), then out (device, 8 float64) =
 * {obj, dual = b^T y, ||A(RR^T) - b||_2, err1, err1_inf, err3, 0, 0}.
 * `work` is device scratch of at least max(n*ld*(element bytes), 8*m) bytes
 * (MaxCut: receives C R; completion: receives A(RR^T)). */
int lrsdp_k_alm(lrsdp_ctx *ctx, const lrsdp_problem *prob, int prec,
                const void *R, int64_t ld, double *y, double sigma, void *work,
                double *out);

/* Allocation-free variant of lrsdp_k_alm, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid it): the same computation and outputs, with the work buffer taken
 * from a static device array of lrsdp_k_alm_noalloc_max_bytes() bytes (64 MiB)
 * that the library holds on each device from the first context created there
 * until the process ends.  The call itself allocates nothing.  ENOMEM (with
 * the sizes in the message) when max(n * ld * (element bytes), 8 * m) exceeds
 * the array.  All calls on one device share the array: calls that overlap on
 * one device (several streams or host threads) race; serialise them. */
int lrsdp_k_alm_noalloc(lrsdp_ctx *ctx, const lrsdp_problem *prob, int prec,
                        const void *R, int64_t ld, double *y, double sigma,
                        double *out);
size_t lrsdp_k_alm_noalloc_max_bytes(void);

/* `iters` splitting iterations (Section 2.2, eqs. 2.2-2.3) in place:
 * U <- argmin_U L(U, V, y), V <- argmin_V L(U, V, y), then
 * y <- y + sigma (b - A(U V^T)).  U, V device n x ld, y device m float64.
 * MaxCut: each half-step solved exactly per row (work unused, may be NULL).
 * Completion and general problems: each half-step solved by conjugate
 * gradients (Algorithm 2), C V formed once per half-step for a general C,
 * from the current iterate until ||r||_F <= cg_tol max(1, ||rhs||_F) or cg_max
 * steps; work: caller device memory, 256-byte aligned, of
 * lrsdp_admm_workspace_bytes; synchronises the stream (the CG scalars are
 * formed on the host).  ENUMERIC if CG meets non-positive curvature. */
int lrsdp_k_admm(lrsdp_ctx *ctx, const lrsdp_problem *prob, int prec, void *U, void *V, int64_t ld,
                 double *y, double sigma, int iters, double cg_tol, int cg_max,
                 void *work, size_t work_bytes);

/* Device workspace of lrsdp_k_admm: 0 for MaxCut; five n x ld arrays (six
 * for a general problem) and three m float64 vectors otherwise. */
int lrsdp_admm_workspace_bytes(const lrsdp_problem *prob, int prec, int64_t ld,
                               size_t *bytes);

/* Compact-form L-BFGS direction (Algorithm 1, H0 = I) for gradient G and k
 * pairs s_t = S[t], y_t = Y[t] (oldest first; S, Y: host arrays of k device
 * pointers each, k <= 8), all n x ld of the element type.  D = -H G, computed
 * as the two-loop recursion on the Gram matrix of {G, s_t, y_t}.  Synchronises
 * the stream (the Gram matrix is checked on the host); returns EINVAL if some
 * <y_t, s_t> <= 0. */
int lrsdp_k_lbfgs_dir(lrsdp_ctx *ctx, int prec, int64_t n, int64_t ld,
                      const void *G, const void *const *S, const void *const *Y,
                      int k, void *D);

/* ---- learned warm start (MaxCut) -------------------------------------------
 * The paper has no warm start; this is the project's extension: a per-node MLP
 * 16 -> 64 -> 64 -> 2 (tanh hidden layers; parameters laid out as W1[64][16],
 * b1[64], W2[64][64], b2[64], W3[2][64], b3[2]) maps 16 local graph features
 * of node i to (t_i, s_i); the warm start is y0_i = -t_i a_i / 4 with
 * a_i = sum_j |w_ij| and t_i limited to [-2, 2] (at an optimum y*_i =
 * -sum_j w_ij (1 - X*_ij) / 4 with |X*_ij| <= 1), and sigma0 = (default
 * sigma0) * exp(m / 2), m the mean of s_i limited to a caller-given range (the
 * range of the training labels): s predicts log(final penalty / default) of a
 * cold solve, and the warm start begins at the geometric mean of the default
 * and that penalty.  The default sigma0 is 4 ||vec(C)||_1 / m.
 * Parameters are float32 (LRSDP_PARAM_F32) or bfloat16 storage
 * (LRSDP_PARAM_BF16, widened exactly to float32 in the kernels; training keeps
 * a float32 master copy).  Activations and sums are float32.  Only MaxCut
 * problems are accepted (others: EUNSUPPORTED).
 */
#define LRSDP_PARAM_F32  0
#define LRSDP_PARAM_BF16 1

/* Number of parameters (5378). */
int lrsdp_mlp_param_count(void);

/* feat (device n x 16 float32, row-major) = node features of the problem's
 * graph; stats: device scratch of 4 float32 per node. */
int lrsdp_ws_features(lrsdp_ctx *ctx, const lrsdp_problem *prob, float *feat, float *stats);

/* Training targets from a solved problem: target (device n x 2 float32) =
 * (-4 y_i / a_i, log(sigma_final / default sigma0)) (first entry 0 for
 * isolated nodes); stats as filled by lrsdp_ws_features, y the solution
 * multipliers (device float64), sigma_final the penalty the cold solve ended
 * with (lrsdp_result.sigma; EINVAL unless positive and finite). */
int lrsdp_ws_targets(lrsdp_ctx *ctx, const lrsdp_problem *prob, const float *stats, const double *y,
                     double sigma_final, float *target);

/* out (device n x 2 float32) = MLP(feat); params of param_dtype. */
int lrsdp_mlp_forward(lrsdp_ctx *ctx, const void *params, int param_dtype, const float *feat, int64_t n,
                      float *out);

/* grad (device nparam float32) and *loss (device float64, may be NULL) of
 * L = (1/n) sum_i ||MLP(feat_i) - target_i||^2, target device n x 2 float32,
 * params of param_dtype.  work: device float32 scratch of 256 * (nparam + 1).
 * Deterministic (fixed-order sums, no atomics). */
int lrsdp_mlp_grad(lrsdp_ctx *ctx, const void *params, int param_dtype, const float *feat, const float *target,
                   int64_t n, float *grad, double *loss, float *work);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on
 * device arrays of nparam float32. */
int lrsdp_mlp_adam(lrsdp_ctx *ctx, float *params, float *m, float *v, const float *grad, int step, float lr);

/* Full-batch training: `steps` Adam steps numbered first_step, first_step + 1,
 * ...  Each step takes the gradient at the bfloat16 parameters params_bf16
 * (device nparam uint16), updates the float32 master copy `master` with the
 * moments m, v (device nparam float32 each, zero before step 1), and rounds
 * the master to params_bf16 (round to nearest even); params_bf16 is first set
 * from master.  feat / target: device n x 16 and n x 2 float32 (nodes of all
 * training graphs stacked).  work: device float32 scratch of
 * lrsdp_mlp_train_work_floats().  loss_hist: NULL or device float64 of
 * `steps` entries, the loss before each step.  Enqueued on the context
 * stream, no synchronisation. */
int lrsdp_mlp_train(lrsdp_ctx *ctx, float *master, uint16_t *params_bf16, float *m, float *v, const float *feat,
                    const float *target, int64_t n, int first_step, int steps, float lr, float *work,
                    double *loss_hist);
int lrsdp_mlp_train_work_floats(void);

/* ---- dual estimate (certificate) --------------------------------------------
 * Smallest eigenvalue of S = C - A*(y) (the dual slack of the error measures,
 * Section 4.2) by block Lanczos on the problem's own SpMM, blocks of 8
 * float64 vectors, no stored basis.  For any y, a lower bound lb on
 * lambda_min(S) gives a lower bound on the optimum: MaxCut (diag(X) = 1, so
 * trace X = n): b^T y + n min(0, lb); completion (C = I): b^T y / max(1, 1 - lb),
 * since 1 - lambda_min is the spectral norm of the n1 x n2 matrix of the y_k.
 * The library uses lb = (smallest Ritz value) - (its residual norm).  That is a
 * bound on the eigenvalue of S nearest the Ritz value; it bounds lambda_min
 * only if Lanczos has not missed a lower eigenvalue, which a Krylov method
 * cannot exclude.  The bound and the gap computed from it are therefore
 * estimates, not proofs.
 */
typedef struct {
    double  lambda_min;  /* smallest Ritz value of S (>= the true lambda_min)     */
    double  resid;       /* residual norm of that Ritz pair                       */
    double  lambda_lb;   /* lambda_min - resid: the value the bound uses          */
    double  dual_bound;  /* estimated lower bound on the optimum from y and
                            lambda_lb (see above)                                 */
    double  err2;        /* max(0, -lambda_min) / (1 + ||vec(C)||_1)              */
    double  by;          /* b^T y                                                 */
    int64_t iters;       /* block Lanczos steps taken                             */
    int     status;      /* 0: resid <= tol; 1: max_iter reached; 2: the Krylov
                            space became invariant (resid = 0, lambda exact up to
                            rounding)                                             */
    int     block;       /* block size (8)                                        */
    double  lambda_max;  /* largest Ritz value (<= the true lambda_max): with
                            lambda_min, a lower estimate of ||S||_2 against
                            which resid can be read                              */
} lrsdp_cert;

/* Device workspace for lrsdp_certify with at most max_iter steps:
 * 4 n x 8 float64 blocks, an n-vector (y in the library's node order), max_iter
 * KB and 0.3 MB of partial sums. */
int lrsdp_certify_workspace_bytes(const lrsdp_problem *prob, int max_iter,
                                  size_t *bytes);

/* Run block Lanczos on S = C - A*(y) (y: device float64, m entries) from a
 * seeded random start block until the residual of the smallest Ritz pair is
 * <= tol (absolute) or max_iter steps; checks every 10 steps.  work: caller
 * device memory, 256-byte aligned, of lrsdp_certify_workspace_bytes.
 * Synchronises the context stream.  Errors: EINVAL (arguments, not uploaded),
 * EUNSUPPORTED (n < 16), ENOMEM (workspace short), ENUMERIC (rank-deficient
 * start block or non-finite values).  The Ritz values are exact up to the loss
 * of orthogonality of the Lanczos basis (re-orthogonalised only against the two
 * previous blocks); the bound built on them is an estimate (above).  y is in
 * the caller's node labels for a problem relabelled by degree.
 */
int lrsdp_certify(lrsdp_ctx *ctx, const lrsdp_problem *prob, const double *y,
                  int max_iter, double tol, uint64_t seed, void *work,
                  size_t work_bytes, lrsdp_cert *out);

/* ---- proof of a lower bound (small problems, host) --------------------------
 * Proves lambda_min(S) >= lambda_lb for S = C - A*(y) (the dual slack of the
 * error measures, Section 4.2), which the Lanczos estimate above cannot: S -
 * shift I is formed densely on the host in float64 and factorised by
 * Cholesky.  If every pivot is positive, the rounding analysis of Cholesky
 * (computed factor R: R^T R = S' + E, |E| <= gamma_{n+1} |R^T||R|, gamma_k =
 * k u / (1 - k u), u = 2^-53; IEEE float64, no underflow) bounds ||E||_2 by
 * gamma_{n+1} ||R||_F^2; with a bound on the rounding of the formation of S'
 * this gives lambda_lb = shift - margin.  dual_bound: the bound on the optimum
 * of lrsdp_certify's formulas taken at lambda_lb and b^T y rounded down
 * (MaxCut, completion; NaN for a general problem).  The caller picks shift,
 * e.g. the Lanczos lambda_lb less a small allowance; a failed factorisation
 * (status 1) says S - shift I is not (numerically) positive definite, i.e. the
 * shift is too high.  Host work only: O(n^3 / 6) multiply-adds (the rows of a
 * 64-row block left of the block on up to 16 host threads, the same
 * operations per entry as one thread) and up to 4.5 n^2 doubles of host memory
 * while S' is formed (2.4 GB at n = 8192), 2 n^2 after; the problem need not be
 * uploaded.  y: host float64,
 * m entries, in the caller's node labels.  Errors: EINVAL (NULL, shift or y
 * not finite), EUNSUPPORTED (n > LRSDP_PROOF_MAX_N).
 */
#define LRSDP_PROOF_MAX_N 8192
typedef struct {
    double  shift;       /* the shift tried                                      */
    double  lambda_lb;   /* status 0: proven lower bound on lambda_min(S)        */
    double  margin;      /* shift - lambda_lb: the rounding allowance            */
    double  dual_bound;  /* status 0: proven lower bound on the optimum          */
    double  by;          /* b^T y as computed                                    */
    int64_t pivot;       /* status 1: index of the first non-positive pivot      */
    int     status;      /* 0: proven; 1: the factorisation failed (no bound)    */
    int     reserved;
} lrsdp_proof;
int lrsdp_certify_dense(const lrsdp_problem *prob, const double *y, double shift,
                        lrsdp_proof *out);

/* Warm start for the problem: y0 (device m float64) and *sigma0 (host), with
 * the mean penalty output limited to [log_ratio_lo, log_ratio_hi] (EINVAL if
 * empty or not finite).  params of param_dtype.  work: device float32 scratch
 * of 22 n.  Synchronises the stream.  Returns LRSDP_ENUMERIC (y0 contents then
 * undefined, *sigma0 untouched) when any predicted multiplier or the penalty
 * is not finite; the caller then solves from the cold start. */
int lrsdp_warmstart(lrsdp_ctx *ctx, const lrsdp_problem *prob, const void *params, int param_dtype,
                    double log_ratio_lo, double log_ratio_hi, float *work, double *y0, double *sigma0);

#ifdef __cplusplus
}
#endif

#endif /* LRSDP_H */
