// C ABI: context, options, device-resident solve driver, kernel entry points.
//
// The solve (Section 2.1 ALM, Algorithm 1 L-BFGS, appendix A.2 exact line
// search) runs entirely on the device.  Per L-BFGS iteration the host enqueues
//   spmm(LS)  -> ls_finalize -> update -> lbfgs_finalize -> combine
// and reads the 3 KB state block back every `check_every` iterations.  Each
// kernel returns at once when the state says the subproblem is finished, so
// the iterations enqueued past convergence cost only their launches.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>

#include "kernels.h"

namespace lrsdp {

int launch_ls_finalize(hipStream_t, SolverState *, const double *, int, const double *, int, int, double);
int launch_lbfgs_finalize(hipStream_t, SolverState *, const double *, int);
int launch_init_finalize(hipStream_t, SolverState *, const double *, int, int);
int launch_alm_finalize(hipStream_t, SolverState *, const double *, int, int, double);
int launch_dscale(hipStream_t, double *, double, int64_t);
int launch_reduce(hipStream_t, const double *, int, int, double *);
int launch_cubic(hipStream_t, const double *, double *);
int launch_update_maxcut(hipStream_t, int, SolverState *, void *, const void *, const double *, const double *,
                         const double *, const double *, const double *, double *, void *const *, void *const *,
                         int, int64_t, int64_t, double *, double *, int *, const PcBufs * = nullptr);
int launch_combine(hipStream_t, int, SolverState *, const double *, const void *const *, int, void *, int64_t,
                   int64_t, double *, double *, int *, uint16_t *, const void * = nullptr, const PcBufs * = nullptr);
int launch_grad_init_maxcut(hipStream_t, int, SolverState *, const void *, const void *, const double *,
                            const double *, double *, void *, int64_t, int64_t, double *, int *,
                            const PcBufs * = nullptr);
int launch_fill(hipStream_t, int, void *, int64_t);
int launch_rank_grow(hipStream_t, int, void *, int64_t, int64_t, int, int, uint64_t, double, const int32_t *);
int launch_avg(hipStream_t, int, const void *, const void *, void *, int64_t);
int launch_dots(hipStream_t, int, const void *, const void *const *, int, int64_t, int64_t, double *, int *);
int launch_rowdot(hipStream_t, int, const void *, const void *, int64_t, int64_t, double *);
int launch_ytil(hipStream_t, const double *, const double *, const double *, double, int64_t, double *);
int launch_ls_out(hipStream_t, const double *, double, double *);
int launch_alm_out(hipStream_t, const double *, double, double, double *);
int launch_two_loop_pairs(hipStream_t, const double *, int, double *, int *);
int launch_gather_gram(hipStream_t, const double *, int, int, double *);
int launch_ls_out_cmp(hipStream_t, const double *, const double *, double, double *);
int cmp_grad(hipStream_t, const DevCompletion &, int, const SolverState *, const void *, const double *,
             void *const *, void *const *, int, int64_t, double *, int, int *, double);
int cmp_sddmm(hipStream_t, const DevCompletion &, int, int, const void *, const void *, int64_t, double *, double *,
              double *, const double *, double *, double, double *, const SolverState *, int *);
int cmp_samples(hipStream_t, const DevCompletion &, const SolverState *, double *, const double *, const double *,
                const double *, double *);
int cmp_ytil(hipStream_t, const DevCompletion &, const SolverState *, double, const double *, const double *,
             double *);
int axpy_state(hipStream_t, int, const SolverState *, void *, const void *, int64_t, int64_t);
int gen_sddmm(hipStream_t, const DevGeneral &, int, int, const void *, const void *, int64_t, double *, double *,
              double *, const double *, double *, double, double, double *, const SolverState *, int *,
              bool dense_sums = true);
int gen_grad(hipStream_t, const DevGeneral &, int, const SolverState *, const void *, const double *, void *const *,
             void *const *, int, int64_t, double *, int, int *, double);
int gen_rank_mask(hipStream_t, const DevGeneral &, int, void *, int64_t);

namespace {

// ctx scratch layout (bytes)
constexpr size_t kStateOff = 0;
constexpr size_t kPartRows = 2 * kMaxBlocks;                 // rows per partials set
constexpr size_t kPartBytes = kPartRows * kMaxSums * sizeof(double);
constexpr size_t kPartLsOff = 8192;
constexpr size_t kPartCbOff = kPartLsOff + kPartBytes;
constexpr size_t kPartUpOff = kPartCbOff + kPartBytes;
constexpr size_t kPartMiscOff = kPartUpOff + kPartBytes;
constexpr size_t kSmallOff = kPartMiscOff + kPartBytes;      // 4096 doubles of small buffers
constexpr size_t kL1Off = kSmallOff + 4096 * sizeof(double);  // first-level sums of the flat sweeps
constexpr size_t kScratchBytes = kL1Off + kL1Bytes;

template <typename T>
T *at(void *base, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

int elem_size(int prec) { return prec == LRSDP_F64 ? 8 : 4; }

int check_prec(int prec) {
    if (prec != LRSDP_F64 && prec != LRSDP_F32 && prec != LRSDP_F32_BF16IN)
        return set_error(LRSDP_EINVAL, "unknown precision %d", prec);
    return LRSDP_OK;
}

int check_ld(int prec, int64_t ld) {
    const int64_t rb = ld * elem_size(prec);
    if (ld <= 0 || rb % 16 != 0 || rb > 256)
        return set_error(LRSDP_EINVAL, "ld = %lld: ld * element size must be a positive multiple of 16, at most 256",
                         (long long)ld);
    return LRSDP_OK;
}

// The per-kernel entry points take per-node arrays in the library's order,
// which is the caller's only for problems built in input order.
static int check_input_order(const lrsdp_problem *p) {
    if (p->csr.perm)
        return set_error(LRSDP_EUNSUPPORTED,
                         "the per-kernel entry points need a problem in input order (LRSDP_ORDER_INPUT); this "
                         "one is relabelled by degree");
    return LRSDP_OK;
}

int check_problem(const lrsdp_problem *p) {
    if (!p) return set_error(LRSDP_EINVAL, "problem is NULL");
    if (!p->uploaded) return set_error(LRSDP_EINVAL, "problem has not been uploaded");
    return LRSDP_OK;
}

// Default initial penalty: 4 ||vec(C)||_1 / m (floored at 1e-8).
double default_sigma0(const lrsdp_problem *p) {
    return std::max(4.0 * p->info.c_l1 / (double)p->info.m, 1e-8);
}

// Algorithmic bytes of one MaxCut line-search SpMM launch (each array once):
// work list + row pointers + column indices (+ values) + gathered D + own rows
// of R and D read once + C D written + ytil + diagonal.
double maxcut_spmm_bytes(const lrsdp_problem *p, int prec, int r) {
    const double n = (double)p->info.n, nnz = (double)p->info.nnz, w = elem_size(prec);
    double b = 4.0 * n + 4.0 * (n + 1) + 4.0 * nnz + 16.0 * n + 3.0 * n * r * w;
    if (p->info.weights == kWGeneral) b += 8.0 * nnz;
    return b;
}

// Algorithmic bytes of one completion gradient SpMM launch: row pointers, per
// entry partner index + sample id + ytil, R read, G written, and the 2T ring
// slots read for the dot products.
double completion_grad_bytes(const lrsdp_problem *p, int prec, int r, int T) {
    const double n = (double)p->info.n, m = (double)p->info.m, w = elem_size(prec);
    return 4.0 * (n + 2) + 2.0 * m * 16.0 + (2.0 + 2.0 * T) * n * r * w;
}

// Algorithmic bytes of one general-problem gradient SpMM launch: row pointers,
// per stored entry its column, position and C value, the transposed stacked
// matrix and ytil once, R read, G written, the 2T ring slots read.
double general_grad_bytes(const lrsdp_problem *p, int prec, int r, int T) {
    const double n = (double)p->info.n, nnz = (double)p->info.nnz, w = elem_size(prec);
    const double nom = (double)p->gen.nom, na = (double)p->gen.nnz_a, m = (double)p->info.m;
    return 4.0 * (n + 1) + 8.0 * nnz + 12.0 * nom + 12.0 * na + 8.0 * m + (2.0 + 2.0 * T) * n * r * w;
}

}  // namespace
}  // namespace lrsdp

using namespace lrsdp;

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int lrsdp_ctx_create(int device, void *hip_stream, lrsdp_ctx **out) {
    clear_error();
    if (!out) return set_error(LRSDP_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    LRSDP_HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return set_error(LRSDP_EINVAL, "device %d not in [0, %d)", device, count);
    LRSDP_HIP_TRY(hipSetDevice(device));
    auto *c = new lrsdp_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->scratch_bytes = kScratchBytes;
    c->pinned_bytes = 8192;
    hipError_t e = hipMalloc(&c->scratch, c->scratch_bytes);
    if (e == hipSuccess) e = hipHostMalloc(&c->pinned, c->pinned_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&c->ev0);
    if (e == hipSuccess) e = hipEventCreate(&c->ev1);
    if (e == hipSuccess) e = hipMemsetAsync(c->scratch, 0, c->scratch_bytes, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        lrsdp_ctx_destroy(c);
        return set_error(LRSDP_EHIP, "context setup failed: %s", hipGetErrorString(e));
    }
    int rc = noalloc_init(device, &c->static_scratch);
    if (rc) {
        lrsdp_ctx_destroy(c);
        return rc;
    }
    *out = c;
    return LRSDP_OK;
}

extern "C" void lrsdp_ctx_destroy(lrsdp_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    if (c->ev0) hipEventDestroy(c->ev0);
    if (c->ev1) hipEventDestroy(c->ev1);
    if (c->scratch) hipFree(c->scratch);
    if (c->pinned) hipHostFree(c->pinned);
    delete c;
}

// ---------------------------------------------------------------------------
// options / workspace
// ---------------------------------------------------------------------------
extern "C" void lrsdp_options_default(lrsdp_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->prec = LRSDP_F64;
    o->rank = 0;
    o->ld = 0;
    o->lbfgs_mem = 1;
    o->tol = 1e-5;
    o->max_outer = 300;
    o->max_inner = 1000;
    o->max_iter_total = 200000;
    o->time_limit_s = 1e30;
    o->sigma0 = 0.0;
    o->sigma_factor = 4.0;
    o->sigma_max_ratio = 1e8;
    o->feas_decrease = 0.25;
    o->eta0 = 1e-1;
    o->eta_factor = 0.25;
    o->eta_min = 1e-9;
    o->check_every = 8;
    o->refresh_every = 0;
    o->profile = 0;
    o->verbose = 0;
    o->phase2 = 0;
    o->switch_err1 = 1e-3;
    o->admm_check = 10;
    o->max_admm = 5000;
    o->precond = 0;
    o->rank_max = 0;
    o->rank_trigger = 1000;
    o->rank_scale = 1e-2;
    o->rank_seed = 15049;
    o->reopt = 0;
    o->reopt_factor = 0.1;
    o->max_reopt = 10;
    o->cert_iters = 300;
}

namespace {

struct WsPlan {
    size_t cd, gring[kMaxMem + 1], dring[kMaxMem], ytil[2], rn, q1, q2, acon, shadow, rho, kap, hdyn, cadmm, csnap,
        yorig, cert, cert_bytes, total;
};

int plan_workspace(const lrsdp_problem *p, const lrsdp_options *o, WsPlan *w) {
    if (!p || !o) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc = check_prec(o->prec);
    if (rc) return rc;
    if (o->lbfgs_mem < 1 || o->lbfgs_mem > kMaxMem)
        return set_error(LRSDP_EINVAL, "lbfgs_mem = %d not in [1, %d]", o->lbfgs_mem, kMaxMem);
    if (o->rank < 1 || o->ld < o->rank) return set_error(LRSDP_EINVAL, "need 1 <= rank <= ld");
    rc = check_ld(o->prec, o->ld);
    if (rc) return rc;
    if (o->precond < 0 || o->precond > 2) return set_error(LRSDP_EINVAL, "precond = %d not in {0, 1, 2}", o->precond);
    if (o->reopt < 0 || o->reopt > 2) return set_error(LRSDP_EINVAL, "reopt = %d not in {0, 1, 2}", o->reopt);
    if (o->reopt && (!(o->reopt_factor > 0.0) || !(o->reopt_factor < 1.0) || o->max_reopt < 0))
        return set_error(LRSDP_EINVAL, "re-optimisation needs 0 < reopt_factor < 1 and max_reopt >= 0");
    if (o->reopt == 2 && o->cert_iters < 1) return set_error(LRSDP_EINVAL, "reopt = 2 needs cert_iters >= 1");
    if (o->reopt == 2 && p->info.n < 16)
        return set_error(LRSDP_EUNSUPPORTED, "reopt = 2 needs the certificate, which needs n >= 16");
    if (o->precond) {
        if (p->info.kind != LRSDP_MAXCUT)
            return set_error(LRSDP_EUNSUPPORTED, "precond (row-block H0) is for MaxCut problems");
        if (o->lbfgs_mem > kPcMem)
            return set_error(LRSDP_EINVAL, "precond needs lbfgs_mem <= %d (got %d)", kPcMem, o->lbfgs_mem);
    }
    const size_t arr = (size_t)p->info.n * o->ld * elem_size(o->prec);
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t r = (off + 255) & ~size_t(255);
        off = r + b;
        return r;
    };
    w->cd = take(arr);
    for (int g = 0; g <= o->lbfgs_mem; ++g) w->gring[g] = take(arr);
    for (int d = 0; d < o->lbfgs_mem; ++d) w->dring[d] = take(arr);
    w->ytil[0] = take((size_t)p->info.m * 8);
    w->ytil[1] = take((size_t)p->info.m * 8);
    w->rn = take((size_t)p->info.n * 8);
    w->q1 = take((size_t)p->info.m * 8);
    w->q2 = take((size_t)p->info.m * 8);
    w->acon = take((size_t)p->info.m * 8);
    w->shadow = take(o->prec == LRSDP_F32_BF16IN ? (size_t)p->info.n * bf16_ld(o->ld) * 2 : 0);
    w->rho = take(o->precond ? (size_t)(o->lbfgs_mem + 1) * p->info.n * 8 : 0);
    w->kap = take(o->precond ? (size_t)p->info.n * 8 : 0);
    w->hdyn = take(o->precond == 2 ? (size_t)p->info.n * 8 : 0);
    // completion / general splitting phase: CG scratch (five n x ld arrays, six
    // for a general problem, three m-vectors; the layout of cmp_admm_layout) and
    // the copy of R kept for the fallback
    const bool cph2 = o->phase2 && (p->info.kind == LRSDP_COMPLETION || p->info.kind == LRSDP_GENERAL);
    const size_t arr256 = (arr + 255) / 256 * 256, vec256 = ((size_t)p->info.m * 8 + 255) / 256 * 256;
    w->cadmm = take(cph2 ? (p->info.kind == LRSDP_GENERAL ? 6 : 5) * arr256 + 3 * vec256 : 0);
    w->csnap = take(cph2 ? arr : 0);
    // strict re-optimisation: multipliers of the original problem and the
    // certificate's workspace
    w->cert_bytes = 0;
    if (o->reopt == 2 && (rc = lrsdp_certify_workspace_bytes(p, o->cert_iters, &w->cert_bytes))) return rc;
    w->yorig = take(o->reopt == 2 ? (size_t)p->info.m * 8 : 0);
    w->cert = take(w->cert_bytes);
    w->total = off + 256;
    return LRSDP_OK;
}

}  // namespace

extern "C" int lrsdp_workspace_bytes(const lrsdp_problem *p, const lrsdp_options *o, size_t *bytes) {
    clear_error();
    if (!bytes) return set_error(LRSDP_EINVAL, "bytes is NULL");
    WsPlan w;
    int rc = plan_workspace(p, o, &w);
    if (rc) return rc;
    *bytes = w.total;
    return LRSDP_OK;
}

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------
namespace {

int read_state(lrsdp_ctx *c, SolverState *h) {
    SolverState *d = at<SolverState>(c->scratch, kStateOff);
    LRSDP_HIP_TRY(hipMemcpyAsync(c->pinned, d, sizeof(SolverState), hipMemcpyDeviceToHost, c->stream));
    LRSDP_HIP_TRY(hipStreamSynchronize(c->stream));
    std::memcpy(h, c->pinned, sizeof(SolverState));
    return LRSDP_OK;
}

int write_state(lrsdp_ctx *c, const SolverState &h) {
    SolverState *d = at<SolverState>(c->scratch, kStateOff);
    std::memcpy(c->pinned, &h, sizeof(SolverState));
    LRSDP_HIP_TRY(hipMemcpyAsync(d, c->pinned, sizeof(SolverState), hipMemcpyHostToDevice, c->stream));
    LRSDP_HIP_TRY(hipStreamSynchronize(c->stream));
    return LRSDP_OK;
}

// One splitting iteration for MaxCut (Section 2.2): U-step from V, V-step from
// U with the multiplier step fused into its epilogue.
int admm_iter(hipStream_t s, const DevCsr &P, int prec, void *U, void *V, int64_t ld, double *y, double sigma) {
    int np = 0, rc;
    SpmmArgs a;
    a.epi = kEpiSplit;
    a.V = V;
    a.Y = U;
    a.y = y;
    a.sigma = sigma;
    a.ld = ld;
    if ((rc = spmm_maxcut(s, P, prec, a, &np))) return rc;
    a.V = U;
    a.Y = V;
    a.R = U;
    return spmm_maxcut(s, P, prec, a, &np);
}

// ---------------------------------------------------------------------------
// Splitting iteration for matrix completion and general problems (Section
// 2.2, eqs. 2.2-2.3): each half-step solves the positive definite system of
// eq. 2.2,
//   A_V(U) = sigma A*(A(U V^T)) V + sigma U = B_V = -C V + A*(y) V + sigma A*(b) V + sigma V,
// by conjugate gradients (Algorithm 2) warm-started at the current U, until
// ||r||_F <= cg_tol max(1, ||B_V||_F).  With S(V, z) = (C - A*(z)) V (the
// completion SpMM with C = I, or the general SpMM on Omega):
// B_V = sigma V - S(V, y + sigma b) and
// A_V(X) = sigma (C V - S(V, A(X V^T))) + sigma X, where C V = S(V, 0) is formed
// once per half-step (C V = V for completion).  The vector updates are combine
// passes (coefficients from the host, dots back to the host).
// ---------------------------------------------------------------------------
struct CmpAdmmBufs {
    void *B, *r, *p, *q, *S;   // n x ld
    void *CV;                   // n x ld: C V of the half-step's fixed factor (general problems; V itself for C = I)
    double *z, *w, *zero;       // m
};

// General problems keep one more n x ld array (C V).
size_t cmp_admm_bytes(const lrsdp_problem *p, int prec, int64_t ld) {
    const size_t arr = ((size_t)p->info.n * ld * elem_size(prec) + 255) / 256 * 256;
    const size_t vec = ((size_t)p->info.m * 8 + 255) / 256 * 256;
    return (p->info.kind == LRSDP_GENERAL ? 6 : 5) * arr + 3 * vec;
}

CmpAdmmBufs cmp_admm_layout(const lrsdp_problem *p, int prec, int64_t ld, char *work) {
    const size_t arr = ((size_t)p->info.n * ld * elem_size(prec) + 255) / 256 * 256;
    const size_t vec = ((size_t)p->info.m * 8 + 255) / 256 * 256;
    const int na = p->info.kind == LRSDP_GENERAL ? 6 : 5;
    CmpAdmmBufs b;
    b.B = work;
    b.r = work + arr;
    b.p = work + 2 * arr;
    b.q = work + 3 * arr;
    b.S = work + 4 * arr;
    b.CV = na == 6 ? work + 5 * arr : nullptr;
    b.z = reinterpret_cast<double *>(work + na * arr);
    b.w = reinterpret_cast<double *>(work + na * arr + vec);
    b.zero = reinterpret_cast<double *>(work + na * arr + 2 * vec);
    return b;
}

// The per-constraint kernels see only m and b: a general problem passes them
// through a completion view.
DevCompletion constraint_view(const lrsdp_problem *p) {
    if (p->info.kind == LRSDP_COMPLETION) return p->cmp;
    DevCompletion v{};
    v.m = p->info.m;
    v.b = p->gen.b;
    return v;
}

// out = A(X V^T) (completion SDDMM or the general compressed outer product)
int split_constraint(lrsdp_ctx *c, const lrsdp_problem *p, int prec, const void *X, const void *V, int64_t ld,
                     double *out) {
    int nb = 0;
    if (p->info.kind == LRSDP_GENERAL)
        return gen_sddmm(c->stream, p->gen, prec, 0, X, V, ld, out, nullptr, nullptr, nullptr, nullptr, 0.0, 1.0,
                         nullptr, nullptr, &nb);
    return cmp_sddmm(c->stream, p->cmp, prec, 0, X, V, ld, out, nullptr, nullptr, nullptr, nullptr, 0.0, nullptr,
                     nullptr, &nb);
}

// Y = (C - A*(z)) V
int split_spmm(lrsdp_ctx *c, const lrsdp_problem *p, int prec, const void *V, int64_t ld, const double *z, void *Y) {
    if (p->info.kind == LRSDP_GENERAL) return spmm_general(c->stream, p->gen, prec, V, ld, z, Y);
    return spmm_completion(c->stream, p->cmp, prec, V, ld, z, Y);
}

// out = sum_j coef_j basis_j; sums[j] = <out, basis_j>, sums[kMaxBasis] = ||out||^2 (host).
// Synchronises the stream.
int cmp_lincomb(lrsdp_ctx *c, int prec, std::initializer_list<const void *> basis, std::initializer_list<double> coef,
                void *out, int64_t n, int64_t ld, double *sums) {
    const void *bs[kMaxBasis];
    double *dcoef = at<double>(c->scratch, kSmallOff);
    double *dred = at<double>(c->scratch, kSmallOff) + 64;
    double *part = at<double>(c->scratch, kPartMiscOff);
    double *hc = reinterpret_cast<double *>(static_cast<char *>(c->pinned) + 6144);
    int nb = 0;
    for (const void *b : basis) bs[nb++] = b;
    int k = 0;
    for (double v : coef) hc[k++] = v;
    LRSDP_HIP_TRY(hipMemcpyAsync(dcoef, hc, nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
    int nblk = 0, rc;
    double *l1 = at<double>(c->scratch, kL1Off);
    if ((rc = launch_combine(c->stream, prec, nullptr, dcoef, bs, nb, out, n, ld, part, l1, &nblk, nullptr))) return rc;
    if ((rc = launch_reduce(c->stream, part, nblk, kMaxBasis + 1, dred))) return rc;
    double *hr = reinterpret_cast<double *>(static_cast<char *>(c->pinned) + 6656);
    LRSDP_HIP_TRY(hipMemcpyAsync(hr, dred, (kMaxBasis + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LRSDP_HIP_TRY(hipStreamSynchronize(c->stream));
    std::memcpy(sums, hr, (kMaxBasis + 1) * sizeof(double));
    return LRSDP_OK;
}

// out = A_V(X) = sigma A*(A(X V^T)) V + sigma X = sigma (C V - S(V, A(X V^T))) + sigma X
// (sums as cmp_lincomb; sums[2] = <out, X>).  cv: C V (V itself for C = I).
int cmp_split_apply(lrsdp_ctx *c, const lrsdp_problem *p, int prec, const void *X, const void *V, const void *cv,
                    int64_t ld, double sigma, const CmpAdmmBufs &b, void *out, double *sums) {
    int rc;
    if ((rc = split_constraint(c, p, prec, X, V, ld, b.z))) return rc;
    if ((rc = split_spmm(c, p, prec, V, ld, b.z, b.S))) return rc;
    return cmp_lincomb(c, prec, {cv, b.S, X}, {sigma, -sigma, sigma}, out, p->info.n, ld, sums);
}

// U <- argmin of the half-step (CG from the current U); returns CG iterations in *its
int cmp_split_half(lrsdp_ctx *c, const lrsdp_problem *p, int prec, void *U, const void *V, int64_t ld,
                   const double *y, double sigma, double cg_tol, int cg_max, const CmpAdmmBufs &b, int *its) {
    const int64_t n = p->info.n;
    double sums[kMaxBasis + 1];
    int rc;
    const DevCompletion cview = constraint_view(p);
    // C V: V itself when C = I, else (C - A*(0)) V once for the half-step
    const void *cv = V;
    if (b.CV) {
        if ((rc = split_spmm(c, p, prec, V, ld, b.zero, b.CV))) return rc;
        cv = b.CV;
    }
    if ((rc = cmp_ytil(c->stream, cview, nullptr, sigma, b.zero, y, b.w))) return rc;     // w = y + sigma b
    if ((rc = split_spmm(c, p, prec, V, ld, b.w, b.S))) return rc;
    if ((rc = cmp_lincomb(c, prec, {V, b.S}, {sigma, -1.0}, b.B, n, ld, sums))) return rc;
    const double eps = cg_tol * std::max(1.0, std::sqrt(std::max(sums[kMaxBasis], 0.0)));
    if ((rc = cmp_split_apply(c, p, prec, U, V, cv, ld, sigma, b, b.q, sums))) return rc;
    if ((rc = cmp_lincomb(c, prec, {b.B, b.q}, {1.0, -1.0}, b.r, n, ld, sums))) return rc;
    double rr = sums[kMaxBasis];
    if ((rc = cmp_lincomb(c, prec, {b.r}, {1.0}, b.p, n, ld, sums))) return rc;
    int k = 0;
    for (; k < cg_max; ++k) {
        if (!(std::sqrt(std::max(rr, 0.0)) > eps)) break;
        if ((rc = cmp_split_apply(c, p, prec, b.p, V, cv, ld, sigma, b, b.q, sums))) return rc;
        const double pq = sums[2];
        if (!(pq > 0.0) || !std::isfinite(pq)) return set_error(LRSDP_ENUMERIC, "splitting CG lost positive curvature");
        const double alpha = rr / pq;
        if ((rc = cmp_lincomb(c, prec, {U, b.p}, {1.0, alpha}, U, n, ld, sums))) return rc;
        if ((rc = cmp_lincomb(c, prec, {b.r, b.q}, {1.0, -alpha}, b.r, n, ld, sums))) return rc;
        const double rr_new = sums[kMaxBasis];
        const double beta = rr_new / rr;
        rr = rr_new;
        if ((rc = cmp_lincomb(c, prec, {b.r, b.p}, {1.0, beta}, b.p, n, ld, sums))) return rc;
    }
    *its = k;
    return LRSDP_OK;
}

// One completion splitting iteration: U-step, V-step, y <- y + sigma (b - A(U V^T)).
int cmp_admm_iter(lrsdp_ctx *c, const lrsdp_problem *p, int prec, void *U, void *V, int64_t ld, double *y,
                  double sigma, double cg_tol, int cg_max, const CmpAdmmBufs &b) {
    int its = 0, rc;
    if ((rc = cmp_split_half(c, p, prec, U, V, ld, y, sigma, cg_tol, cg_max, b, &its))) return rc;
    if ((rc = cmp_split_half(c, p, prec, V, U, ld, y, sigma, cg_tol, cg_max, b, &its))) return rc;
    if ((rc = split_constraint(c, p, prec, U, V, ld, b.z))) return rc;
    return cmp_ytil(c->stream, constraint_view(p), nullptr, sigma, b.z, y, y);
}

int solve_impl(lrsdp_ctx *c, lrsdp_problem *p, const lrsdp_options *o, char *ws, void *R, double *y,
               lrsdp_result *res) {
    const bool mc = p->info.kind == LRSDP_MAXCUT;
    const bool gen = p->info.kind == LRSDP_GENERAL;
    const bool cmp = p->info.kind == LRSDP_COMPLETION;
    // per-constraint kernels (acon, ytil updates) of the sample families see
    // only m and b: a general problem passes them through a completion view
    DevCompletion gview{};
    gview.m = p->info.m;
    gview.b = p->gen.b;
    const DevCompletion &cv = gen ? gview : p->cmp;
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    const int prec = o->prec == LRSDP_F64 ? LRSDP_F64 : LRSDP_F32;
    const int T = o->lbfgs_mem;
    const int64_t n = p->info.n, ld = o->ld;
    hipStream_t s = c->stream;
    WsPlan w;
    int rc = plan_workspace(p, o, &w);
    if (rc) return rc;
    void *CD = ws + w.cd;
    void *gring[kMaxMem + 1] = {};
    void *dring[kMaxMem] = {};
    for (int g = 0; g <= T; ++g) gring[g] = ws + w.gring[g];
    for (int d = 0; d < T; ++d) dring[d] = ws + w.dring[d];
    double *ytil[2] = {reinterpret_cast<double *>(ws + w.ytil[0]), reinterpret_cast<double *>(ws + w.ytil[1])};
    double *rn = reinterpret_cast<double *>(ws + w.rn);
    double *q1 = reinterpret_cast<double *>(ws + w.q1);
    double *q2 = reinterpret_cast<double *>(ws + w.q2);
    double *acon = reinterpret_cast<double *>(ws + w.acon);
    const bool bf = o->prec == LRSDP_F32_BF16IN && mc;
    uint16_t *shadow = bf ? reinterpret_cast<uint16_t *>(ws + w.shadow) : nullptr;
    PcBufs pcb{reinterpret_cast<double *>(ws + w.rho), reinterpret_cast<double *>(ws + w.kap), p->csr.hrow, n,
               o->precond, p->csr.diag, reinterpret_cast<double *>(ws + w.hdyn), 1.0};
    const PcBufs *pc = (mc && o->precond) ? &pcb : nullptr;
    SolverState *st = at<SolverState>(c->scratch, kStateOff);
    double *part_ls = at<double>(c->scratch, kPartLsOff);
    double *part_cb = at<double>(c->scratch, kPartCbOff);
    double *part_up = at<double>(c->scratch, kPartUpOff);
    double *part_misc = at<double>(c->scratch, kPartMiscOff);
    double *l1 = at<double>(c->scratch, kL1Off);
    const void *basis[kMaxBasis];
    for (int g = 0; g <= T; ++g) basis[g] = gring[g];
    for (int d = 0; d < T; ++d) basis[T + 1 + d] = dring[d];

    const double sigma0 = o->sigma0 > 0 ? o->sigma0 : default_sigma0(p);
    SolverState h{};
    h.sigma = sigma0;
    h.sigma_cap = sigma0 * o->sigma_max_ratio;
    h.eta = o->eta0;
    h.gfloor = 1.0;
    h.err1_prev = INFINITY;
    h.tol = o->tol;
    h.sigma_factor = o->sigma_factor;
    h.feas_decrease = o->feas_decrease;
    h.eta_factor = o->eta_factor;
    h.eta_min = o->eta_min;
    h.b_l1 = p->info.b_l1;
    h.precond = (mc && o->precond) ? 1 : 0;
    h.b_inf = p->info.b_inf;
    h.max_inner = o->max_inner;
    h.T = T;
    h.stop_rule = o->reopt ? 1 : 0;
    rc = write_state(c, h);
    if (rc) return rc;
    // zero the rings so stale slots hold finite values
    for (int g = 0; g <= T; ++g)
        if ((rc = launch_fill(s, prec, gring[g], n * ld))) return rc;
    for (int d = 0; d < T; ++d)
        if ((rc = launch_fill(s, prec, dring[d], n * ld))) return rc;
    if (bf && (rc = launch_fill(s, LRSDP_F32, shadow, n * bf16_ld(ld) / 2))) return rc;

    // profiling events
    const int B = std::max(1, o->check_every);
    std::vector<hipEvent_t> evs;
    if (o->profile) {
        evs.resize(2 * B);
        for (auto &e : evs) LRSDP_HIP_TRY(hipEventCreate(&e));
    }
    auto free_events = [&]() {
        for (auto &e : evs) hipEventDestroy(e);
        evs.clear();
    };
    double spmm_ms = 0.0;
    int spmm_n = 0;
    // objective scale of the current re-optimisation round: the round solves
    // the problem with cs C in place of C
    double cs = 1.0;

    // ALM measures at R, with the multiplier step y <- y + sigma (b - A(RR^T))
    // when sigma > 0.  MaxCut: exact C R (into CD), ||R_i||^2; completion:
    // constraint values a = A(RR^T) and ||R||_F^2.
    auto alm_refresh = [&](double sigma, int mode) -> int {
        int r2 = 0, np = 0;
        if (mc) {
            SpmmArgs ref;
            ref.epi = kEpiRefresh;
            ref.V = R;
            ref.Y = CD;
            ref.y = y;
            ref.rn = rn;
            ref.sigma = sigma;
            ref.cs = cs;
            ref.ld = ld;
            ref.partials = part_misc;
            if ((r2 = spmm_maxcut(s, p->csr, prec, ref, &np))) return r2;
        } else if (gen) {
            if ((r2 = gen_sddmm(s, p->gen, prec, 2, R, nullptr, ld, acon, nullptr, nullptr, nullptr, y, sigma, cs,
                                part_misc, nullptr, &np)))
                return r2;
        } else {
            int nb1 = 0, nb2 = 0;
            if ((r2 = cmp_sddmm(s, p->cmp, prec, 2, R, nullptr, ld, acon, nullptr, nullptr, nullptr, y, sigma,
                                part_misc, nullptr, &nb1)))
                return r2;
            const void *rb[1] = {R};
            if ((r2 = launch_dots(s, prec, R, rb, 1, n, ld, part_misc + (size_t)nb1 * kMaxSums, &nb2))) return r2;
            np = nb1 + nb2;
        }
        return launch_alm_finalize(s, st, part_misc, np, mode, cmp ? cs : 1.0);
    };
    // block ranks (general problems): the entries of R past a block's rank start at zero
    if (gen && (rc = gen_rank_mask(s, p->gen, prec, R, ld))) return rc;
    if ((rc = alm_refresh(0.0, 0))) return rc;

    int status = LRSDP_NOT_CONVERGED;
    int64_t admm_iters = 0, admm_fallbacks = 0;
    bool phase2_on = o->phase2 != 0;
    int rank_cur = o->rank;
    const int rank_cap = (int)std::min<int64_t>(
        {(int64_t)std::max(o->rank_max, o->rank), ld, (int64_t)std::floor(std::sqrt(2.0 * (double)p->info.m))});
    int64_t outer = 0;
    int64_t total_inner = 0;
    double sigma_host = sigma0;
    int reopt_rounds = 0;
    double err2 = NAN;
    // Re-optimisation (Section 4.1), after a round met err1 <= tol: test the
    // final criteria on the original problem, whose objective and multipliers
    // are those of the round divided by cs.  Returns 0 when they hold, 1 when a
    // limit stops the solve, 2 when a new round has been set up (C <- factor C
    // and y <- factor y, the multipliers of the scaled problem; R, the penalty
    // and the rank carry over; the inner tolerance factor takes one more
    // schedule step and the inner stop's floor moves to the objective scale;
    // the penalty rule's err1 reference restarts; no splitting phase), or an
    // error code.
    auto reopt_check = [&](SolverState &hs) -> int {
        const double err3o = (hs.obj - hs.dual) / (cs + std::fabs(hs.obj) + std::fabs(hs.dual));
        bool ok = std::fabs(err3o) <= o->tol;
        int r2 = 0;
        if (ok && o->reopt == 2) {
            // dual infeasibility from the certified lower bound on
            // lambda_min(C - A*(y / cs))
            double *yo = reinterpret_cast<double *>(ws + w.yorig);
            LRSDP_HIP_TRY(hipMemcpyAsync(yo, y, p->info.m * sizeof(double), hipMemcpyDeviceToDevice, s));
            if (cs != 1.0 && (r2 = launch_dscale(s, yo, 1.0 / cs, p->info.m))) return r2;
            lrsdp_cert ct{};
            if ((r2 = certify_lib_order(c, p, yo, o->cert_iters, 0.1 * o->tol * (1.0 + p->info.c_l1), 15049,
                                        ws + w.cert, w.cert_bytes, &ct)))
                return r2;
            err2 = std::max(0.0, -ct.lambda_lb) / (1.0 + p->info.c_l1);
            ok = err2 <= o->tol;
        }
        if (o->verbose)
            fprintf(stderr, "[lrsdp] re-opt round %d (scale %.3e): err1 %.3e err3 % .3e err2 %.3e %s\n", reopt_rounds,
                    cs, hs.err1, err3o, err2, ok ? "met" : "not met");
        if (ok) return 0;
        if (reopt_rounds >= o->max_reopt || hs.inner_total >= o->max_iter_total || outer >= o->max_outer ||
            elapsed() > o->time_limit_s)
            return 1;
        ++reopt_rounds;
        cs *= o->reopt_factor;
        pcb.cs = cs;
        phase2_on = false;
        if ((r2 = launch_dscale(s, y, o->reopt_factor, p->info.m))) return r2;
        if ((r2 = alm_refresh(0.0, 0))) return r2;
        if ((r2 = read_state(c, &hs))) return r2;
        hs.eta = std::max(hs.eta * o->eta_factor, o->eta_min);
        hs.gfloor = cs;
        hs.err1_prev = INFINITY;
        hs.converged = 0;
        if ((r2 = write_state(c, hs))) return r2;
        return 2;
    };
    for (outer = 1; outer <= o->max_outer; ++outer) {
        // subproblem start: ytil, G_0, D_0 = -G_0
        int nb = 0, ncb = 0;
        if (mc) {
            if ((rc = launch_grad_init_maxcut(s, prec, st, R, CD, y, rn, ytil[0], gring[0], n, ld, part_misc, &nb,
                                              pc)))
                break;
        } else {
            if ((rc = cmp_ytil(s, cv, st, 0.0, acon, y, ytil[0]))) break;
            if (gen) rc = gen_grad(s, p->gen, prec, st, R, ytil[0], gring, dring, T, ld, part_misc, 0, &nb, cs);
            else rc = cmp_grad(s, p->cmp, prec, st, R, ytil[0], gring, dring, T, ld, part_misc, 0, &nb, cs);
            if (rc) break;
        }
        int64_t left = o->max_iter_total - total_inner;
        int k_limit = (int)std::min<int64_t>(o->max_inner, std::max<int64_t>(left, 0));
        if ((rc = launch_init_finalize(s, st, part_misc, nb, k_limit))) break;
        if ((rc = launch_combine(s, prec, st, nullptr, basis, 2 * T + 1, nullptr, n, ld, part_cb, l1, &ncb, shadow, R,
                                 pc)))
            break;
        // L-BFGS iterations in batches of B.  `it` indexes the ring slots (reset
        // by a gradient refresh); `done_it` counts every enqueued iteration.
        int64_t it = 0, done_it = 0, since_refresh = 0;
        SolverState hs{};
        for (;;) {
            if (o->refresh_every > 0 && since_refresh >= o->refresh_every) {
                // exact C R (MaxCut) / constraint values (completion), gradient,
                // memory restart; same multipliers, penalty and target
                since_refresh = 0;
                it = 0;
                int nb2 = 0;
                if (mc) {
                    SpmmArgs ref;
                    ref.epi = kEpiRefresh;
                    ref.V = R;
                    ref.Y = CD;
                    ref.y = y;
                    ref.rn = rn;
                    ref.sigma = 0.0;
                    ref.cs = cs;
                    ref.ld = ld;
                    ref.partials = part_misc;
                    int np2 = 0;
                    if ((rc = spmm_maxcut(s, p->csr, prec, ref, &np2))) break;
                    if ((rc = launch_grad_init_maxcut(s, prec, st, R, CD, y, rn, ytil[0], gring[0], n, ld, part_misc,
                                                      &nb2, pc)))
                        break;
                } else {
                    if (gen)
                        rc = gen_sddmm(s, p->gen, prec, 2, R, nullptr, ld, acon, nullptr, nullptr, nullptr, y, 0.0, cs,
                                       part_misc, nullptr, &nb2);
                    else
                        rc = cmp_sddmm(s, p->cmp, prec, 2, R, nullptr, ld, acon, nullptr, nullptr, nullptr, y, 0.0,
                                       part_misc, nullptr, &nb2);
                    if (rc) break;
                    if ((rc = cmp_ytil(s, cv, st, 0.0, acon, y, ytil[0]))) break;
                    if (gen)
                        rc = gen_grad(s, p->gen, prec, st, R, ytil[0], gring, dring, T, ld, part_misc, 0, &nb2, cs);
                    else
                        rc = cmp_grad(s, p->cmp, prec, st, R, ytil[0], gring, dring, T, ld, part_misc, 0, &nb2, cs);
                    if (rc) break;
                }
                if ((rc = launch_init_finalize(s, st, part_misc, nb2, -1))) break;
                if ((rc = launch_combine(s, prec, st, nullptr, basis, 2 * T + 1, nullptr, n, ld, part_cb, l1, &ncb,
                                         shadow, R, pc)))
                    break;
            }
            for (int b = 0; b < B && !mc; ++b, ++it, ++done_it, ++since_refresh) {
                int nls = 0, nup = 0;
                if (gen)
                    rc = gen_sddmm(s, p->gen, prec, 1, R, dring[it % T], ld, nullptr, q1, q2, ytil[0], nullptr, 0.0,
                                   cs, part_ls, st, &nls);
                else
                    rc = cmp_sddmm(s, p->cmp, prec, 1, R, dring[it % T], ld, nullptr, q1, q2, ytil[0], nullptr, 0.0,
                                   part_ls, st, &nls);
                if (rc) break;
                if ((rc = launch_ls_finalize(s, st, part_ls, nls, part_cb, ncb, p->info.kind, cs))) break;
                if (gen) {
                    // general problems recompute A(RR^T) at the new R (one more
                    // compressed pass) instead of the recurrence a += tau (q1 +
                    // tau q2): with float32 storage of R the recurrence drifts
                    // from the constraint values of the rounded R
                    // (its partial sums are not read here: no dense C product for <C, RR^T>)
                    int nrf = 0;
                    if ((rc = axpy_state(s, prec, st, R, dring[it % T], n, ld))) break;
                    if ((rc = gen_sddmm(s, p->gen, prec, 2, R, nullptr, ld, acon, nullptr, nullptr, nullptr, y, 0.0,
                                        cs, part_misc, st, &nrf, false)))
                        break;
                    if ((rc = cmp_ytil(s, cv, st, 0.0, acon, y, ytil[0]))) break;
                } else {
                    if ((rc = cmp_samples(s, cv, st, acon, q1, q2, y, ytil[0]))) break;
                    if ((rc = axpy_state(s, prec, st, R, dring[it % T], n, ld))) break;
                }
                if (o->profile) LRSDP_HIP_TRY(hipEventRecord(evs[2 * b], s));
                if (gen)
                    rc = gen_grad(s, p->gen, prec, st, R, ytil[0], gring, dring, T, ld, part_up, -1, &nup, cs);
                else
                    rc = cmp_grad(s, p->cmp, prec, st, R, ytil[0], gring, dring, T, ld, part_up, -1, &nup, cs);
                if (rc) break;
                if (o->profile) LRSDP_HIP_TRY(hipEventRecord(evs[2 * b + 1], s));
                if ((rc = launch_lbfgs_finalize(s, st, part_up, nup))) break;
                if ((rc = launch_combine(s, prec, st, nullptr, basis, 2 * T + 1, nullptr, n, ld, part_cb, l1, &ncb,
                                         shadow)))
                    break;
            }
            for (int b = 0; b < B && mc; ++b, ++it, ++done_it, ++since_refresh) {
                SpmmArgs ls;
                ls.epi = kEpiLS;
                ls.V = bf ? (const void *)shadow : dring[it % T];
                ls.Vown = dring[it % T];
                ls.Y = CD;
                ls.R = R;
                ls.ytil = ytil[it % 2];
                ls.q1 = q1;
                ls.q2 = q2;
                ls.rn = rn;
                ls.ld = ld;
                ls.cs = cs;
                ls.partials = part_ls;
                ls.st = st;
                int nls = 0;
                if (o->profile) LRSDP_HIP_TRY(hipEventRecord(evs[2 * b], s));
                if ((rc = spmm_maxcut(s, p->csr, bf ? LRSDP_F32_BF16IN : prec, ls, &nls))) break;
                if (o->profile) LRSDP_HIP_TRY(hipEventRecord(evs[2 * b + 1], s));
                if ((rc = launch_ls_finalize(s, st, part_ls, nls, part_cb, ncb, LRSDP_MAXCUT, 1.0))) break;
                int nup = 0;
                if ((rc = launch_update_maxcut(s, prec, st, R, CD, y, rn, q1, q2, ytil[it % 2], ytil[(it + 1) % 2],
                                               gring, dring, T, n, ld, part_up, l1, &nup, pc)))
                    break;
                if ((rc = launch_lbfgs_finalize(s, st, part_up, nup))) break;
                if ((rc = launch_combine(s, prec, st, nullptr, basis, 2 * T + 1, nullptr, n, ld, part_cb, l1, &ncb,
                                         shadow, R, pc)))
                    break;
            }
            if (rc) break;
            int64_t k_before = hs.k;
            if ((rc = read_state(c, &hs))) break;
            if (o->profile) {
                int ran = (int)std::min<int64_t>(B, std::max<int64_t>(0, hs.k - k_before));
                for (int b = 0; b < ran; ++b) {
                    float ms = 0.f;
                    LRSDP_HIP_TRY(hipEventElapsedTime(&ms, evs[2 * b], evs[2 * b + 1]));
                    spmm_ms += ms;
                    spmm_n += 1;
                }
            }
            if (hs.done || hs.numeric) break;
            if (elapsed() > o->time_limit_s) break;
            if (done_it > (int64_t)k_limit + 2 * B) {
                rc = set_error(LRSDP_EHIP, "device state did not advance (iteration %lld)", (long long)done_it);
                break;
            }
        }
        if (rc) break;
        total_inner = hs.inner_total;
        if (hs.numeric) {
            rc = set_error(LRSDP_ENUMERIC, "NaN/Inf in the L-BFGS iteration (outer %lld)", (long long)outer);
            break;
        }
        // ALM step: y <- y + sigma (b - A(RR^T)), exact C R, measures
        if ((rc = alm_refresh(sigma_host, 1))) break;
        if ((rc = read_state(c, &hs))) break;
        if (o->verbose)
            fprintf(stderr, "[lrsdp] outer %3lld inner %6lld sigma %.3e obj % .10e err1 %.3e err3 % .3e gnorm %.3e t %.3fs\n",
                    (long long)outer, (long long)hs.inner_total, sigma_host, hs.obj, hs.err1, hs.err3, hs.gnorm,
                    elapsed());
        const double sigma_sub = sigma_host;  // penalty of the subproblem just solved
        sigma_host = hs.sigma;
        if (hs.numeric) {
            rc = set_error(LRSDP_ENUMERIC, "NaN/Inf in the ALM measures (outer %lld)", (long long)outer);
            break;
        }
        if (hs.converged) {
            const int d = o->reopt ? reopt_check(hs) : 0;
            if (d < 0) {
                rc = d;
                break;
            }
            if (d == 0) status = LRSDP_OK;
            if (d != 2) break;
            continue;
        }
        if (rank_cur < rank_cap && hs.k >= o->rank_trigger) {
            // dynamic rank: the subproblem just solved took rank_trigger L-BFGS
            // iterations or more; grow R in place (new columns from the seeded
            // generator), then exact C R and measures for the new R
            const int r_new = std::min<int64_t>(rank_cap, (3 * (int64_t)rank_cur + 1) / 2);
            if ((rc = launch_rank_grow(s, prec, R, n, ld, rank_cur, r_new, (uint64_t)o->rank_seed, o->rank_scale,
                                       mc ? p->csr.perm : nullptr)))
                break;
            if (gen && (rc = gen_rank_mask(s, p->gen, prec, R, ld))) break;   // up to each block's rank
            if (o->verbose) fprintf(stderr, "[lrsdp] rank %d -> %d\n", rank_cur, r_new);
            rank_cur = r_new;
            if ((rc = alm_refresh(0.0, 0))) break;
            if ((rc = read_state(c, &hs))) break;
            // the new columns move err1; the penalty rule restarts its reference
            // so that the jump is not read as a stall
            hs.err1_prev = INFINITY;
            if ((rc = write_state(c, hs))) break;
        }
        if ((cmp || gen) && phase2_on && hs.err1 <= o->switch_err1) {
            // completion / general splitting phase: CG half-steps (Algorithm 2),
            // same measures, stop test and fallback as the MaxCut phase below
            void *U = gring[0];
            void *Ravg = gring[1];
            const int64_t bytes = n * ld * (prec == LRSDP_F64 ? 8 : 4);
            const SolverState snap = hs;
            const CmpAdmmBufs cb = cmp_admm_layout(p, prec, ld, ws + w.cadmm);
            LRSDP_HIP_TRY(hipMemcpyAsync(ws + w.csnap, R, bytes, hipMemcpyDeviceToDevice, s));
            LRSDP_HIP_TRY(hipMemcpyAsync(ytil[1], y, p->info.m * sizeof(double), hipMemcpyDeviceToDevice, s));
            LRSDP_HIP_TRY(hipMemcpyAsync(U, R, bytes, hipMemcpyDeviceToDevice, s));
            if ((rc = launch_fill(s, LRSDP_F64, cb.zero, p->info.m))) break;
            const int chk = std::max(1, o->admm_check);
            int64_t it2 = 0;
            bool done2 = false, diverged = false;
            while (it2 < o->max_admm) {
                for (int b = 0; b < chk && rc == 0; ++b, ++it2)
                    rc = cmp_admm_iter(c, p, prec, U, R, ld, y, sigma_sub, 1e-10, 200, cb);
                if (rc) break;
                if ((rc = launch_avg(s, prec, U, R, Ravg, n * ld))) break;
                int nb1 = 0, nb2 = 0;
                if (gen) {
                    // objective (cs C inside the pass), constraint values, no multiplier step
                    if ((rc = gen_sddmm(s, p->gen, prec, 2, Ravg, nullptr, ld, acon, nullptr, nullptr, nullptr, y,
                                        0.0, cs, part_misc, nullptr, &nb1)))
                        break;
                } else {
                    if ((rc = cmp_sddmm(s, p->cmp, prec, 2, Ravg, nullptr, ld, acon, nullptr, nullptr, nullptr, y,
                                        0.0, part_misc, nullptr, &nb1)))
                        break;
                    const void *rb[1] = {Ravg};
                    if ((rc = launch_dots(s, prec, Ravg, rb, 1, n, ld, part_misc + (size_t)nb1 * kMaxSums, &nb2)))
                        break;
                }
                if ((rc = launch_alm_finalize(s, st, part_misc, nb1 + nb2, 0, 1.0))) break;
                if ((rc = read_state(c, &hs))) break;
                if (o->verbose)
                    fprintf(stderr, "[lrsdp] admm %6lld obj % .10e err1 %.3e err3 % .3e t %.3fs\n", (long long)it2,
                            hs.obj, hs.err1, hs.err3, elapsed());
                if (!std::isfinite(hs.obj) || !std::isfinite(hs.err1) || hs.err1 > 10.0 * snap.err1) {
                    diverged = true;
                    break;
                }
                if (hs.err1 <= o->tol && (o->reopt || std::fabs(hs.err3) <= o->tol)) {
                    done2 = true;
                    break;
                }
                if (elapsed() > o->time_limit_s) break;
            }
            admm_iters += it2;
            if (rc == LRSDP_ENUMERIC) {
                // CG lost positive curvature: treat as a diverged splitting phase
                rc = 0;
                diverged = true;
                clear_error();
            }
            if (rc) break;
            if (done2) {
                LRSDP_HIP_TRY(hipMemcpyAsync(R, Ravg, bytes, hipMemcpyDeviceToDevice, s));
                const int d = o->reopt ? reopt_check(hs) : 0;
                if (d < 0) {
                    rc = d;
                    break;
                }
                if (d == 0) status = LRSDP_OK;
                if (d != 2) break;
                continue;
            }
            if (elapsed() > o->time_limit_s && !diverged) {
                LRSDP_HIP_TRY(hipMemcpyAsync(R, Ravg, bytes, hipMemcpyDeviceToDevice, s));
                break;
            }
            ++admm_fallbacks;
            phase2_on = false;
            LRSDP_HIP_TRY(hipMemcpyAsync(R, ws + w.csnap, bytes, hipMemcpyDeviceToDevice, s));
            LRSDP_HIP_TRY(hipMemcpyAsync(y, ytil[1], p->info.m * sizeof(double), hipMemcpyDeviceToDevice, s));
            if ((rc = write_state(c, snap))) break;
            if ((rc = alm_refresh(0.0, 0))) break;
            if ((rc = read_state(c, &hs))) break;
            if (o->verbose)
                fprintf(stderr, "[lrsdp] splitting phase %s after %lld iterations: back to the ALM\n",
                        diverged ? "diverged" : "did not converge", (long long)it2);
        }
        if (mc && phase2_on && hs.err1 <= o->switch_err1) {
            // splitting phase from U = V = R with the current y and the penalty of the
            // subproblem just solved; measures
            // at R = (U + V)/2 every admm_check iterations (R holds V, the first G
            // slot holds U).  R, y and the solver state are kept (first D slot,
            // second ytil buffer, host copy) for the fallback below.
            void *U = gring[0];
            const int64_t bytes = n * ld * (prec == LRSDP_F64 ? 8 : 4);
            const SolverState snap = hs;
            LRSDP_HIP_TRY(hipMemcpyAsync(dring[0], R, bytes, hipMemcpyDeviceToDevice, s));
            LRSDP_HIP_TRY(hipMemcpyAsync(ytil[1], y, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            LRSDP_HIP_TRY(hipMemcpyAsync(U, R, bytes, hipMemcpyDeviceToDevice, s));
            const int chk = std::max(1, o->admm_check);
            int64_t it2 = 0;
            bool done2 = false, diverged = false;
            while (it2 < o->max_admm) {
                for (int b = 0; b < chk && rc == 0; ++b, ++it2) rc = admm_iter(s, p->csr, prec, U, R, ld, y, sigma_sub);
                if (rc) break;
                if ((rc = launch_avg(s, prec, U, R, gring[1], n * ld))) break;
                SpmmArgs ref;
                ref.epi = kEpiRefresh;
                ref.V = gring[1];
                ref.Y = CD;
                ref.y = y;
                ref.rn = rn;
                ref.sigma = 0.0;
                ref.ld = ld;
                ref.partials = part_misc;
                int np = 0;
                if ((rc = spmm_maxcut(s, p->csr, prec, ref, &np))) break;
                if ((rc = launch_alm_finalize(s, st, part_misc, np, 0, 1.0))) break;
                if ((rc = read_state(c, &hs))) break;
                if (o->verbose)
                    fprintf(stderr, "[lrsdp] admm %6lld obj % .10e err1 %.3e err3 % .3e t %.3fs\n", (long long)it2,
                            hs.obj, hs.err1, hs.err3, elapsed());
                if (!std::isfinite(hs.obj) || !std::isfinite(hs.err1) || hs.err1 > 10.0 * snap.err1) {
                    diverged = true;
                    break;
                }
                if (hs.err1 <= o->tol && (o->reopt || std::fabs(hs.err3) <= o->tol)) {
                    done2 = true;
                    break;
                }
                if (elapsed() > o->time_limit_s) break;
            }
            admm_iters += it2;
            if (rc) break;
            if (done2) {
                LRSDP_HIP_TRY(hipMemcpyAsync(R, gring[1], bytes, hipMemcpyDeviceToDevice, s));
                const int d = o->reopt ? reopt_check(hs) : 0;
                if (d < 0) {
                    rc = d;
                    break;
                }
                if (d == 0) status = LRSDP_OK;
                if (d != 2) break;
                continue;
            }
            if (elapsed() > o->time_limit_s && !diverged) {
                LRSDP_HIP_TRY(hipMemcpyAsync(R, gring[1], bytes, hipMemcpyDeviceToDevice, s));
                break;
            }
            // Fallback (diverged, or max_admm without convergence): restore R, y and
            // the ALM state of the switch, recompute C R, and go on with the ALM
            // alone.
            ++admm_fallbacks;
            phase2_on = false;
            LRSDP_HIP_TRY(hipMemcpyAsync(R, dring[0], bytes, hipMemcpyDeviceToDevice, s));
            LRSDP_HIP_TRY(hipMemcpyAsync(y, ytil[1], n * sizeof(double), hipMemcpyDeviceToDevice, s));
            if ((rc = write_state(c, snap))) break;
            if ((rc = alm_refresh(0.0, 0))) break;
            if ((rc = read_state(c, &hs))) break;
            if (o->verbose)
                fprintf(stderr, "[lrsdp] splitting phase %s after %lld iterations: back to the ALM\n",
                        diverged ? "diverged" : "did not converge", (long long)it2);
        }
        if (hs.inner_total >= o->max_iter_total || elapsed() > o->time_limit_s) break;
    }
    free_events();
    if (rc < 0) return rc;
    SolverState hs{};
    if ((rc = read_state(c, &hs))) return rc;
    // back to the original problem after re-optimisation rounds: objective,
    // multipliers and penalty divided by cs (L for cs C equals cs times L for C
    // with y / cs and sigma / cs)
    if (cs != 1.0 && (rc = launch_dscale(s, y, 1.0 / cs, p->info.m))) return rc;
    LRSDP_HIP_TRY(hipStreamSynchronize(s));
    std::memset(res, 0, sizeof(*res));
    res->obj = hs.obj / cs;
    res->dual = hs.dual / cs;
    res->err1 = hs.err1;
    res->err1_inf = hs.err1_inf;
    res->err3 = (hs.obj - hs.dual) / (cs + std::fabs(hs.obj) + std::fabs(hs.dual));
    res->sigma = hs.sigma / cs;
    res->seconds = elapsed();
    res->outer = std::min<int64_t>(outer, o->max_outer);
    res->inner = hs.inner_total;
    res->status = status;
    res->spmm_launches = spmm_n;
    res->spmm_ms = spmm_ms;
    res->spmm_bytes = mc    ? maxcut_spmm_bytes(p, prec, o->rank)
                      : gen ? general_grad_bytes(p, prec, o->rank, T)
                            : completion_grad_bytes(p, prec, o->rank, T);
    res->admm_iters = admm_iters;
    res->admm_fallbacks = admm_fallbacks;
    res->rank_final = rank_cur;
    res->reopt_rounds = reopt_rounds;
    res->err2 = err2;
    return status;
}

}  // namespace

extern "C" int lrsdp_solve(lrsdp_ctx *c, lrsdp_problem *p, const lrsdp_options *o, void *ws, size_t ws_bytes,
                           void *R, double *y, lrsdp_result *res) {
    clear_error();
    if (!c || !o || !ws || !R || !y || !res) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc = check_problem(p);
    if (rc) return rc;
    WsPlan w;
    if ((rc = plan_workspace(p, o, &w))) return rc;
    if (ws_bytes < w.total) return set_error(LRSDP_ENOMEM, "workspace needs %zu bytes, %zu given", w.total, ws_bytes);
    LRSDP_HIP_TRY(hipSetDevice(c->device));
    const int32_t *perm = p->info.kind == LRSDP_MAXCUT ? p->csr.perm : nullptr;
    if (!perm) return solve_impl(c, p, o, static_cast<char *>(ws), R, y, res);
    // A problem relabelled by degree: R and y move into the library's node
    // order for the solve and back afterwards (also after a failed solve),
    // through the front of the workspace, which the solve has not yet taken or
    // no longer needs.
    const int64_t n = p->info.n;
    const size_t rbytes = (size_t)o->ld * elem_size(o->prec), fbytes = (size_t)n * rbytes;
    const size_t yoff = (fbytes + 255) / 256 * 256;
    if (w.total < yoff + (size_t)n * sizeof(double))
        return set_error(LRSDP_ENOMEM, "workspace of %zu bytes cannot stage the node-order moves", w.total);
    char *tmp = static_cast<char *>(ws);
    double *ytmp = reinterpret_cast<double *>(tmp + yoff);
    hipStream_t s = c->stream;
    if ((rc = launch_permute_rows(s, R, tmp, perm, n, (int64_t)rbytes, 0))) return rc;
    if ((rc = launch_permute_vec(s, y, ytmp, perm, n, 0))) return rc;
    LRSDP_HIP_TRY(hipMemcpyAsync(R, tmp, fbytes, hipMemcpyDeviceToDevice, s));
    LRSDP_HIP_TRY(hipMemcpyAsync(y, ytmp, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    const int rc_solve = solve_impl(c, p, o, static_cast<char *>(ws), R, y, res);
    if ((rc = launch_permute_rows(s, R, tmp, perm, n, (int64_t)rbytes, 1))) return rc;
    if ((rc = launch_permute_vec(s, y, ytmp, perm, n, 1))) return rc;
    LRSDP_HIP_TRY(hipMemcpyAsync(R, tmp, fbytes, hipMemcpyDeviceToDevice, s));
    LRSDP_HIP_TRY(hipMemcpyAsync(y, ytmp, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    LRSDP_HIP_TRY(hipStreamSynchronize(s));
    return rc_solve;
}

// ---------------------------------------------------------------------------
// kernel entry points
// ---------------------------------------------------------------------------
extern "C" int lrsdp_k_spmm(lrsdp_ctx *c, const lrsdp_problem *p, int prec, const void *V, int64_t ld,
                            const double *ytil, void *Y) {
    clear_error();
    if (!c || !V || !Y) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_problem(p)) || (rc = check_input_order(p)) || (rc = check_prec(prec)) ||
        (rc = check_ld(prec, ld)))
        return rc;
    if (V == Y) return set_error(LRSDP_EINVAL, "Y must not alias V");
    const int pr = prec == LRSDP_F64 ? LRSDP_F64 : LRSDP_F32;
    if (p->info.kind == LRSDP_MAXCUT) {
        SpmmArgs a;
        a.epi = kEpiPlain;
        a.V = V;
        a.Y = Y;
        a.ytil = ytil;
        a.ld = ld;
        int np = 0;
        return spmm_maxcut(c->stream, p->csr, prec, a, &np);
    }
    if (prec == LRSDP_F32_BF16IN)
        return set_error(LRSDP_EUNSUPPORTED, "bfloat16 input is implemented for the MaxCut SpMM only");
    if (p->info.kind == LRSDP_GENERAL) return spmm_general(c->stream, p->gen, pr, V, ld, ytil, Y);
    return spmm_completion(c->stream, p->cmp, pr, V, ld, ytil, Y);
}

extern "C" int lrsdp_k_constraint(lrsdp_ctx *c, const lrsdp_problem *p, int prec, const void *U, const void *V,
                                  int64_t ld, double *out) {
    clear_error();
    if (!c || !U || !out) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_problem(p)) || (rc = check_input_order(p)) || (rc = check_prec(prec)) ||
        (rc = check_ld(prec, ld)))
        return rc;
    const int pr = prec == LRSDP_F64 ? LRSDP_F64 : LRSDP_F32;
    if (!V) V = U;
    if (p->info.kind == LRSDP_MAXCUT) return launch_rowdot(c->stream, pr, U, V, p->info.n, ld, out);
    int nb = 0;
    if (p->info.kind == LRSDP_GENERAL)
        return gen_sddmm(c->stream, p->gen, pr, 0, U, V, ld, out, nullptr, nullptr, nullptr, nullptr, 0.0, 1.0,
                         nullptr, nullptr, &nb);
    return cmp_sddmm(c->stream, p->cmp, pr, 0, U, V, ld, out, nullptr, nullptr, nullptr, nullptr, 0.0, nullptr,
                     nullptr, &nb);
}

extern "C" int lrsdp_k_ls_coeffs(lrsdp_ctx *c, const lrsdp_problem *p, int prec, const void *R, const void *D,
                                 int64_t ld, const double *y, double sigma, void *work, double *out, double *q1,
                                 double *q2) {
    clear_error();
    if (!c || !R || !D || !y || !work || !out) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_problem(p)) || (rc = check_input_order(p)) || (rc = check_prec(prec)) ||
        (rc = check_ld(prec, ld)))
        return rc;
    const int pr = prec == LRSDP_F64 ? LRSDP_F64 : LRSDP_F32;
    const int64_t n = p->info.n;
    const size_t arr = (size_t)n * ld * elem_size(pr);
    char *wk = static_cast<char *>(work);
    if (p->info.kind == LRSDP_GENERAL) {
        // a = A(RR^T), ytil = y + sigma (b - a), then the C-weighted and
        // per-constraint line-search terms in one compressed pass
        const int64_t m = p->info.m;
        double *acon = reinterpret_cast<double *>(wk);
        double *yt = acon + m;
        double *part = at<double>(c->scratch, kPartLsOff);
        double *sums = at<double>(c->scratch, kSmallOff);
        hipStream_t s = c->stream;
        DevCompletion v{};
        v.m = m;
        v.b = p->gen.b;
        int nb = 0;
        if ((rc = gen_sddmm(s, p->gen, pr, 0, R, R, ld, acon, nullptr, nullptr, nullptr, nullptr, 0.0, 1.0, nullptr,
                            nullptr, &nb)))
            return rc;
        if ((rc = cmp_ytil(s, v, nullptr, sigma, acon, y, yt))) return rc;
        if ((rc = gen_sddmm(s, p->gen, pr, 1, R, D, ld, nullptr, q1, q2, yt, nullptr, 0.0, 1.0, part, nullptr, &nb)))
            return rc;
        if ((rc = launch_reduce(s, part, nb, kLsSums, sums))) return rc;
        return launch_ls_out(s, sums, sigma, out);
    }
    if (p->info.kind == LRSDP_COMPLETION) {
        // a = A(RR^T), ytil = y + sigma (b - a), sample terms, then p1 = 2<R,D>, p2 = ||D||^2
        const int64_t m = p->info.m;
        double *acon = reinterpret_cast<double *>(wk);
        double *yt = acon + m;
        double *part = at<double>(c->scratch, kPartLsOff);
        double *sums = at<double>(c->scratch, kSmallOff);
        double *d2 = sums + 16;
        hipStream_t s = c->stream;
        int nb = 0;
        if ((rc = cmp_sddmm(s, p->cmp, pr, 0, R, R, ld, acon, nullptr, nullptr, nullptr, nullptr, 0.0, nullptr,
                            nullptr, &nb)))
            return rc;
        if ((rc = cmp_ytil(s, p->cmp, nullptr, sigma, acon, y, yt))) return rc;
        if ((rc = cmp_sddmm(s, p->cmp, pr, 1, R, D, ld, nullptr, q1, q2, yt, nullptr, 0.0, part, nullptr, &nb)))
            return rc;
        if ((rc = launch_reduce(s, part, nb, kLsSums, sums))) return rc;
        const void *rd[2] = {R, D};
        double *part2 = at<double>(c->scratch, kPartMiscOff);
        if ((rc = launch_dots(s, pr, D, rd, 2, n, ld, part2, &nb))) return rc;
        if ((rc = launch_reduce(s, part2, nb, 2, d2))) return rc;
        return launch_ls_out_cmp(s, sums, d2, sigma, out);
    }
    void *CR = wk, *CDv = wk + arr;
    double *ytil = reinterpret_cast<double *>(wk + 2 * arr);
    double *part = at<double>(c->scratch, kPartLsOff);
    double *sums = at<double>(c->scratch, kSmallOff);
    hipStream_t s = c->stream;
    // ytil = y + sigma (1 - ||R_i||^2)
    if ((rc = launch_rowdot(s, pr, R, R, n, ld, ytil))) return rc;
    if ((rc = launch_ytil(s, y, ytil, nullptr, sigma, n, ytil))) return rc;
    SpmmArgs a;
    a.epi = kEpiPlain;
    a.V = R;
    a.Y = CR;
    a.ld = ld;
    int np = 0;
    if ((rc = spmm_maxcut(s, p->csr, pr, a, &np))) return rc;
    SpmmArgs b;
    b.epi = kEpiLS;
    b.V = D;
    b.Y = CDv;
    b.R = R;
    b.aux = CR;
    b.ytil = ytil;
    b.q1 = q1;
    b.q2 = q2;
    b.ld = ld;
    b.partials = part;
    if ((rc = spmm_maxcut(s, p->csr, pr, b, &np))) return rc;
    if ((rc = launch_reduce(s, part, np, kLsSums, sums))) return rc;
    return launch_ls_out(s, sums, sigma, out);
}

extern "C" int lrsdp_k_cubic(lrsdp_ctx *c, const double *a, double *tau) {
    clear_error();
    if (!c || !a || !tau) return set_error(LRSDP_EINVAL, "NULL argument");
    return launch_cubic(c->stream, a, tau);
}

extern "C" int lrsdp_k_alm(lrsdp_ctx *c, const lrsdp_problem *p, int prec, const void *R, int64_t ld, double *y,
                           double sigma, void *work, double *out) {
    clear_error();
    if (!c || !R || !y || !work || !out) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_problem(p)) || (rc = check_input_order(p)) || (rc = check_prec(prec)) ||
        (rc = check_ld(prec, ld)))
        return rc;
    const int pr = prec == LRSDP_F64 ? LRSDP_F64 : LRSDP_F32;
    double *part = at<double>(c->scratch, kPartMiscOff);
    double *sums = at<double>(c->scratch, kSmallOff);
    if (p->info.kind == LRSDP_GENERAL) {
        int nb = 0;
        if ((rc = gen_sddmm(c->stream, p->gen, pr, 2, R, nullptr, ld, static_cast<double *>(work), nullptr, nullptr,
                            nullptr, y, sigma, 1.0, part, nullptr, &nb)))
            return rc;
        if ((rc = launch_reduce(c->stream, part, nb, 3, sums))) return rc;
        return launch_alm_out(c->stream, sums, p->info.b_l1, p->info.b_inf, out);
    }
    if (p->info.kind == LRSDP_COMPLETION) {
        int nb1 = 0, nb2 = 0;
        if ((rc = cmp_sddmm(c->stream, p->cmp, pr, 2, R, nullptr, ld, static_cast<double *>(work), nullptr, nullptr,
                            nullptr, y, sigma, part, nullptr, &nb1)))
            return rc;
        const void *rb[1] = {R};
        if ((rc = launch_dots(c->stream, pr, R, rb, 1, p->info.n, ld, part + (size_t)nb1 * kMaxSums, &nb2))) return rc;
        if ((rc = launch_reduce(c->stream, part, nb1 + nb2, 3, sums))) return rc;
        return launch_alm_out(c->stream, sums, p->info.b_l1, p->info.b_inf, out);
    }
    SpmmArgs a;
    a.epi = kEpiRefresh;
    a.V = R;
    a.Y = work;
    a.y = y;
    a.sigma = sigma;
    a.ld = ld;
    a.partials = part;
    int np = 0;
    if ((rc = spmm_maxcut(c->stream, p->csr, pr, a, &np))) return rc;
    if ((rc = launch_reduce(c->stream, part, np, 3, sums))) return rc;
    return launch_alm_out(c->stream, sums, p->info.b_l1, p->info.b_inf, out);
}

extern "C" int lrsdp_k_lbfgs_dir(lrsdp_ctx *c, int prec, int64_t n, int64_t ld, const void *G,
                                 const void *const *S, const void *const *Y, int k, void *D) {
    clear_error();
    if (!c || !G || !D || (k > 0 && (!S || !Y))) return set_error(LRSDP_EINVAL, "NULL argument");
    if (k < 0 || k > kMaxMem) return set_error(LRSDP_EINVAL, "k = %d not in [0, %d]", k, kMaxMem);
    int rc;
    if ((rc = check_prec(prec)) || (rc = check_ld(prec, ld))) return rc;
    const int pr = prec == LRSDP_F64 ? LRSDP_F64 : LRSDP_F32;
    const int nb = 2 * k + 1;
    const void *basis[kMaxBasis];
    basis[0] = G;
    for (int t = 0; t < k; ++t) {
        basis[1 + t] = S[t];
        basis[1 + k + t] = Y[t];
    }
    hipStream_t s = c->stream;
    double *part = at<double>(c->scratch, kPartMiscOff);
    double *small = at<double>(c->scratch, kSmallOff);
    double *red = small;                      // nb sums
    double *gram = small + 64;                // nb x nb
    double *coef = small + 64 + 512;          // nb
    int *flag = reinterpret_cast<int *>(small + 64 + 512 + 64);
    for (int i = 0; i < nb; ++i) {
        int nblk = 0;
        if ((rc = launch_dots(s, pr, basis[i], basis, nb, n, ld, part, &nblk))) return rc;
        if ((rc = launch_reduce(s, part, nblk, nb, red))) return rc;
        if ((rc = launch_gather_gram(s, red, nb, i, gram))) return rc;
    }
    if ((rc = launch_two_loop_pairs(s, gram, k, coef, flag))) return rc;
    int nblk = 0;
    double *l1 = at<double>(c->scratch, kL1Off);
    if ((rc = launch_combine(s, pr, nullptr, coef, basis, nb, D, n, ld, part, l1, &nblk, nullptr))) return rc;
    int hflag = 0;
    LRSDP_HIP_TRY(hipMemcpyAsync(c->pinned, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    LRSDP_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(&hflag, c->pinned, sizeof(int));
    if (hflag) return set_error(LRSDP_EINVAL, "a pair has <y_t, s_t> <= 0");
    return LRSDP_OK;
}

// ---------------------------------------------------------------------------
// learned warm start
// ---------------------------------------------------------------------------
namespace lrsdp {
int ws_features(hipStream_t, const DevCsr &, float *, float4 *);
int mlp_forward(hipStream_t, const void *, int, const float *, int64_t, float *);
int mlp_grad(hipStream_t, const void *, int, const float *, const float *, int64_t, float *, double *, float *);
int mlp_adam(hipStream_t, float *, float *, float *, const float *, int, float, uint16_t *);
int to_bf16(hipStream_t, const float *, int64_t, uint16_t *);
int warm_y0(hipStream_t, const float *, const float4 *, int64_t, double *, double *, double *);
int mlp_param_count();
int ws_targets(hipStream_t, const float4 *, const double *, int64_t, double, float *);
}  // namespace lrsdp

extern "C" int lrsdp_ws_targets(lrsdp_ctx *c, const lrsdp_problem *p, const float *stats, const double *y,
                                double sigma_final, float *target) {
    clear_error();
    if (!c || !stats || !y || !target) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (p->info.kind != LRSDP_MAXCUT) return set_error(LRSDP_EUNSUPPORTED, "warm start is for MaxCut problems");
    if (!(sigma_final > 0.0) || !std::isfinite(sigma_final))
        return set_error(LRSDP_EINVAL, "sigma_final must be positive and finite");
    return ws_targets(c->stream, reinterpret_cast<const float4 *>(stats), y, p->info.n,
                      std::log(sigma_final / default_sigma0(p)), target);
}

extern "C" int lrsdp_mlp_param_count(void) { return mlp_param_count(); }

extern "C" int lrsdp_ws_features(lrsdp_ctx *c, const lrsdp_problem *p, float *feat, float *stats) {
    clear_error();
    if (!c || !feat || !stats) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (p->info.kind != LRSDP_MAXCUT) return set_error(LRSDP_EUNSUPPORTED, "warm start is for MaxCut problems");
    if (((uintptr_t)feat | (uintptr_t)stats) % 16) return set_error(LRSDP_EINVAL, "buffers must be 16-byte aligned");
    return ws_features(c->stream, p->csr, feat, reinterpret_cast<float4 *>(stats));
}

static int check_param_dtype(int dtype) {
    if (dtype != LRSDP_PARAM_F32 && dtype != LRSDP_PARAM_BF16)
        return set_error(LRSDP_EINVAL, "parameter dtype %d is neither LRSDP_PARAM_F32 nor LRSDP_PARAM_BF16", dtype);
    return LRSDP_OK;
}

extern "C" int lrsdp_mlp_forward(lrsdp_ctx *c, const void *params, int param_dtype, const float *feat, int64_t n,
                                 float *out) {
    clear_error();
    if (!c || !params || !feat || !out || n < 0) return set_error(LRSDP_EINVAL, "bad argument");
    int rc;
    if ((rc = check_param_dtype(param_dtype))) return rc;
    if (n == 0) return LRSDP_OK;
    return mlp_forward(c->stream, params, param_dtype == LRSDP_PARAM_BF16, feat, n, out);
}

extern "C" int lrsdp_mlp_grad(lrsdp_ctx *c, const void *params, int param_dtype, const float *feat,
                              const float *target, int64_t n, float *grad, double *loss, float *work) {
    clear_error();
    if (!c || !params || !feat || !target || !grad || !work || n <= 0) return set_error(LRSDP_EINVAL, "bad argument");
    int rc;
    if ((rc = check_param_dtype(param_dtype))) return rc;
    return mlp_grad(c->stream, params, param_dtype == LRSDP_PARAM_BF16, feat, target, n, grad, loss, work);
}

extern "C" int lrsdp_mlp_adam(lrsdp_ctx *c, float *params, float *m, float *v, const float *grad, int step, float lr) {
    clear_error();
    if (!c || !params || !m || !v || !grad || step < 1) return set_error(LRSDP_EINVAL, "bad argument");
    return mlp_adam(c->stream, params, m, v, grad, step, lr, nullptr);
}

extern "C" int lrsdp_mlp_train(lrsdp_ctx *c, float *master, uint16_t *params_bf16, float *m, float *v,
                               const float *feat, const float *target, int64_t n, int first_step, int steps,
                               float lr, float *work, double *loss_hist) {
    clear_error();
    if (!c || !master || !params_bf16 || !m || !v || !feat || !target || !work || n <= 0 || first_step < 1 ||
        steps < 0 || !(lr > 0.0f))
        return set_error(LRSDP_EINVAL, "bad argument");
    const int P = mlp_param_count();
    float *grad = work;                            // P floats, then the gradient partials
    float *partials = work + ((P + 63) / 64) * 64;
    hipStream_t s = c->stream;
    int rc;
    if ((rc = to_bf16(s, master, P, params_bf16))) return rc;
    for (int k = 0; k < steps; ++k) {
        if ((rc = mlp_grad(s, params_bf16, 1, feat, target, n, grad, loss_hist ? loss_hist + k : nullptr, partials)))
            return rc;
        if ((rc = mlp_adam(s, master, m, v, grad, first_step + k, lr, params_bf16))) return rc;
    }
    return LRSDP_OK;
}

extern "C" int lrsdp_mlp_train_work_floats(void) {
    const int P = mlp_param_count();
    return ((P + 63) / 64) * 64 + 256 * (P + 1);
}

extern "C" int lrsdp_warmstart(lrsdp_ctx *c, const lrsdp_problem *p, const void *params, int param_dtype,
                               double log_ratio_lo, double log_ratio_hi, float *work, double *y0, double *sigma0) {
    clear_error();
    if (!c || !params || !work || !y0 || !sigma0) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_param_dtype(param_dtype))) return rc;
    if ((rc = check_problem(p))) return rc;
    if (p->info.kind != LRSDP_MAXCUT) return set_error(LRSDP_EUNSUPPORTED, "warm start is for MaxCut problems");
    if ((uintptr_t)work % 16) return set_error(LRSDP_EINVAL, "work must be 16-byte aligned");
    if (!(log_ratio_lo <= log_ratio_hi) || !std::isfinite(log_ratio_lo) || !std::isfinite(log_ratio_hi))
        return set_error(LRSDP_EINVAL, "the penalty range [%g, %g] is empty or not finite", log_ratio_lo,
                         log_ratio_hi);
    const int64_t n = p->info.n;
    float *feat = work;
    float4 *stats = reinterpret_cast<float4 *>(work + 16 * n);
    float *out = work + 20 * n;
    double *part = at<double>(c->scratch, kPartMiscOff);
    double *sum = at<double>(c->scratch, kSmallOff);
    hipStream_t s = c->stream;
    if ((rc = ws_features(s, p->csr, feat, stats))) return rc;
    if ((rc = mlp_forward(s, params, param_dtype == LRSDP_PARAM_BF16, feat, n, out))) return rc;
    if ((rc = warm_y0(s, out, stats, n, y0, part, sum))) return rc;
    double hsum[2] = {0.0, 0.0};
    LRSDP_HIP_TRY(hipMemcpyAsync(c->pinned, sum, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    LRSDP_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(hsum, c->pinned, 2 * sizeof(double));
    const double mean = n > 0 ? hsum[0] / (double)n : 0.0;
    if (!std::isfinite(mean) || !std::isfinite(hsum[1]))
        return set_error(LRSDP_ENUMERIC, "warm-start prediction is not finite");
    // the network predicts log(final penalty / default) of a cold solve; the
    // warm start begins halfway there on the log scale, leaving the penalty
    // rule room to raise it (starting at the final penalty made the first
    // subproblems too stiff to solve within their iteration limit)
    *sigma0 = default_sigma0(p) * std::exp(0.5 * std::max(log_ratio_lo, std::min(log_ratio_hi, mean)));
    return LRSDP_OK;
}

extern "C" int lrsdp_admm_workspace_bytes(const lrsdp_problem *p, int prec, int64_t ld, size_t *bytes) {
    clear_error();
    if (!p || !bytes) return set_error(LRSDP_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_prec(prec)) || (rc = check_ld(prec, ld))) return rc;
    *bytes = p->info.kind == LRSDP_MAXCUT ? 0 : cmp_admm_bytes(p, prec == LRSDP_F64 ? LRSDP_F64 : LRSDP_F32, ld);
    return LRSDP_OK;
}

extern "C" int lrsdp_k_admm(lrsdp_ctx *c, const lrsdp_problem *p, int prec, void *U, void *V, int64_t ld, double *y,
                            double sigma, int iters, double cg_tol, int cg_max, void *work, size_t work_bytes) {
    clear_error();
    if (!c || !U || !V || !y || iters < 0 || !(sigma > 0)) return set_error(LRSDP_EINVAL, "bad argument");
    int rc;
    if ((rc = check_problem(p)) || (rc = check_input_order(p)) || (rc = check_prec(prec)) ||
        (rc = check_ld(prec, ld)))
        return rc;
    const int pr = prec == LRSDP_F64 ? LRSDP_F64 : LRSDP_F32;
    if (p->info.kind == LRSDP_MAXCUT) {
        for (int k = 0; k < iters; ++k)
            if ((rc = admm_iter(c->stream, p->csr, pr, U, V, ld, y, sigma))) return rc;
        return LRSDP_OK;
    }
    if (!(cg_tol > 0.0) || cg_max < 1) return set_error(LRSDP_EINVAL, "need cg_tol > 0 and cg_max >= 1");
    const size_t need = cmp_admm_bytes(p, pr, ld);
    if (!work || work_bytes < need)
        return set_error(LRSDP_ENOMEM, "splitting workspace needs %zu bytes, got %zu", need, work_bytes);
    if ((uintptr_t)work % 256) return set_error(LRSDP_EINVAL, "workspace must be 256-byte aligned");
    const CmpAdmmBufs b = cmp_admm_layout(p, pr, ld, static_cast<char *>(work));
    if ((rc = launch_fill(c->stream, LRSDP_F64, b.zero, p->info.m))) return rc;
    for (int k = 0; k < iters; ++k)
        if ((rc = cmp_admm_iter(c, p, pr, U, V, ld, y, sigma, cg_tol, cg_max, b))) return rc;
    return LRSDP_OK;
}
