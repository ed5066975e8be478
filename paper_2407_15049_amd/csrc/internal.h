// Internal declarations of the lrsdp library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lrsdp.h"

namespace lrsdp {

// ---------------------------------------------------------------------------
// Error handling: every ABI function returns an int status and leaves a
// thread-local message.
// ---------------------------------------------------------------------------
int set_error(int code, const char *fmt, ...);
void clear_error();

// Takes the device address of the allocation-free entry point's static array
// on `device` (current) once; lrsdp_ctx_create calls it.
int noalloc_init(int device, void **ptr);

#define LRSDP_HIP_TRY(expr)                                                      \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess)                                                    \
            return ::lrsdp::set_error(LRSDP_EHIP, "%s failed: %s (%s:%d)", #expr, \
                                      hipGetErrorString(e_), __FILE__, __LINE__);\
    } while (0)

#define LRSDP_CHECK_LAUNCH()                                                     \
    do {                                                                         \
        hipError_t e_ = hipGetLastError();                                       \
        if (e_ != hipSuccess)                                                    \
            return ::lrsdp::set_error(LRSDP_EHIP, "kernel launch failed: %s (%s:%d)", \
                                      hipGetErrorString(e_), __FILE__, __LINE__);\
    } while (0)

// Launch geometry shared by the grid-stride kernels.
constexpr int kBlock = 256;          // threads per workgroup (4 wave64s)
constexpr int kMaxBlocks = 2048;     // fixed grid of the reduction kernels
constexpr int kMaxSums = 32;         // doubles of partial sums per block
constexpr int kMaxMem = 8;           // largest L-BFGS memory
constexpr int kMaxBasis = 2 * kMaxMem + 1;
constexpr int kSegLen = 128;         // rows longer than this are split into segments
// The flat streaming sweeps (L-BFGS update and combine) run one 16-byte chunk
// per thread over as many workgroups as the array needs (fewer, grid-stride,
// past kL1Bytes of first-level sums), each workgroup storing one compact row
// of its dot products; a second kernel adds kL1PerL2 consecutive rows at a
// time, in a fixed order, into the kMaxSums-stride rows the finalize kernels read.
constexpr size_t kL1Bytes = size_t(16) << 20;
constexpr int kL1PerL2 = kBlock;

// Weight encodings of the MaxCut off-diagonal values C_ij = w_ij / 4.
enum WeightMode { kWUnit = 0, kWSign = 1, kWGeneral = 2 };

// ---------------------------------------------------------------------------
// Problem: host build + device views.
// ---------------------------------------------------------------------------
struct DevCsr {
    // Symmetric off-diagonal part of the SpMM operator in CSR.
    const int32_t *row_ptr = nullptr;   // n + 1
    const int32_t *col = nullptr;       // nnz; bit 31 = negative weight (kWSign)
    const double *val = nullptr;        // nnz (kWGeneral only)
    const double *diag = nullptr;       // n   (C_ii)
    const double *hrow = nullptr;       // n   2 max(sum_j |C_ij|, 1e-3 ||vec(C)||_1 / n) (row-block H0)
    const int32_t *perm = nullptr;      // n   caller label of internal node k (LRSDP_ORDER_DEGREE), else null
    // Work lists.  Light rows (<= kSegLen nonzeros) sorted by decreasing length
    // inside windows of consecutive rows; heavy rows split into segments.
    const int4 *light = nullptr;        // n_light {row, begin, end, 0}
    const int4 *seg = nullptr;          // n_seg {row, begin, end, slot}
    const int32_t *heavy = nullptr;     // n_heavy row ids
    const int32_t *heavy_seg = nullptr; // n_heavy + 1 offsets into seg
    void *seg_buf = nullptr;            // n_seg x 32 float64 segment partial sums
    int64_t n = 0, nnz = 0, n_light = 0, n_seg = 0, n_heavy = 0;
    int wmode = kWUnit;
};

// Completion: X has order n = n1 + n2; sample k = (i, j) sits at column n1 + j.
struct DevCompletion {
    const int32_t *top_ptr = nullptr;   // n1 + 1, samples sorted by (i, j)
    const int32_t *top_col = nullptr;   // m: j (column block index)
    const int32_t *top_eid = nullptr;   // m: sample id k of each top entry
    const int32_t *bot_ptr = nullptr;   // n2 + 1
    const int32_t *bot_row = nullptr;   // m: i
    const int32_t *bot_eid = nullptr;   // m: sample id k of each bottom entry
    const int32_t *samp_i = nullptr;    // m
    const int32_t *samp_j = nullptr;    // m
    const double *b = nullptr;          // m: 2 M_ij
    int64_t n1 = 0, n2 = 0, m = 0;
};

// Constraint rows of a general problem longer than this are reduced by a
// whole workgroup (a trace constraint spans n positions).
constexpr int kLongRow = 512;

// Dense C of a general problem: largest order accepted, largest order chosen
// automatically, the fraction of nonzero upper-triangle positions from which
// the automatic choice takes dense storage, the bytes per row of the dense
// product and its split-k partials (64 float64 columns: ld <= 32 in float64,
// <= 64 in float32), and the largest k split.
constexpr int64_t kDenseMaxN = 16384;
constexpr int64_t kDenseAutoN = 8192;
constexpr double kDenseFrac = 0.1;
constexpr size_t kDenseRowBytes = 64 * sizeof(double);
constexpr int kDenseMaxSplit = 8;

// General problem (Section 3.4 compression).  Omega: positions (a, b), a <= b,
// that are nonzero in C or in some A_k; the stacked constraint matrix keeps
// only its nonzero columns, indexed by position in Omega.
struct DevGeneral {
    const int32_t *om_a = nullptr;      // |Omega| row of each position
    const int32_t *om_b = nullptr;      // |Omega| column (>= row)
    const double *cval = nullptr;       // |Omega| C_ab (0 where only constraints touch)
    const int32_t *a_ptr = nullptr;     // m + 1: constraint rows of the stacked matrix
    const int32_t *a_idx = nullptr;     // nnz_a: Omega index
    const double *a_val = nullptr;      // nnz_a: A_k,ab
    const int32_t *at_ptr = nullptr;    // |Omega| + 1: the transpose, rows = positions
    const int32_t *at_idx = nullptr;    // nnz_a: constraint index
    const double *at_val = nullptr;     // nnz_a
    const int32_t *s_ptr = nullptr;     // n + 1: symmetric pattern of Omega by rows
    const int32_t *s_col = nullptr;     // nnz_s: column
    const int32_t *s_om = nullptr;      // nnz_s: Omega index of the entry
    const double *b = nullptr;          // m
    const int32_t *con_short = nullptr; // constraints whose row has <= kLongRow entries (a thread each)
    const int32_t *con_long = nullptr;  // the longer ones (a workgroup each)
    int64_t n_short = 0, n_long = 0;
    // Dense storage of C (Section 3.5, last paragraph; null with sparse storage):
    const double *cd = nullptr;         // n x n, row-major, both triangles
    double *dw = nullptr;               // n rows of kDenseRowBytes: the dense product cs C V
    double *dpart = nullptr;            // kDenseMaxSplit x n rows of kDenseRowBytes: split-k partials
    const int32_t *row_rank = nullptr;  // n: columns row i of R may use (block ranks), or null: all
    double *x1 = nullptr;               // |Omega| compressed outer products, and (x2) the values of
    double *x2 = nullptr;               // C - A*(y) for the SpMM (problem-owned scratch: calls on one
                                        // problem must not overlap)
    int64_t n = 0, m = 0, nom = 0, nnz_a = 0, nnz_s = 0;
};

// General problem: Y = (C - A*(ytil)) V on the symmetric pattern of Omega.
int spmm_general(hipStream_t s, const DevGeneral &P, int prec, const void *V, int64_t ld, const double *ytil,
                 void *Y);

// Node-order moves of a relabelled MaxCut problem (perm[k] = caller label of
// internal node k).  scatter == 0: dst[k] = src[perm[k]] (caller -> library
// order); scatter == 1: dst[perm[k]] = src[k] (library -> caller order).
// Rows of row_bytes (a multiple of 16) for factors, float64 entries for vectors.
int launch_permute_rows(hipStream_t s, const void *src, void *dst, const int32_t *perm, int64_t n,
                        int64_t row_bytes, int scatter);
int launch_permute_vec(hipStream_t s, const double *src, double *dst, const int32_t *perm, int64_t n, int scatter);

// lrsdp_certify with y in the library's node order (the solver's own calls).
int certify_lib_order(lrsdp_ctx *c, const lrsdp_problem *p, const double *y, int max_iter, double tol,
                      uint64_t seed, void *work, size_t work_bytes, lrsdp_cert *out);

}  // namespace lrsdp

struct lrsdp_problem {
    lrsdp_problem_info info{};
    // host data
    std::vector<int32_t> row_ptr, col, heavy, heavy_seg, perm;
    std::vector<int4> light;
    std::vector<int4> seg;
    std::vector<double> val, diag, hrow;
    std::vector<int32_t> top_ptr, top_col, top_eid, bot_ptr, bot_row, bot_eid, samp_i, samp_j;
    std::vector<double> b;
    std::vector<int32_t> om_a, om_b, a_ptr, a_idx, at_ptr, at_idx, s_ptr, s_col, s_om, con_short, con_long;
    std::vector<double> cval, a_val, at_val, cdense;
    std::vector<int64_t> block_off;     // general problems of several blocks: row offsets (nblocks + 1)
    std::vector<int32_t> row_rank;      // general problems with block ranks: columns of R per row
    // device views (valid after upload)
    lrsdp::DevCsr csr;
    lrsdp::DevCompletion cmp;
    lrsdp::DevGeneral gen;
    void *dev = nullptr;
    size_t dev_bytes = 0;
    bool uploaded = false;
};

struct lrsdp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void *scratch = nullptr;      // device: partial sums + solver state
    size_t scratch_bytes = 0;
    void *pinned = nullptr;       // host pinned read-back block
    size_t pinned_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    void *static_scratch = nullptr;  // device address of the allocation-free entry point's array
};
