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
    // Work lists.  Light rows (<= kSegLen nonzeros) sorted by decreasing length
    // inside windows of consecutive rows; heavy rows split into segments.
    const int32_t *light = nullptr;     // n_light row ids
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

}  // namespace lrsdp

struct lrsdp_problem {
    lrsdp_problem_info info{};
    // host data
    std::vector<int32_t> row_ptr, col, light, heavy, heavy_seg;
    std::vector<int4> seg;
    std::vector<double> val, diag, hrow;
    std::vector<int32_t> top_ptr, top_col, top_eid, bot_ptr, bot_row, bot_eid, samp_i, samp_j;
    std::vector<double> b;
    // device views (valid after upload)
    lrsdp::DevCsr csr;
    lrsdp::DevCompletion cmp;
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
};
