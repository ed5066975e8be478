// General problems: the compressed linear map of Section 3.4 on the GPU.
//
// Omega holds the positions (a, b), a <= b, that are nonzero in C or in some
// A_k.  The constraint map runs in two passes:
//   k_gen_xbar  one lane group per position: the compressed outer product
//               xbar_o = X_ab + X_ba (a < b) or X_aa for X = U V^T (the
//               paper's CompressedOuterProduct, over every position of Omega
//               so that the C-weighted sums of the objective and the line
//               search come out of the same pass);
//   k_gen_cons  one thread per constraint: its row of the stacked matrix
//               (nonzero columns only) times xbar, plus the line-search or
//               ALM row terms; rows longer than kLongRow (a trace
//               constraint) go to k_gen_cons_long, a workgroup per row.
// The operator C - A*(y) is applied on the symmetric pattern of Omega in two
// passes: k_gen_sv streams over the positions and forms their values
// cs C_o - sum_k A_k,o y_k from the transposed stacked matrix (eq. At with the
// index set Omega) into the problem's second compressed buffer, then
// k_gen_spmm gathers one value and one row of V per stored entry.
//
// Dense storage of C (Section 3.5, last paragraph): Omega then holds the
// constraint positions only (C's entries there are zero) and C enters through
// the dense product W = cs C V (k_dense_mfma, float64 matrix cores, split over
// k, then k_dense_finish adds the splits in a fixed order).  The SpMM adds W
// to the sparse part row by row; the objective and line-search sums
// <C, U V^T> = sum_i U_i . (C V)_i come from the rows of the product.
#include <algorithm>

#include "device.h"
#include "kernels.h"

namespace lrsdp {
namespace {

int gen_grid(int64_t items, int per_block) {
    const int64_t need = (items + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, kMaxBlocks));
}

enum { kGenA = 0, kGenLS = 1, kGenRefresh = 2 };

template <typename S>
struct XbarArgs {
    const S *U;
    const S *V;         // kGenA: V; kGenLS: D (U = R); kGenRefresh: unused (U = R)
    int64_t ld;
    double *x1, *x2;    // per position: A: xbar(U V^T); LS: xbar(RD^T + DR^T), xbar(DD^T); refresh: xbar(RR^T)
    double cs;          // objective scale
    double *partials;   // LS: s[0] = <C, DD^T>, s[6] = <C, RD^T + DR^T>; refresh: s[0] = <C, RR^T>
    const SolverState *st;
};

template <typename S, int GS, int MODE>
__global__ __launch_bounds__(kBlock) void k_gen_xbar(DevGeneral P, XbarArgs<S> a) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    if (a.st && a.st->done) return;
    const int lane = threadIdx.x % GS, grp = threadIdx.x / GS;
    const bool active = lane * NV < a.ld;
    const CV zero = vzero(CV{});
    double s[kLsSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t o = (int64_t)blockIdx.x * GPB + grp; o < P.nom; o += (int64_t)gridDim.x * GPB) {
        const int32_t ia = P.om_a[o], ib = P.om_b[o];
        // a diagonal position counts X_aa once: half of the symmetric formula
        const double w = ia == ib ? 0.5 : 1.0;
        const int64_t ra = (int64_t)ia * a.ld, rb = (int64_t)ib * a.ld;
        const CV ua = chunk_or_zero(a.U + ra, lane, active);
        const CV ub = chunk_or_zero(a.U + rb, lane, active);
        if constexpr (MODE == kGenRefresh) {
            const double x = w * 2.0 * group_sum<GS>(vdot(ua, ub));
            if (lane == 0) {
                a.x1[o] = x;
                s[0] += a.cs * P.cval[o] * x;
            }
        } else {
            const CV va = chunk_or_zero(a.V + ra, lane, active);
            const CV vb = chunk_or_zero(a.V + rb, lane, active);
            if constexpr (MODE == kGenA) {
                const double x = w * group_sum<GS>(vdot(ua, vb) + vdot(ub, va));
                if (lane == 0) a.x1[o] = x;
            } else {
                const double q1 = w * 2.0 * group_sum<GS>(vdot(ua, vb) + vdot(ub, va));
                const double q2 = w * 2.0 * group_sum<GS>(vdot(va, vb));
                if (lane == 0) {
                    a.x1[o] = q1;
                    a.x2[o] = q2;
                    const double c = a.cs * P.cval[o];
                    s[0] += c * q2;
                    s[6] += c * q1;
                }
            }
        }
    }
    if constexpr (MODE != kGenA) block_sums_store<kLsSums>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

struct ConsArgs {
    const double *x1, *x2;
    double *out;          // A: A(U V^T); refresh: constraint values (nullable)
    double *q1, *q2;      // LS outputs (nullable)
    const double *ytil;   // LS
    double *y;            // refresh: multipliers
    double sigma;         // refresh: y <- y + sigma (b - a) when > 0
    double *partials;
    const SolverState *st;
};

// the terms of constraint k once its row sums t1 (and t2) are known
template <int MODE>
__device__ __forceinline__ void cons_epilogue(const DevGeneral &P, const ConsArgs &a, int64_t k, double t1,
                                              double t2, double (&s)[kLsSums]) {
    if constexpr (MODE == kGenA) {
        a.out[k] = t1;
    } else if constexpr (MODE == kGenLS) {
        if (a.q1) a.q1[k] = t1;
        if (a.q2) a.q2[k] = t2;
        const double yt = a.ytil[k];
        s[1] += yt * t2;
        s[2] += yt * t1;
        s[3] += t2 * t2;
        s[4] += t1 * t2;
        s[5] += t1 * t1;
    } else {
        const double res = t1 - P.b[k];
        double yk = a.y[k];
        if (a.sigma > 0.0) {
            yk -= a.sigma * res;
            a.y[k] = yk;
        }
        if (a.out) a.out[k] = t1;
        s[1] += P.b[k] * yk;
        s[2] += res * res;
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_gen_cons(DevGeneral P, ConsArgs a) {
    if (a.st && a.st->done) return;
    double s[kLsSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P.n_short; i += (int64_t)gridDim.x * kBlock) {
        const int64_t k = P.con_short[i];
        double t1 = 0.0, t2 = 0.0;
        for (int t = P.a_ptr[k]; t < P.a_ptr[k + 1]; ++t) {
            const double v = P.a_val[t];
            const int32_t o = P.a_idx[t];
            t1 = fma(v, a.x1[o], t1);
            if constexpr (MODE == kGenLS) t2 = fma(v, a.x2[o], t2);
        }
        cons_epilogue<MODE>(P, a, k, t1, t2, s);
    }
    if constexpr (MODE != kGenA) block_sums_store<kLsSums>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

// One workgroup per long constraint row: the threads stride over the row, a
// fixed wavefront/LDS tree adds their sums (deterministic), thread 0 takes the
// epilogue.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_gen_cons_long(DevGeneral P, ConsArgs a) {
    if (a.st && a.st->done) return;
    __shared__ double sh[kBlock / 64][2];
    double s[kLsSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t i = blockIdx.x; i < P.n_long; i += gridDim.x) {
        const int64_t k = P.con_long[i];
        double t1 = 0.0, t2 = 0.0;
        for (int t = P.a_ptr[k] + threadIdx.x; t < P.a_ptr[k + 1]; t += kBlock) {
            const double v = P.a_val[t];
            const int32_t o = P.a_idx[t];
            t1 = fma(v, a.x1[o], t1);
            if constexpr (MODE == kGenLS) t2 = fma(v, a.x2[o], t2);
        }
        t1 = wave_sum(t1);
        t2 = wave_sum(t2);
        __syncthreads();                      // sh of the previous row has been read
        if (lane == 0) {
            sh[wave][0] = t1;
            sh[wave][1] = t2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double r1 = 0.0, r2 = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) {
                r1 += sh[w][0];
                r2 += sh[w][1];
            }
            cons_epilogue<MODE>(P, a, k, r1, r2, s);
        }
    }
    if constexpr (MODE != kGenA) block_sums_store<kLsSums>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

template <typename S>
struct GenSpmmArgs {
    const S *V;
    S *Y;
    const double *ytil;   // nullable: then the operator is cs C
    double cs;
    int64_t ld;
    const SolverState *st;
    int force_slot;       // >= 0: write G into this slot and ignore st->done (subproblem start)
    Rings<S> rings;
    double *partials;
    const S *addw;        // dense C: the rows of cs C V, added to the sparse part (nullable)
};

// x2[o] = value of cs C - A*(ytil) at position o (skipped when st says the
// subproblem is finished)
__global__ __launch_bounds__(kBlock) void k_gen_sv(DevGeneral P, const double *ytil, double cs,
                                                   const SolverState *st) {
    if (st && st->done) return;
    for (int64_t o = (int64_t)blockIdx.x * kBlock + threadIdx.x; o < P.nom; o += (int64_t)gridDim.x * kBlock) {
        double v = cs * P.cval[o];
        if (ytil)
            for (int t = P.at_ptr[o]; t < P.at_ptr[o + 1]; ++t) v = fma(-P.at_val[t], ytil[P.at_idx[t]], v);
        P.x2[o] = v;
    }
}

// GRAD = false: Y = (cs C - A*(ytil)) V.  GRAD = true: G_{k+1} = 2 (cs C - A*(ytil)) R
// into G slot (gk+1) mod (T+1), plus its dots with every ring slot.  TM: the
// largest memory the instance handles (T <= TM); the ring loops run to TM, so
// the common T <= 2 build keeps its ring pointers in registers.
template <typename S, int GS, bool GRAD, int TM>
__global__ __launch_bounds__(kBlock) void k_gen_spmm(DevGeneral P, GenSpmmArgs<S> a) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    int T = 0, gk1 = 0;
    S *Gn = nullptr;
    if constexpr (GRAD) {
        if (a.force_slot < 0 && a.st->done) return;
        T = a.st->T;
        gk1 = a.force_slot >= 0 ? a.force_slot : (a.st->gk + 1) % (T + 1);
#pragma unroll
        for (int g = 0; g <= TM; ++g)
            if (g == gk1) Gn = a.rings.g[g];
    }
    const int lane = threadIdx.x % GS, grp = threadIdx.x / GS;
    const bool active = lane * NV < a.ld;
    const CV zero = vzero(CV{});
    double s[kMaxBasis];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j) s[j] = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * GPB + grp; row < P.n; row += (int64_t)gridDim.x * GPB) {
        D4 acc{{0.0, 0.0, 0.0, 0.0}};
        const int e0 = P.s_ptr[row], e1 = P.s_ptr[row + 1];
        int e = e0;
        for (; e + 4 <= e1; e += 4) {
            CV v[4];
            double w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v[q] = chunk_or_zero(a.V + (int64_t)P.s_col[e + q] * a.ld, lane, active);
                w[q] = P.x2[P.s_om[e + q]];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const D4 vq = widen(v[q]);
#pragma unroll
                for (int c = 0; c < 4; ++c) acc.v[c] = fma(w[q], vq.v[c], acc.v[c]);
            }
        }
        for (; e < e1; ++e) {
            const CV v0 = chunk_or_zero(a.V + (int64_t)P.s_col[e] * a.ld, lane, active);
            const double w0 = P.x2[P.s_om[e]];
            const D4 vq = widen(v0);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc.v[c] = fma(w0, vq.v[c], acc.v[c]);
        }
        const int64_t rbase = row * a.ld, off = rbase + lane * NV;
        if (a.addw) {
            const D4 wv = widen(chunk_or_zero(a.addw + rbase, lane, active));
#pragma unroll
            for (int c = 0; c < 4; ++c) acc.v[c] += wv.v[c];
        }
        D4 o;
#pragma unroll
        for (int c = 0; c < 4; ++c) o.v[c] = GRAD ? 2.0 * acc.v[c] : acc.v[c];
        if constexpr (GRAD) {
            if (P.row_rank) {   // block ranks: the gradient of the free entries only
                const int lim = P.row_rank[row];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (lane * NV + c >= lim) o.v[c] = 0.0;
            }
        }
        CV os;
        narrow(o, os);
        if constexpr (!GRAD) {
            if (active) *reinterpret_cast<CV *>(a.Y + off) = os;
        } else {
            if (active) *reinterpret_cast<CV *>(Gn + off) = os;
#pragma unroll
            for (int g = 0; g <= TM; ++g) {
                if (g <= T) {
                    CV bsl = (g == gk1) ? os : chunk_or_zero<S>(a.rings.g[g] + rbase, lane, active);
                    s[g] += vdot(os, bsl);
                }
            }
#pragma unroll
            for (int d = 0; d < TM; ++d) {
                if (d < T) {
                    CV bsl = chunk_or_zero<S>(a.rings.d[d] + rbase, lane, active);
                    s[kMaxMem + 1 + d] += vdot(os, bsl);
                }
            }
        }
    }
    if constexpr (GRAD) block_sums_store<kMaxBasis>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

// ---------------------------------------------------------------------------
// Dense C: W = C V on float64 matrix cores.  A workgroup of four wavefronts
// owns kDBM = 64 rows of C and one range of k; each wavefront owns 16 rows and
// every 16-column tile of V (NT tiles, ld <= 16 NT), and runs
// v_mfma_f64_16x16x4f64 over the range: A operand lane l = C[row l%16][k + l/16],
// B operand lane l = V[k + l/16][col l%16], result register i of lane l holds
// row l/16 + 4 i, column l%16.  C and V go through LDS in stages of kDKC = 64
// values of k: a stage reads 64 rows x 512 contiguous bytes of C (each
// iteration of the load loop four whole 512-byte row segments), all of them
// issued before the first is stored, then 16 MFMA steps per tile.
// ---------------------------------------------------------------------------
constexpr int kDBM = 64;
constexpr int kDKC = 64;

typedef double dense_acc_t __attribute__((ext_vector_type(4)));

template <typename S, int NT>
__global__ __launch_bounds__(kBlock) void k_dense_mfma(const double *__restrict__ C, const S *__restrict__ V,
                                                       int64_t n, int64_t ld, int64_t kspan,
                                                       double *__restrict__ part, const SolverState *st) {
    if (st && st->done) return;
    constexpr int LDP = 16 * NT;
    constexpr int CL = kDBM * kDKC / kBlock;   // C values per thread per stage
    constexpr int VL = kDKC * LDP / kBlock;    // V values per thread per stage
    __shared__ double Cs[kDBM][kDKC + 1];
    __shared__ double Vs[kDKC][LDP + 1];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int64_t r0 = (int64_t)blockIdx.x * kDBM;
    const int64_t k0 = (int64_t)blockIdx.y * kspan, k1 = min(n, k0 + kspan);
    dense_acc_t acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = dense_acc_t{0.0, 0.0, 0.0, 0.0};
    for (int64_t kb = k0; kb < k1; kb += kDKC) {
        double cv[CL], vv[VL];
#pragma unroll
        for (int e = 0; e < CL; ++e) {
            const int t = threadIdx.x + e * kBlock;
            const int rr = t / kDKC, kk = t % kDKC;
            const int64_t gr = r0 + rr, gk = kb + kk;
            const bool use = gr < n && gk < k1;
            const double x = C[(use ? gr : r0) * n + (use ? gk : k0)];   // a valid address either way
            cv[e] = use ? x : 0.0;
        }
#pragma unroll
        for (int e = 0; e < VL; ++e) {
            const int t = threadIdx.x + e * kBlock;
            const int kk = t / LDP, cc = t % LDP;
            const int64_t gk = kb + kk;
            const bool use = gk < k1 && cc < ld;
            const double x = (double)V[(use ? gk : k0) * ld + (use ? cc : 0)];
            vv[e] = use ? x : 0.0;
        }
#pragma unroll
        for (int e = 0; e < CL; ++e) {
            const int t = threadIdx.x + e * kBlock;
            Cs[t / kDKC][t % kDKC] = cv[e];
        }
#pragma unroll
        for (int e = 0; e < VL; ++e) {
            const int t = threadIdx.x + e * kBlock;
            Vs[t / LDP][t % LDP] = vv[e];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kDKC; kk += 4) {
            const double a = Cs[wave * 16 + (lane % 16)][kk + lane / 16];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double b = Vs[kk + lane / 16][t * 16 + lane % 16];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    constexpr int RW = (int)(kDenseRowBytes / sizeof(double));
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = r0 + wave * 16 + lane / 16 + 4 * i;
            if (row < n) part[((int64_t)blockIdx.y * n + row) * RW + t * 16 + lane % 16] = acc[t][i];
        }
    }
}

enum { kDenseStore = 0, kDenseLS = 1, kDenseRefresh = 2 };

// Adds the k splits of each row in split order and scales by cs.  kDenseStore:
// W_i = cs (C V)_i in the storage type; kDenseLS (V = D): s[0] += D_i . cs (C D)_i,
// s[6] += 2 R_i . cs (C D)_i; kDenseRefresh (V = R): s[0] += R_i . cs (C R)_i.
// A group of GS lanes per row, one column each (GS >= ld), so that the split
// partials and the rows of U, V, W are read and written as contiguous segments;
// the row dots are summed by the block's fixed tree.
template <typename S, int MODE, int GS>
__global__ __launch_bounds__(kBlock) void k_dense_finish(const double *__restrict__ part, int ks, int64_t n,
                                                         int64_t ld, double cs, S *W, const S *U, const S *V,
                                                         double *partials, const SolverState *st) {
    if (st && st->done) return;
    constexpr int RW = (int)(kDenseRowBytes / sizeof(double));
    constexpr int GPB = kBlock / GS;
    const int lane = threadIdx.x % GS, grp = threadIdx.x / GS;
    const bool act = lane < ld;
    const int c = act ? lane : 0;
    double s[kLsSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t row = (int64_t)blockIdx.x * GPB + grp; row < n; row += (int64_t)gridDim.x * GPB) {
        double v = 0.0;
        for (int k = 0; k < ks; ++k) v += part[((int64_t)k * n + row) * RW + c];
        v *= cs;
        if constexpr (MODE == kDenseStore) {
            if (act) W[row * ld + c] = (S)v;
        } else if constexpr (MODE == kDenseLS) {
            const double dv = (double)V[row * ld + c], du = (double)U[row * ld + c];
            s[0] += act ? dv * v : 0.0;
            s[6] += act ? 2.0 * du * v : 0.0;
        } else {
            const double du = (double)U[row * ld + c];
            s[0] += act ? du * v : 0.0;
        }
    }
    if constexpr (MODE != kDenseStore) block_sums_store<kLsSums>(s, partials + (size_t)blockIdx.x * kMaxSums);
}

constexpr int kDenseFinishBlocks = 256;

template <typename S, int GS>
void finish_launch(hipStream_t s, const DevGeneral &P, int mode, int ks, int64_t ld, double cs, const S *U,
                   const S *V, double *partials, const SolverState *st, int *nf) {
    const int64_t n = P.n;
    const int64_t need = (n + kBlock / GS - 1) / (kBlock / GS);
    *nf = (int)std::min<int64_t>(need, kDenseFinishBlocks);
    if (mode == kDenseStore)
        hipLaunchKernelGGL((k_dense_finish<S, kDenseStore, GS>), dim3(*nf), dim3(kBlock), 0, s, P.dpart, ks, n, ld,
                           cs, (S *)P.dw, U, V, partials, st);
    else if (mode == kDenseLS)
        hipLaunchKernelGGL((k_dense_finish<S, kDenseLS, GS>), dim3(*nf), dim3(kBlock), 0, s, P.dpart, ks, n, ld, cs,
                           (S *)nullptr, U, V, partials, st);
    else
        hipLaunchKernelGGL((k_dense_finish<S, kDenseRefresh, GS>), dim3(*nf), dim3(kBlock), 0, s, P.dpart, ks, n, ld,
                           cs, (S *)nullptr, U, V, partials, st);
}

// W = cs C V (MODE kDenseStore) or the dense sums of the LS / refresh pass into
// partial rows (*nb rows written).  V, U: n x ld of S.
template <typename S>
int dense_product(hipStream_t s, const DevGeneral &P, int mode, const S *V, const S *U, int64_t ld, double cs,
                  double *partials, const SolverState *st, int *nb) {
    *nb = 0;
    const int64_t n = P.n;
    const int64_t rb = (n + kDBM - 1) / kDBM;
    int ks = (int)std::min<int64_t>(kDenseMaxSplit, std::max<int64_t>(1, (512 + rb - 1) / rb));
    ks = (int)std::max<int64_t>(1, std::min<int64_t>(ks, (n + kDKC - 1) / kDKC));
    const int64_t kspan = ((n + ks - 1) / ks + kDKC - 1) / kDKC * kDKC;
    ks = (int)((n + kspan - 1) / kspan);
    const dim3 g((unsigned)rb, (unsigned)ks);
    if (ld <= 16) hipLaunchKernelGGL((k_dense_mfma<S, 1>), g, dim3(kBlock), 0, s, P.cd, V, n, ld, kspan, P.dpart, st);
    else if (ld <= 32) hipLaunchKernelGGL((k_dense_mfma<S, 2>), g, dim3(kBlock), 0, s, P.cd, V, n, ld, kspan, P.dpart, st);
    else hipLaunchKernelGGL((k_dense_mfma<S, 4>), g, dim3(kBlock), 0, s, P.cd, V, n, ld, kspan, P.dpart, st);
    LRSDP_CHECK_LAUNCH();
    int nf = 0;
    if (ld <= 32) finish_launch<S, 32>(s, P, mode, ks, ld, cs, U, V, partials, st, &nf);
    else finish_launch<S, 64>(s, P, mode, ks, ld, cs, U, V, partials, st, &nf);
    LRSDP_CHECK_LAUNCH();
    if (mode != kDenseStore) *nb = nf;
    return LRSDP_OK;
}

template <typename S>
int gs_of_gen(int64_t ld) {
    const int ch = (int)(ld * (int64_t)sizeof(S) / 16);
    return ch <= 4 ? 4 : (ch <= 8 ? 8 : 16);
}

template <typename S, int MODE>
int xbar_t(hipStream_t s, const DevGeneral &P, const XbarArgs<S> &a, int *nb) {
    const int gs = gs_of_gen<S>(a.ld);
    // with dense C the dense sums take partial rows after the constraint rows:
    // the positions pass keeps to half the grid so that all stay within
    // 2 kMaxBlocks rows
    *nb = std::min(gen_grid(P.nom, kBlock / gs), P.cd ? kMaxBlocks / 2 : kMaxBlocks);
    if (gs == 4) hipLaunchKernelGGL((k_gen_xbar<S, 4, MODE>), dim3(*nb), dim3(kBlock), 0, s, P, a);
    else if (gs == 8) hipLaunchKernelGGL((k_gen_xbar<S, 8, MODE>), dim3(*nb), dim3(kBlock), 0, s, P, a);
    else hipLaunchKernelGGL((k_gen_xbar<S, 16, MODE>), dim3(*nb), dim3(kBlock), 0, s, P, a);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

// With long rows present the two constraint kernels use at most kMaxBlocks / 2
// workgroups each, so that with the positions pass the partial rows stay
// within 2 kMaxBlocks; without them the short-row kernel keeps the full grid.
template <int MODE>
int cons_t(hipStream_t s, const DevGeneral &P, const ConsArgs &a, int *nb) {
    const int nb_short = std::min(gen_grid(P.n_short, kBlock), P.n_long > 0 ? kMaxBlocks / 2 : kMaxBlocks);
    hipLaunchKernelGGL((k_gen_cons<MODE>), dim3(nb_short), dim3(kBlock), 0, s, P, a);
    *nb = nb_short;
    if (P.n_long > 0) {
        ConsArgs b = a;
        if (b.partials) b.partials += (size_t)nb_short * kMaxSums;
        const int nb_long = (int)std::min<int64_t>(P.n_long, kMaxBlocks / 2);
        hipLaunchKernelGGL((k_gen_cons_long<MODE>), dim3(nb_long), dim3(kBlock), 0, s, P, b);
        *nb += nb_long;
    }
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

template <typename S, int MODE>
int sddmm_t(hipStream_t s, const DevGeneral &P, const void *U, const void *V, int64_t ld, double *out, double *q1,
            double *q2, const double *ytil, double *y, double sigma, double cs, double *partials,
            const SolverState *st, int *nb, bool dense_sums) {
    XbarArgs<S> xa{(const S *)U, (const S *)V, ld, P.x1, P.x2, cs, partials, st};
    int nb1 = 0, nb2 = 0, rc;
    if ((rc = xbar_t<S, MODE>(s, P, xa, &nb1))) return rc;
    if (MODE == kGenA) nb1 = 0;   // no partial sums from the first pass
    ConsArgs ca{P.x1, P.x2, out, q1, q2, ytil, y, sigma, partials ? partials + (size_t)nb1 * kMaxSums : nullptr,
                st};
    if ((rc = cons_t<MODE>(s, P, ca, &nb2))) return rc;
    int nb3 = 0;
    if (P.cd && MODE != kGenA && dense_sums) {
        // <C, DD^T>, <C, RD^T + DR^T> (LS, V = D) or <C, RR^T> (refresh) from the dense product
        const S *Vd = MODE == kGenLS ? (const S *)V : (const S *)U;
        if ((rc = dense_product<S>(s, P, MODE == kGenLS ? kDenseLS : kDenseRefresh, Vd, (const S *)U, ld, cs,
                                   partials + (size_t)(nb1 + nb2) * kMaxSums, st, &nb3)))
            return rc;
    }
    *nb = MODE == kGenA ? 0 : nb1 + nb2 + nb3;
    return LRSDP_OK;
}

template <typename S, bool GRAD, int TM>
int gen_spmm_tm(hipStream_t s, const DevGeneral &P, const GenSpmmArgs<S> &a, int *nb) {
    // values first (the gradient call of a finished subproblem skips both)
    const SolverState *skip = (GRAD && a.force_slot < 0) ? a.st : nullptr;
    GenSpmmArgs<S> b = a;
    if (P.cd) {
        int nbd = 0, rc;
        if ((rc = dense_product<S>(s, P, kDenseStore, a.V, nullptr, a.ld, a.cs, nullptr, skip, &nbd))) return rc;
        b.addw = (const S *)P.dw;
    }
    hipLaunchKernelGGL(k_gen_sv, dim3(gen_grid(P.nom, kBlock)), dim3(kBlock), 0, s, P, a.ytil, a.cs, skip);
    const int gs = gs_of_gen<S>(a.ld);
    *nb = gen_grid(P.n, kBlock / gs);
    if (gs == 4) hipLaunchKernelGGL((k_gen_spmm<S, 4, GRAD, TM>), dim3(*nb), dim3(kBlock), 0, s, P, b);
    else if (gs == 8) hipLaunchKernelGGL((k_gen_spmm<S, 8, GRAD, TM>), dim3(*nb), dim3(kBlock), 0, s, P, b);
    else hipLaunchKernelGGL((k_gen_spmm<S, 16, GRAD, TM>), dim3(*nb), dim3(kBlock), 0, s, P, b);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

// Block ranks: zero the entries of R past its row's rank (n x ld, storage type).
template <typename S>
__global__ __launch_bounds__(kBlock) void k_gen_rank_mask(const int32_t *row_rank, S *R, int64_t n, int64_t ld) {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * ld; e += (int64_t)gridDim.x * kBlock) {
        const int64_t i = e / ld, c = e - i * ld;
        if (c >= row_rank[i]) R[e] = (S)0;
    }
}

// T: L-BFGS memory of the gradient call (0 for the plain SpMM)
template <typename S, bool GRAD>
int gen_spmm_t(hipStream_t s, const DevGeneral &P, const GenSpmmArgs<S> &a, int *nb, int T = 0) {
    if (!GRAD) return gen_spmm_tm<S, false, 0>(s, P, a, nb);
    if (T <= 2) return gen_spmm_tm<S, GRAD, 2>(s, P, a, nb);
    return gen_spmm_tm<S, GRAD, kMaxMem>(s, P, a, nb);
}

}  // namespace

int gen_rank_mask(hipStream_t s, const DevGeneral &P, int prec, void *R, int64_t ld) {
    if (!P.row_rank || P.n <= 0) return LRSDP_OK;
    const int nb = gen_grid(P.n * ld, kBlock);
    if (prec == LRSDP_F64)
        hipLaunchKernelGGL(k_gen_rank_mask<double>, dim3(nb), dim3(kBlock), 0, s, P.row_rank, (double *)R, P.n, ld);
    else
        hipLaunchKernelGGL(k_gen_rank_mask<float>, dim3(nb), dim3(kBlock), 0, s, P.row_rank, (float *)R, P.n, ld);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

// mode 0: out = A(U V^T); mode 1: line-search terms of direction V at U with
// ytil (partials: {<C,DD^T>, ytil.q2, ytil.q1, q2.q2, q1.q2, q1.q1, <C,RD^T+DR^T>});
// mode 2: constraint values (into out when given) and the multiplier step,
// partials {<C,RR^T>, b.y, ||A(RR^T) - b||^2}.  *nb = partial rows written.
// dense_sums = false: a refresh pass whose partial sums the caller does not
// read (constraint values only) skips the dense C product for <C, RR^T>.
int gen_sddmm(hipStream_t s, const DevGeneral &P, int prec, int mode, const void *U, const void *V, int64_t ld,
              double *out, double *q1, double *q2, const double *ytil, double *y, double sigma, double cs,
              double *partials, const SolverState *st, int *nb, bool dense_sums) {
    const bool ds = dense_sums || mode != kGenRefresh;
    if (prec == LRSDP_F64) {
        if (mode == kGenA)
            return sddmm_t<double, kGenA>(s, P, U, V, ld, out, q1, q2, ytil, y, sigma, cs, partials, st, nb, ds);
        if (mode == kGenLS)
            return sddmm_t<double, kGenLS>(s, P, U, V, ld, out, q1, q2, ytil, y, sigma, cs, partials, st, nb, ds);
        return sddmm_t<double, kGenRefresh>(s, P, U, V, ld, out, q1, q2, ytil, y, sigma, cs, partials, st, nb, ds);
    }
    if (mode == kGenA)
        return sddmm_t<float, kGenA>(s, P, U, V, ld, out, q1, q2, ytil, y, sigma, cs, partials, st, nb, ds);
    if (mode == kGenLS)
        return sddmm_t<float, kGenLS>(s, P, U, V, ld, out, q1, q2, ytil, y, sigma, cs, partials, st, nb, ds);
    return sddmm_t<float, kGenRefresh>(s, P, U, V, ld, out, q1, q2, ytil, y, sigma, cs, partials, st, nb, ds);
}

int spmm_general(hipStream_t s, const DevGeneral &P, int prec, const void *V, int64_t ld, const double *ytil,
                 void *Y) {
    int nb = 0;
    if (prec == LRSDP_F64) {
        GenSpmmArgs<double> a{(const double *)V, (double *)Y, ytil, 1.0, ld, nullptr, -1, {}, nullptr, nullptr};
        return gen_spmm_t<double, false>(s, P, a, &nb);
    }
    GenSpmmArgs<float> a{(const float *)V, (float *)Y, ytil, 1.0, ld, nullptr, -1, {}, nullptr, nullptr};
    return gen_spmm_t<float, false>(s, P, a, &nb);
}

int gen_grad(hipStream_t s, const DevGeneral &P, int prec, const SolverState *st, const void *R,
             const double *ytil, void *const *gring, void *const *dring, int T, int64_t ld, double *partials,
             int force_slot, int *nb, double cs) {
    if (prec == LRSDP_F64) {
        GenSpmmArgs<double> a{(const double *)R, nullptr, ytil, cs, ld, st, force_slot, {}, partials, nullptr};
        for (int g = 0; g <= T; ++g) a.rings.g[g] = (double *)gring[g];
        for (int d = 0; d < T; ++d) a.rings.d[d] = (double *)dring[d];
        return gen_spmm_t<double, true>(s, P, a, nb, T);
    }
    GenSpmmArgs<float> a{(const float *)R, nullptr, ytil, cs, ld, st, force_slot, {}, partials, nullptr};
    for (int g = 0; g <= T; ++g) a.rings.g[g] = (float *)gring[g];
    for (int d = 0; d < T; ++d) a.rings.d[d] = (float *)dring[d];
    return gen_spmm_t<float, true>(s, P, a, nb, T);
}

}  // namespace lrsdp
