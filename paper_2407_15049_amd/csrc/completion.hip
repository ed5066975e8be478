// Matrix-completion kernels (paper, matrix-completion section): X of order
// n = n1 + n2, C = I, sample k = (i, j) with A_k = E_{i,n1+j} + E_{n1+j,i} and
// b_k = 2 M_ij.
//
//  * SpMM  Y = (I - A*(ytil)) V  (eq. At): top row i gathers the rows n1+j of its
//    samples, bottom row n1+j gathers the rows i of its samples, each weighted by
//    -ytil_k (sample id from the CSR).  One lane group per row, rows in order.
//  * SDDMM over samples (the compressed outer product of Section 3.3): a lane
//    group owns a top row i, keeps U_i (and D_i) in registers and walks the row's
//    samples, gathering the partner rows n1+j:
//      kSddA        out_k = <A_k, U V^T> = U_i . V_{n1+j} + U_{n1+j} . V_i
//      kSddLS       q1_k = 2 (R_i . D_{n1+j} + D_i . R_{n1+j}), q2_k = 2 D_i . D_{n1+j},
//                   sums ytil.q2, ytil.q1, q2.q2, q1.q2, q1.q1 (appendix A.2)
//      kSddRefresh  a_k = 2 R_i . R_{n1+j}, optional multiplier step
//                   y_k <- y_k - sigma (a_k - b_k); sums b.y, ||a - b||^2
//  * the gradient SpMM of the solve, G = 2 (I - A*(ytil)) R, whose epilogue also
//    takes the dot products of the new G with every L-BFGS ring slot.
#include "device.h"
#include "kernels.h"

namespace lrsdp {
namespace {

enum { kSddA = 0, kSddLS = 1, kSddRefresh = 2 };

template <typename S>
struct CmpSpmmArgs {
    const S *V;
    S *Y;
    const double *ytil;   // m (nullable: then Y = V)
    int64_t ld;
    // gradient mode
    const SolverState *st;
    int force_slot;       // >= 0: write G into this slot and ignore st->done (subproblem start)
    Rings<S> rings;       // G slots 0..T, D slots 0..T-1
    double *partials;
    double cs;            // objective scale: C = cs I
};

// acc += sum over the row's samples of ytil_k * V_partner  (this lane's chunk).
// The GS lanes of the group take the row's samples PW at a time: each lane
// loads the partner index and the weight ytil_k of PW / GS samples (coalesced
// index loads, the ytil gathers of all of them in flight at once), then the
// partner rows are fetched eight at a time with the indices and weights handed
// round by lane shuffles.  The products are added in sample order, which
// rounds exactly as a sequential walk over the row does.
template <typename S, int GS>
__device__ __forceinline__ void cmp_gather(const int32_t *__restrict__ ptr, const int32_t *__restrict__ nbr,
                                           const int32_t *__restrict__ eid, int row, int64_t base,
                                           const double *__restrict__ ytil, const S *__restrict__ V, int64_t ld,
                                           int lane, bool active, typename Chunk<S>::V &acc) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int PW = GS < 16 ? 16 : GS;   // samples per pass
    constexpr int NT = PW / GS;             // samples per lane and pass
    constexpr int KB = 8;                   // partner rows in flight per lane
    const int b = ptr[row], e = ptr[row + 1];
    if (b >= e) return;
    // Indices and weights of the pass starting at k (k < e): every lane loads,
    // past the row's end repeating the last sample (the gather below stops at
    // the pass's count, so those entries are never used), so that no load sits
    // behind a branch: all index loads, then all ytil gathers, are in flight
    // together.
    auto load_pass = [&](int k, int32_t(&j)[NT], double(&w)[NT]) {
        const int cnt = min(PW, e - k);
        int32_t ev[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int q = min(lane + t * GS, cnt - 1);
            j[t] = nbr[k + q];
            ev[t] = eid[k + q];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) w[t] = ytil[ev[t]];
    };
    // indices and weights of the first pass; each pass loads the next one's
    // before its own partner rows, so their latency overlaps the gather (the
    // next weights stay float64 until the pass ends, so that no conversion
    // waits for them early)
    int32_t jj[NT];
    S ww[NT];
    {
        double w0[NT];
        load_pass(b, jj, w0);
#pragma unroll
        for (int t = 0; t < NT; ++t) ww[t] = (S)w0[t];
    }
    for (int k0 = b; k0 < e; k0 += PW) {
        const int cnt = min(PW, e - k0);     // the same for every lane of the group
        int32_t jn[NT] = {};
        double wn[NT] = {};
        const int k1 = k0 + PW;
        if (k1 < e) load_pass(k1, jn, wn);
#pragma unroll
        for (int q0 = 0; q0 < PW; q0 += KB) {
            if (q0 >= cnt) break;
            int64_t j[KB];
            S w[KB];
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                j[q] = base + __shfl(jj[(q0 + q) / GS], (q0 + q) % GS, GS);
                w[q] = __shfl(ww[(q0 + q) / GS], (q0 + q) % GS, GS);
            }
            if (active) {
                CV v[KB];
#pragma unroll
                for (int q = 0; q < KB; ++q)
                    if (q0 + q < cnt) v[q] = *reinterpret_cast<const CV *>(V + j[q] * ld + lane * NV);
#pragma unroll
                for (int q = 0; q < KB; ++q)
                    if (q0 + q < cnt) vfma(acc, w[q], v[q]);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            jj[t] = jn[t];
            ww[t] = (S)wn[t];
        }
    }
}

// GRAD = false: Y = cs V - A*(ytil) V.  GRAD = true: G_{k+1} = 2 (cs R - A*(ytil) R)
// into G slot (gk+1) mod (T+1), plus its dots with every ring slot.  TM: the
// largest memory the build handles (T <= TM).
template <typename S, int GS, bool GRAD, int TM>
__global__ __launch_bounds__(kBlock) void k_cmp_spmm(DevCompletion P, CmpSpmmArgs<S> a) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    int T = 0, gk = 0, gk1 = 0;
    S *Gn = nullptr;
    if constexpr (GRAD) {
        if (a.force_slot < 0 && a.st->done) return;
        T = a.st->T;
        gk = a.st->gk;
        gk1 = a.force_slot >= 0 ? a.force_slot : (gk + 1) % (T + 1);
#pragma unroll
        for (int g = 0; g <= TM; ++g)
            if (g == gk1) Gn = a.rings.g[g];
    }
    const int lane = threadIdx.x % GS, grp = threadIdx.x / GS;
    const bool active = lane * NV < a.ld;
    const CV zero = vzero(CV{});
    const int64_t n = P.n1 + P.n2;
    double s[kMaxBasis];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j) s[j] = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * GPB + grp; row < n; row += (int64_t)gridDim.x * GPB) {
        CV acc = zero;
        if (a.ytil) {
            if (row < P.n1)
                cmp_gather<S, GS>(P.top_ptr, P.top_col, P.top_eid, (int)row, P.n1, a.ytil, a.V, a.ld, lane, active, acc);
            else
                cmp_gather<S, GS>(P.bot_ptr, P.bot_row, P.bot_eid, (int)(row - P.n1), 0, a.ytil, a.V, a.ld, lane, active,
                              acc);
        }
        const int64_t rb = row * a.ld, off = rb + lane * NV;
        const CV v = chunk_or_zero(a.V + rb, lane, active);
        D4 vv = widen(v), aa = widen(acc), o;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double cv = a.cs * vv.v[c];
            o.v[c] = GRAD ? 2.0 * (cv - aa.v[c]) : cv - aa.v[c];
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
                    CV bsl = (g == gk1) ? os : chunk_or_zero<S>(a.rings.g[g] + rb, lane, active);
                    s[g] += vdot(os, bsl);
                }
            }
#pragma unroll
            for (int d = 0; d < TM; ++d) {
                if (d < T) {
                    CV bsl = chunk_or_zero<S>(a.rings.d[d] + rb, lane, active);
                    s[kMaxMem + 1 + d] += vdot(os, bsl);
                }
            }
        }
    }
    if constexpr (GRAD) block_sums_store<kMaxBasis>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

template <typename S>
struct SddArgs {
    const S *U;           // kSddA: U; LS / refresh: R
    const S *V;           // kSddA: V; LS: D
    int64_t ld;
    double *out;          // kSddA: A(UV^T); refresh: a (constraint values)
    double *q1, *q2;      // kSddLS outputs
    const double *ytil;   // kSddLS
    double *y;            // kSddRefresh
    double sigma;         // kSddRefresh
    double *partials;
    const SolverState *st;
};

template <typename S, int GS, int MODE>
__global__ __launch_bounds__(kBlock) void k_cmp_sddmm(DevCompletion P, SddArgs<S> a) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    if (a.st && a.st->done) return;
    const int lane = threadIdx.x % GS, grp = threadIdx.x / GS;
    const bool active = lane * NV < a.ld;
    const CV zero = vzero(CV{});
    double s[kLsSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * GPB + grp; i < P.n1; i += (int64_t)gridDim.x * GPB) {
        const int64_t ib = i * a.ld;
        const CV ui = chunk_or_zero(a.U + ib, lane, active);
        const CV vi = MODE != kSddRefresh ? chunk_or_zero(a.V + ib, lane, active) : zero;
        const int b = P.top_ptr[i], e = P.top_ptr[i + 1];
        // The row's samples PW at a time: each lane loads the partner index and
        // sample id of NT of them (coalesced; past the row's end it repeats the
        // last sample), then SS = 4 samples per step take them by lane shuffles,
        // with all eight partner-row loads in flight before the first reduction
        // (a step past the end repeats the last sample's loads and skips its
        // outputs).  NT = 2 for float64 rows; float32 rows keep one: the extra
        // index registers cost the float32 line-search build a wave per SIMD,
        // and eight samples per step with two index registers measured 682 us
        // against 500 us (mode A, n = 1e6, m = 1e7).  The next pass's indices
        // are loaded before this pass's partner rows, so their latency overlaps
        // the gather.
        constexpr int NT = sizeof(S) == 8 ? 2 : 1;
        constexpr int PW = NT * GS;
        constexpr int SS = 4;   // samples per step
        int32_t cc[NT], ee[NT];
        if (b < e) {
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const int tq = b + min(lane + u * GS, min(PW, e - b) - 1);
                cc[u] = P.top_col[tq];
                ee[u] = P.top_eid[tq];
            }
        }
        for (int t0 = b; t0 < e; t0 += PW) {
          const int cnt0 = min(PW, e - t0);
          int32_t cn[NT] = {}, en[NT] = {};
          const int t1 = t0 + PW;
          if (t1 < e) {
#pragma unroll
              for (int u = 0; u < NT; ++u) {
                  const int tq = t1 + min(lane + u * GS, min(PW, e - t1) - 1);
                  cn[u] = P.top_col[tq];
                  en[u] = P.top_eid[tq];
              }
          }
#pragma unroll
          for (int s0 = 0; s0 < PW; s0 += SS) {
            if (s0 >= cnt0) break;
            const int cnt = min(SS, cnt0 - s0);
            int64_t pj[SS];
            int kk[SS];
#pragma unroll
            for (int q = 0; q < SS; ++q) {
                const int src = s0 + q;   // compile-time register and lane
                pj[q] = (P.n1 + __shfl(cc[src / GS], src % GS, GS)) * a.ld;
                kk[q] = __shfl(ee[src / GS], src % GS, GS);
            }
            CV xu[SS], xv[SS];
#pragma unroll
            for (int q = 0; q < SS; ++q) {
                xu[q] = chunk_or_zero(a.U + pj[q], lane, active);
                xv[q] = MODE != kSddRefresh ? chunk_or_zero(a.V + pj[q], lane, active) : zero;
            }
            // the samples' own scalars, loaded by every lane with the rows (a
            // repeated sample past the row's end is a valid index) and taken
            // through selects, so that no load waits inside a lane-0 branch
            double sv0[SS], sv1[SS];
#pragma unroll
            for (int q = 0; q < SS; ++q) {
                if constexpr (MODE == kSddLS) sv0[q] = a.ytil[kk[q]];
                if constexpr (MODE == kSddRefresh) {
                    sv0[q] = P.b[kk[q]];
                    sv1[q] = a.y[kk[q]];
                }
            }
#pragma unroll
            for (int q = 0; q < SS; ++q) {
                const int k = kk[q];
                const bool own = lane == 0 && q < cnt;
                if constexpr (MODE == kSddA) {
                    // <A_k, U V^T> = U_i . V_{n1+j} + U_{n1+j} . V_i
                    const double d = group_sum<GS>(vdot(ui, xv[q]) + vdot(xu[q], vi));
                    if (own) a.out[k] = d;
                } else if constexpr (MODE == kSddLS) {
                    // R rows in xu, D rows in xv
                    const double q1 = 2.0 * group_sum<GS>(vdot(ui, xv[q]) + vdot(vi, xu[q]));
                    const double q2 = 2.0 * group_sum<GS>(vdot(vi, xv[q]));
                    const double yt = sv0[q];
                    s[1] += own ? yt * q2 : 0.0;
                    s[2] += own ? yt * q1 : 0.0;
                    s[3] += own ? q2 * q2 : 0.0;
                    s[4] += own ? q1 * q2 : 0.0;
                    s[5] += own ? q1 * q1 : 0.0;
                    if (own) {
                        if (a.q1) a.q1[k] = q1;
                        if (a.q2) a.q2[k] = q2;
                    }
                } else {
                    const double ak = 2.0 * group_sum<GS>(vdot(ui, xu[q]));
                    const double bk = sv0[q], res = ak - bk;
                    const double yk = a.sigma > 0.0 ? sv1[q] - a.sigma * res : sv1[q];
                    s[1] += own ? bk * yk : 0.0;
                    s[2] += own ? res * res : 0.0;
                    if (own) {
                        if (a.sigma > 0.0) a.y[k] = yk;
                        if (a.out) a.out[k] = ak;
                    }
                }
            }
          }
#pragma unroll
          for (int u = 0; u < NT; ++u) {
              cc[u] = cn[u];
              ee[u] = en[u];
          }
        }
    }
    if constexpr (MODE != kSddA) block_sums_store<kLsSums>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

// per sample: a_k += tau (q1_k + tau q2_k); ytil_k = y_k + sigma (b_k - a_k)
__global__ __launch_bounds__(kBlock) void k_cmp_samples(DevCompletion P, const SolverState *st, double *acon,
                                                        const double *q1, const double *q2, const double *y,
                                                        double *ytil) {
    if (st->done) return;
    const double tau = st->tau, sigma = st->sigma;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < P.m; k += (int64_t)gridDim.x * kBlock) {
        const double ak = acon[k] + tau * (q1[k] + tau * q2[k]);
        acon[k] = ak;
        ytil[k] = y[k] + sigma * (P.b[k] - ak);
    }
}

// ytil_k = y_k + sigma (b_k - a_k) with sigma from the state
__global__ __launch_bounds__(kBlock) void k_cmp_ytil(DevCompletion P, const SolverState *st, double sigma_arg,
                                                     const double *acon, const double *y, double *ytil) {
    const double sigma = st ? st->sigma : sigma_arg;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < P.m; k += (int64_t)gridDim.x * kBlock)
        ytil[k] = y[k] + sigma * (P.b[k] - acon[k]);
}

// R <- R + tau D (flat over 16-byte chunks), tau from the state
template <typename S>
__global__ __launch_bounds__(kBlock) void k_axpy_state(const SolverState *st, S *R, const S *D, int64_t nchunks) {
    using CV = typename Chunk<S>::V;
    if (st->done) return;
    const double tau = st->tau;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nchunks; c += (int64_t)gridDim.x * kBlock) {
        D4 r = widen(reinterpret_cast<const CV *>(R)[c]), d = widen(reinterpret_cast<const CV *>(D)[c]);
#pragma unroll
        for (int e = 0; e < 4; ++e) r.v[e] = fma(tau, d.v[e], r.v[e]);
        CV o;
        narrow(r, o);
        reinterpret_cast<CV *>(R)[c] = o;
    }
}

int grid(int64_t items, int per_block) {
    int64_t need = (items + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, kMaxBlocks));
}

template <typename S>
int gs_of(int64_t ld) {
    const int ch = (int)(ld * (int64_t)sizeof(S) / 16);
    return ch <= 4 ? 4 : (ch <= 8 ? 8 : 16);
}

template <typename S, bool GRAD, int TM>
int cmp_spmm_tm(hipStream_t s, const DevCompletion &P, const CmpSpmmArgs<S> &a, int *nb) {
    const int gs = gs_of<S>(a.ld);
    const int64_t n = P.n1 + P.n2;
    *nb = grid(n, kBlock / gs);
    if (gs == 4) hipLaunchKernelGGL((k_cmp_spmm<S, 4, GRAD, TM>), dim3(*nb), dim3(kBlock), 0, s, P, a);
    else if (gs == 8) hipLaunchKernelGGL((k_cmp_spmm<S, 8, GRAD, TM>), dim3(*nb), dim3(kBlock), 0, s, P, a);
    else hipLaunchKernelGGL((k_cmp_spmm<S, 16, GRAD, TM>), dim3(*nb), dim3(kBlock), 0, s, P, a);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

// The gradient build keeps the loops to kMaxMem for every T: the T <= 2 build
// (more waves per SIMD, more random row fetches in flight) measured 850 us
// against 749 us per launch at m = 1e7, rank 16, float64.
template <typename S, bool GRAD>
int cmp_spmm_t(hipStream_t s, const DevCompletion &P, const CmpSpmmArgs<S> &a, int *nb) {
    if (!GRAD) return cmp_spmm_tm<S, false, 0>(s, P, a, nb);
    return cmp_spmm_tm<S, GRAD, kMaxMem>(s, P, a, nb);
}

template <typename S, int MODE>
int cmp_sddmm_t(hipStream_t s, const DevCompletion &P, const SddArgs<S> &a, int *nb) {
    const int gs = gs_of<S>(a.ld);
    *nb = grid(P.n1, kBlock / gs);
    if (gs == 4) hipLaunchKernelGGL((k_cmp_sddmm<S, 4, MODE>), dim3(*nb), dim3(kBlock), 0, s, P, a);
    else if (gs == 8) hipLaunchKernelGGL((k_cmp_sddmm<S, 8, MODE>), dim3(*nb), dim3(kBlock), 0, s, P, a);
    else hipLaunchKernelGGL((k_cmp_sddmm<S, 16, MODE>), dim3(*nb), dim3(kBlock), 0, s, P, a);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

}  // namespace

int spmm_completion(hipStream_t s, const DevCompletion &P, int prec, const void *V, int64_t ld, const double *ytil,
                    void *Y) {
    int nb = 0;
    if (prec == LRSDP_F64) {
        CmpSpmmArgs<double> a{(const double *)V, (double *)Y, ytil, ld, nullptr, -1, {}, nullptr, 1.0};
        return cmp_spmm_t<double, false>(s, P, a, &nb);
    }
    CmpSpmmArgs<float> a{(const float *)V, (float *)Y, ytil, ld, nullptr, -1, {}, nullptr, 1.0};
    return cmp_spmm_t<float, false>(s, P, a, &nb);
}

int cmp_grad(hipStream_t s, const DevCompletion &P, int prec, const SolverState *st, const void *R,
             const double *ytil, void *const *gring, void *const *dring, int T, int64_t ld, double *partials,
             int force_slot, int *nb, double cs) {
    if (prec == LRSDP_F64) {
        CmpSpmmArgs<double> a{(const double *)R, nullptr, ytil, ld, st, force_slot, {}, partials, cs};
        for (int g = 0; g <= T; ++g) a.rings.g[g] = (double *)gring[g];
        for (int d = 0; d < T; ++d) a.rings.d[d] = (double *)dring[d];
        return cmp_spmm_t<double, true>(s, P, a, nb);
    }
    CmpSpmmArgs<float> a{(const float *)R, nullptr, ytil, ld, st, force_slot, {}, partials, cs};
    for (int g = 0; g <= T; ++g) a.rings.g[g] = (float *)gring[g];
    for (int d = 0; d < T; ++d) a.rings.d[d] = (float *)dring[d];
    return cmp_spmm_t<float, true>(s, P, a, nb);
}

// mode 0: out = A(U V^T); mode 1: line-search terms of direction V at U with
// ytil; mode 2: constraint values + multiplier step.
int cmp_sddmm(hipStream_t s, const DevCompletion &P, int prec, int mode, const void *U, const void *V, int64_t ld,
              double *out, double *q1, double *q2, const double *ytil, double *y, double sigma, double *partials,
              const SolverState *st, int *nb) {
    if (prec == LRSDP_F64) {
        SddArgs<double> a{(const double *)U, (const double *)V, ld, out, q1, q2, ytil, y, sigma, partials, st};
        if (mode == kSddA) return cmp_sddmm_t<double, kSddA>(s, P, a, nb);
        if (mode == kSddLS) return cmp_sddmm_t<double, kSddLS>(s, P, a, nb);
        return cmp_sddmm_t<double, kSddRefresh>(s, P, a, nb);
    }
    SddArgs<float> a{(const float *)U, (const float *)V, ld, out, q1, q2, ytil, y, sigma, partials, st};
    if (mode == kSddA) return cmp_sddmm_t<float, kSddA>(s, P, a, nb);
    if (mode == kSddLS) return cmp_sddmm_t<float, kSddLS>(s, P, a, nb);
    return cmp_sddmm_t<float, kSddRefresh>(s, P, a, nb);
}

int cmp_samples(hipStream_t s, const DevCompletion &P, const SolverState *st, double *acon, const double *q1,
                const double *q2, const double *y, double *ytil) {
    hipLaunchKernelGGL(k_cmp_samples, dim3(grid(P.m, kBlock)), dim3(kBlock), 0, s, P, st, acon, q1, q2, y, ytil);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int cmp_ytil(hipStream_t s, const DevCompletion &P, const SolverState *st, double sigma, const double *acon,
             const double *y, double *ytil) {
    hipLaunchKernelGGL(k_cmp_ytil, dim3(grid(P.m, kBlock)), dim3(kBlock), 0, s, P, st, sigma, acon, y, ytil);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int axpy_state(hipStream_t s, int prec, const SolverState *st, void *R, const void *D, int64_t n, int64_t ld) {
    const int64_t nch = n * ld * (prec == LRSDP_F64 ? 8 : 4) / 16;
    if (prec == LRSDP_F64)
        hipLaunchKernelGGL(k_axpy_state<double>, dim3(grid(nch, kBlock)), dim3(kBlock), 0, s, st, (double *)R,
                           (const double *)D, nch);
    else
        hipLaunchKernelGGL(k_axpy_state<float>, dim3(grid(nch, kBlock)), dim3(kBlock), 0, s, st, (float *)R,
                           (const float *)D, nch);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

}  // namespace lrsdp
