// MaxCut SpMM  Y = C V  with C = -L/4 (paper eq. At for A = diag), fused with
// the per-row epilogues of the ALM iteration.
//
// Design (gfx950, bandwidth bound, no MFMA):
//  * A lane group of GS lanes (GS = power of two >= 16-byte chunks per row)
//    owns one output row; lane c accumulates chunk c of the row, so every
//    neighbour row V_j is fetched as GS contiguous 16-byte loads (coalesced).
//  * Rows with at most kSegLen nonzeros ("light") are walked in an order
//    sorted by length inside windows of consecutive rows, so the groups of a
//    wavefront finish together.  Longer rows are cut into kSegLen segments
//    processed like light rows; their partial sums go to a per-segment buffer
//    and a fixup kernel (one workgroup per heavy row) adds them in a fixed
//    order: no floating-point atomics, bitwise reproducible.
//  * Off-diagonal values are implicit for unit and +-1 weights (the sign sits
//    in bit 31 of the column index); the diagonal C_ii is a separate vector
//    applied in the epilogue together with the shift by -ytil_i.
//  * Epilogues:
//      kEpiPlain    Y_i = (C V)_i - ytil_i V_i
//      kEpiLS       CD_i = (C D)_i, plus the row terms of the exact line search
//                   (appendix A.2) for MaxCut: p2_i = CD_i.D_i, q1_i = 2 R_i.D_i,
//                   q2_i = ||D_i||^2, summed as p2, ytil.q2, ytil.q1, q2.q2,
//                   q1.q2, q1.q1 and (optionally) p1 = 2 sum CR_i.D_i; optionally
//                   stores q1_i, q2_i and ||R_i||^2 per row
//      kEpiRefresh  CR_i = (C R)_i, obj_i = R_i.CR_i, res_i = ||R_i||^2 - 1,
//                   optional multiplier step y_i <- y_i - sigma res_i; sums
//                   obj, b^T y, ||res||^2
//  * Per-block sums go to a fixed-grid partials array (deterministic).
#include "device.h"
#include "kernels.h"

namespace lrsdp {
namespace {

template <typename S, int W>
__device__ __forceinline__ S edge_weight(const DevCsr &P, int e, int32_t c) {
    if constexpr (W == kWUnit) {
        return (S)0.25;
    } else if constexpr (W == kWSign) {
        return c < 0 ? (S)-0.25 : (S)0.25;
    } else {
        return (S)P.val[e];
    }
}

// acc += sum_{e in [beg, end)} C_{row, col[e]} V_{col[e]}  (this lane's chunk)
template <typename S, int W>
__device__ __forceinline__ void gather(const DevCsr &P, const S *__restrict__ V, int64_t ld,
                                       int beg, int end, int lane, bool active,
                                       typename Chunk<S>::V &acc) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    const int32_t *__restrict__ col = P.col;
    int e = beg;
    for (; e + 4 <= end; e += 4) {
        int32_t c0 = col[e], c1 = col[e + 1], c2 = col[e + 2], c3 = col[e + 3];
        S w0 = edge_weight<S, W>(P, e, c0), w1 = edge_weight<S, W>(P, e + 1, c1);
        S w2 = edge_weight<S, W>(P, e + 2, c2), w3 = edge_weight<S, W>(P, e + 3, c3);
        if (active) {
            const CV v0 = *reinterpret_cast<const CV *>(V + (int64_t)(c0 & 0x7fffffff) * ld + lane * NV);
            const CV v1 = *reinterpret_cast<const CV *>(V + (int64_t)(c1 & 0x7fffffff) * ld + lane * NV);
            const CV v2 = *reinterpret_cast<const CV *>(V + (int64_t)(c2 & 0x7fffffff) * ld + lane * NV);
            const CV v3 = *reinterpret_cast<const CV *>(V + (int64_t)(c3 & 0x7fffffff) * ld + lane * NV);
            vfma(acc, w0, v0);
            vfma(acc, w1, v1);
            vfma(acc, w2, v2);
            vfma(acc, w3, v3);
        }
    }
    for (; e < end; ++e) {
        int32_t c0 = col[e];
        S w0 = edge_weight<S, W>(P, e, c0);
        if (active) {
            const CV v0 = *reinterpret_cast<const CV *>(V + (int64_t)(c0 & 0x7fffffff) * ld + lane * NV);
            vfma(acc, w0, v0);
        }
    }
}

// Per-row epilogue.  Every lane of the group calls it (inactive lanes hold
// zero chunks); lane 0 of the group adds the row's terms into s[].
template <typename S, int GS, int EPI>
__device__ __forceinline__ void epilogue(const DevCsr &P, const SpmmArgs &a, int row, int lane,
                                         bool active, typename Chunk<S>::V acc, double (&s)[kLsSums]) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    const int64_t off = (int64_t)row * a.ld + lane * NV;
    const S dg = (S)P.diag[row];
    CV zero = vzero(CV{});
    if constexpr (EPI == kEpiPlain) {
        const CV v = active ? *reinterpret_cast<const CV *>((const S *)a.V + off) : zero;
        S shift = dg;
        if (a.ytil) shift = (S)((double)P.diag[row] - a.ytil[row]);
        vfma(acc, shift, v);
        if (active) *reinterpret_cast<CV *>((S *)a.Y + off) = acc;
    } else if constexpr (EPI == kEpiLS) {
        const CV d = active ? *reinterpret_cast<const CV *>((const S *)a.V + off) : zero;
        const CV r = active ? *reinterpret_cast<const CV *>((const S *)a.R + off) : zero;
        vfma(acc, dg, d);
        if (active) *reinterpret_cast<CV *>((S *)a.Y + off) = acc;
        double p2 = group_sum<GS>(vdot(acc, d));
        double q1 = 2.0 * group_sum<GS>(vdot(r, d));
        double q2 = group_sum<GS>(vdot(d, d));
        double rr = a.rn ? group_sum<GS>(vdot(r, r)) : 0.0;
        double p1 = 0.0;
        if (a.aux) {
            const CV cr = active ? *reinterpret_cast<const CV *>((const S *)a.aux + off) : zero;
            p1 = 2.0 * group_sum<GS>(vdot(cr, d));
        }
        if (lane == 0) {
            const double yt = a.ytil[row];
            s[0] += p2;
            s[1] += yt * q2;
            s[2] += yt * q1;
            s[3] += q2 * q2;
            s[4] += q1 * q2;
            s[5] += q1 * q1;
            s[6] += p1;
            if (a.q1) a.q1[row] = q1;
            if (a.q2) a.q2[row] = q2;
            if (a.rn) a.rn[row] = rr;
        }
    } else {  // kEpiRefresh: V = R
        const CV r = active ? *reinterpret_cast<const CV *>((const S *)a.V + off) : zero;
        vfma(acc, dg, r);
        if (active && a.Y) *reinterpret_cast<CV *>((S *)a.Y + off) = acc;
        double obj = group_sum<GS>(vdot(r, acc));
        double rn = group_sum<GS>(vdot(r, r));
        if (lane == 0) {
            double res = rn - 1.0;
            double yi = a.y[row];
            if (a.sigma > 0.0) {
                yi = yi - a.sigma * res;
                a.y[row] = yi;
            }
            if (a.rn) a.rn[row] = rn;
            s[0] += obj;
            s[1] += yi;           // b^T y with b = 1
            s[2] += res * res;
        }
    }
}

template <typename S, int GS, int W, int EPI>
__global__ __launch_bounds__(kBlock) void k_spmm_light(DevCsr P, SpmmArgs a) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    if (a.st && a.st->done) return;
    const int lane = threadIdx.x % GS;
    const int grp = threadIdx.x / GS;
    const bool active = lane * NV < a.ld;
    double s[kLsSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    const S *V = (const S *)a.V;
    for (int64_t it = (int64_t)blockIdx.x * GPB + grp; it < P.n_light; it += (int64_t)gridDim.x * GPB) {
        const int row = P.light[it];
        const int beg = P.row_ptr[row], end = P.row_ptr[row + 1];
        CV acc = vzero(CV{});
        gather<S, W>(P, V, a.ld, beg, end, lane, active, acc);
        epilogue<S, GS, EPI>(P, a, row, lane, active, acc, s);
    }
    if constexpr (EPI != kEpiPlain) block_sums_store<kLsSums>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

// Segments of heavy rows: partial sums to seg_buf (256 bytes per segment).
template <typename S, int GS, int W>
__global__ __launch_bounds__(kBlock) void k_spmm_segments(DevCsr P, SpmmArgs a) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    if (a.st && a.st->done) return;
    const int lane = threadIdx.x % GS;
    const int grp = threadIdx.x / GS;
    const bool active = lane * NV < a.ld;
    const S *V = (const S *)a.V;
    CV *buf = (CV *)P.seg_buf;
    for (int64_t it = (int64_t)blockIdx.x * GPB + grp; it < P.n_seg; it += (int64_t)gridDim.x * GPB) {
        const int4 sg = P.seg[it];
        CV acc = vzero(CV{});
        gather<S, W>(P, V, a.ld, sg.y, sg.z, lane, active, acc);
        if (active) buf[(int64_t)sg.w * 16 + lane] = acc;
    }
}

// One workgroup per heavy row: add its segment sums in a fixed order, then run
// the epilogue with lane group 0.
template <typename S, int GS, int EPI>
__global__ __launch_bounds__(kBlock) void k_spmm_fixup(DevCsr P, SpmmArgs a, int part_base) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    if (a.st && a.st->done) return;
    const int lane = threadIdx.x % GS;
    const int grp = threadIdx.x / GS;
    const bool active = lane * NV < a.ld;
    const CV *buf = (const CV *)P.seg_buf;
    __shared__ CV sh[GPB][GS];
    double s[kLsSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t h = blockIdx.x; h < P.n_heavy; h += gridDim.x) {
        const int row = P.heavy[h];
        const int s0 = P.heavy_seg[h], s1 = P.heavy_seg[h + 1];
        CV acc = vzero(CV{});
        for (int q = s0 + grp; q < s1; q += GPB) {
            if (active) {
                const CV v = buf[(int64_t)q * 16 + lane];
                vfma(acc, (S)1, v);
            }
        }
        sh[grp][lane] = acc;
        __syncthreads();
        if (grp == 0) {
            CV t = vzero(CV{});
#pragma unroll 4
            for (int g = 0; g < GPB; ++g) vfma(t, (S)1, sh[g][lane]);
            epilogue<S, GS, EPI>(P, a, row, lane, active, t, s);
        }
        __syncthreads();
    }
    if constexpr (EPI != kEpiPlain)
        block_sums_store<kLsSums>(s, a.partials + (size_t)(part_base + blockIdx.x) * kMaxSums);
}

template <typename S, int GS, int W, int EPI>
int launch(hipStream_t st, const DevCsr &P, const SpmmArgs &a, int *nparts) {
    constexpr int GPB = kBlock / GS;
    int nb1 = 0, nb3 = 0;
    if (P.n_light > 0) {
        int64_t need = (P.n_light + GPB - 1) / GPB;
        nb1 = (int)std::min<int64_t>(need, kMaxBlocks);
        hipLaunchKernelGGL((k_spmm_light<S, GS, W, EPI>), dim3(nb1), dim3(kBlock), 0, st, P, a);
        LRSDP_CHECK_LAUNCH();
    }
    if (P.n_heavy > 0) {
        int64_t need = (P.n_seg + GPB - 1) / GPB;
        int nb2 = (int)std::min<int64_t>(need, 4 * kMaxBlocks);
        hipLaunchKernelGGL((k_spmm_segments<S, GS, W>), dim3(nb2), dim3(kBlock), 0, st, P, a);
        LRSDP_CHECK_LAUNCH();
        nb3 = (int)std::min<int64_t>(P.n_heavy, kMaxBlocks);
        hipLaunchKernelGGL((k_spmm_fixup<S, GS, EPI>), dim3(nb3), dim3(kBlock), 0, st, P, a, nb1);
        LRSDP_CHECK_LAUNCH();
    }
    *nparts = nb1 + nb3;
    return LRSDP_OK;
}

template <typename S, int GS, int EPI>
int launch_w(hipStream_t st, const DevCsr &P, const SpmmArgs &a, int *nparts) {
    switch (P.wmode) {
        case kWUnit: return launch<S, GS, kWUnit, EPI>(st, P, a, nparts);
        case kWSign: return launch<S, GS, kWSign, EPI>(st, P, a, nparts);
        default: return launch<S, GS, kWGeneral, EPI>(st, P, a, nparts);
    }
}

template <typename S, int EPI>
int launch_gs(hipStream_t st, const DevCsr &P, const SpmmArgs &a, int *nparts) {
    const int chunks = (int)(a.ld * (int64_t)sizeof(S) / 16);
    if (chunks <= 4) return launch_w<S, 4, EPI>(st, P, a, nparts);
    if (chunks <= 8) return launch_w<S, 8, EPI>(st, P, a, nparts);
    return launch_w<S, 16, EPI>(st, P, a, nparts);
}

template <typename S>
int launch_epi(hipStream_t st, const DevCsr &P, const SpmmArgs &a, int *nparts) {
    switch (a.epi) {
        case kEpiPlain: return launch_gs<S, kEpiPlain>(st, P, a, nparts);
        case kEpiLS: return launch_gs<S, kEpiLS>(st, P, a, nparts);
        default: return launch_gs<S, kEpiRefresh>(st, P, a, nparts);
    }
}

}  // namespace

int spmm_maxcut(hipStream_t st, const DevCsr &P, int prec, const SpmmArgs &a, int *nparts) {
    const int64_t esz = prec == LRSDP_F64 ? 8 : 4;
    if (a.ld <= 0 || (a.ld * esz) % 16 != 0 || a.ld * esz > 256)
        return set_error(LRSDP_EINVAL, "ld = %lld: row bytes must be a positive multiple of 16, at most 256",
                         (long long)a.ld);
    if (prec == LRSDP_F64) return launch_epi<double>(st, P, a, nparts);
    return launch_epi<float>(st, P, a, nparts);
}

}  // namespace lrsdp
