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
//      kEpiSplit    splitting half-step (Section 2.2, eq. 2.2 for A = diag): with
//                   b_i = -(C V)_i + (y_i + 2 sigma) V_i the block of the operator
//                   for row i is sigma (V_i V_i^T + I), so the exact solve is
//                   U_i = (b_i - (V_i . b_i) / (1 + ||V_i||^2) V_i) / sigma (written
//                   to Y); when R is given (the V-step, R = U) the multiplier step
//                   y_i <- y_i + sigma (1 - R_i . Y_i) follows
//  * Per-block sums go to a fixed-grid partials array (deterministic).
//  * BF16 input (float32 path only): the gathered operand is a bfloat16 copy
//    (row stride ldb = ld rounded up to 8); a lane then covers 8 columns, i.e.
//    two float32 chunks of the output, and accumulates in float32.
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

// 8 bfloat16 values (16 bytes) -> two float4
__device__ __forceinline__ void bf16x8_to_f32(const uint4 &u, float4 &lo, float4 &hi) {
    lo.x = __uint_as_float(u.x << 16);
    lo.y = __uint_as_float(u.x & 0xffff0000u);
    lo.z = __uint_as_float(u.y << 16);
    lo.w = __uint_as_float(u.y & 0xffff0000u);
    hi.x = __uint_as_float(u.z << 16);
    hi.y = __uint_as_float(u.z & 0xffff0000u);
    hi.z = __uint_as_float(u.w << 16);
    hi.w = __uint_as_float(u.w & 0xffff0000u);
}

// One gathered neighbour row chunk: NC = 1 -> one 16-byte chunk of S; NC = 2
// (BF16 input) -> 8 bfloat16 values widened to two float4.
template <typename S, int NC>
__device__ __forceinline__ void load_nbr(const void *V, int64_t j, int64_t ldv, int lane,
                                         typename Chunk<S>::V (&v)[NC]) {
    using CV = typename Chunk<S>::V;
    if constexpr (NC == 1) {
        v[0] = *reinterpret_cast<const CV *>((const S *)V + j * ldv + lane * Chunk<S>::N);
    } else {
        const uint4 u = *reinterpret_cast<const uint4 *>((const uint16_t *)V + j * ldv + lane * 8);
        bf16x8_to_f32(u, v[0], v[1]);
    }
}

// acc += sum_{e in [beg, end)} C_{row, col[e]} V_{col[e]}  (this lane's chunks).
// The GS lanes of the group fetch up to GS column indices of the row with one
// coalesced load and hand them round by lane shuffles, so a batch of up to
// eight neighbour-row loads per lane is issued back to back instead of each
// waiting behind its own index load.  The products are added in edge order,
// which rounds exactly as a sequential walk over the row does.
template <typename S, int GS, int W, int NC>
__device__ __forceinline__ void gather(const DevCsr &P, const void *__restrict__ V, int64_t ldv, int beg, int end,
                                       int lane, bool active, typename Chunk<S>::V (&acc)[NC]) {
    using CV = typename Chunk<S>::V;
    constexpr int KB = GS < 8 ? GS : 8;   // neighbour rows in flight per lane
    for (int e0 = beg; e0 < end; e0 += GS) {
        const int cnt = min(GS, end - e0);   // the same for every lane of the group
        int32_t mc = 0;
        S mw = (S)0;
        if (lane < cnt) {
            mc = P.col[e0 + lane];
            if constexpr (W == kWGeneral) mw = edge_weight<S, W>(P, e0 + lane, mc);
        }
#pragma unroll
        for (int k0 = 0; k0 < GS; k0 += KB) {
            if (k0 >= cnt) break;
            int32_t c[KB];
            S w[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                c[k] = __shfl(mc, k0 + k, GS);
                if constexpr (W == kWGeneral) w[k] = __shfl(mw, k0 + k, GS);
                else w[k] = edge_weight<S, W>(P, 0, c[k]);
            }
            if (active) {
                CV v[KB][NC];
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    if (k0 + k < cnt) load_nbr<S, NC>(V, c[k] & 0x7fffffff, ldv, lane, v[k]);
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    if (k0 + k < cnt) {
#pragma unroll
                        for (int q = 0; q < NC; ++q) vfma(acc[q], w[k], v[k][q]);
                    }
                }
            }
        }
    }
}

// Operands of the line-search epilogue that do not depend on the gather (the
// row's own D and R chunks, C_ii, ytil_i), loaded before it so that their
// latency overlaps the neighbour loads.  The other epilogues load in place.
template <typename S, int NC>
struct OwnRow {
    typename Chunk<S>::V d[NC], r[NC];
    double diag = 0.0, ytil = 0.0;
};

template <typename S, int EPI, int NC>
__device__ __forceinline__ void load_own(const DevCsr &P, const SpmmArgs &a, int row, int lane, bool active,
                                         OwnRow<S, NC> &o) {
    if constexpr (EPI == kEpiLS) {
        using CV = typename Chunk<S>::V;
        constexpr int NV = Chunk<S>::N;
        const S *Dn = (const S *)(NC == 1 ? a.V : a.Vown);   // own row of D in the storage type
        const CV zero = vzero(CV{});
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int ci = lane * NC + q;
            const bool act = active && ci * NV < a.ld;
            const int64_t rb = (int64_t)row * a.ld;
            o.d[q] = chunk_or_zero(Dn + rb, ci, act);
            o.r[q] = chunk_or_zero((const S *)a.R + rb, ci, act);
        }
        o.diag = P.diag[row];
        o.ytil = a.ytil[row];
    }
}

// Per-row epilogue.  Every lane of the group calls it (inactive chunks hold
// zeros); lane 0 of the group adds the row's terms into s[].  Lane `lane` owns
// output chunks lane*NC + q, q < NC.
template <typename S, int GS, int EPI, int NC>
__device__ __forceinline__ void epilogue(const DevCsr &P, const SpmmArgs &a, int row, int lane, bool active,
                                         const OwnRow<S, NC> &own, typename Chunk<S>::V (&acc)[NC],
                                         double (&s)[kLsSums]) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    // operator cs C: the gathered off-diagonal sum and the diagonal both take the
    // objective scale (cs = 1 leaves every value unchanged)
    const S cs = (S)a.cs;
#pragma unroll
    for (int q = 0; q < NC; ++q) vscale(acc[q], cs);
    const S dg = (S)(a.cs * (EPI == kEpiLS ? own.diag : P.diag[row]));
    const CV zero = vzero(CV{});
    const int64_t rb = (int64_t)row * a.ld;
    int64_t off[NC];
    bool act[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int ci = lane * NC + q;
        act[q] = active && ci * NV < a.ld;
        off[q] = rb + ci * NV;
    }
    if constexpr (EPI == kEpiPlain) {
        CV v[NC];
        if constexpr (NC == 1) {
            v[0] = chunk_or_zero((const S *)a.V + rb, lane, act[0]);
        } else {
            // own row from the bfloat16 input (lanes past the row hold zeros)
#pragma unroll
            for (int q = 0; q < NC; ++q) v[q] = zero;
            if (active) load_nbr<S, NC>(a.V, row, a.ldv, lane, v);
        }
        S shift = dg;
        if (a.ytil) shift = (S)(a.cs * P.diag[row] - a.ytil[row]);
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            vfma(acc[q], shift, v[q]);
            if (act[q]) *reinterpret_cast<CV *>((S *)a.Y + off[q]) = acc[q];
        }
    } else if constexpr (EPI == kEpiLS) {
        double p2 = 0.0, q1 = 0.0, q2 = 0.0, rr = 0.0, p1 = 0.0;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const CV d = own.d[q];
            const CV r = own.r[q];
            vfma(acc[q], dg, d);
            if (act[q]) *reinterpret_cast<CV *>((S *)a.Y + off[q]) = acc[q];
            p2 += vdot(acc[q], d);
            q1 += vdot(r, d);
            q2 += vdot(d, d);
            if (a.rn) rr += vdot(r, r);
            if (a.aux) {
                const CV cr = chunk_or_zero((const S *)a.aux + rb, lane * NC + q, act[q]);
                p1 += vdot(cr, d);
            }
        }
        p2 = group_sum<GS>(p2);
        q1 = 2.0 * group_sum<GS>(q1);
        q2 = group_sum<GS>(q2);
        if (a.rn) rr = group_sum<GS>(rr);
        if (a.aux) p1 = 2.0 * group_sum<GS>(p1);
        if (lane == 0) {
            const double yt = own.ytil;
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
    } else if constexpr (EPI == kEpiSplit) {  // NC = 1
        const CV v = chunk_or_zero((const S *)a.V + rb, lane, act[0]);
        vfma(acc[0], dg, v);                                   // (C V)_i
        const double coef = a.y[row] + 2.0 * a.sigma;
        D4 vv4 = widen(v), cv4 = widen(acc[0]), b4;
#pragma unroll
        for (int c = 0; c < 4; ++c) b4.v[c] = fma(coef, vv4.v[c], -cv4.v[c]);
        double vb = 0.0, vv = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            vb = fma(vv4.v[c], b4.v[c], vb);
            vv = fma(vv4.v[c], vv4.v[c], vv);
        }
        vb = group_sum<GS>(vb);
        vv = group_sum<GS>(vv);
        const double f = vb / (1.0 + vv), is = 1.0 / a.sigma;
        D4 u4;
#pragma unroll
        for (int c = 0; c < 4; ++c) u4.v[c] = (b4.v[c] - f * vv4.v[c]) * is;
        CV us;
        narrow(u4, us);
        if (act[0]) *reinterpret_cast<CV *>((S *)a.Y + off[0]) = us;
        if (a.R) {
            const CV r = chunk_or_zero((const S *)a.R + rb, lane, act[0]);
            const double ru = group_sum<GS>(vdot(r, us));
            if (lane == 0) a.y[row] += a.sigma * (1.0 - ru);
        }
    } else {  // kEpiRefresh: V = R (storage type, NC = 1)
        double obj = 0.0, rn = 0.0;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const CV r = chunk_or_zero((const S *)a.V + rb, lane * NC + q, act[q]);
            vfma(acc[q], dg, r);
            if (act[q] && a.Y) *reinterpret_cast<CV *>((S *)a.Y + off[q]) = acc[q];
            obj += vdot(r, acc[q]);
            rn += vdot(r, r);
        }
        obj = group_sum<GS>(obj);
        rn = group_sum<GS>(rn);
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

// lane owns gathered chunk `lane` (NC = 1: chunk of S; NC = 2: 8 bfloat16)
template <typename S, int NC>
__device__ __forceinline__ bool lane_active(const SpmmArgs &a, int lane) {
    return NC == 1 ? lane * Chunk<S>::N < a.ld : lane * 8 < a.ld;
}

template <typename S, int GS, int W, int EPI, int NC>
__global__ __launch_bounds__(kBlock) void k_spmm_light(DevCsr P, SpmmArgs a) {
    using CV = typename Chunk<S>::V;
    constexpr int GPB = kBlock / GS;
    if (a.st && a.st->done) return;
    const int lane = threadIdx.x % GS;
    const int grp = threadIdx.x / GS;
    const bool active = lane_active<S, NC>(a, lane);
    double s[kLsSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * GPB;
    int64_t it = (int64_t)blockIdx.x * GPB + grp;
    // work-list entries {row, begin, end} (no dependent row_ptr load); the next
    // row's entry is loaded before this row's gather, off the critical path
    int4 wl = it < P.n_light ? P.light[it] : make_int4(0, 0, 0, 0);
    for (; it < P.n_light; it += stride) {
        const int4 wn = it + stride < P.n_light ? P.light[it + stride] : make_int4(0, 0, 0, 0);
        const int row = wl.x, beg = wl.y, end = wl.z;
        CV acc[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] = vzero(CV{});
        OwnRow<S, NC> own;
        load_own<S, EPI, NC>(P, a, row, lane, active, own);
        gather<S, GS, W, NC>(P, a.V, a.ldv, beg, end, lane, active, acc);
        epilogue<S, GS, EPI, NC>(P, a, row, lane, active, own, acc, s);
        wl = wn;
    }
    if constexpr (EPI == kEpiLS || EPI == kEpiRefresh)
        block_sums_store<kLsSums>(s, a.partials + (size_t)blockIdx.x * kMaxSums);
}

// Segments of heavy rows: partial sums to seg_buf (16 chunks = 256 bytes per segment).
template <typename S, int GS, int W, int NC>
__global__ __launch_bounds__(kBlock) void k_spmm_segments(DevCsr P, SpmmArgs a) {
    using CV = typename Chunk<S>::V;
    constexpr int GPB = kBlock / GS;
    if (a.st && a.st->done) return;
    const int lane = threadIdx.x % GS;
    const int grp = threadIdx.x / GS;
    const bool active = lane_active<S, NC>(a, lane);
    CV *buf = (CV *)P.seg_buf;
    for (int64_t it = (int64_t)blockIdx.x * GPB + grp; it < P.n_seg; it += (int64_t)gridDim.x * GPB) {
        const int4 sg = P.seg[it];
        CV acc[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] = vzero(CV{});
        gather<S, GS, W, NC>(P, a.V, a.ldv, sg.y, sg.z, lane, active, acc);
        if (active) {
#pragma unroll
            for (int q = 0; q < NC; ++q) buf[(int64_t)sg.w * 16 + lane * NC + q] = acc[q];
        }
    }
}

// One workgroup per heavy row: add its segment sums in a fixed order, then run
// the epilogue with lane group 0.
template <typename S, int GS, int EPI, int NC>
__global__ __launch_bounds__(kBlock) void k_spmm_fixup(DevCsr P, SpmmArgs a, int part_base) {
    using CV = typename Chunk<S>::V;
    constexpr int GPB = kBlock / GS;
    if (a.st && a.st->done) return;
    const int lane = threadIdx.x % GS;
    const int grp = threadIdx.x / GS;
    const bool active = lane_active<S, NC>(a, lane);
    const CV *buf = (const CV *)P.seg_buf;
    __shared__ CV sh[GPB][GS * NC];
    double s[kLsSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t h = blockIdx.x; h < P.n_heavy; h += gridDim.x) {
        const int row = P.heavy[h];
        const int s0 = P.heavy_seg[h], s1 = P.heavy_seg[h + 1];
        CV acc[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] = vzero(CV{});
        for (int g = s0 + grp; g < s1; g += GPB) {
            if (active) {
#pragma unroll
                for (int q = 0; q < NC; ++q) vfma(acc[q], (S)1, buf[(int64_t)g * 16 + lane * NC + q]);
            }
        }
#pragma unroll
        for (int q = 0; q < NC; ++q) sh[grp][lane * NC + q] = acc[q];
        __syncthreads();
        if (grp == 0) {
            CV t[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                t[q] = vzero(CV{});
#pragma unroll 4
                for (int g = 0; g < GPB; ++g) vfma(t[q], (S)1, sh[g][lane * NC + q]);
            }
            OwnRow<S, NC> own;
            load_own<S, EPI, NC>(P, a, row, lane, active, own);
            epilogue<S, GS, EPI, NC>(P, a, row, lane, active, own, t, s);
        }
        __syncthreads();
    }
    if constexpr (EPI == kEpiLS || EPI == kEpiRefresh)
        block_sums_store<kLsSums>(s, a.partials + (size_t)(part_base + blockIdx.x) * kMaxSums);
}

template <typename S, int GS, int W, int EPI, int NC>
int launch(hipStream_t st, const DevCsr &P, const SpmmArgs &a, int *nparts) {
    constexpr int GPB = kBlock / GS;
    int nb1 = 0, nb3 = 0;
    if (P.n_light > 0) {
        int64_t need = (P.n_light + GPB - 1) / GPB;
        nb1 = (int)std::min<int64_t>(need, kMaxBlocks);
        hipLaunchKernelGGL((k_spmm_light<S, GS, W, EPI, NC>), dim3(nb1), dim3(kBlock), 0, st, P, a);
        LRSDP_CHECK_LAUNCH();
    }
    if (P.n_heavy > 0) {
        int64_t need = (P.n_seg + GPB - 1) / GPB;
        int nb2 = (int)std::min<int64_t>(need, 4 * kMaxBlocks);
        hipLaunchKernelGGL((k_spmm_segments<S, GS, W, NC>), dim3(nb2), dim3(kBlock), 0, st, P, a);
        LRSDP_CHECK_LAUNCH();
        nb3 = (int)std::min<int64_t>(P.n_heavy, kMaxBlocks);
        hipLaunchKernelGGL((k_spmm_fixup<S, GS, EPI, NC>), dim3(nb3), dim3(kBlock), 0, st, P, a, nb1);
        LRSDP_CHECK_LAUNCH();
    }
    *nparts = nb1 + nb3;
    return LRSDP_OK;
}

template <typename S, int GS, int EPI, int NC>
int launch_w(hipStream_t st, const DevCsr &P, const SpmmArgs &a, int *nparts) {
    switch (P.wmode) {
        case kWUnit: return launch<S, GS, kWUnit, EPI, NC>(st, P, a, nparts);
        case kWSign: return launch<S, GS, kWSign, EPI, NC>(st, P, a, nparts);
        default: return launch<S, GS, kWGeneral, EPI, NC>(st, P, a, nparts);
    }
}

template <typename S, int EPI, int NC>
int launch_gs(hipStream_t st, const DevCsr &P, const SpmmArgs &a, int *nparts) {
    // gathered 16-byte chunks per row
    const int chunks = NC == 1 ? (int)(a.ld * (int64_t)sizeof(S) / 16) : (int)((a.ld + 7) / 8);
    if (chunks <= 4) return launch_w<S, 4, EPI, NC>(st, P, a, nparts);
    if (chunks <= 8) return launch_w<S, 8, EPI, NC>(st, P, a, nparts);
    return launch_w<S, 16, EPI, NC>(st, P, a, nparts);
}

template <typename S, int NC>
int launch_epi(hipStream_t st, const DevCsr &P, const SpmmArgs &a, int *nparts) {
    switch (a.epi) {
        case kEpiPlain: return launch_gs<S, kEpiPlain, NC>(st, P, a, nparts);
        case kEpiLS: return launch_gs<S, kEpiLS, NC>(st, P, a, nparts);
        case kEpiSplit: return launch_gs<S, kEpiSplit, 1>(st, P, a, nparts);
        default: return launch_gs<S, kEpiRefresh, 1>(st, P, a, nparts);
    }
}

}  // namespace

int spmm_maxcut(hipStream_t st, const DevCsr &P, int prec, const SpmmArgs &a_in, int *nparts) {
    const int64_t esz = prec == LRSDP_F64 ? 8 : 4;
    SpmmArgs a = a_in;
    if (a.ld <= 0 || (a.ld * esz) % 16 != 0 || a.ld * esz > 256)
        return set_error(LRSDP_EINVAL, "ld = %lld: row bytes must be a positive multiple of 16, at most 256",
                         (long long)a.ld);
    const bool bf = prec == LRSDP_F32_BF16IN && a.epi != kEpiRefresh && a.epi != kEpiSplit;
    if (bf && a.epi == kEpiLS && !a.Vown)
        return set_error(LRSDP_EINVAL, "bfloat16 line-search SpMM needs the float32 operand");
    a.ldv = bf ? bf16_ld(a.ld) : a.ld;
    if (prec == LRSDP_F64) return launch_epi<double, 1>(st, P, a, nparts);
    if (bf) return launch_epi<float, 2>(st, P, a, nparts);
    return launch_epi<float, 1>(st, P, a, nparts);
}

}  // namespace lrsdp
