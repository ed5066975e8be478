// Learned warm start for MaxCut: per-node features, a 16-64-64-2 tanh MLP
// (forward, gradient, Adam), and the multiplier / penalty prediction.
//
// Features of node i (d degree, s = sum_j w_ij, a = sum_j |w_ij|, l = log(1+d),
// b = s / max(a, 1), dbar = 2|E|/n; w_ij = 4 C_ij):
//   0 l_i   1 b_i   2 log(1+a_i)   3 mean_j l_j   4 std_j l_j   5 mean_j w_ij b_j
//   6 mean_j 1/(1+d_j)   7 log(1 + d_i/dbar)   8 1/(1+d_i)   9 a_i/max(d_i,1)
//  10 mean_j w_ij   11 log(n)/20   12 log(1+dbar)   13 max_j l_j - l_i
//  14 mean_j d_j/(d_i+d_j)   15 1
// Output 0 predicts t_i = -4 y_i / a_i (so y0_i = -t_i a_i / 4); output 1 the
// log of the initial penalty relative to the default.
//
// Parameters (float32, flat): W1[64][16] b1[64] W2[64][64] b2[64] W3[2][64] b3[2].
// The gradient kernel processes tiles of 128 nodes per workgroup: the tile's
// activations live in LDS, each thread owns a fixed set of weight entries and
// accumulates their gradient over the tiles it visits; per-workgroup partial
// gradients are then summed in a fixed order (deterministic, no atomics).
#include "device.h"
#include "kernels.h"

namespace lrsdp {

constexpr int kNF = 16, kH = 64, kNO = 2;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kNF, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kNO * kH, kNParam = kOffB3 + kNO;
constexpr int kTile = 128;           // nodes per tile of the gradient kernel
constexpr int kGradBlocks = 256;     // workgroups of the gradient kernel

namespace {

template <int W>
__device__ __forceinline__ float edge_w(const DevCsr &P, int e, int32_t c) {
    if constexpr (W == kWUnit) return 1.0f;
    else if constexpr (W == kWSign) return c < 0 ? -1.0f : 1.0f;
    else return (float)(4.0 * P.val[e]);
}

// The 16 features of one node from its stats and neighbour sums (sl = sum of
// l_j - l_i, sl2 = its squares, swb = sum w_ij b_j, sinv = sum 1/(1+d_j),
// sw = sum w_ij, sdd = sum d_j/(d_i+d_j), lmax = max l_j).
__device__ __forceinline__ void write_features(const float4 si, int deg, double sl, double sl2, double swb,
                                               double sinv, double sw, double sdd, float lmax, float dbar,
                                               float logn20, float *out) {
    const float d = si.x, a = si.z, l = si.w;
    float f[kNF];
    f[0] = l;
    f[1] = si.y / fmaxf(a, 1.f);
    f[2] = log1pf(a);
    f[7] = dbar > 0.f ? log1pf(d / dbar) : 0.f;
    f[8] = 1.f / (1.f + d);
    f[9] = a / fmaxf(d, 1.f);
    f[11] = logn20;
    f[12] = log1pf(dbar);
    f[15] = 1.f;
    if (deg > 0) {
        const double inv = 1.0 / (double)deg;
        const double ml = sl * inv;  // mean of l_j - l_i
        f[3] = (float)((double)l + ml);
        f[4] = (float)sqrt(fmax(sl2 * inv - ml * ml, 0.0));
        f[5] = (float)(swb * inv);
        f[6] = (float)(sinv * inv);
        f[10] = (float)(sw * inv);
        f[13] = lmax - l;
        f[14] = (float)(sdd * inv);
    } else {
        f[3] = f[4] = f[5] = f[6] = f[10] = f[13] = f[14] = 0.f;
    }
#pragma unroll
    for (int q = 0; q < kNF; q += 4)
        *reinterpret_cast<float4 *>(out + q) = make_float4(f[q], f[q + 1], f[q + 2], f[q + 3]);
}

// Caller label of internal node i: per-node outputs and the statistics table
// are in the caller's order for a problem relabelled by degree.
__device__ __forceinline__ int64_t lab(const DevCsr &P, int64_t i) { return P.perm ? (int64_t)P.perm[i] : i; }

// pass 1: per-node (d, s, a, l)
template <int W>
__global__ __launch_bounds__(kBlock) void k_node_stats(DevCsr P, float4 *stats) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * kBlock) {
        const int b = P.row_ptr[i], e = P.row_ptr[i + 1];
        if (e - b > kSegLen) continue;   // hub rows: k_node_stats_heavy
        double s = 0.0, a = 0.0;
        for (int k = b; k < e; ++k) {
            const double w = edge_w<W>(P, k, P.col[k]);
            s += w;
            a += fabs(w);
        }
        const float d = (float)(e - b);
        stats[lab(P, i)] = make_float4(d, (float)s, (float)a, (float)log1p((double)(e - b)));
    }
}

// pass 2: neighbour statistics -> 16 features per node
template <int W>
__global__ __launch_bounds__(kBlock) void k_features(DevCsr P, const float4 *stats, float dbar, float logn20,
                                                     float *F) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * kBlock) {
        const int b = P.row_ptr[i], e = P.row_ptr[i + 1];
        if (e - b > kSegLen) continue;   // hub rows: k_features_heavy
        const float4 si = stats[lab(P, i)];
        const float d = si.x, l = si.w;
        // Neighbour sums in double: the spread feature (std of l over the
        // neighbours) cancels badly in float for hubs whose neighbours have
        // near-equal degrees.  This pass runs once per graph.
        double sl = 0.0, sl2 = 0.0, swb = 0.0, sinv = 0.0, sw = 0.0, sdd = 0.0;
        float lmax = -1e30f;
        for (int k = b; k < e; ++k) {
            const int32_t c = P.col[k];
            const double w = edge_w<W>(P, k, c);
            const float4 sj = stats[lab(P, c & 0x7fffffff)];
            const double lj = (double)sj.w - (double)l;
            sl += lj;
            sl2 += lj * lj;
            swb += w * (double)(sj.y / fmaxf(sj.z, 1.f));
            sinv += 1.0 / (1.0 + (double)sj.x);
            sw += w;
            lmax = fmaxf(lmax, sj.w);
            sdd += (double)sj.x / ((double)d + (double)sj.x);
        }
        write_features(si, e - b, sl, sl2, swb, sinv, sw, sdd, lmax, dbar, logn20, F + lab(P, i) * kNF);
    }
}

// One workgroup per hub row (more than kSegLen neighbours): the threads stride
// over the neighbours, the sums go through a fixed wavefront / LDS tree.
template <int W>
__global__ __launch_bounds__(kBlock) void k_node_stats_heavy(DevCsr P, float4 *stats) {
    __shared__ double sh[kBlock / 64][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t h = blockIdx.x; h < P.n_heavy; h += gridDim.x) {
        const int64_t i = P.heavy[h];
        const int b = P.row_ptr[i], e = P.row_ptr[i + 1];
        double s = 0.0, a = 0.0;
        for (int k = b + threadIdx.x; k < e; k += kBlock) {
            const double w = edge_w<W>(P, k, P.col[k]);
            s += w;
            a += fabs(w);
        }
        s = wave_sum(s);
        a = wave_sum(a);
        __syncthreads();
        if (lane == 0) {
            sh[wave][0] = s;
            sh[wave][1] = a;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ts = 0.0, ta = 0.0;
#pragma unroll
            for (int q = 0; q < kBlock / 64; ++q) {
                ts += sh[q][0];
                ta += sh[q][1];
            }
            stats[lab(P, i)] = make_float4((float)(e - b), (float)ts, (float)ta, (float)log1p((double)(e - b)));
        }
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_features_heavy(DevCsr P, const float4 *stats, float dbar, float logn20,
                                                           float *F) {
    __shared__ double sh[kBlock / 64][6];
    __shared__ float shm[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t h = blockIdx.x; h < P.n_heavy; h += gridDim.x) {
        const int64_t i = P.heavy[h];
        const int b = P.row_ptr[i], e = P.row_ptr[i + 1];
        const float4 si = stats[lab(P, i)];
        const float d = si.x, l = si.w;
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // sl, sl2, swb, sinv, sw, sdd
        float lmax = -1e30f;
        for (int k = b + threadIdx.x; k < e; k += kBlock) {
            const int32_t c = P.col[k];
            const double w = edge_w<W>(P, k, c);
            const float4 sj = stats[lab(P, c & 0x7fffffff)];
            const double lj = (double)sj.w - (double)l;
            v[0] += lj;
            v[1] += lj * lj;
            v[2] += w * (double)(sj.y / fmaxf(sj.z, 1.f));
            v[3] += 1.0 / (1.0 + (double)sj.x);
            v[4] += w;
            lmax = fmaxf(lmax, sj.w);
            v[5] += (double)sj.x / ((double)d + (double)sj.x);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) v[q] = wave_sum(v[q]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lmax = fmaxf(lmax, __shfl_xor(lmax, o, 64));
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 6; ++q) sh[wave][q] = v[q];
            shm[wave] = lmax;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double t[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            float tm = -1e30f;
            for (int w = 0; w < kBlock / 64; ++w) {
#pragma unroll
                for (int q = 0; q < 6; ++q) t[q] += sh[w][q];
                tm = fmaxf(tm, shm[w]);
            }
            write_features(si, e - b, t[0], t[1], t[2], t[3], t[4], t[5], tm, dbar, logn20, F + lab(P, i) * kNF);
        }
    }
}

__device__ __forceinline__ float param_at(const float *g, int k) { return g[k]; }
__device__ __forceinline__ float param_at(const uint16_t *g, int k) { return bf16_to_f32(g[k]); }

// parameters (float32, or bfloat16 storage widened exactly) into LDS as float32
template <typename PT>
__device__ __forceinline__ void load_params(const PT *g, float *sh) {
    for (int k = threadIdx.x; k < kNParam; k += blockDim.x) sh[k] = param_at(g, k);
}

// One node: h1 = tanh(W1 x + b1) kept in registers (fully unrolled, static
// indices), h2 = tanh(W2 h1 + b2) produced one unit at a time (optionally
// stored to h2 in LDS), out = W3 h2 + b3.  P points to the parameters in LDS.
__device__ __forceinline__ void mlp_node(const float *P, const float (&x)[kNF], float (&h1)[kH], float *h2,
                                         float (&out)[kNO]) {
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float z = P[kOffB1 + o];
#pragma unroll
        for (int k = 0; k < kNF; ++k) z = fmaf(P[kOffW1 + o * kNF + k], x[k], z);
        h1[o] = tanhf(z);
    }
    float o0 = P[kOffB3], o1 = P[kOffB3 + 1];
    for (int o = 0; o < kH; ++o) {
        float z = P[kOffB2 + o];
#pragma unroll
        for (int k = 0; k < kH; ++k) z = fmaf(P[kOffW2 + o * kH + k], h1[k], z);
        const float h = tanhf(z);
        if (h2) h2[o] = h;
        o0 = fmaf(P[kOffW3 + o], h, o0);
        o1 = fmaf(P[kOffW3 + kH + o], h, o1);
    }
    out[0] = o0;
    out[1] = o1;
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_mlp_forward(const PT *params, const float *F, int64_t n, float *out) {
    __shared__ float P[kNParam];
    load_params(params, P);
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        float x[kNF], h1[kH], o[kNO];
#pragma unroll
        for (int k = 0; k < kNF; ++k) x[k] = F[i * kNF + k];
        mlp_node(P, x, h1, nullptr, o);
        out[2 * i] = o[0];
        out[2 * i + 1] = o[1];
    }
}

// Gradient of L = (1/N) sum_i ||out_i - T_i||^2 (N = number of nodes) with
// respect to the parameters, plus L itself; per-workgroup partials.
// blockDim = kTile = 128.  Thread t owns dW3[t/64][t%64], db3[t] (t < 2),
// dW2[t/2][(t%2)*32 + q] (q < 32), db2[t] and db1[t] (t < 64),
// dW1[t/2][(t%2)*8 + q] (q < 8).
template <typename PT>
__global__ __launch_bounds__(kTile) void k_mlp_grad(const PT *params, const float *F, const float *T, int64_t n,
                                                    float *partials /* gridDim x (kNParam + 1) */) {
    constexpr int SX = kNF + 1, SH = kH + 1;   // padded LDS rows (no bank conflicts)
    __shared__ float P[kNParam];
    __shared__ float xs[kTile * SX];
    __shared__ float h1s[kTile * SH];           // h1, later g_z1
    __shared__ float h2s[kTile * SH];           // h2, later g_z2
    __shared__ float gos[kTile * 2];
    __shared__ float red[kTile];
    load_params(params, P);
    const int t = threadIdx.x;
    float aW3 = 0.f, aB3 = 0.f, aW2[32], aB2 = 0.f, aW1[8], aB1 = 0.f, aLoss = 0.f;
#pragma unroll
    for (int q = 0; q < 32; ++q) aW2[q] = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) aW1[q] = 0.f;
    const float invN = 1.f / (float)n;
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * kTile; base < n; base += (int64_t)gridDim.x * kTile) {
        const int64_t i = base + t;
        const bool live = i < n;
        {   // A: forward of this thread's node (nodes past n run on x = 0 with a
            // zero output gradient, so they add nothing), loss, output gradient
            float x[kNF], h1[kH], o[kNO];
#pragma unroll
            for (int k = 0; k < kNF; ++k) x[k] = live ? F[i * kNF + k] : 0.f;
            mlp_node(P, x, h1, &h2s[t * SH], o);
            float g0 = 0.f, g1 = 0.f;
            if (live) {
                const float e0 = o[0] - T[2 * i], e1 = o[1] - T[2 * i + 1];
                aLoss += (e0 * e0 + e1 * e1) * invN;
                g0 = 2.f * e0 * invN;
                g1 = 2.f * e1 * invN;
            }
#pragma unroll
            for (int k = 0; k < kNF; ++k) xs[t * SX + k] = x[k];
#pragma unroll
            for (int k = 0; k < kH; ++k) h1s[t * SH + k] = h1[k];
            gos[2 * t] = g0;
            gos[2 * t + 1] = g1;
        }
        __syncthreads();
        {   // B: dW3, db3
            const int c = t / kH, o = t % kH;
            float acc = 0.f;
            for (int m = 0; m < kTile; ++m) acc = fmaf(gos[2 * m + c], h2s[m * SH + o], acc);
            aW3 += acc;
            if (t < kNO) {
                float b = 0.f;
                for (int m = 0; m < kTile; ++m) b += gos[2 * m + t];
                aB3 += b;
            }
        }
        __syncthreads();
        // C: g_z2 = (W3^T g_out) * (1 - h2^2), overwriting h2 (own row)
        for (int o = 0; o < kH; ++o) {
            const float h = h2s[t * SH + o];
            const float gh = P[kOffW3 + o] * gos[2 * t] + P[kOffW3 + kH + o] * gos[2 * t + 1];
            h2s[t * SH + o] = gh * (1.f - h * h);
        }
        __syncthreads();
        {   // D: dW2[o][k] = sum_m gz2[m][o] h1[m][k], db2
            const int o = t / 2, k0 = (t % 2) * 32;
            for (int m = 0; m < kTile; ++m) {
                const float g = h2s[m * SH + o];
#pragma unroll
                for (int q = 0; q < 32; ++q) aW2[q] = fmaf(g, h1s[m * SH + k0 + q], aW2[q]);
            }
            if (t < kH) {
                float b = 0.f;
                for (int m = 0; m < kTile; ++m) b += h2s[m * SH + t];
                aB2 += b;
            }
        }
        __syncthreads();
        // E: g_z1 = (W2^T g_z2) * (1 - h1^2), overwriting h1 (own row)
        for (int k = 0; k < kH; ++k) {
            float gh = 0.f;
            for (int o = 0; o < kH; ++o) gh = fmaf(P[kOffW2 + o * kH + k], h2s[t * SH + o], gh);
            const float h = h1s[t * SH + k];
            h1s[t * SH + k] = gh * (1.f - h * h);
        }
        __syncthreads();
        {   // F: dW1[o][f] = sum_m gz1[m][o] x[m][f], db1
            const int o = t / 2, f0 = (t % 2) * 8;
            for (int m = 0; m < kTile; ++m) {
                const float g = h1s[m * SH + o];
#pragma unroll
                for (int q = 0; q < 8; ++q) aW1[q] = fmaf(g, xs[m * SX + f0 + q], aW1[q]);
            }
            if (t < kH) {
                float b = 0.f;
                for (int m = 0; m < kTile; ++m) b += h1s[m * SH + t];
                aB1 += b;
            }
        }
        __syncthreads();
    }
    float *out = partials + (size_t)blockIdx.x * (kNParam + 1);
    out[kOffW3 + t] = aW3;
    if (t < kNO) out[kOffB3 + t] = aB3;
    {
        const int o = t / 2, k0 = (t % 2) * 32, f0 = (t % 2) * 8;
#pragma unroll
        for (int q = 0; q < 32; ++q) out[kOffW2 + o * kH + k0 + q] = aW2[q];
#pragma unroll
        for (int q = 0; q < 8; ++q) out[kOffW1 + o * kNF + f0 + q] = aW1[q];
    }
    if (t < kH) {
        out[kOffB2 + t] = aB2;
        out[kOffB1 + t] = aB1;
    }
    red[t] = aLoss;
    __syncthreads();
    for (int h = kTile / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) out[kNParam] = red[0];
}

// grad[p] = sum_b partials[b][p] (fixed order); loss = sum_b partials[b][kNParam]
__global__ __launch_bounds__(kBlock) void k_grad_reduce(const float *partials, int nb, float *grad, double *loss) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p > kNParam) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += (double)partials[(size_t)b * (kNParam + 1) + p];
    if (p < kNParam) grad[p] = (float)acc;
    else if (loss) *loss = acc;
}

// Adam (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// theta <- theta - lr mhat / (sqrt(vhat) + eps) with bias-corrected mhat, vhat.
// With `store`, the updated float32 master is also rounded to bfloat16 there.
__global__ __launch_bounds__(kBlock) void k_adam(float *theta, float *m, float *v, const float *g, int step, float lr,
                                                 float b1, float b2, float eps, uint16_t *store) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= kNParam) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const float mh = mp / (1.f - powf(b1, (float)step));
    const float vh = vp / (1.f - powf(b2, (float)step));
    const float th = theta[p] - lr * mh / (sqrtf(vh) + eps);
    theta[p] = th;
    if (store) store[p] = bf16_rne(th);
}

__global__ __launch_bounds__(kBlock) void k_to_bf16(const float *x, int64_t n, uint16_t *out) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = bf16_rne(x[i]);
}

// y0_i = -t_i * a_i / 4 with t_i = out_i0 limited to [-2, 2] (the range of
// -4 y*_i / a_i at an optimum, where y*_i = -sum_j w_ij (1 - X*_ij) / 4 and
// |X*_ij| <= 1); s = sum_i out_i1 (per-block partials).  A NaN output stays
// NaN (fmin/fmax would drop it), so the finiteness test below still sees it.
__global__ __launch_bounds__(kBlock) void k_warm_y0(const float *out, const float4 *stats, int64_t n, double *y0,
                                                    double *partials) {
    double s[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double o = (double)out[2 * i];
        const double t = o != o ? o : (o > 2.0 ? 2.0 : (o < -2.0 ? -2.0 : o));
        const double yi = -0.25 * t * (double)stats[i].z;
        y0[i] = yi;
        s[0] += (double)out[2 * i + 1];
        s[1] += yi;  // only read for finiteness: a NaN or Inf anywhere shows here
    }
    block_sums_store<2>(s, partials + (size_t)blockIdx.x * kMaxSums);
}

// training targets: t_i = -4 y_i / a_i (0 for isolated nodes), s_i = s
__global__ __launch_bounds__(kBlock) void k_ws_targets(const float4 *stats, const double *y, int64_t n, float s,
                                                       float *target) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double a = (double)stats[i].z;
        target[2 * i] = a > 0.0 ? (float)(-4.0 * y[i] / a) : 0.f;
        target[2 * i + 1] = s;
    }
}

}  // namespace

int launch_reduce(hipStream_t, const double *, int, int, double *);

int ws_targets(hipStream_t st, const float4 *stats, const double *y, int64_t n, double s, float *target) {
    int64_t need = (n + kBlock - 1) / kBlock;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(need, kMaxBlocks));
    hipLaunchKernelGGL(k_ws_targets, dim3(nb), dim3(kBlock), 0, st, stats, y, n, (float)s, target);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

static int blocks_for(int64_t items) {
    int64_t need = (items + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, kMaxBlocks));
}

int ws_features(hipStream_t s, const DevCsr &P, float *F, float4 *stats) {
    const int nb = blocks_for(P.n);
    const float dbar = P.n > 0 ? (float)((double)P.nnz / (double)P.n) : 0.f;
    const float logn20 = (float)(std::log((double)P.n) / 20.0);
    const int nh = (int)std::max<int64_t>(1, std::min<int64_t>(P.n_heavy, kMaxBlocks));
    switch (P.wmode) {
        case kWUnit:
            hipLaunchKernelGGL(k_node_stats<kWUnit>, dim3(nb), dim3(kBlock), 0, s, P, stats);
            hipLaunchKernelGGL(k_node_stats_heavy<kWUnit>, dim3(nh), dim3(kBlock), 0, s, P, stats);
            hipLaunchKernelGGL(k_features<kWUnit>, dim3(nb), dim3(kBlock), 0, s, P, stats, dbar, logn20, F);
            hipLaunchKernelGGL(k_features_heavy<kWUnit>, dim3(nh), dim3(kBlock), 0, s, P, stats, dbar, logn20, F);
            break;
        case kWSign:
            hipLaunchKernelGGL(k_node_stats<kWSign>, dim3(nb), dim3(kBlock), 0, s, P, stats);
            hipLaunchKernelGGL(k_node_stats_heavy<kWSign>, dim3(nh), dim3(kBlock), 0, s, P, stats);
            hipLaunchKernelGGL(k_features<kWSign>, dim3(nb), dim3(kBlock), 0, s, P, stats, dbar, logn20, F);
            hipLaunchKernelGGL(k_features_heavy<kWSign>, dim3(nh), dim3(kBlock), 0, s, P, stats, dbar, logn20, F);
            break;
        default:
            hipLaunchKernelGGL(k_node_stats<kWGeneral>, dim3(nb), dim3(kBlock), 0, s, P, stats);
            hipLaunchKernelGGL(k_node_stats_heavy<kWGeneral>, dim3(nh), dim3(kBlock), 0, s, P, stats);
            hipLaunchKernelGGL(k_features<kWGeneral>, dim3(nb), dim3(kBlock), 0, s, P, stats, dbar, logn20, F);
            hipLaunchKernelGGL(k_features_heavy<kWGeneral>, dim3(nh), dim3(kBlock), 0, s, P, stats, dbar, logn20,
                               F);
    }
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int mlp_forward(hipStream_t s, const void *params, int bf16, const float *F, int64_t n, float *out) {
    if (bf16)
        hipLaunchKernelGGL(k_mlp_forward<uint16_t>, dim3(blocks_for(n)), dim3(kBlock), 0, s,
                           (const uint16_t *)params, F, n, out);
    else
        hipLaunchKernelGGL(k_mlp_forward<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s, (const float *)params, F,
                           n, out);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int mlp_grad(hipStream_t s, const void *params, int bf16, const float *F, const float *T, int64_t n, float *grad,
             double *loss, float *partials) {
    int64_t tiles = (n + kTile - 1) / kTile;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, kGradBlocks));
    if (bf16)
        hipLaunchKernelGGL(k_mlp_grad<uint16_t>, dim3(nb), dim3(kTile), 0, s, (const uint16_t *)params, F, T, n,
                           partials);
    else
        hipLaunchKernelGGL(k_mlp_grad<float>, dim3(nb), dim3(kTile), 0, s, (const float *)params, F, T, n, partials);
    LRSDP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_grad_reduce, dim3((kNParam + 1 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, partials, nb,
                       grad, loss);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int mlp_adam(hipStream_t s, float *theta, float *m, float *v, const float *g, int step, float lr, uint16_t *store) {
    hipLaunchKernelGGL(k_adam, dim3((kNParam + kBlock - 1) / kBlock), dim3(kBlock), 0, s, theta, m, v, g, step, lr,
                       0.9f, 0.999f, 1e-8f, store);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int to_bf16(hipStream_t s, const float *x, int64_t n, uint16_t *out) {
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(kBlock), 0, s, x, n, out);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int warm_y0(hipStream_t s, const float *out, const float4 *stats, int64_t n, double *y0, double *partials,
            double *mean_out1) {
    const int nb = blocks_for(n);
    hipLaunchKernelGGL(k_warm_y0, dim3(nb), dim3(kBlock), 0, s, out, stats, n, y0, partials);
    LRSDP_CHECK_LAUNCH();
    return launch_reduce(s, partials, nb, 2, mean_out1);
}

int mlp_param_count() { return kNParam; }

}  // namespace lrsdp
