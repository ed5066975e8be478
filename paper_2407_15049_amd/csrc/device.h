// Device helpers shared by the lrsdp kernels: 16-byte row chunks, lane-group
// and wavefront reductions (64-wide wavefronts), deterministic block sums.
#pragma once

#include "internal.h"

namespace lrsdp {

// A row of an n x ld array is processed in 16-byte chunks: 2 doubles or 4 floats.
template <typename S> struct Chunk;
template <> struct Chunk<double> {
    using V = double2;
    static constexpr int N = 2;
};
template <> struct Chunk<float> {
    using V = float4;
    static constexpr int N = 4;
};

__device__ __forceinline__ double2 vzero(double2) { return make_double2(0.0, 0.0); }
__device__ __forceinline__ float4 vzero(float4) { return make_float4(0.f, 0.f, 0.f, 0.f); }

// Chunk `lane` of the row starting at `row`, or zero when the lane holds no
// chunk of the row (act false).  The load is unconditional: an inactive lane
// reads the row's first chunk (in bounds whenever the row is) and discards it.
// A conditional load would be a branch around each load, into which the
// compiler sinks the consumers and their waits, one memory round trip each.
template <typename S>
__device__ __forceinline__ typename Chunk<S>::V chunk_or_zero(const S *row, int lane, bool act) {
    using CV = typename Chunk<S>::V;
    const CV t = *reinterpret_cast<const CV *>(row + (act ? lane * Chunk<S>::N : 0));
    return act ? t : vzero(CV{});
}

// The same for a row given as an array of chunks.
template <typename CV>
__device__ __forceinline__ CV vchunk_or_zero(const CV *row_chunks, int lane, bool act) {
    const CV t = row_chunks[act ? lane : 0];
    return act ? t : vzero(CV{});
}

// a += w * b
__device__ __forceinline__ void vfma(double2 &a, double w, const double2 &b) {
    a.x = fma(w, b.x, a.x);
    a.y = fma(w, b.y, a.y);
}
__device__ __forceinline__ void vfma(float4 &a, float w, const float4 &b) {
    a.x = fmaf(w, b.x, a.x);
    a.y = fmaf(w, b.y, a.y);
    a.z = fmaf(w, b.z, a.z);
    a.w = fmaf(w, b.w, a.w);
}

// float64 dot product of two chunks (float inputs promoted before the products)
__device__ __forceinline__ void vscale(double2 &a, double w) {
    a.x *= w;
    a.y *= w;
}
__device__ __forceinline__ void vscale(float4 &a, float w) {
    a.x *= w;
    a.y *= w;
    a.z *= w;
    a.w *= w;
}
__device__ __forceinline__ double vdot(const double2 &a, const double2 &b) {
    return fma(a.x, b.x, a.y * b.y);
}
__device__ __forceinline__ double vdot(const float4 &a, const float4 &b) {
    double s = (double)a.x * (double)b.x;
    s = fma((double)a.y, (double)b.y, s);
    s = fma((double)a.z, (double)b.z, s);
    s = fma((double)a.w, (double)b.w, s);
    return s;
}

// Chunk <-> 4 doubles (x, y, z, w; unused lanes zero for double2)
struct D4 {
    double v[4];
};
__device__ __forceinline__ D4 widen(const double2 &a) { return D4{{a.x, a.y, 0.0, 0.0}}; }
__device__ __forceinline__ D4 widen(const float4 &a) {
    return D4{{(double)a.x, (double)a.y, (double)a.z, (double)a.w}};
}
__device__ __forceinline__ void narrow(const D4 &d, double2 &a) {
    a.x = d.v[0];
    a.y = d.v[1];
}
__device__ __forceinline__ void narrow(const D4 &d, float4 &a) {
    a.x = (float)d.v[0];
    a.y = (float)d.v[1];
    a.z = (float)d.v[2];
    a.w = (float)d.v[3];
}

template <typename V>
__device__ __forceinline__ V ldg(const V *p) {
    return *p;
}

// Sum over an aligned group of GS lanes (GS a power of two <= 64).
template <int GS>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = GS / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, GS);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Reduce K per-thread sums over the block (kBlock threads) and write them to
// out[0..K) (one row of the partials array).  Fixed order: deterministic.
template <int K>
__device__ __forceinline__ void block_sums_store(const double (&s)[K], double *out) {
    __shared__ double sh[kBlock / 64][K > 0 ? K : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double v = wave_sum(s[k]);
        if (lane == 0) sh[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// Inside a single-block kernel (blockDim.x == kBlock): out[k] = sum over rows b
// < nrows of part[b * kMaxSums + k], k < K.  Each thread walks rows t, t+kBlock,
// ... accumulating K sums, then a fixed wavefront/LDS tree: deterministic.
// `out` is shared memory, valid for every thread on return.
template <int K>
__device__ __forceinline__ void reduce_rows(const double *part, int nrows, double *out) {
    __shared__ double sh[kBlock / 64][K];
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nrows; b += kBlock) {
        const double *p = part + (size_t)b * kMaxSums;
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += p[k];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double v = wave_sum(acc[k]);
        if (lane == 0) sh[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// Cooperative copy of a POD struct between global and shared memory.
template <typename T>
__device__ __forceinline__ void block_copy(T *dst, const T *src) {
    static_assert(sizeof(T) % 8 == 0, "struct size must be a multiple of 8");
    const uint64_t *s = reinterpret_cast<const uint64_t *>(src);
    uint64_t *d = reinterpret_cast<uint64_t *>(dst);
    for (int i = threadIdx.x; i < (int)(sizeof(T) / 8); i += blockDim.x) d[i] = s[i];
}

// float32 -> bfloat16, round to nearest, ties to even (NaN kept quiet)
__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// bfloat16 bits -> float32 (exact)
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

}  // namespace lrsdp
