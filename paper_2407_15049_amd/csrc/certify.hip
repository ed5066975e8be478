// Dual certificate: the smallest eigenvalue of S = C - A*(y).
//
// Any multipliers y give a lower bound on the SDP optimum once the smallest
// eigenvalue of S is known (the error measures of Section 4.2 use it for the
// dual infeasibility err2):
//   MaxCut (trace X = n):   <C,X> = <S,X> + b^T y >= n min(0, lambda_min) + b^T y
//   completion (C = I):     lambda_min(I - A*(y)) = 1 - ||Y||_2, where Y is the
//                           n1 x n2 sparse matrix of the y_k, so y / max(1, ||Y||_2)
//                           is dual feasible and b^T y / max(1, 1 - lambda_min)
//                           bounds the optimum from below.
//
// lambda_min comes from block Lanczos with blocks of kCB = 8 vectors in
// float64 (a 64-byte row: one 4-lane group of the SpMM).  Per step:
//   W = S Q_j                                   (the problem's own SpMM)
//   A_j = Q_j^T W                               (Gram kernel + reduction)
//   W <- W - Q_j A_j - Q_{j-1} B_{j-1}^T        (fused with Q_j^T W, Q_{j-1}^T W)
//   W <- W - Q_j (Q_j^T W) - Q_{j-1} (Q_{j-1}^T W)   (one local re-orthogonalisation,
//                                                  fused with the Gram W^T W)
//   W = Q_{j+1} B_j                             (Cholesky QR applied twice, so that
//                                                Q_{j+1} stays orthonormal when W is
//                                                ill conditioned; B_j upper triangular)
// S Q_j = Q_{j-1} B_{j-1}^T + Q_j A_j + Q_{j+1} B_j, so T_k, the block
// tridiagonal matrix of the A_j and B_j, is S projected on the Krylov space.
// No basis is kept (memory: four n x 8 blocks) and there is no global
// re-orthogonalisation: the extreme Ritz values converge regardless (copies of
// converged ones may appear; they do not lower the smallest).  Within a step
// orthonormality is kept: a single Cholesky QR of an ill-conditioned W (common
// once the large eigenvalues of hub rows have converged) loses it and then the
// Ritz values leave the spectrum.  The smallest
// eigenvalue theta of T_k is found on the host by bisection on the inertia of
// the band LDL^T of T_k - sigma I, its eigenvector s by inverse iteration, and
// the residual of the Ritz pair is ||B_k s_last|| (s_last = last block of s).
// lambda_lb = theta - residual bounds the eigenvalue of S nearest theta from
// below; it bounds lambda_min(S) only if no lower eigenvalue was missed, which
// Lanczos cannot rule out, so the dual bound built on it is an estimate.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "device.h"
#include "internal.h"
#include "kernels.h"

namespace lrsdp {
namespace {

constexpr int kCB = 8;              // block size
constexpr int kCS = kCB * kCB;      // entries of a b x b block
constexpr int kCertGrid = 512;      // workgroups of the Gram kernels
constexpr int kCertCheck = 10;      // steps between convergence checks

struct CertStep {
    double A[kCS];   // Q_j^T S Q_j, symmetrised
    double B[kCS];   // upper-triangular factor of W_j = Q_{j+1} B_j
};

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// uniform(-1, 1) entries from a counter-based generator
__global__ __launch_bounds__(kBlock) void k_cert_random(double *Q, int64_t count, uint64_t seed) {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < count; e += (int64_t)gridDim.x * kBlock) {
        const uint64_t h = splitmix64(seed * 0xD1B54A32D192ED03ull + (uint64_t)e);
        Q[e] = (double)(h >> 11) * 0x1.0p-52 - 1.0;
    }
}

// Partial sums of a Gram kernel: per workgroup, kCP doubles (two 8 x 8
// matrices; single-matrix kernels fill the first kCS).
constexpr int kCP = 2 * kCS;

// Sum the per-lane accumulators acc[k] (column c = lane & 7 of the left
// operand, column k of the right one) over the wave and the workgroup and
// store (X^T Y)[c][k] at part[blockIdx.x * kCP + off + c * 8 + k].  Fixed order.
__device__ __forceinline__ void gram_store(double (&acc)[kCB], double *part, int off, double (*sh)[kCP]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c = threadIdx.x & 7;
#pragma unroll
    for (int k = 0; k < kCB; ++k) {
        double v = acc[k];
        v += __shfl_xor(v, 8, 64);
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (lane < kCB) sh[wave][off + c * kCB + k] = v;
    }
}

__device__ __forceinline__ void part_store(double *part, int count, double (*sh)[kCP]) {
    __syncthreads();
    if (threadIdx.x < count) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
        part[(size_t)blockIdx.x * kCP + threadIdx.x] = t;
    }
}

// Row i of an n x 8 block is owned by eight consecutive lanes, lane c holding
// entry c; other entries of the row come by shuffles inside the 8-lane group
// (the eight lanes share the row, so all of them are active together).
#define CERT_ROWS(i)                                                                           \
    for (int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kCB; i < n;                \
         i += (int64_t)gridDim.x * (kBlock / kCB))

// part <- partials of Q1^T Y (entries 0..63) and, if Q2 is given, Q2^T Y (64..127).
__global__ __launch_bounds__(kBlock) void k_cert_proj(const double *__restrict__ Q1, const double *__restrict__ Q2,
                                                      const double *__restrict__ Y, int64_t n, double *part) {
    __shared__ double sh[kBlock / 64][kCP];
    const int lane = threadIdx.x & 63, c = threadIdx.x & 7, base = lane & ~7;
    double a1[kCB] = {0, 0, 0, 0, 0, 0, 0, 0}, a2[kCB] = {0, 0, 0, 0, 0, 0, 0, 0};
    CERT_ROWS(i) {
        const double y = Y[i * kCB + c];
        const double x1 = Q1[i * kCB + c];
        const double x2 = Q2 ? Q2[i * kCB + c] : 0.0;
#pragma unroll
        for (int k = 0; k < kCB; ++k) {
            const double yk = __shfl(y, base | k, 64);
            a1[k] = fma(x1, yk, a1[k]);
            a2[k] = fma(x2, yk, a2[k]);
        }
    }
    gram_store(a1, part, 0, sh);
    gram_store(a2, part, kCS, sh);
    part_store(part, kCP, sh);
}

// Sum the partial rows into LDS g[0..K) with all kBlock threads (kBlock / K
// threads per entry over interleaved rows, combined in a fixed order).
template <int K>
__device__ __forceinline__ void reduce_part(const double *part, int np, double *g) {
    constexpr int P = kBlock / K;
    __shared__ double sh[P][K];
    const int e = threadIdx.x % K, q = threadIdx.x / K;
    double t = 0.0;
    for (int b = q; b < np; b += P) t += part[(size_t)b * kCP + e];
    sh[q][e] = t;
    __syncthreads();
    if (threadIdx.x < K) {
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < P; ++r) v += sh[r][threadIdx.x];
        g[threadIdx.x] = v;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_cert_fin_a(const double *part, int np, CertStep *steps, int j) {
    __shared__ double g[kCS];
    reduce_part<kCS>(part, np, g);
    if (threadIdx.x < kCS) {
        const int r = threadIdx.x / kCB, c = threadIdx.x % kCB;
        steps[j].A[threadIdx.x] = 0.5 * (g[r * kCB + c] + g[c * kCB + r]);
    }
}

// out[0..128) <- the reduced pair of projections (no symmetrisation)
__global__ __launch_bounds__(kBlock) void k_cert_fin_c(const double *part, int np, double *out) {
    __shared__ double g[kCP];
    reduce_part<kCP>(part, np, g);
    if (threadIdx.x < kCP) out[threadIdx.x] = g[threadIdx.x];
}

// W <- W - Q1 M1 - Q2 M2' with M2' = M2^T if trans2 else M2 (row times 8 x 8
// matrix; Q2 may be null).  Then mode 0: partials of Q1^T W and Q2^T W;
// mode 1: partials of W^T W.
__global__ __launch_bounds__(kBlock) void k_cert_sub(double *__restrict__ W, const double *__restrict__ Q1,
                                                     const double *M1, const double *__restrict__ Q2,
                                                     const double *M2, int trans2, int mode, int64_t n,
                                                     double *part) {
    __shared__ double sh[kBlock / 64][kCP];
    __shared__ double m1[kCS], m2[kCS];
    if (threadIdx.x < kCS) {
        const int r = threadIdx.x / kCB, c = threadIdx.x % kCB;
        m1[threadIdx.x] = M1[threadIdx.x];
        m2[threadIdx.x] = Q2 ? (trans2 ? M2[c * kCB + r] : M2[threadIdx.x]) : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, c = threadIdx.x & 7, base = lane & ~7;
    double a1[kCB] = {0, 0, 0, 0, 0, 0, 0, 0}, a2[kCB] = {0, 0, 0, 0, 0, 0, 0, 0};
    CERT_ROWS(i) {
        const double q1 = Q1[i * kCB + c];
        const double q2 = Q2 ? Q2[i * kCB + c] : 0.0;
        double w = W[i * kCB + c];
#pragma unroll
        for (int k = 0; k < kCB; ++k) {
            w = fma(-__shfl(q1, base | k, 64), m1[k * kCB + c], w);
            w = fma(-__shfl(q2, base | k, 64), m2[k * kCB + c], w);
        }
        W[i * kCB + c] = w;
        if (mode == 0) {
#pragma unroll
            for (int k = 0; k < kCB; ++k) {
                const double wk = __shfl(w, base | k, 64);
                a1[k] = fma(q1, wk, a1[k]);
                a2[k] = fma(q2, wk, a2[k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < kCB; ++k) a1[k] = fma(w, __shfl(w, base | k, 64), a1[k]);
        }
    }
    gram_store(a1, part, 0, sh);
    if (mode == 0) gram_store(a2, part, kCS, sh);
    part_store(part, mode == 0 ? kCP : kCS, sh);
}

// Cholesky factor R (upper, G = R^T R) of the reduced Gram matrix and R^{-1}.
// `scale2` bounds the squared size of the step (for the breakdown test):
// steps[j].A and steps[j-1].B when j >= 0 and first_pass, else the Gram
// diagonal.  Breakdown (a pivot at or below 1e-24 scale2, or not finite): the
// Krylov space is invariant; *flag records the first such step as j + 2 (1:
// the start block) and R, R^{-1} are zeroed so later steps stay finite.  If
// Rprev is given, B_j = R Rprev is stored in steps[j].B (the second pass of
// Cholesky QR).
__global__ __launch_bounds__(kBlock) void k_cert_chol(const double *part, int np, CertStep *steps, int j,
                                                      int first_pass, double *Rout, double *Rinv,
                                                      const double *Rprev, int *flag) {
    __shared__ double g[kCS];
    reduce_part<kCS>(part, np, g);
    if (threadIdx.x != 0) return;
    double scale = 0.0;
    for (int k = 0; k < kCB; ++k) scale = fmax(scale, g[k * kCB + k]);
    if (j >= 0 && first_pass) {
        double s = 0.0;
        for (int e = 0; e < kCS; ++e) {
            s = fmax(s, fabs(steps[j].A[e]));
            if (j > 0) s = fmax(s, fabs(steps[j - 1].B[e]));
        }
        scale = fmax(scale, s * s);
    }
    double R[kCS], Ri[kCS];
    for (int e = 0; e < kCS; ++e) R[e] = Ri[e] = 0.0;
    bool ok = scale > 0.0 && isfinite(scale);
    for (int p = 0; p < kCB && ok; ++p) {
        double d = g[p * kCB + p];
        for (int k = 0; k < p; ++k) d -= R[k * kCB + p] * R[k * kCB + p];
        if (!(d > 1e-24 * scale) || !isfinite(d)) {
            ok = false;
            break;
        }
        const double rpp = sqrt(d);
        R[p * kCB + p] = rpp;
        for (int q = p + 1; q < kCB; ++q) {
            double v = 0.5 * (g[p * kCB + q] + g[q * kCB + p]);
            for (int k = 0; k < p; ++k) v -= R[k * kCB + p] * R[k * kCB + q];
            R[p * kCB + q] = v / rpp;
        }
    }
    if (ok) {
        // inverse of the upper-triangular R by back substitution, column by column
        for (int c = 0; c < kCB; ++c) {
            for (int r = c; r >= 0; --r) {
                double v = (r == c) ? 1.0 : 0.0;
                for (int k = r + 1; k <= c; ++k) v -= R[r * kCB + k] * Ri[k * kCB + c];
                Ri[r * kCB + c] = v / R[r * kCB + r];
            }
        }
    } else {
        for (int e = 0; e < kCS; ++e) R[e] = Ri[e] = 0.0;
        if (*flag == 0) *flag = j + 2;
    }
    for (int e = 0; e < kCS; ++e) {
        Rout[e] = R[e];
        Rinv[e] = Ri[e];
    }
    if (Rprev && j >= 0) {
        for (int r = 0; r < kCB; ++r)
            for (int c = 0; c < kCB; ++c) {
                double v = 0.0;
                for (int k = r; k <= c; ++k) v += R[r * kCB + k] * Rprev[k * kCB + c];
                steps[j].B[r * kCB + c] = v;
            }
    }
}

// Qo_i = W_i Rinv (row times upper-triangular inverse; Qo may equal W), and if
// part is given the partials of Qo^T Qo.
__global__ __launch_bounds__(kBlock) void k_cert_scale(const double *W, const double *Rinv, double *Qo, int64_t n,
                                                       double *part) {
    __shared__ double sh[kBlock / 64][kCP];
    __shared__ double Ri[kCS];
    if (threadIdx.x < kCS) Ri[threadIdx.x] = Rinv[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, c = threadIdx.x & 7, base = lane & ~7;
    double acc[kCB] = {0, 0, 0, 0, 0, 0, 0, 0};
    CERT_ROWS(i) {
        const double w = W[i * kCB + c];
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < kCB; ++k) v = fma(__shfl(w, base | k, 64), Ri[k * kCB + c], v);
        Qo[i * kCB + c] = v;
        if (part) {
#pragma unroll
            for (int k = 0; k < kCB; ++k) acc[k] = fma(v, __shfl(v, base | k, 64), acc[k]);
        }
    }
    if (part) {
        gram_store(acc, part, 0, sh);
        part_store(part, kCS, sh);
    }
}

// b^T y: MaxCut b = 1 (b null), completion b_k = 2 M_ij.  One workgroup.
__global__ __launch_bounds__(kBlock) void k_cert_by(const double *b, const double *y, int64_t m, double *out) {
    double s[1] = {0.0};
    for (int64_t k = threadIdx.x; k < m; k += kBlock) s[0] += (b ? b[k] : 1.0) * y[k];
    block_sums_store<1>(s, out);
}

int grid_rows(int64_t n) {
    const int64_t need = (n * kCB + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, kCertGrid));
}

// ---------------------------------------------------------------------------
// Host: smallest eigenvalue of the block tridiagonal T_k (half-bandwidth kCB)
// ---------------------------------------------------------------------------

// Lower band of T_k: band[i * (kCB + 1) + d] = T[i][i - d].
std::vector<double> assemble_band(const std::vector<CertStep> &st, int k) {
    const int N = k * kCB, W = kCB + 1;
    std::vector<double> band((size_t)N * W, 0.0);
    for (int j = 0; j < k; ++j) {
        for (int p = 0; p < kCB; ++p)
            for (int q = 0; q <= p; ++q) band[(size_t)(j * kCB + p) * W + (p - q)] = st[j].A[p * kCB + q];
        if (j + 1 < k)
            for (int p = 0; p < kCB; ++p)
                for (int q = p; q < kCB; ++q)
                    band[(size_t)((j + 1) * kCB + p) * W + (kCB + p - q)] = st[j].B[p * kCB + q];
    }
    return band;
}

// Number of eigenvalues of T below sigma: negative pivots of the band LDL^T of
// T - sigma I (Sylvester's law of inertia).  A zero pivot is replaced by a
// tiny negative number (sigma is then taken as just above an eigenvalue).
int count_below(const std::vector<double> &band, int N, double sigma, double tiny) {
    const int W = kCB + 1;
    std::vector<double> M(band);
    int neg = 0;
    for (int i = 0; i < N; ++i) M[(size_t)i * W] -= sigma;
    for (int k = 0; k < N; ++k) {
        double d = M[(size_t)k * W];
        if (d == 0.0) d = -tiny;
        if (d < 0.0) ++neg;
        const int last = std::min(N - 1, k + kCB);
        for (int i = k + 1; i <= last; ++i) {
            const double lik = M[(size_t)i * W + (i - k)] / d;
            if (lik == 0.0) continue;
            for (int jj = k + 1; jj <= i; ++jj) M[(size_t)i * W + (i - jj)] -= lik * M[(size_t)jj * W + (jj - k)];
        }
    }
    return neg;
}

// Solve (T - sigma I) x = rhs in place for symmetric positive definite
// T - sigma I by band Cholesky.  Returns false if a pivot is not positive.
bool band_spd_solve(const std::vector<double> &band, int N, double sigma, std::vector<double> &x) {
    const int W = kCB + 1;
    std::vector<double> L(band);
    for (int i = 0; i < N; ++i) L[(size_t)i * W] -= sigma;
    for (int k = 0; k < N; ++k) {
        double d = L[(size_t)k * W];
        for (int p = std::max(0, k - kCB); p < k; ++p) d -= L[(size_t)k * W + (k - p)] * L[(size_t)k * W + (k - p)];
        if (!(d > 0.0)) return false;
        const double lkk = std::sqrt(d);
        L[(size_t)k * W] = lkk;
        const int last = std::min(N - 1, k + kCB);
        for (int i = k + 1; i <= last; ++i) {
            double v = L[(size_t)i * W + (i - k)];
            for (int p = std::max(0, i - kCB); p < k; ++p) v -= L[(size_t)i * W + (i - p)] * L[(size_t)k * W + (k - p)];
            L[(size_t)i * W + (i - k)] = v / lkk;
        }
    }
    for (int i = 0; i < N; ++i) {  // L z = x
        double v = x[i];
        for (int p = std::max(0, i - kCB); p < i; ++p) v -= L[(size_t)i * W + (i - p)] * x[p];
        x[i] = v / L[(size_t)i * W];
    }
    for (int i = N - 1; i >= 0; --i) {  // L^T x = z
        double v = x[i];
        for (int q = i + 1; q <= std::min(N - 1, i + kCB); ++q) v -= L[(size_t)q * W + (q - i)] * x[q];
        x[i] = v / L[(size_t)i * W];
    }
    return true;
}

// theta = lambda_min(T_k) and the residual norm ||B_last s_last|| of its Ritz
// pair (0 when has_next is false: the Krylov space is invariant).
void ritz_min(const std::vector<CertStep> &st, int k, bool has_next, double *theta, double *resid,
              double *theta_max = nullptr) {
    const int N = k * kCB, W = kCB + 1;
    const std::vector<double> band = assemble_band(st, k);
    double lo = INFINITY, hi = -INFINITY, amax = 0.0;
    for (int i = 0; i < N; ++i) {  // Gershgorin
        double off = 0.0;
        for (int d = 1; d <= kCB && d <= i; ++d) off += std::fabs(band[(size_t)i * W + d]);
        for (int d = 1; d <= kCB && i + d < N; ++d) off += std::fabs(band[(size_t)(i + d) * W + d]);
        const double a = band[(size_t)i * W];
        lo = std::min(lo, a - off);
        hi = std::max(hi, a + off);
        amax = std::max(amax, std::fabs(a) + off);
    }
    const double tiny = 1e-300 + 1e-30 * amax;
    // bisection for inf { sigma : count_below(sigma) >= 1 }
    double a = lo - 1e-12 * (amax + 1.0), b = hi + 1e-12 * (amax + 1.0);
    for (int it = 0; it < 200 && b - a > 4e-16 * std::max(std::fabs(a), std::fabs(b)) + 1e-300; ++it) {
        const double mid = 0.5 * (a + b);
        if (count_below(band, N, mid, tiny) >= 1) b = mid;
        else a = mid;
    }
    *theta = 0.5 * (a + b);
    if (theta_max) {  // the largest Ritz value: inf { sigma : count_below(sigma) >= N }
        double a2 = lo - 1e-12 * (amax + 1.0), b2 = hi + 1e-12 * (amax + 1.0);
        for (int it = 0; it < 200 && b2 - a2 > 4e-16 * std::max(std::fabs(a2), std::fabs(b2)) + 1e-300; ++it) {
            const double mid = 0.5 * (a2 + b2);
            if (count_below(band, N, mid, tiny) >= N) b2 = mid;
            else a2 = mid;
        }
        *theta_max = 0.5 * (a2 + b2);
    }
    *resid = 0.0;
    if (!has_next) return;
    // inverse iteration just below theta
    const double shift = *theta - (1e-10 * (amax + 1e-300) + 1e-12 * std::fabs(*theta));
    std::vector<double> x(N, 1.0), y(N);
    for (int i = 0; i < N; ++i) x[i] = 1.0 + 1e-3 * (double)((i * 7919) % 101);
    for (int it = 0; it < 3; ++it) {
        if (!band_spd_solve(band, N, shift, x)) break;
        double nrm = 0.0;
        for (double v : x) nrm += v * v;
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) break;
        for (double &v : x) v /= nrm;
    }
    // ||B_{k-1} s_last||
    const CertStep &last = st[k - 1];
    double r2 = 0.0;
    for (int p = 0; p < kCB; ++p) {
        double v = 0.0;
        for (int q = p; q < kCB; ++q) v += last.B[p * kCB + q] * x[(k - 1) * kCB + q];
        r2 += v * v;
    }
    *resid = std::sqrt(r2);
}

struct CertLayout {
    size_t q[3], w, part, steps, small, flag, by, yperm, total;
};

CertLayout cert_layout(int64_t n, int max_iter) {
    CertLayout L{};
    const size_t blk = (size_t)n * kCB * sizeof(double);
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t o = 0;
    for (int i = 0; i < 3; ++i) { L.q[i] = o; o += al(blk); }
    L.w = o; o += al(blk);
    L.part = o; o += al((size_t)kCertGrid * kCP * sizeof(double));
    L.steps = o; o += al((size_t)max_iter * sizeof(CertStep));
    L.small = o; o += al(6 * kCS * sizeof(double));   // C (2 blocks), R1, R1^{-1}, R2, R2^{-1}
    L.flag = o; o += 256;
    L.by = o; o += 256;
    L.yperm = o; o += al((size_t)n * sizeof(double));   // y in the library's node order (relabelled MaxCut)
    L.total = o;
    return L;
}

// Device addresses of the A and B blocks of step j (address arithmetic only).
const double *step_a(const CertStep *steps, int j) {
    return reinterpret_cast<const double *>(reinterpret_cast<const char *>(steps) + (size_t)j * sizeof(CertStep) +
                                            offsetof(CertStep, A));
}
const double *step_b(const CertStep *steps, int j) {
    return reinterpret_cast<const double *>(reinterpret_cast<const char *>(steps) + (size_t)j * sizeof(CertStep) +
                                            offsetof(CertStep, B));
}

int apply_s(hipStream_t s, const lrsdp_problem *p, const double *V, const double *y, double *Y) {
    if (p->info.kind == LRSDP_MAXCUT) {
        SpmmArgs a;
        a.epi = kEpiPlain;
        a.V = V;
        a.Y = Y;
        a.ytil = y;
        a.ld = kCB;
        int np = 0;
        return spmm_maxcut(s, p->csr, LRSDP_F64, a, &np);
    }
    if (p->info.kind == LRSDP_GENERAL) return spmm_general(s, p->gen, LRSDP_F64, V, kCB, y, Y);
    return spmm_completion(s, p->cmp, LRSDP_F64, V, kCB, y, Y);
}

}  // namespace
}  // namespace lrsdp

using namespace lrsdp;

extern "C" int lrsdp_certify_workspace_bytes(const lrsdp_problem *p, int max_iter, size_t *bytes) {
    clear_error();
    if (!p || !bytes || max_iter < 1) return set_error(LRSDP_EINVAL, "bad argument");
    *bytes = cert_layout(p->info.n, max_iter).total;
    return LRSDP_OK;
}

// y_lib: y is in the library's node order already (the solver's own calls);
// otherwise a relabelled MaxCut problem's y is moved into that order first.
static int certify_run(lrsdp_ctx *c, const lrsdp_problem *p, const double *y, int max_iter, double tol,
                       uint64_t seed, void *work, size_t work_bytes, lrsdp_cert *out, bool y_lib) {
    if (!c || !p || !y || !work || !out || max_iter < 1 || !(tol >= 0.0))
        return set_error(LRSDP_EINVAL, "bad argument");
    if (!p->uploaded) return set_error(LRSDP_EINVAL, "problem has not been uploaded");
    const int64_t n = p->info.n;
    if (n < 2 * kCB) return set_error(LRSDP_EUNSUPPORTED, "certificate needs n >= %d (got %lld)", 2 * kCB, (long long)n);
    const CertLayout L = cert_layout(n, max_iter);
    if (work_bytes < L.total)
        return set_error(LRSDP_ENOMEM, "certificate workspace needs %zu bytes, got %zu", L.total, work_bytes);
    if ((uintptr_t)work % 256) return set_error(LRSDP_EINVAL, "workspace must be 256-byte aligned");
    char *ws = static_cast<char *>(work);
    double *Q[3] = {reinterpret_cast<double *>(ws + L.q[0]), reinterpret_cast<double *>(ws + L.q[1]),
                    reinterpret_cast<double *>(ws + L.q[2])};
    double *Wb = reinterpret_cast<double *>(ws + L.w);
    double *part = reinterpret_cast<double *>(ws + L.part);
    CertStep *steps = reinterpret_cast<CertStep *>(ws + L.steps);
    double *small = reinterpret_cast<double *>(ws + L.small);
    double *Cm = small, *R1 = small + 2 * kCS, *R1i = small + 3 * kCS, *R2 = small + 4 * kCS, *R2i = small + 5 * kCS;
    int *flag = reinterpret_cast<int *>(ws + L.flag);
    double *by = reinterpret_cast<double *>(ws + L.by);
    hipStream_t s = c->stream;
    const int g = grid_rows(n);
    int rc;
    if (!y_lib && p->info.kind == LRSDP_MAXCUT && p->csr.perm) {
        double *yp = reinterpret_cast<double *>(ws + L.yperm);
        if ((rc = launch_permute_vec(s, y, yp, p->csr.perm, n, 0))) return rc;
        y = yp;
    }

    LRSDP_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
    const bool mc = p->info.kind == LRSDP_MAXCUT;
    const double *bvec = mc ? nullptr : (p->info.kind == LRSDP_GENERAL ? p->gen.b : p->cmp.b);
    hipLaunchKernelGGL(k_cert_by, dim3(1), dim3(kBlock), 0, s, bvec, y, p->info.m, by);
    LRSDP_CHECK_LAUNCH();
    // start block: random, orthonormalised by Cholesky QR applied twice
    hipLaunchKernelGGL(k_cert_random, dim3(g), dim3(kBlock), 0, s, Wb, n * kCB, seed);
    hipLaunchKernelGGL(k_cert_proj, dim3(g), dim3(kBlock), 0, s, Wb, nullptr, Wb, n, part);
    hipLaunchKernelGGL(k_cert_chol, dim3(1), dim3(kBlock), 0, s, part, g, steps, -1, 1, R1, R1i, nullptr, flag);
    hipLaunchKernelGGL(k_cert_scale, dim3(g), dim3(kBlock), 0, s, Wb, R1i, Wb, n, part);
    hipLaunchKernelGGL(k_cert_chol, dim3(1), dim3(kBlock), 0, s, part, g, steps, -1, 0, R2, R2i, nullptr, flag);
    hipLaunchKernelGGL(k_cert_scale, dim3(g), dim3(kBlock), 0, s, Wb, R2i, Q[0], n, nullptr);
    LRSDP_CHECK_LAUNCH();

    std::vector<CertStep> host;
    int cur = 0, prev = -1;
    int64_t done = 0;
    double theta = NAN, resid = NAN, theta_max = NAN;
    int status = 1;
    for (int j = 0; j < max_iter; ++j) {
        if ((rc = apply_s(s, p, Q[cur], y, Wb))) return rc;
        const double *Qp = prev >= 0 ? Q[prev] : nullptr;
        const double *Aj = step_a(steps, j);
        const double *Bp = j > 0 ? step_b(steps, j - 1) : nullptr;
        // A_j = Q_j^T S Q_j
        hipLaunchKernelGGL(k_cert_proj, dim3(g), dim3(kBlock), 0, s, Q[cur], nullptr, Wb, n, part);
        hipLaunchKernelGGL(k_cert_fin_a, dim3(1), dim3(kBlock), 0, s, part, g, steps, j);
        // three-term recurrence, then one re-orthogonalisation against Q_j, Q_{j-1}
        hipLaunchKernelGGL(k_cert_sub, dim3(g), dim3(kBlock), 0, s, Wb, Q[cur], Aj, Qp, Bp, 1, 0, n, part);
        hipLaunchKernelGGL(k_cert_fin_c, dim3(1), dim3(kBlock), 0, s, part, g, Cm);
        hipLaunchKernelGGL(k_cert_sub, dim3(g), dim3(kBlock), 0, s, Wb, Q[cur], Cm, Qp, Cm + kCS, 0, 1, n, part);
        // Cholesky QR twice: W = Q_{j+1} R2 R1, B_j = R2 R1
        hipLaunchKernelGGL(k_cert_chol, dim3(1), dim3(kBlock), 0, s, part, g, steps, j, 1, R1, R1i, nullptr, flag);
        hipLaunchKernelGGL(k_cert_scale, dim3(g), dim3(kBlock), 0, s, Wb, R1i, Wb, n, part);
        hipLaunchKernelGGL(k_cert_chol, dim3(1), dim3(kBlock), 0, s, part, g, steps, j, 0, R2, R2i, R1, flag);
        const int nxt = prev < 0 ? (cur + 1) % 3 : 3 - cur - prev;  // the buffer holding neither Q_j nor Q_{j-1}
        hipLaunchKernelGGL(k_cert_scale, dim3(g), dim3(kBlock), 0, s, Wb, R2i, Q[nxt], n, nullptr);
        LRSDP_CHECK_LAUNCH();
        prev = cur;
        cur = nxt;
        done = j + 1;
        if (done % kCertCheck != 0 && done != max_iter) continue;
        int hflag = 0;
        host.resize(done);
        LRSDP_HIP_TRY(hipMemcpyAsync(host.data(), steps, done * sizeof(CertStep), hipMemcpyDeviceToHost, s));
        LRSDP_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        LRSDP_HIP_TRY(hipStreamSynchronize(s));
        if (hflag == 1) return set_error(LRSDP_ENUMERIC, "certificate start block is rank deficient");
        if (hflag > 1) {
            // breakdown in step hflag - 2: its A is valid, the space is invariant
            const int k = hflag - 1;
            ritz_min(host, k, false, &theta, &resid);
            done = k;
            status = 2;
            break;
        }
        ritz_min(host, (int)done, true, &theta, &resid);
        if (!std::isfinite(theta)) return set_error(LRSDP_ENUMERIC, "certificate produced a non-finite eigenvalue");
        if (resid <= tol) {
            status = 0;
            break;
        }
    }
    if (done > 0 && (int64_t)host.size() >= done) {   // the largest Ritz value of the final space (once)
        double t2 = 0.0, r2 = 0.0;
        ritz_min(host, (int)done, false, &t2, &r2, &theta_max);
    }
    double hby = 0.0;
    LRSDP_HIP_TRY(hipMemcpyAsync(&hby, by, sizeof(double), hipMemcpyDeviceToHost, s));
    LRSDP_HIP_TRY(hipStreamSynchronize(s));
    out->lambda_min = theta;
    out->resid = resid;
    out->lambda_lb = theta - resid;
    out->by = hby;
    out->err2 = std::max(0.0, -theta) / (1.0 + p->info.c_l1);
    if (mc) out->dual_bound = hby + (double)n * std::min(0.0, out->lambda_lb);
    else if (p->info.kind == LRSDP_COMPLETION) out->dual_bound = hby / std::max(1.0, 1.0 - out->lambda_lb);
    else out->dual_bound = NAN;   // needs a bound on trace X, which a general problem does not state
    out->iters = done;
    out->status = status;
    out->block = kCB;
    out->lambda_max = theta_max;
    return LRSDP_OK;
}

extern "C" int lrsdp_certify(lrsdp_ctx *c, const lrsdp_problem *p, const double *y, int max_iter, double tol,
                             uint64_t seed, void *work, size_t work_bytes, lrsdp_cert *out) {
    clear_error();
    return certify_run(c, p, y, max_iter, tol, seed, work, work_bytes, out, false);
}

int lrsdp::certify_lib_order(lrsdp_ctx *c, const lrsdp_problem *p, const double *y, int max_iter, double tol,
                             uint64_t seed, void *work, size_t work_bytes, lrsdp_cert *out) {
    return certify_run(c, p, y, max_iter, tol, seed, work, work_bytes, out, true);
}
