// Small kernels used by the per-kernel entry points: row dots of the MaxCut
// constraint map, the multiplier estimate, assembly of the line-search
// coefficients and ALM measures from reduced sums, and the two-loop recursion
// for explicitly stored pairs.
#include "device.h"
#include "kernels.h"

namespace lrsdp {

double exact_step_host(double a1, double a2, double a3, double a4);

namespace {

// out_i = U_i . V_i  (MaxCut A(U V^T) = diag(U V^T)); lane group per row
template <typename S, int GS>
__global__ __launch_bounds__(kBlock) void k_rowdot(const S *U, const S *V, int64_t n, int64_t ld, double *out) {
    using CV = typename Chunk<S>::V;
    constexpr int NV = Chunk<S>::N;
    constexpr int GPB = kBlock / GS;
    const int lane = threadIdx.x % GS, grp = threadIdx.x / GS;
    const bool active = lane * NV < ld;
    for (int64_t row = (int64_t)blockIdx.x * GPB + grp; row < n; row += (int64_t)gridDim.x * GPB) {
        double t = 0.0;
        if (active) {
            const int64_t off = row * ld + lane * NV;
            t = vdot(*reinterpret_cast<const CV *>(U + off), *reinterpret_cast<const CV *>(V + off));
        }
        t = group_sum<GS>(t);
        if (lane == 0) out[row] = t;
    }
}

// ytil = y + sigma (b - a)  (elementwise, length m; b = 1 when b == nullptr)
__global__ void k_ytil(const double *y, const double *a, const double *b, double sigma, int64_t m, double *ytil) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        ytil[i] = y[i] + sigma * ((b ? b[i] : 1.0) - a[i]);
}

// out = {a1, a2, a3, a4, p1, p2, ||q1||^2, ||q2||^2} from the reduced sums
// {p2, ytil.q2, ytil.q1, q2.q2, q1.q2, q1.q1, p1}
__global__ void k_ls_out(const double *s, double sigma, double *out) {
    if (threadIdx.x != 0) return;
    out[0] = 0.5 * sigma * s[3];
    out[1] = sigma * s[4];
    out[2] = s[0] - s[1] + 0.5 * sigma * s[5];
    out[3] = s[6] - s[2];
    out[4] = s[6];
    out[5] = s[0];
    out[6] = s[5];
    out[7] = s[3];
}

// completion: sums {0, ytil.q2, ytil.q1, q2.q2, q1.q2, q1.q1, 0} and d = {<D,R>, <D,D>}
__global__ void k_ls_out_cmp(const double *s, const double *d, double sigma, double *out) {
    if (threadIdx.x != 0) return;
    const double p1 = 2.0 * d[0], p2 = d[1];
    out[0] = 0.5 * sigma * s[3];
    out[1] = sigma * s[4];
    out[2] = p2 - s[1] + 0.5 * sigma * s[5];
    out[3] = p1 - s[2];
    out[4] = p1;
    out[5] = p2;
    out[6] = s[5];
    out[7] = s[3];
}

// out = {obj, dual, ||res||, err1, err1_inf, err3, 0, 0} from {obj, b.y, ||res||^2}
__global__ void k_alm_out(const double *s, double b_l1, double b_inf, double *out) {
    if (threadIdx.x != 0) return;
    const double obj = s[0], dual = s[1], rn = sqrt(fmax(s[2], 0.0));
    out[0] = obj;
    out[1] = dual;
    out[2] = rn;
    out[3] = rn / (1.0 + b_l1);
    out[4] = rn / (1.0 + b_inf);
    out[5] = (obj - dual) / (1.0 + fabs(obj) + fabs(dual));
    out[6] = 0.0;
    out[7] = 0.0;
}

// Two-loop recursion of Algorithm 1 on coefficients for the layout
// basis = [G, S_0..S_{k-1}, Y_0..Y_{k-1}]; gram is nb x nb (row stride nb).
// flag = 1 if some <y_t, s_t> <= 0.
__global__ void k_two_loop_pairs(const double *gram, int k, double *coef, int *flag) {
    if (threadIdx.x != 0) return;
    const int nb = 2 * k + 1;
    double q[kMaxBasis], alpha[kMaxMem], beta[kMaxMem];
    for (int j = 0; j < nb; ++j) q[j] = 0.0;
    q[0] = -1.0;
    *flag = 0;
    auto dot_basis = [&](int i, const double *v) {  // <basis_i, v>
        double t = 0.0;
        for (int j = 0; j < nb; ++j) t += gram[i * nb + j] * v[j];
        return t;
    };
    for (int t = 0; t < k; ++t) {
        double ys = gram[(1 + k + t) * nb + (1 + t)];
        if (!(ys > 0.0)) *flag = 1;
        beta[t] = 1.0 / ys;
    }
    for (int t = k - 1; t >= 0; --t) {
        alpha[t] = beta[t] * dot_basis(1 + t, q);
        q[1 + k + t] -= alpha[t];
    }
    for (int t = 0; t < k; ++t) {
        double c = alpha[t] - beta[t] * dot_basis(1 + k + t, q);
        q[1 + t] += c;
    }
    for (int j = 0; j < nb; ++j) coef[j] = q[j];
}

__global__ void k_gather_gram(const double *red, int nb, int row, double *gram) {
    // red: nb sums <x_row, basis_j>
    for (int j = threadIdx.x; j < nb; j += blockDim.x) gram[row * nb + j] = red[j];
}

}  // namespace

int launch_rowdot(hipStream_t s, int prec, const void *U, const void *V, int64_t n, int64_t ld, double *out) {
    const int cpr = (int)(ld * (prec == LRSDP_F64 ? 8 : 4) / 16);
    const int gs = cpr <= 4 ? 4 : (cpr <= 8 ? 8 : 16);
    int64_t need = (n + kBlock / gs - 1) / (kBlock / gs);
    int nb = (int)std::max<int64_t>(1, std::min<int64_t>(need, kMaxBlocks));
    if (prec == LRSDP_F64) {
        if (gs == 4) hipLaunchKernelGGL((k_rowdot<double, 4>), dim3(nb), dim3(kBlock), 0, s, (const double *)U, (const double *)V, n, ld, out);
        else if (gs == 8) hipLaunchKernelGGL((k_rowdot<double, 8>), dim3(nb), dim3(kBlock), 0, s, (const double *)U, (const double *)V, n, ld, out);
        else hipLaunchKernelGGL((k_rowdot<double, 16>), dim3(nb), dim3(kBlock), 0, s, (const double *)U, (const double *)V, n, ld, out);
    } else {
        if (gs == 4) hipLaunchKernelGGL((k_rowdot<float, 4>), dim3(nb), dim3(kBlock), 0, s, (const float *)U, (const float *)V, n, ld, out);
        else if (gs == 8) hipLaunchKernelGGL((k_rowdot<float, 8>), dim3(nb), dim3(kBlock), 0, s, (const float *)U, (const float *)V, n, ld, out);
        else hipLaunchKernelGGL((k_rowdot<float, 16>), dim3(nb), dim3(kBlock), 0, s, (const float *)U, (const float *)V, n, ld, out);
    }
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_ytil(hipStream_t s, const double *y, const double *a, const double *b, double sigma, int64_t m,
                double *ytil) {
    int64_t need = (m + kBlock - 1) / kBlock;
    int nb = (int)std::max<int64_t>(1, std::min<int64_t>(need, kMaxBlocks));
    hipLaunchKernelGGL(k_ytil, dim3(nb), dim3(kBlock), 0, s, y, a, b, sigma, m, ytil);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_ls_out(hipStream_t s, const double *sums, double sigma, double *out) {
    hipLaunchKernelGGL(k_ls_out, dim3(1), dim3(64), 0, s, sums, sigma, out);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_ls_out_cmp(hipStream_t s, const double *sums, const double *d, double sigma, double *out) {
    hipLaunchKernelGGL(k_ls_out_cmp, dim3(1), dim3(64), 0, s, sums, d, sigma, out);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_alm_out(hipStream_t s, const double *sums, double b_l1, double b_inf, double *out) {
    hipLaunchKernelGGL(k_alm_out, dim3(1), dim3(64), 0, s, sums, b_l1, b_inf, out);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_two_loop_pairs(hipStream_t s, const double *gram, int k, double *coef, int *flag) {
    hipLaunchKernelGGL(k_two_loop_pairs, dim3(1), dim3(64), 0, s, gram, k, coef, flag);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

int launch_gather_gram(hipStream_t s, const double *red, int nb, int row, double *gram) {
    hipLaunchKernelGGL(k_gather_gram, dim3(1), dim3(64), 0, s, red, nb, row, gram);
    LRSDP_CHECK_LAUNCH();
    return LRSDP_OK;
}

}  // namespace lrsdp
