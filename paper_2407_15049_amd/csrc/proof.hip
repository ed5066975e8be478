// Proof of a lower bound on lambda_min(C - A*(y)) for small problems, on the
// host in float64 (no device work).
//
// For the error measures of Section 4.2 the dual slack S = C - A*(y) must be
// positive semidefinite; a lower bound lb on lambda_min(S) turns the
// multipliers into a bound on the optimum (MaxCut: trace X = n; completion:
// C = I).  The block Lanczos estimate of the certificate cannot exclude a
// missed eigenvalue below its Ritz values.  Here S - shift I is formed densely
// and factorised by Cholesky; if every pivot is positive the standard
// rounding analysis of Cholesky (any order of the inner products, no
// underflow) gives R^T R = S' + E with |E| <= gamma_{n+1} |R^T| |R|, so
//   ||E||_2 <= gamma_{n+1} || |R| ||_F^2,  gamma_k = k u / (1 - k u),  u = 2^-53,
// and lambda_min(S) >= shift - ||E||_2 - ||F||_2, where F is the rounding of
// the entries of S' when it is formed (bounded entry by entry, then in the
// Frobenius norm).  Every floating-point sum entering the margin is itself
// enlarged by its own gamma factor.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.h"

using namespace lrsdp;

namespace {

constexpr double kU = 1.1102230246251565e-16;   // 2^-53

inline double gamma_k(double k) { return k * kU / (1.0 - k * kU); }

// Dense S - shift I (row-major, both triangles) and, per entry, a bound on the
// rounding of its formation (sum of |terms| times gamma of the term count).
struct Dense {
    int64_t n = 0;
    std::vector<double> a;     // n x n
    std::vector<double> err;   // n x n
};

// a[i][j] += v (and a[j][i] when i != j), err bookkeeping: `terms` counts the
// values summed into each entry, `absum` their absolute values.
struct Acc {
    Dense &d;
    std::vector<double> absum, extra;
    std::vector<int32_t> terms;
    explicit Acc(Dense &dd) : d(dd), absum(dd.a.size(), 0.0), extra(dd.a.size(), 0.0), terms(dd.a.size(), 0) {}
    // a rounding already made in a value before it is added (a product)
    void add_err(int64_t i, int64_t j, double e) {
        extra[i * d.n + j] += e;
        if (i != j) extra[j * d.n + i] += e;
    }
    void add(int64_t i, int64_t j, double v) {
        const int64_t n = d.n;
        d.a[i * n + j] += v;
        absum[i * n + j] += std::fabs(v);
        terms[i * n + j] += 1;
        if (i != j) {
            d.a[j * n + i] += v;
            absum[j * n + i] += std::fabs(v);
            terms[j * n + i] += 1;
        }
    }
    // rounding bound of each entry: a sum of t values has error <= gamma_{t-1}
    // sum |values|, plus the roundings made inside the values
    void finish() {
        for (size_t e = 0; e < d.a.size(); ++e)
            d.err[e] = (terms[e] > 1 ? gamma_k((double)terms[e] - 1.0) * absum[e] : 0.0) + extra[e] * (1.0 + kU);
    }
};

int build_dense(const lrsdp_problem *p, const double *y, double shift, Dense &d) {
    const int64_t n = p->info.n;
    d.n = n;
    d.a.assign((size_t)(n * n), 0.0);
    d.err.assign((size_t)(n * n), 0.0);
    Acc acc(d);
    if (p->info.kind == LRSDP_MAXCUT) {
        // internal node k is the caller's node perm[k] (degree order) or k
        auto lab = [&](int64_t k) -> int64_t { return p->perm.empty() ? k : p->perm[k]; };
        for (int64_t i = 0; i < n; ++i) {
            acc.add(i, i, p->diag[i]);
            acc.add(i, i, -y[lab(i)]);
            acc.add(i, i, -shift);
            for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
                const uint32_t raw = (uint32_t)p->col[e];
                const int64_t j = (int64_t)(raw & 0x7fffffffu);
                if (j <= i) continue;   // each edge once; add() writes both triangles
                double c;
                if (p->info.weights == kWGeneral) c = p->val[e];
                else c = (raw & 0x80000000u) ? -0.25 : 0.25;
                acc.add(i, j, c);
            }
        }
    } else if (p->info.kind == LRSDP_COMPLETION) {
        // C = I; A_k = E_{i, n1+j} + E_{n1+j, i}
        for (int64_t i = 0; i < n; ++i) {
            acc.add(i, i, 1.0);
            acc.add(i, i, -shift);
        }
        const int64_t n1 = p->info.n1;
        for (int64_t k = 0; k < p->info.m; ++k) acc.add(p->samp_i[k], n1 + p->samp_j[k], -y[k]);
    } else {
        // general: C on Omega (or dense), A_k on Omega, both symmetric
        if (!p->cdense.empty()) {
            for (int64_t i = 0; i < n; ++i)
                for (int64_t j = i; j < n; ++j) acc.add(i, j, p->cdense[(size_t)(i * n + j)]);
        } else {
            for (size_t o = 0; o < p->om_a.size(); ++o)
                if (p->cval[o] != 0.0) acc.add(p->om_a[o], p->om_b[o], p->cval[o]);
        }
        for (int64_t k = 0; k < p->info.m; ++k)
            for (int32_t e = p->a_ptr[k]; e < p->a_ptr[k + 1]; ++e) {
                const int32_t o = p->a_idx[e];
                const double t = -y[k] * p->a_val[e];
                acc.add(p->om_a[o], p->om_b[o], t);
                acc.add_err(p->om_a[o], p->om_b[o], kU * std::fabs(t));   // the product's own rounding
            }
        for (int64_t i = 0; i < n; ++i) acc.add(i, i, -shift);
    }
    acc.finish();
    return LRSDP_OK;
}

// Cholesky-Banachiewicz in place on the lower triangle (row-major), by blocks
// of kPB rows: the entries of a block's rows left of the block depend only on
// earlier blocks, so host threads take those rows in parallel (each row's
// entries in column order); the block's own triangle follows on one thread.
// Every entry is the same sequence of operations as the one-thread algorithm,
// so the rounding analysis is unchanged.  Returns -1 on success, else the index
// of the first non-positive (or non-finite) pivot.
constexpr int64_t kPB = 64;

void row_left(std::vector<double> &a, int64_t n, int64_t i, int64_t j1) {
    double *ri = &a[(size_t)(i * n)];
    for (int64_t j = 0; j < j1; ++j) {
        const double *rj = &a[(size_t)(j * n)];
        double s = ri[j];
        for (int64_t k = 0; k < j; ++k) s -= ri[k] * rj[k];
        ri[j] = s / rj[j];
    }
}

int64_t cholesky_rows(std::vector<double> &a, int64_t n) {
    const int nt = (int)std::max<int64_t>(
        1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(), kPB}));
    for (int64_t b0 = 0; b0 < n; b0 += kPB) {
        const int64_t b1 = std::min(n, b0 + kPB);
        if (b0 > 0) {
            // rows of the block, columns [0, b0): independent rows
            std::vector<std::thread> pool;
            for (int t = 0; t < nt; ++t)
                pool.emplace_back([&, t]() {
                    for (int64_t i = b0 + t; i < b1; i += nt) row_left(a, n, i, b0);
                });
            for (auto &th : pool) th.join();
        }
        // the block's own triangle, row by row
        for (int64_t i = b0; i < b1; ++i) {
            double *ri = &a[(size_t)(i * n)];
            for (int64_t j = b0; j <= i; ++j) {
                const double *rj = &a[(size_t)(j * n)];
                double s = ri[j];
                for (int64_t k = 0; k < j; ++k) s -= ri[k] * rj[k];
                if (j < i) {
                    ri[j] = s / rj[j];
                } else {
                    if (!(s > 0.0) || !std::isfinite(s)) return i;
                    ri[i] = std::sqrt(s);
                }
            }
        }
    }
    return -1;
}

}  // namespace

extern "C" int lrsdp_certify_dense(const lrsdp_problem *p, const double *y, double shift, lrsdp_proof *out) {
    clear_error();
    if (!p || !y || !out) return set_error(LRSDP_EINVAL, "NULL argument");
    if (!std::isfinite(shift)) return set_error(LRSDP_EINVAL, "shift is not finite");
    const int64_t n = p->info.n;
    if (n < 1 || n > LRSDP_PROOF_MAX_N)
        return set_error(LRSDP_EUNSUPPORTED, "dense proof for n <= %d (n = %lld)", LRSDP_PROOF_MAX_N, (long long)n);
    for (int64_t k = 0; k < p->info.m; ++k)
        if (!std::isfinite(y[k])) return set_error(LRSDP_EINVAL, "y[%lld] is not finite", (long long)k);
    std::memset(out, 0, sizeof(*out));
    out->shift = shift;
    Dense d;
    int rc = build_dense(p, y, shift, d);
    if (rc) return rc;
    // ||F||_2 <= ||F||_F from the entry bounds (scaled by the largest, so that
    // no square underflows)
    double emax = 0.0;
    for (double e : d.err) emax = std::max(emax, e);
    double f2 = 0.0;
    if (emax > 0.0)
        for (double e : d.err) f2 += (e / emax) * (e / emax);
    const double form = emax * std::sqrt(f2 * (1.0 + gamma_k((double)d.err.size() + 2.0))) * (1.0 + 4.0 * kU);
    // b^T y and its rounding
    double by = 0.0, byabs = 0.0;
    for (int64_t k = 0; k < p->info.m; ++k) {
        const double bk = p->info.kind == LRSDP_MAXCUT ? 1.0 : p->b[k];
        by += bk * y[k];
        byabs += std::fabs(bk * y[k]);
    }
    const double by_lo = by - gamma_k((double)p->info.m + 1.0) * byabs;
    out->by = by;
    const int64_t piv = cholesky_rows(d.a, n);
    if (piv >= 0) {
        out->status = 1;
        out->pivot = piv;
        out->lambda_lb = NAN;
        out->margin = NAN;
        out->dual_bound = NAN;
        return LRSDP_OK;
    }
    // || |R| ||_F^2 from the computed factor (lower triangle), rounded up
    double fro = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            const double r = d.a[(size_t)(i * n + j)];
            fro += r * r;
        }
    const double npos = (double)n * (double)(n + 1) / 2.0;
    fro = fro / (1.0 - gamma_k(npos));
    const double chol = gamma_k((double)n + 1.0) * fro;
    const double margin = (chol + form) * (1.0 + 8.0 * kU) + 2.0 * kU * std::fabs(shift);
    const double lb = shift - margin;
    out->status = 0;
    out->pivot = -1;
    out->margin = margin;
    out->lambda_lb = lb;
    const double lam = std::min(0.0, lb);
    if (p->info.kind == LRSDP_MAXCUT) {
        // b^T y + n min(0, lb), rounded down
        const double v = by_lo + (double)n * lam;
        out->dual_bound = v - 4.0 * kU * (std::fabs(by_lo) + (double)n * std::fabs(lam));
    } else if (p->info.kind == LRSDP_COMPLETION) {
        // y / (1 - min(0, lb)) is dual feasible: bound b^T y / (1 - min(0, lb)), rounded down
        const double den = 1.0 - lam;
        const double q = by_lo >= 0.0 ? by_lo / (den * (1.0 + 2.0 * kU)) : by_lo / (den * (1.0 - 2.0 * kU));
        out->dual_bound = q - 2.0 * kU * std::fabs(q);
    } else {
        out->dual_bound = NAN;   // needs a bound on trace X, which a general problem does not state
    }
    return LRSDP_OK;
}
