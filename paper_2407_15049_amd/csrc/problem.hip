// Host-side problem build (CSR of the SpMM operator, work lists) and upload.
//
// MaxCut (paper, MaxCut section): C = -L(G,w)/4 with the Laplacian
// L_ij = -w_ij on edges and L_ii = sum_k w_ik, so C_ij = w_ij/4 off the
// diagonal and C_ii = -sum_k w_ik/4; A(X) = diag(X), b = 1.
//
// Completion (paper, matrix-completion section): X = [[W1, M], [M^T, W2]] of
// order n1 + n2, C = I, sample k = (i, j) gives A_k = E_{i,n1+j} + E_{n1+j,i}
// and b_k = 2 M_ij.  The operator C - A*(y) then has unit diagonal and the
// off-diagonal entries -y_k at (i, n1+j) and (n1+j, i), stored as a "top" CSR
// (rows i, column j) and a "bottom" CSR (rows j, column i, sample id).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <thread>

#include "internal.h"

namespace lrsdp {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

}  // namespace lrsdp

using namespace lrsdp;

extern "C" const char *lrsdp_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *lrsdp_version(void) { return "lrsdp 0.1 (gfx950)"; }

namespace {

// Host threads for a build pass over `work` entries: one per 2^20 entries, at
// most 16 and at most the hardware's count.
int host_threads(int64_t work) {
    int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
    return (int)std::max<int64_t>(1, std::min<int64_t>({16, hw, work >> 20}));
}

// Light rows sorted by decreasing length inside windows of consecutive rows, so
// a wavefront's groups walk rows of similar length while touching nearby rows.
constexpr int64_t kWindow = 8192;

void build_work_lists(lrsdp_problem *p, int64_t n) {
    const auto &rp = p->row_ptr;
    p->light.clear();
    p->heavy.clear();
    p->seg.clear();
    p->heavy_seg.assign(1, 0);
    std::vector<int32_t> win;
    for (int64_t w0 = 0; w0 < n; w0 += kWindow) {
        int64_t w1 = std::min(n, w0 + kWindow);
        win.clear();
        for (int64_t i = w0; i < w1; ++i) {
            int64_t len = rp[i + 1] - rp[i];
            if (len <= kSegLen) {
                win.push_back((int32_t)i);
            } else {
                p->heavy.push_back((int32_t)i);
                for (int64_t b = rp[i]; b < rp[i + 1]; b += kSegLen) {
                    int4 s;
                    s.x = (int32_t)i;
                    s.y = (int32_t)b;
                    s.z = (int32_t)std::min<int64_t>(b + kSegLen, rp[i + 1]);
                    s.w = (int32_t)p->seg.size();
                    p->seg.push_back(s);
                }
                p->heavy_seg.push_back((int32_t)p->seg.size());
            }
        }
        std::stable_sort(win.begin(), win.end(), [&](int32_t a, int32_t b) {
            return (rp[a + 1] - rp[a]) > (rp[b + 1] - rp[b]);
        });
        for (int32_t i : win) p->light.push_back(make_int4(i, rp[i], rp[i + 1], 0));
    }
}

}  // namespace

extern "C" int lrsdp_problem_maxcut(int64_t n, int64_t n_edges, const int32_t *u,
                                    const int32_t *v, const double *w,
                                    lrsdp_problem **out) {
    return lrsdp_problem_maxcut_ex(n, n_edges, u, v, w, LRSDP_ORDER_INPUT, out);
}

extern "C" int lrsdp_problem_maxcut_ex(int64_t n, int64_t n_edges, const int32_t *u, const int32_t *v,
                                       const double *w, int node_order, lrsdp_problem **out) {
    clear_error();
    if (!out) return set_error(LRSDP_EINVAL, "out is NULL");
    if (node_order != LRSDP_ORDER_INPUT && node_order != LRSDP_ORDER_DEGREE)
        return set_error(LRSDP_EINVAL, "node_order %d is neither LRSDP_ORDER_INPUT nor LRSDP_ORDER_DEGREE",
                         node_order);
    *out = nullptr;
    if (n < 1 || n > INT32_MAX - 1) return set_error(LRSDP_EINVAL, "n = %lld out of range", (long long)n);
    if (n_edges < 0) return set_error(LRSDP_EINVAL, "n_edges < 0");
    if (n_edges > 0 && (!u || !v)) return set_error(LRSDP_EINVAL, "edge arrays are NULL");
    if (2 * n_edges > (int64_t)INT32_MAX) return set_error(LRSDP_EUNSUPPORTED, "2*n_edges exceeds int32 indexing");

    int mode = kWUnit;
    if (w) {
        mode = kWSign;
        for (int64_t e = 0; e < n_edges; ++e) {
            if (!std::isfinite(w[e])) return set_error(LRSDP_EINVAL, "weight %lld is not finite", (long long)e);
            if (w[e] != 1.0 && w[e] != -1.0) mode = kWGeneral;
        }
    }
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t e = 0; e < n_edges; ++e) {
        int64_t a = u[e], b = v[e];
        if (a < 0 || a >= n || b < 0 || b >= n)
            return set_error(LRSDP_EINVAL, "edge %lld = (%lld, %lld) has an endpoint outside [0, %lld)",
                             (long long)e, (long long)a, (long long)b, (long long)n);
        if (a == b) return set_error(LRSDP_EINVAL, "edge %lld is a self loop at node %lld", (long long)e, (long long)a);
        deg[a]++;
        deg[b]++;
    }
    auto *p = new lrsdp_problem();
    // Node order.  With LRSDP_ORDER_DEGREE, internal node k is the caller's
    // node perm[k], nodes taken by decreasing degree and increasing label: the
    // factor rows of the high-degree nodes, gathered by most rows of the
    // SpMM, then sit next to each other in memory and share cache lines.
    std::vector<int32_t> newid;   // caller label -> internal label (empty: the identity)
    if (node_order == LRSDP_ORDER_DEGREE) {
        int64_t dmax = 0;
        for (int64_t i = 0; i < n; ++i) dmax = std::max(dmax, deg[i]);
        std::vector<int64_t> start(dmax + 2, 0);   // counting sort by decreasing degree, stable in the label
        for (int64_t i = 0; i < n; ++i) start[dmax - deg[i] + 1]++;
        for (int64_t d = 0; d <= dmax; ++d) start[d + 1] += start[d];
        p->perm.resize(n);
        newid.resize(n);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t k = start[dmax - deg[i]]++;
            p->perm[k] = (int32_t)i;
            newid[i] = (int32_t)k;
        }
        std::vector<int64_t> d2(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) d2[newid[i]] = deg[i];
        deg.swap(d2);
    }
    p->row_ptr.resize(n + 1);
    p->row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) p->row_ptr[i + 1] = (int32_t)(p->row_ptr[i] + deg[i]);
    const int64_t nnz = p->row_ptr[n];
    std::vector<int32_t> fill(p->row_ptr.begin(), p->row_ptr.end() - 1);
    std::vector<double> wv(nnz);
    p->col.resize(nnz);
    const bool relabel = !newid.empty();
    for (int64_t e = 0; e < n_edges; ++e) {
        double we = w ? w[e] : 1.0;
        int32_t a = relabel ? newid[u[e]] : u[e], b = relabel ? newid[v[e]] : v[e];
        int32_t pa = fill[a]++, pb = fill[b]++;
        p->col[pa] = b;
        p->col[pb] = a;
        wv[pa] = we;
        wv[pb] = we;
    }
    // sort each row by column (deterministic layout, duplicate detection); rows
    // are independent, so blocks of rows go to host threads, and the per-row
    // terms of ||vec(C)||_1 are added in row order afterwards (the same sum
    // whatever the thread count)
    p->diag.assign(n, 0.0);
    p->hrow.assign(n, 0.0);
    std::vector<double> row_l1(n, 0.0);
    std::vector<int64_t> dup_row(1, -1);
    auto sort_rows = [&](int64_t r0, int64_t r1, int64_t *first_dup) {
        std::vector<std::pair<int32_t, double>> ent;
        for (int64_t i = r0; i < r1; ++i) {
            int64_t b0 = p->row_ptr[i], b1 = p->row_ptr[i + 1];
            int64_t len = b1 - b0;
            ent.resize(len);
            for (int64_t k = 0; k < len; ++k) ent[k] = {p->col[b0 + k], wv[b0 + k]};
            std::sort(ent.begin(), ent.end(),
                      [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
                          return x.first < y.first;
                      });
            double wsum = 0.0, wabs = 0.0, l1 = 0.0;
            for (int64_t k = 0; k < len; ++k) {
                if (k > 0 && ent[k].first == ent[k - 1].first) {
                    *first_dup = i;
                    return;
                }
                p->col[b0 + k] = ent[k].first;
                wv[b0 + k] = ent[k].second;
                wsum += ent[k].second;
                wabs += std::fabs(ent[k].second);
                l1 += std::fabs(ent[k].second) * 0.25;
            }
            p->diag[i] = -0.25 * wsum;
            row_l1[i] = l1 + std::fabs(p->diag[i]);
            p->hrow[i] = 0.25 * wabs + std::fabs(p->diag[i]);   // sum_j |C_ij|, finished below
        }
    };
    {
        const int nt = host_threads(nnz);
        std::vector<int64_t> first_dup(nt, -1);
        std::vector<std::thread> pool;
        const int64_t chunk = (n + nt - 1) / nt;
        for (int t = 0; t < nt; ++t) {
            int64_t r0 = std::min<int64_t>(n, t * chunk), r1 = std::min<int64_t>(n, r0 + chunk);
            pool.emplace_back(sort_rows, r0, r1, &first_dup[t]);
        }
        for (auto &th : pool) th.join();
        for (int t = 0; t < nt; ++t)
            if (first_dup[t] >= 0) {
                int64_t i = first_dup[t];
                std::vector<int32_t> c(p->col.begin() + p->row_ptr[i], p->col.begin() + p->row_ptr[i + 1]);
                std::sort(c.begin(), c.end());
                int32_t d = c[std::adjacent_find(c.begin(), c.end()) - c.begin()];
                const long long ci = p->perm.empty() ? (long long)i : (long long)p->perm[i];
                const int cd = p->perm.empty() ? d : p->perm[d];
                delete p;
                return set_error(LRSDP_EINVAL, "edge (%lld, %d) appears more than once", ci, cd);
            }
    }
    double c_l1 = 0.0;
    int64_t max_row = 0;
    for (int64_t i = 0; i < n; ++i) {
        c_l1 += row_l1[i];
        max_row = std::max<int64_t>(max_row, p->row_ptr[i + 1] - p->row_ptr[i]);
    }
    // h_i of the row-block H0 of the L-BFGS direction (solve option precond)
    const double hfloor = n > 0 ? 1e-3 * c_l1 / (double)n : 0.0;
    for (int64_t i = 0; i < n; ++i) p->hrow[i] = 2.0 * std::max(p->hrow[i], hfloor);
    if (mode == kWSign) {
        for (int64_t k = 0; k < nnz; ++k)
            if (wv[k] < 0) p->col[k] = (int32_t)((uint32_t)p->col[k] | 0x80000000u);
    } else if (mode == kWGeneral) {
        p->val.resize(nnz);
        for (int64_t k = 0; k < nnz; ++k) p->val[k] = 0.25 * wv[k];
    }
    build_work_lists(p, n);
    auto &I = p->info;
    I.kind = LRSDP_MAXCUT;
    I.n = n;
    I.m = n;
    I.nnz = nnz;
    I.weights = mode;
    I.max_row_nnz = max_row;
    I.c_l1 = c_l1;
    I.b_l1 = (double)n;
    I.b_inf = 1.0;
    I.node_order = node_order;
    *out = p;
    return LRSDP_OK;
}

extern "C" int lrsdp_problem_completion(int64_t n1, int64_t n2, int64_t m, const int32_t *i,
                                        const int32_t *j, const double *Mij,
                                        lrsdp_problem **out) {
    clear_error();
    if (!out) return set_error(LRSDP_EINVAL, "out is NULL");
    *out = nullptr;
    if (n1 < 1 || n2 < 1 || n1 + n2 > INT32_MAX - 1) return set_error(LRSDP_EINVAL, "bad block sizes");
    if (m < 0 || m > (int64_t)INT32_MAX) return set_error(LRSDP_EINVAL, "bad sample count");
    if (m > 0 && (!i || !j || !Mij)) return set_error(LRSDP_EINVAL, "sample arrays are NULL");
    for (int64_t k = 0; k < m; ++k) {
        if (i[k] < 0 || i[k] >= n1 || j[k] < 0 || j[k] >= n2)
            return set_error(LRSDP_EINVAL, "sample %lld = (%d, %d) out of range", (long long)k, i[k], j[k]);
        if (!std::isfinite(Mij[k])) return set_error(LRSDP_EINVAL, "value %lld is not finite", (long long)k);
    }
    auto *p = new lrsdp_problem();
    p->samp_i.assign(i, i + m);
    p->samp_j.assign(j, j + m);
    p->b.resize(m);
    double b_l1 = 0.0, b_inf = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        p->b[k] = 2.0 * Mij[k];
        b_l1 += std::fabs(p->b[k]);
        b_inf = std::max(b_inf, std::fabs(p->b[k]));
    }
    // top CSR: rows i, entries sorted by j, holding (j, k)
    std::vector<int32_t> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return i[a] != i[b] ? i[a] < i[b] : j[a] < j[b];
    });
    for (int64_t t = 1; t < m; ++t)
        if (i[ord[t]] == i[ord[t - 1]] && j[ord[t]] == j[ord[t - 1]]) {
            delete p;
            return set_error(LRSDP_EINVAL, "sample (%d, %d) appears more than once", i[ord[t]], j[ord[t]]);
        }
    p->top_ptr.assign(n1 + 1, 0);
    for (int64_t k = 0; k < m; ++k) p->top_ptr[i[k] + 1]++;
    for (int64_t r = 0; r < n1; ++r) p->top_ptr[r + 1] += p->top_ptr[r];
    p->top_col.resize(m);
    p->top_eid.resize(m);
    for (int64_t t = 0; t < m; ++t) {
        p->top_col[t] = j[ord[t]];
        p->top_eid[t] = ord[t];
    }
    // bottom CSR: rows j, entries sorted by i, holding (i, k)
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return j[a] != j[b] ? j[a] < j[b] : i[a] < i[b];
    });
    p->bot_ptr.assign(n2 + 1, 0);
    for (int64_t k = 0; k < m; ++k) p->bot_ptr[j[k] + 1]++;
    for (int64_t r = 0; r < n2; ++r) p->bot_ptr[r + 1] += p->bot_ptr[r];
    p->bot_row.resize(m);
    p->bot_eid.resize(m);
    for (int64_t t = 0; t < m; ++t) {
        p->bot_row[t] = i[ord[t]];
        p->bot_eid[t] = ord[t];
    }
    int64_t max_row = 0;
    for (int64_t r = 0; r < n1; ++r) max_row = std::max<int64_t>(max_row, p->top_ptr[r + 1] - p->top_ptr[r]);
    for (int64_t r = 0; r < n2; ++r) max_row = std::max<int64_t>(max_row, p->bot_ptr[r + 1] - p->bot_ptr[r]);
    auto &I = p->info;
    I.kind = LRSDP_COMPLETION;
    I.n = n1 + n2;
    I.m = m;
    I.nnz = 2 * m;
    I.n1 = n1;
    I.n2 = n2;
    I.weights = 0;
    I.max_row_nnz = max_row;
    I.c_l1 = (double)(n1 + n2);
    I.b_l1 = b_l1;
    I.b_inf = b_inf;
    *out = p;
    return LRSDP_OK;
}

extern "C" void lrsdp_problem_destroy(lrsdp_problem *prob) { delete prob; }

extern "C" int lrsdp_problem_get_info(const lrsdp_problem *prob, lrsdp_problem_info *out) {
    clear_error();
    if (!prob || !out) return set_error(LRSDP_EINVAL, "NULL argument");
    *out = prob->info;
    return LRSDP_OK;
}

extern "C" int lrsdp_problem_general_ex(int64_t n, int64_t c_nnz, const int32_t *c_row, const int32_t *c_col,
                                        const double *c_val, int64_t m, int64_t a_nnz, const int32_t *a_con,
                                        const int32_t *a_row, const int32_t *a_col, const double *a_val,
                                        const double *b, int c_storage, lrsdp_problem **out) {
    clear_error();
    if (!out) return set_error(LRSDP_EINVAL, "out is NULL");
    *out = nullptr;
    if (c_storage != LRSDP_C_AUTO && c_storage != LRSDP_C_SPARSE && c_storage != LRSDP_C_DENSE)
        return set_error(LRSDP_EINVAL, "c_storage = %d", c_storage);
    if (c_storage == LRSDP_C_DENSE && n > kDenseMaxN)
        return set_error(LRSDP_EINVAL, "dense C storage is for n <= %lld (n = %lld)", (long long)kDenseMaxN,
                         (long long)n);
    if (n < 1 || n > INT32_MAX - 1) return set_error(LRSDP_EINVAL, "n = %lld out of range", (long long)n);
    if (m < 1 || m > INT32_MAX - 1) return set_error(LRSDP_EINVAL, "m = %lld out of range", (long long)m);
    if (c_nnz < 0 || a_nnz < 0 || a_nnz > INT32_MAX) return set_error(LRSDP_EINVAL, "bad entry counts");
    if ((c_nnz > 0 && (!c_row || !c_col || !c_val)) || (a_nnz > 0 && (!a_con || !a_row || !a_col || !a_val)) || !b)
        return set_error(LRSDP_EINVAL, "input arrays are NULL");
    for (int64_t t = 0; t < c_nnz; ++t) {
        if (c_row[t] < 0 || c_row[t] >= n || c_col[t] < 0 || c_col[t] >= n)
            return set_error(LRSDP_EINVAL, "C entry %lld = (%d, %d) out of range", (long long)t, c_row[t], c_col[t]);
        if (!std::isfinite(c_val[t])) return set_error(LRSDP_EINVAL, "C value %lld is not finite", (long long)t);
    }
    for (int64_t t = 0; t < a_nnz; ++t) {
        if (a_con[t] < 0 || a_con[t] >= m)
            return set_error(LRSDP_EINVAL, "A entry %lld names constraint %d", (long long)t, a_con[t]);
        if (a_row[t] < 0 || a_row[t] >= n || a_col[t] < 0 || a_col[t] >= n)
            return set_error(LRSDP_EINVAL, "A entry %lld = (%d, %d) out of range", (long long)t, a_row[t], a_col[t]);
        if (!std::isfinite(a_val[t])) return set_error(LRSDP_EINVAL, "A value %lld is not finite", (long long)t);
    }
    for (int64_t k = 0; k < m; ++k)
        if (!std::isfinite(b[k])) return set_error(LRSDP_EINVAL, "b[%lld] is not finite", (long long)k);
    auto key = [n](int32_t r, int32_t c) {
        const int64_t a = std::min(r, c), bb = std::max(r, c);
        return a * n + bb;
    };
    // C: positions of the upper triangle, repeated positions summed
    std::vector<std::pair<int64_t, double>> ce(c_nnz);
    for (int64_t t = 0; t < c_nnz; ++t) ce[t] = {key(c_row[t], c_col[t]), c_val[t]};
    std::sort(ce.begin(), ce.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
    std::vector<std::pair<int64_t, double>> cs;
    for (const auto &e : ce) {
        if (!cs.empty() && cs.back().first == e.first) cs.back().second += e.second;
        else cs.push_back(e);
    }
    // A: (constraint, position) pairs, repeated ones summed
    struct AE {
        int32_t k;
        int64_t pos;
        double v;
    };
    std::vector<AE> ae(a_nnz);
    for (int64_t t = 0; t < a_nnz; ++t) ae[t] = {a_con[t], key(a_row[t], a_col[t]), a_val[t]};
    std::sort(ae.begin(), ae.end(), [](const AE &x, const AE &y) { return x.k != y.k ? x.k < y.k : x.pos < y.pos; });
    std::vector<AE> as;
    for (const auto &e : ae) {
        if (!as.empty() && as.back().k == e.k && as.back().pos == e.pos) as.back().v += e.v;
        else as.push_back(e);
    }
    // Storage of C (Section 3.5, last paragraph): a small C with many nonzeros
    // is kept as a dense n x n matrix applied by a dense product; then Omega
    // holds the nonzero columns of the stacked constraint matrix only.
    const double tri = 0.5 * (double)n * (double)(n + 1);
    const bool dense = c_storage == LRSDP_C_DENSE ||
                       (c_storage == LRSDP_C_AUTO && n <= kDenseAutoN && (double)cs.size() >= kDenseFrac * tri);
    // Omega = positions of C (sparse storage) and of the nonzero columns of the stacked matrix
    std::vector<int64_t> om;
    om.reserve((dense ? 0 : cs.size()) + as.size());
    if (!dense)
        for (const auto &e : cs) om.push_back(e.first);
    for (const auto &e : as) om.push_back(e.pos);
    std::sort(om.begin(), om.end());
    om.erase(std::unique(om.begin(), om.end()), om.end());
    if ((int64_t)om.size() > INT32_MAX / 2) return set_error(LRSDP_EINVAL, "|Omega| = %zu too large", om.size());
    auto idx = [&](int64_t pos) { return (int32_t)(std::lower_bound(om.begin(), om.end(), pos) - om.begin()); };
    const int64_t nom = (int64_t)om.size();
    auto *p = new lrsdp_problem();
    p->om_a.resize(nom);
    p->om_b.resize(nom);
    p->cval.assign(nom, 0.0);
    for (int64_t o = 0; o < nom; ++o) {
        p->om_a[o] = (int32_t)(om[o] / n);
        p->om_b[o] = (int32_t)(om[o] % n);
    }
    double c_l1 = 0.0;
    if (dense) {
        p->cdense.assign((size_t)n * (size_t)n, 0.0);
        for (const auto &e : cs) {
            const int64_t a = e.first / n, bb = e.first % n;
            p->cdense[(size_t)a * n + bb] = e.second;
            p->cdense[(size_t)bb * n + a] = e.second;
            c_l1 += (a == bb ? 1.0 : 2.0) * std::fabs(e.second);
        }
    } else {
        for (const auto &e : cs) {
            const int32_t o = idx(e.first);
            p->cval[o] = e.second;
            c_l1 += (p->om_a[o] == p->om_b[o] ? 1.0 : 2.0) * std::fabs(e.second);
        }
    }
    // stacked constraint matrix by constraint rows (sorted by Omega index)
    p->a_ptr.assign(m + 1, 0);
    p->a_idx.resize(as.size());
    p->a_val.resize(as.size());
    for (size_t t = 0; t < as.size(); ++t) {
        p->a_ptr[as[t].k + 1]++;
        p->a_idx[t] = idx(as[t].pos);
        p->a_val[t] = as[t].v;
    }
    for (int64_t k = 0; k < m; ++k) p->a_ptr[k + 1] += p->a_ptr[k];
    for (int64_t k = 0; k < m; ++k)
        (p->a_ptr[k + 1] - p->a_ptr[k] > kLongRow ? p->con_long : p->con_short).push_back((int32_t)k);
    // its transpose by positions (sorted by constraint)
    p->at_ptr.assign(nom + 1, 0);
    for (size_t t = 0; t < as.size(); ++t) p->at_ptr[p->a_idx[t] + 1]++;
    for (int64_t o = 0; o < nom; ++o) p->at_ptr[o + 1] += p->at_ptr[o];
    p->at_idx.resize(as.size());
    p->at_val.resize(as.size());
    {
        std::vector<int32_t> fill(p->at_ptr.begin(), p->at_ptr.end() - 1);
        for (size_t t = 0; t < as.size(); ++t) {
            const int32_t o = p->a_idx[t];
            p->at_idx[fill[o]] = as[t].k;
            p->at_val[fill[o]] = as[t].v;
            fill[o]++;
        }
    }
    // symmetric pattern of Omega by rows: (a, b) in row a and, off the diagonal,
    // (b, a) in row b, each with its Omega index; columns ascending
    std::vector<std::pair<int64_t, int32_t>> se;   // (row * n + col, omega)
    se.reserve(2 * nom);
    for (int64_t o = 0; o < nom; ++o) {
        const int64_t a = p->om_a[o], bb = p->om_b[o];
        se.push_back({a * n + bb, (int32_t)o});
        if (a != bb) se.push_back({bb * n + a, (int32_t)o});
    }
    std::sort(se.begin(), se.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
    if ((int64_t)se.size() > INT32_MAX) {
        delete p;
        return set_error(LRSDP_EINVAL, "symmetric pattern too large");
    }
    p->s_ptr.assign(n + 1, 0);
    p->s_col.resize(se.size());
    p->s_om.resize(se.size());
    for (size_t t = 0; t < se.size(); ++t) {
        p->s_ptr[se[t].first / n + 1]++;
        p->s_col[t] = (int32_t)(se[t].first % n);
        p->s_om[t] = se[t].second;
    }
    int64_t max_row = 0;
    for (int64_t r = 0; r < n; ++r) {
        max_row = std::max<int64_t>(max_row, p->s_ptr[r + 1]);
        p->s_ptr[r + 1] += p->s_ptr[r];
    }
    p->b.assign(b, b + m);
    double b_l1 = 0.0, b_inf = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        b_l1 += std::fabs(b[k]);
        b_inf = std::max(b_inf, std::fabs(b[k]));
    }
    auto &I = p->info;
    I.kind = LRSDP_GENERAL;
    I.n = n;
    I.m = m;
    I.nnz = (int64_t)se.size();
    I.weights = kWGeneral;
    I.c_dense = dense ? 1 : 0;
    I.max_row_nnz = max_row;
    I.c_l1 = c_l1;
    I.b_l1 = b_l1;
    I.b_inf = b_inf;
    *out = p;
    return LRSDP_OK;
}

extern "C" int lrsdp_problem_general(int64_t n, int64_t c_nnz, const int32_t *c_row, const int32_t *c_col,
                                     const double *c_val, int64_t m, int64_t a_nnz, const int32_t *a_con,
                                     const int32_t *a_row, const int32_t *a_col, const double *a_val,
                                     const double *b, lrsdp_problem **out) {
    return lrsdp_problem_general_ex(n, c_nnz, c_row, c_col, c_val, m, a_nnz, a_con, a_row, a_col, a_val, b,
                                    LRSDP_C_AUTO, out);
}

extern "C" int lrsdp_problem_general_blocks(int64_t nblocks, const int64_t *block_n, int64_t c_nnz,
                                            const int32_t *c_blk, const int32_t *c_row, const int32_t *c_col,
                                            const double *c_val, int64_t m, int64_t a_nnz, const int32_t *a_con,
                                            const int32_t *a_blk, const int32_t *a_row, const int32_t *a_col,
                                            const double *a_val, const double *b, lrsdp_problem **out) {
    clear_error();
    if (!out) return set_error(LRSDP_EINVAL, "out is NULL");
    *out = nullptr;
    if (nblocks < 1 || !block_n) return set_error(LRSDP_EINVAL, "need at least one block");
    if (c_nnz < 0 || a_nnz < 0) return set_error(LRSDP_EINVAL, "bad entry counts");
    if ((c_nnz > 0 && (!c_blk || !c_row || !c_col)) || (a_nnz > 0 && (!a_blk || !a_row || !a_col)))
        return set_error(LRSDP_EINVAL, "input arrays are NULL");
    std::vector<int64_t> off(nblocks + 1, 0);
    for (int64_t j = 0; j < nblocks; ++j) {
        if (block_n[j] < 1) return set_error(LRSDP_EINVAL, "block %lld has order %lld", (long long)j,
                                             (long long)block_n[j]);
        off[j + 1] = off[j] + block_n[j];
        if (off[j + 1] > INT32_MAX - 1) return set_error(LRSDP_EINVAL, "total order too large");
    }
    auto place = [&](int64_t cnt, const int32_t *blk, const int32_t *r, const int32_t *c, std::vector<int32_t> &gr,
                     std::vector<int32_t> &gc, const char *what) -> int {
        gr.resize(cnt);
        gc.resize(cnt);
        for (int64_t t = 0; t < cnt; ++t) {
            const int32_t j = blk[t];
            if (j < 0 || j >= nblocks)
                return set_error(LRSDP_EINVAL, "%s entry %lld names block %d", what, (long long)t, j);
            if (r[t] < 0 || r[t] >= block_n[j] || c[t] < 0 || c[t] >= block_n[j])
                return set_error(LRSDP_EINVAL, "%s entry %lld = (%d, %d) outside block %d", what, (long long)t, r[t],
                                 c[t], j);
            gr[t] = (int32_t)(off[j] + r[t]);
            gc[t] = (int32_t)(off[j] + c[t]);
        }
        return LRSDP_OK;
    };
    std::vector<int32_t> cr, cc, ar, ac;
    int rc;
    if ((rc = place(c_nnz, c_blk, c_row, c_col, cr, cc, "C"))) return rc;
    if ((rc = place(a_nnz, a_blk, a_row, a_col, ar, ac, "A"))) return rc;
    rc = lrsdp_problem_general(off[nblocks], c_nnz, cr.data(), cc.data(), c_val, m, a_nnz, a_con, ar.data(),
                               ac.data(), a_val, b, out);
    if (rc == LRSDP_OK) (*out)->block_off = off;
    return rc;
}

extern "C" int lrsdp_problem_block_ranks(lrsdp_problem *p, const int32_t *block_rank) {
    clear_error();
    if (!p || !block_rank) return set_error(LRSDP_EINVAL, "NULL argument");
    if (p->info.kind != LRSDP_GENERAL)
        return set_error(LRSDP_EUNSUPPORTED, "block ranks apply to general problems");
    if (p->uploaded) return set_error(LRSDP_EINVAL, "set the block ranks before the upload");
    std::vector<int64_t> off = p->block_off;
    if (off.empty()) off = {0, p->info.n};   // lrsdp_problem_general: one block
    const int64_t nb = (int64_t)off.size() - 1;
    for (int64_t j = 0; j < nb; ++j)
        if (block_rank[j] < 1)
            return set_error(LRSDP_EINVAL, "block %lld has rank %d", (long long)j, block_rank[j]);
    p->row_rank.resize(p->info.n);
    for (int64_t j = 0; j < nb; ++j)
        for (int64_t i = off[j]; i < off[j + 1]; ++i) p->row_rank[i] = block_rank[j];
    return LRSDP_OK;
}

namespace {

struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = (off + 255) & ~size_t(255);
        off = o + bytes;
        return o;
    }
};

// Fills offsets for every device array of the problem; returns total bytes.
size_t plan_device(const lrsdp_problem *p, size_t *offs) {
    Layout L;
    int k = 0;
    auto add = [&](size_t bytes) { offs[k++] = L.take(bytes); };
    if (p->info.kind == LRSDP_MAXCUT) {
        add(p->row_ptr.size() * 4);
        add(p->col.size() * 4);
        add(p->val.size() * 8);
        add(p->diag.size() * 8);
        add(p->light.size() * sizeof(int4));
        add(p->seg.size() * sizeof(int4));
        add(p->heavy.size() * 4);
        add(p->heavy_seg.size() * 4);
        add(p->seg.size() * 256);      // segment partial sums (<= 256 B per row)
        add(p->hrow.size() * 8);
        add(p->perm.size() * 4);
    } else if (p->info.kind == LRSDP_GENERAL) {
        add(p->om_a.size() * 4);
        add(p->om_b.size() * 4);
        add(p->cval.size() * 8);
        add(p->a_ptr.size() * 4);
        add(p->a_idx.size() * 4);
        add(p->a_val.size() * 8);
        add(p->at_ptr.size() * 4);
        add(p->at_idx.size() * 4);
        add(p->at_val.size() * 8);
        add(p->s_ptr.size() * 4);
        add(p->s_col.size() * 4);
        add(p->s_om.size() * 4);
        add(p->b.size() * 8);
        add(p->om_a.size() * 8);       // compressed outer products (two per position)
        add(p->om_a.size() * 8);
        add(p->con_short.size() * 4);
        add(p->con_long.size() * 4);
        add(p->cdense.size() * 8);                                      // dense C
        add(p->cdense.empty() ? 0 : (size_t)p->info.n * kDenseRowBytes);  // dense product, one row per node
        add(p->cdense.empty() ? 0 : (size_t)kDenseMaxSplit * p->info.n * kDenseRowBytes);  // split-k partials
        add(p->row_rank.size() * 4);                                     // per-row rank (block ranks)
    } else {
        add(p->top_ptr.size() * 4);
        add(p->top_col.size() * 4);
        add(p->top_eid.size() * 4);
        add(p->bot_ptr.size() * 4);
        add(p->bot_row.size() * 4);
        add(p->bot_eid.size() * 4);
        add(p->samp_i.size() * 4);
        add(p->samp_j.size() * 4);
        add(p->b.size() * 8);
    }
    return L.off + 256;
}

}  // namespace

extern "C" int lrsdp_problem_device_bytes(const lrsdp_problem *prob, size_t *bytes) {
    clear_error();
    if (!prob || !bytes) return set_error(LRSDP_EINVAL, "NULL argument");
    size_t offs[24];
    *bytes = plan_device(prob, offs);
    return LRSDP_OK;
}

extern "C" int lrsdp_problem_upload(lrsdp_ctx *ctx, lrsdp_problem *p, void *dev, size_t bytes) {
    clear_error();
    if (!ctx || !p || !dev) return set_error(LRSDP_EINVAL, "NULL argument");
    size_t offs[24];
    size_t need = plan_device(p, offs);
    if (bytes < need)
        return set_error(LRSDP_ENOMEM, "problem needs %zu device bytes, %zu given", need, bytes);
    LRSDP_HIP_TRY(hipSetDevice(ctx->device));
    char *base = static_cast<char *>(dev);
    auto put = [&](size_t off, const void *src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, ctx->stream);
    };
    if (p->info.kind == LRSDP_MAXCUT) {
        LRSDP_HIP_TRY(put(offs[0], p->row_ptr.data(), p->row_ptr.size() * 4));
        LRSDP_HIP_TRY(put(offs[1], p->col.data(), p->col.size() * 4));
        LRSDP_HIP_TRY(put(offs[2], p->val.data(), p->val.size() * 8));
        LRSDP_HIP_TRY(put(offs[3], p->diag.data(), p->diag.size() * 8));
        LRSDP_HIP_TRY(put(offs[4], p->light.data(), p->light.size() * sizeof(int4)));
        LRSDP_HIP_TRY(put(offs[5], p->seg.data(), p->seg.size() * sizeof(int4)));
        LRSDP_HIP_TRY(put(offs[6], p->heavy.data(), p->heavy.size() * 4));
        LRSDP_HIP_TRY(put(offs[7], p->heavy_seg.data(), p->heavy_seg.size() * 4));
        LRSDP_HIP_TRY(put(offs[9], p->hrow.data(), p->hrow.size() * 8));
        LRSDP_HIP_TRY(put(offs[10], p->perm.data(), p->perm.size() * 4));
        DevCsr &c = p->csr;
        c.row_ptr = (const int32_t *)(base + offs[0]);
        c.col = (const int32_t *)(base + offs[1]);
        c.val = p->val.empty() ? nullptr : (const double *)(base + offs[2]);
        c.diag = (const double *)(base + offs[3]);
        c.light = (const int4 *)(base + offs[4]);
        c.seg = (const int4 *)(base + offs[5]);
        c.heavy = (const int32_t *)(base + offs[6]);
        c.heavy_seg = (const int32_t *)(base + offs[7]);
        c.seg_buf = base + offs[8];
        c.hrow = (const double *)(base + offs[9]);
        c.perm = p->perm.empty() ? nullptr : (const int32_t *)(base + offs[10]);
        c.n = p->info.n;
        c.nnz = p->info.nnz;
        c.n_light = (int64_t)p->light.size();
        c.n_seg = (int64_t)p->seg.size();
        c.n_heavy = (int64_t)p->heavy.size();
        c.wmode = p->info.weights;
    } else if (p->info.kind == LRSDP_GENERAL) {
        LRSDP_HIP_TRY(put(offs[0], p->om_a.data(), p->om_a.size() * 4));
        LRSDP_HIP_TRY(put(offs[1], p->om_b.data(), p->om_b.size() * 4));
        LRSDP_HIP_TRY(put(offs[2], p->cval.data(), p->cval.size() * 8));
        LRSDP_HIP_TRY(put(offs[3], p->a_ptr.data(), p->a_ptr.size() * 4));
        LRSDP_HIP_TRY(put(offs[4], p->a_idx.data(), p->a_idx.size() * 4));
        LRSDP_HIP_TRY(put(offs[5], p->a_val.data(), p->a_val.size() * 8));
        LRSDP_HIP_TRY(put(offs[6], p->at_ptr.data(), p->at_ptr.size() * 4));
        LRSDP_HIP_TRY(put(offs[7], p->at_idx.data(), p->at_idx.size() * 4));
        LRSDP_HIP_TRY(put(offs[8], p->at_val.data(), p->at_val.size() * 8));
        LRSDP_HIP_TRY(put(offs[9], p->s_ptr.data(), p->s_ptr.size() * 4));
        LRSDP_HIP_TRY(put(offs[10], p->s_col.data(), p->s_col.size() * 4));
        LRSDP_HIP_TRY(put(offs[11], p->s_om.data(), p->s_om.size() * 4));
        LRSDP_HIP_TRY(put(offs[12], p->b.data(), p->b.size() * 8));
        DevGeneral &g = p->gen;
        g.om_a = (const int32_t *)(base + offs[0]);
        g.om_b = (const int32_t *)(base + offs[1]);
        g.cval = (const double *)(base + offs[2]);
        g.a_ptr = (const int32_t *)(base + offs[3]);
        g.a_idx = (const int32_t *)(base + offs[4]);
        g.a_val = (const double *)(base + offs[5]);
        g.at_ptr = (const int32_t *)(base + offs[6]);
        g.at_idx = (const int32_t *)(base + offs[7]);
        g.at_val = (const double *)(base + offs[8]);
        g.s_ptr = (const int32_t *)(base + offs[9]);
        g.s_col = (const int32_t *)(base + offs[10]);
        g.s_om = (const int32_t *)(base + offs[11]);
        g.b = (const double *)(base + offs[12]);
        g.x1 = (double *)(base + offs[13]);
        g.x2 = (double *)(base + offs[14]);
        LRSDP_HIP_TRY(put(offs[15], p->con_short.data(), p->con_short.size() * 4));
        LRSDP_HIP_TRY(put(offs[16], p->con_long.data(), p->con_long.size() * 4));
        g.con_short = (const int32_t *)(base + offs[15]);
        g.con_long = (const int32_t *)(base + offs[16]);
        LRSDP_HIP_TRY(put(offs[17], p->cdense.data(), p->cdense.size() * 8));
        g.cd = p->cdense.empty() ? nullptr : (const double *)(base + offs[17]);
        g.dw = p->cdense.empty() ? nullptr : (double *)(base + offs[18]);
        g.dpart = p->cdense.empty() ? nullptr : (double *)(base + offs[19]);
        LRSDP_HIP_TRY(put(offs[20], p->row_rank.data(), p->row_rank.size() * 4));
        g.row_rank = p->row_rank.empty() ? nullptr : (const int32_t *)(base + offs[20]);
        g.n_short = (int64_t)p->con_short.size();
        g.n_long = (int64_t)p->con_long.size();
        g.n = p->info.n;
        g.m = p->info.m;
        g.nom = (int64_t)p->om_a.size();
        g.nnz_a = (int64_t)p->a_idx.size();
        g.nnz_s = (int64_t)p->s_col.size();
    } else {
        LRSDP_HIP_TRY(put(offs[0], p->top_ptr.data(), p->top_ptr.size() * 4));
        LRSDP_HIP_TRY(put(offs[1], p->top_col.data(), p->top_col.size() * 4));
        LRSDP_HIP_TRY(put(offs[2], p->top_eid.data(), p->top_eid.size() * 4));
        LRSDP_HIP_TRY(put(offs[3], p->bot_ptr.data(), p->bot_ptr.size() * 4));
        LRSDP_HIP_TRY(put(offs[4], p->bot_row.data(), p->bot_row.size() * 4));
        LRSDP_HIP_TRY(put(offs[5], p->bot_eid.data(), p->bot_eid.size() * 4));
        LRSDP_HIP_TRY(put(offs[6], p->samp_i.data(), p->samp_i.size() * 4));
        LRSDP_HIP_TRY(put(offs[7], p->samp_j.data(), p->samp_j.size() * 4));
        LRSDP_HIP_TRY(put(offs[8], p->b.data(), p->b.size() * 8));
        DevCompletion &c = p->cmp;
        c.top_ptr = (const int32_t *)(base + offs[0]);
        c.top_col = (const int32_t *)(base + offs[1]);
        c.top_eid = (const int32_t *)(base + offs[2]);
        c.bot_ptr = (const int32_t *)(base + offs[3]);
        c.bot_row = (const int32_t *)(base + offs[4]);
        c.bot_eid = (const int32_t *)(base + offs[5]);
        c.samp_i = (const int32_t *)(base + offs[6]);
        c.samp_j = (const int32_t *)(base + offs[7]);
        c.b = (const double *)(base + offs[8]);
        c.n1 = p->info.n1;
        c.n2 = p->info.n2;
        c.m = p->info.m;
    }
    LRSDP_HIP_TRY(hipStreamSynchronize(ctx->stream));
    p->dev = dev;
    p->dev_bytes = bytes;
    p->uploaded = true;
    return LRSDP_OK;
}
