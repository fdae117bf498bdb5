// Host: SP2 of the whole matrix in numerically thresholded sparse algebra,
// the standard scheme that gives the initial density matrix before any
// graph or partition exists (Fig. 1 description in the Introduction: the
// first P comes from thresholded sparse SP2; the threshold is the same kind
// of parameter as the graph's tau, Methods, "Graph Theory").
//
// The steps are those of the dense run: Gershgorin bounds of H, eq. (1),
// then per product Y = X X, e = Tr X - Tr Y, the stop rule, the trace rule
// for the branch and eq. (2); every iterate (X0 included) keeps only the
// entries with |x| > eps.  The products are sparse-sparse (Gustavson: row i
// of Y accumulates x_ik times row k of X in a dense per-thread accumulator,
// k in ascending order, so every entry's sum has a fixed order and the
// result does not depend on the number of threads).  Rows are split over
// host threads.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <thread>
#include <vector>

#include "gsp2_internal.hpp"

namespace gsp2 {

namespace {

struct Csr {
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

// Run f(first_row, last_row, thread) over contiguous row ranges.
template <typename F>
void parallel_rows(int32_t n, int n_threads, F &&f) {
    if (n_threads <= 1 || n < 2 * n_threads) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < n_threads; ++t) {
        const int32_t a = (int32_t)((int64_t)n * t / n_threads), b = (int32_t)((int64_t)n * (t + 1) / n_threads);
        th.emplace_back([&, a, b, t] { f(a, b, t); });
    }
    for (auto &x : th) x.join();
}

// Assemble per-row entry lists (already sorted by column) into CSR.
Csr assemble(int32_t n, const std::vector<std::vector<int32_t>> &rc, const std::vector<std::vector<double>> &rv) {
    Csr m;
    m.ptr.assign((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) m.ptr[i + 1] = m.ptr[i] + (int64_t)rc[i].size();
    m.col.resize((size_t)m.ptr[n]);
    m.val.resize((size_t)m.ptr[n]);
    for (int32_t i = 0; i < n; ++i) {
        std::copy(rc[i].begin(), rc[i].end(), m.col.begin() + m.ptr[i]);
        std::copy(rv[i].begin(), rv[i].end(), m.val.begin() + m.ptr[i]);
    }
    return m;
}

double trace(const Csr &m, int32_t n) {
    double t = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = m.ptr[i]; e < m.ptr[i + 1]; ++e)
            if (m.col[e] == i) t += m.val[e];
    return t;
}

}  // namespace

SparseSP2Result sparse_sp2(int32_t n, const int64_t *rp, const int32_t *ci, const double *hv, double n_occ,
                           double eps, int32_t max_iter, double trace_tol, int n_threads) {
    SparseSP2Result r;
    // Gershgorin bounds of H (Methods, SP2 section)
    double emin = INFINITY, emax = -INFINITY;
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0, rad = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] == i) d += hv[e];
            else rad += std::fabs(hv[e]);
        }
        emin = std::min(emin, d - rad);
        emax = std::max(emax, d + rad);
    }
    r.eps_min = emin;
    r.eps_max = emax;
    const double D = emax - emin;
    // eq. (1), thresholded: row i holds (emax delta_ij - H_ij) / D for j in H's row and i
    std::vector<std::vector<int32_t>> rc(n);
    std::vector<std::vector<double>> rv(n);
    parallel_rows(n, n_threads, [&](int32_t a, int32_t b, int) {
        std::vector<std::pair<int32_t, double>> row;
        for (int32_t i = a; i < b; ++i) {
            row.clear();
            bool diag = false;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                if (ci[e] == i) diag = true;
                row.emplace_back(ci[e], ((ci[e] == i ? emax : 0.0) - hv[e]) / D);
            }
            if (!diag) row.emplace_back(i, emax / D);
            std::sort(row.begin(), row.end());
            for (const auto &p : row)
                if (std::fabs(p.second) > eps) {
                    rc[i].push_back(p.first);
                    rv[i].push_back(p.second);
                }
        }
    });
    Csr X = assemble(n, rc, rv);
    double tr = trace(X, n);
    std::vector<double> errors;
    const double floor = std::max(1.0, n * 0x1p-53);
    r.status = GSP2_E_NOT_CONVERGED;
    for (int32_t t = 0; t < max_iter; ++t) {
        // Y = X X, row by row; then the stop test, the branch and eq. (2)
        std::vector<std::vector<int32_t>> yc(n);
        std::vector<std::vector<double>> yv(n);
        std::vector<double> row_diag(n, 0.0);
        parallel_rows(n, n_threads, [&](int32_t a, int32_t b, int) {
            std::vector<double> acc(n, 0.0);
            std::vector<char> seen(n, 0);
            std::vector<int32_t> cols;
            for (int32_t i = a; i < b; ++i) {
                cols.clear();
                for (int64_t e = X.ptr[i]; e < X.ptr[i + 1]; ++e) {
                    const int32_t k = X.col[e];
                    const double x = X.val[e];
                    for (int64_t f = X.ptr[k]; f < X.ptr[k + 1]; ++f) {
                        const int32_t j = X.col[f];
                        if (!seen[j]) { seen[j] = 1; cols.push_back(j); }
                        acc[j] += x * X.val[f];
                    }
                }
                std::sort(cols.begin(), cols.end());
                yc[i] = cols;
                yv[i].resize(cols.size());
                for (size_t q = 0; q < cols.size(); ++q) {
                    yv[i][q] = acc[cols[q]];
                    if (cols[q] == i) row_diag[i] = acc[cols[q]];
                    acc[cols[q]] = 0.0;
                    seen[cols[q]] = 0;
                }
            }
        });
        double trY = 0.0;
        for (int32_t i = 0; i < n; ++i) trY += row_diag[i];
        const double e = tr - trY;
        errors.push_back(e);
        r.n_products = t + 1;
        if (!std::isfinite(e)) break;
        if (t >= 2 && std::fabs(e) >= std::fabs(errors[t - 2]) && std::fabs(errors[t - 2]) < floor) {
            r.status = std::fabs(tr - n_occ) <= trace_tol ? GSP2_OK : GSP2_E_WRONG_TRACE;
            r.idempotency = e;
            break;
        }
        const int alpha = tr <= n_occ ? 1 : -1;
        r.alphas.push_back((int8_t)alpha);
        // eq. (2): X' = X + alpha (X - Y), merged row by row, thresholded
        std::vector<std::vector<int32_t>> nc(n);
        std::vector<std::vector<double>> nv(n);
        parallel_rows(n, n_threads, [&](int32_t a, int32_t b, int) {
            for (int32_t i = a; i < b; ++i) {
                int64_t p = X.ptr[i];
                size_t q = 0;
                const int64_t pe = X.ptr[i + 1];
                const size_t qe = yc[i].size();
                while (p < pe || q < qe) {
                    int32_t j;
                    double x = 0.0, y = 0.0;
                    if (q >= qe || (p < pe && X.col[p] < yc[i][q])) {
                        j = X.col[p]; x = X.val[p]; ++p;
                    } else if (p >= pe || yc[i][q] < X.col[p]) {
                        j = yc[i][q]; y = yv[i][q]; ++q;
                    } else {
                        j = X.col[p]; x = X.val[p]; y = yv[i][q]; ++p; ++q;
                    }
                    const double v = x + alpha * (x - y);
                    if (std::fabs(v) > eps) {
                        nc[i].push_back(j);
                        nv[i].push_back(v);
                    }
                }
            }
        });
        X = assemble(n, nc, nv);
        tr = trace(X, n);
    }
    r.trace = tr;
    if (r.status == GSP2_E_NOT_CONVERGED) r.idempotency = errors.empty() ? NAN : errors.back();
    r.ptr = std::move(X.ptr);
    r.col = std::move(X.col);
    r.val = std::move(X.val);
    return r;
}

}  // namespace gsp2
