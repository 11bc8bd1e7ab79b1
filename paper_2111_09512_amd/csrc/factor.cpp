// Host-side incomplete LU factorizations (set-up for the scaled-ILU smoother).
//
// ILU(k) (symbolic level-of-fill phase + numeric phase, Section 3.1) and
// ILUT(tau, p) (threshold + fill-per-row, Sections 4.2 and 6.1), both without
// pivoting.  The row being eliminated lives in a dense work row indexed by
// column with a touched list; the lower columns still to be eliminated are
// kept in a min-heap, so fill created while eliminating column k (always at
// columns > k) is visited in increasing order.  Row sums are formed in
// ascending column order and every update is w_j <- w_j - l_ik * u_kj, so the
// factors do not depend on the data structures used here.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <queue>
#include <vector>

#include "../../include/scaled_ilu.h"
#include "../../include/silu_factor.h"

namespace {

using idx_t = int32_t;

// A factor under construction: rows appended in order.
struct Growing {
    std::vector<idx_t> rp{0};
    std::vector<idx_t> col;
    std::vector<double> val;
    std::vector<uint16_t> lev;  // level of fill (ILU(k) symbolic phase only)
};

int export_csr(int64_t n, Growing &g, silu_host_csr *out)
{
    out->n = n;
    out->nnz = (int64_t)g.col.size();
    size_t nn = (size_t)n + 1, nz = g.col.size() ? g.col.size() : 1;
    out->row_ptr = (int32_t *)std::malloc(nn * sizeof(int32_t));
    out->col_idx = (int32_t *)std::malloc(nz * sizeof(int32_t));
    out->val = (double *)std::malloc(nz * sizeof(double));
    if (!out->row_ptr || !out->col_idx || !out->val) {
        silu_host_csr_free(out);
        return SILU_ERR_NOMEM;
    }
    std::memcpy(out->row_ptr, g.rp.data(), nn * sizeof(int32_t));
    if (!g.col.empty()) {
        std::memcpy(out->col_idx, g.col.data(), g.col.size() * sizeof(int32_t));
        std::memcpy(out->val, g.val.data(), g.val.size() * sizeof(double));
    }
    return SILU_OK;
}

int check_input(const silu_host_csr *A)
{
    if (!A || !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)) || A->n < 0 || A->n >= INT32_MAX)
        return SILU_ERR_ARG;
    if (A->row_ptr[0] != 0 || A->row_ptr[A->n] != A->nnz) return SILU_ERR_PATTERN;
    for (int64_t i = 0; i < A->n; i++) {
        if (A->row_ptr[i + 1] < A->row_ptr[i]) return SILU_ERR_PATTERN;
        for (int32_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; p++) {
            if (A->col_idx[p] < 0 || A->col_idx[p] >= A->n) return SILU_ERR_PATTERN;
            if (p > A->row_ptr[i] && A->col_idx[p] <= A->col_idx[p - 1]) return SILU_ERR_PATTERN;
        }
    }
    return SILU_OK;
}

using MinHeap = std::priority_queue<idx_t, std::vector<idx_t>, std::greater<idx_t>>;

int iluk_impl(const silu_host_csr *A, int K, silu_host_csr *Lout, silu_host_csr *Uout, int64_t *bad_row)
{
    const idx_t n = (idx_t)A->n;
    const uint16_t ABSENT = 0xFFFF;
    if (K < 0 || K > 0xFFFE) return SILU_ERR_ARG;
    Growing L, U;
    L.rp.reserve((size_t)n + 1);
    U.rp.reserve((size_t)n + 1);
    std::vector<uint16_t> lev((size_t)n, ABSENT);
    std::vector<idx_t> touched;
    touched.reserve(256);
    MinHeap pend;

    // ---- symbolic phase: the level-k pattern, row by row ----
    for (idx_t i = 0; i < n; i++) {
        touched.clear();
        bool diag = false;
        for (int32_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; p++) {
            idx_t j = A->col_idx[p];
            lev[j] = 0;
            touched.push_back(j);
            if (j < i) pend.push(j);
            diag |= (j == i);
        }
        if (!diag) {
            if (bad_row) *bad_row = i;
            return SILU_ERR_PATTERN;
        }
        while (!pend.empty()) {
            idx_t k = pend.top();
            pend.pop();
            const unsigned lk = lev[k];
            for (int32_t q = U.rp[k] + 1; q < U.rp[k + 1]; q++) {  // strictly upper part of row k
                const unsigned nl = lk + U.lev[q] + 1u;
                if (nl > (unsigned)K) continue;
                idx_t j = U.col[q];
                if (lev[j] == ABSENT) {
                    touched.push_back(j);
                    if (j < i) pend.push(j);
                    lev[j] = (uint16_t)nl;
                } else if (nl < lev[j]) {
                    lev[j] = (uint16_t)nl;
                }
            }
        }
        std::sort(touched.begin(), touched.end());
        for (idx_t j : touched) {
            Growing &g = j < i ? L : U;
            g.col.push_back(j);
            g.lev.push_back(lev[j]);
            lev[j] = ABSENT;
        }
        L.rp.push_back((idx_t)L.col.size());
        U.rp.push_back((idx_t)U.col.size());
    }
    U.lev.clear();
    U.lev.shrink_to_fit();
    L.lev.clear();
    L.lev.shrink_to_fit();
    L.val.assign(L.col.size(), 0.0);
    U.val.assign(U.col.size(), 0.0);

    // ---- numeric phase on the fixed pattern ----
    std::vector<double> w((size_t)n, 0.0);
    std::vector<uint8_t> inpat((size_t)n, 0);
    for (idx_t i = 0; i < n; i++) {
        for (int32_t p = L.rp[i]; p < L.rp[i + 1]; p++) inpat[L.col[p]] = 1;
        for (int32_t p = U.rp[i]; p < U.rp[i + 1]; p++) inpat[U.col[p]] = 1;
        for (int32_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; p++) w[A->col_idx[p]] = A->val[p];
        for (int32_t p = L.rp[i]; p < L.rp[i + 1]; p++) {
            const idx_t k = L.col[p];
            const double lik = w[k] / U.val[U.rp[k]];
            w[k] = lik;
            for (int32_t q = U.rp[k] + 1; q < U.rp[k + 1]; q++) {
                const idx_t j = U.col[q];
                if (inpat[j]) w[j] = w[j] - lik * U.val[q];
            }
        }
        for (int32_t p = L.rp[i]; p < L.rp[i + 1]; p++) {
            L.val[p] = w[L.col[p]];
            w[L.col[p]] = 0.0;
            inpat[L.col[p]] = 0;
        }
        for (int32_t p = U.rp[i]; p < U.rp[i + 1]; p++) {
            U.val[p] = w[U.col[p]];
            w[U.col[p]] = 0.0;
            inpat[U.col[p]] = 0;
        }
        const double piv = U.val[U.rp[i]];
        if (!(piv != 0.0) || !std::isfinite(piv)) {
            if (bad_row) *bad_row = i;
            return SILU_ERR_ZERO_PIVOT;
        }
    }
    int st = export_csr(n, L, Lout);
    if (st) return st;
    st = export_csr(n, U, Uout);
    if (st) silu_host_csr_free(Lout);
    return st;
}

struct Cand {
    double key;
    idx_t col;
};
// total order: larger magnitude first, then smaller column
inline bool cand_before(const Cand &a, const Cand &b) { return a.key > b.key || (a.key == b.key && a.col < b.col); }

int ilut_impl(const silu_host_csr *A, double tau, int p, silu_host_csr *Lout, silu_host_csr *Uout,
              int64_t *bad_row)
{
    const idx_t n = (idx_t)A->n;
    if (p < 0 || !(tau >= 0.0)) return SILU_ERR_ARG;
    Growing L, U;
    L.rp.reserve((size_t)n + 1);
    U.rp.reserve((size_t)n + 1);
    L.col.reserve((size_t)n * std::min(p, 32));
    L.val.reserve((size_t)n * std::min(p, 32));
    U.col.reserve((size_t)n * (std::min(p, 32) + 1));
    U.val.reserve((size_t)n * (std::min(p, 32) + 1));
    std::vector<double> w((size_t)n, 0.0), before((size_t)n, 0.0);
    // state of a column in the current row: 0 absent, 1 present, 2 dropped lower entry
    std::vector<uint8_t> state((size_t)n, 0);
    std::vector<idx_t> touched, lower;
    std::vector<Cand> cand;
    MinHeap pend;

    for (idx_t i = 0; i < n; i++) {
        touched.clear();
        lower.clear();
        double nrm2 = 0.0;
        for (int32_t q = A->row_ptr[i]; q < A->row_ptr[i + 1]; q++) {
            const idx_t j = A->col_idx[q];
            const double a = A->val[q];
            w[j] = a;
            state[j] = 1;
            touched.push_back(j);
            if (j < i) pend.push(j);
            nrm2 = nrm2 + a * a;
        }
        const double tau_i = tau * std::sqrt(nrm2);
        if (!state[i]) {
            w[i] = 0.0;
            state[i] = 1;
            touched.push_back(i);
        }
        while (!pend.empty()) {
            const idx_t k = pend.top();
            pend.pop();
            const double v = w[k];
            if (std::fabs(v) < tau_i) {  // dropped: no elimination with row k
                w[k] = 0.0;
                state[k] = 2;
                continue;
            }
            const double lik = v / U.val[U.rp[k]];
            w[k] = lik;
            before[k] = v;
            lower.push_back(k);
            for (int32_t q = U.rp[k] + 1; q < U.rp[k + 1]; q++) {
                const idx_t j = U.col[q];
                if (!state[j]) {
                    state[j] = 1;
                    w[j] = 0.0;
                    touched.push_back(j);
                    if (j < i) pend.push(j);
                }
                w[j] = w[j] - lik * U.val[q];
            }
        }
        // L part: `lower` is already ascending (heap order)
        cand.clear();
        for (idx_t k : lower) cand.push_back({std::fabs(before[k]), k});
        if ((int)cand.size() > p) {
            std::nth_element(cand.begin(), cand.begin() + p, cand.end(), cand_before);
            cand.resize((size_t)p);
        }
        std::sort(cand.begin(), cand.end(), [](const Cand &a, const Cand &b) { return a.col < b.col; });
        for (const Cand &c : cand) {
            L.col.push_back(c.col);
            L.val.push_back(w[c.col]);
        }
        L.rp.push_back((idx_t)L.col.size());
        // U part: diagonal first, then the kept off-diagonal entries
        const double piv = w[i];
        if (!(piv != 0.0) || !std::isfinite(piv)) {
            if (bad_row) *bad_row = i;
            return SILU_ERR_ZERO_PIVOT;
        }
        cand.clear();
        for (idx_t j : touched)
            if (j > i && std::fabs(w[j]) >= tau_i) cand.push_back({std::fabs(w[j]), j});
        if ((int)cand.size() > p) {
            std::nth_element(cand.begin(), cand.begin() + p, cand.end(), cand_before);
            cand.resize((size_t)p);
        }
        std::sort(cand.begin(), cand.end(), [](const Cand &a, const Cand &b) { return a.col < b.col; });
        U.col.push_back(i);
        U.val.push_back(piv);
        for (const Cand &c : cand) {
            U.col.push_back(c.col);
            U.val.push_back(w[c.col]);
        }
        U.rp.push_back((idx_t)U.col.size());
        for (idx_t j : touched) {
            w[j] = 0.0;
            state[j] = 0;
        }
    }
    int st = export_csr(n, L, Lout);
    if (st) return st;
    st = export_csr(n, U, Uout);
    if (st) silu_host_csr_free(Lout);
    return st;
}

}  // namespace

extern "C" {

int silu_factor_iluk(const silu_host_csr *A, int k, silu_host_csr *L, silu_host_csr *U, int64_t *bad_row)
{
    if (bad_row) *bad_row = -1;
    if (!L || !U) return SILU_ERR_ARG;
    std::memset(L, 0, sizeof(*L));
    std::memset(U, 0, sizeof(*U));
    int st = check_input(A);
    if (st) return st;
    try {
        return iluk_impl(A, k, L, U, bad_row);
    } catch (const std::bad_alloc &) {
        return SILU_ERR_NOMEM;
    }
}

int silu_factor_ilut(const silu_host_csr *A, double tau, int p, silu_host_csr *L, silu_host_csr *U,
                     int64_t *bad_row)
{
    if (bad_row) *bad_row = -1;
    if (!L || !U) return SILU_ERR_ARG;
    std::memset(L, 0, sizeof(*L));
    std::memset(U, 0, sizeof(*U));
    int st = check_input(A);
    if (st) return st;
    try {
        return ilut_impl(A, tau, p, L, U, bad_row);
    } catch (const std::bad_alloc &) {
        return SILU_ERR_NOMEM;
    }
}

void silu_host_csr_free(silu_host_csr *m)
{
    if (!m) return;
    std::free(m->row_ptr);
    std::free(m->col_idx);
    std::free(m->val);
    m->row_ptr = nullptr;
    m->col_idx = nullptr;
    m->val = nullptr;
    m->nnz = 0;
}

}  // extern "C"
