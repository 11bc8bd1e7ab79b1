// Host-code driver for the sanitizer build: the library's host-side set-up
// (ILU(k) and ILUT factorizations, the reverse Cuthill-McKee locality order)
// linked on its own with AddressSanitizer and UndefinedBehaviorSanitizer, run
// over valid inputs of several shapes and over every rejected input.  Prints
// one line per case and exits non-zero on the first failed check; the
// sanitizers abort on the first memory or undefined-behaviour error (and
// report leaks at exit).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../include/scaled_ilu.h"
#include "../include/silu_factor.h"

namespace {

struct Csr {
    int64_t n = 0;
    std::vector<int32_t> rp{0}, col;
    std::vector<double> val;
    silu_host_csr view()
    {
        silu_host_csr h;
        h.n = n;
        h.nnz = (int64_t)col.size();
        h.row_ptr = rp.data();
        h.col_idx = col.data();
        h.val = val.data();
        return h;
    }
};

int failures = 0;

void check(bool ok, const char *what, const char *name)
{
    if (!ok) {
        std::printf("FAIL %s: %s\n", name, what);
        failures++;
    }
}

// 7-point Laplacian on an N^3 grid, Dirichlet (out-of-grid neighbours dropped).
Csr poisson7(int N)
{
    Csr A;
    A.n = (int64_t)N * N * N;
    for (int z = 0; z < N; z++)
        for (int y = 0; y < N; y++)
            for (int x = 0; x < N; x++) {
                const int i = x + N * (y + N * z);
                const int off[7][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
                for (auto &o : off) {
                    const int xx = x + o[0], yy = y + o[1], zz = z + o[2];
                    if (xx < 0 || yy < 0 || zz < 0 || xx >= N || yy >= N || zz >= N) continue;
                    const int j = xx + N * (yy + N * zz);
                    A.col.push_back(j);
                    A.val.push_back(i == j ? 6.0 : -1.0);
                }
                A.rp.push_back((int32_t)A.col.size());
            }
    return A;
}

// Random symmetric, strictly diagonally dominant sparse matrix; some rows
// hold only their diagonal.
Csr random_dd(int n, double density, unsigned seed)
{
    std::mt19937 g(seed);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::vector<std::vector<std::pair<int, double>>> rows((size_t)n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < i; j++)
            if (u(g) < density) {
                const double v = -u(g);
                rows[(size_t)i].push_back({j, v});
                rows[(size_t)j].push_back({i, v});
            }
    Csr A;
    A.n = n;
    for (int i = 0; i < n; i++) {
        double s = 1.0;
        for (auto &e : rows[(size_t)i]) s += std::fabs(e.second);
        rows[(size_t)i].push_back({i, s});
        std::sort(rows[(size_t)i].begin(), rows[(size_t)i].end());
        for (auto &e : rows[(size_t)i]) {
            A.col.push_back(e.first);
            A.val.push_back(e.second);
        }
        A.rp.push_back((int32_t)A.col.size());
    }
    return A;
}

// L strictly lower with sorted columns; U starts every row with its diagonal,
// then strictly upper sorted columns; every value finite.
void check_factors(const silu_host_csr &L, const silu_host_csr &U, int64_t n, int p, const char *name)
{
    check(L.n == n && U.n == n, "factor sizes", name);
    check(L.row_ptr[0] == 0 && U.row_ptr[0] == 0, "row_ptr[0]", name);
    check(L.row_ptr[n] == L.nnz && U.row_ptr[n] == U.nnz, "nnz", name);
    for (int64_t i = 0; i < n; i++) {
        for (int32_t e = L.row_ptr[i]; e < L.row_ptr[i + 1]; e++) {
            check(L.col_idx[e] < i && L.col_idx[e] >= 0, "L not strictly lower", name);
            if (e > L.row_ptr[i]) check(L.col_idx[e] > L.col_idx[e - 1], "L columns unsorted", name);
            check(std::isfinite(L.val[e]), "L value not finite", name);
        }
        check(U.row_ptr[i + 1] > U.row_ptr[i] && U.col_idx[U.row_ptr[i]] == i, "U row without leading diagonal",
              name);
        for (int32_t e = U.row_ptr[i] + 1; e < U.row_ptr[i + 1]; e++) {
            check(U.col_idx[e] > i && U.col_idx[e] < n, "U not strictly upper", name);
            if (e > U.row_ptr[i] + 1) check(U.col_idx[e] > U.col_idx[e - 1], "U columns unsorted", name);
            check(std::isfinite(U.val[e]), "U value not finite", name);
        }
        if (p > 0) {
            check(L.row_ptr[i + 1] - L.row_ptr[i] <= p, "ILUT L row over p", name);
            check(U.row_ptr[i + 1] - U.row_ptr[i] - 1 <= p, "ILUT U row over p", name);
        }
    }
}

// ILU(0): (L U)_ij = a_ij on the pattern of A (dense product; small n only).
void check_ilu0_characterization(Csr &A, const silu_host_csr &L, const silu_host_csr &U, const char *name)
{
    const int64_t n = A.n;
    std::vector<double> Ld((size_t)(n * n), 0.0), Ud((size_t)(n * n), 0.0);
    for (int64_t i = 0; i < n; i++) {
        Ld[(size_t)(i * n + i)] = 1.0;
        for (int32_t e = L.row_ptr[i]; e < L.row_ptr[i + 1]; e++) Ld[(size_t)(i * n + L.col_idx[e])] = L.val[e];
        for (int32_t e = U.row_ptr[i]; e < U.row_ptr[i + 1]; e++) Ud[(size_t)(i * n + U.col_idx[e])] = U.val[e];
    }
    double worst = 0.0;
    for (int64_t i = 0; i < n; i++)
        for (int32_t e = A.rp[(size_t)i]; e < A.rp[(size_t)i + 1]; e++) {
            const int64_t j = A.col[(size_t)e];
            double s = 0.0;
            for (int64_t k = 0; k < n; k++) s += Ld[(size_t)(i * n + k)] * Ud[(size_t)(k * n + j)];
            worst = std::fmax(worst, std::fabs(s - A.val[(size_t)e]));
        }
    check(worst < 1e-12, "(LU)_ij != a_ij on the pattern", name);
}

void factor_cases()
{
    struct C {
        const char *name;
        Csr A;
    };
    std::vector<C> cases;
    cases.push_back({"poisson7 N=4", poisson7(4)});
    cases.push_back({"poisson7 N=7", poisson7(7)});
    cases.push_back({"random n=150", random_dd(150, 0.04, 3)});
    cases.push_back({"random n=1", random_dd(1, 0.5, 4)});
    cases.push_back({"random n=40 dense", random_dd(40, 0.5, 5)});
    for (auto &c : cases) {
        silu_host_csr Av = c.A.view(), L, U;
        int64_t bad;
        for (int k = 0; k <= 2; k++) {
            const int st = silu_factor_iluk(&Av, k, &L, &U, &bad);
            check(st == SILU_OK && bad == -1, "ILU(k) status", c.name);
            if (st == SILU_OK) {
                check_factors(L, U, c.A.n, 0, c.name);
                if (k == 0 && c.A.n <= 400) check_ilu0_characterization(c.A, L, U, c.name);
            }
            silu_host_csr_free(&L);
            silu_host_csr_free(&U);
        }
        const double taus[3] = {0.0, 1e-3, 1e-1};
        const int ps[3] = {1, 5, 1000};
        for (double tau : taus)
            for (int p : ps) {
                const int st = silu_factor_ilut(&Av, tau, p, &L, &U, &bad);
                check(st == SILU_OK, "ILUT status", c.name);
                if (st == SILU_OK) check_factors(L, U, c.A.n, p, c.name);
                silu_host_csr_free(&L);
                silu_host_csr_free(&U);
            }
        std::printf("ok factor %s (n=%lld)\n", c.name, (long long)c.A.n);
    }
}

void factor_rejects()
{
    silu_host_csr L, U;
    int64_t bad;
    // a row without its diagonal
    Csr A = poisson7(3);
    Csr B;
    B.n = A.n;
    for (int64_t i = 0; i < A.n; i++) {
        for (int32_t e = A.rp[(size_t)i]; e < A.rp[(size_t)i + 1]; e++)
            if (!(i == 5 && A.col[(size_t)e] == 5)) {
                B.col.push_back(A.col[(size_t)e]);
                B.val.push_back(A.val[(size_t)e]);
            }
        B.rp.push_back((int32_t)B.col.size());
    }
    silu_host_csr Bv = B.view();
    int st = silu_factor_iluk(&Bv, 0, &L, &U, &bad);
    check(st != SILU_OK, "missing diagonal accepted by ILU(k)", "rejects");
    silu_host_csr_free(&L);
    silu_host_csr_free(&U);
    // ILUT forms the diagonal by elimination (fill may create it), so a row
    // stored without one either factors or reports a zero pivot at that row
    st = silu_factor_ilut(&Bv, 1e-3, 5, &L, &U, &bad);
    check(st == SILU_OK || (st == SILU_ERR_ZERO_PIVOT && bad == 5), "ILUT on a row without a stored diagonal",
          "rejects");
    if (st == SILU_OK) check_factors(L, U, B.n, 5, "ILUT without a stored diagonal");
    silu_host_csr_free(&L);
    silu_host_csr_free(&U);
    // a zero pivot: the 2x2 matrix [[0 1] [1 0]] with both diagonals stored as 0
    Csr Z;
    Z.n = 2;
    Z.rp = {0, 2, 4};
    Z.col = {0, 1, 0, 1};
    Z.val = {0.0, 1.0, 1.0, 0.0};
    silu_host_csr Zv = Z.view();
    st = silu_factor_iluk(&Zv, 0, &L, &U, &bad);
    check(st == SILU_ERR_ZERO_PIVOT && bad == 0, "zero pivot not reported", "rejects");
    silu_host_csr_free(&L);
    silu_host_csr_free(&U);
    // null outputs, null input
    check(silu_factor_iluk(&Zv, 0, nullptr, &U, &bad) == SILU_ERR_ARG, "null L accepted", "rejects");
    check(silu_factor_iluk(nullptr, 0, &L, &U, &bad) != SILU_OK, "null A accepted", "rejects");
    silu_host_csr_free(&L);
    silu_host_csr_free(&U);
    std::printf("ok factor rejects\n");
}

bool is_permutation(const std::vector<int32_t> &o)
{
    std::vector<char> seen(o.size(), 0);
    for (int32_t v : o) {
        if (v < 0 || (size_t)v >= o.size() || seen[(size_t)v]) return false;
        seen[(size_t)v] = 1;
    }
    return true;
}

void order_cases()
{
    struct C {
        const char *name;
        Csr A;
    };
    std::vector<C> cases;
    cases.push_back({"poisson7 N=6", poisson7(6)});
    cases.push_back({"random n=300 sparse", random_dd(300, 0.004, 7)});  // many components, lone rows
    cases.push_back({"random n=64", random_dd(64, 0.1, 8)});
    cases.push_back({"random n=1", random_dd(1, 0.1, 9)});
    for (auto &c : cases) {
        for (double theta : {0.0, 0.25, 1.0, 2.0}) {
            std::vector<int32_t> order((size_t)c.A.n, -1);
            const int st = silu_reorder_rcm(c.A.n, c.A.rp.data(), c.A.col.data(), c.A.val.data(), theta,
                                            order.data());
            check(st == SILU_OK, "RCM status", c.name);
            check(is_permutation(order), "RCM order is not a permutation", c.name);
        }
        std::printf("ok order %s\n", c.name);
    }
    // rejected inputs: column out of range, decreasing row pointers, bad theta, n < 0
    Csr A = poisson7(3);
    std::vector<int32_t> order((size_t)A.n);
    std::vector<int32_t> col = A.col;
    col[4] = (int32_t)A.n;
    check(silu_reorder_rcm(A.n, A.rp.data(), col.data(), A.val.data(), 0.25, order.data()) == SILU_ERR_PATTERN,
          "column out of range accepted", "order rejects");
    col[4] = -1;
    check(silu_reorder_rcm(A.n, A.rp.data(), col.data(), A.val.data(), 0.25, order.data()) == SILU_ERR_PATTERN,
          "negative column accepted", "order rejects");
    std::vector<int32_t> rp = A.rp;
    rp[3] = rp[2] - 1;
    check(silu_reorder_rcm(A.n, rp.data(), A.col.data(), A.val.data(), 0.25, order.data()) == SILU_ERR_PATTERN,
          "decreasing row pointers accepted", "order rejects");
    check(silu_reorder_rcm(A.n, A.rp.data(), A.col.data(), A.val.data(), std::nan(""), order.data()) == SILU_ERR_ARG,
          "NaN theta accepted", "order rejects");
    check(silu_reorder_rcm(-1, A.rp.data(), A.col.data(), A.val.data(), 0.25, order.data()) == SILU_ERR_ARG,
          "negative n accepted", "order rejects");
    check(silu_reorder_rcm(0, A.rp.data(), nullptr, nullptr, 0.25, nullptr) == SILU_OK, "n = 0 rejected",
          "order rejects");
    std::printf("ok order rejects\n");
}

}  // namespace

int main()
{
    factor_cases();
    factor_rejects();
    order_cases();
    if (failures) {
        std::printf("%d checks failed\n", failures);
        return 1;
    }
    std::printf("all host checks passed\n");
    return 0;
}
