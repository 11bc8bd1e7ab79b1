// Locality order for the sweeps' relabeled copies (SILU_REORDER): host code.
//
// Reverse Cuthill-McKee on the graph of strong couplings (|a_ij| >= theta *
// max_{k != i} |a_ik|, the strength of connection of algebraic multigrid,
// Section 3), which ignores weak long-range couplings that would otherwise
// collapse the BFS levels.  Plain C++ (no HIP), so it builds and is checked
// under the host sanitizers like the factorizations.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/scaled_ilu.h"

namespace silu {

// Reverse Cuthill-McKee on the strong-coupling graph (host).  Components are
// started from their unvisited row of least strong degree; each row's
// unvisited strong neighbours are queued by increasing degree (ties: lower
// index).  order[k] = the row placed at position k.
int rcm_strength_order(int64_t n, const int32_t *rp, const int32_t *col, const double *val, double theta,
                       int32_t *order)
{
    if (n <= 0) return SILU_OK;
    std::vector<int32_t> deg((size_t)n, 0), srp((size_t)n + 1, 0);
    std::vector<int32_t> sadj;
    sadj.reserve((size_t)rp[n]);
    for (int64_t i = 0; i < n; i++) {
        double mx = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; e++)
            if (col[e] != i) mx = std::max(mx, std::fabs(val[e]));
        for (int32_t e = rp[i]; e < rp[i + 1]; e++) {
            const int32_t j = col[e];
            if (j < 0 || j >= n) return SILU_ERR_PATTERN;
            if (j != i && mx > 0.0 && std::fabs(val[e]) >= theta * mx) sadj.push_back(j);
        }
        srp[(size_t)i + 1] = (int32_t)sadj.size();
        deg[(size_t)i] = srp[(size_t)i + 1] - srp[(size_t)i];
    }
    // rows by increasing degree (counting sort, stable in the index)
    int32_t maxd = 0;
    for (int32_t d : deg) maxd = std::max(maxd, d);
    std::vector<int64_t> cnt((size_t)maxd + 2, 0);
    for (int32_t d : deg) cnt[(size_t)d + 1]++;
    for (size_t d = 1; d < cnt.size(); d++) cnt[d] += cnt[d - 1];
    std::vector<int32_t> by_deg((size_t)n);
    for (int64_t i = 0; i < n; i++) by_deg[(size_t)cnt[(size_t)deg[(size_t)i]]++] = (int32_t)i;
    std::vector<char> seen((size_t)n, 0);
    int64_t head = 0, tail = 0;
    std::vector<int32_t> nb;
    for (int64_t s = 0; s < n; s++) {
        const int32_t start = by_deg[(size_t)s];
        if (seen[(size_t)start]) continue;
        seen[(size_t)start] = 1;
        order[tail++] = start;
        while (head < tail) {
            const int32_t u = order[head++];
            nb.clear();
            for (int32_t e = srp[(size_t)u]; e < srp[(size_t)u + 1]; e++) {
                const int32_t v = sadj[(size_t)e];
                if (!seen[(size_t)v]) {
                    seen[(size_t)v] = 1;
                    nb.push_back(v);
                }
            }
            std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
                return deg[(size_t)a] != deg[(size_t)b] ? deg[(size_t)a] < deg[(size_t)b] : a < b;
            });
            for (int32_t v : nb) order[tail++] = v;
        }
    }
    std::reverse(order, order + n);
    return SILU_OK;
}

} // namespace silu

extern "C" int silu_reorder_rcm(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                                double theta, int32_t *order)
{
    if (n < 0 || n >= INT32_MAX || (n > 0 && (!row_ptr || !order)) || !(theta >= 0.0)) return SILU_ERR_ARG;
    if (n > 0 && row_ptr[n] > 0 && (!col_idx || !val)) return SILU_ERR_ARG;
    for (int64_t i = 0; i < n; i++)
        if (row_ptr[i + 1] < row_ptr[i] || row_ptr[0] != 0) return SILU_ERR_PATTERN;
    return silu::rcm_strength_order(n, row_ptr, col_idx, val, theta, order);
}
