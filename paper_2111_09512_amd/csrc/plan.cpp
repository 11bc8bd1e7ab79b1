// Plan of a persistent serving launch: see plan.h.
#include "plan.h"

#include <algorithm>
#include <numeric>

namespace silu {

bool persist_plan(const std::vector<int64_t> &rows, const std::vector<int> &ops, int rpb, int max_wg,
                  std::vector<int> &order, std::vector<int32_t> &first, std::vector<int32_t> &dep, int64_t *grid)
{
    const size_t nreq = rows.size();
    if (ops.size() != nreq || rpb < 1 || max_wg < 1) return false;
    order.resize(nreq);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return rows[(size_t)a] * ops[(size_t)a] < rows[(size_t)b] * ops[(size_t)b]; });
    int64_t nops = 0, tiles = 0, g = 0;
    for (size_t r = 0; r < nreq; r++) {
        if (rows[r] < 1 || ops[r] < 1) return false;
        const int64_t t = (rows[r] + rpb - 1) / rpb;
        nops += ops[r];
        tiles += t * ops[r];
        g += 2 * t;
    }
    if (nops > (1 << 24) || tiles > INT32_MAX - (1 << 20)) return false;
    first.assign((size_t)nops + 1, 0);
    dep.assign((size_t)nops, -1);
    int64_t i = 0, t0 = 0;
    for (int r : order) {
        const int64_t t = (rows[(size_t)r] + rpb - 1) / rpb;
        for (int j = 0; j < ops[(size_t)r]; j++, i++) {
            first[(size_t)i] = (int32_t)t0;
            dep[(size_t)i] = j == 0 ? -1 : (int32_t)(i - 1);
            t0 += t;
        }
    }
    first[(size_t)nops] = (int32_t)tiles;
    *grid = std::min<int64_t>(g, max_wg);
    return true;
}

} // namespace silu
