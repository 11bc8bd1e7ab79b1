// Plan of a persistent serving launch (host code, no HIP): the tiles of every
// op of a batch of requests numbered into one queue.  Shared by the serving
// runtime and the host-thread model of the launch's protocol in the tests.
#ifndef SILU_PLAN_H
#define SILU_PLAN_H

#include <cstdint>
#include <vector>

namespace silu {

// Requests (rows[r], ops[r]) are ordered by their work rows * ops, smallest
// first (stable), into `order`; request order[k] then contributes ops[order[k]]
// consecutive ops, each of ceil(rows / rpb) tiles, op j depending on op j - 1
// of the same request.  first[i] = the first tile of op i (first[nops] = all
// tiles), dep[i] = the op op i waits for (-1 for a request's first op).  grid =
// two ops' tiles per request (one at work, the next waiting), at most max_wg.
// Returns false when the plan would not fit 32-bit tile numbers or 2^24 ops.
bool persist_plan(const std::vector<int64_t> &rows, const std::vector<int> &ops, int rpb, int max_wg,
                  std::vector<int> &order, std::vector<int32_t> &first, std::vector<int32_t> &dep, int64_t *grid);

} // namespace silu

#endif
