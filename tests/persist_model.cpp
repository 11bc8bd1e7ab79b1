// Host-thread model of the persistent serving launch's protocol (the kernel
// that runs a batch's chains of sweeps in one launch), on the plan the
// serving runtime builds (persist_plan, linked from the library's sources).
// Each thread plays a workgroup: it takes the next tile number from a shared
// counter, finds the tile's op (the largest op whose first tile is at or below
// it), waits until the op it depends on has counted all of its tiles, "runs"
// the tile and counts it for its op -- the kernel's steps in the kernel's
// order.  Running a tile reads every tile record of the op it depends on
// (plain, non-atomic memory: in the kernel, the gathers of the previous
// iterate) and writes its own, so a tile run before its dependency has
// finished is caught here by the check and, under ThreadSanitizer, as a data
// race.  The kernel's relaxed counter updates with a device fence before the
// increment and after the wait are written as release increments and acquire
// loads, their C++ counterparts (ThreadSanitizer does not follow stand-alone
// fences).  Each wait is bounded by a wall-clock deadline, as in the kernel;
// an expired wait is reported and fails the run.
//
// Built with -DPLANT_NO_WAIT the wait is skipped (a deliberate protocol
// mistake), which the checks must catch.
//
// Input (stdin): the worker count, then one line "rows ops" per request in
// submission order.  Prints the plan's sizes and "model ok", or what failed,
// and exits non-zero on a failure.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <thread>
#include <vector>

#include "../paper_2111_09512_amd/csrc/plan.h"

int main()
{
    int workers = 0;
    if (std::scanf("%d", &workers) != 1 || workers < 1) return 2;
    std::vector<int64_t> rows;
    std::vector<int> ops;
    long long r;
    int o;
    while (std::scanf("%lld %d", &r, &o) == 2) {
        rows.push_back(r);
        ops.push_back(o);
    }
    std::vector<int> order;
    std::vector<int32_t> first, dep;
    int64_t grid = 0;
    if (!silu::persist_plan(rows, ops, 256, workers, order, first, dep, &grid)) {
        std::printf("FAIL: plan refused\n");
        return 1;
    }
    const int nops = (int)dep.size(), total = first[(size_t)nops];
    // the plan itself: tiles of each op = ceil(rows / 256), chains in order
    {
        int i = 0;
        std::vector<int> seen(rows.size(), 0);
        for (int q : order) {
            if (seen[(size_t)q]++) {
                std::printf("FAIL: request %d planned twice\n", q);
                return 1;
            }
            const int t = (int)((rows[(size_t)q] + 255) / 256);
            for (int j = 0; j < ops[(size_t)q]; j++, i++) {
                if (first[(size_t)i + 1] - first[(size_t)i] != t || dep[(size_t)i] != (j == 0 ? -1 : i - 1)) {
                    std::printf("FAIL: op %d of request %d planned wrongly\n", i, q);
                    return 1;
                }
            }
        }
        if (i != nops || first[0] != 0) {
            std::printf("FAIL: op count\n");
            return 1;
        }
    }
    std::atomic<int> next{0}, expired{0}, misordered{0};
    std::vector<std::atomic<int>> done((size_t)nops);
    for (auto &d : done) d.store(0);
    std::vector<int> tile_rec((size_t)total, 0); // plain memory: each tile's "output"
    const auto deadline_per_wait = std::chrono::seconds(20);
    auto body = [&]() {
        for (;;) {
            const int t = next.fetch_add(1, std::memory_order_relaxed);
            if (t >= total) return;
            const int op = (int)(std::upper_bound(first.begin(), first.end(), t) - first.begin()) - 1;
            const int d = dep[(size_t)op];
            bool skip = false;
            if (d >= 0) {
                const int need = first[(size_t)d + 1] - first[(size_t)d];
                const auto t0 = std::chrono::steady_clock::now();
#ifdef PLANT_NO_WAIT // a protocol mistake planted on purpose: the wait is skipped
                while (false) {
#else
                while (done[(size_t)d].load(std::memory_order_acquire) < need) {
#endif
                    std::this_thread::yield();
                    if (std::chrono::steady_clock::now() - t0 > deadline_per_wait) {
                        expired.fetch_add(1);
                        skip = true;
                        break;
                    }
                }
                if (!skip)
                    for (int u = first[(size_t)d]; u < first[(size_t)d + 1]; u++)
                        if (tile_rec[(size_t)u] != d + 1) misordered.fetch_add(1);
            }
            tile_rec[(size_t)t] = op + 1;
            done[(size_t)op].fetch_add(1, std::memory_order_release);
        }
    };
    std::vector<std::thread> pool;
    for (int w = 0; w < (int)grid; w++) pool.emplace_back(body);
    for (auto &th : pool) th.join();
    int unfinished = 0;
    for (int i = 0; i < nops; i++)
        if (done[(size_t)i].load() != first[(size_t)i + 1] - first[(size_t)i]) unfinished++;
    std::printf("requests %zu ops %d tiles %d workers %lld: expired waits %d, tiles before their dependency %d, "
                "ops not fully counted %d\n",
                rows.size(), nops, total, (long long)grid, expired.load(), misordered.load(), unfinished);
    if (expired.load() || misordered.load() || unfinished) {
        std::printf("FAIL\n");
        return 1;
    }
    std::printf("model ok\n");
    return 0;
}
