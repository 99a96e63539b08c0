// Host worker pool of fedfem_precompute_many: `threads` workers (the calling
// thread among them) take items 0..n-1 from one atomic counter, so a slow
// item never holds up the others; each worker's layout builds are capped at
// `inner` host threads, so workers running side by side share the cores.
#include <algorithm>
#include <atomic>
#include <system_error>
#include <thread>
#include <vector>

#include "internal.h"

namespace fedfem {

void run_workers(int32_t n, int32_t threads, int inner, const std::function<void(int32_t)>& fn) {
    std::atomic<int32_t> next{0};
    auto work = [&] {
        const int prev = set_layout_threads(inner);
        for (;;) {
            const int32_t j = next.fetch_add(1);
            if (j >= n) break;
            fn(j);
        }
        set_layout_threads(prev);
    };
    std::vector<std::thread> pool;
    try {
        for (int32_t t = 1; t < threads; t++) pool.emplace_back(work);
    } catch (const std::system_error&) {
        // fewer workers than asked: the remaining ones share the work
    }
    work();
    for (auto& t : pool) t.join();
}

}  // namespace fedfem
