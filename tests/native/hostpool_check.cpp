// Stress check of the host worker pool (csrc/hostpool.hpp): three threads run
// loops of varying length concurrently (one of them at a time gets the pool,
// the others run alone), each loop starts a nested loop from inside a chunk,
// and every index must be visited exactly once.  Exit status 0 on success.
#include "../../paper_1303_5466_amd/csrc/hostpool.hpp"

#include <cstdio>
#include <thread>
#include <vector>

int main() {
    auto& pool = rsd::HostPool::get();
    std::atomic<long> errors{0};
    auto body = [&](int seed) {
        for (int it = 0; it < 1500; ++it) {
            const int64_t n = 1 + (it * 7919 + seed * 104729) % 40000;
            std::vector<int> hit(n, 0);
            pool.parallel_for(n, 1000, [&](int64_t lo, int64_t hi) {
                for (int64_t i = lo; i < hi; ++i) hit[i]++;
                if (lo == 0) {
                    std::atomic<int> inner{0};
                    pool.parallel_for(64, 1, [&](int64_t a, int64_t b) { inner += (int)(b - a); });
                    if (inner != 64) errors++;
                }
            });
            for (int64_t i = 0; i < n; ++i)
                if (hit[i] != 1) errors++;
        }
    };
    std::thread t1(body, 1), t2(body, 2);
    body(3);
    t1.join();
    t2.join();
    std::printf("threads %d errors %ld\n", pool.threads(), errors.load());
    return errors.load() == 0 ? 0 : 1;
}
