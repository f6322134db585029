// Persistent host worker threads for the data-parallel loops of a build's
// host phase (grid detection, coefficient permutation, level-table
// generation).  These loops sit between the call and the first launch, so
// the device idles while they run; threads spawned per call would cost about
// as much as the loops at moderate sizes.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <system_error>
#include <thread>
#include <vector>

namespace rsd {

class HostPool {
public:
    static HostPool& get() {
        static HostPool* pool = new HostPool();   // never destroyed: outlives static destructors
        return *pool;
    }
    int threads() const { return (int)workers_.size() + 1; }

    // fn(lo, hi) over [0, n) in about 4 chunks per thread of at least `grain`
    // items, on the workers and the calling thread; returns when every chunk
    // is done.  One loop runs at a time: a caller that finds the pool busy
    // runs its loop alone.  fn must not throw.
    void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& fn) {
        if (n <= 0) return;
        const int64_t chunks = std::min<int64_t>((n + std::max<int64_t>(grain, 1) - 1) / std::max<int64_t>(grain, 1),
                                                 4 * (int64_t)threads());
        // a loop started from inside a chunk (or while this thread runs one)
        // runs alone
        if (chunks <= 1 || workers_.empty() || in_chunk()) {
            fn(0, n);
            return;
        }
        std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
        if (!busy.owns_lock()) {
            fn(0, n);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &fn;
            n_ = n;
            step_ = (n + chunks - 1) / chunks;
            chunks_ = chunks;
            next_.store(0);
            done_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        const int64_t mine = run_chunks();
        std::unique_lock<std::mutex> lk(mu_);
        done_ += mine;
        // every chunk done and no worker still inside this job: only then may
        // the next job reset the chunk counter
        done_cv_.wait(lk, [&] { return done_ == chunks_ && active_ == 0; });
        job_ = nullptr;
    }

private:
    HostPool() {
        const unsigned hw = std::thread::hardware_concurrency();
        const int nw = (int)std::min<unsigned>(hw > 1 ? hw - 1 : 0, 7);
        for (int i = 0; i < nw; ++i) {
            try {
                workers_.emplace_back([this] { loop(); });
            } catch (const std::system_error&) {
                break;
            }
        }
        for (auto& t : workers_) t.detach();
    }
    static bool& in_chunk() {
        static thread_local bool flag = false;
        return flag;
    }
    int64_t run_chunks() {
        int64_t c;
        int64_t finished = 0;
        in_chunk() = true;
        while ((c = next_.fetch_add(1)) < chunks_) {
            const int64_t lo = c * step_, hi = std::min(n_, lo + step_);
            if (lo < hi) (*job_)(lo, hi);
            ++finished;
        }
        in_chunk() = false;
        return finished;
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen && job_ != nullptr; });
                seen = gen_;
                ++active_;
            }
            const int64_t finished = run_chunks();
            {
                std::lock_guard<std::mutex> lk(mu_);
                done_ += finished;
                --active_;
            }
            done_cv_.notify_all();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex run_mu_;             // one loop at a time
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int64_t, int64_t)>* job_ = nullptr;
    int64_t n_ = 0, step_ = 0, chunks_ = 0, done_ = 0;
    int active_ = 0;                // workers inside the current job
    std::atomic<int64_t> next_{0};
    uint64_t gen_ = 0;
};

}  // namespace rsd
