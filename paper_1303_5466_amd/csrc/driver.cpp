// Factor object, level-by-level build, inverse apply and the C interface.
//
// Build (Algorithm 1 in the block form of Algorithm 2, fine-to-coarse):
//   interpolation  T for every box type: proxy matrices, pivoted QR (k_qr)
//   per level      F_i = D_i (leaves) or [E_c1 K12; K21 E_c2] (k_gen)
//                  F'_sr = F_sr - F_ss T                        (GEMM)
//                  F'_rr = F_rr - F_rs T - T^T F'_sr            (GEMM, 2 terms)
//                  F'_rs = F'_sr^T                              (transpose)
//                  [F'_rr | F'_rs] -> [G | W], G = F'_rr^{-1}   (Gauss-Jordan)
//                  E_i = F_ss - F'_sr W                         (GEMM)
//   top            the root is eliminated the same way with its first child
//                  as residual and T = 0, and the remaining block inverted.
// E_i here equals (R_i F_i^{-1} L_i)^{-1} of Algorithm 1: F' = P^{-T} F P^{-1}
// with P = [I T; 0 I] is a congruence, and the skeleton block of F'^{-1} is
// the inverse of the Schur complement F'_ss - F'_sr F'_rr^{-1} F'_rs.
//
// Solve (Algorithm 6 in the same variables), per box:
//   up    f'_r = f_r - T^T f_s ;  y = G f'_r ;  g = f_s - W^T f'_r  -> parent
//   top   phi = G_top g
//   down  s'_r = y - W phi ;  s_s = phi - T s'_r ;  s_r = s'_r      -> children
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <condition_variable>
#include <type_traits>
#include <vector>

#include "../../include/rsd.h"
#include "common.hpp"
#include "hostpool.hpp"
#include "plan.hpp"

namespace rsd {

struct Error : std::runtime_error {
    rsd_status code;
    Error(rsd_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

static thread_local std::string g_last_error;

// ----------------------------------------------------------------------------
// device memory
// ----------------------------------------------------------------------------
// Caching allocator: device blocks freed by one factor, solve or build are
// kept per device and handed out again to a later request of about the same
// size, so repeated builds do not pay hipMalloc / hipFree for their arenas
// (freeing a large arena synchronises and unmaps, about a millisecond).
// A block is cached only once its last use has completed: a release inside
// an IdleScope (its owner has synchronised every stream that used it) is
// immediate, any other release synchronises the device first, as hipFree
// does.  At most `limit` bytes stay cached per device; an allocation that
// fails returns the device's cache to HIP and tries again.
static thread_local int g_idle_depth = 0;
struct IdleScope {
    IdleScope() { ++g_idle_depth; }
    ~IdleScope() { --g_idle_depth; }
};

// Runs `work` on the calling thread and on up to n - 1 more, then joins them.
// The callers share their items through an atomic counter, so a thread
// that cannot be started only leaves its share to the others.
template <typename Fn>
static void run_on_threads(int n, Fn&& work) {
    std::vector<std::thread> ts;
    for (int i = 1; i < n; ++i) {
        try {
            ts.emplace_back(work);
        } catch (const std::system_error&) {
            break;
        }
    }
    work();
    for (auto& t : ts) t.join();
}

class DevicePool {
public:
    static DevicePool& get() {
        static DevicePool* pool = new DevicePool();   // outlives static destructors
        return *pool;
    }
    // size class: 512 B minimum, powers of two up to 1 MiB, then 2 MiB multiples
    static size_t size_class(size_t n) {
        if (n <= 512) return 512;
        if (n <= (size_t(1) << 20)) {
            size_t c = 512;
            while (c < n) c <<= 1;
            return c;
        }
        const size_t g = size_t(2) << 20;
        return (n + g - 1) / g * g;
    }
    void* take(int dev, size_t want, size_t& cap) {
        const size_t c = size_class(want);
        {
            std::lock_guard<std::mutex> lk(mu_);
            Dev& d = devs_[dev];
            auto it = d.blocks.lower_bound(c);
            // small classes match exactly; large blocks up to 1/8 above the request
            if (it != d.blocks.end() && it->first <= c + (c > (size_t(1) << 20) ? c / 8 : 0)) {
                void* p = it->second;
                cap = it->first;
                d.cached -= cap;
                d.blocks.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, c);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim(dev);
            e = hipMalloc(&p, c);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        cap = c;
        return p;
    }
    void give(int dev, void* p, size_t cap) {
        if (g_idle_depth == 0) (void)hipDeviceSynchronize();
        std::vector<void*> drop;
        {
            std::lock_guard<std::mutex> lk(mu_);
            Dev& d = devs_[dev];
            const size_t lim = limit(dev);
            if (cap > lim) {
                drop.push_back(p);
            } else {
                d.blocks.emplace(cap, p);
                d.cached += cap;
                while (d.cached > lim) {          // evict the largest blocks first
                    auto it = std::prev(d.blocks.end());
                    d.cached -= it->first;
                    drop.push_back(it->second);
                    d.blocks.erase(it);
                }
            }
        }
        for (void* q : drop) (void)hipFree(q);
    }
    // hands every cached block of a device (dev < 0: all devices) back to HIP
    void trim(int dev) {
        std::vector<std::pair<int, void*>> drop;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (auto& kv : devs_) {
                if (dev >= 0 && kv.first != dev) continue;
                for (auto& b : kv.second.blocks) drop.emplace_back(kv.first, b.second);
                kv.second.blocks.clear();
                kv.second.cached = 0;
            }
        }
        int cur = 0;
        (void)hipGetDevice(&cur);
        for (auto& q : drop) {
            (void)hipSetDevice(q.first);
            (void)hipFree(q.second);
        }
        (void)hipSetDevice(cur);
    }
    int64_t cached(int dev) {
        std::lock_guard<std::mutex> lk(mu_);
        int64_t t = 0;
        for (auto& kv : devs_)
            if (dev < 0 || kv.first == dev) t += (int64_t)kv.second.cached;
        return t;
    }
    void set_limit(int64_t bytes) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            user_limit_ = bytes;
        }
        if (bytes >= 0) {
            // apply at once: drop what no longer fits
            std::vector<std::pair<int, void*>> drop;
            {
                std::lock_guard<std::mutex> lk(mu_);
                for (auto& kv : devs_) {
                    Dev& d = kv.second;
                    while (d.cached > (size_t)bytes && !d.blocks.empty()) {
                        auto it = std::prev(d.blocks.end());
                        d.cached -= it->first;
                        drop.emplace_back(kv.first, it->second);
                        d.blocks.erase(it);
                    }
                }
            }
            int cur = 0;
            (void)hipGetDevice(&cur);
            for (auto& q : drop) {
                (void)hipSetDevice(q.first);
                (void)hipFree(q.second);
            }
            (void)hipSetDevice(cur);
        }
    }

private:
    struct Dev {
        std::multimap<size_t, void*> blocks;
        size_t cached = 0;
        size_t total = 0;     // device memory, read once
    };
    // default: min(16 GiB, 1/8 of the device memory); called with mu_ held
    size_t limit(int dev) {
        if (user_limit_ >= 0) return (size_t)user_limit_;
        Dev& d = devs_[dev];
        if (d.total == 0) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
                (void)hipGetLastError();
                tot = size_t(8) << 30;
            }
            d.total = tot;
        }
        return std::min<size_t>(size_t(16) << 30, d.total / 8);
    }
    std::mutex mu_;
    std::map<int, Dev> devs_;
    int64_t user_limit_ = -1;
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;     // requested size
    size_t cap = 0;       // size of the pool block
    int dev = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) DevicePool::get().give(dev, p, cap);
        p = nullptr;
        bytes = cap = 0;
    }
    void alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        RSD_HIP(hipGetDevice(&dev));
        p = DevicePool::get().take(dev, n, cap);
        if (!p) throw Error(RSD_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
        bytes = n;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Host tables packed into one byte buffer (each at a 256-byte boundary) so
// that they go to the device in one copy.
struct HostPack {
    std::vector<unsigned char> bytes;
    template <typename T>
    size_t add(const std::vector<T>& v) {
        const size_t o = (bytes.size() + 255) / 256 * 256;
        bytes.resize(o + std::max<size_t>(v.size() * sizeof(T), 1));
        if (!v.empty()) std::memcpy(bytes.data() + o, v.data(), v.size() * sizeof(T));
        return o;
    }
};

template <typename T>
static void upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    b.alloc(v.size() * sizeof(T));
    if (!v.empty()) RSD_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Non-blocking streams, kept per device and handed to later factors and
// builds: creating and destroying the streams of a build costs a few hundred
// microseconds of host time each, a large share of a small grid's build.  A
// stream handed back may still hold queued work; its next owner's launches
// queue behind it.
class StreamPool {
public:
    static StreamPool& get() {
        static StreamPool* pool = new StreamPool();   // outlives static destructors
        return *pool;
    }
    // a stream of the current device
    hipStream_t take() {
        int dev = 0;
        RSD_HIP(hipGetDevice(&dev));
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto& v = free_[dev];
            if (!v.empty()) {
                hipStream_t q = v.back();
                v.pop_back();
                return q;
            }
        }
        hipStream_t q = nullptr;
        RSD_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        return q;
    }
    void give(int dev, hipStream_t q) {
        if (!q) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_[dev].push_back(q);
    }

private:
    std::mutex mu_;
    std::map<int, std::vector<hipStream_t>> free_;
};

// Pinned host blocks for staging large uploads: a copy from pinned memory is
// asynchronous, one from pageable memory returns only when it is done.  The
// blocks are kept for reuse (pinning costs about a millisecond per block);
// a holder returns its block only after the copy has completed.
class PinnedPool {
public:
    static PinnedPool& get() {
        static PinnedPool* pool = new PinnedPool();   // outlives static destructors
        return *pool;
    }
    void* take(size_t n, size_t& cap) {
        cap = std::max<size_t>((n + (size_t(1) << 20) - 1) >> 20 << 20, size_t(1) << 20);
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(cap);
            if (it != free_.end() && it->first <= 2 * cap) {
                void* p = it->second;
                cap = it->first;
                free_.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        RSD_HIP(hipHostMalloc(&p, cap, hipHostMallocDefault));
        return p;
    }
    void give(void* p, size_t cap) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_.emplace(cap, p);
    }

private:
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
};

// Pinned host words (flags read back by the host), handed out from 4 KiB
// pages that live until the process ends: pinning and unpinning a page
// costs hundreds of microseconds, more than a small solve.
class PinnedWords {
public:
    static PinnedWords& get() {
        static PinnedWords* w = new PinnedWords();   // outlives static destructors
        return *w;
    }
    int* take() {
        std::lock_guard<std::mutex> lk(mu_);
        if (free_.empty()) {
            void* page = nullptr;
            RSD_HIP(hipHostMalloc(&page, 4096, hipHostMallocDefault));
            for (int i = 0; i < 4096 / 64; ++i) free_.push_back(static_cast<int*>(page) + 16 * i);
        }
        int* w = free_.back();
        free_.pop_back();
        return w;
    }
    void give(int* w) {
        if (!w) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_.push_back(w);
    }

private:
    std::mutex mu_;
    std::vector<int*> free_;   // one word per 64-byte line
};

static bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// ----------------------------------------------------------------------------
// kernel-class profiler (HIP events around launches, enabled on demand)
// ----------------------------------------------------------------------------
struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
    int64_t groups;     // work-groups of the launch (0: not recorded)
};
struct Profiler {
    bool on = false;
    bool paused = false;        // on, but nothing bracketed until resumed (records kept)
    uint32_t mask = ~0u;        // classes bracketed while on
    std::mutex mu;              // solves of different factors may run on several threads
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        std::lock_guard<std::mutex> lk(mu);
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e;
        RSD_HIP(hipEventCreate(&e));
        return e;
    }
    void clear() {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
        recs.clear();
    }
    void add(const ProfRec& r) {
        std::lock_guard<std::mutex> lk(mu);
        recs.push_back(r);
    }
};
static Profiler g_prof;

static bool prof_active(int cls) { return g_prof.on && !g_prof.paused && cls >= 0 && cls < 32 && ((g_prof.mask >> cls) & 1u); }

struct ProfScope {
    bool act;
    ProfRec rec;
    hipStream_t s;
    ProfScope(int cls, hipStream_t st, double flops = 0, double bytes = 0, int64_t groups = 0)
        : act(prof_active(cls)), s(st) {
        if (!act) return;
        rec.cls = cls; rec.flops = flops; rec.bytes = bytes; rec.groups = groups;
        rec.a = g_prof.get();
        rec.b = g_prof.get();
        RSD_HIP(hipEventRecord(rec.a, s));
    }
    ~ProfScope() {
        if (!act) return;
        if (hipEventRecord(rec.b, s) == hipSuccess) g_prof.add(rec);
    }
};

// ----------------------------------------------------------------------------
// GEMM batches: descriptors + tile tables, uploaded once
// ----------------------------------------------------------------------------
// ---- tile autotuner -----------------------------------------------------------
// The grouped GEMM launches of the factor levels choose a tile width (64 or
// 128) and a split-K target (how many work-groups per compute unit long K
// ranges are split for, or none).  The built-in rule is a heuristic; the
// tuner replaces it per launch shape: a launch's shape bucket is (element
// size, log2 of its 64-wide tile count, log2 of its longest K, log2 of its
// flops), and rsd_autotune times every candidate on real builds and keeps the
// fastest per bucket.  The table can be saved to and loaded from a text file
// (one "bucket tile split" line per entry; RSD_TUNE_FILE names a file loaded
// at the first build).
struct TuneChoice {
    int tile = 64;
    int split = 2;      // split target in work-groups per compute unit (0: never split)
};
constexpr int TUNE_CANDIDATES = 6;
static const TuneChoice kTuneCand[TUNE_CANDIDATES] = {{64, 2}, {64, 0}, {64, 4}, {128, 2}, {128, 0}, {128, 4}};

class Tuner {
public:
    static Tuner& get() {
        static Tuner t;
        return t;
    }
    static uint64_t key(int es, int64_t t64, int kmax, double flops) {
        auto lg = [](double v) { return v < 1 ? 0 : (int)std::floor(std::log2(v)); };
        return (uint64_t)es | ((uint64_t)std::min(lg((double)t64), 63) << 8) |
               ((uint64_t)std::min(lg((double)kmax), 63) << 16) | ((uint64_t)std::min(lg(flops), 127) << 24);
    }
    // the choice for a launch: the forced candidate while tuning, else the
    // table's entry, else false (heuristic)
    bool choice(uint64_t k, TuneChoice& c) {
        std::lock_guard<std::mutex> lk(mu_);
        load_env();
        if (forced_ >= 0) {
            c = kTuneCand[forced_];
            return true;
        }
        auto it = table_.find(k);
        if (it == table_.end()) return false;
        c = it->second;
        return true;
    }
    void set_forced(int cand) {
        std::lock_guard<std::mutex> lk(mu_);
        forced_ = cand;
    }
    bool recording() const { return recording_.load(std::memory_order_relaxed); }
    void set_recording(bool on) { recording_.store(on); }
    // one timed launch (events recorded on its stream)
    void record(uint64_t k, hipEvent_t a, hipEvent_t b) {
        std::lock_guard<std::mutex> lk(mu_);
        pending_.push_back({k, forced_, a, b});
    }
    hipEvent_t event() {
        std::lock_guard<std::mutex> lk(mu_);
        if (!free_ev_.empty()) {
            hipEvent_t e = free_ev_.back();
            free_ev_.pop_back();
            return e;
        }
        hipEvent_t e;
        RSD_HIP(hipEventCreate(&e));
        return e;
    }
    // after a device synchronisation: fold the recorded launches into the
    // per-bucket, per-candidate totals
    void collect() {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto& r : pending_) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && r.cand >= 0) {
                auto& v = times_[r.k];
                v.resize(TUNE_CANDIDATES, 0.0);
                v[r.cand] += ms;
            } else {
                (void)hipGetLastError();
            }
            free_ev_.push_back(r.a);
            free_ev_.push_back(r.b);
        }
        pending_.clear();
    }
    // picks the fastest candidate of every bucket timed under all candidates
    int commit() {
        std::lock_guard<std::mutex> lk(mu_);
        int n = 0;
        for (auto& kv : times_) {
            const auto& v = kv.second;
            int best = -1;
            for (int c = 0; c < TUNE_CANDIDATES; ++c)
                if (v[c] > 0 && (best < 0 || v[c] < v[best])) best = c;
            bool all = true;
            for (int c = 0; c < TUNE_CANDIDATES; ++c) all = all && v[c] > 0;
            if (best >= 0 && all) {
                table_[kv.first] = kTuneCand[best];
                ++n;
            }
        }
        times_.clear();
        return n;
    }
    void clear() {
        std::lock_guard<std::mutex> lk(mu_);
        table_.clear();
        times_.clear();
    }
    int64_t size() {
        std::lock_guard<std::mutex> lk(mu_);
        return (int64_t)table_.size();
    }
    void save(const char* path) {
        std::lock_guard<std::mutex> lk(mu_);
        FILE* fp = std::fopen(path, "w");
        if (!fp) throw Error(RSD_EINVAL, std::string("cannot write ") + path);
        for (auto& kv : table_)
            std::fprintf(fp, "%llu %d %d\n", (unsigned long long)kv.first, kv.second.tile, kv.second.split);
        std::fclose(fp);
    }
    void load(const char* path) {
        std::lock_guard<std::mutex> lk(mu_);
        load_file(path);
    }

private:
    struct Rec {
        uint64_t k;
        int cand;
        hipEvent_t a, b;
    };
    void load_file(const char* path) {
        FILE* fp = std::fopen(path, "r");
        if (!fp) throw Error(RSD_EINVAL, std::string("cannot read ") + path);
        unsigned long long k;
        int tile, split;
        while (std::fscanf(fp, "%llu %d %d", &k, &tile, &split) == 3)
            if ((tile == 64 || tile == 128) && split >= 0 && split <= 16) table_[k] = {tile, split};
        std::fclose(fp);
    }
    void load_env() {
        if (env_done_) return;
        env_done_ = true;
        const char* p = std::getenv("RSD_TUNE_FILE");
        if (p && *p) {
            try {
                load_file(p);
            } catch (const std::exception&) {
            }
        }
    }
    std::mutex mu_;
    std::map<uint64_t, TuneChoice> table_;
    std::map<uint64_t, std::vector<double>> times_;
    std::vector<Rec> pending_;
    std::vector<hipEvent_t> free_ev_;
    std::atomic<bool> recording_{false};
    int forced_ = -1;
    bool env_done_ = false;
};

template <typename T>
struct GemmBatch {
    std::vector<GemmDesc<T>> descs;
    std::vector<TileRef> tiles;            // built by finalize(): one per work-group
    std::vector<TileRef> slots;            // split tiles (reduce dispatch), one each
    const GemmDesc<T>* d_descs = nullptr;
    const TileRef* d_tiles = nullptr;
    const TileRef* d_slots = nullptr;
    T* d_ws = nullptr;                     // split-K partial tiles (shared by a batch list)
    int tile = 64;
    int64_t ws_elems = 0;                  // partial-tile elements
    double flops = 0, bytes = 0;
    int prof_cls = -1;
    int role = -1;      // kernel instantiation (see launch_gemm); -1: from prof_cls
    int max_split = 16; // 1: no split K, so every product's rounding is independent of the batch
    int wg_waves = 0;   // solve products: > 0, one work-group of this many waves per 16-row item
    uint64_t tune_key = 0;  // shape bucket of a tuned launch (0: not tuned)
    void add(const GemmDesc<T>& d) {
        if (d.M <= 0 || d.N <= 0) return;
        descs.push_back(d);
        const double kk = (double)(std::max(d.K, 0) + std::max(d.K2, 0));
        flops += 2.0 * d.M * d.N * kk;
        bytes += sizeof(T) * ((double)d.M * kk + kk * d.N + 2.0 * d.M * d.N);
    }
    bool empty() const { return descs.empty(); }
    // Tile table.  128-wide tiles when the products are large, have K > 128
    // and give every compute unit two tiles; otherwise 64.  When even the 64-wide tiles
    // cannot give every compute unit one, long K ranges are split (at least
    // eight panels per split, at most 16 splits) and summed by a second
    // dispatch.
    void finalize() {
        constexpr int CUS = 256;
        // the kernel addresses each operand with 32-bit byte offsets from the
        // tile's first row / column (at most 128 of them, all of K)
        auto reach = [](int rows, int cols, int ld, int tr) {
            if (rows <= 0 || cols <= 0) return (int64_t)0;
            rows = std::min(rows, 128);   // rows: the tile's dimension; cols: K
            return (int64_t)sizeof(T) * ((tr ? (int64_t)(cols - 1) + (int64_t)(rows - 1) * ld
                                             : (int64_t)(rows - 1) + (int64_t)(cols - 1) * ld) + 1);
        };
        for (auto& d : descs) {
            // A is M x K (tA: stored K x M), B is K x N (tB: stored N x K)
            int64_t e = std::max(reach(d.M, d.K, d.lda, d.tA), reach(d.N, d.K, d.ldb, !d.tB));
            if (d.K2 > 0) e = std::max({e, reach(d.M, d.K2, d.lda2, d.tA2), reach(d.N, d.K2, d.ldb2, !d.tB2)});
            e = std::max(e, reach(std::min(d.M, 128), std::min(d.N, 128), d.ldc, 0));
            if (e + 16 > (int64_t)GEMM_MAX_OPERAND_BYTES)
                throw Error(RSD_EINVAL, "matrix block too large for the GEMM kernel (2 GiB reach of a tile)");
        }
        tiles.clear();
        slots.clear();
        ws_elems = 0;
        // the solve's products over at most 16 right-hand sides: one 16-row
        // block per wave, K split until there are about four per compute
        // unit; a split item's waves form one work-group and sum their parts
        // in LDS (no second dispatch)
        bool skinny = kernel_role() == 2;
        for (auto& d : descs) skinny = skinny && d.N <= 16;
        wg_waves = 0;
        if (skinny) {
            tile = 16;
            int64_t blocks = 0;
            for (auto& d : descs) blocks += (d.M + 15) / 16;
            std::vector<int> S(descs.size(), 1);
            int smax = 1;
            for (int id = 0; id < (int)descs.size(); ++id) {
                const auto& d = descs[id];
                const int ksteps = (std::max(d.K, 0) + 3) / 4 + (std::max(d.K2, 0) + 3) / 4;
                if (blocks < 4 * CUS)
                    S[id] = std::max(1, std::min<int>({(int)((4 * CUS + blocks - 1) / blocks), ksteps / 16,
                                                       SKINNY_WG_WAVES}));
                smax = std::max(smax, S[id]);
            }
            if (smax > 1) wg_waves = smax;
            for (int id = 0; id < (int)descs.size(); ++id)
                for (int rb = 0; rb < (descs[id].M + 15) / 16; ++rb) tiles.push_back({id, rb, 0, 0, S[id], 0});
            return;
        }
        int64_t t64 = 0, t128 = 0;
        double big = 0, tot = 0;
        int kmax = 0;
        for (auto& d : descs) {
            kmax = std::max(kmax, std::max(d.K, 0) + std::max(d.K2, 0));
            t64 += (int64_t)((d.M + 63) / 64) * ((d.N + 63) / 64);
            t128 += (int64_t)((d.M + 127) / 128) * ((d.N + 127) / 128);
            const double w = (double)d.M * d.N * (std::max(d.K, 0) + std::max(d.K2, 0));
            tot += w;
            if (d.M >= 128 && d.N >= 128) big += w;
        }
        // short-K launches (the Gauss-Jordan updates) are bound by their C
        // traffic: the 64-wide tiles load C before the K loop
        tile = (t128 >= 2 * CUS && big >= 0.8 * tot && kmax > 128) ? 128 : 64;
        int split_target = 2;
        tune_key = 0;
        if (kernel_role() == 0 && max_split > 1) {
            // the factor levels' launches: the tuned choice for this shape
            const uint64_t k = Tuner::key((int)sizeof(T), t64, kmax, flops);
            TuneChoice c;
            if (Tuner::get().choice(k, c)) {
                tile = c.tile;
                split_target = c.split;
            }
            tune_key = k;
        }
        const int64_t nt = tile == 128 ? t128 : t64;
        const int bk = (sizeof(T) == 8 && tile == 128) ? 8 : 16;
        for (int id = 0; id < (int)descs.size(); ++id) {
            const auto& d = descs[id];
            const int steps = (std::max(d.K, 0) + bk - 1) / bk + (std::max(d.K2, 0) + bk - 1) / bk;
            int S = 1;
            if (split_target > 0 && nt < (int64_t)split_target * CUS / 2)
                S = std::max(1, std::min<int>({(int)((split_target * CUS + nt - 1) / nt), steps / 8, max_split}));
            const int tm = (d.M + tile - 1) / tile, tn = (d.N + tile - 1) / tile;
            for (int i = 0; i < tm; ++i)
                for (int j = 0; j < tn; ++j) {
                    if (S == 1) {
                        tiles.push_back({id, i, j, 0, 1, 0});
                        continue;
                    }
                    const int pbase = (int)(ws_elems / ((int64_t)tile * tile));
                    for (int sp = 0; sp < S; ++sp) tiles.push_back({id, i, j, sp, S, pbase});
                    slots.push_back({id, i, j, 0, S, pbase});
                    ws_elems += (int64_t)S * tile * tile;
                }
        }
    }
    int kernel_role() const {
        return role >= 0 ? role
             : (prof_cls == RSD_PROF_FACTOR_GEMM_F64 || prof_cls == RSD_PROF_FACTOR_GEMM_F32) ? 0
             : (prof_cls == RSD_PROF_SOLVE_GEMM ? 2 : 1);
    }
    void run(hipStream_t s) const {
        if (tiles.empty()) return;
        const int r = kernel_role();
        hipEvent_t ta = nullptr, tb = nullptr;
        Tuner& tu = Tuner::get();
        if (tune_key && tu.recording()) {
            ta = tu.event();
            tb = tu.event();
            RSD_HIP(hipEventRecord(ta, s));
        }
        // profiled launches carry their timing events in the dispatch itself
        // (kernel start and end, no marker packets between the kernels)
        if (prof_active(prof_cls)) {
            ProfRec rec{prof_cls, g_prof.get(), g_prof.get(), flops, bytes, (int64_t)tiles.size()};
            launch_gemm<T>(d_descs, d_tiles, (int)tiles.size(), tile, d_ws, -wg_waves, s, r, rec.a, rec.b);
            g_prof.add(rec);
            if (!slots.empty()) {
                ProfRec red{prof_cls, g_prof.get(), g_prof.get(), 0, 0, (int64_t)slots.size()};
                launch_gemm<T>(d_descs, d_slots, (int)slots.size(), tile, d_ws, 1, s, r, red.a, red.b);
                g_prof.add(red);
            }
        } else {
            launch_gemm<T>(d_descs, d_tiles, (int)tiles.size(), tile, d_ws, -wg_waves, s, r);
            if (!slots.empty()) launch_gemm<T>(d_descs, d_slots, (int)slots.size(), tile, d_ws, 1, s, r);
        }
        if (ta) {
            RSD_HIP(hipEventRecord(tb, s));
            tu.record(tune_key, ta, tb);
        }
    }
};

template <typename T>
static GemmDesc<T> gdesc(int M, int N, int K, const T* A, int lda, int tA, const T* B, int ldb,
                         int tB, T* C, int ldc, T alpha, T beta) {
    GemmDesc<T> d;
    std::memset(&d, 0, sizeof(d));
    d.M = M; d.N = N; d.K = K; d.K2 = 0;
    d.A = A; d.lda = lda; d.tA = tA;
    d.B = B; d.ldb = ldb; d.tB = tB;
    d.A2 = nullptr; d.B2 = nullptr; d.lda2 = 1; d.ldb2 = 1;
    d.C = C; d.ldc = ldc;
    d.alpha = alpha; d.beta = beta;
    d.zc0 = d.zc1 = 0;
    d.guard = nullptr;
    return d;
}

// Pinned staging block held until its copy has completed (the holder's
// owner drains the stream first).
struct PinnedBlock {
    void* p = nullptr;
    size_t cap = 0;
    PinnedBlock() = default;
    PinnedBlock(const PinnedBlock&) = delete;
    PinnedBlock& operator=(const PinnedBlock&) = delete;
    ~PinnedBlock() { release(); }
    void release() {
        PinnedPool::get().give(p, cap);
        p = nullptr;
        cap = 0;
    }
};

// Uploads every batch of a list into one buffer and fixes their device
// pointers.  The batches of one list run one after another on one stream, so
// they share one split-K workspace, sized for the largest.  With `pinned`,
// the tables are staged in a pinned block (filled on `threads` threads) and
// the upload is asynchronous; the block must stay alive until the stream has
// passed the copy.
template <typename T>
static void upload_batches(DevBuf& buf, std::vector<GemmBatch<T>*>& bs, hipStream_t s, bool finalized = false,
                           PinnedBlock* pinned = nullptr, int threads = 1) {
    size_t nd = 0, nt = 0;
    int64_t max_ws = 0;
    size_t n_descs = 0;
    for (auto* b : bs) n_descs += b->descs.size();
    // large lists only: below that, waking the pool costs more than it saves
    const bool pooled = n_descs >= 16384;
    if (!finalized && !pooled) {
        for (auto* b : bs) b->finalize();
    } else if (!finalized) {
        // tile tables of the batches on the host pool (a reach error is
        // rethrown here)
        std::mutex emu;
        std::exception_ptr err;
        HostPool::get().parallel_for((int64_t)bs.size(), 4, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) {
                try {
                    bs[i]->finalize();
                } catch (...) {
                    std::lock_guard<std::mutex> lk(emu);
                    if (!err) err = std::current_exception();
                }
            }
        });
        if (err) std::rethrow_exception(err);
    }
    for (auto* b : bs) {
        nd += b->descs.size();
        nt += b->tiles.size() + b->slots.size();
        max_ws = std::max(max_ws, b->ws_elems);
    }
    auto up = [](size_t x, size_t a) { return (x + a - 1) / a * a; };
    const size_t o_tiles = up(nd * sizeof(GemmDesc<T>), 16);
    const size_t o_ws = up(o_tiles + nt * sizeof(TileRef), 256);
    const size_t host_bytes = o_tiles + nt * sizeof(TileRef);
    std::vector<unsigned char> pageable;
    unsigned char* host = nullptr;
    if (pinned && host_bytes > 0) {
        pinned->p = PinnedPool::get().take(host_bytes, pinned->cap);
        host = static_cast<unsigned char*>(pinned->p);
    } else {
        pageable.resize(host_bytes);
        host = pageable.data();
    }
    buf.alloc(o_ws + (size_t)max_ws * sizeof(T));
    unsigned char* base = buf.as<unsigned char>();
    std::vector<size_t> od(bs.size()), ot(bs.size());
    {
        size_t d = 0, t = o_tiles;
        for (size_t i = 0; i < bs.size(); ++i) {
            od[i] = d;
            ot[i] = t;
            d += bs[i]->descs.size() * sizeof(GemmDesc<T>);
            t += (bs[i]->tiles.size() + bs[i]->slots.size()) * sizeof(TileRef);
        }
    }
    auto fill = [&](size_t i) {
        GemmBatch<T>* b = bs[i];
        std::memcpy(host + od[i], b->descs.data(), b->descs.size() * sizeof(GemmDesc<T>));
        b->d_descs = reinterpret_cast<const GemmDesc<T>*>(base + od[i]);
        const size_t ts = b->tiles.size() * sizeof(TileRef);
        std::memcpy(host + ot[i], b->tiles.data(), ts);
        b->d_tiles = reinterpret_cast<const TileRef*>(base + ot[i]);
        std::memcpy(host + ot[i] + ts, b->slots.data(), b->slots.size() * sizeof(TileRef));
        b->d_slots = reinterpret_cast<const TileRef*>(base + ot[i] + ts);
        b->d_ws = reinterpret_cast<T*>(base + o_ws);
    };
    if (threads > 1 && bs.size() > 1) {
        std::atomic<size_t> next{0};
        auto work = [&]() {
            for (size_t i = next++; i < bs.size(); i = next++) fill(i);
        };
        run_on_threads(threads, work);
    } else if (pooled) {
        HostPool::get().parallel_for((int64_t)bs.size(), 4, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) fill((size_t)i);
        });
    } else {
        for (size_t i = 0; i < bs.size(); ++i) fill(i);
    }
    if (host_bytes > 0) RSD_HIP(hipMemcpyAsync(buf.p, host, host_bytes, hipMemcpyHostToDevice, s));
}

constexpr int GJ_NB = 64;   // Gauss-Jordan panel width (matches k_gj)

// The Gauss-Jordan kernel addresses its block with 32-bit byte offsets.
template <typename T>
static void check_gj_block(const GJDesc<T>& g) {
    // the pivot kernel addresses 64 rows x 64 columns from one descriptor base
    const int64_t bytes = (int64_t)sizeof(T) * ((int64_t)GJ_NB + (int64_t)GJ_NB * g.ld);
    if (bytes + 16 > (int64_t)GEMM_MAX_OPERAND_BYTES)
        throw Error(RSD_EINVAL, "matrix block too large for the Gauss-Jordan kernel (leading dimension)");
}

// ----------------------------------------------------------------------------
// per-level execution plan (one precision per level)
// ----------------------------------------------------------------------------
template <typename T>
struct LevelExec {
    int level = 0;
    std::vector<int> ids;        // box ids
    int max_m = 0, max_k = 0, max_r = 0, max_chunks = 0;
    GemmBatch<T> g_sr, g_rr, g_E;
    std::vector<GemmBatch<T>> g_gj;   // one per Gauss-Jordan step
    GemmBatch<T> g_top;               // root only: unused placeholder
    std::vector<GJDesc<T>> gj;        // per box
    const GJDesc<T>* d_gj = nullptr;
    std::vector<GemmBatch<T>> g_topgj;   // root: inversion of the remaining block
    std::vector<GJDesc<T>> topgj;
    const GJDesc<T>* d_topgj = nullptr;
    int top_chunks = 0;
    int gj_steps = 0, topgj_steps = 0;
};

template <typename T>
struct SolveLevel {
    GemmBatch<T> up1, up2, dn1, dn2, top;
};

struct SolvePlan {
    int nrhs = 0;
    DevBuf V32, V64, Y32, Y64, tmp, in, out, gemm32, gemm64;
    DevBuf refine_work, refine_norms;   // refinement vectors, allocated on first use
    std::vector<SolveLevel<float>> L32;
    std::vector<SolveLevel<double>> L64;
    hipGraphExec_t sweeps = nullptr;    // the sweeps between leaf gather and scatter, captured once
    bool sweeps_failed = false;         // capture or instantiation refused: launched one by one
    SolvePlan() = default;
    SolvePlan(const SolvePlan&) = delete;
    SolvePlan& operator=(const SolvePlan&) = delete;
    ~SolvePlan() {
        if (sweeps) (void)hipGraphExecDestroy(sweeps);
    }
};

struct Factor {
    Plan plan;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int precision = RSD_PREC_FP64;
    int max_refine = 0;
    double refine_tol = 0;
    double tol = 0;
    int64_t N = 0, nx = 0, ny = 0;
    double h = 0;
    int cplx = 0;
    int top = 0;                    // root level
    int flags = 0;
    KernelDesc kd{};                // the factored matrix (generation kernels)
    KernelDesc kd_res{};            // the exact operator (residuals, rsd_matvec)
    std::vector<int> level_prec;    // 0 fp64, 1 fp32
    // device tables
    DevBuf d_boxes, d_layouts, d_lu, d_lv, d_srcc, d_srci, d_inv, d_perm, d_ident, d_a, d_sb,
        d_level_ids, d_err, d_table, d_spec, d_fftwork, d_flag;
    DevBuf d_interp;                // per layout, 4 x (kept rank, |R_11| reference, sectors)
    std::vector<int8_t> layout_damped;   // per layout: interpolation solved as damped least squares
    int fft_mx = 0, fft_my = 0;     // circulant sizes of the FFT product (0: not set up)
    std::mutex use_mu;              // solves and products of one factor run one at a time
    std::vector<int> level_id_off;
    bool dedup = false;                         // one block per (level, layout)
    std::vector<std::vector<int>> build_levels; // boxes built per level (representatives)
    std::vector<int> build_id_off;
    DevBuf F64, F32, T64, T32, SR, SC, gemm64, gemm32, gemm64e, gemm32e, gj64, gj32;
    hipStream_t qr_stream[2] = {nullptr, nullptr};   // interpolation chains run here
    std::vector<hipEvent_t> tmp_events;
    hipEvent_t build_ev[2] = {nullptr, nullptr};     // start / end of the device build
    std::vector<std::unique_ptr<DevBuf>> scratch;   // freed after the build
    std::vector<LevelExec<double>> L64;
    std::vector<LevelExec<float>> L32;
    std::vector<BoxDev> hboxes;
    std::vector<LayoutDev> hlayouts;
    std::map<int, std::unique_ptr<SolvePlan>> solve_plans;
    int* h_flag = nullptr;          // pinned word for the right-hand side check
    std::vector<GemmBatch<double>*> tables64;   // the level products, uploaded by enqueue_single
    std::vector<GemmBatch<float>*> tables32;
    PinnedBlock staged[6];          // their pinned staging, returned by build_finish
    std::vector<int> exec_index;    // level -> index into L64 or L32
    std::vector<int> layout_level;  // layout -> level of its boxes
    double gemm_flops = 0;          // flops of the level products
    int layers = 0;
    rsd_factor_stats stats{};
    ~Factor() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (auto q : qr_stream)
            if (q) (void)hipStreamSynchronize(q);
        {
            // every stream that touched the factor's memory has drained
            IdleScope idle;
            solve_plans.clear();
            scratch.clear();
            for (DevBuf* b : {&d_boxes, &d_layouts, &d_lu, &d_lv, &d_srcc, &d_srci, &d_inv, &d_perm,
                              &d_ident, &d_a, &d_sb, &d_level_ids, &d_err, &d_table, &d_spec, &d_fftwork,
                              &d_flag, &d_interp, &F64, &F32, &T64, &T32, &SR, &SC, &gemm64, &gemm32, &gemm64e, &gemm32e, &gj64, &gj32})
                b->release();
        }
        PinnedWords::get().give(h_flag);
        for (auto e : tmp_events) (void)hipEventDestroy(e);
        for (auto e : build_ev)
            if (e) (void)hipEventDestroy(e);
        for (auto q : qr_stream) StreamPool::get().give(device, q);
        if (own_stream) StreamPool::get().give(device, stream);
    }
    DevBuf& tmp() {
        scratch.push_back(std::make_unique<DevBuf>());
        return *scratch.back();
    }
    const int* ids(int t) const { return d_level_ids.as<int>() + level_id_off[t]; }
    const int* bids(int t) const { return d_level_ids.as<int>() + build_id_off[t]; }
};

template <typename T> static T* Fbase(Factor& f);
template <> double* Fbase<double>(Factor& f) { return f.F64.as<double>(); }
template <> float* Fbase<float>(Factor& f) { return f.F32.as<float>(); }
template <typename T> static T* Tbase(Factor& f);
template <> double* Tbase<double>(Factor& f) { return f.T64.as<double>(); }
template <> float* Tbase<float>(Factor& f) { return f.T32.as<float>(); }

// ----------------------------------------------------------------------------
// interpolation matrices for every box type (one problem per layout)
// ----------------------------------------------------------------------------
// Truncation threshold of the float64 interpolation problems.  With two or
// more skeleton layers the proxy problems are numerically full rank down to
// 1e-10 relative (measured: rank = k at every level of the benchmark grids),
// so they are truncated at min(tol, 1e-10): every column is kept and T is the
// problem's unique least-squares solution, at least as accurate as one
// truncated at a looser tol.  With one layer the truncation is active and
// follows tol.
// Truncation threshold of the float64 interpolation problems.  The skeleton
// is fixed by the layers, so truncation only zeroes rows of T; it is kept
// where the proxy problems are (nearly) full rank: 1e-10 with two layers,
// 1e-12 with three.  The window pivoting decides truncation per sub-panel
// and stops earlier than greedy column pivoting once many columns fall
// below the threshold (three layers at 1e-10: a few hundred of 1116 columns
// kept, T entries 10^3 times too large, the solve wrong), which these
// thresholds avoid; the truncation record of every box type
// (rsd_factor_interp_info) exposes the kept ranks.
static double interp_tol64(const Factor& f) {
    if (f.layers >= 3) return std::min(f.tol, 1e-12);
    return f.layers >= 2 ? std::min(f.tol, 1e-10) : f.tol;
}

// Skeleton layers m: from tol (layers_for_tol), one more for the oscillatory
// Helmholtz kernel below tol 1e-6 (Sec. 5.3: more layers than for Laplace
// at high accuracy), at most three.
static int default_layers(double tol, int kernel_type) {
    const int m = layers_for_tol(tol);
    return kernel_type == RSD_KERNEL_HELMHOLTZ && tol < 1e-6 ? std::min(m + 1, 3) : m;
}

// The symmetry split is used where the proxy problems are full rank or
// nearly (float64 interpolation truncated at 1e-9 or below), so the sector
// solutions are the whole problem's least-squares solution up to rounding.
// Where truncation decides the rank (float32 interpolation, one layer) the
// whole problem is solved: the window pivoting's truncation test sees only a
// sub-panel's columns, and on the small sector problems that stops too early.
// (Three layers at 1e-12: the largest types keep a few percent fewer columns
// in sectors than whole, with interpolation residuals still near 1e-14.)
static bool split_sym(const Factor& f, const IDProblem& I, int prec) {
    return I.sym && prec == 0 && interp_tol64(f) <= 1e-9;
}

// Precision of the interpolation problems of a level (0 float64, 1 float32).
static int interp_prec(const Factor& f, int level) {
    return f.level_prec[level] && (f.flags & RSD_FLAG_FP32_INTERP) ? 1 : 0;
}

// The sector problems of one interpolation problem, appended to a chain's
// problem list: nsec consecutive entries that share the group start g0 (the
// list index of the first) and size gn = nsec, labelled by the group's
// characters in order -- all four for two reflections, 0 and 1 for the u
// reflection alone, 0 and 2 for the v reflection alone -- or one entry with
// sec = -1 when the problem is solved whole.  Sizes are the problem's divided
// by nsec; the caller fills in the offsets.
static void append_sector_problems(std::vector<QRProblemDev>& qp, const IDProblem& I, bool sym) {
    const int nsec = sym ? I.nsec() : 1;
    const int g0 = (int)qp.size();
    for (int sc = 0; sc < nsec; ++sc) {
        QRProblemDev q{};
        q.p = I.p / nsec;
        q.pz = q.p;
        q.k = I.k / nsec;
        q.r = I.r / nsec;
        q.sec = sym ? (I.grp == 2 ? 2 * sc : sc) : -1;
        q.g0 = g0;
        q.gn = nsec;
        qp.push_back(q);
    }
}

// Checks the sector groups of a chain's problem list before any kernel reads
// them: every problem's group [g0, g0 + gn) lies inside the list, contains the
// problem, and is made of gn consecutive sectors of one interpolation problem
// (owner[i]: the member problem i came from) with distinct characters of one
// group (gn = 4: 0..3; gn = 2: {0, 1} or {0, 2}; gn = 1: unsplit, sec = -1).
static void check_sector_groups(const std::vector<QRProblemDev>& qp, const std::vector<int>& owner) {
    const int np = (int)qp.size();
    if ((int)owner.size() != np) throw Error(RSD_EINVAL, "interpolation groups: owner table size");
    for (int i = 0; i < np; ++i) {
        const QRProblemDev& q = qp[i];
        const bool ok_range = q.gn >= 1 && q.g0 >= 0 && q.g0 + q.gn <= np && i >= q.g0 && i < q.g0 + q.gn;
        if (!ok_range)
            throw Error(RSD_EINVAL, "interpolation problem " + std::to_string(i) + ": sector group [" +
                                        std::to_string(q.g0) + ", " + std::to_string(q.g0 + q.gn) +
                                        ") outside the list of " + std::to_string(np));
        if (q.gn != 1 && q.gn != 2 && q.gn != 4)
            throw Error(RSD_EINVAL, "interpolation problem " + std::to_string(i) + ": group of " +
                                        std::to_string(q.gn) + " sectors");
        unsigned seen = 0;
        for (int j = q.g0; j < q.g0 + q.gn; ++j) {
            const QRProblemDev& o = qp[j];
            const bool same = owner[j] == owner[i] && o.g0 == q.g0 && o.gn == q.gn && o.p == q.p &&
                              o.k == q.k && o.r == q.r;
            const bool lab = q.gn == 1 ? o.sec == -1 : (o.sec >= 0 && o.sec < 4);
            if (!same || !lab || (lab && q.gn > 1 && (seen >> o.sec) & 1u))
                throw Error(RSD_EINVAL, "interpolation problem " + std::to_string(i) +
                                            ": sectors of its group are not one problem's");
            if (q.gn > 1) seen |= 1u << o.sec;
        }
        const bool chars = q.gn == 1 || (q.gn == 4 && seen == 0xFu) ||
                           (q.gn == 2 && (seen == 0x3u || seen == 0x5u));
        if (!chars)
            throw Error(RSD_EINVAL, "interpolation problem " + std::to_string(i) +
                                        ": group characters do not form one reflection group");
    }
    // a member's problems form exactly one group
    for (int i = 0; i < np;) {
        const QRProblemDev& q = qp[i];
        if (q.g0 != i) throw Error(RSD_EINVAL, "interpolation groups are not consecutive");
        for (int j = i + q.gn; j < np && owner[j] == owner[i]; ++j)
            throw Error(RSD_EINVAL, "interpolation problem split across groups");
        i += q.gn;
    }
}

// One interpolation problem of a chain: the box type `id` of factor `f`,
// whose level `level` needs its T; `tag` is reported when it is solved.
struct ChainMember {
    Factor* f;
    int id, level, tag;
};

// One chain of interpolation problems: every problem of the chain advances
// window by window through the same launches on the chain's stream, and the
// problems finished after a window get their back substitution right after
// it, on the same stream.  The problems may belong to several factors (a
// batch of grids): one launch then serves the same window of all of them.
template <typename T>
struct QRChain {
    Factor* f = nullptr;               // first member's factor (tolerance, kernel, T arena)
    bool several = false;              // problems of several factors: every solution staged
    std::vector<std::unique_ptr<DevBuf>>* owner = nullptr;   // holds the chain's device buffers
    hipStream_t s = nullptr;
    std::vector<QRProblemDev> qp;
    std::vector<int> prob_tag;         // the member's tag of every (sector) problem
    int S = 0, np = 0, max_k = 0, max_n = 0, max_nch = 0, max_subs = 0;
    DevBuf *dA = nullptr, *daux = nullptr, *diaux = nullptr, *dws = nullptr, *dsec = nullptr;
    // the chain's tables, uploaded together (one copy)
    const QRProblemDev* q_dev = nullptr;
    const int *list_dev = nullptr, *solve_dev = nullptr, *orb_dev = nullptr, *refl_dev = nullptr;
    const SymCombineDesc* comb_dev = nullptr;
    std::vector<int64_t> sym_sec0;     // staging-arena offset of every staged problem
    std::vector<int> staged_prec;      // precision of its T arena (0 float64, 1 float32)
    std::vector<int> comb_off[2];      // staging descriptors per window, per destination precision
    int comb_max_kr = 0;
    std::vector<GemmBatch<T>> g1, gt, g2;
    std::vector<std::vector<GemmBatch<T>>> gsolve;
    static constexpr int NWIDTH = 5;   // sub-panel width classes 16, 8, 4, 2, 1
    std::vector<int> lists[NWIDTH];
    int off[NWIDTH] = {0, 0, 0, 0, 0}, maxp[NWIDTH] = {0, 0, 0, 0, 0};
    std::vector<int> sflat, soff;
    bool any_damp = false;
    double flops = 0, bytes = 0;

    DevBuf& tmp() {
        owner->push_back(std::make_unique<DevBuf>());
        return *owner->back();
    }

    // members: the problems, each with its factor, level and tag (reported by
    // window() when it is solved).  With members of several factors every
    // solution goes through the staging arena, whose combine step writes it
    // into its own factor's T arena.
    void setup(const std::vector<ChainMember>& members, bool of_several,
               std::vector<std::unique_ptr<DevBuf>>& buffers, hipStream_t stream) {
        f = members.front().f;
        several = of_several;
        owner = &buffers;
        s = stream;
        std::vector<int64_t> offA;
        std::vector<double> lgh;
        std::vector<Factor*> staged_fac;
        std::vector<int> pof, kof, rof, zoff, xoff, zu, zv, xu, xv, geo;
        int64_t A_el = 0, aux_el = 0, iaux_el = 0, ws_el = 0, sec_el = 0;
        int max_pn = 0, max_r = 0;
        // a symmetric interpolation problem becomes its four sector problems
        // (orbit representatives; their solutions are combined into T after
        // the back substitution)
        // staged solutions: symmetric problems (sectors, then combined) and
        // problems whose level keeps T in another precision than this chain
        std::vector<int> staged_ids, staged_sym;
        std::vector<int> owner;            // member index of every (sector) problem
        for (size_t pi = 0; pi < members.size(); ++pi) {
            Factor& F = *members[pi].f;
            const int id = members[pi].id, lev = members[pi].level;
            const IDProblem& I = F.plan.idps[id];
            const Layout& L = F.plan.layouts[I.layout];
            const int chain_prec = std::is_same<T, double>::value ? 0 : 1;
            const bool sym = split_sym(F, I, chain_prec);
            const bool convert = F.level_prec[lev] != chain_prec;
            const bool staged = sym || convert || several;
            const int nsec = sym ? I.nsec() : 1;
            const int64_t sec0 = sec_el;
            if (staged) {
                sec_el += (int64_t)I.k * I.r / nsec;
                staged_ids.push_back(id);
                staged_sym.push_back(sym ? 1 : 0);
                sym_sec0.push_back(sec0);
                staged_prec.push_back(F.level_prec[lev]);
                staged_fac.push_back(&F);
            }
            // the sectors (characters of the reflection group, bit 0: u, bit 1: v)
            // are appended with their group; offsets follow
            const size_t base = qp.size();
            append_sector_problems(qp, I, sym);
            // truncation, or damped least squares where truncation would be
            // active (three layers in float64, float32 interpolation): the
            // window pivoting tests truncation per sub-panel and stops too
            // early there, the damped problem needs no truncation
            const bool f32 = !std::is_same<T, double>::value;
            const double plain_tol = f32 ? std::max(F.tol, 1e-6) : interp_tol64(F);
            const double damp_rel = f32 ? std::max(F.tol, 1e-6) : F.tol;
            const bool want_damp = (f32 || F.layers >= 3 || F.cplx) && !(F.flags & RSD_FLAG_NO_DAMPING);
            for (int sc = 0; sc < nsec; ++sc) {
                QRProblemDev& q = qp[base + sc];
                q.staged = staged ? 1 : 0;
                q.ttol = plain_tol;
                if (want_damp && qr_panel_width(q.pz + q.k, (int)sizeof(T)) > 0) {
                    q.p = q.pz + q.k;
                    q.damp = damp_rel;
                    q.ttol = 1e-3 * damp_rel;    // a guard only: no pivot falls below damp |R_11|
                    any_damp = true;
                } else if (want_damp && F.cplx) {
                    // complex factors are not accurate with truncation alone (their
                    // least-squares solutions turn ill-conditioned)
                    throw Error(RSD_EINVAL, "interpolation problem of a " + std::to_string(L.ax) + "x" +
                                                std::to_string(L.ay) + " box type (" + std::to_string(q.pz) +
                                                " x " + std::to_string(q.k) +
                                                ") too large for the damped least squares; use fewer interface "
                                                "points or RSD_FLAG_FP32_INTERP");
                }
                if ((size_t)I.layout < F.layout_damped.size()) F.layout_damped[I.layout] = q.damp > 0 ? 1 : 0;
                q.nb = qr_panel_width(q.p, (int)sizeof(T));
                if (q.nb == 0) throw Error(RSD_EINVAL, "box too large for the interpolation kernels");
                const int n = q.k + q.r;
                const int nch = (q.p + QR_RC - 1) / QR_RC;
                q.offA = A_el;
                q.offT = staged ? sec0 + (int64_t)sc * q.k * q.r : F.hlayouts[I.layout].offT;
                q.offAux = aux_el;
                q.offIaux = iaux_el;
                q.rec = F.d_interp.as<double>() + 12 * (int64_t)I.layout + 3 * sc;
                q.offV = ws_el;
                q.offTmp = q.offV + (int64_t)q.p * QR_WIN;
                q.offW = q.offTmp + (int64_t)q.p * 2 * QR_WIN;
                q.offWs = q.offW + (int64_t)nch * QR_WIN * (QR_WIN + n);
                ws_el = q.offWs + (int64_t)QR_WIN * (QR_WIN + n);
                A_el += (int64_t)q.p * n;
                aux_el += 2 * q.k + QR_NB * QR_NB + QR_WIN * QR_WIN + 8;
                iaux_el += q.k + 8 + 4 * QR_WIN;
                owner.push_back((int)pi);
                prob_tag.push_back(members[pi].tag);
                lgh.push_back(F.kd.logh);
                offA.push_back(q.offA);
                pof.push_back(q.p); kof.push_back(q.k); rof.push_back(q.r);
                zoff.push_back((int)zu.size());
                xoff.push_back((int)xu.size());
                if (sym) {
                    zu.insert(zu.end(), I.zr_u.begin(), I.zr_u.end());
                    zv.insert(zv.end(), I.zr_v.begin(), I.zr_v.end());
                    xu.insert(xu.end(), I.skr_u.begin(), I.skr_u.end());
                    xu.insert(xu.end(), I.rsr_u.begin(), I.rsr_u.end());
                    xv.insert(xv.end(), I.skr_v.begin(), I.skr_v.end());
                    xv.insert(xv.end(), I.rsr_v.begin(), I.rsr_v.end());
                } else {
                    zu.insert(zu.end(), I.zu.begin(), I.zu.end());
                    zv.insert(zv.end(), I.zv.begin(), I.zv.end());
                    xu.insert(xu.end(), L.u.begin(), L.u.end());
                    xv.insert(xv.end(), L.v.begin(), L.v.end());
                }
                geo.push_back(L.ax); geo.push_back(L.ay); geo.push_back(q.sec); geo.push_back(sym ? I.grp : 0);
                geo.push_back(q.pz);
                max_pn = std::max(max_pn, q.p * n);
                max_k = std::max(max_k, q.k);
                max_r = std::max(max_r, q.r);
                max_n = std::max(max_n, n);
                max_nch = std::max(max_nch, nch);
                S = std::max(S, (q.k + QR_WIN - 1) / QR_WIN);
            }
        }
        np = (int)qp.size();
        check_sector_groups(qp, owner);
        DevBuf& dgemm = tmp();
        dA = &tmp(); daux = &tmp(); diaux = &tmp(); dws = &tmp(); dsec = &tmp();
        HostPack pk;
        const size_t o_logh = several ? pk.add(lgh) : 0;
        dA->alloc(A_el * sizeof(T));
        daux->alloc(aux_el * sizeof(T));
        diaux->alloc(iaux_el * sizeof(int));
        dws->alloc(ws_el * sizeof(T));
        dsec->alloc(std::max<int64_t>(sec_el, 1) * sizeof(T));
        const size_t o_q = pk.add(qp), o_offA = pk.add(offA), o_p = pk.add(pof), o_k = pk.add(kof),
                     o_r = pk.add(rof), o_zo = pk.add(zoff), o_zu = pk.add(zu), o_zv = pk.add(zv),
                     o_xo = pk.add(xoff), o_xu = pk.add(xu), o_xv = pk.add(xv), o_geo = pk.add(geo);
        size_t o_comb = 0, o_orb = 0, o_refl = 0;
        // staged solutions into the T arenas (combined for symmetric types,
        // converted to the level's precision), grouped by the window after
        // which their problems are complete, one list per destination precision
        {
            std::vector<int> orb, refl;
            std::vector<std::vector<SymCombineDesc>> by_win[2];
            for (size_t si = 0; si < staged_ids.size(); ++si) {
                Factor& F = *staged_fac[si];
                const IDProblem& I = F.plan.idps[staged_ids[si]];
                const bool sym = staged_sym[si] != 0;
                SymCombineDesc cd;
                cd.offT = F.hlayouts[I.layout].offT;
                cd.dst = nullptr;
                if (several)
                    cd.dst = staged_prec[si] ? static_cast<void*>(Tbase<float>(F) + cd.offT)
                                             : static_cast<void*>(Tbase<double>(F) + cd.offT);
                cd.offS = sym_sec0[si];
                cd.k = I.k;
                cd.r = I.r;
                cd.sym = sym ? 1 : 0;
                cd.grp = sym ? I.grp : 0;
                cd.off_sk = (int)orb.size();
                cd.off_rs = (int)orb.size();
                if (sym) {
                    orb.insert(orb.end(), I.sk_orb.begin(), I.sk_orb.end());
                    refl.insert(refl.end(), I.sk_g.begin(), I.sk_g.end());
                    cd.off_rs = (int)orb.size();
                    orb.insert(orb.end(), I.rs_orb.begin(), I.rs_orb.end());
                    refl.insert(refl.end(), I.rs_g.begin(), I.rs_g.end());
                }
                const int kq = sym ? I.k / I.nsec() : I.k;
                const int w = (kq + QR_WIN - 1) / QR_WIN - 1;
                auto& bw = by_win[staged_prec[si]];
                if ((int)bw.size() <= w) bw.resize(w + 1);
                bw[w].push_back(cd);
                comb_max_kr = std::max(comb_max_kr, I.k * I.r);
            }
            std::vector<SymCombineDesc> flatc;
            for (int pr = 0; pr < 2; ++pr) {
                comb_off[pr].assign(S + 1, 0);
                for (int w = 0; w < S; ++w) {
                    comb_off[pr][w] = (int)flatc.size();
                    if (w < (int)by_win[pr].size()) flatc.insert(flatc.end(), by_win[pr][w].begin(), by_win[pr][w].end());
                }
                comb_off[pr][S] = (int)flatc.size();
            }
            orb.push_back(0);
            refl.push_back(0);
            o_comb = pk.add(flatc);
            o_orb = pk.add(orb);
            o_refl = pk.add(refl);
        }
        // trailing-update products of every window, guarded by the problem's skip flag
        T* Ab = dA->as<T>();
        T* W = dws->as<T>();
        g1.resize(S); gt.resize(S); g2.resize(S);
        for (size_t i = 0; i < qp.size(); ++i) {
            const QRProblemDev& q = qp[i];
            const int n = q.k + q.r;
            const int* guard = diaux->as<int>() + q.offIaux + q.k + 1;
            T* V = W + q.offV;
            T* Wp = W + q.offW;
            T* Ws = W + q.offWs;
            T* Tw = daux->as<T>() + q.offAux + 2 * q.k + QR_NB * QR_NB;
            const int64_t chunk = (int64_t)QR_WIN * (QR_WIN + n);
            for (int sw = 0; sw * QR_WIN < q.k; ++sw) {
                const int J0 = sw * QR_WIN, WO = std::min(QR_WIN, q.k - J0);
                const int ntrail = n - J0 - WO, pr = q.p - J0;
                const int nch = (pr + QR_RC - 1) / QR_RC;
                for (int c = 0; c < nch; ++c) {
                    const int r0 = J0 + c * QR_RC, kr = std::min(QR_RC, q.p - r0);
                    GemmDesc<T> da = gdesc<T>(QR_WIN, QR_WIN, kr, V + r0, q.p, 1, V + r0, q.p, 0,
                                              Wp + c * chunk, QR_WIN, T(1), T(0));
                    da.guard = guard;
                    g1[sw].add(da);
                    if (ntrail > 0) {
                        GemmDesc<T> db = gdesc<T>(QR_WIN, ntrail, kr, V + r0, q.p, 1,
                                                  Ab + q.offA + r0 + (int64_t)(J0 + WO) * q.p, q.p, 0,
                                                  Wp + c * chunk + QR_WIN * QR_WIN, QR_WIN, T(1), T(0));
                        db.guard = guard;
                        g1[sw].add(db);
                    }
                }
                if (ntrail > 0) {
                    GemmDesc<T> dt = gdesc<T>(QR_WIN, ntrail, QR_WIN, Tw, QR_WIN, 1, Ws + QR_WIN * QR_WIN,
                                              QR_WIN, 0, Wp, QR_WIN, T(1), T(0));
                    dt.guard = guard;
                    gt[sw].add(dt);
                    GemmDesc<T> d2 = gdesc<T>(pr, ntrail, QR_WIN, V + J0, q.p, 0, Wp, QR_WIN, 0,
                                              Ab + q.offA + J0 + (int64_t)(J0 + WO) * q.p, q.p, T(-1), T(1));
                    d2.guard = guard;
                    g2[sw].add(d2);
                }
            }
            const double p = q.p, k = q.k, r = q.r;
            flops += 2 * k * k * (p - k / 3) + 4 * p * k * r - 2 * k * k * r + k * k * r;
            bytes += sizeof(T) * (2 * p * (k + r) + k * r);
        }
        // problems grouped by the window after which they are complete
        std::vector<std::vector<int>> done_after(S);
        for (int i = 0; i < np; ++i) done_after[(qp[i].k + QR_WIN - 1) / QR_WIN - 1].push_back(i);
        // blocked back substitution per group: after solving 64-row block I in
        // place, the rows above take  B[0:64I, :] -= R[0:64I, block I] X_I
        gsolve.resize(S);
        for (int sw = 0; sw < S; ++sw) {
            int nblk = 0;
            for (int i : done_after[sw]) nblk = std::max(nblk, (qp[i].k + 63) / 64);
            gsolve[sw].resize(nblk);
            for (int i : done_after[sw]) {
                const QRProblemDev& q = qp[i];
                const int nb_i = (q.k + 63) / 64;
                T* Aq = Ab + q.offA;
                for (int st = 0; st < nb_i; ++st) {
                    const int I = nb_i - 1 - st;
                    if (I == 0) continue;
                    const int i0 = I * 64, kb = std::min(64, q.k - i0);
                    gsolve[sw][st].add(gdesc<T>(i0, q.r, kb, Aq + (int64_t)i0 * q.p, q.p, 0,
                                                Aq + (int64_t)q.k * q.p + i0, q.p, 0,
                                                Aq + (int64_t)q.k * q.p, q.p, T(-1), T(1)));
                }
            }
        }
        // no split K: a problem's solution must not depend on the other
        // problems of its chain (a grid built alone or in a batch gets the
        // same bits)
        std::vector<GemmBatch<T>*> all;
        for (int sw = 0; sw < S; ++sw) { all.push_back(&g1[sw]); all.push_back(&gt[sw]); all.push_back(&g2[sw]); }
        for (auto& v : gsolve)
            for (auto& b : v) all.push_back(&b);
        for (auto* b : all) b->max_split = 1;
        upload_batches<T>(dgemm, all, s);
        // sub-panel width classes
        const int widths[NWIDTH] = {16, 8, 4, 2, 1};
        for (int i = 0; i < np; ++i) {
            int c = 0;
            while (widths[c] != qp[i].nb) ++c;
            lists[c].push_back(i);
            maxp[c] = std::max(maxp[c], qp[i].p);
        }
        std::vector<int> flat;
        for (int c = 0; c < NWIDTH; ++c) {
            off[c] = (int)flat.size();
            flat.insert(flat.end(), lists[c].begin(), lists[c].end());
            if (!lists[c].empty()) max_subs = std::max(max_subs, QR_WIN / widths[c]);
        }
        const size_t o_list = pk.add(flat);
        soff.assign(S + 1, 0);
        for (int sw = 0; sw < S; ++sw) {
            soff[sw] = (int)sflat.size();
            sflat.insert(sflat.end(), done_after[sw].begin(), done_after[sw].end());
        }
        soff[S] = (int)sflat.size();
        const size_t o_solve = pk.add(sflat);
        DevBuf& dpk = tmp();
        dpk.alloc(pk.bytes.size());
        RSD_HIP(hipMemcpyAsync(dpk.p, pk.bytes.data(), pk.bytes.size(), hipMemcpyHostToDevice, s));
        auto at = [&](size_t o) { return static_cast<const void*>(dpk.as<unsigned char>() + o); };
        q_dev = static_cast<const QRProblemDev*>(at(o_q));
        list_dev = static_cast<const int*>(at(o_list));
        solve_dev = static_cast<const int*>(at(o_solve));
        comb_dev = static_cast<const SymCombineDesc*>(at(o_comb));
        orb_dev = static_cast<const int*>(at(o_orb));
        refl_dev = static_cast<const int*>(at(o_refl));
        auto ints = [&](size_t o) { return static_cast<const int*>(at(o)); };
        launch_proxy_matrix<T>(Ab, static_cast<const int64_t*>(at(o_offA)), ints(o_p), ints(o_k), ints(o_r),
                               ints(o_zo), ints(o_zu), ints(o_zv), ints(o_xo), ints(o_xu), ints(o_xv),
                               ints(o_geo), several ? static_cast<const double*>(at(o_logh)) : nullptr, np,
                               max_pn, f->kd, s);
        launch_qr_init<T>(Ab, daux->as<T>(), diaux->as<int>(), q_dev, np, max_k, s);
        if (any_damp) launch_qr_damp<T>(Ab, daux->as<T>(), diaux->as<int>(), q_dev, np, max_k, s);
    }

    // Enqueues window sw.  For the problems that finish in it, the back
    // substitutions follow on the chain's stream, then an event: returned,
    // with the tag of every finished (sector) problem appended to `done`
    // (nullptr and nothing appended when no problem finishes).
    hipEvent_t window(int sw, std::vector<int>& done) {
        if (sw >= S) return nullptr;
        T* Ab = dA->as<T>();
        T* W = dws->as<T>();
        T* aux = daux->as<T>();
        int* iaux = diaux->as<int>();
        const QRProblemDev* q = q_dev;
        const int widths[NWIDTH] = {16, 8, 4, 2, 1};
        launch_qr_select<T>(Ab, aux, iaux, W, q, np, sw, max_k, s);
        launch_qr_move<T>(Ab, iaux, W, q, np, 0, s);
        launch_qr_move<T>(Ab, iaux, W, q, np, 1, s);
        for (int sub = 0; sub < max_subs; ++sub)
            for (int c = 0; c < NWIDTH; ++c) {
                if (lists[c].empty() || sub * widths[c] >= QR_WIN) continue;
                launch_qr_panel<T>(Ab, aux, iaux, W, q, list_dev + off[c], (int)lists[c].size(),
                                   widths[c], maxp[c], sw, sub, s);
                launch_qr_inner<T>(Ab, aux, iaux, W, q, list_dev + off[c], (int)lists[c].size(),
                                   widths[c], sw, sub, s);
            }
        g1[sw].run(s);
        launch_qr_wsum<T>(aux, iaux, W, q, np, sw, max_n, max_nch, s);
        gt[sw].run(s);
        g2[sw].run(s);
        launch_qr_norms<T>(Ab, aux, iaux, q, np, sw, max_k, s);
        const int ng = soff[sw + 1] - soff[sw];
        if (ng == 0) return nullptr;
        // back substitution for the problems finished in this window, on the
        // chain's stream
        int gr = 0;
        for (int g = soff[sw]; g < soff[sw + 1]; ++g) gr = std::max(gr, qp[sflat[g]].r);
        for (int st = 0; st < (int)gsolve[sw].size(); ++st) {
            launch_qr_trsm<T>(Ab, aux, iaux, Tbase<T>(*f), dsec->as<T>(), q, solve_dev + soff[sw], ng,
                              gr, st, s);
            gsolve[sw][st].run(s);
        }
        launch_sym_combine<T, double>(Tbase<double>(*f), dsec->as<T>(), comb_dev + comb_off[0][sw],
                                      comb_off[0][sw + 1] - comb_off[0][sw], orb_dev, refl_dev,
                                      comb_max_kr, s);
        launch_sym_combine<T, float>(Tbase<float>(*f), dsec->as<T>(), comb_dev + comb_off[1][sw],
                                     comb_off[1][sw + 1] - comb_off[1][sw], orb_dev, refl_dev,
                                     comb_max_kr, s);
        hipEvent_t solved;
        RSD_HIP(hipEventCreateWithFlags(&solved, hipEventDisableTiming));
        RSD_HIP(hipEventRecord(solved, s));
        for (int g = soff[sw]; g < soff[sw + 1]; ++g) done.push_back(prob_tag[sflat[g]]);
        return solved;
    }
};

// ----------------------------------------------------------------------------
// level plans
// ----------------------------------------------------------------------------
template <typename T>
static void plan_level(Factor& f, LevelExec<T>& L, int t, std::vector<GemmBatch<T>*>& all,
                       int64_t& sr_need, int64_t& sc_need) {
    Plan& P = f.plan;
    L.level = t;
    L.ids = f.build_levels.empty() ? P.levels[t] : f.build_levels[t];
    T* F = Fbase<T>(f);
    T* Tb = Tbase<T>(f);
    int64_t sr = 0, sc = 0;
    for (int id : L.ids) {
        const Box& b = P.boxes[id];
        const LayoutDev& LD = f.hlayouts[b.layout];
        const int k = b.k, r = b.r, m = k + r;
        L.max_m = std::max(L.max_m, m);
        L.max_k = std::max(L.max_k, k);
        L.max_r = std::max(L.max_r, r);
        T* Fb = F + b.offF;
        T* Fss = Fb;
        T* Fsr = Fb + (int64_t)k * m;
        T* Frs = Fb + k;
        T* Frr = Fb + k + (int64_t)k * m;
        const T* Tm = LD.offT >= 0 ? Tb + LD.offT : nullptr;
        if (r > 0 && Tm) {
            L.g_sr.add(gdesc<T>(k, r, k, Fss, m, 0, Tm, k, 0, Fsr, m, T(-1), T(1)));
            GemmDesc<T> d = gdesc<T>(r, r, k, Frs, m, 0, Tm, k, 0, Frr, m, T(-1), T(1));
            d.K2 = k; d.A2 = Tm; d.lda2 = k; d.tA2 = 1; d.B2 = Fsr; d.ldb2 = m; d.tB2 = 0;
            L.g_rr.add(d);
        }
        if (r > 0) {
            GJDesc<T> g;
            g.X = Frs; g.ld = m; g.n = r; g.ncols = m; g.pcol = k;
            check_gj_block(g);
            g.SR = nullptr; g.SC = nullptr; g.box = id;
            L.gj.push_back(g);
            sr += (int64_t)GJ_NB * m;
            sc += (int64_t)r * GJ_NB;
            L.g_E.add(gdesc<T>(k, k, r, Fsr, m, 0, Frs, m, 0, Fss, m, T(-1), T(1)));
        }
    }
    // side buffers (shared by every level, sized for the largest)
    sr_need = std::max(sr_need, sr);
    sc_need = std::max(sc_need, sc);
    L.gj_steps = (L.max_r + GJ_NB - 1) / GJ_NB;
    L.max_chunks = (L.max_m + 63) / 64;
    const int cls = std::is_same<T, double>::value ? RSD_PROF_FACTOR_GEMM_F64 : RSD_PROF_FACTOR_GEMM_F32;
    L.g_sr.prof_cls = L.g_rr.prof_cls = L.g_E.prof_cls = cls;
    all.push_back(&L.g_sr);
    all.push_back(&L.g_rr);
    all.push_back(&L.g_E);
}

template <typename T>
static void finish_gj(Factor& f, LevelExec<T>& L, T* SRb, T* SCb, std::vector<GemmBatch<T>*>& all,
                      std::vector<GJDesc<T>>& gjall) {
    int64_t osr = 0, osc = 0;
    for (auto& g : L.gj) {
        g.SR = SRb + osr;
        g.SC = SCb + osc;
        osr += (int64_t)GJ_NB * g.ncols;
        osc += (int64_t)g.n * GJ_NB;
    }
    L.g_gj.resize(L.gj_steps);
    for (int st = 0; st < L.gj_steps; ++st) {
        for (auto& g : L.gj) {
            const int j0 = st * GJ_NB;
            if (j0 >= g.n) continue;
            const int nbe = std::min(GJ_NB, g.n - j0);
            GemmDesc<T> d = gdesc<T>(g.n, g.ncols, nbe, g.SC, g.n, 0, g.SR, GJ_NB, 0, g.X, g.ld,
                                     T(-1), T(1));
            d.zc0 = g.pcol + j0;
            d.zc1 = g.pcol + j0 + nbe;
            L.g_gj[st].add(d);
        }
    }
    for (auto& b : L.g_gj) {
        b.prof_cls = std::is_same<T, double>::value ? RSD_PROF_FACTOR_GEMM_F64 : RSD_PROF_FACTOR_GEMM_F32;
        all.push_back(&b);
    }
    (void)f;
    (void)gjall;
}

template <typename T>
static void plan_top(Factor& f, LevelExec<T>& L, T* SRb, T* SCb, std::vector<GemmBatch<T>*>& all) {
    // invert the remaining k x k block of the root in place
    const Box& b = f.plan.boxes[f.plan.root];
    const int k = b.k, m = b.k + b.r;
    T* Fss = Fbase<T>(f) + b.offF;
    GJDesc<T> g;
    g.X = Fss; g.ld = m; g.n = k; g.ncols = k; g.pcol = 0; g.SR = SRb; g.SC = SCb; g.box = f.plan.root;
    check_gj_block(g);
    L.topgj.push_back(g);
    L.topgj_steps = (k + GJ_NB - 1) / GJ_NB;
    L.top_chunks = (k + 63) / 64;
    L.g_topgj.resize(L.topgj_steps);
    for (int st = 0; st < L.topgj_steps; ++st) {
        const int j0 = st * GJ_NB;
        const int nbe = std::min(GJ_NB, k - j0);
        GemmDesc<T> d = gdesc<T>(k, k, nbe, SCb, k, 0, SRb, GJ_NB, 0, Fss, m, T(-1), T(1));
        d.zc0 = j0;
        d.zc1 = j0 + nbe;
        L.g_topgj[st].add(d);
    }
    for (auto& bb : L.g_topgj) {
        bb.prof_cls = RSD_PROF_FACTOR_GEMM_F64;
        all.push_back(&bb);
    }
}

template <typename T>
static void upload_gj(DevBuf& buf, std::vector<LevelExec<T>>& Ls, hipStream_t s, PinnedBlock* pinned = nullptr) {
    size_t n = 0;
    for (auto& L : Ls) n += L.gj.size() + L.topgj.size();
    std::vector<GJDesc<T>> host;
    host.reserve(n);
    for (auto& L : Ls) { host.insert(host.end(), L.gj.begin(), L.gj.end()); }
    for (auto& L : Ls) { host.insert(host.end(), L.topgj.begin(), L.topgj.end()); }
    buf.alloc(std::max<size_t>(1, host.size()) * sizeof(GJDesc<T>));
    if (!host.empty()) {
        const size_t bytes = host.size() * sizeof(GJDesc<T>);
        const void* src = host.data();
        if (pinned) {
            pinned->p = PinnedPool::get().take(bytes, pinned->cap);
            std::memcpy(pinned->p, src, bytes);
            src = pinned->p;
        }
        RSD_HIP(hipMemcpyAsync(buf.p, src, bytes, hipMemcpyHostToDevice, s));
    }
    size_t o = 0;
    for (auto& L : Ls) { L.d_gj = buf.as<GJDesc<T>>() + o; o += L.gj.size(); }
    for (auto& L : Ls) { L.d_topgj = buf.as<GJDesc<T>>() + o; o += L.topgj.size(); }
}

// F of every box of the level: leaf blocks, or the parent blocks assembled
// from the children's E and the generated sibling blocks.
template <typename T>
static void run_assembly(Factor& f, LevelExec<T>& L, hipStream_t s) {
    const int t = L.level;
    const int n = (int)L.ids.size();
    T* F = Fbase<T>(f);
    const BoxDev* B = f.d_boxes.as<BoxDev>();
    const LayoutDev* LD = f.d_layouts.as<LayoutDev>();
    ProfScope ps(RSD_PROF_ASSEMBLY, s);
    if (t == 0) {
        launch_leaf_F<T>(F, B, f.bids(t), n, LD, f.d_lu.as<int>(), f.d_lv.as<int>(), f.kd, L.max_m, s);
    } else {
        const int child_prec = f.level_prec[t - 1];
        if constexpr (std::is_same<T, float>::value) {
            launch_assemble_F<float, float>(F, f.F32.as<float>(), B, f.bids(t), n, LD, f.d_lu.as<int>(),
                                            f.d_lv.as<int>(), f.d_srcc.as<int>(), f.d_srci.as<int>(),
                                            f.kd, L.max_m, s);
        } else if (child_prec == 1) {
            launch_assemble_F<float, double>(F, f.F32.as<float>(), B, f.bids(t), n, LD, f.d_lu.as<int>(),
                                             f.d_lv.as<int>(), f.d_srcc.as<int>(), f.d_srci.as<int>(),
                                             f.kd, L.max_m, s);
        } else {
            launch_assemble_F<double, double>(F, f.F64.as<double>(), B, f.bids(t), n, LD,
                                              f.d_lu.as<int>(), f.d_lv.as<int>(), f.d_srcc.as<int>(),
                                              f.d_srci.as<int>(), f.kd, L.max_m, s);
        }
    }
}

// F'_rs = (F'_sr)^T for the level's boxes
template <typename T>
static void run_transpose(Factor& f, LevelExec<T>& L, hipStream_t s) {
    if (L.g_sr.empty()) return;
    ProfScope ps(RSD_PROF_ASSEMBLY, s);
    launch_transpose_sr<T>(Fbase<T>(f), f.d_boxes.as<BoxDev>(), f.bids(L.level), (int)L.ids.size(),
                           L.max_k, L.max_r, s);
}

template <typename T>
static void run_level(Factor& f, LevelExec<T>& L, hipStream_t s, bool assemble = true) {
    if (assemble) run_assembly<T>(f, L, s);
    L.g_sr.run(s);
    L.g_rr.run(s);
    run_transpose<T>(f, L, s);
    for (int st = 0; st < L.gj_steps; ++st) {
        {
            ProfScope ps(RSD_PROF_GJ_PIVOT, s);
            launch_gj_pivot<T>(L.d_gj, (int)L.gj.size(), st, GJ_NB, L.max_chunks, f.d_err.as<int>(), f.cplx, s);
        }
        L.g_gj[st].run(s);
    }
    L.g_E.run(s);
    for (int st = 0; st < L.topgj_steps; ++st) {
        {
            ProfScope ps(RSD_PROF_GJ_PIVOT, s);
            launch_gj_pivot<T>(L.d_topgj, 1, st, GJ_NB, L.top_chunks, f.d_err.as<int>(), f.cplx, s);
        }
        L.g_topgj[st].run(s);
    }
}

// One level (and precision) of every factor of a batch group: each product
// and each Gauss-Jordan step is one launch for the boxes of all of them.
// Every descriptor keeps its own factor's addresses (and its error flag), so
// merging changes nothing but the launch count and, through the tile table,
// the split of long K ranges.
template <typename T>
struct GroupLevel {
    std::vector<std::pair<Factor*, LevelExec<T>*>> members;
    GemmBatch<T> g_sr, g_rr, g_E;
    std::vector<GemmBatch<T>> g_gj, g_topgj;
    std::vector<GJDesc<T>> gj, topgj;
    const GJDesc<T>* d_gj = nullptr;
    const GJDesc<T>* d_topgj = nullptr;
    int gj_steps = 0, topgj_steps = 0, max_chunks = 0, top_chunks = 0;
    // assembly and transposes: per-member tables, and the boxes by the
    // precision of their children (0 float64, 1 float32; leaves under 0)
    int level = 0, max_m = 0, max_k = 0, max_r = 0;
    std::vector<AsmInst> ainst;
    std::vector<GroupItem> items[2], titems;
    const AsmInst* d_ainst = nullptr;
    const GroupItem* d_items[2] = {nullptr, nullptr};
    const GroupItem* d_titems = nullptr;

    void add(Factor& F, LevelExec<T>& L) {
        members.push_back({&F, &L});
        {
            const int inst = (int)ainst.size();
            const int child_prec = L.level > 0 ? F.level_prec[L.level - 1] : 0;
            AsmInst a;
            a.F = Fbase<T>(F);
            a.Fc = L.level == 0 ? nullptr : (child_prec ? F.F32.p : F.F64.p);
            a.boxes = F.d_boxes.as<BoxDev>();
            a.layouts = F.d_layouts.as<LayoutDev>();
            a.lu = F.d_lu.as<int>();
            a.lv = F.d_lv.as<int>();
            a.src_c = F.d_srcc.as<int>();
            a.src_i = F.d_srci.as<int>();
            a.kd = F.kd;
            ainst.push_back(a);
            for (int id : L.ids) {
                items[child_prec].push_back({inst, id});
                if (!L.g_sr.empty()) titems.push_back({inst, id});
            }
            level = L.level;
            max_m = std::max(max_m, L.max_m);
            max_k = std::max(max_k, L.max_k);
            max_r = std::max(max_r, L.max_r);
        }
        for (auto& d : L.g_sr.descs) g_sr.add(d);
        for (auto& d : L.g_rr.descs) g_rr.add(d);
        for (auto& d : L.g_E.descs) g_E.add(d);
        if ((int)g_gj.size() < L.gj_steps) g_gj.resize(L.gj_steps);
        for (int st = 0; st < L.gj_steps; ++st)
            for (auto& d : L.g_gj[st].descs) g_gj[st].add(d);
        if ((int)g_topgj.size() < L.topgj_steps) g_topgj.resize(L.topgj_steps);
        for (int st = 0; st < L.topgj_steps; ++st)
            for (auto& d : L.g_topgj[st].descs) g_topgj[st].add(d);
        for (auto g : L.gj) {
            g.err = F.d_err.as<int>();
            gj.push_back(g);
        }
        for (auto g : L.topgj) {
            g.err = F.d_err.as<int>();
            topgj.push_back(g);
        }
        gj_steps = std::max(gj_steps, L.gj_steps);
        topgj_steps = std::max(topgj_steps, L.topgj_steps);
        max_chunks = std::max(max_chunks, L.max_chunks);
        top_chunks = std::max(top_chunks, L.top_chunks);
    }
    void batches(std::vector<GemmBatch<T>*>& all) {
        const int cls = std::is_same<T, double>::value ? RSD_PROF_FACTOR_GEMM_F64 : RSD_PROF_FACTOR_GEMM_F32;
        for (auto* b : {&g_sr, &g_rr, &g_E}) {
            b->prof_cls = cls;
            all.push_back(b);
        }
        for (auto& b : g_gj) { b.prof_cls = cls; all.push_back(&b); }
        for (auto& b : g_topgj) { b.prof_cls = RSD_PROF_FACTOR_GEMM_F64; all.push_back(&b); }
    }
    void run(hipStream_t s) {
        if (members.empty()) return;
        int* err0 = members.front().first->d_err.template as<int>();
        const int cplx = members.front().first->cplx;   // groups hold one kind of factor
        {
            ProfScope ps(RSD_PROF_ASSEMBLY, s);
            if (level == 0) {
                launch_leaf_F_group<T>(d_ainst, d_items[0], (int)items[0].size(), max_m, s);
            } else {
                if (!items[1].empty())
                    launch_assemble_F_group<float, T>(d_ainst, d_items[1], (int)items[1].size(), max_m, s);
                if constexpr (std::is_same<T, double>::value) {
                    if (!items[0].empty())
                        launch_assemble_F_group<double, double>(d_ainst, d_items[0], (int)items[0].size(), max_m, s);
                } else if (!items[0].empty()) {
                    throw Error(RSD_EINVAL, "internal: float32 level above a float64 level");
                }
            }
        }
        g_sr.run(s);
        g_rr.run(s);
        if (!titems.empty()) {
            ProfScope ps(RSD_PROF_ASSEMBLY, s);
            launch_transpose_group<T>(d_ainst, d_titems, (int)titems.size(), max_k, max_r, s);
        }
        for (int st = 0; st < gj_steps; ++st) {
            {
                ProfScope ps(RSD_PROF_GJ_PIVOT, s);
                launch_gj_pivot<T>(d_gj, (int)gj.size(), st, GJ_NB, max_chunks, err0, cplx, s);
            }
            g_gj[st].run(s);
        }
        g_E.run(s);
        for (int st = 0; st < topgj_steps; ++st) {
            {
                ProfScope ps(RSD_PROF_GJ_PIVOT, s);
                launch_gj_pivot<T>(d_topgj, (int)topgj.size(), st, GJ_NB, top_chunks, err0, cplx, s);
            }
            g_topgj[st].run(s);
        }
    }
};

template <typename T>
static void upload_group_asm(DevBuf& ibuf, DevBuf& tbuf, std::vector<GroupLevel<T>>& G, hipStream_t s) {
    std::vector<AsmInst> insts;
    std::vector<GroupItem> items;
    for (auto& g : G) {
        insts.insert(insts.end(), g.ainst.begin(), g.ainst.end());
        for (int c = 0; c < 2; ++c) items.insert(items.end(), g.items[c].begin(), g.items[c].end());
        items.insert(items.end(), g.titems.begin(), g.titems.end());
    }
    upload(ibuf, insts, s);
    upload(tbuf, items, s);
    size_t oi = 0, ot = 0;
    for (auto& g : G) {
        g.d_ainst = ibuf.as<AsmInst>() + oi;
        oi += g.ainst.size();
        for (int c = 0; c < 2; ++c) {
            g.d_items[c] = tbuf.as<GroupItem>() + ot;
            ot += g.items[c].size();
        }
        g.d_titems = tbuf.as<GroupItem>() + ot;
        ot += g.titems.size();
    }
}

template <typename T>
static void upload_group_gj(DevBuf& buf, std::vector<GroupLevel<T>>& G, hipStream_t s) {
    std::vector<GJDesc<T>> host;
    for (auto& g : G) host.insert(host.end(), g.gj.begin(), g.gj.end());
    for (auto& g : G) host.insert(host.end(), g.topgj.begin(), g.topgj.end());
    upload(buf, host, s);
    size_t o = 0;
    for (auto& g : G) { g.d_gj = buf.as<GJDesc<T>>() + o; o += g.gj.size(); }
    for (auto& g : G) { g.d_topgj = buf.as<GJDesc<T>>() + o; o += g.topgj.size(); }
}

// ----------------------------------------------------------------------------
// build
// ----------------------------------------------------------------------------
// Spacing in grid cells of the interface skeleton points of a Helmholtz
// factor with ppw points per wavelength 2 pi / k (Sec. 5.3), at least one
// cell; 0 (none) for Laplace or ppw = 0.
static int interface_step(int ktype, double k, double h, double ppw) {
    if (!(ppw >= 0) || !std::isfinite(ppw)) throw Error(RSD_EINVAL, "interface_ppw must be finite and >= 0");
    if (ktype != RSD_KERNEL_HELMHOLTZ || ppw == 0) return 0;
    const double cells = std::floor(2.0 * M_PI / (k * h * ppw));
    return cells < 1 ? 1 : (cells > 1e6 ? 1000000 : (int)cells);
}

// The plan depends on the grid's shape, the leaf side, the layer count and
// the interface spacing only; the last few plans are kept (building one is most of a build's host
// planning, ~0.9 ms at 256x256, copying it a fraction of that).
static Plan cached_plan(int64_t nx, int64_t ny, int leaf, int m, int iface) {
    struct Entry {
        int64_t nx, ny;
        int leaf, m, iface;
        std::shared_ptr<const Plan> plan;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;   // most recent last
    constexpr size_t KEEP = 8;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < cache.size(); ++i) {
            const Entry& e = cache[i];
            if (e.nx == nx && e.ny == ny && e.leaf == leaf && e.m == m && e.iface == iface) {
                Entry hit = e;
                cache.erase(cache.begin() + i);
                cache.push_back(hit);
                return *hit.plan;
            }
        }
    }
    auto plan = std::make_shared<const Plan>(make_plan(nx, ny, leaf, m, iface));
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({nx, ny, leaf, m, iface, plan});
    if (cache.size() > KEEP) cache.erase(cache.begin());
    return *plan;
}

// Plan of a complex factor: every box type's dof block lists each point
// twice, its plane-0 and plane-1 dofs adjacent, skeleton points first (the
// real symmetric J form of the complex symmetric matrix, see KernelDesc; the
// pairing makes the pivot-free elimination pivot on complex entries), so k, r
// and the interpolation problems double (rows: proxy points of plane 0 then
// plane 1) and the children-to-parent maps point at the child's dof of the
// same plane.  The interpolation problems are solved whole (no symmetry
// sectors).
static Plan expand_planes(const Plan& P) {
    Plan Q = P;
    for (size_t li = 0; li < Q.layouts.size(); ++li) {
        Layout& L = Q.layouts[li];
        const Layout& O = P.layouts[li];
        const int k = O.k, r = O.r;
        std::vector<int32_t> u, v, sc, si;
        auto put = [&](int q, int plane) {
            u.push_back(O.u[q]);
            v.push_back(O.v[q]);
            if (!O.src_c.empty()) {
                sc.push_back(O.src_c[q]);
                si.push_back(2 * O.src_i[q] + plane);   // the child's skeleton dofs are paired too
            }
        };
        for (int q = 0; q < k + r; ++q) {
            put(q, 0);
            put(q, 1);
        }
        L.u = std::move(u);
        L.v = std::move(v);
        L.src_c = std::move(sc);
        L.src_i = std::move(si);
        L.k = 2 * k;
        L.r = 2 * r;
    }
    for (auto& b : Q.boxes) { b.k *= 2; b.r *= 2; }
    for (auto& I : Q.idps) {
        I.p *= 2; I.k *= 2; I.r *= 2;
        I.sym = false;
        I.grp = 0;
    }
    Q.F_elems = Q.V_elems = Q.Vr_elems = 0;
    for (auto& b : Q.boxes) {
        Q.F_elems += (int64_t)(b.k + b.r) * (b.k + b.r);
        Q.V_elems += b.k + b.r;
        Q.Vr_elems += b.r;
    }
    return Q;
}

// Integral of the kernel over the square cell of side h centred on its point
// (the diagonal of the Nystrom matrix, Sec. 5).  Laplace: closed form
// h^2 (log h + J) / 2pi, J = -log(2)/2 - 3/2 + pi/4 (eight triangles in polar
// coordinates).  Helmholtz (i/4) H0^(1)(k r): written as -(1/2pi) log r plus
// the bounded remainder R(r) = G(r) + (1/2pi) log r, whose integral over the
// eight triangles r < h / (2 cos t), 0 < t < pi/4 is taken by tensor
// Gauss-Legendre quadrature with r = rmax s^2 (the remainder behaves like
// r^2 log r at 0, the substitution smooths it).
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int j = 2; j <= n; ++j) {
            const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

static void self_cell_integral(int type, double h, double k, double& re, double& im) {
    const double J = -0.5 * std::log(2.0) - 1.5 + M_PI / 4.0;
    const double lap = h * h * (std::log(h) + J) / (2.0 * M_PI);
    if (type == RSD_KERNEL_LAPLACE) {
        re = lap;
        im = 0.0;
        return;
    }
    std::vector<double> gx, gw;
    gauss_legendre(40, gx, gw);
    double sr = 0.0, si = 0.0;
    for (int a = 0; a < 40; ++a) {
        const double t = 0.125 * M_PI * (gx[a] + 1.0), wt = 0.125 * M_PI * gw[a];
        const double rmax = h / (2.0 * std::cos(t));
        for (int b = 0; b < 40; ++b) {
            const double sq = 0.5 * (gx[b] + 1.0), ws = 0.5 * gw[b];
            const double rr = rmax * sq * sq;           // r = rmax s^2, dr = 2 rmax s ds
            const double jac = 2.0 * rmax * sq * rr;    // dr * r
            const double z = k * rr;
            const double gre = -0.25 * std::cyl_neumann(0.0, z) + std::log(rr) / (2.0 * M_PI);
            const double gim = 0.25 * std::cyl_bessel_j(0.0, z);
            sr += wt * ws * jac * gre;
            si += wt * ws * jac * gim;
        }
    }
    re = -lap + 8.0 * sr;
    im = 8.0 * si;
}

// Host planning of a build and the uploads of its tables (on the factor's
// stream); no kernel is launched yet.
// Grid detection of the most recent distinct point set: repeated builds on
// one grid (new coefficients, tolerances or kernels) compare the points with
// it exactly and reuse its result, which is a function of the points alone.
struct GridCache {
    std::mutex mu;
    std::vector<double> pts;
    int64_t nx = 0, ny = 0;
    double h = 0, x0 = 0, y0 = 0;
    std::vector<int64_t> perm;
};
static bool detect_grid_cached(const double* pts, int64_t n, int64_t& nx, int64_t& ny, double& h, double& x0,
                               double& y0, std::vector<int64_t>& perm, std::string& why) {
    static GridCache* cache = new GridCache();   // outlives static destructors
    {
        std::lock_guard<std::mutex> lk(cache->mu);
        if ((int64_t)cache->pts.size() == 2 * n && std::memcmp(cache->pts.data(), pts, 2 * n * sizeof(double)) == 0) {
            nx = cache->nx; ny = cache->ny; h = cache->h; x0 = cache->x0; y0 = cache->y0;
            perm = cache->perm;
            return true;
        }
    }
    if (!detect_grid(pts, n, nx, ny, h, x0, y0, perm, why)) return false;
    std::lock_guard<std::mutex> lk(cache->mu);
    cache->pts.assign(pts, pts + 2 * n);
    cache->nx = nx; cache->ny = ny; cache->h = h; cache->x0 = x0; cache->y0 = y0;
    cache->perm = perm;
    return true;
}

static std::unique_ptr<Factor> build_prepare(const double* points, int64_t n, const rsd_kernel* kernel,
                                             const double* a, double tol, const rsd_options* opt,
                                             bool allow_dedup = true) {
    if (!points || n <= 0) throw Error(RSD_EINVAL, "points must be non-null and n_points > 0");
    if (!(tol > 0) || !std::isfinite(tol)) throw Error(RSD_EINVAL, "tol must be a positive number");
    rsd_options o{};
    if (opt) o = *opt;
    auto f = std::make_unique<Factor>();
    if (o.device >= 0) RSD_HIP(hipSetDevice(o.device));
    RSD_HIP(hipGetDevice(&f->device));
    if (o.hip_stream) f->stream = static_cast<hipStream_t>(o.hip_stream);
    else {
        f->stream = StreamPool::get().take();
        f->own_stream = true;
    }
    hipStream_t s = f->stream;
    f->tol = tol;
    f->flags = o.flags;
    f->precision = o.precision == RSD_PREC_FP32_REFINE ? RSD_PREC_FP32_REFINE : RSD_PREC_FP64;
    if (o.precision != RSD_PREC_FP64 && o.precision != RSD_PREC_FP32_REFINE)
        throw Error(RSD_EINVAL, "unknown precision");
    f->max_refine = o.max_refine < 0 ? 0 : (o.max_refine == 0 ? (f->precision == RSD_PREC_FP32_REFINE ? 10 : 0) : o.max_refine);
    f->refine_tol = o.refine_tol > 0 ? o.refine_tol : tol;
    const int leaf = o.leaf_side > 0 ? o.leaf_side : 8;
    const int ktype = kernel ? kernel->type : RSD_KERNEL_LAPLACE;
    const int m = o.layers > 0 ? o.layers : default_layers(tol, ktype);
    if (ktype != RSD_KERNEL_LAPLACE && ktype != RSD_KERNEL_HELMHOLTZ) throw Error(RSD_EINVAL, "unknown kernel type");
    const double wavenumber = ktype == RSD_KERNEL_HELMHOLTZ ? kernel->wavenumber : 0.0;
    if (ktype == RSD_KERNEL_HELMHOLTZ && !(wavenumber > 0 && std::isfinite(wavenumber)))
        throw Error(RSD_EINVAL, "the Helmholtz kernel needs a positive finite wavenumber");
    f->cplx = ktype == RSD_KERNEL_HELMHOLTZ ? 1 : 0;
    // host views of the inputs: device arrays are read back into a pinned
    // block (a direct copy), host arrays are read in place
    const double* bptr = kernel ? kernel->contrast_b : nullptr;
    PinnedBlock in_pin;
    const double* pts = points;
    const double* ha = a;
    const double* hb = bptr;
    {
        const bool pdev = is_device_ptr(points), adev = a && is_device_ptr(a), bdev = bptr && is_device_ptr(bptr);
        if (pdev || adev || bdev) {
            const size_t np = pdev ? 2 * (size_t)n : 0, na = adev ? (size_t)n : 0, nb = bdev ? (size_t)n : 0;
            in_pin.p = PinnedPool::get().take((np + na + nb) * sizeof(double), in_pin.cap);
            double* w = static_cast<double*>(in_pin.p);
            if (pdev) {
                RSD_HIP(hipMemcpy(w, points, np * sizeof(double), hipMemcpyDeviceToHost));
                pts = w;
            }
            if (adev) {
                RSD_HIP(hipMemcpy(w + np, a, na * sizeof(double), hipMemcpyDeviceToHost));
                ha = w + np;
            }
            if (bdev) {
                RSD_HIP(hipMemcpy(w + np + na, bptr, nb * sizeof(double), hipMemcpyDeviceToHost));
                hb = w + np + na;
            }
        }
    }
    HostPool& pool = HostPool::get();
    // below about 10^5 points waking the pool costs more than the loops
    const int64_t GRAIN = n >= (int64_t(1) << 17) ? 16384 : n;
    // every point's value checked on the host pool (flags, no throws inside)
    auto all_of = [&](const double* v, auto pred) {
        std::atomic<int> bad{0};
        pool.parallel_for(n, GRAIN, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i)
                if (!pred(v[i])) { bad.store(1, std::memory_order_relaxed); return; }
        });
        return bad.load() == 0;
    };
    if (ha && !all_of(ha, [](double x) { return std::isfinite(x); }))
        throw Error(RSD_EINVAL, "non-finite value in a");
    // contrast (scattering) form A = I + S K S, S = diag sqrt(b) (Sec. 5.4):
    // factored as A = S M S with M = diag(1/b) + K, whose off-diagonal part is
    // the translation-invariant kernel (one T per box type); needs b > 0
    if (hb) {
        if (ha) throw Error(RSD_EINVAL, "the contrast form takes a = NULL (identity coefficient 1)");
        if (!all_of(hb, [](double x) { return std::isfinite(x) && x > 0; }))
            throw Error(RSD_EINVAL, "the contrast b must be finite and positive at every point");
    }
    int64_t nx, ny;
    double h, x0, y0;
    std::vector<int64_t> perm;
    std::string why;
    if (!detect_grid_cached(pts, n, nx, ny, h, x0, y0, perm, why)) throw Error(RSD_ENOTGRID, why);
    f->N = n; f->nx = nx; f->ny = ny; f->h = h;
    try {
        f->plan = cached_plan(nx, ny, leaf, m, interface_step(ktype, wavenumber, h, o.interface_ppw));
    } catch (const std::exception& e) {
        throw Error(RSD_EINVAL, e.what());
    }
    if (f->cplx) f->plan = expand_planes(f->plan);
    Plan& P = f->plan;
    if (o.flags & RSD_FLAG_NO_SYMMETRY)
        for (auto& I : P.idps) I.sym = false;
    const int nlev = (int)P.levels.size();
    f->top = nlev - 1;
    f->level_prec.assign(nlev, 0);
    if (f->precision == RSD_PREC_FP32_REFINE)
        for (int t = 0; t < f->top; ++t) f->level_prec[t] = 1;
    // ---- grid-ordered coefficients -----------------------------------------
    // ag: diagonal coefficient of the factored matrix (a, or 1/b for the
    // contrast form); sbg: sqrt(b) for the contrast form (residual operator
    // and the scaling around the solve)
    std::vector<double> ag, sbg;
    if (ha) {
        ag.resize(n);
        pool.parallel_for(n, GRAIN, [&](int64_t lo, int64_t hi) {
            for (int64_t g = lo; g < hi; ++g) ag[g] = ha[perm[g]];
        });
    }
    if (hb) {
        ag.resize(n);
        sbg.resize(n);
        pool.parallel_for(n, GRAIN, [&](int64_t lo, int64_t hi) {
            for (int64_t g = lo; g < hi; ++g) {
                ag[g] = 1.0 / hb[perm[g]];
                sbg[g] = std::sqrt(hb[perm[g]]);
            }
        });
    }
    // ---- device tables ------------------------------------------------------
    std::vector<int> lu, lv, srcc, srci, inv;
    f->hlayouts.resize(P.layouts.size());
    int64_t offT64 = 0, offT32 = 0;
    for (size_t li = 0; li < P.layouts.size(); ++li) {
        const Layout& L = P.layouts[li];
        LayoutDev& D = f->hlayouts[li];
        D.k = L.k; D.r = L.r;
        D.off_uv = (int)lu.size();
        lu.insert(lu.end(), L.u.begin(), L.u.end());
        lv.insert(lv.end(), L.v.begin(), L.v.end());
        if (L.src_c.empty()) { srcc.insert(srcc.end(), L.u.size(), 0); srci.insert(srci.end(), L.u.size(), 0); }
        else { srcc.insert(srcc.end(), L.src_c.begin(), L.src_c.end()); srci.insert(srci.end(), L.src_i.begin(), L.src_i.end()); }
        D.off_inv0 = D.off_inv1 = 0;
        if (L.child[0] >= 0) {
            const int k0 = P.layouts[L.child[0]].k, k1 = P.layouts[L.child[1]].k;
            D.off_inv0 = (int)inv.size();
            inv.resize(inv.size() + k0 + k1, -1);
            D.off_inv1 = D.off_inv0 + k0;
            for (int q = 0; q < L.k + L.r; ++q)
                inv[(L.src_c[q] == 0 ? D.off_inv0 : D.off_inv1) + L.src_i[q]] = q;
        }
        D.idp = L.idp;
        D.offT = -1;
    }
    // precision of each layout = precision of the level its boxes sit on
    std::vector<int> layout_level(P.layouts.size(), -1);
    for (auto& b : P.boxes) layout_level[b.layout] = b.level;
    for (size_t li = 0; li < P.layouts.size(); ++li) {
        const Layout& L = P.layouts[li];
        if (L.idp < 0) continue;
        const int prec = f->level_prec[layout_level[li]];
        int64_t& o2 = prec ? offT32 : offT64;
        f->hlayouts[li].offT = o2;
        o2 += (int64_t)L.k * L.r;
    }
    // Translation-invariant deduplication (Sec. 5.1.2): with a constant
    // diagonal coefficient and no contrast, every box of one layout on one
    // level has the same F_i (kernel blocks depend on relative positions only,
    // the children's E_c are equal by induction), hence the same E_i, G and W.
    // Only one representative per (level, layout) is built; every box's block
    // offset points at its representative's block.
    bool const_a = !hb;
    if (ha && const_a) {
        const double a0 = ha[0];
        const_a = all_of(ha, [a0](double x) { return x == a0; });
    }
    f->dedup = allow_dedup && const_a && !(o.flags & RSD_FLAG_NO_DEDUP);
    std::vector<int> rep(P.boxes.size());
    for (size_t i = 0; i < P.boxes.size(); ++i) rep[i] = (int)i;
    if (f->dedup) {
        std::map<std::pair<int, int>, int> first;     // (level, layout) -> representative
        for (size_t i = 0; i < P.boxes.size(); ++i) {
            const auto key = std::make_pair(P.boxes[i].level, P.boxes[i].layout);
            auto it = first.find(key);
            if (it == first.end()) first.emplace(key, (int)i);
            else rep[i] = it->second;
        }
    }
    // boxes: F offsets per precision arena, vector offsets per precision
    int64_t offF64 = 0, offF32 = 0;
    f->hboxes.resize(P.boxes.size());
    std::vector<int64_t> offV(2, 0), offY(2, 0);
    for (size_t i = 0; i < P.boxes.size(); ++i) {
        const Box& b = P.boxes[i];
        BoxDev& D = f->hboxes[i];
        D.x0 = b.x0; D.y0 = b.y0; D.k = b.k; D.r = b.r; D.layout = b.layout;
        D.parent = b.parent; D.pos = b.pos_in_parent; D.child0 = b.child[0]; D.child1 = b.child[1];
        D.level = b.level;
        const int prec = f->level_prec[b.level];
        const int64_t mm = (int64_t)b.k + b.r;
        if (rep[i] == (int)i) {
            int64_t& oF = prec ? offF32 : offF64;
            D.offF = oF;
            oF += mm * mm;
        } else {
            D.offF = f->hboxes[rep[i]].offF;      // representatives come first in box order
        }
        P.boxes[i].offF = D.offF;
        D.offV = offV[prec];
        offV[prec] += mm;
        D.offY = offY[prec];
        offY[prec] += b.r;
    }
    f->F64.alloc(std::max<int64_t>(offF64, 1) * sizeof(double));
    f->F32.alloc(std::max<int64_t>(offF32, 1) * sizeof(float));
    f->T64.alloc(std::max<int64_t>(offT64, 1) * sizeof(double));
    f->T32.alloc(std::max<int64_t>(offT32, 1) * sizeof(float));
    std::vector<int> lid, bid;
    f->build_levels.assign(nlev, {});
    for (int t = 0; t < nlev; ++t) {
        f->level_id_off.push_back((int)lid.size());
        lid.insert(lid.end(), P.levels[t].begin(), P.levels[t].end());
        for (int id : P.levels[t])
            if (rep[id] == id) f->build_levels[t].push_back(id);
    }
    for (int t = 0; t < nlev; ++t) {
        f->build_id_off.push_back((int)(lid.size() + bid.size()));
        bid.insert(bid.end(), f->build_levels[t].begin(), f->build_levels[t].end());
    }
    lid.insert(lid.end(), bid.begin(), bid.end());   // one device table: all boxes, then the built ones
    std::vector<int64_t> ident(f->cplx ? 2 * n : n);
    for (int64_t g = 0; g < (int64_t)ident.size(); ++g) ident[g] = g;
    upload(f->d_boxes, f->hboxes, s);
    upload(f->d_layouts, f->hlayouts, s);
    upload(f->d_lu, lu, s);
    upload(f->d_lv, lv, s);
    upload(f->d_srcc, srcc, s);
    upload(f->d_srci, srci, s);
    upload(f->d_inv, inv, s);
    upload(f->d_perm, perm, s);
    upload(f->d_ident, ident, s);
    upload(f->d_level_ids, lid, s);
    if (!ag.empty()) upload(f->d_a, ag, s);
    if (!sbg.empty()) upload(f->d_sb, sbg, s);
    f->d_err.alloc(sizeof(int) * 4);
    RSD_HIP(hipMemsetAsync(f->d_err.p, 0, sizeof(int) * 4, s));
    // every interpolation problem writes its record (no clearing needed)
    f->d_interp.alloc(std::max<size_t>(P.layouts.size(), 1) * 12 * sizeof(double));
    f->layout_damped.assign(P.layouts.size(), 0);
    // kernel descriptions: kd generates the factored matrix (diagonal ag,
    // no scaling), kd_res is the exact operator of the residual (contrast
    // scaling when given)
    KernelDesc& kd = f->kd;
    kd.type = ktype == RSD_KERNEL_HELMHOLTZ ? 1 : 0;
    kd.has_b = 0;
    kd.h = h;
    kd.logh = std::log(h);
    kd.k = wavenumber;
    self_cell_integral(ktype, h, wavenumber, kd.sc_re, kd.sc_im);
    kd.a = ag.empty() ? nullptr : f->d_a.as<double>();
    kd.sb = nullptr;
    kd.ny = ny;
    kd.cplx = f->cplx;
    f->kd_res = kd;
    if (!sbg.empty()) {
        f->kd_res.has_b = 1;
        f->kd_res.a = nullptr;
        f->kd_res.sb = f->d_sb.as<double>();
    }
    // ---- level plans ----------------------------------------------------------
    std::vector<GemmBatch<double>*> b64;
    std::vector<GemmBatch<float>*> b32;
    int64_t sr64 = 0, sc64 = 0, sr32 = 0, sc32 = 0;
    f->L64.clear();
    f->L32.clear();
    f->L64.reserve(nlev);
    f->L32.reserve(nlev);
    std::vector<int> exec_index(nlev);
    for (int t = 0; t < nlev; ++t) {
        if (f->level_prec[t]) { exec_index[t] = (int)f->L32.size(); f->L32.emplace_back(); }
        else { exec_index[t] = (int)f->L64.size(); f->L64.emplace_back(); }
    }
    for (int t = 0; t < nlev; ++t) {
        if (f->level_prec[t]) plan_level<float>(*f, f->L32[exec_index[t]], t, b32, sr32, sc32);
        else plan_level<double>(*f, f->L64[exec_index[t]], t, b64, sr64, sc64);
    }
    {   // root: remaining block inverted in place
        const Box& rb = P.boxes[P.root];
        sr64 = std::max<int64_t>(sr64, (int64_t)GJ_NB * rb.k);
        sc64 = std::max<int64_t>(sc64, (int64_t)rb.k * GJ_NB);
    }
    const int64_t sr_el = std::max(sr64, sr32), sc_el = std::max(sc64, sc32);
    f->SR.alloc(std::max<int64_t>(sr_el, 1) * sizeof(double));
    f->SC.alloc(std::max<int64_t>(sc_el, 1) * sizeof(double));
    std::vector<GJDesc<double>> gj64;
    std::vector<GJDesc<float>> gj32;
    for (auto& L : f->L64) finish_gj<double>(*f, L, f->SR.as<double>(), f->SC.as<double>(), b64, gj64);
    for (auto& L : f->L32) finish_gj<float>(*f, L, f->SR.as<float>(), f->SC.as<float>(), b32, gj32);
    plan_top<double>(*f, f->L64[exec_index[f->top]], f->SR.as<double>(), f->SC.as<double>(), b64);
    // uploaded by enqueue_single once the first interpolation window is
    // under way (a factor built in a group runs from the group's tables)
    f->tables64 = b64;
    f->tables32 = b32;
    f->exec_index = exec_index;
    f->layout_level = layout_level;
    f->layers = m;
    for (auto* b : b64) f->gemm_flops += b->flops;
    for (auto* b : b32) f->gemm_flops += b->flops;
    RSD_HIP(hipEventCreate(&f->build_ev[0]));
    RSD_HIP(hipEventCreate(&f->build_ev[1]));
    RSD_HIP(hipEventRecord(f->build_ev[0], s));
    return f;
}

// Chain class of a box type's interpolation problem, and how many (sector)
// problems it makes.  Class 0 holds the problems done after one window (the
// lowest levels, needed first), class 3 those done after two to four (the
// middle levels), class 1 the longer ones (the top levels), class 2 the boxes
// too tall for 16-column sub-panels.  A window's launches last as long as
// their largest problem, so the middle levels do not wait for the top
// levels' windows.
constexpr int CHAIN_CLASSES = 4;
static int chain_class(const Factor& f, const IDProblem& I, int ip, int& nprob) {
    nprob = split_sym(f, I, ip) ? I.nsec() : 1;
    const bool narrow = qr_panel_width(I.p / nprob, ip ? 4 : 8) < 16;
    const int windows = (I.k / nprob + QR_WIN - 1) / QR_WIN;
    return narrow ? 2 : (windows <= 1 ? 0 : (windows <= 4 ? 3 : 1));
}

// Every launch of a single build: the interpolation chains on two streams of
// their own and the level pipeline on the factor's stream, each level as
// soon as the events of its box types exist.
static void enqueue_single(Factor& fr) {
    Factor* f = &fr;
    Plan& P = f->plan;
    hipStream_t s = f->stream;
    const int nlev = (int)P.levels.size();
    const std::vector<int>& exec_index = f->exec_index;
    const std::vector<int>& layout_level = f->layout_level;
    // interpolation problems on their own streams, overlapping the level pipeline
    for (auto& q : f->qr_stream) q = StreamPool::get().take();
    {
        hipEvent_t go;
        RSD_HIP(hipEventCreateWithFlags(&go, hipEventDisableTiming));
        RSD_HIP(hipEventRecord(go, s));
        for (auto q : f->qr_stream) RSD_HIP(hipStreamWaitEvent(q, go, 0));
        (void)hipEventDestroy(go);
    }
    // chains: (precision, class) -> problems (chain_class); every chain
    // advances its problems window by window, so the short problems do
    // not wait for the first windows of the large ones.  Classes 0, 2 and 3
    // share a stream (class 0 is done almost at once), class 1 has the other:
    // with the level pipeline's stream that is three streams, one hardware
    // queue each under HIP's default of four per process (one is taken by
    // the default stream).
    constexpr int NCH = CHAIN_CLASSES;
    auto chain_stream = [&](int c) { return f->qr_stream[c == 1 ? 1 : 0]; };
    std::vector<ChainMember> cp[2][NCH];
    std::vector<int> pending(nlev, 0);
    for (size_t li = 0; li < P.layouts.size(); ++li) {
        if (P.layouts[li].idp < 0) continue;
        const int lev = layout_level[li];
        // T depends on geometry only (one problem per box type), so it is
        // computed in float64 and rounded into a float32 level's arena,
        // unless the caller asks for float32 interpolation as well
        const int ip = interp_prec(*f, lev);
        int nprob = 1;
        const int cls = chain_class(*f, P.idps[P.layouts[li].idp], ip, nprob);
        cp[ip][cls].push_back({f, P.layouts[li].idp, lev, lev});
        pending[lev] += nprob;     // one per (sector) problem
    }
    // Levels are enqueued as soon as the events of their box types exist, so
    // the level pipeline runs alongside the interpolation problems.  The
    // chains' windows are enqueued by a second host thread (its launches go to
    // the chain streams only), so neither the windows nor the levels wait for
    // the host to enqueue the other; pending counts and events are shared
    // under a lock.
    std::vector<std::vector<hipEvent_t>> level_waits(nlev);
    std::mutex mu;
    std::condition_variable cv;
    bool chains_done = false;
    auto publish = [&](hipEvent_t ev, const std::vector<int>& done) {
        if (!ev) return;
        {
            std::lock_guard<std::mutex> lk(mu);
            f->tmp_events.push_back(ev);
            for (int lev : done) {
                if (level_waits[lev].empty() || level_waits[lev].back() != ev) level_waits[lev].push_back(ev);
                --pending[lev];
            }
        }
        cv.notify_all();
    };
    int next_level = 0;
    // enqueues the next level once its problems are done (block: wait for it)
    auto enqueue_next = [&](bool block) {
        std::vector<hipEvent_t> waits;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (block) cv.wait(lk, [&] { return pending[next_level] == 0 || chains_done; });
            if (pending[next_level] != 0) return false;
            waits = level_waits[next_level];
        }
        const int t = next_level++;
        // the level's F blocks need only the level below: assembled before
        // the wait for the level's interpolation
        if (f->level_prec[t]) {
            run_assembly<float>(*f, f->L32[exec_index[t]], s);
            for (auto e : waits) RSD_HIP(hipStreamWaitEvent(s, e, 0));
            run_level<float>(*f, f->L32[exec_index[t]], s, false);
        } else {
            run_assembly<double>(*f, f->L64[exec_index[t]], s);
            for (auto e : waits) RSD_HIP(hipStreamWaitEvent(s, e, 0));
            run_level<double>(*f, f->L64[exec_index[t]], s, false);
        }
        return true;
    };
    {
        QRChain<double> c64[NCH];
        QRChain<float> c32[NCH];
        int S = 0;
        double fl = 0, by = 0;
        ProfScope ps(RSD_PROF_INTERP, f->qr_stream[1]);   // flops and bytes filled in below
        auto set_up = [&](int c) {
            if (!cp[0][c].empty()) { c64[c].setup(cp[0][c], false, f->scratch, chain_stream(c)); S = std::max(S, c64[c].S); }
            if (!cp[1][c].empty()) { c32[c].setup(cp[1][c], false, f->scratch, chain_stream(c)); S = std::max(S, c32[c].S); }
            fl += c64[c].flops + c32[c].flops;
            by += c64[c].bytes + c32[c].bytes;
        };
        // the one-window chain first, on this thread: set up and enqueued
        // before anything else, since the lowest level waits for it
        set_up(0);
        {
            std::vector<int> done;
            publish(c32[0].window(0, done), done);
            done.clear();
            publish(c64[0].window(0, done), done);
        }
        // then the other chains, whose enqueue threads start before the
        // level tables are built (the top levels' chain is the longest)
        for (int c = 1; c < NCH; ++c) set_up(c);
        ps.rec.flops = fl;
        ps.rec.bytes = by;
        // two enqueue threads, one per chain stream: the long class 1 chain
        // (the top levels, many launches per window) on its own, so that its
        // enqueue does not hold back the windows that finish the middle
        // levels, which the level pipeline reaches first
        std::exception_ptr chain_err[2];
        const int dev = f->device;
        int running = 2;
        auto chain_thread = [&](int which) {
            try {
                RSD_HIP(hipSetDevice(dev));
                for (int sw = 0; sw < S; ++sw)
                    for (int c = 0; c < NCH; ++c) {
                        if ((c == 1) != (which == 1)) continue;
                        if (c == 0 && sw == 0) continue;
                        std::vector<int> done;
                        publish(c32[c].window(sw, done), done);
                        done.clear();
                        publish(c64[c].window(sw, done), done);
                    }
            } catch (...) {
                chain_err[which] = std::current_exception();
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                if (--running == 0) chains_done = true;
            }
            cv.notify_all();
        };
        std::thread chains0(chain_thread, 0);
        std::thread chains1;
        try {
            chains1 = std::thread(chain_thread, 1);
        } catch (const std::system_error&) {
            chain_thread(1);   // no second thread: the same work on this one
        }
        std::exception_ptr level_err;
        try {
            // the level tables, staged in pinned memory (a copy from pageable
            // memory would wait for the kernels of a stream sharing the
            // hardware queue), while the chain threads enqueue their windows:
            // first the Gauss-Jordan descriptors and the tables of the lowest
            // levels, whose interpolation the first window published, which
            // are enqueued at once, then the other levels' tables
            upload_gj<double>(f->gj64, f->L64, s, &f->staged[2]);
            upload_gj<float>(f->gj32, f->L32, s, &f->staged[3]);
            int n_early = 0;
            {
                std::lock_guard<std::mutex> lk(mu);
                while (n_early < nlev - 1 && pending[n_early] == 0) ++n_early;
            }
            std::vector<GemmBatch<double>*> e64, r64;
            std::vector<GemmBatch<float>*> e32, r32;
            auto split = [&](auto& all, auto& Ls, int prec, auto& early, auto& rest) {
                std::vector<const void*> mine;
                for (int t = 0; t < n_early; ++t) {
                    if (f->level_prec[t] != prec) continue;
                    auto& L = Ls[exec_index[t]];
                    for (const void* b : {(const void*)&L.g_sr, (const void*)&L.g_rr, (const void*)&L.g_E})
                        mine.push_back(b);
                    for (auto& b : L.g_gj) mine.push_back(&b);
                    for (auto& b : L.g_topgj) mine.push_back(&b);
                }
                for (auto* b : all)
                    (std::find(mine.begin(), mine.end(), (const void*)b) != mine.end() ? early : rest).push_back(b);
            };
            split(f->tables64, f->L64, 0, e64, r64);
            split(f->tables32, f->L32, 1, e32, r32);
            if (n_early > 0) {
                upload_batches<double>(f->gemm64e, e64, s, false, &f->staged[4], 1);
                upload_batches<float>(f->gemm32e, e32, s, false, &f->staged[5], 1);
                while (next_level < n_early && enqueue_next(false)) {
                }
            }
            upload_batches<double>(f->gemm64, r64, s, false, &f->staged[0], 1);
            upload_batches<float>(f->gemm32, r32, s, false, &f->staged[1], 1);
            while (next_level < nlev && enqueue_next(true)) {
            }
        } catch (...) {
            level_err = std::current_exception();
        }
        chains0.join();
        if (chains1.joinable()) chains1.join();
        for (auto& e : chain_err)
            if (e) std::rethrow_exception(e);
        if (level_err) std::rethrow_exception(level_err);
        // the interpolation profile ends when both streams have
        hipEvent_t done;
        RSD_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        RSD_HIP(hipEventRecord(done, f->qr_stream[0]));
        RSD_HIP(hipStreamWaitEvent(f->qr_stream[1], done, 0));
        f->tmp_events.push_back(done);
    }
    while (next_level < nlev && enqueue_next(false)) {
    }
    if (next_level != nlev) throw Error(RSD_EINVAL, "internal: interpolation problems left unsolved");
    RSD_HIP(hipEventRecord(f->build_ev[1], s));
}

// Sizes and flop / byte counts of a prepared factor (the build time is
// filled in by build_finish).
static void build_stats(Factor& fr) {
    Factor* f = &fr;
    Plan& P = f->plan;
    rsd_factor_stats& st = f->stats;
    st.n_points = f->N; st.nx = f->nx; st.ny = f->ny;
    st.n_levels = (int)P.levels.size();
    st.n_boxes = (int)P.boxes.size();
    st.layers = f->layers;
    st.precision = f->precision;
    st.complex_values = f->cplx;
    st.factor_bytes = (int64_t)(f->F64.bytes + f->F32.bytes + f->T64.bytes + f->T32.bytes);
    double fl = f->gemm_flops;
    for (auto& I : P.idps) {
        const double ns = split_sym(*f, I, interp_prec(*f, f->layout_level[I.layout])) ? I.nsec() : 1;
        const double p = I.p / ns, k = I.k / ns, r = I.r / ns;
        fl += ns * (2 * k * k * (p - k / 3) + 4 * p * k * r - 2 * k * k * r + k * k * r);
    }
    st.factor_flops = fl;
    double sb = 0;
    for (auto& b : P.boxes) {
        const int es = f->level_prec[b.level] ? 4 : 8;
        sb += (double)es * ((double)b.r * b.r + 2.0 * b.r * b.k);   // G, W twice
        if (b.level == f->top) sb += (double)es * b.k * b.k;
    }
    st.solve_bytes = sb;
}

// Host planning, uploads and every launch of a build; returns without waiting
// for the device (build_finish does).
static std::unique_ptr<Factor> build_enqueue(const double* points, int64_t n, const rsd_kernel* kernel,
                                             const double* a, double tol, const rsd_options* opt) {
    auto f = build_prepare(points, n, kernel, a, tol, opt);
    enqueue_single(*f);
    build_stats(*f);
    return f;
}

// Waits for an enqueued build, releases its temporaries and reports a singular
// pivot block if one was met.
// Right-hand-side count of the most recent solve.  While a build runs on the
// device, the host prepares the new factor's solve plan for that count (a
// repeated workload then finds it ready); a failure there is left to the
// first solve to report.
static std::atomic<int> g_last_nrhs{0};
static SolvePlan& get_solve_plan(Factor& f, int nrhs);

static void build_finish(Factor& f, bool plan_solve = true) {
    // the error word comes back with the stream's own completion
    if (!f.h_flag) f.h_flag = PinnedWords::get().take();
    RSD_HIP(hipMemcpyAsync(f.h_flag, f.d_err.p, sizeof(int), hipMemcpyDeviceToHost, f.stream));
    if (const int n = g_last_nrhs.load(std::memory_order_relaxed); plan_solve && n > 0 && n <= 64) {
        try {
            get_solve_plan(f, n);
        } catch (const std::exception&) {
            f.solve_plans.erase(n);
        }
    }
    RSD_HIP(hipStreamSynchronize(f.stream));
    for (auto q : f.qr_stream)
        if (q) RSD_HIP(hipStreamSynchronize(q));
    {
        IdleScope idle;     // the build's streams have drained
        f.scratch.clear();
    }
    for (auto& b : f.staged) b.release();
    for (auto e : f.tmp_events) (void)hipEventDestroy(e);
    f.tmp_events.clear();
    float ms = 0;
    if (f.build_ev[0] && f.build_ev[1]) RSD_HIP(hipEventElapsedTime(&ms, f.build_ev[0], f.build_ev[1]));
    for (auto& e : f.build_ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    f.stats.build_ms = ms;
    if (const int err = *f.h_flag; err != 0) {
        const int bx = err - 1;
        throw Error(RSD_ESINGULAR, "singular pivot block in box " + std::to_string(bx) + " at level " +
                                       std::to_string(f.plan.boxes[bx].level));
    }
}

// Streams and device buffers shared by the factors of a batch group (the
// interpolation chains and the merged levels).  Released only after the
// streams have drained, and before any factor of the group may be freed
// (they write into the factors' arenas).
struct GroupChains {
    hipStream_t qs[3] = {nullptr, nullptr, nullptr};   // two chain streams, the level stream
    int dev = 0;
    std::vector<std::unique_ptr<DevBuf>> buffers;
    PinnedBlock pinned[2];     // staged level tables; returned after the body has drained the streams
    std::vector<hipEvent_t> events;
    DevBuf& buffer() {
        buffers.push_back(std::make_unique<DevBuf>());
        return *buffers.back();
    }
    ~GroupChains() {
        for (auto q : qs)
            if (q) (void)hipStreamSynchronize(q);
        {
            IdleScope idle;
            buffers.clear();
        }
        for (auto e : events) (void)hipEventDestroy(e);
        for (auto q : qs) StreamPool::get().give(dev, q);
    }
};

// Enqueues the builds of a group of prepared factors together.  The
// interpolation problems of all of them form one set of chains, so every
// window is one launch per kernel for the whole group; then the levels,
// counted from the leaves, each merged over the group (one launch per
// product and per Gauss-Jordan step for the boxes of every factor), after
// the events of their box types.  A factor's T is bitwise what a build of
// its own computes; the merged level products may split long K ranges
// differently, which changes only the rounding order.
static void enqueue_group(const std::vector<Factor*>& group, GroupChains& gc) {
    constexpr int NCH = CHAIN_CLASSES;
    constexpr int TAG_LEVELS = 256;   // tag = member * TAG_LEVELS + level
    RSD_HIP(hipGetDevice(&gc.dev));
    for (auto& q : gc.qs) q = StreamPool::get().take();
    const int ng = (int)group.size();
    std::vector<ChainMember> cp[2][NCH];
    std::vector<std::vector<int>> pending(ng);
    std::vector<std::vector<std::vector<hipEvent_t>>> waits(ng);
    int max_lev = 0;
    for (int i = 0; i < ng; ++i) {
        Factor& F = *group[i];
        Plan& P = F.plan;
        const int nlev = (int)P.levels.size();
        if (nlev > TAG_LEVELS) throw Error(RSD_EINVAL, "internal: too many levels");
        max_lev = std::max(max_lev, nlev);
        pending[i].assign(nlev, 0);
        waits[i].resize(nlev);
        for (size_t li = 0; li < P.layouts.size(); ++li) {
            if (P.layouts[li].idp < 0) continue;
            const int lev = F.layout_level[li];
            const int ip = interp_prec(F, lev);
            int nprob = 1;
            const int cls = chain_class(F, P.idps[P.layouts[li].idp], ip, nprob);
            cp[ip][cls].push_back({&F, P.layouts[li].idp, lev, i * TAG_LEVELS + lev});
            pending[i][lev] += nprob;
        }
    }
    // the merged levels run on the group's level stream, after every factor's
    // uploads; their tables are built and staged by a second host thread
    // while this one sets up the chains, and go up before any window is
    // enqueued
    hipStream_t ls = gc.qs[2];
    for (auto* F : group) {
        hipEvent_t up;
        RSD_HIP(hipEventCreateWithFlags(&up, hipEventDisableTiming));
        gc.events.push_back(up);
        RSD_HIP(hipEventRecord(up, F->stream));
        RSD_HIP(hipStreamWaitEvent(ls, up, 0));
    }
    std::vector<GroupLevel<float>> G32(max_lev);
    std::vector<GroupLevel<double>> G64(max_lev);
    DevBuf &d32 = gc.buffer(), &d64 = gc.buffer(), &j32 = gc.buffer(), &j64 = gc.buffer();
    DevBuf &ai32 = gc.buffer(), &at32 = gc.buffer(), &ai64 = gc.buffer(), &at64 = gc.buffer();
    std::exception_ptr table_err;
    std::thread tables([&] {
        try {
            RSD_HIP(hipSetDevice(gc.dev));
            for (auto* F : group)
                for (int t = 0; t < (int)F->plan.levels.size(); ++t) {
                    if (F->level_prec[t]) G32[t].add(*F, F->L32[F->exec_index[t]]);
                    else G64[t].add(*F, F->L64[F->exec_index[t]]);
                }
            std::vector<GemmBatch<float>*> b32;
            std::vector<GemmBatch<double>*> b64;
            for (auto& g : G32) g.batches(b32);
            for (auto& g : G64) g.batches(b64);
            // tile tables on a few threads (hundreds of thousands of products)
            std::atomic<size_t> next{0};
            const size_t n32 = b32.size(), nall = b32.size() + b64.size();
            std::vector<std::exception_ptr> errs(nall);
            auto work = [&]() {
                for (size_t k = next++; k < nall; k = next++) {
                    try {
                        if (k < n32) b32[k]->finalize();
                        else b64[k - n32]->finalize();
                    } catch (...) {
                        errs[k] = std::current_exception();
                    }
                }
            };
            run_on_threads(6, work);
            for (auto& e : errs)
                if (e) std::rethrow_exception(e);
            upload_batches<float>(d32, b32, ls, true, &gc.pinned[0], 6);
            upload_batches<double>(d64, b64, ls, true, &gc.pinned[1], 6);
            upload_group_gj<float>(j32, G32, ls);
            upload_group_gj<double>(j64, G64, ls);
            upload_group_asm<float>(ai32, at32, G32, ls);
            upload_group_asm<double>(ai64, at64, G64, ls);
        } catch (...) {
            table_err = std::current_exception();
        }
    });
    auto chain_stream = [&](int c) { return gc.qs[c == 1 ? 1 : 0]; };
    QRChain<double> c64[NCH];
    QRChain<float> c32[NCH];
    int S = 0;
    double fl = 0, by = 0;
    std::exception_ptr setup_err;
    try {
        for (int c = 0; c < NCH; ++c) {
            if (!cp[0][c].empty()) { c64[c].setup(cp[0][c], true, gc.buffers, chain_stream(c)); S = std::max(S, c64[c].S); }
            if (!cp[1][c].empty()) { c32[c].setup(cp[1][c], true, gc.buffers, chain_stream(c)); S = std::max(S, c32[c].S); }
            fl += c64[c].flops + c32[c].flops;
            by += c64[c].bytes + c32[c].bytes;
        }
    } catch (...) {
        setup_err = std::current_exception();
    }
    tables.join();
    if (setup_err) std::rethrow_exception(setup_err);
    if (table_err) std::rethrow_exception(table_err);
    auto publish = [&](hipEvent_t ev, const std::vector<int>& done) {
        if (!ev) return;
        gc.events.push_back(ev);
        for (int tag : done) {
            const int i = tag / TAG_LEVELS, lev = tag % TAG_LEVELS;
            auto& w = waits[i][lev];
            if (w.empty() || w.back() != ev) w.push_back(ev);
            --pending[i][lev];
        }
    };
    // Each merged level is enqueued as soon as the windows that solve its box
    // types are: streams beyond the hardware queues share them in order of
    // submission, so a level enqueued after all windows would wait behind
    // every window on a shared queue.
    int next_t = 0;
    auto enqueue_ready = [&]() {
        for (; next_t < max_lev; ++next_t) {
            const int t = next_t;
            std::vector<hipEvent_t> w;
            for (int i = 0; i < ng; ++i) {
                if (t >= (int)group[i]->plan.levels.size()) continue;
                if (pending[i][t] != 0) return;
                for (auto e : waits[i][t])
                    if (std::find(w.begin(), w.end(), e) == w.end()) w.push_back(e);
            }
            for (auto e : w) RSD_HIP(hipStreamWaitEvent(ls, e, 0));
            G32[t].run(ls);
            G64[t].run(ls);
            for (auto* F : group)
                if (t + 1 == (int)F->plan.levels.size()) {
                    RSD_HIP(hipEventRecord(F->build_ev[1], ls));
                    RSD_HIP(hipStreamWaitEvent(F->stream, F->build_ev[1], 0));
                }
        }
    };
    {
        ProfScope ps(RSD_PROF_INTERP, gc.qs[1], fl, by);
        for (int sw = 0; sw < S; ++sw)
            for (int c = 0; c < NCH; ++c) {
                std::vector<int> done;
                publish(c32[c].window(sw, done), done);
                done.clear();
                publish(c64[c].window(sw, done), done);
                enqueue_ready();
            }
        hipEvent_t joined;
        RSD_HIP(hipEventCreateWithFlags(&joined, hipEventDisableTiming));
        gc.events.push_back(joined);
        RSD_HIP(hipEventRecord(joined, gc.qs[0]));
        RSD_HIP(hipStreamWaitEvent(gc.qs[1], joined, 0));
    }
    enqueue_ready();
    if (next_t != max_lev) throw Error(RSD_EINVAL, "internal: interpolation problems left unsolved");
}

static std::unique_ptr<Factor> build(const double* points, int64_t n, const rsd_kernel* kernel,
                                     const double* a, double tol, const rsd_options* opt) {
    auto f = build_enqueue(points, n, kernel, a, tol, opt);
    build_finish(*f);
    return f;
}

// ----------------------------------------------------------------------------
// solve
// ----------------------------------------------------------------------------
template <typename T> static T* Vbase(SolvePlan& sp);
template <> double* Vbase<double>(SolvePlan& sp) { return sp.V64.as<double>(); }
template <> float* Vbase<float>(SolvePlan& sp) { return sp.V32.as<float>(); }
template <typename T> static T* Ybase(SolvePlan& sp);
template <> double* Ybase<double>(SolvePlan& sp) { return sp.Y64.as<double>(); }
template <> float* Ybase<float>(SolvePlan& sp) { return sp.Y32.as<float>(); }

template <typename T>
static void plan_solve_level(Factor& f, SolvePlan& sp, SolveLevel<T>& SL, int t,
                             std::vector<GemmBatch<T>*>& all) {
    Plan& P = f.plan;
    const int nr = sp.nrhs;
    T* F = Fbase<T>(f);
    T* Tb = Tbase<T>(f);
    T* V = Vbase<T>(sp);
    T* Y = Ybase<T>(sp);
    for (int id : P.levels[t]) {
        const BoxDev& b = f.hboxes[id];
        const LayoutDev& LD = f.hlayouts[b.layout];
        const int k = b.k, r = b.r, m = k + r;
        T* Fb = F + b.offF;
        T* G = Fb + k + (int64_t)k * m;
        T* W = Fb + k;
        T* Vs = V + b.offV * nr;
        T* Vr = Vs + k;
        T* Yb = Y + b.offY * nr;
        const T* Tm = LD.offT >= 0 ? Tb + LD.offT : nullptr;
        if (r > 0) {
            if (Tm) SL.up1.add(gdesc<T>(r, nr, k, Tm, k, 1, Vs, m, 0, Vr, m, T(-1), T(1)));
            SL.up2.add(gdesc<T>(r, nr, r, G, m, 0, Vr, m, 0, Yb, r, T(1), T(0)));
            SL.up2.add(gdesc<T>(k, nr, r, W, m, 1, Vr, m, 0, Vs, m, T(-1), T(1)));
            SL.dn1.add(gdesc<T>(r, nr, k, W, m, 0, Vs, m, 0, Yb, r, T(-1), T(1)));
            if (Tm) SL.dn2.add(gdesc<T>(k, nr, r, Tm, k, 0, Yb, r, 0, Vs, m, T(-1), T(1)));
        }
        if (t == f.top) {
            // phi = G_top g  (g in Vs, result via tmp)
            T* tmp = reinterpret_cast<T*>(sp.tmp.p);
            SL.top.add(gdesc<T>(k, nr, k, Fb, m, 0, Vs, m, 0, tmp, k, T(1), T(0)));
        }
    }
    for (auto* b : {&SL.up1, &SL.up2, &SL.dn1, &SL.dn2, &SL.top}) {
        b->prof_cls = RSD_PROF_SOLVE_GEMM;
        all.push_back(b);
    }
}

static SolvePlan& get_solve_plan(Factor& f, int nrhs) {
    auto it = f.solve_plans.find(nrhs);
    if (it != f.solve_plans.end()) return *it->second;
    auto sp = std::make_unique<SolvePlan>();
    sp->nrhs = nrhs;
    int64_t v[2] = {0, 0}, y[2] = {0, 0};
    for (auto& b : f.hboxes) {
        const int prec = f.level_prec[b.level];
        v[prec] += b.k + b.r;
        y[prec] += b.r;
    }
    sp->V64.alloc(std::max<int64_t>(v[0] * nrhs, 1) * sizeof(double));
    sp->V32.alloc(std::max<int64_t>(v[1] * nrhs, 1) * sizeof(float));
    sp->Y64.alloc(std::max<int64_t>(y[0] * nrhs, 1) * sizeof(double));
    sp->Y32.alloc(std::max<int64_t>(y[1] * nrhs, 1) * sizeof(float));
    const Box& rb = f.plan.boxes[f.plan.root];
    sp->tmp.alloc(std::max<int64_t>((int64_t)rb.k * nrhs, 1) * sizeof(double));
    sp->in.alloc(f.N * nrhs * sizeof(double) * (f.cplx ? 2 : 1));
    sp->out.alloc(f.N * nrhs * sizeof(double) * (f.cplx ? 2 : 1));
    const int nlev = (int)f.plan.levels.size();
    sp->L32.resize(nlev);
    sp->L64.resize(nlev);
    std::vector<GemmBatch<double>*> b64;
    std::vector<GemmBatch<float>*> b32;
    for (int t = 0; t < nlev; ++t) {
        if (f.level_prec[t]) plan_solve_level<float>(f, *sp, sp->L32[t], t, b32);
        else plan_solve_level<double>(f, *sp, sp->L64[t], t, b64);
    }
    upload_batches<double>(sp->gemm64, b64, f.stream);
    upload_batches<float>(sp->gemm32, b32, f.stream);
    auto& ref = *sp;
    f.solve_plans[nrhs] = std::move(sp);
    return ref;
}

// x (grid or caller order per `perm`) = A^{-1} f, both device buffers with ld N
// The up sweep, the root and the down sweep of the inverse apply (Algorithm
// 6) between the leaf gather and the leaf scatter: every launch reads and
// writes only the solve plan's buffers and the factor's blocks.
static void apply_sweeps(Factor& f, SolvePlan& sp, hipStream_t s) {
    const int nr = sp.nrhs;
    const BoxDev* B = f.d_boxes.as<BoxDev>();
    const LayoutDev* LD = f.d_layouts.as<LayoutDev>();
    const int* inv = f.d_inv.as<int>();
    const int nlev = (int)f.plan.levels.size();
    auto nb = [&](int t) { return (int)f.plan.levels[t].size(); };
    auto maxk = [&](int t) { int m = 0; for (int id : f.plan.levels[t]) m = std::max(m, f.hboxes[id].k); return m; };
    for (int t = 0; t < nlev; ++t) {
        const int p = f.level_prec[t];
        if (p) { sp.L32[t].up1.run(s); sp.L32[t].up2.run(s); }
        else { sp.L64[t].up1.run(s); sp.L64[t].up2.run(s); }
        if (t < f.top) {
            const int pp = f.level_prec[t + 1];
            if (p && pp) launch_scatter_up<float, float>(sp.V32.as<float>(), sp.V32.as<float>(), nr, B, f.ids(t), nb(t), LD, inv, maxk(t), s);
            else if (p && !pp) launch_scatter_up<float, double>(sp.V64.as<double>(), sp.V32.as<float>(), nr, B, f.ids(t), nb(t), LD, inv, maxk(t), s);
            else launch_scatter_up<double, double>(sp.V64.as<double>(), sp.V64.as<double>(), nr, B, f.ids(t), nb(t), LD, inv, maxk(t), s);
        }
    }
    // top: phi = G_top g -> tmp, copy back into the root's skeleton part
    {
        sp.L64[f.top].top.run(s);
        const BoxDev& rb = f.hboxes[f.plan.root];
        const int m = rb.k + rb.r;
        double* Vs = sp.V64.as<double>() + rb.offV * nr;
        RSD_HIP(hipMemcpy2DAsync(Vs, m * sizeof(double), sp.tmp.p, rb.k * sizeof(double),
                                 rb.k * sizeof(double), nr, hipMemcpyDeviceToDevice, s));
    }
    for (int t = f.top; t >= 0; --t) {
        const int p = f.level_prec[t];
        if (t < f.top) {
            const int pp = f.level_prec[t + 1];
            if (p && pp) launch_gather_down<float, float>(sp.V32.as<float>(), sp.V32.as<float>(), sp.Y32.as<float>(), nr, B, f.ids(t), nb(t), LD, inv, maxk(t), s);
            else if (p && !pp) launch_gather_down<double, float>(sp.V32.as<float>(), sp.V64.as<double>(), sp.Y64.as<double>(), nr, B, f.ids(t), nb(t), LD, inv, maxk(t), s);
            else launch_gather_down<double, double>(sp.V64.as<double>(), sp.V64.as<double>(), sp.Y64.as<double>(), nr, B, f.ids(t), nb(t), LD, inv, maxk(t), s);
        }
        if (p) { sp.L32[t].dn1.run(s); sp.L32[t].dn2.run(s); }
        else { sp.L64[t].dn1.run(s); sp.L64[t].dn2.run(s); }
    }
}

// Whether the sweeps run as a captured graph: asked for, no profiler or
// tuner events to record, and a non-blocking stream (no implicit
// synchronisation with other threads' default-stream work during capture).
static bool sweeps_as_graph(const Factor& f) {
    if (!(f.flags & RSD_FLAG_SOLVE_GRAPH) || g_prof.on || Tuner::get().recording()) return false;
    unsigned int fl = 0;
    if (!f.stream || hipStreamGetFlags(f.stream, &fl) != hipSuccess) return false;
    return (fl & hipStreamNonBlocking) != 0;
}

// Captures the sweeps of a solve plan into a graph on first use (about a
// hundred launches replayed as one); falls back to launching them one by one
// when the runtime refuses the capture.
static void run_sweeps(Factor& f, SolvePlan& sp, hipStream_t s) {
    if (!sp.sweeps_failed && !sp.sweeps && sweeps_as_graph(f)) {
        hipGraph_t g = nullptr;
        RSD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            apply_sweeps(f, sp, s);
        } catch (...) {
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        const hipError_t e = hipStreamEndCapture(s, &g);
        hipGraphExec_t ge = nullptr;
        if (e == hipSuccess && g && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess) sp.sweeps = ge;
        else {
            (void)hipGetLastError();
            sp.sweeps_failed = true;
        }
        if (g) (void)hipGraphDestroy(g);
    }
    if (sp.sweeps && sweeps_as_graph(f)) RSD_HIP(hipGraphLaunch(sp.sweeps, s));
    else apply_sweeps(f, sp, s);
}

static void apply_inverse(Factor& f, SolvePlan& sp, const double* fin, double* xout,
                          const int64_t* perm) {
    hipStream_t s = f.stream;
    const int nr = sp.nrhs;
    const BoxDev* B = f.d_boxes.as<BoxDev>();
    const LayoutDev* LD = f.d_layouts.as<LayoutDev>();
    const int* lu = f.d_lu.as<int>();
    const int* lv = f.d_lv.as<int>();
    const int nb0 = (int)f.plan.levels[0].size();
    int maxm0 = 0;
    for (int id : f.plan.levels[0]) maxm0 = std::max(maxm0, f.hboxes[id].k + f.hboxes[id].r);
    // leaves (complex factors: fin holds the two dof planes of each column,
    // ld 2N, plane 1 at offset N)
    const int64_t ldv = f.cplx ? 2 * f.N : f.N, poff = f.cplx ? f.N : 0;
    if (f.level_prec[0]) launch_gather_leaf<double, float>(sp.V32.as<float>(), fin, ldv, nr, B, f.ids(0), nb0, LD, lu, lv, perm, f.ny, poff, maxm0, s);
    else launch_gather_leaf<double, double>(sp.V64.as<double>(), fin, ldv, nr, B, f.ids(0), nb0, LD, lu, lv, perm, f.ny, poff, maxm0, s);
    run_sweeps(f, sp, s);
    if (f.level_prec[0]) launch_scatter_leaf<float, double>(xout, ldv, sp.V32.as<float>(), sp.Y32.as<float>(), nr, B, f.ids(0), nb0, LD, lu, lv, perm, f.ny, poff, maxm0, s);
    else launch_scatter_leaf<double, double>(xout, ldv, sp.V64.as<double>(), sp.Y64.as<double>(), nr, B, f.ids(0), nb0, LD, lu, lv, perm, f.ny, poff, maxm0, s);
}

static void ensure_table(Factor& f) {
    if (f.d_table.p) return;
    if (f.cplx) throw Error(RSD_EINVAL, "the exact complex product needs grid sides of at most 2048 (FFT form)");
    f.d_table.alloc(f.N * sizeof(double));
    launch_matvec_table(f.d_table.as<double>(), f.nx, f.ny, f.kd_res, f.stream);
}

// y = A x, grid-ordered device vectors (interleaved complex for complex
// factors): the FFT form (circulant embedding) when the grid sides allow it,
// else the direct sum
static void matvec_grid(Factor& f, const double* x, double* y, int nrhs) {
    int mx = 0, my = 0;
    if (fft_matvec_sizes(f.nx, f.ny, &mx, &my)) {
        const double n = (double)mx * my;
        if (!f.fft_mx) {
            f.d_spec.alloc((size_t)n * sizeof(double) * (f.cplx ? 2 : 1));
            f.d_fftwork.alloc((size_t)n * 2 * sizeof(double));
            launch_fft_spectrum(f.d_spec.as<double>(), f.d_fftwork.as<double2>(), f.nx, f.ny, mx, my, f.kd_res,
                                f.stream);
            f.fft_mx = mx;
            f.fft_my = my;
        }
        const double fields = f.cplx ? nrhs : (nrhs + 1) / 2;
        ProfScope ps(RSD_PROF_MATVEC, f.stream, fields * 2 * 5.0 * n * std::log2(n), fields * 10.0 * 16.0 * n);
        launch_fft_matvec(y, x, nrhs, f.d_spec.as<double>(), f.d_fftwork.as<double2>(), f.nx, f.ny, mx, my,
                          f.kd_res, f.stream);
        return;
    }
    ensure_table(f);
    const double nn = (double)f.N;
    ProfScope ps(RSD_PROF_MATVEC, f.stream, 2.0 * nn * nn * nrhs, 16.0 * nn * nrhs);
    launch_matvec(y, x, nrhs, f.d_table.as<double>(), f.nx, f.ny, f.kd_res, 0, f.stream);
}

// Enqueues the finiteness check of a right-hand side; its flag reaches a
// pinned host word asynchronously, read by finite_check_failed after the
// next synchronisation of the factor's stream (so the check costs no round
// trip of its own).
static void start_finite_check(Factor& f, const double* x, int64_t n) {
    DevBuf& flag = f.d_flag;
    if (!flag.p) flag.alloc(sizeof(int));
    if (!f.h_flag) f.h_flag = PinnedWords::get().take();
    RSD_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), f.stream));
    launch_check_finite(x, n, flag.as<int>(), f.stream);
    RSD_HIP(hipMemcpyAsync(f.h_flag, flag.p, sizeof(int), hipMemcpyDeviceToHost, f.stream));
}

static void finite_check_failed(const Factor& f) {
    if (*f.h_flag) throw Error(RSD_EINVAL, "non-finite value in the right-hand side");
}

static rsd_status solve(Factor& f, const double* rhs, int64_t nrhs, double* x, rsd_solve_info* info) {
    std::lock_guard<std::mutex> use(f.use_mu);   // one solve plan and stream per factor
    if (nrhs < 0) throw Error(RSD_EINVAL, "nrhs < 0");
    if (info) { info->refine_iters = 0; info->rel_residual = -1; }
    if (nrhs == 0) return RSD_OK;
    if (!rhs || !x) throw Error(RSD_EINVAL, "null rhs or x");
    if (nrhs > 4096) throw Error(RSD_EINVAL, "nrhs > 4096");
    RSD_HIP(hipSetDevice(f.device));
    hipStream_t s = f.stream;
    g_last_nrhs.store((int)nrhs, std::memory_order_relaxed);
    SolvePlan& sp = get_solve_plan(f, (int)nrhs);
    const int w = f.cplx ? 2 : 1;                 // doubles per entry (interleaved complex)
    const int64_t tot = f.N * nrhs * w;
    const bool rdev = is_device_ptr(rhs), xdev = is_device_ptr(x);
    const double* fin = rhs;
    if (!rdev) {
        RSD_HIP(hipMemcpyAsync(sp.in.p, rhs, tot * sizeof(double), hipMemcpyHostToDevice, s));
        fin = sp.in.as<double>();
    }
    start_finite_check(f, fin, tot);
    double* xo = xdev ? x : sp.out.as<double>();
    rsd_status status = RSD_OK;
    // complex and contrast-form factors solve through the factored matrix M:
    // x = S^-1 M~^-1 S^-1 f, with the complex vectors carried on the two dof
    // planes of J(M)
    const bool scaled = f.cplx || f.kd_res.has_b;
    if (f.max_refine <= 0 && !scaled) {
        apply_inverse(f, sp, fin, xo, f.d_perm.as<int64_t>());
    } else {
        // grid-ordered work vectors fg, xg, rg, dg, ax and the plane blocks R, X
        if (!sp.refine_work.p) {
            sp.refine_work.alloc(7 * tot * sizeof(double));
            sp.refine_norms.alloc((2 + COLNORM_WS_PER_COL) * nrhs * sizeof(double));
        }
        double* fg = sp.refine_work.as<double>();
        double* xg = fg + tot;
        double* rg = xg + tot;
        double* dg = rg + tot;
        double* ax = dg + tot;
        double* R = ax + tot;
        double* X = R + tot;
        const double* sb = f.kd_res.has_b ? f.kd_res.sb : nullptr;
        auto inv = [&](const double* src, double* dst) {      // dst = A~^-1 src (grid order)
            if (!scaled) {
                apply_inverse(f, sp, src, dst, f.d_ident.as<int64_t>());
                return;
            }
            launch_scale_split(R, src, sb, f.N, (int)nrhs, f.cplx, s);
            apply_inverse(f, sp, R, X, f.d_ident.as<int64_t>());
            launch_scale_merge(dst, X, sb, f.N, (int)nrhs, f.cplx, s);
        };
        launch_permute(fg, fin, f.d_perm.as<int64_t>(), f.N, (int)nrhs, w, 1, s);
        inv(fg, xg);
        if (f.max_refine > 0) {
            DevBuf& nb = sp.refine_norms;
            double* nws = nb.as<double>() + 2 * nrhs;       // the norms' partial sums
            launch_col_norms2(nb.as<double>(), fg, f.N * w, (int)nrhs, nws, s);
            std::vector<double> fn(nrhs), rn(nrhs);
            RSD_HIP(hipMemcpyAsync(fn.data(), nb.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
            int it = 0;
            double worst = 0;
            for (;;) {
                matvec_grid(f, xg, ax, (int)nrhs);
                launch_axpy_resid(rg, fg, ax, tot, s);
                launch_col_norms2(nb.as<double>() + nrhs, rg, f.N * w, (int)nrhs, nws, s);
                RSD_HIP(hipMemcpyAsync(rn.data(), nb.as<double>() + nrhs, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
                RSD_HIP(hipStreamSynchronize(s));
                finite_check_failed(f);
                worst = 0;
                for (int c = 0; c < nrhs; ++c) {
                    const double rel = fn[c] > 0 ? std::sqrt(rn[c] / fn[c]) : std::sqrt(rn[c]);
                    if (!(rel <= worst)) worst = rel;      // a NaN residual stays NaN (never converged)
                }
                if (worst <= f.refine_tol || it >= f.max_refine) break;
                inv(rg, dg);
                launch_add(xg, dg, tot, s);
                ++it;
            }
            if (info) { info->refine_iters = it; info->rel_residual = worst; }
            if (worst > f.refine_tol) status = RSD_ENOCONV;
        }
        launch_permute(xo, xg, f.d_perm.as<int64_t>(), f.N, (int)nrhs, w, 0, s);
        RSD_HIP(hipStreamSynchronize(s));
    }
    if (!xdev) RSD_HIP(hipMemcpyAsync(x, xo, tot * sizeof(double), hipMemcpyDeviceToHost, s));
    RSD_HIP(hipStreamSynchronize(s));
    finite_check_failed(f);
    if (status == RSD_ENOCONV)
        throw Error(RSD_ENOCONV, "iterative refinement did not reach the tolerance");
    return status;
}

static void matvec(Factor& f, const double* xin, int64_t nrhs, double* y) {
    std::lock_guard<std::mutex> use(f.use_mu);
    if (nrhs < 0 || !xin || !y) throw Error(RSD_EINVAL, "bad matvec arguments");
    if (nrhs == 0) return;
    RSD_HIP(hipSetDevice(f.device));
    hipStream_t s = f.stream;
    const int w = f.cplx ? 2 : 1;
    const int64_t tot = f.N * nrhs * w;
    DevBuf buf;
    buf.alloc(3 * tot * sizeof(double));
    double* xi = buf.as<double>();
    double* xg = xi + tot;
    double* yg = xg + tot;
    if (is_device_ptr(xin)) RSD_HIP(hipMemcpyAsync(xi, xin, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
    else RSD_HIP(hipMemcpyAsync(xi, xin, tot * sizeof(double), hipMemcpyHostToDevice, s));
    launch_permute(xg, xi, f.d_perm.as<int64_t>(), f.N, (int)nrhs, w, 1, s);
    matvec_grid(f, xg, yg, (int)nrhs);
    launch_permute(xi, yg, f.d_perm.as<int64_t>(), f.N, (int)nrhs, w, 0, s);
    if (is_device_ptr(y)) RSD_HIP(hipMemcpyAsync(y, xi, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
    else RSD_HIP(hipMemcpyAsync(y, xi, tot * sizeof(double), hipMemcpyDeviceToHost, s));
    RSD_HIP(hipStreamSynchronize(s));
}

// ---- the compressed forward product (Sec. 2.3) ----------------------------------
// y ~ A x through the factor's skeletonization: charges up the tree, sibling
// blocks across, potentials down, the dense leaf blocks at the bottom (see
// k_hmatvec.hip).  O(N) work; accurate to the factor's interpolation.
static void matvec_compressed(Factor& f, const double* xin, int64_t nrhs, double* y) {
    std::lock_guard<std::mutex> use(f.use_mu);
    if (nrhs < 0 || !xin || !y) throw Error(RSD_EINVAL, "bad matvec arguments");
    if (f.cplx || f.kd.has_b || f.kd.type != 0)
        throw Error(RSD_EINVAL, "the compressed product is built for Laplace factors without a contrast");
    if (nrhs == 0) return;
    if (nrhs > 4096) throw Error(RSD_EINVAL, "nrhs > 4096");
    RSD_HIP(hipSetDevice(f.device));
    hipStream_t s = f.stream;
    const Plan& P = f.plan;
    const int nlev = (int)P.levels.size();
    const int64_t tot = f.N * nrhs;
    // box offsets count separately on float32 and float64 levels (as in the
    // solve's arenas): float32-level boxes first, float64-level ones after
    int64_t v[2] = {0, 0};
    for (auto& b : f.hboxes) v[f.level_prec[b.level]] += b.k + b.r;
    const int64_t varena = std::max<int64_t>(v[0] + v[1], 1) * nrhs;
    DevBuf buf;
    buf.alloc((2 * tot + 3 * varena) * sizeof(double));
    double* xi = buf.as<double>();
    double* yo = xi + tot;
    double* X = yo + tot;
    double* Y = X + varena;
    double* Pot = Y + varena;
    const bool xdev = is_device_ptr(xin), ydev = is_device_ptr(y);
    RSD_HIP(hipMemcpyAsync(xi, xin, tot * sizeof(double), xdev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    RSD_HIP(hipMemsetAsync(Pot, 0, varena * sizeof(double), s));
    const BoxDev* B = f.d_boxes.as<BoxDev>();
    const LayoutDev* LD = f.d_layouts.as<LayoutDev>();
    const int* lu = f.d_lu.as<int>();
    const int* lv = f.d_lv.as<int>();
    const int* inv = f.d_inv.as<int>();
    const int64_t* perm = f.d_perm.as<int64_t>();
    auto nb = [&](int t) { return (int)P.levels[t].size(); };
    auto maxk = [&](int t) { int m = 0; for (int id : P.levels[t]) m = std::max(m, f.hboxes[id].k); return m; };
    auto maxm = [&](int t) { int m = 0; for (int id : P.levels[t]) m = std::max(m, f.hboxes[id].k + f.hboxes[id].r); return m; };
    auto maxkk = [&](int t) {   // children's skeletons of a parent level
        int m = 0;
        for (int id : P.levels[t]) {
            const Box& b = P.boxes[id];
            if (b.child[0] >= 0) m = std::max(m, P.boxes[b.child[0]].k + P.boxes[b.child[1]].k);
        }
        return m;
    };
    // base of a level's boxes in each arena
    const int64_t o64 = v[1] * nrhs;
    auto at = [&](double* arena, int t) { return arena + (f.level_prec[t] ? 0 : o64); };
    launch_gather_leaf<double, double>(at(X, 0), xi, f.N, (int)nrhs, B, f.ids(0), nb(0), LD, lu, lv, perm, f.ny, 0,
                                       maxm(0), s);
    for (int t = 0; t < f.top; ++t) {   // charges up
        if (f.level_prec[t])
            launch_hmv_up<float>(at(X, t), at(X, t + 1), Tbase<float>(f), (int)nrhs, B, f.ids(t), nb(t), LD, inv,
                                 maxk(t), s);
        else
            launch_hmv_up<double>(at(X, t), at(X, t + 1), Tbase<double>(f), (int)nrhs, B, f.ids(t), nb(t), LD, inv,
                                  maxk(t), s);
    }
    for (int t = 1; t < nlev; ++t)      // sibling blocks across
        launch_hmv_sibling(at(Pot, t - 1), at(X, t), (int)nrhs, B, f.ids(t), nb(t), LD, lu, lv, inv, maxkk(t), f.kd, s);
    for (int t = f.top - 1; t >= 1; --t) {   // potentials down
        if (f.level_prec[t])
            launch_hmv_spread<float>(at(Y, t), at(Pot, t), Tbase<float>(f), (int)nrhs, B, f.ids(t), nb(t), LD, maxm(t), s);
        else
            launch_hmv_spread<double>(at(Y, t), at(Pot, t), Tbase<double>(f), (int)nrhs, B, f.ids(t), nb(t), LD, maxm(t), s);
        launch_hmv_push(at(Pot, t - 1), at(Y, t), (int)nrhs, B, f.ids(t - 1), nb(t - 1), LD, inv, maxk(t - 1), s);
    }
    if (f.level_prec[0])
        launch_hmv_leaf<float>(yo, f.N, at(X, 0), at(Pot, 0), Tbase<float>(f), (int)nrhs, B, f.ids(0), nb(0), LD, lu,
                               lv, perm, maxm(0), f.kd, s);
    else
        launch_hmv_leaf<double>(yo, f.N, at(X, 0), at(Pot, 0), Tbase<double>(f), (int)nrhs, B, f.ids(0), nb(0), LD,
                                lu, lv, perm, maxm(0), f.kd, s);
    RSD_HIP(hipMemcpyAsync(y, yo, tot * sizeof(double), ydev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    RSD_HIP(hipStreamSynchronize(s));
}

// ---- the exact product without device allocations ---------------------------
// Work space of rsd_matvec_noalloc: the grid-ordered copies of x and y, the
// circulant spectrum and the FFT field (or the direct sum's kernel table), in
// one file-scope device array per GPU.  Host code never passes the array's
// name to a kernel: its device address is looked up once per device
// (noalloc_scratch) and only that address is used.
constexpr int64_t NOALLOC_SCRATCH_BYTES = 64ll << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

static double* noalloc_scratch(int device) {
    static std::mutex mu;
    static std::vector<double*> ptrs;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)ptrs.size() <= device) ptrs.resize(device + 1, nullptr);
    if (!ptrs[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw Error(RSD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        ptrs[device] = static_cast<double*>(p);
    }
    return ptrs[device];
}

static void matvec_noalloc(Factor& f, const double* x, int64_t nrhs, double* y) {
    if (nrhs < 0 || !x || !y) throw Error(RSD_EINVAL, "bad matvec arguments");
    if (nrhs == 0) return;
    RSD_HIP(hipSetDevice(f.device));
    if (!is_device_ptr(x) || !is_device_ptr(y))
        throw Error(RSD_EINVAL, "rsd_matvec_noalloc takes device buffers only");
    const int w = f.cplx ? 2 : 1;                  // doubles per entry
    const int64_t tot = f.N * nrhs * w;
    int mx = 0, my = 0;
    const bool fft = fft_matvec_sizes(f.nx, f.ny, &mx, &my);
    if (!fft && f.cplx) throw Error(RSD_EINVAL, "the exact complex product needs grid sides of at most 2048");
    const int64_t n = (int64_t)mx * my;
    const int64_t need = 2 * tot + (fft ? (w + 2) * n : f.N);   // doubles
    const int64_t cap = NOALLOC_SCRATCH_BYTES / (int64_t)sizeof(double);
    if (need > cap)
        throw Error(RSD_EINVAL, "rsd_matvec_noalloc: " + std::to_string(need * 8) + " bytes of work space for N = " +
                                    std::to_string(f.N) + ", nrhs = " + std::to_string(nrhs) + " exceed its " +
                                    std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte maximum");
    double* base = noalloc_scratch(f.device);
    hipStream_t s = f.stream;
    double* xg = base;
    double* yg = xg + tot;
    double* rest = yg + tot;
    launch_permute(xg, x, f.d_perm.as<int64_t>(), f.N, (int)nrhs, w, 1, s);
    if (fft) {
        double* spec = rest;                                     // n (real) or 2n (complex) doubles
        double2* work = reinterpret_cast<double2*>(spec + w * n);   // 16-byte aligned: 2 tot and n are even
        launch_fft_spectrum(spec, work, f.nx, f.ny, mx, my, f.kd_res, s);
        launch_fft_matvec(yg, xg, (int)nrhs, spec, work, f.nx, f.ny, mx, my, f.kd_res, s);
    } else {
        double* table = rest;
        launch_matvec_table(table, f.nx, f.ny, f.kd_res, s);
        launch_matvec(yg, xg, (int)nrhs, table, f.nx, f.ny, f.kd_res, 0, s);
    }
    launch_permute(y, yg, f.d_perm.as<int64_t>(), f.N, (int)nrhs, w, 0, s);
    RSD_HIP(hipStreamSynchronize(s));
}

// ---- dense building blocks exposed for direct use ---------------------------
template <typename T>
static void dense_gemm(int M, int N, int K, int tA, int tB, double alpha, const void* A, int lda,
                       const void* B, int ldb, double beta, void* C, int ldc) {
    if (M < 0 || N < 0 || K < 0) throw Error(RSD_EINVAL, "negative size");
    if (M == 0 || N == 0) return;
    const int ra = tA ? K : M, ca = tA ? M : K, rb = tB ? N : K, cb = tB ? K : N;
    if (lda < std::max(1, ra) || ldb < std::max(1, rb) || ldc < std::max(1, M))
        throw Error(RSD_EINVAL, "leading dimension too small");
    hipStream_t s = nullptr;
    DevBuf dA, dB, dC, dd;
    const T* pA = static_cast<const T*>(A);
    const T* pB = static_cast<const T*>(B);
    T* pC = static_cast<T*>(C);
    const bool hc = !is_device_ptr(C);
    if (!is_device_ptr(A)) { dA.alloc((size_t)lda * ca * sizeof(T)); RSD_HIP(hipMemcpy(dA.p, A, (size_t)lda * ca * sizeof(T), hipMemcpyHostToDevice)); pA = dA.as<T>(); }
    if (!is_device_ptr(B)) { dB.alloc((size_t)ldb * cb * sizeof(T)); RSD_HIP(hipMemcpy(dB.p, B, (size_t)ldb * cb * sizeof(T), hipMemcpyHostToDevice)); pB = dB.as<T>(); }
    if (hc) { dC.alloc((size_t)ldc * N * sizeof(T)); RSD_HIP(hipMemcpy(dC.p, C, (size_t)ldc * N * sizeof(T), hipMemcpyHostToDevice)); pC = dC.as<T>(); }
    GemmBatch<T> b;
    b.role = 3;
    b.add(gdesc<T>(M, N, K, pA, lda, tA, pB, ldb, tB, pC, ldc, (T)alpha, (T)beta));
    std::vector<GemmBatch<T>*> all{&b};
    upload_batches<T>(dd, all, s);
    b.run(s);
    RSD_HIP(hipStreamSynchronize(s));
    if (hc) RSD_HIP(hipMemcpy(C, pC, (size_t)ldc * N * sizeof(T), hipMemcpyDeviceToHost));
}

template <typename T>
static void dense_gj(int n, void* A, int lda, int pair) {
    if (n < 0 || lda < std::max(1, n)) throw Error(RSD_EINVAL, "bad size");
    if (pair && (n & 1)) throw Error(RSD_EINVAL, "paired pivots need an even n");
    if (n == 0) return;
    hipStream_t s = nullptr;
    DevBuf dA, sr, sc, err, dd, dg;
    T* pA = static_cast<T*>(A);
    const bool host = !is_device_ptr(A);
    if (host) { dA.alloc((size_t)lda * n * sizeof(T)); RSD_HIP(hipMemcpy(dA.p, A, (size_t)lda * n * sizeof(T), hipMemcpyHostToDevice)); pA = dA.as<T>(); }
    sr.alloc((size_t)GJ_NB * n * sizeof(T));
    sc.alloc((size_t)n * GJ_NB * sizeof(T));
    err.alloc(4 * sizeof(int));
    RSD_HIP(hipMemset(err.p, 0, 4 * sizeof(int)));
    GJDesc<T> g;
    g.X = pA; g.ld = lda; g.n = n; g.ncols = n; g.pcol = 0; g.SR = sr.as<T>(); g.SC = sc.as<T>(); g.box = 0;
    check_gj_block(g);
    dg.alloc(sizeof(g));
    RSD_HIP(hipMemcpy(dg.p, &g, sizeof(g), hipMemcpyHostToDevice));
    const int steps = (n + GJ_NB - 1) / GJ_NB;
    std::vector<GemmBatch<T>> bs(steps);
    std::vector<GemmBatch<T>*> all;
    for (int st = 0; st < steps; ++st) {
        const int j0 = st * GJ_NB, nbe = std::min(GJ_NB, n - j0);
        GemmDesc<T> d = gdesc<T>(n, n, nbe, g.SC, n, 0, g.SR, GJ_NB, 0, pA, lda, T(-1), T(1));
        d.zc0 = j0; d.zc1 = j0 + nbe;
        bs[st].add(d);
        all.push_back(&bs[st]);
    }
    upload_batches<T>(dd, all, s);
    for (int st = 0; st < steps; ++st) {
        launch_gj_pivot<T>(dg.as<GJDesc<T>>(), 1, st, GJ_NB, (n + 63) / 64, err.as<int>(), pair, s);
        bs[st].run(s);
    }
    RSD_HIP(hipStreamSynchronize(s));
    int e[4];
    RSD_HIP(hipMemcpy(e, err.p, sizeof(e), hipMemcpyDeviceToHost));
    if (host) RSD_HIP(hipMemcpy(A, pA, (size_t)lda * n * sizeof(T), hipMemcpyDeviceToHost));
    if (e[0]) throw Error(RSD_ESINGULAR, "singular pivot block");
}

}  // namespace rsd

// ============================================================================
// C interface
// ============================================================================
struct rsd_factor {
    std::unique_ptr<rsd::Factor> impl;
};
struct rsd_plan {
    rsd::Plan plan;
};

using rsd::g_last_error;

template <typename Fn>
static rsd_status guarded(Fn&& fn) {
    try {
        g_last_error.clear();
        return fn();
    } catch (const rsd::Error& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const rsd::HipError& e) {
        g_last_error = e.what();
        return RSD_EDEVICE;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return RSD_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return RSD_EINVAL;
    }
}

extern "C" {

rsd_status rsd_pool_trim(int32_t device) {
    return guarded([&]() {
        rsd::DevicePool::get().trim(device);
        return RSD_OK;
    });
}

rsd_status rsd_pool_set_limit(int64_t bytes) {
    return guarded([&]() {
        rsd::DevicePool::get().set_limit(bytes < 0 ? -1 : bytes);
        return RSD_OK;
    });
}

rsd_status rsd_pool_cached_bytes(int32_t device, int64_t* out) {
    return guarded([&]() {
        if (!out) throw rsd::Error(RSD_EINVAL, "out is null");
        *out = rsd::DevicePool::get().cached(device);
        return RSD_OK;
    });
}

rsd_status rsd_build_factor(const double* points, int64_t n_points, const rsd_kernel* kernel,
                            const double* a, double tol, const rsd_options* opt, rsd_factor** out) {
    if (out) *out = nullptr;
    return guarded([&]() {
        if (!out) throw rsd::Error(RSD_EINVAL, "out is null");
        auto f = rsd::build(points, n_points, kernel, a, tol, opt);
        *out = new rsd_factor{std::move(f)};
        return RSD_OK;
    });
}

rsd_status rsd_build_factor_batched(int32_t n_inst, const double* const* points,
                                    const int64_t* n_points, const rsd_kernel* kernel,
                                    const double* const* a, double tol, const rsd_options* opt,
                                    int32_t max_inflight, rsd_factor** out) {
    if (out && n_inst > 0)
        for (int32_t i = 0; i < n_inst; ++i) out[i] = nullptr;
    std::vector<std::unique_ptr<rsd::Factor>> fs;
    int32_t where = -1;
    const rsd_status st = guarded([&]() {
        if (!out || !points || !n_points) throw rsd::Error(RSD_EINVAL, "null argument");
        if (kernel && (kernel->type != RSD_KERNEL_LAPLACE || kernel->contrast_b))
            throw rsd::Error(RSD_EINVAL, "batched builds take the Laplace kernel without contrast");
        if (n_inst <= 0) throw rsd::Error(RSD_EINVAL, "n_inst must be positive");
        if (opt && opt->hip_stream) throw rsd::Error(RSD_EINVAL, "batched builds use their own streams");
        const int32_t group = max_inflight > 0 ? max_inflight : 64;
        fs.resize(n_inst);
        for (int32_t g0 = 0; g0 < n_inst; g0 += group) {
            const int32_t g1 = std::min(n_inst, g0 + group);
            // destroyed (its streams drained) before any factor can be freed
            rsd::GroupChains chains;
            // host planning of the group's instances on a few threads
            {
                int dev = 0;
                RSD_HIP(hipGetDevice(&dev));
                const int nw = (int)std::min<int64_t>(g1 - g0, 8);
                std::vector<std::exception_ptr> errs(g1 - g0);
                std::atomic<int32_t> next{g0};
                auto work = [&]() {
                    const bool on_dev = hipSetDevice(dev) == hipSuccess;
                    for (int32_t i = next++; i < g1; i = next++) {
                        try {
                            if (!on_dev) throw rsd::HipError("hipSetDevice failed on a planning thread");
                            fs[i] = rsd::build_prepare(points[i], n_points[i], kernel, a ? a[i] : nullptr, tol, opt,
                                                       false);
                        } catch (...) {
                            errs[i - g0] = std::current_exception();
                        }
                    }
                };
                rsd::run_on_threads(nw, work);
                for (int32_t i = g0; i < g1; ++i)
                    if (errs[i - g0]) {
                        where = i;
                        std::rethrow_exception(errs[i - g0]);
                    }
            }
            std::vector<rsd::Factor*> members;
            for (int32_t i = g0; i < g1; ++i) members.push_back(fs[i].get());
            where = g0;
            rsd::enqueue_group(members, chains);
            for (int32_t i = g0; i < g1; ++i) {
                where = i;
                rsd::build_stats(*fs[i]);
                // (the batched solve makes its plans on several threads)
                rsd::build_finish(*fs[i], false);
            }
        }
        return RSD_OK;
    });
    if (st != RSD_OK) {
        const std::string msg = rsd::g_last_error;
        fs.clear();
        rsd::g_last_error = "instance " + std::to_string(where) + ": " + msg;
        return st;
    }
    for (int32_t i = 0; i < n_inst; ++i) out[i] = new rsd_factor{std::move(fs[i])};
    return RSD_OK;
}

rsd_status rsd_solve(rsd_factor* f, const double* rhs, int64_t nrhs, double* x, rsd_solve_info* info) {
    return guarded([&]() {
        if (!f) throw rsd::Error(RSD_EINVAL, "factor is null");
        return rsd::solve(*f->impl, rhs, nrhs, x, info);
    });
}

rsd_status rsd_solve_batched(int32_t n, rsd_factor* const* factors, const double* const* rhs, int64_t nrhs,
                             double* const* x, rsd_solve_info* info) {
    std::vector<rsd_status> st(n > 0 ? n : 0, RSD_OK);
    std::vector<std::string> msg(st.size());
    const rsd_status pre = guarded([&]() {
        if (n <= 0) throw rsd::Error(RSD_EINVAL, "n must be positive");
        if (!factors || !rhs || !x) throw rsd::Error(RSD_EINVAL, "null argument");
        std::vector<rsd_factor*> sorted(factors, factors + n);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            throw rsd::Error(RSD_EINVAL, "a factor appears twice");
        for (auto* f : sorted)
            if (!f) throw rsd::Error(RSD_EINVAL, "factor is null");
        return RSD_OK;
    });
    if (pre != RSD_OK) return pre;
    // every factor has its own stream: a few host threads keep several
    // solves (and their refinement round trips) in flight at once
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        for (int32_t i = next++; i < n; i = next++) {
            st[i] = guarded([&]() {
                return rsd::solve(*factors[i]->impl, rhs[i], nrhs, x[i], info ? &info[i] : nullptr);
            });
            if (st[i] != RSD_OK) msg[i] = rsd::g_last_error;
        }
    };
    rsd::run_on_threads(std::min<int32_t>(n, 8), work);
    rsd::g_last_error.clear();
    for (int32_t i = 0; i < n; ++i)
        if (st[i] != RSD_OK) {
            rsd::g_last_error = "instance " + std::to_string(i) + ": " + msg[i];
            return st[i];
        }
    return RSD_OK;
}

rsd_status rsd_matvec(rsd_factor* f, const double* x, int64_t nrhs, double* y) {
    return guarded([&]() {
        if (!f) throw rsd::Error(RSD_EINVAL, "factor is null");
        rsd::matvec(*f->impl, x, nrhs, y);
        return RSD_OK;
    });
}

rsd_status rsd_matvec_compressed(rsd_factor* f, const double* x, int64_t nrhs, double* y) {
    return guarded([&]() {
        if (!f) throw rsd::Error(RSD_EINVAL, "factor is null");
        rsd::matvec_compressed(*f->impl, x, nrhs, y);
        return RSD_OK;
    });
}

rsd_status rsd_autotune(int32_t n_inst, const double* const* points, const int64_t* n_points,
                        const rsd_kernel* kernel, const double* const* a, double tol, const rsd_options* opt,
                        int32_t reps, int32_t* n_entries) {
    if (n_entries) *n_entries = 0;
    return guarded([&]() {
        if (n_inst <= 0 || !points || !n_points) throw rsd::Error(RSD_EINVAL, "no instances to tune on");
        if (reps <= 0) reps = 1;
        rsd::Tuner& tu = rsd::Tuner::get();
        struct Reset {
            rsd::Tuner& t;
            ~Reset() {
                t.set_forced(-1);
                t.set_recording(false);
                t.collect();
            }
        } reset{tu};
        for (int c = 0; c < rsd::TUNE_CANDIDATES; ++c)
            for (int r = 0; r < reps; ++r) {
                tu.set_forced(c);
                tu.set_recording(true);
                if (n_inst == 1) {
                    rsd_factor* f = nullptr;
                    const rsd_status st = rsd_build_factor(points[0], n_points[0], kernel, a ? a[0] : nullptr, tol, opt, &f);
                    if (st != RSD_OK) throw rsd::Error(st, rsd::g_last_error);
                    rsd_free(f);
                } else {
                    std::vector<rsd_factor*> fs(n_inst, nullptr);
                    const rsd_status st = rsd_build_factor_batched(n_inst, points, n_points, kernel, a, tol, opt, 0, fs.data());
                    if (st != RSD_OK) throw rsd::Error(st, rsd::g_last_error);
                    for (auto* f : fs) rsd_free(f);
                }
                tu.set_recording(false);
                RSD_HIP(hipDeviceSynchronize());
                tu.collect();
            }
        tu.set_forced(-1);
        const int n = tu.commit();
        if (n_entries) *n_entries = n;
        return RSD_OK;
    });
}

rsd_status rsd_tune_save(const char* path) {
    return guarded([&]() {
        if (!path) throw rsd::Error(RSD_EINVAL, "null path");
        rsd::Tuner::get().save(path);
        return RSD_OK;
    });
}

rsd_status rsd_tune_load(const char* path) {
    return guarded([&]() {
        if (!path) throw rsd::Error(RSD_EINVAL, "null path");
        rsd::Tuner::get().load(path);
        return RSD_OK;
    });
}

rsd_status rsd_tune_clear(int64_t* n_entries_before) {
    return guarded([&]() {
        if (n_entries_before) *n_entries_before = rsd::Tuner::get().size();
        rsd::Tuner::get().clear();
        return RSD_OK;
    });
}

rsd_status rsd_matvec_noalloc(rsd_factor* f, const double* x, int64_t nrhs, double* y) {
    return guarded([&]() {
        if (!f) throw rsd::Error(RSD_EINVAL, "factor is null");
        rsd::matvec_noalloc(*f->impl, x, nrhs, y);
        return RSD_OK;
    });
}

void rsd_free(rsd_factor* f) { delete f; }

rsd_status rsd_profile_enable(int32_t on) {
    return guarded([&]() {
        if (!rsd::g_prof.recs.empty()) RSD_HIP(hipDeviceSynchronize());
        rsd::g_prof.clear();
        rsd::g_prof.on = on != 0;
        rsd::g_prof.paused = false;
        rsd::g_prof.mask = ~0u;
        return RSD_OK;
    });
}

rsd_status rsd_profile_enable_mask(uint32_t mask) {
    return guarded([&]() {
        if (!rsd::g_prof.recs.empty()) RSD_HIP(hipDeviceSynchronize());
        rsd::g_prof.clear();
        rsd::g_prof.on = mask != 0;
        rsd::g_prof.paused = false;
        rsd::g_prof.mask = mask;
        return RSD_OK;
    });
}

rsd_status rsd_profile_pause(int32_t paused) {
    return guarded([&]() {
        rsd::g_prof.paused = paused != 0;
        return RSD_OK;
    });
}

rsd_status rsd_profile_query(int32_t cls, double* total_ms, int64_t* launches, double* flops,
                             double* bytes) {
    return guarded([&]() {
        if (cls < 0 || cls >= RSD_PROF_NCLASS) throw rsd::Error(RSD_EINVAL, "unknown class");
        double ms = 0, fl = 0, by = 0;
        int64_t n = 0;
        for (auto& r : rsd::g_prof.recs) {
            if (r.cls != cls) continue;
            RSD_HIP(hipEventSynchronize(r.b));
            float e = 0;
            RSD_HIP(hipEventElapsedTime(&e, r.a, r.b));
            ms += e;
            fl += r.flops;
            by += r.bytes;
            ++n;
        }
        if (total_ms) *total_ms = ms;
        if (launches) *launches = n;
        if (flops) *flops = fl;
        if (bytes) *bytes = by;
        return RSD_OK;
    });
}

rsd_status rsd_profile_record_count(int64_t* n) {
    return guarded([&]() {
        if (!n) throw rsd::Error(RSD_EINVAL, "n is null");
        std::lock_guard<std::mutex> lk(rsd::g_prof.mu);
        *n = (int64_t)rsd::g_prof.recs.size();
        return RSD_OK;
    });
}

rsd_status rsd_profile_record(int64_t i, int32_t* cls, double* ms, double* flops, double* bytes,
                              int64_t* groups) {
    return guarded([&]() {
        rsd::ProfRec r;
        {
            std::lock_guard<std::mutex> lk(rsd::g_prof.mu);
            if (i < 0 || i >= (int64_t)rsd::g_prof.recs.size()) throw rsd::Error(RSD_EINVAL, "no such record");
            r = rsd::g_prof.recs[(size_t)i];
        }
        RSD_HIP(hipEventSynchronize(r.b));
        float e = 0;
        RSD_HIP(hipEventElapsedTime(&e, r.a, r.b));
        if (cls) *cls = r.cls;
        if (ms) *ms = e;
        if (flops) *flops = r.flops;
        if (bytes) *bytes = r.bytes;
        if (groups) *groups = r.groups;
        return RSD_OK;
    });
}

rsd_status rsd_gemm(int32_t dtype, int32_t M, int32_t N, int32_t K, int32_t tA, int32_t tB,
                    double alpha, const void* A, int32_t lda, const void* B, int32_t ldb,
                    double beta, void* C, int32_t ldc) {
    return guarded([&]() {
        if (!A || !B || !C) throw rsd::Error(RSD_EINVAL, "null matrix");
        if (dtype == 0) rsd::dense_gemm<double>(M, N, K, tA, tB, alpha, A, lda, B, ldb, beta, C, ldc);
        else if (dtype == 1) rsd::dense_gemm<float>(M, N, K, tA, tB, alpha, A, lda, B, ldb, beta, C, ldc);
        else throw rsd::Error(RSD_EINVAL, "dtype must be 0 or 1");
        return RSD_OK;
    });
}

rsd_status rsd_gj_invert(int32_t dtype, int32_t n, void* A, int32_t lda) {
    return guarded([&]() {
        if (!A) throw rsd::Error(RSD_EINVAL, "null matrix");
        if (dtype & ~3) throw rsd::Error(RSD_EINVAL, "dtype must be 0..3");
        const int pair = (dtype & 2) ? 1 : 0;
        if (dtype & 1) rsd::dense_gj<float>(n, A, lda, pair);
        else rsd::dense_gj<double>(n, A, lda, pair);
        return RSD_OK;
    });
}

const char* rsd_last_error(void) { return g_last_error.c_str(); }

rsd_status rsd_factor_get_stats(const rsd_factor* f, rsd_factor_stats* out) {
    return guarded([&]() {
        if (!f || !out) throw rsd::Error(RSD_EINVAL, "null argument");
        rsd::Factor& F = *f->impl;
        *out = F.stats;
        std::lock_guard<std::mutex> use(F.use_mu);
        out->solve_graphs = 0;
        for (const auto& kv : F.solve_plans) out->solve_graphs += kv.second->sweeps ? 1 : 0;
        return RSD_OK;
    });
}

rsd_status rsd_factor_box_info(const rsd_factor* f, int32_t box, rsd_box_info* out) {
    return guarded([&]() {
        if (!f || !out) throw rsd::Error(RSD_EINVAL, "null argument");
        const auto& P = f->impl->plan;
        if (box < 0 || box >= (int)P.boxes.size()) throw rsd::Error(RSD_EINVAL, "box out of range");
        const auto& b = P.boxes[box];
        *out = {b.level, b.x0, b.y0, b.ax, b.ay, b.k, b.r, b.parent};
        return RSD_OK;
    });
}

rsd_status rsd_factor_interp_info(const rsd_factor* fc, int32_t box, rsd_interp_info* out) {
    return guarded([&]() {
        if (!fc || !out) throw rsd::Error(RSD_EINVAL, "null argument");
        rsd::Factor& f = *fc->impl;
        const auto& P = f.plan;
        if (box < 0 || box >= (int)P.boxes.size()) throw rsd::Error(RSD_EINVAL, "box out of range");
        const int li = P.boxes[box].layout;
        *out = rsd_interp_info{};
        if (li < 0 || f.hlayouts[li].offT < 0) return RSD_OK;
        RSD_HIP(hipStreamSynchronize(f.stream));
        double rec[12];
        RSD_HIP(hipMemcpy(rec, f.d_interp.as<double>() + 12 * (int64_t)li, sizeof(rec), hipMemcpyDeviceToHost));
        const int n = (int)rec[2];
        if (n != 1 && n != 2 && n != 4) throw rsd::Error(RSD_EINVAL, "internal: no interpolation record for this box type");
        out->n_problems = n;
        out->damped = f.layout_damped[li];
        for (int sc = 0; sc < n; ++sc) {
            out->rank[sc] = (int32_t)rec[3 * sc];
            out->scale[sc] = rec[3 * sc + 1];
        }
        return RSD_OK;
    });
}

rsd_status rsd_factor_get_block(const rsd_factor* fc, int32_t box, int32_t which, void* dst) {
    return guarded([&]() {
        if (!fc || !dst) throw rsd::Error(RSD_EINVAL, "null argument");
        rsd::Factor& f = *fc->impl;
        const auto& P = f.plan;
        if (box < 0 || box >= (int)P.boxes.size()) throw rsd::Error(RSD_EINVAL, "box out of range");
        const auto& b = P.boxes[box];
        const auto& LD = f.hlayouts[b.layout];
        const int prec = f.level_prec[b.level];
        RSD_HIP(hipStreamSynchronize(f.stream));
        if (which == 2) {
            auto pts = rsd::box_points(P, box);
            std::memcpy(dst, pts.data(), pts.size() * sizeof(int64_t));
            return RSD_OK;
        }
        int64_t rows, cols, ld;
        const void* src;
        size_t es = prec ? sizeof(float) : sizeof(double);
        if (which == 0) {
            if (LD.offT < 0) throw rsd::Error(RSD_EINVAL, "this box has no interpolation matrix");
            rows = b.k; cols = b.r; ld = b.k;
            src = prec ? (const void*)(f.T32.as<float>() + LD.offT) : (const void*)(f.T64.as<double>() + LD.offT);
        } else if (which == 1) {
            if (!(f.flags & RSD_FLAG_KEEP_E)) throw rsd::Error(RSD_EINVAL, "build with RSD_FLAG_KEEP_E to read E blocks");
            if (box == P.root) throw rsd::Error(RSD_EINVAL, "the root has no E block");
            rows = b.k; cols = b.k; ld = b.k + b.r;
            src = prec ? (const void*)(f.F32.as<float>() + b.offF) : (const void*)(f.F64.as<double>() + b.offF);
        } else {
            throw rsd::Error(RSD_EINVAL, "unknown block kind");
        }
        std::vector<unsigned char> tmp(es * ld * cols);
        RSD_HIP(hipMemcpy(tmp.data(), src, tmp.size(), hipMemcpyDeviceToHost));
        double* d = static_cast<double*>(dst);
        for (int64_t j = 0; j < cols; ++j)
            for (int64_t i = 0; i < rows; ++i) {
                const size_t e = (size_t)(i + j * ld);
                d[i + j * rows] = prec ? (double)reinterpret_cast<float*>(tmp.data())[e]
                                       : reinterpret_cast<double*>(tmp.data())[e];
            }
        return RSD_OK;
    });
}

rsd_status rsd_plan_create(int64_t nx, int64_t ny, int32_t leaf_side, int32_t layers,
                           int32_t interface_step, rsd_plan** out) {
    if (out) *out = nullptr;
    return guarded([&]() {
        if (!out) throw rsd::Error(RSD_EINVAL, "out is null");
        if (interface_step < 0) throw rsd::Error(RSD_EINVAL, "interface_step must be >= 0");
        auto p = std::make_unique<rsd_plan>();
        p->plan = rsd::make_plan(nx, ny, leaf_side > 0 ? leaf_side : 8, layers > 0 ? layers : 2, interface_step);
        *out = p.release();
        return RSD_OK;
    });
}

rsd_status rsd_estimate_factor_bytes(int64_t nx, int64_t ny, const rsd_kernel* kernel, double tol,
                                     const rsd_options* opt, int64_t* bytes) {
    return guarded([&]() {
        if (!bytes) throw rsd::Error(RSD_EINVAL, "bytes is null");
        *bytes = 0;
        if (nx <= 0 || ny <= 0) throw rsd::Error(RSD_EINVAL, "grid sides must be positive");
        if (!(tol > 0) || !std::isfinite(tol)) throw rsd::Error(RSD_EINVAL, "tol must be a positive number");
        rsd_options o{};
        if (opt) o = *opt;
        if (o.precision != RSD_PREC_FP64 && o.precision != RSD_PREC_FP32_REFINE)
            throw rsd::Error(RSD_EINVAL, "unknown precision");
        const int leaf = o.leaf_side > 0 ? o.leaf_side : 8;
        const int m = o.layers > 0 ? o.layers : rsd::default_layers(tol, kernel ? kernel->type : RSD_KERNEL_LAPLACE);
        rsd::Plan P;
        try {
            // the interface spacing takes the unit-square spacing h = 1 / max(nx, ny)
            P = rsd::cached_plan(nx, ny, leaf, m,
                                 rsd::interface_step(kernel ? kernel->type : RSD_KERNEL_LAPLACE,
                                                     kernel ? kernel->wavenumber : 0.0,
                                                     1.0 / (double)std::max(nx, ny), o.interface_ppw));
        } catch (const std::exception& e) {
            throw rsd::Error(RSD_EINVAL, e.what());
        }
        // the arenas build_prepare allocates: one (k + r)^2 block per box and
        // one k x r interpolation block per layout that has one, in the
        // precision of the level (float32 below the root for FP32_REFINE)
        const int top = (int)P.levels.size() - 1;
        auto es = [&](int level) -> int64_t {
            return o.precision == RSD_PREC_FP32_REFINE && level < top ? 4 : 8;
        };
        int64_t f64 = 0, f32 = 0, t64 = 0, t32 = 0;
        std::vector<int> layout_level(P.layouts.size(), -1);
        for (auto& b : P.boxes) {
            layout_level[b.layout] = b.level;
            const int64_t mm = (int64_t)b.k + b.r;
            (es(b.level) == 4 ? f32 : f64) += mm * mm;
        }
        for (size_t li = 0; li < P.layouts.size(); ++li) {
            const rsd::Layout& L = P.layouts[li];
            if (L.idp < 0) continue;
            (es(layout_level[li]) == 4 ? t32 : t64) += (int64_t)L.k * L.r;
        }
        // complex factors hold every block on two dofs per point: 4x the entries
        const int64_t cx = kernel && kernel->type == RSD_KERNEL_HELMHOLTZ ? 4 : 1;
        *bytes = 8 * (std::max<int64_t>(cx * f64, 1) + std::max<int64_t>(cx * t64, 1)) +
                 4 * (std::max<int64_t>(cx * f32, 1) + std::max<int64_t>(cx * t32, 1));
        return RSD_OK;
    });
}

rsd_status rsd_self_cell_integral(int32_t kernel_type, double h, double k, double* re, double* im) {
    return guarded([&]() {
        if (!re || !im) throw rsd::Error(RSD_EINVAL, "null output");
        if (!(h > 0) || (kernel_type == RSD_KERNEL_HELMHOLTZ && !(k > 0)))
            throw rsd::Error(RSD_EINVAL, "h and the wavenumber must be positive");
        if (kernel_type != RSD_KERNEL_LAPLACE && kernel_type != RSD_KERNEL_HELMHOLTZ)
            throw rsd::Error(RSD_EINVAL, "unknown kernel type");
        rsd::self_cell_integral(kernel_type, h, k, *re, *im);
        return RSD_OK;
    });
}

int32_t rsd_plan_n_boxes(const rsd_plan* p) { return p ? (int32_t)p->plan.boxes.size() : 0; }
int32_t rsd_plan_n_levels(const rsd_plan* p) { return p ? (int32_t)p->plan.levels.size() : 0; }

rsd_status rsd_plan_box_info(const rsd_plan* p, int32_t box, rsd_box_info* out) {
    return guarded([&]() {
        if (!p || !out) throw rsd::Error(RSD_EINVAL, "null argument");
        if (box < 0 || box >= (int)p->plan.boxes.size()) throw rsd::Error(RSD_EINVAL, "box out of range");
        const auto& b = p->plan.boxes[box];
        *out = {b.level, b.x0, b.y0, b.ax, b.ay, b.k, b.r, b.parent};
        return RSD_OK;
    });
}

rsd_status rsd_plan_box_points(const rsd_plan* p, int32_t box, int64_t* dst) {
    return guarded([&]() {
        if (!p || !dst) throw rsd::Error(RSD_EINVAL, "null argument");
        if (box < 0 || box >= (int)p->plan.boxes.size()) throw rsd::Error(RSD_EINVAL, "box out of range");
        auto v = rsd::box_points(p->plan, box);
        std::memcpy(dst, v.data(), v.size() * sizeof(int64_t));
        return RSD_OK;
    });
}

rsd_status rsd_plan_box_symmetry(const rsd_plan* p, int32_t box, int32_t* group) {
    return guarded([&]() {
        if (!p || !group) throw rsd::Error(RSD_EINVAL, "null argument");
        if (box < 0 || box >= (int)p->plan.boxes.size()) throw rsd::Error(RSD_EINVAL, "box out of range");
        const auto& L = p->plan.layouts[p->plan.boxes[box].layout];
        *group = 0;
        if (L.idp >= 0) {
            const auto& I = p->plan.idps[L.idp];
            if (I.sym) *group = I.grp;
        }
        return RSD_OK;
    });
}

rsd_status rsd_plan_interp_groups(const rsd_plan* p, int32_t split, int32_t* n_problems,
                                  int32_t* table) {
    return guarded([&]() {
        if (!p || !n_problems) throw rsd::Error(RSD_EINVAL, "null argument");
        std::vector<rsd::QRProblemDev> qp;
        std::vector<int> owner;
        for (size_t id = 0; id < p->plan.idps.size(); ++id) {
            const rsd::IDProblem& I = p->plan.idps[id];
            rsd::append_sector_problems(qp, I, split != 0 && I.sym);
            owner.resize(qp.size(), (int)id);
        }
        rsd::check_sector_groups(qp, owner);
        *n_problems = (int32_t)qp.size();
        if (table)
            for (size_t i = 0; i < qp.size(); ++i) {
                int32_t* t = table + 7 * i;
                t[0] = owner[i]; t[1] = qp[i].sec; t[2] = qp[i].g0; t[3] = qp[i].gn;
                t[4] = qp[i].p; t[5] = qp[i].k; t[6] = qp[i].r;
            }
        return RSD_OK;
    });
}

rsd_status rsd_check_interp_groups(int32_t n_problems, const int32_t* table) {
    return guarded([&]() {
        if (n_problems < 0 || (n_problems > 0 && !table)) throw rsd::Error(RSD_EINVAL, "bad table");
        std::vector<rsd::QRProblemDev> qp(n_problems);
        std::vector<int> owner(n_problems);
        for (int i = 0; i < n_problems; ++i) {
            const int32_t* t = table + 7 * i;
            owner[i] = t[0];
            qp[i] = rsd::QRProblemDev{};
            qp[i].sec = t[1]; qp[i].g0 = t[2]; qp[i].gn = t[3];
            qp[i].p = t[4]; qp[i].k = t[5]; qp[i].r = t[6];
        }
        rsd::check_sector_groups(qp, owner);
        return RSD_OK;
    });
}

void rsd_plan_free(rsd_plan* p) { delete p; }

rsd_status rsd_detect_grid(const double* points_host, int64_t n_points, int64_t* nx, int64_t* ny,
                           double* h, int64_t* perm) {
    return guarded([&]() {
        if (!points_host || !nx || !ny || !h || !perm) throw rsd::Error(RSD_EINVAL, "null argument");
        std::vector<int64_t> pv;
        std::string why;
        double x0, y0;
        if (!rsd::detect_grid(points_host, n_points, *nx, *ny, *h, x0, y0, pv, why))
            throw rsd::Error(RSD_ENOTGRID, why);
        std::memcpy(perm, pv.data(), pv.size() * sizeof(int64_t));
        return RSD_OK;
    });
}

}  // extern "C"
