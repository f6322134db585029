// Serving runtime: resident factors in device memory, queued solve requests
// coalesced per factor and answered by worker threads (the inverse apply of
// Algorithm 6 for many clients), and factor requests admitted by memory and
// slots as they free up and built by a builder thread beside the solves.
// Built only on the public interface of the library (rsd_build_factor /
// rsd_solve / rsd_free / rsd_estimate_factor_bytes / rsd_detect_grid) plus
// HIP streams and copies, so a factor here is exactly what a direct call
// would build.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <stdexcept>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rsd.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    int64_t fid = 0;
    const double* rhs = nullptr;
    double* x = nullptr;
    int64_t nrhs = 0;
    Clock::time_point t_submit, t_done;
    bool done = false;
    rsd_status status = RSD_OK;
    rsd_solve_info info{0, -1.0};
};

// A factor request's inputs, owned by the server from submission until the
// build (the caller's buffers are borrowed for the submit call only).
struct FactorJob {
    std::vector<double> points, a, b;
    rsd_kernel kernel{};
    double tol = 0;
    rsd_options opt{};
};

enum SlotState { QUEUED = 0, BUILDING = 1, READY = 2 };

struct Slot {
    int state = QUEUED;
    std::unique_ptr<FactorJob> job;  // QUEUED and BUILDING
    rsd_factor* f = nullptr;
    hipStream_t stream = nullptr;
    int64_t n = 0;
    int w = 1;                       // doubles per vector entry (2: complex factor)
    int64_t bytes = 0;               // admission size (estimate until built)
    bool busy = false;
    Clock::time_point last_use;
    std::deque<int64_t> pending;     // tickets, oldest first
    double* dbuf = nullptr;          // in | out, n x cap columns each
    int64_t cap = 0;
};

int64_t pow2_at_least(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

struct rsd_server {
    rsd_server_options opt{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_build;
    std::map<int64_t, Slot> slots;                 // QUEUED, BUILDING and READY factors
    std::map<int64_t, rsd_status> failed;          // ids whose build failed
    std::unordered_map<int64_t, Request> reqs;
    std::vector<std::thread> workers;
    std::thread builder;
    bool stop = false;
    int64_t next_fid = 1, next_ticket = 1;
    int64_t resident = 0;                          // READY + BUILDING bytes
    // statistics
    int64_t n_requests = 0, n_done = 0, n_batches = 0, n_evicted = 0, rhs_done = 0, rhs_batched = 0;
    int64_t n_built = 0;
    std::vector<double> lat_ms;
    bool started = false;
    Clock::time_point t_first;

    int64_t n_ready() const {
        int64_t c = 0;
        for (auto& kv : slots) c += kv.second.state != QUEUED;
        return c;
    }

    // READY slot with queued work, not busy, whose oldest request is the oldest overall
    Slot* ready(int64_t* fid) {
        Slot* best = nullptr;
        int64_t best_ticket = INT64_MAX;
        for (auto& kv : slots) {
            Slot& sl = kv.second;
            if (sl.state != READY || sl.busy || sl.pending.empty()) continue;
            if (sl.pending.front() < best_ticket) {
                best_ticket = sl.pending.front();
                best = &sl;
                *fid = kv.first;
            }
        }
        return best;
    }

    void free_slot(Slot& sl) {
        if (sl.f) rsd_free(sl.f);
        if (sl.dbuf) (void)hipFree(sl.dbuf);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        sl = Slot{};
    }

    void complete(Request& r, rsd_status st, Clock::time_point now) {
        r.done = true;
        r.t_done = now;
        r.status = st;
        lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r.t_submit).count());
        rhs_done += r.nrhs;
        ++n_done;
    }

    // Frees room for `bytes` more (and one more slot) by evicting least
    // recently used idle READY factors when allowed; true when it fits.
    bool make_room(int64_t bytes) {
        for (;;) {
            if (n_ready() < opt.max_slots && resident + bytes <= opt.mem_budget) return true;
            if (!opt.evict_idle) return false;
            auto victim = slots.end();
            for (auto it = slots.begin(); it != slots.end(); ++it) {
                const Slot& v = it->second;
                if (v.state == READY && !v.busy && v.pending.empty() &&
                    (victim == slots.end() || v.last_use < victim->second.last_use))
                    victim = it;
            }
            if (victim == slots.end()) return false;
            resident -= victim->second.bytes;
            free_slot(victim->second);
            slots.erase(victim);
            ++n_evicted;
        }
    }

    // Admits queued factor requests in submission order as memory and slots
    // free up, and builds them one at a time on their own streams (the solve
    // workers keep serving resident factors meanwhile).
    void build_loop() {
        if (opt.device >= 0) (void)hipSetDevice(opt.device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            int64_t fid = 0;
            Slot* sl = nullptr;
            cv_build.wait(lk, [&] {
                sl = nullptr;
                for (auto& kv : slots)
                    if (kv.second.state == QUEUED) { sl = &kv.second; fid = kv.first; break; }
                return stop || (sl && make_room(sl->bytes));
            });
            if (!sl) return;   // stop and nothing queued
            if (!make_room(sl->bytes)) {
                // stopping with a request that cannot be admitted: fail it
                fail_slot(fid, RSD_ENOMEM);
                continue;
            }
            sl->state = BUILDING;
            resident += sl->bytes;
            FactorJob* job = sl->job.get();
            lk.unlock();
            rsd_factor* fac = nullptr;
            hipStream_t stream = nullptr;
            rsd_status st = RSD_OK;
            if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
                (void)hipGetLastError();
                stream = nullptr;
                st = RSD_EDEVICE;
            } else {
                rsd_options o = job->opt;
                o.hip_stream = stream;
                if (opt.device >= 0) o.device = opt.device;
                rsd_kernel kd = job->kernel;
                kd.contrast_b = job->b.empty() ? nullptr : job->b.data();
                st = rsd_build_factor(job->points.data(), (int64_t)job->points.size() / 2, &kd,
                                      job->a.empty() ? nullptr : job->a.data(), job->tol, &o, &fac);
            }
            rsd_factor_stats fs{};
            if (st == RSD_OK) (void)rsd_factor_get_stats(fac, &fs);
            lk.lock();
            ++n_built;
            Slot& s2 = slots[fid];      // BUILDING slots are never erased
            resident -= s2.bytes;
            s2.job.reset();
            if (st != RSD_OK) {
                if (fac) rsd_free(fac);
                if (stream) (void)hipStreamDestroy(stream);
                fail_slot(fid, st);
            } else {
                s2.f = fac;
                s2.stream = stream;
                s2.bytes = fs.factor_bytes + batch_bytes(s2.n * s2.w);
                resident += s2.bytes;
                s2.state = READY;
                s2.last_use = Clock::now();
            }
            cv_done.notify_all();
            cv_work.notify_all();
            cv_build.notify_all();
        }
    }

    // removes a QUEUED or BUILDING slot whose build failed; its queued solves
    // complete with the build's status
    void fail_slot(int64_t fid, rsd_status st) {
        auto it = slots.find(fid);
        if (it == slots.end()) return;
        const auto now = Clock::now();
        for (int64_t tk : it->second.pending) complete(reqs[tk], st, now);
        it->second.pending.clear();
        slots.erase(it);
        failed[fid] = st;
        cv_done.notify_all();
        cv_work.notify_all();
    }

    int64_t batch_bytes(int64_t n) const {
        return (int64_t)(6 * n * opt.max_coalesce) * (int64_t)sizeof(double);
    }

    void worker() {
        if (opt.device >= 0) (void)hipSetDevice(opt.device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            int64_t fid = 0;
            Slot* sl = nullptr;
            cv_work.wait(lk, [&] { return (sl = ready(&fid)) != nullptr || (stop && !building_or_queued()); });
            if (!sl) return;   // stop and nothing left
            sl->busy = true;
            std::vector<int64_t> batch;
            int64_t cols = 0;
            while (!sl->pending.empty()) {
                const int64_t tk = sl->pending.front();
                const int64_t c = reqs[tk].nrhs;
                if (!batch.empty() && cols + c > opt.max_coalesce) break;
                batch.push_back(tk);
                cols += c;
                sl->pending.pop_front();
            }
            std::vector<Request*> rq;
            for (int64_t tk : batch) rq.push_back(&reqs[tk]);   // stable: nodes of an unordered_map
            lk.unlock();
            rsd_status st = run_batch(*sl, rq, cols);
            lk.lock();
            const auto now = Clock::now();
            for (Request* r : rq) complete(*r, (st != RSD_OK && r->status == RSD_OK) ? st : r->status, now);
            n_batches += 1;
            rhs_batched += cols;
            sl->busy = false;
            sl->last_use = now;
            (void)fid;
            cv_done.notify_all();
            cv_work.notify_all();
            cv_build.notify_all();     // an idle factor may now be evicted
        }
    }

    bool building_or_queued() const {
        for (auto& kv : slots)
            if (kv.second.state != READY) return true;
        return false;
    }

    // one coalesced solve: gather the right-hand sides into n x P columns (P a
    // power of two, zero padding), solve, scatter the solutions back
    rsd_status run_batch(Slot& sl, std::vector<Request*>& rq, int64_t cols) {
        const int64_t n = sl.n * sl.w;   // doubles per column
        const int64_t P = pow2_at_least(cols);
        if (P > sl.cap) {
            if (sl.dbuf) (void)hipFree(sl.dbuf);
            sl.dbuf = nullptr;
            if (hipMalloc(&sl.dbuf, (size_t)(2 * n * P) * sizeof(double)) != hipSuccess) {
                (void)hipGetLastError();
                sl.cap = 0;
                for (Request* r : rq) r->status = RSD_ENOMEM;
                return RSD_ENOMEM;
            }
            sl.cap = P;
        }
        double* in = sl.dbuf;
        double* out = sl.dbuf + n * sl.cap;
        int64_t off = 0;
        for (Request* r : rq) {
            (void)hipMemcpyAsync(in + off * n, r->rhs, (size_t)(n * r->nrhs) * sizeof(double),
                                 hipMemcpyDefault, sl.stream);
            off += r->nrhs;
        }
        if (P > cols)
            (void)hipMemsetAsync(in + cols * n, 0, (size_t)((P - cols) * n) * sizeof(double), sl.stream);
        rsd_solve_info info{0, -1.0};
        const rsd_status st = rsd_solve(sl.f, in, P, out, &info);
        if (st == RSD_OK || st == RSD_ENOCONV) {
            off = 0;
            for (Request* r : rq) {
                (void)hipMemcpyAsync(r->x, out + off * n, (size_t)(n * r->nrhs) * sizeof(double),
                                     hipMemcpyDefault, sl.stream);
                off += r->nrhs;
                r->info = info;
                r->status = st;
            }
        } else {
            for (Request* r : rq) r->status = st;
        }
        if (hipStreamSynchronize(sl.stream) != hipSuccess) {
            (void)hipGetLastError();
            for (Request* r : rq) r->status = RSD_EDEVICE;
            return RSD_EDEVICE;
        }
        return st;
    }
};

// No C++ exception crosses the C interface: a failed allocation inside a
// call is reported as RSD_ENOMEM.
template <typename Fn>
static rsd_status no_throw(Fn&& fn) {
    try {
        return fn();
    } catch (const std::bad_alloc&) {
        return RSD_ENOMEM;
    } catch (const std::exception&) {
        return RSD_EINVAL;
    }
}

extern "C" {

rsd_status rsd_server_create(const rsd_server_options* opt, rsd_server** out) {
    if (!out) return RSD_EINVAL;
    *out = nullptr;
    auto* s = new (std::nothrow) rsd_server();
    if (!s) return RSD_ENOMEM;
    if (opt) s->opt = *opt;
    if (s->opt.device >= 0 && hipSetDevice(s->opt.device) != hipSuccess) {
        delete s;
        return RSD_EDEVICE;
    }
    if (s->opt.max_slots <= 0) s->opt.max_slots = 16;
    if (s->opt.n_workers <= 0) s->opt.n_workers = 2;
    if (s->opt.max_coalesce <= 0) s->opt.max_coalesce = 64;
    s->opt.evict_idle = s->opt.evict_idle ? 1 : 0;
    if (s->opt.mem_budget <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return RSD_EDEVICE;
        }
        s->opt.mem_budget = (int64_t)(fr / 4 * 3);
    }
    try {
        s->builder = std::thread([s] { s->build_loop(); });
        for (int i = 0; i < s->opt.n_workers; ++i) s->workers.emplace_back([s] { s->worker(); });
    } catch (const std::exception&) {
        rsd_server_destroy(s);     // stops and joins the threads started so far
        return RSD_ENOMEM;
    }
    *out = s;
    return RSD_OK;
}

static void copy_in(std::vector<double>& dst, const double* src, int64_t n) {
    dst.resize((size_t)n);
    if (n == 0) return;
    hipPointerAttribute_t at{};
    bool dev = false;
    if (hipPointerGetAttributes(&at, src) == hipSuccess)
        dev = at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
    else
        (void)hipGetLastError();
    if (dev) {
        if (hipMemcpy(dst.data(), src, (size_t)n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            (void)hipGetLastError();
            throw std::runtime_error("copy of a device input failed");
        }
    } else {
        std::memcpy(dst.data(), src, (size_t)n * sizeof(double));
    }
}

rsd_status rsd_server_submit_factor(rsd_server* s, const double* points, int64_t n_points,
                                    const rsd_kernel* kernel, const double* a, double tol,
                                    const rsd_options* opt, int64_t* factor_id) {
    return no_throw([&]() -> rsd_status {
        if (!s || !factor_id || !points || n_points <= 0) return RSD_EINVAL;
        if (opt && opt->hip_stream) return RSD_EINVAL;
        if (!(tol > 0)) return RSD_EINVAL;
        auto job = std::make_unique<FactorJob>();
        if (s->opt.device >= 0) (void)hipSetDevice(s->opt.device);
        copy_in(job->points, points, 2 * n_points);
        if (a) copy_in(job->a, a, n_points);
        if (kernel) {
            job->kernel = *kernel;
            if (kernel->contrast_b) copy_in(job->b, kernel->contrast_b, n_points);
        } else {
            job->kernel.type = RSD_KERNEL_LAPLACE;
        }
        job->kernel.contrast_b = nullptr;
        job->tol = tol;
        if (opt) job->opt = *opt;
        job->opt.hip_stream = nullptr;
        // grid and size now, so that a request that can never be built or
        // admitted fails here rather than in the queue
        int64_t nx = 0, ny = 0, est = 0;
        double h = 0;
        std::vector<int64_t> perm((size_t)n_points);
        rsd_status st = rsd_detect_grid(job->points.data(), n_points, &nx, &ny, &h, perm.data());
        if (st != RSD_OK) return st;
        st = rsd_estimate_factor_bytes(nx, ny, &job->kernel, tol, &job->opt, &est);
        if (st != RSD_OK) return st;
        const int w = job->kernel.type == RSD_KERNEL_HELMHOLTZ ? 2 : 1;
        std::lock_guard<std::mutex> lk(s->mu);
        const int64_t bytes = est + s->batch_bytes(n_points * w);
        if (bytes > s->opt.mem_budget) return RSD_ENOMEM;
        const int64_t id = s->next_fid++;
        Slot& sl = s->slots[id];
        sl.job = std::move(job);
        sl.n = n_points;
        sl.w = w;
        sl.bytes = bytes;
        sl.state = QUEUED;
        *factor_id = id;
        s->cv_build.notify_all();
        return RSD_OK;
    });
}

rsd_status rsd_server_wait_factor(rsd_server* s, int64_t factor_id, int32_t timeout_ms) {
    return no_throw([&]() -> rsd_status {
        if (!s) return RSD_EINVAL;
        std::unique_lock<std::mutex> lk(s->mu);
        auto settled = [&] {
            auto it = s->slots.find(factor_id);
            return it == s->slots.end() || it->second.state == READY;
        };
        if (timeout_ms < 0) s->cv_done.wait(lk, settled);
        else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), settled)) return RSD_EAGAIN;
        if (s->slots.count(factor_id)) return RSD_OK;
        auto f = s->failed.find(factor_id);
        return f != s->failed.end() ? f->second : RSD_EINVAL;
    });
}

rsd_status rsd_server_release_factor(rsd_server* s, int64_t factor_id) {
    return no_throw([&]() -> rsd_status {
        if (!s) return RSD_EINVAL;
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->slots.find(factor_id);
        if (it == s->slots.end()) return RSD_EINVAL;
        Slot& sl = it->second;
        if (sl.state == BUILDING || sl.busy || !sl.pending.empty()) return RSD_EAGAIN;
        if (sl.state == READY) s->resident -= sl.bytes;
        s->free_slot(sl);
        s->slots.erase(it);
        s->cv_build.notify_all();     // memory and a slot freed: admit the next request
        return RSD_OK;
    });
}

rsd_status rsd_server_submit_solve(rsd_server* s, int64_t factor_id, const double* rhs,
                                   int64_t nrhs, double* x, int64_t* ticket) {
    return no_throw([&]() -> rsd_status {
        if (!s || !ticket || !rhs || !x || nrhs <= 0) return RSD_EINVAL;
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->slots.find(factor_id);
        if (it == s->slots.end()) return RSD_EINVAL;
        if (nrhs > s->opt.max_coalesce) return RSD_EINVAL;
        const int64_t tk = s->next_ticket++;
        Request& r = s->reqs[tk];
        r.fid = factor_id;
        r.rhs = rhs;
        r.x = x;
        r.nrhs = nrhs;
        r.t_submit = Clock::now();
        if (!s->started) {
            s->started = true;
            s->t_first = r.t_submit;
        }
        it->second.pending.push_back(tk);
        ++s->n_requests;
        *ticket = tk;
        s->cv_work.notify_one();
        return RSD_OK;
    });
}

rsd_status rsd_server_wait(rsd_server* s, int64_t ticket, int32_t timeout_ms, rsd_solve_info* info) {
    return no_throw([&]() -> rsd_status {
        if (!s) return RSD_EINVAL;
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return RSD_EINVAL;
        auto is_done = [&] { return s->reqs[ticket].done; };
        if (timeout_ms < 0) s->cv_done.wait(lk, is_done);
        else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), is_done)) return RSD_EAGAIN;
        Request r = s->reqs[ticket];
        s->reqs.erase(ticket);
        if (info) *info = r.info;
        return r.status;
    });
}

int32_t rsd_server_poll(rsd_server* s, int64_t ticket) {
    if (!s) return -1;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return -1;
    return it->second.done ? 1 : 0;
}

rsd_status rsd_server_get_stats(rsd_server* s, rsd_server_stats* out) {
    return no_throw([&]() -> rsd_status {
        if (!s || !out) return RSD_EINVAL;
        std::lock_guard<std::mutex> lk(s->mu);
        std::memset(out, 0, sizeof(*out));
        out->n_requests = s->n_requests;
        out->n_done = s->n_done;
        out->n_batches = s->n_batches;
        int64_t ready = 0, queued = 0;
        for (auto& kv : s->slots) (kv.second.state == READY ? ready : queued) += 1;
        out->n_factors = ready;
        out->n_queued_factors = queued;
        out->n_built = s->n_built;
        out->n_evicted = s->n_evicted;
        out->resident_bytes = s->resident;
        if (!s->lat_ms.empty()) {
            std::vector<double> v = s->lat_ms;
            std::sort(v.begin(), v.end());
            auto pct = [&](double q) {
                const size_t i = (size_t)std::min<double>((double)v.size() - 1, q * (double)(v.size() - 1) + 0.5);
                return v[i];
            };
            out->p50_ms = pct(0.50);
            out->p99_ms = pct(0.99);
        }
        out->mean_batch_rhs = s->n_batches ? (double)s->rhs_batched / (double)s->n_batches : 0.0;
        if (s->started) {
            const double el = std::chrono::duration<double>(Clock::now() - s->t_first).count();
            out->rhs_per_s = el > 0 ? (double)s->rhs_done / el : 0.0;
        }
        return RSD_OK;
    });
}

void rsd_server_destroy(rsd_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_build.notify_all();
    s->cv_work.notify_all();
    if (s->builder.joinable()) s->builder.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->slots) s->free_slot(kv.second);
    delete s;
}

}  // extern "C"
