// Continuous-batching server for edge-posterior solves (bn_server_* calls).
//
// A worker thread owns the device side. Submitted requests (inputs copied at
// submit) wait in a FIFO queue; the worker admits the head whenever its
// device footprint fits in the memory budget and fewer than max_active
// solves are in flight. Each admitted solve is enqueued whole on one of
// several HIP streams, so requests that arrive while others run are started
// as soon as a slot and memory free up and their kernels overlap on the
// device. Completion is observed through an event per request; the worker
// then releases the request's device memory and admits more.
//
// The budget is charged with the device bytes a request really holds (its
// block from the cache may be larger than the plan). When an admitted
// request cannot get device memory while other solves are running, it goes
// back to the head of the queue and admission pauses until one of them
// completes; only a request that fails with nothing else on the device
// resolves to BN_ENOMEM.
//
// The device work sits behind an Executor interface. BN_SERVE_FAKE=1 at
// server creation selects a CPU executor (timed placeholder results) so the
// scheduling logic -- admission, ordering, cancellation, failure paths --
// can be tested without a GPU (BN_SERVE_FAKE_MS fixes its per-request
// duration). BN_SERVE_FAIL_ALLOC=k makes the k-th
// allocation (1-based) fail, to test that path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bn.h"
#include "bn_arena.h"
#include "bn_solver.h"

namespace bnk {

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t ticket = 0;
    enum State { PENDING, RUNNING, DONE } state = PENDING;
    bn_status status = BN_EAGAIN;
    // copied inputs
    bn_problem p{};
    std::vector<uint8_t> data, arity;
    std::vector<double> log_rho, log_q;
    bn_precision prec = BN_FP32_SCALED;
    size_t footprint = 0;   // admission estimate (the plan, rounded as allocated)
    size_t charged = 0;     // bytes counted against the budget while admitted
    // results
    std::vector<double> post;
    bn_report rep{};
    double t_submit = 0, t_admit = 0, t_done = 0;
    // executor state
    void *ws = nullptr, *hpin = nullptr;
    size_t ws_bytes = 0, hpin_bytes = 0;   // sizes of the (cached) blocks held
    hipStream_t st = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double fake_until = 0;
};

class Executor {
   public:
    virtual ~Executor() = default;
    virtual size_t footprint(const Req &r) = 0;
    // Starts the solve; returns false (with r.status set) on failure.
    virtual bool start(Req &r) = 0;
    // Device bytes the started request actually holds (a cached block may
    // be larger than its footprint).
    virtual size_t held(const Req &r) { return r.footprint; }
    // True once the solve has finished (results then written into r).
    virtual bool done(Req &r) = 0;
    virtual void release(Req &r) = 0;

    int fail_at = -1;   // 1-based index of an allocation to fail (test hook)
    int allocs = 0;
    bool alloc_fails() { return ++allocs == fail_at; }
};

// ------------------------------------------------------------ device arena
// Workspaces come from the chunked arena of bn_arena.h over device memory.
struct HipMem {
    static bool alloc(size_t bytes, void **p) {
        if (hipMalloc(p, bytes) == hipSuccess) return true;
        (void)hipGetLastError();
        return false;
    }
    static void release(void *p) { (void)hipFree(p); }
};
using DeviceArena = Arena<HipMem>;

// ------------------------------------------------------------ GPU executor
// Device workspaces come from the arena above; pinned host blocks and events
// of finished requests are kept for reuse (a request takes the smallest
// cached host block that fits and is at most 1.25 times its size).
class GpuExecutor : public Executor {
   public:
    GpuExecutor(int dev, int nstreams, size_t budget) : dev_(dev), arena_(budget) {
        (void)hipSetDevice(dev_);
        for (int k = 0; k < nstreams; ++k) {
            hipStream_t s;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess)
                streams_.push_back(s);
        }
    }
    ~GpuExecutor() override {
        (void)hipSetDevice(dev_);
        for (auto s : streams_) (void)hipStreamDestroy(s);
        for (auto &kv : host_cache_) (void)hipHostFree(kv.second);
        for (auto e : events_) (void)hipEventDestroy(e);
    }
    bool ok() const { return !streams_.empty(); }
    size_t footprint(const Req &r) override {
        return round_up(make_plan(r.p.n, r.p.d, r.p.m, r.prec, true, true).total,
                        DeviceArena::kGranule);
    }
    size_t held(const Req &r) override { return r.ws_bytes; }
    bool start(Req &r) override {
        (void)hipSetDevice(dev_);
        const Plan P = make_plan(r.p.n, r.p.d, r.p.m, r.prec, true, true);
        const size_t nn = (size_t)r.p.n * r.p.n, dbytes = (size_t)r.p.n * r.p.m;
        if (alloc_fails() || !arena_.get(P.total, &r.ws, &r.ws_bytes)) {
            r.ws = nullptr;
            r.status = BN_ENOMEM;
            return false;
        }
        // pinned host block: post (n*n), diag (16), data (n*m)
        if (!get_host((nn + 16) * 8 + dbytes + 8, &r.hpin, &r.hpin_bytes)) {
            arena_.put(r.ws, r.ws_bytes);
            r.ws = nullptr;
            r.status = BN_ENOMEM;
            return false;
        }
        double *hpost = reinterpret_cast<double *>(r.hpin);
        double *hdiag = hpost + nn;
        uint8_t *hdata = reinterpret_cast<uint8_t *>(hdiag + 16);
        if (dbytes) memcpy(hdata, r.data.data(), dbytes);
        r.st = streams_[next_++ % streams_.size()];
        r.ev0 = get_event();
        r.ev1 = get_event();
        char *ws = reinterpret_cast<char *>(r.ws);
        uint8_t *ddata = reinterpret_cast<uint8_t *>(ws + P.o_data);
        double *dpost = reinterpret_cast<double *>(ws + P.o_post);
        double *ddiag = reinterpret_cast<double *>(ws + P.o_diag);
        bool ok = hipEventRecord(r.ev0, r.st) == hipSuccess;
        if (ok && dbytes)
            ok = hipMemcpyAsync(ddata, hdata, dbytes, hipMemcpyHostToDevice, r.st) == hipSuccess;
        if (ok) ok = enqueue_solve(P, &r.p, ddata, ws, r.st, dpost, ddiag, nullptr) == BN_OK;
        if (ok)
            ok = hipMemcpyAsync(hpost, dpost, nn * 8, hipMemcpyDeviceToHost, r.st) == hipSuccess &&
                 hipMemcpyAsync(hdiag, ddiag, 8 * 8, hipMemcpyDeviceToHost, r.st) == hipSuccess;
        if (ok) ok = hipEventRecord(r.ev1, r.st) == hipSuccess;
        if (!ok) {
            (void)hipStreamSynchronize(r.st);
            release(r);
            r.status = BN_EDEVICE;
            return false;
        }
        return true;
    }
    bool done(Req &r) override {
        const hipError_t q = hipEventQuery(r.ev1);
        if (q == hipErrorNotReady) return false;
        if (q != hipSuccess) {
            r.status = BN_EDEVICE;
            return true;
        }
        const size_t nn = (size_t)r.p.n * r.p.n;
        const double *hpost = reinterpret_cast<const double *>(r.hpin);
        const double *hdiag = hpost + nn;
        r.post.assign(hpost, hpost + nn);
        memset(&r.rep, 0, sizeof(r.rep));
        r.rep.log_LV = hdiag[0];
        r.rep.max_invariant_residual = hdiag[1];
        r.rep.saturated = (uint64_t)hdiag[2];
        r.rep.flushed = (uint64_t)hdiag[3];
        r.rep.fallback_tiles = (uint64_t)hdiag[7];
        float ms = 0;
        (void)hipEventElapsedTime(&ms, r.ev0, r.ev1);
        r.rep.ms_total = ms;
        r.status = BN_OK;
        return true;
    }
    void release(Req &r) override {
        if (r.ev0) events_.push_back(r.ev0);
        if (r.ev1) events_.push_back(r.ev1);
        if (r.hpin) host_cache_.emplace(r.hpin_bytes, r.hpin);
        if (r.ws) arena_.put(r.ws, r.ws_bytes);
        r.ev0 = r.ev1 = nullptr;
        r.hpin = r.ws = nullptr;
    }

   private:
    static size_t round_up(size_t x, size_t g) { return (x + g - 1) / g * g; }
    static bool take(std::multimap<size_t, void *> &c, size_t need, void **p, size_t *got) {
        auto it = c.lower_bound(need);
        if (it == c.end() || it->first > need + need / 4) return false;
        *p = it->second;
        *got = it->first;
        c.erase(it);
        return true;
    }
    bool get_host(size_t bytes, void **p, size_t *got) {
        const size_t need = round_up(bytes, (size_t)64 << 10);
        if (take(host_cache_, need, p, got)) return true;
        if (hipHostMalloc(p, need) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        *got = need;
        return true;
    }
    hipEvent_t get_event() {
        if (!events_.empty()) {
            hipEvent_t e = events_.back();
            events_.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }

    int dev_;
    std::vector<hipStream_t> streams_;
    size_t next_ = 0;
    DeviceArena arena_;
    std::multimap<size_t, void *> host_cache_;
    std::vector<hipEvent_t> events_;
};

// ------------------------------------------------------------ CPU executor
// Test executor: holds a request for a time that grows with n 2^n and
// returns placeholder posteriors that depend only on the request.
class FakeExecutor : public Executor {
   public:
    size_t footprint(const Req &r) override {
        return make_plan(r.p.n, r.p.d, r.p.m, r.prec, true, true).total;
    }
    bool start(Req &r) override {
        if (alloc_fails()) {
            r.status = BN_ENOMEM;
            return false;
        }
        r.fake_until = now_ms() + (fixed_ms_ > 0 ? fixed_ms_
                                                 : 0.2 + 1e-6 * (double)r.p.n * (double)(1ull << r.p.n));
        return true;
    }
    bool done(Req &r) override {
        if (now_ms() < r.fake_until) return false;
        const int n = r.p.n;
        r.post.assign((size_t)n * n, 0.0);
        for (int u = 0; u < n; ++u)
            for (int v = 0; v < n; ++v)
                if (u != v) r.post[(size_t)u * n + v] = ((u * 31 + v * 17 + n + r.p.m) % 97) / 97.0;
        memset(&r.rep, 0, sizeof(r.rep));
        r.rep.log_LV = -(double)(n + r.p.m);
        r.status = BN_OK;
        return true;
    }
    void release(Req &) override {}
    double fixed_ms_ = 0;   // BN_SERVE_FAKE_MS: fixed duration of every request
};

// ------------------------------------------------------------------ server
class Server {
   public:
    Server(size_t budget, int max_active, std::unique_ptr<Executor> ex)
        : budget_(budget), max_active_(max_active), ex_(std::move(ex)) {
        worker_ = std::thread([this] { loop(); });
    }
    ~Server() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            for (Req *r : pending_) {
                r->state = Req::DONE;
                r->status = BN_ECANCELED;
            }
            pending_.clear();
        }
        cv_work_.notify_all();
        cv_done_.notify_all();
        worker_.join();                    // finishes the requests already on the device
        std::unique_lock<std::mutex> lk(mu_);
        cv_done_.wait(lk, [this] { return pollers_ == 0; });
        for (auto &kv : all_) delete kv.second;
        all_.clear();
    }

    bn_status submit(const bn_problem *p, bn_precision prec, uint64_t *ticket) {
        if (!ticket) return BN_EINVAL;
        if (prec != BN_FP64_LOG && prec != BN_FP32_SCALED) return BN_EINVAL;
        bn_status s = validate(p, true, true);
        if (s != BN_OK) return s;
        auto r = std::make_unique<Req>();
        r->p = *p;
        r->prec = prec;
        const int n = p->n, d = std::min(p->d, n - 1);
        r->arity.assign(p->arity, p->arity + n);
        if (p->m > 0) r->data.assign(p->data, p->data + (size_t)n * p->m);
        if (p->log_rho) r->log_rho.assign(p->log_rho, p->log_rho + d + 1);
        if (p->log_q) r->log_q.assign(p->log_q, p->log_q + n);
        r->p.data = r->data.empty() ? nullptr : r->data.data();
        r->p.arity = r->arity.data();
        r->p.log_rho = p->log_rho ? r->log_rho.data() : nullptr;
        r->p.log_q = p->log_q ? r->log_q.data() : nullptr;
        r->footprint = ex_->footprint(*r);
        if (r->footprint > budget_) return BN_ENOMEM;   // could never be admitted
        r->t_submit = now_ms();
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stop_) return BN_ECANCELED;
            r->ticket = next_ticket_++;
            *ticket = r->ticket;
            Req *raw = r.release();
            all_[raw->ticket] = raw;
            pending_.push_back(raw);
        }
        cv_work_.notify_all();
        return BN_OK;
    }

    bn_status poll(uint64_t ticket, double *post, bn_report *rep, int32_t timeout_us) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = all_.find(ticket);
        if (it == all_.end()) return BN_EINVAL;
        Req *r = it->second;
        ++pollers_;
        if (r->state != Req::DONE && timeout_us != 0) {
            auto pred = [r] { return r->state == Req::DONE; };
            if (timeout_us < 0)
                cv_done_.wait(lk, pred);
            else
                cv_done_.wait_for(lk, std::chrono::microseconds(timeout_us), pred);
        }
        bn_status s = BN_EAGAIN;
        if (r->state == Req::DONE) {
            s = r->status;
            if (s == BN_OK) {
                if (post) memcpy(post, r->post.data(), r->post.size() * sizeof(double));
                if (rep) {
                    *rep = r->rep;
                    rep->ms_queue = r->t_admit - r->t_submit;
                    rep->ms_latency = r->t_done - r->t_submit;
                }
            }
            all_.erase(ticket);
            delete r;
        }
        --pollers_;
        if (pollers_ == 0) cv_done_.notify_all();
        return s;
    }

   private:
    void finish(Req *r) {   // with mu_ held
        r->state = Req::DONE;
        r->t_done = now_ms();
    }

    void loop() {
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            // admit in arrival order while the head fits (and no admitted
            // request is waiting for device memory to come back)
            while (!stop_ && !mem_wait_ && !pending_.empty() &&
                   (int)running_.size() < max_active_ &&
                   used_ + pending_.front()->footprint <= budget_) {
                Req *r = pending_.front();
                pending_.pop_front();
                used_ += r->footprint;
                r->state = Req::RUNNING;
                r->t_admit = now_ms();
                lk.unlock();
                const bool ok = ex_->start(*r);
                lk.lock();
                used_ -= r->footprint;
                if (ok) {
                    // charge what the request really holds
                    r->charged = ex_->held(*r);
                    used_ += r->charged;
                    running_.push_back(r);
                } else if (r->status == BN_ENOMEM && !running_.empty()) {
                    // the device is short while other solves hold memory:
                    // the request goes back to the head of the queue and
                    // admission waits for the next completion
                    r->state = Req::PENDING;
                    r->status = BN_EAGAIN;
                    pending_.push_front(r);
                    mem_wait_ = true;
                } else {
                    finish(r);
                    cv_done_.notify_all();
                }
            }
            // completions
            bool any = false;
            for (size_t k = 0; k < running_.size();) {
                Req *r = running_[k];
                lk.unlock();
                const bool fin = ex_->done(*r);
                if (fin) ex_->release(*r);
                lk.lock();
                if (fin) {
                    used_ -= r->charged;
                    mem_wait_ = false;
                    finish(r);
                    running_.erase(running_.begin() + k);
                    any = true;
                } else {
                    ++k;
                }
            }
            if (any) cv_done_.notify_all();
            if (stop_ && running_.empty()) break;
            if (running_.empty()) {
                cv_work_.wait(lk, [this] { return stop_ || !pending_.empty(); });
            } else if (!any) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        }
    }

    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<Req *> pending_;
    std::vector<Req *> running_;
    std::unordered_map<uint64_t, Req *> all_;
    size_t budget_, used_ = 0;
    int max_active_;
    uint64_t next_ticket_ = 1;
    bool stop_ = false;
    bool mem_wait_ = false;   // an admitted request found the device short of memory
    int pollers_ = 0;
    std::unique_ptr<Executor> ex_;
    std::thread worker_;
};

}  // namespace bnk

extern "C" {

bn_status bn_server_create(size_t mem_budget_bytes, int32_t max_active, void **server) {
    if (!server || max_active < 1) return BN_EINVAL;
    *server = nullptr;
    std::unique_ptr<bnk::Executor> ex;
    size_t budget = mem_budget_bytes;
    const char *fake = getenv("BN_SERVE_FAKE");
    if (fake && fake[0] == '1') {
        auto *f = new bnk::FakeExecutor();
        if (const char *ms = getenv("BN_SERVE_FAKE_MS")) f->fixed_ms_ = atof(ms);
        ex.reset(f);
        if (!budget) budget = (size_t)1 << 40;
    } else {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return BN_EDEVICE;
        if (!budget) {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return BN_EDEVICE;
            budget = free_b / 10 * 9;
        }
        auto *g = new bnk::GpuExecutor(dev, std::min(max_active, 8), budget);
        if (!g->ok()) {
            delete g;
            return BN_EDEVICE;
        }
        ex.reset(g);
    }
    if (const char *f = getenv("BN_SERVE_FAIL_ALLOC")) ex->fail_at = atoi(f);
    *server = new bnk::Server(budget, max_active, std::move(ex));
    return BN_OK;
}

bn_status bn_serve_submit(void *server, const bn_problem *p, bn_precision prec, uint64_t *ticket) {
    if (!server) return BN_EINVAL;
    return static_cast<bnk::Server *>(server)->submit(p, prec, ticket);
}

bn_status bn_serve_poll(void *server, uint64_t ticket, double *post, bn_report *rep,
                        int32_t timeout_us) {
    if (!server) return BN_EINVAL;
    return static_cast<bnk::Server *>(server)->poll(ticket, post, rep, timeout_us);
}

bn_status bn_server_destroy(void *server) {
    if (!server) return BN_EINVAL;
    delete static_cast<bnk::Server *>(server);
    return BN_OK;
}

}  // extern "C"
