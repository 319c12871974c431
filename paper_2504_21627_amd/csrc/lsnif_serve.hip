// Serving loop: continuous batching of queries that arrive over time.
//
// One host thread per context owns the device side.  Each turn it
//  - drops waiting requests whose admission timeout has passed,
//  - admits waiting requests in arrival order while a slot is free and their
//    query workspace fits in the budget arena (first fit, 256-byte granules),
//    enqueueing each on the next of several HIP streams, so the kernels of
//    different requests overlap on the device,
//  - retires requests whose completion event has fired: the slot and the
//    workspace return to the pool, which may admit the next request.
// The first waiting request blocks the ones behind it (no overtaking), so a
// large request is not starved by a stream of small ones.
//
// Small requests that wait together are merged: the request at the head of
// the queue and the ones right behind it that query the same target (the same
// object, or pairs over the same instance array), each of at most merge_rays
// rays, up to merge_max of them and 2^23 rays in all, are admitted as one
// launch: their rays and pairs are staged into one batch (k_serve.hip), one
// query answers it, and each request's answers are copied back to its own
// output.  Every member completes when the launch does.  A ray's answer does
// not depend on its batch, so merged and direct answers are the same bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lsnif_internal.hpp"

namespace lsnif {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) in 256-byte granules.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        size_ = size;
        if (size) free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = (bytes + 255) / 256 * 256;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) / 256 * 256;
        if (bytes == 0) bytes = 256;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t peak() const { return peak_; }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

struct Req {
    lsnif_request r{};
    int32_t state = LSNIF_REQ_QUEUED;   // or a negative final status
    size_t need = 0, off = 0;
    Clock::time_point t_submit, t_admit, t_done;
    hipEvent_t done_ev = nullptr;
    int stream = 0;
    std::vector<uint64_t> members;      // a merged launch's first request: the others it answers
    uint64_t launch_rays = 0;           // rays of the whole launch (dry runs: its duration)
};

constexpr uint32_t kMergeRays = 1u << 18;     // default largest request that may be merged
constexpr uint64_t kMergeTotal = 1ull << 23;  // rays of one merged launch at most

inline size_t al256s(size_t x) { return (x + 255) / 256 * 256; }

// Staging of a merged launch: rays, pair ray and instance indices, answers.
inline size_t merge_stage_bytes(uint64_t rays, uint64_t pairs)
{
    return al256s(rays * sizeof(lsnif_ray)) + 2 * al256s(pairs * 4) + al256s(rays * sizeof(lsnif_hit));
}

class Server {
public:
    Server(lsnif_ctx *ctx, const lsnif_serve_cfg &cfg) : ctx_(ctx), cfg_(cfg) {}

    lsnif_status start()
    {
        if (!cfg_.max_inflight) cfg_.max_inflight = 8;
        if (!cfg_.hbm_budget) cfg_.hbm_budget = 4ull << 30;
        if (!cfg_.n_streams) cfg_.n_streams = 4;
        if (!cfg_.max_queue) cfg_.max_queue = 65536;
        if (!cfg_.merge_rays) cfg_.merge_rays = kMergeRays;
        if (!cfg_.merge_max || cfg_.merge_max > kMergeMax) cfg_.merge_max = kMergeMax;
        dry_ = cfg_.dry_run_ns_per_ray > 0;
        if (!dry_) {
            if (ctx_->device < 0) return fail(LSNIF_E_INVALID, "a host-only context serves dry runs only");
            DeviceGuard g(ctx_->device);
            streams_.resize(cfg_.n_streams, nullptr);
            for (auto &s : streams_)
                if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
                    return fail(LSNIF_E_DEVICE, "hipStreamCreate failed");
            if (hipMalloc(&base_, cfg_.hbm_budget) != hipSuccess)
                return fail(LSNIF_E_NOMEM, "serving workspace of %llu bytes", (unsigned long long)cfg_.hbm_budget);
        }
        arena_.reset(cfg_.hbm_budget);
        t0_ = Clock::now();
        worker_ = std::thread([this] { loop(); });
        return LSNIF_OK;
    }

    lsnif_status submit(const lsnif_request &r, uint64_t &ticket)
    {
        size_t need = 0;
        lsnif_status st = sizing(r, need);
        std::unique_lock<std::mutex> lk(mu_);
        ++submitted_;
        if (st) {
            ++rejected_;
            return st;
        }
        if (need > arena_.size()) {
            ++rejected_;
            return fail(LSNIF_E_NOMEM, "request needs %llu bytes of workspace, the budget is %llu",
                        (unsigned long long)need, (unsigned long long)arena_.size());
        }
        if (queue_.size() >= cfg_.max_queue) {
            ++rejected_;
            return fail(LSNIF_E_BUSY, "serving queue is full (%u)", cfg_.max_queue);
        }
        if (stopping_) return fail(LSNIF_E_CANCELLED, "serving is stopping");
        ticket = next_ticket_++;
        Req &q = reqs_[ticket];
        q.r = r;
        q.need = need;
        q.t_submit = Clock::now();
        queue_.push_back(ticket);
        cv_work_.notify_one();
        return LSNIF_OK;
    }

    lsnif_status poll(uint64_t ticket, int32_t &state)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return fail(LSNIF_E_NOTFOUND, "no request %llu", (unsigned long long)ticket);
        state = it->second.state;
        return LSNIF_OK;
    }

    lsnif_status wait(uint64_t ticket, int64_t timeout_ns)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return fail(LSNIF_E_NOTFOUND, "no request %llu", (unsigned long long)ticket);
        const Req &q = it->second;   // element references survive rehashing, iterators do not
        auto finished = [&] { return q.state == LSNIF_REQ_DONE || q.state < 0; };
        if (timeout_ns < 0) cv_done_.wait(lk, finished);
        else if (!cv_done_.wait_for(lk, std::chrono::nanoseconds(timeout_ns), finished))
            return fail(LSNIF_E_TIMEOUT, "request %llu not finished", (unsigned long long)ticket);
        return q.state == LSNIF_REQ_DONE ? LSNIF_OK : q.state;
    }

    lsnif_status cancel(uint64_t ticket)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return fail(LSNIF_E_NOTFOUND, "no request %llu", (unsigned long long)ticket);
        if (it->second.state != LSNIF_REQ_QUEUED) return fail(LSNIF_E_BUSY, "request already admitted");
        queue_.erase(std::remove(queue_.begin(), queue_.end(), ticket), queue_.end());
        it->second.state = LSNIF_E_CANCELLED;
        ++cancelled_;
        cv_done_.notify_all();
        cv_work_.notify_one();
        return LSNIF_OK;
    }

    void stats(lsnif_serve_stats &s)
    {
        std::unique_lock<std::mutex> lk(mu_);
        s = lsnif_serve_stats{};
        s.submitted = submitted_;
        s.admitted = admitted_;
        s.completed = completed_;
        s.rejected = rejected_;
        s.cancelled = cancelled_;
        s.timed_out = timed_out_;
        s.failed = failed_;
        s.queued = queue_.size();
        s.inflight = inflight_.size();
        s.rays_completed = rays_done_;
        s.ws_bytes_peak = arena_.peak();
        if (!lat_ms_.empty()) {
            std::vector<double> v = lat_ms_;
            std::sort(v.begin(), v.end());
            auto pct = [&](double p) {
                const double x = p * (double)(v.size() - 1);
                const size_t i = (size_t)x;
                const double f = x - (double)i;
                return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
            };
            s.p50_ms = pct(0.50);
            s.p99_ms = pct(0.99);
            double sum = 0.0;
            for (double x : v) sum += x;
            s.mean_ms = sum / (double)v.size();
            s.max_ms = v.back();
        }
        s.elapsed_s = std::chrono::duration<double>(Clock::now() - t0_).count();
        s.launches = launches_;
    }

    // Finish admitted work, cancel waiting requests, join the thread, free resources.
    void stop()
    {
        {
            std::unique_lock<std::mutex> lk(mu_);
            stopping_ = true;
            for (uint64_t t : queue_) {
                reqs_[t].state = LSNIF_E_CANCELLED;
                ++cancelled_;
            }
            queue_.clear();
            cv_work_.notify_one();
            cv_done_.notify_all();
        }
        if (worker_.joinable()) worker_.join();
        if (!dry_) {
            DeviceGuard g(ctx_->device);
            for (auto &kv : reqs_)
                if (kv.second.done_ev) (void)hipEventDestroy(kv.second.done_ev);
            for (hipEvent_t e : spare_ev_) (void)hipEventDestroy(e);
            for (auto s : streams_)
                if (s) (void)hipStreamDestroy(s);
            (void)hipFree(base_);
        }
    }

private:
    // Workspace bytes of a request, or an error for a request that can never run.
    lsnif_status sizing(const lsnif_request &r, size_t &need)
    {
        if (r.n_rays == 0) {
            need = 0;
            return LSNIF_OK;
        }
        if (!r.d_rays || !r.d_out) return fail(LSNIF_E_INVALID, "rays or output is NULL");
        if (r.kind != LSNIF_REQ_SINGLE && r.kind != LSNIF_REQ_PAIRS)
            return fail(LSNIF_E_INVALID, "unknown request kind %d", r.kind);
        if (r.kind == LSNIF_REQ_PAIRS) {
            if (r.n_pairs && (!r.d_pair_ray || !r.d_pair_inst || !r.d_inst))
                return fail(LSNIF_E_INVALID, "pair buffers are NULL");
            if (dry_) {
                need = pairs_ws_bytes(r.n_rays, r.n_pairs, r.n_inst + 1, kMaxList, 4);   // the default grouping
                return LSNIF_OK;
            }
            std::lock_guard<std::recursive_mutex> g(ctx_->mu);
            PairsSetup ps;
            lsnif_status st = pairs_setup(ctx_, ps);
            if (st) return st;
            need = pairs_ws_bytes(r.n_rays, r.n_pairs, ps.n_objs, ps.maxH >> 1, ps.pair_bits);
            return LSNIF_OK;
        }
        uint32_t bits = 5, cap = kMaxList;   // dry runs: the default resolution, the longest lists
        if (!dry_) {
            std::lock_guard<std::recursive_mutex> g(ctx_->mu);
            auto it = ctx_->objects.find(r.object_id);
            if (it == ctx_->objects.end()) return fail(LSNIF_E_NOTFOUND, "no object %u", r.object_id);
            bits = it->second.geom.sort_bits;
            cap = (uint32_t)it->second.geom.H >> 1;
        }
        need = query_ws_bytes(r.n_rays, bits, cap);
        return LSNIF_OK;
    }

    // A request that may share a launch with its neighbours in the queue.
    bool mergeable(const lsnif_request &r) const
    {
        return r.n_rays > 0 && r.n_rays <= cfg_.merge_rays &&
               (r.kind == LSNIF_REQ_SINGLE || (r.kind == LSNIF_REQ_PAIRS && r.n_pairs > 0));
    }
    static bool same_target(const lsnif_request &a, const lsnif_request &b)
    {
        if (a.kind != b.kind) return false;
        if (a.kind == LSNIF_REQ_SINGLE) return a.object_id == b.object_id;
        return a.d_inst == b.d_inst && a.n_inst == b.n_inst;
    }

    // Workspace of a merged launch of `rays` rays and `pairs` pairs like `r` (ctx->mu held).
    lsnif_status group_sizing(const lsnif_request &r, uint64_t rays, uint64_t pairs, size_t &need)
    {
        if (rays > 0xffffffffull || pairs > 0xffffffffull) return fail(LSNIF_E_INVALID, "merged launch too large");
        if (dry_) {   // the default resolution and grouping, the longest lists
            need = merge_stage_bytes(rays, pairs) +
                   (r.kind == LSNIF_REQ_PAIRS ? pairs_ws_bytes((uint32_t)rays, (uint32_t)pairs, r.n_inst + 1, kMaxList, 4)
                                              : query_ws_bytes((uint32_t)rays, 5, kMaxList));
            return LSNIF_OK;
        }
        if (r.kind == LSNIF_REQ_PAIRS) {
            PairsSetup ps;
            const lsnif_status st = pairs_setup(ctx_, ps);
            if (st) return st;
            need = merge_stage_bytes(rays, pairs) +
                   pairs_ws_bytes((uint32_t)rays, (uint32_t)pairs, ps.n_objs, ps.maxH >> 1, ps.pair_bits);
            return LSNIF_OK;
        }
        auto it = ctx_->objects.find(r.object_id);
        if (it == ctx_->objects.end()) return fail(LSNIF_E_NOTFOUND, "no object %u", r.object_id);
        need = merge_stage_bytes(rays, 0) +
               query_ws_bytes((uint32_t)rays, it->second.geom.sort_bits, (uint32_t)it->second.geom.H >> 1);
        return LSNIF_OK;
    }

    // Enqueue a merged launch: the leader q and its members, `rays` and `pairs` in all
    // (mu_ and ctx->mu held).
    lsnif_status launch_group(Req &q, uint64_t rays, uint64_t pairs)
    {
        if (dry_) return LSNIF_OK;
        hipStream_t s = streams_[q.stream];
        char *w = static_cast<char *>(base_) + q.off;
        MergeArgs M{};
        M.rays = reinterpret_cast<float4 *>(w);
        w += al256s(rays * sizeof(lsnif_ray));
        M.pair_ray = reinterpret_cast<uint32_t *>(w);
        w += al256s(pairs * 4);
        M.pair_inst = reinterpret_cast<uint32_t *>(w);
        w += al256s(pairs * 4);
        M.out = reinterpret_cast<lsnif_hit *>(w);
        w += al256s(rays * sizeof(lsnif_hit));
        M.n_rays = (uint32_t)rays;
        M.n_pairs = (uint32_t)pairs;
        uint32_t r0 = 0, p0 = 0;
        auto add = [&](const lsnif_request &r) {
            MergeMember &m = M.m[M.n_members++];
            m.rays = reinterpret_cast<const float4 *>(r.d_rays);
            m.out = r.d_out;
            m.pair_ray = r.d_pair_ray;
            m.pair_inst = r.d_pair_inst;
            m.ray0 = r0;
            m.pair0 = p0;
            m.n_rays = r.n_rays;
            m.n_pairs = r.kind == LSNIF_REQ_PAIRS ? r.n_pairs : 0;
            r0 += m.n_rays;
            p0 += m.n_pairs;
        };
        add(q.r);
        for (uint64_t t : q.members) add(reqs_[t].r);
        for (uint32_t k = 0; k < M.n_members; ++k)
            if (reinterpret_cast<uintptr_t>(M.m[k].rays) % 16 || reinterpret_cast<uintptr_t>(M.m[k].out) % 4)
                return fail(LSNIF_E_INVALID, "rays must be 16-byte and hits 4-byte aligned");
        if (launch_merge_pack(M, s) != hipSuccess) return fail(LSNIF_E_DEVICE, "merge pack launch failed");
        lsnif_status st;
        const lsnif_ray *srays = reinterpret_cast<const lsnif_ray *>(M.rays);
        if (q.r.kind == LSNIF_REQ_PAIRS) {
            PairsSetup ps;
            st = pairs_setup(ctx_, ps);
            if (!st)
                st = enqueue_pairs(ctx_, ps, srays, M.n_rays, M.pair_ray, M.pair_inst, M.n_pairs, q.r.d_inst,
                                   q.r.n_inst, M.out, s, w, 1);
        } else {
            auto it = ctx_->objects.find(q.r.object_id);
            st = it == ctx_->objects.end() ? fail(LSNIF_E_NOTFOUND, "no object %u", q.r.object_id)
                                           : enqueue_query(ctx_, it->second, srays, M.n_rays, M.out, nullptr, s, w, 1);
        }
        if (st) return st;
        if (launch_merge_unpack(M, s) != hipSuccess) return fail(LSNIF_E_DEVICE, "merge unpack launch failed");
        q.done_ev = take_event();
        if (!q.done_ev) return fail(LSNIF_E_DEVICE, "hipEventCreate failed");
        if (hipEventRecord(q.done_ev, s) != hipSuccess) return fail(LSNIF_E_DEVICE, "hipEventRecord failed");
        return LSNIF_OK;
    }

    hipEvent_t take_event()
    {
        if (!spare_ev_.empty()) {
            hipEvent_t e = spare_ev_.back();
            spare_ev_.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    // Enqueue an admitted request on its stream (mu_ held).
    lsnif_status launch(Req &q)
    {
        if (dry_ || q.r.n_rays == 0) return LSNIF_OK;
        hipStream_t s = streams_[q.stream];
        void *ws = static_cast<char *>(base_) + q.off;
        lsnif_status st;
        {
            std::lock_guard<std::recursive_mutex> g(ctx_->mu);
            if (q.r.kind == LSNIF_REQ_PAIRS) {
                PairsSetup ps;
                st = pairs_setup(ctx_, ps);
                if (!st)
                    st = enqueue_pairs(ctx_, ps, q.r.d_rays, q.r.n_rays, q.r.d_pair_ray, q.r.d_pair_inst, q.r.n_pairs,
                                       q.r.d_inst, q.r.n_inst, q.r.d_out, s, ws, 1);   // streams overlap requests
            } else {
                auto it = ctx_->objects.find(q.r.object_id);
                st = it == ctx_->objects.end()
                         ? fail(LSNIF_E_NOTFOUND, "no object %u", q.r.object_id)
                         : enqueue_query(ctx_, it->second, q.r.d_rays, q.r.n_rays, q.r.d_out, nullptr, s, ws, 1);
            }
        }
        if (st) return st;
        q.done_ev = take_event();
        if (!q.done_ev) return fail(LSNIF_E_DEVICE, "hipEventCreate failed");
        if (hipEventRecord(q.done_ev, s) != hipSuccess) return fail(LSNIF_E_DEVICE, "hipEventRecord failed");
        return LSNIF_OK;
    }

    void finish(uint64_t ticket, Req &q, int32_t state)
    {
        q.state = state;
        q.t_done = Clock::now();
        arena_.release(q.off, q.need);
        if (q.done_ev) {
            spare_ev_.push_back(q.done_ev);
            q.done_ev = nullptr;
        }
        auto account = [&](Req &x) {
            if (state == LSNIF_REQ_DONE) {
                ++completed_;
                rays_done_ += x.r.n_rays;
                lat_ms_.push_back(std::chrono::duration<double, std::milli>(x.t_done - x.t_submit).count());
            } else {
                ++failed_;
            }
        };
        account(q);
        for (uint64_t m : q.members) {   // the requests a merged launch answered end with it
            Req &x = reqs_[m];
            x.state = state;
            x.t_done = q.t_done;
            account(x);
        }
        q.members.clear();
        inflight_.erase(std::remove(inflight_.begin(), inflight_.end(), ticket), inflight_.end());
    }

    void loop()
    {
        if (!dry_) (void)hipSetDevice(ctx_->device);
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            bool changed = false;
            const auto now = Clock::now();
            // admission timeouts
            for (auto it = queue_.begin(); it != queue_.end();) {
                Req &q = reqs_[*it];
                if (q.r.timeout_ns > 0 && now - q.t_submit > std::chrono::nanoseconds(q.r.timeout_ns)) {
                    q.state = LSNIF_E_TIMEOUT;
                    ++timed_out_;
                    it = queue_.erase(it);
                    changed = true;
                } else {
                    ++it;
                }
            }
            // admission, in arrival order.  The workspace is sized again here, under the
            // context's lock held until the request is enqueued: a build, release or tuning
            // change since submit may have changed the layout the query will use.
            while (!queue_.empty() && inflight_.size() < cfg_.max_inflight) {
                const uint64_t t = queue_.front();
                Req &q = reqs_[t];
                std::unique_lock<std::recursive_mutex> cg(ctx_->mu, std::defer_lock);
                if (!dry_) cg.lock();
                // the requests right behind it that can share its launch
                std::vector<uint64_t> grp{t};
                uint64_t g_rays = q.r.n_rays, g_pairs = q.r.n_pairs;
                if (mergeable(q.r)) {
                    for (size_t i = 1; i < queue_.size() && grp.size() < cfg_.merge_max; ++i) {
                        const Req &o = reqs_[queue_[i]];
                        if (!mergeable(o.r) || !same_target(q.r, o.r) || g_rays + o.r.n_rays > kMergeTotal) break;
                        g_rays += o.r.n_rays;
                        g_pairs += o.r.n_pairs;
                        grp.push_back(queue_[i]);
                    }
                }
                size_t need = 0;
                lsnif_status zst = LSNIF_OK;
                if (grp.size() > 1) {
                    zst = group_sizing(q.r, g_rays, g_pairs, need);
                    if (zst || need > arena_.size()) {   // alone, then
                        grp.resize(1);
                        g_rays = q.r.n_rays;
                        g_pairs = q.r.n_pairs;
                        zst = LSNIF_OK;
                    }
                }
                if (grp.size() == 1) {
                    zst = sizing(q.r, need);
                    if (!zst && need > arena_.size())
                        zst = fail(LSNIF_E_NOMEM, "request needs %llu bytes of workspace, the budget is %llu",
                                   (unsigned long long)need, (unsigned long long)arena_.size());
                }
                if (zst) {   // it can no longer run: it ends without holding a slot
                    queue_.pop_front();
                    q.state = zst;
                    q.t_done = Clock::now();
                    ++failed_;
                    changed = true;
                    continue;
                }
                if (!arena_.alloc(need, q.off)) break;
                q.need = need;
                const auto now_admit = Clock::now();
                q.members.assign(grp.begin() + 1, grp.end());
                q.launch_rays = g_rays;
                for (uint64_t m : grp) {
                    Req &x = reqs_[m];
                    x.t_admit = now_admit;
                    x.state = LSNIF_REQ_RUNNING;
                    ++admitted_;
                }
                queue_.erase(queue_.begin(), queue_.begin() + (std::ptrdiff_t)grp.size());
                q.stream = (int)(next_stream_++ % std::max<uint32_t>(1, cfg_.n_streams));
                inflight_.push_back(t);
                ++launches_;
                const lsnif_status st = q.members.empty() ? launch(q) : launch_group(q, g_rays, g_pairs);
                if (st) finish(t, q, st);
                changed = true;
            }
            // completions
            for (size_t i = 0; i < inflight_.size();) {
                const uint64_t t = inflight_[i];
                Req &q = reqs_[t];
                bool done = false;
                int32_t state = LSNIF_REQ_DONE;
                if (dry_ || q.r.n_rays == 0 || !q.done_ev) {
                    const auto due = q.t_admit + std::chrono::nanoseconds(cfg_.dry_run_ns_per_ray * q.launch_rays);
                    done = dry_ ? now >= due : true;
                } else {
                    const hipError_t e = hipEventQuery(q.done_ev);
                    if (e == hipSuccess) done = true;
                    else if (e != hipErrorNotReady) {
                        done = true;
                        state = LSNIF_E_DEVICE;
                    }
                }
                if (done) {
                    finish(t, q, state);
                    changed = true;
                } else {
                    ++i;
                }
            }
            if (changed) cv_done_.notify_all();
            if (stopping_ && queue_.empty() && inflight_.empty()) break;
            if (!changed) {
                // nothing moved: sleep briefly (requests in flight) or until new work arrives
                const auto nap = inflight_.empty() && queue_.empty() ? std::chrono::microseconds(2000)
                                                                      : std::chrono::microseconds(20);
                cv_work_.wait_for(lk, nap);
            }
        }
    }

    lsnif_ctx *ctx_;
    lsnif_serve_cfg cfg_;
    bool dry_ = false;
    std::vector<hipStream_t> streams_;
    void *base_ = nullptr;
    Arena arena_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::thread worker_;
    bool stopping_ = false;
    std::deque<uint64_t> queue_;
    std::vector<uint64_t> inflight_;
    std::unordered_map<uint64_t, Req> reqs_;
    std::vector<hipEvent_t> spare_ev_;
    std::vector<double> lat_ms_;
    uint64_t next_ticket_ = 1, next_stream_ = 0;
    uint64_t submitted_ = 0, admitted_ = 0, completed_ = 0, rejected_ = 0, cancelled_ = 0, timed_out_ = 0,
             failed_ = 0, rays_done_ = 0, launches_ = 0;
    Clock::time_point t0_;
};

void destroy_server(lsnif_ctx *ctx)
{
    if (ctx && ctx->server) {
        ctx->server->stop();
        delete ctx->server;
        ctx->server = nullptr;
    }
}

}  // namespace lsnif

using namespace lsnif;

extern "C" {

lsnif_status lsnif_serve_start(lsnif_ctx *ctx, const lsnif_serve_cfg *cfg)
{
    if (!ctx || !cfg) return fail(LSNIF_E_INVALID, "ctx or cfg is NULL");
    if (ctx->server) return fail(LSNIF_E_BUSY, "serving already started");
    Server *s = new (std::nothrow) Server(ctx, *cfg);
    if (!s) return fail(LSNIF_E_NOMEM, "host allocation failed");
    const lsnif_status st = s->start();
    if (st) {
        s->stop();
        delete s;
        return st;
    }
    ctx->server = s;
    return LSNIF_OK;
}

lsnif_status lsnif_serve_submit(lsnif_ctx *ctx, const lsnif_request *req, uint64_t *ticket)
{
    if (!ctx || !req || !ticket) return fail(LSNIF_E_INVALID, "NULL argument");
    if (!ctx->server) return fail(LSNIF_E_INVALID, "serving not started");
    return ctx->server->submit(*req, *ticket);
}

lsnif_status lsnif_serve_poll(lsnif_ctx *ctx, uint64_t ticket, int32_t *state)
{
    if (!ctx || !state) return fail(LSNIF_E_INVALID, "NULL argument");
    if (!ctx->server) return fail(LSNIF_E_INVALID, "serving not started");
    return ctx->server->poll(ticket, *state);
}

lsnif_status lsnif_serve_wait(lsnif_ctx *ctx, uint64_t ticket, int64_t timeout_ns)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    if (!ctx->server) return fail(LSNIF_E_INVALID, "serving not started");
    return ctx->server->wait(ticket, timeout_ns);
}

lsnif_status lsnif_serve_cancel(lsnif_ctx *ctx, uint64_t ticket)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    if (!ctx->server) return fail(LSNIF_E_INVALID, "serving not started");
    return ctx->server->cancel(ticket);
}

lsnif_status lsnif_serve_stats_get(lsnif_ctx *ctx, lsnif_serve_stats *stats)
{
    if (!ctx || !stats) return fail(LSNIF_E_INVALID, "NULL argument");
    if (!ctx->server) return fail(LSNIF_E_INVALID, "serving not started");
    ctx->server->stats(*stats);
    return LSNIF_OK;
}

lsnif_status lsnif_serve_stop(lsnif_ctx *ctx)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    if (!ctx->server) return fail(LSNIF_E_INVALID, "serving not started");
    destroy_server(ctx);
    return LSNIF_OK;
}

}  // extern "C"
