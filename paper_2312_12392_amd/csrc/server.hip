// Continuous-batching render server.
//
// Requests (a camera, image size, pass count and displacement, any mode)
// enter a FIFO queue.  A scheduler thread admits them in order while their output
// images fit in a device pool of fixed size (the HBM budget), packs every
// admitted request of the oldest one's size class that is not yet running
// into one batched launch (rcp_render_batch's kernel: each pixel's pass
// chain is independent, so requests of any size and pass count can share a
// launch), and keeps up to
// `max_inflight` launches running at once on separate streams.  Requests
// that arrive while others are on the GPU join the next launch as soon as
// pool space and a launch slot free up, and that launch overlaps the running
// ones.  Finished requests keep their images in the pool until released.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <sys/prctl.h>

#include "rcp_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

// Most requests in one batched launch (the batch entry point's limit).
constexpr int kMaxBatch = 1024;

struct Req {
    rcp_request r;
    size_t bytes = 0;
    size_t offset = 0;            // in the pool, once admitted
    bool in_pool = false;
    int state = RCP_REQ_QUEUED;
    double t_submit = 0, t_start = 0, t_done = 0;
};

// Size classes of requests: more than 2^24 pixel-passes (1080p with 8
// passes is below) is big.
constexpr uint64_t kBigPixelPasses = uint64_t(1) << 24;

inline bool is_big(const Req& r) { return (uint64_t)r.r.W * (uint64_t)r.r.H * (uint64_t)r.r.K > kBigPixelPasses; }

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    rcp::BatchWorkspace ws;
    std::vector<uint64_t> tickets;
    std::vector<rcp_view> views;   // the launch's views (capacity kMaxBatch, reserved at creation)
    bool busy = false;
    bool launching = false;     // its launch is being enqueued (lock released)
};

}  // namespace

struct rcp_server {
    rcp_scene* scene = nullptr;
    int device = 0;
    char* pool = nullptr;
    size_t pool_bytes = 0;
    std::map<size_t, size_t> free_list;          // offset -> size
    int max_inflight = 2;
    int queue_capacity = 1024;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> queue;                  // submitted, not yet admitted
    std::vector<uint64_t> admitted;              // admitted, not yet launched
    std::vector<Slot> slots;
    Clock::time_point t0;
    uint64_t launches = 0;
    uint64_t generation = 0;                     // bumped by submit, release and stop

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    bool pool_alloc(size_t bytes, size_t& off) {
        for (auto it = free_list.begin(); it != free_list.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                // the block's own map node carries the remainder (no allocation)
                auto node = free_list.extract(it);
                if (rest) {
                    node.key() = off + bytes;
                    node.mapped() = rest;
                    free_list.insert(std::move(node));
                }
                return true;
            }
        }
        return false;
    }

    void pool_free(size_t off, size_t bytes) {
        auto it = free_list.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_list.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_list.erase(next);
        }
        if (it != free_list.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_list.erase(it);
            }
        }
    }
};

namespace rcp {

size_t request_bytes(const rcp_request& r) {
    const size_t n = (size_t)r.W * (size_t)r.H * (size_t)r.K;
    const size_t img = (12 * n + 255) & ~(size_t)255;
    const size_t ids = r.with_ids ? (4 * n + 255) & ~(size_t)255 : 0;
    return img + ids;
}

namespace {

// One scheduling round, entered with the lock held: retire finished
// launches, admit queued requests in order while they fit, launch the
// admitted ones.  The launch itself is enqueued with the lock released (the
// slot is marked busy first, and only this thread schedules), so submit and
// poll never wait for it.  It allocates nothing, on the device or the host:
// every slot's device buffers were sized when the server was created, and its
// host arrays hold a full batch (admission stops at one batch of requests
// waiting for a slot).
void schedule(rcp_server* s, std::unique_lock<std::mutex>& lk) {
    for (Slot& sl : s->slots) {
        if (!sl.busy || sl.launching) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        const double t = s->now();
        // a ray that ran out of its step budget (a malformed tree) fails the
        // requests of the launch that reported it
        const bool ok = q == hipSuccess && take_device_error(s->scene) == RCP_OK;
        for (uint64_t id : sl.tickets) {
            Req& r = s->reqs[id];
            r.state = ok ? RCP_REQ_DONE : RCP_REQ_FAILED;
            r.t_done = t;
        }
        if (q != hipSuccess) (void)hipGetLastError();
        sl.tickets.clear();
        sl.busy = false;
    }
    while (!s->queue.empty() && s->admitted.size() < (size_t)kMaxBatch) {
        Req& r = s->reqs[s->queue.front()];
        size_t off = 0;
        if (!s->pool_alloc(r.bytes, off)) break;       // first in, first served: wait for space
        r.offset = off;
        r.in_pool = true;
        s->admitted.push_back(s->queue.front());
        s->queue.pop_front();
    }
    if (s->admitted.empty()) return;
    Slot* free_slot = nullptr;
    for (Slot& sl : s->slots)
        if (!sl.busy) { free_slot = &sl; break; }
    if (!free_slot) return;
    // The launch takes the admitted requests of the oldest one's size class,
    // in admission order: a small request does not wait for a 4K one in the
    // same launch, and the oldest request still goes first.
    const bool big = is_big(s->reqs[s->admitted.front()]);
    size_t n = 0;
    for (size_t i = 0; i < s->admitted.size() && n < (size_t)kMaxBatch; ++i)
        if (is_big(s->reqs[s->admitted[i]]) == big) std::swap(s->admitted[n++], s->admitted[i]);
    std::sort(s->admitted.begin() + (long)n, s->admitted.end());   // the rest in admission (ticket) order
    std::vector<rcp_view>& views = free_slot->views;
    views.resize(n);
    for (size_t i = 0; i < n; ++i) {
        Req& r = s->reqs[s->admitted[i]];
        rcp_view& v = views[i];
        v.camera = r.r.camera;
        v.W = r.r.W; v.H = r.r.H; v.K = r.r.K;
        v.disp = r.r.disp;
        v.out_images = (float*)(s->pool + r.offset);
        v.out_ids = r.r.with_ids
                        ? (int32_t*)(s->pool + r.offset + ((12 * (size_t)r.r.W * r.r.H * r.r.K + 255) & ~(size_t)255))
                        : nullptr;
    }
    free_slot->tickets.assign(s->admitted.begin(), s->admitted.begin() + (long)n);
    s->admitted.erase(s->admitted.begin(), s->admitted.begin() + (long)n);
    free_slot->busy = true;
    free_slot->launching = true;
    const double t_launch = s->now();
    for (uint64_t id : free_slot->tickets) {
        Req& r = s->reqs[id];
        r.state = RCP_REQ_RUNNING;
        r.t_start = t_launch;
    }
    lk.unlock();
    rcp_status st = render_batch(s->scene, views.data(), (int)n, free_slot->ws, free_slot->stream);
    const bool recorded = st == RCP_OK && hipEventRecord(free_slot->done, free_slot->stream) == hipSuccess;
    lk.lock();
    free_slot->launching = false;
    const double t = s->now();
    if (!recorded) {
        // nothing of a failed launch can still be running on the slot's
        // stream once it is synchronised
        (void)hipStreamSynchronize(free_slot->stream);
        (void)hipGetLastError();
        for (uint64_t id : free_slot->tickets) {
            Req& r = s->reqs[id];
            r.state = RCP_REQ_FAILED;
            r.t_done = t;
        }
        free_slot->tickets.clear();
        free_slot->busy = false;
        return;
    }
    ++s->launches;
}

// Launches in flight are looked at again after this many microseconds (their
// completion events cannot wake the scheduler).
constexpr int kPollMicros = 10;

void run(rcp_server* s) {
    (void)hipSetDevice(s->device);
    // Linux lengthens each timed sleep of an ordinary thread by its timer
    // slack, 50 us by default: five times the poll interval.  A request's
    // completion is noticed up to one sleep late, so the slack went straight
    // into the served latency.
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);   // 1 us
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        schedule(s, lk);
        bool running = false;
        for (const Slot& sl : s->slots) running = running || sl.busy;
        if (s->stop && !running && (s->queue.empty() && s->admitted.empty())) break;
        if (s->stop && !running) {
            // requests left in the queue when stopping can never start
            for (uint64_t id : s->queue) s->reqs[id].state = RCP_REQ_FAILED;
            s->queue.clear();
            break;
        }
        if (running) {
            // launches in flight: look again shortly (events cannot notify)
            s->cv.wait_for(lk, std::chrono::microseconds(kPollMicros));
        } else {
            // nothing on the GPU: sleep until a submit, release or stop
            const uint64_t seen = s->generation;
            s->cv.wait(lk, [&] { return s->stop || s->generation != seen; });
        }
    }
}

}  // namespace

rcp_status server_create(rcp_scene* scene, size_t pool_bytes, int max_inflight, int queue_capacity,
                         rcp_server** out) {
    rcp_server* s = new rcp_server();
    s->scene = scene;
    s->device = scene->device;
    s->max_inflight = max_inflight;
    s->queue_capacity = queue_capacity;
    s->t0 = Clock::now();
    s->pool_bytes = pool_bytes;
    rcp_status st = dev_alloc((void**)&s->pool, pool_bytes);
    if (st != RCP_OK) {
        delete s;
        return st;
    }
    s->free_list[0] = pool_bytes;
    s->admitted.reserve((size_t)kMaxBatch);
    s->slots.resize((size_t)max_inflight);
    for (Slot& sl : s->slots) {
        sl.tickets.reserve((size_t)kMaxBatch);
        sl.views.reserve((size_t)kMaxBatch);
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            server_destroy(s);
            return hip_status(e, "server stream", __FILE__, __LINE__);
        }
        // every buffer a launch of this slot uses, sized for the largest batch
        st = prepare_batch_workspace(scene, sl.ws, kMaxBatch, true, sl.stream);
        if (st == RCP_OK && hipStreamSynchronize(sl.stream) != hipSuccess) st = RCP_ERR_DEVICE;
        if (st != RCP_OK) {
            const std::string msg = rcp_last_error();
            server_destroy(s);
            set_error("%s", msg.c_str());
            return st;
        }
    }
    s->worker = std::thread(run, s);
    *out = s;
    return RCP_OK;
}

void server_destroy(rcp_server* s) {
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
            ++s->generation;
        }
        s->cv.notify_all();
        s->worker.join();
    }
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        free_batch_workspace(sl.ws, sl.stream);
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->pool) (void)hipFree(s->pool);
    delete s;
}

rcp_status server_submit(rcp_server* s, const rcp_request& r, uint64_t& ticket) {
    const size_t bytes = request_bytes(r);
    if (bytes > s->pool_bytes) {
        set_error("request needs %zu bytes of output, more than the whole pool (%zu)", bytes, s->pool_bytes);
        return RCP_ERR_INVALID_ARGUMENT;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int)s->queue.size() >= s->queue_capacity) {
            set_error("the request queue is full (%d)", s->queue_capacity);
            return RCP_ERR_QUEUE_FULL;
        }
        ticket = s->next_ticket++;
        Req q;
        q.r = r;
        q.bytes = bytes;
        q.t_submit = s->now();
        s->reqs.emplace(ticket, q);
        s->queue.push_back(ticket);
        ++s->generation;
    }
    s->cv.notify_all();
    return RCP_OK;
}

rcp_status server_poll(rcp_server* s, uint64_t ticket, int32_t& state, double times[3]) {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return RCP_ERR_INVALID_ARGUMENT;
    }
    state = it->second.state;
    if (times) {
        times[0] = it->second.t_submit;
        times[1] = it->second.t_start;
        times[2] = it->second.t_done;
    }
    return RCP_OK;
}

rcp_status server_result(rcp_server* s, uint64_t ticket, float** images, int32_t** ids) {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return RCP_ERR_INVALID_ARGUMENT;
    }
    const Req& r = it->second;
    if (r.state == RCP_REQ_FAILED) {
        set_error("request %llu failed", (unsigned long long)ticket);
        return RCP_ERR_DEVICE;
    }
    if (r.state != RCP_REQ_DONE) {
        set_error("request %llu is not done", (unsigned long long)ticket);
        return RCP_ERR_NOT_READY;
    }
    if (images) *images = (float*)(s->pool + r.offset);
    if (ids)
        *ids = r.r.with_ids
                   ? (int32_t*)(s->pool + r.offset + ((12 * (size_t)r.r.W * r.r.H * r.r.K + 255) & ~(size_t)255))
                   : nullptr;
    return RCP_OK;
}

rcp_status server_result_copy(rcp_server* s, uint64_t ticket, float* images, int32_t* ids, hipStream_t stream) {
    float* src = nullptr;
    int32_t* src_ids = nullptr;
    rcp_status st = server_result(s, ticket, &src, &src_ids);
    if (st != RCP_OK) return st;
    size_t n = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const Req& r = s->reqs[ticket];
        n = (size_t)r.r.W * (size_t)r.r.H * (size_t)r.r.K;
    }
    if (images) RCP_HIP(hipMemcpyAsync(images, src, 12 * n, hipMemcpyDeviceToDevice, stream));
    if (ids) {
        if (!src_ids) {
            set_error("request %llu was submitted without ids", (unsigned long long)ticket);
            return RCP_ERR_INVALID_ARGUMENT;
        }
        RCP_HIP(hipMemcpyAsync(ids, src_ids, 4 * n, hipMemcpyDeviceToDevice, stream));
    }
    return RCP_OK;
}

rcp_status server_release(rcp_server* s, uint64_t ticket) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) {
            set_error("unknown ticket %llu", (unsigned long long)ticket);
            return RCP_ERR_INVALID_ARGUMENT;
        }
        if (it->second.state != RCP_REQ_DONE && it->second.state != RCP_REQ_FAILED) {
            set_error("request %llu is still queued or running", (unsigned long long)ticket);
            return RCP_ERR_NOT_READY;
        }
        if (it->second.in_pool) s->pool_free(it->second.offset, it->second.bytes);
        s->reqs.erase(it);
        ++s->generation;
    }
    s->cv.notify_all();
    return RCP_OK;
}

rcp_status server_stats(rcp_server* s, uint64_t out[4]) {
    std::lock_guard<std::mutex> lk(s->mu);
    size_t free_bytes = 0;
    for (auto& f : s->free_list) free_bytes += f.second;
    out[0] = s->launches;
    out[1] = s->queue.size() + s->admitted.size();
    out[2] = s->pool_bytes - free_bytes;
    out[3] = s->reqs.size();
    return RCP_OK;
}

}  // namespace rcp
