// server.cpp -- the serving engine of include/ctserve.h: a request queue, admission against a
// device arena, merging of queued requests that share a plan into one batched call, and
// concurrent calls on per-slot HIP streams, driven by one host thread.
#include "engine.h"
#include "serve_host.h"

#include "../../include/ctserve.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

bool valid_dtype(ctp_dtype d) { return d == CTP_F32 || d == CTP_BF16 || d == CTP_F16; }

struct Batch;

struct Request {
    uint64_t id = 0;
    const ctp_plan *plan = nullptr;
    ctp_direction dir = CTP_FORWARD;
    const void *input = nullptr;
    ctp_dtype in_dt = CTP_F32, out_dt = CTP_F32;
    size_t in_bytes = 0, out_bytes = 0;
    double work = 0.0;                     // voxel-view updates: the cost estimate
    hipEvent_t ready = nullptr;            // recorded on the producer's stream at submit
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    enum State { kQueued, kRunning, kDone, kFailed } state = kQueued;
    ctp_status err = CTP_OK;
    std::string msg;
    std::shared_ptr<Batch> batch;
    int index = 0;
};

struct Batch {
    std::vector<Request *> items;
    int slot = -1;
    size_t out_off = ctp::Arena::kFail, scratch_off = ctp::Arena::kFail;
    size_t in_item = 0, out_item = 0, staging = 0, ws_bytes = 0;
    int live = 0;                             // items whose output is not yet released
    std::vector<hipEvent_t> release_events;   // the consumers' last uses of the outputs
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::shared_ptr<Batch> batch;             // running call, or empty
};

ctp::BatchKey key_of(const Request *r)
{
    return ctp::BatchKey{r->plan, (int)r->dir, (int)r->in_dt, (int)r->out_dt};
}

// workspace of one call of n items
ctp_status call_workspace(const Request *r, int64_t n, size_t *bytes)
{
    const ctp_dtype vol_dt = r->dir == CTP_FORWARD ? r->in_dt : r->out_dt;
    const ctp_dtype sino_dt = r->dir == CTP_FORWARD ? r->out_dt : r->in_dt;
    return ctp_workspace_bytes(r->plan, r->dir, vol_dt, sino_dt, n, bytes);
}

}  // namespace

// Interval at which the server thread looks at the completion events of running calls.
constexpr int kPollUs = 50;

struct ctp_server {
    int device = -1;
    char *arena = nullptr;
    int max_batch = 1;
    int64_t age_cap_ns = 0;             // 0: strict first come, first served
    double express_work = 0.0;          // > 0: the last slot takes only calls this short, and
                                        // longer calls run one at a time
    double launch_work = 0.0;           // > 0: most voxel-view updates per kernel launch
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable wake;       // worker: new request, release or stop
    std::condition_variable done_cv;    // waiters: a request finished
    bool stop = false;
    ctp::Arena alloc;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::vector<std::shared_ptr<Batch>> releasing;   // all outputs released, events pending
    std::vector<hipEvent_t> event_pool;
    uint64_t next_id = 1;
    ctp_server_stats stats{};
    std::thread worker;

    // ---- helpers (mu held) -------------------------------------------------------------------
    int running() const
    {
        int n = 0;
        for (const Slot &s : slots)
            n += s.batch ? 1 : 0;
        return n;
    }
    bool is_express(int slot) const
    {
        return express_work > 0.0 && slots.size() >= 2 && slot == (int)slots.size() - 1;
    }
    bool is_long(const Request *r) const { return express_work > 0.0 && r->work > express_work; }
    bool long_running() const
    {
        for (const Slot &s : slots)
            if (s.batch && is_long(s.batch->items.front()))
                return true;
        return false;
    }
    void free_batch_scratch(Batch &b)
    {
        if (b.scratch_off != ctp::Arena::kFail)
            alloc.release(b.scratch_off);
        b.scratch_off = ctp::Arena::kFail;
    }
    void free_batch_output(Batch &b)
    {
        if (b.out_off != ctp::Arena::kFail)
            alloc.release(b.out_off);
        b.out_off = ctp::Arena::kFail;
        for (hipEvent_t e : b.release_events)
            event_pool.push_back(e);
        b.release_events.clear();
    }

    // Completed calls and outputs whose consumers have finished.  Returns true on progress.
    bool poll()
    {
        bool progress = false;
        for (Slot &s : slots) {
            if (!s.batch)
                continue;
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady)
                continue;
            std::shared_ptr<Batch> b = std::move(s.batch);
            s.batch.reset();
            const int64_t t = now_ns();
            for (Request *r : b->items) {
                r->t_done = t;
                if (q == hipSuccess) {
                    r->state = Request::kDone;
                    ++stats.completed;
                } else {
                    r->state = Request::kFailed;
                    r->err = CTP_EDEVICE;
                    r->msg = std::string("call failed on the device: ") + hipGetErrorString(q);
                    ++stats.failed;
                }
                event_pool.push_back(r->ready);
                r->ready = nullptr;
            }
            free_batch_scratch(*b);
            progress = true;
        }
        for (size_t i = 0; i < releasing.size();) {
            Batch &b = *releasing[i];
            bool all = true;
            for (hipEvent_t e : b.release_events)
                if (hipEventQuery(e) == hipErrorNotReady) {
                    all = false;
                    break;
                }
            if (!all) {
                ++i;
                continue;
            }
            free_batch_output(b);
            releasing.erase(releasing.begin() + (std::ptrdiff_t)i);
            progress = true;
        }
        if (progress)
            done_cv.notify_all();
        return progress;
    }

    // Choose the next call: try heads in ctp::head_order (requests older than the age cap
    // first, oldest first; then the rest cheapest first), each with the queued requests that
    // may join its call, and reserve the memory and the slot of the first that fits.  A young
    // head that does not fit is passed over; an aged one is not (the memory that frees up is
    // kept for it), so no request waits behind later ones for longer than the cap.  Returns an
    // empty pointer if nothing may start now.
    // The express slot considers only short requests, and an aged long request does not hold
    // it (it can never run there).  Long requests run one at a time (each fills the device on
    // its own, and while two run the hardware hands the compute units freed by one to the
    // other before a third stream's work); one that waits for the running long call does not
    // hold the other slots either.
    std::shared_ptr<Batch> admit(int slot)
    {
        size_t n_aged = 0;
        const std::vector<size_t> order = ctp::head_order(
            queue, now_ns(), age_cap_ns,
            [](const Request *r) { return std::make_pair(r->work, r->t_submit); }, &n_aged);
        const bool express = is_express(slot);
        const bool long_busy = long_running();
        for (size_t k = 0; k < order.size(); ++k) {
            if (express && queue[order[k]]->work > express_work)
                continue;
            if (long_busy && is_long(queue[order[k]]))
                continue;
            std::shared_ptr<Batch> b = try_admit(order[k], slot);
            if (b || k < n_aged)
                return b;
        }
        return nullptr;
    }

    // Reserve a call headed by queue[head_pos] with as many of its batch candidates as fit.
    std::shared_ptr<Batch> try_admit(size_t head_pos, int slot)
    {
        // a call on the express slot stays short: at most express_work in all
        int cap = max_batch;
        if (is_express(slot) && queue[head_pos]->work > 0.0)
            cap = std::max(1, (int)std::min((double)max_batch, express_work / queue[head_pos]->work));
        std::vector<size_t> pos = ctp::batch_candidates(queue, head_pos, cap, key_of);
        const Request *head = queue[head_pos];
        for (int64_t n = (int64_t)pos.size(); n >= 1; --n) {
            size_t ws = 0;
            if (call_workspace(head, n, &ws) != CTP_OK)
                continue;
            const size_t staging = n > 1 ? ctp::Arena::round_up(head->in_bytes * (size_t)n) : 0;
            const size_t out_off = alloc.alloc(head->out_bytes * (size_t)n);
            if (out_off == ctp::Arena::kFail)
                continue;
            size_t scratch_off = ctp::Arena::kFail;
            if (staging + ws > 0) {
                // scratch lives only while the call runs: take it from the top of the arena
                scratch_off = alloc.alloc_high(staging + ws);
                if (scratch_off == ctp::Arena::kFail) {
                    alloc.release(out_off);
                    continue;
                }
            }
            auto b = std::make_shared<Batch>();
            b->slot = slot;
            b->out_off = out_off;
            b->scratch_off = scratch_off;
            b->in_item = head->in_bytes;
            b->out_item = head->out_bytes;
            b->staging = staging;
            b->ws_bytes = ws;
            // remove the chosen requests from the queue (highest position first keeps the
            // others valid)
            std::vector<Request *> items;
            for (int64_t i = 0; i < n; ++i)
                items.push_back(queue[pos[(size_t)i]]);
            std::vector<size_t> del(pos.begin(), pos.begin() + n);
            std::sort(del.begin(), del.end());
            for (auto it = del.rbegin(); it != del.rend(); ++it)
                queue.erase(queue.begin() + (std::ptrdiff_t)*it);
            const int64_t t = now_ns();
            for (int64_t i = 0; i < n; ++i) {
                Request *r = items[(size_t)i];
                r->state = Request::kRunning;
                r->batch = b;
                r->index = (int)i;
                r->t_admit = t;
            }
            b->items = std::move(items);
            b->live = (int)n;
            slots[(size_t)slot].batch = b;
            ++stats.calls;
            stats.max_running = std::max(stats.max_running, running());
            stats.max_batch_seen = std::max(stats.max_batch_seen, (int32_t)n);
            stats.arena_peak = alloc.peak();
            return b;
        }
        return nullptr;
    }

    // Enqueue a reserved call on its slot's stream (mu not held).  Returns false and the
    // message if nothing could be enqueued.
    bool launch(Batch &b, std::string &msg)
    {
        const Slot &s = slots[(size_t)b.slot];
        const Request *head = b.items.front();
        const int64_t n = (int64_t)b.items.size();
        hipError_t e = hipSuccess;
        for (const Request *r : b.items)
            if (e == hipSuccess)
                e = hipStreamWaitEvent(s.stream, r->ready, 0);
        const void *in = head->input;
        char *scratch = b.scratch_off == ctp::Arena::kFail ? nullptr : arena + b.scratch_off;
        if (n > 1) {
            for (int64_t i = 0; i < n && e == hipSuccess; ++i)
                e = hipMemcpyAsync(scratch + (size_t)i * b.in_item, b.items[(size_t)i]->input,
                                   b.in_item, hipMemcpyDeviceToDevice, s.stream);
            in = scratch;
        }
        if (e != hipSuccess) {
            msg = std::string("input staging: ") + hipGetErrorString(e);
            return false;
        }
        void *ws = b.ws_bytes > 0 ? scratch + b.staging : nullptr;
        void *out = arena + b.out_off;
        // split the call over view ranges so that no launch holds the device much longer than
        // launch_work updates take (the other slots' work starts between launches)
        const int nv = ctp::plan_views(head->plan);
        int vpl = nv;
        if (launch_work > 0.0 && head->work > 0.0) {
            const double per_view = head->work * (double)n / (double)nv;
            vpl = (int)std::max(1.0, std::min((double)nv, std::floor(launch_work / per_view)));
        }
        const ctp_status st =
            head->dir == CTP_FORWARD
                ? ctp::project_sliced(head->plan, in, head->in_dt, out, head->out_dt, n, ws,
                                      b.ws_bytes, vpl, s.stream)
                : ctp::backproject_sliced(head->plan, in, head->in_dt, out, head->out_dt, n, ws,
                                          b.ws_bytes, vpl, s.stream);
        if (st != CTP_OK) {
            msg = ctp_last_error();
            return false;
        }
        e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) {
            msg = std::string("event record: ") + hipGetErrorString(e);
            return false;
        }
        return true;
    }

    void fail_batch(std::shared_ptr<Batch> b, const std::string &msg)
    {
        // wait for whatever was enqueued before reusing the memory
        (void)hipStreamSynchronize(slots[(size_t)b->slot].stream);
        std::lock_guard<std::mutex> lk(mu);
        slots[(size_t)b->slot].batch.reset();
        const int64_t t = now_ns();
        for (Request *r : b->items) {
            r->state = Request::kFailed;
            r->err = CTP_EDEVICE;
            r->msg = msg;
            r->t_done = t;
            r->batch.reset();
            event_pool.push_back(r->ready);
            r->ready = nullptr;
            ++stats.failed;
        }
        free_batch_scratch(*b);
        free_batch_output(*b);
        done_cv.notify_all();
    }

    void run()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            poll();
            // free slots in order (the express slot, the last, after the others): each takes
            // the next call it may run; when a regular slot can start nothing, no other regular
            // slot can, and only the express slot is still tried
            for (size_t slot = 0; slot < slots.size() && !queue.empty(); ++slot) {
                if (slots[slot].batch)
                    continue;
                std::shared_ptr<Batch> b = admit((int)slot);
                if (!b) {
                    if (express_work > 0.0 && slots.size() >= 2 && slot + 1 < slots.size() - 1)
                        slot = slots.size() - 2;       // next: the express slot
                    continue;
                }
                lk.unlock();
                std::string msg;
                const bool ok = launch(*b, msg);
                if (!ok)
                    fail_batch(b, msg);
                lk.lock();
            }
            const bool busy = running() > 0 || !releasing.empty();
            if (stop && !busy) {
                // nothing runs and nothing will be freed: what is still queued cannot start
                const int64_t t = now_ns();
                for (Request *r : queue) {
                    r->state = Request::kFailed;
                    r->err = CTP_ENOMEM;
                    r->msg = "server stopped with the request still queued (arena full)";
                    r->t_done = t;
                    ++stats.failed;
                }
                queue.clear();
                done_cv.notify_all();
                return;
            }
            if (busy) {
                // calls in flight: look at their events again after a short sleep, or at once
                // when a request arrives, is released or cancelled
                wake.wait_for(lk, std::chrono::microseconds(kPollUs));
            } else {
                wake.wait(lk);
            }
        }
    }

    hipEvent_t take_event()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (!event_pool.empty()) {
                hipEvent_t e = event_pool.back();
                event_pool.pop_back();
                return e;
            }
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return nullptr;
        return e;
    }
};

extern "C" {

ctp_status ctp_server_create(const ctp_server_config *cfg, ctp_server **out)
{
    ctp::clear_error();
    if (cfg == nullptr || out == nullptr)
        return ctp::set_error(CTP_EINVAL, "NULL config or output pointer");
    if (cfg->arena == nullptr || cfg->arena_bytes < ctp::Arena::kAlign)
        return ctp::set_error(CTP_EINVAL, "arena must be non-NULL and at least 256 bytes");
    if (((uintptr_t)cfg->arena & (ctp::Arena::kAlign - 1)) != 0)
        return ctp::set_error(CTP_EINVAL, "arena must be 256-byte aligned");
    if (cfg->n_slots < 1 || cfg->n_slots > 16)
        return ctp::set_error(CTP_EINVAL, "n_slots must be in 1..16");
    if (cfg->max_batch < 1 || cfg->max_batch > 1024)
        return ctp::set_error(CTP_EINVAL, "max_batch must be in 1..1024");
    if (cfg->age_cap_us < 0)
        return ctp::set_error(CTP_EINVAL, "age_cap_us must be >= 0");
    if (!(cfg->express_work >= 0.0))
        return ctp::set_error(CTP_EINVAL, "express_work must be >= 0");
    if (!(cfg->launch_work >= 0.0))
        return ctp::set_error(CTP_EINVAL, "launch_work must be >= 0");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess)
        return ctp::set_error(CTP_EDEVICE, "no HIP device");
    ctp_server *s = new (std::nothrow) ctp_server();
    if (s == nullptr)
        return ctp::set_error(CTP_ENOMEM, "host allocation failed");
    s->device = dev;
    s->arena = static_cast<char *>(cfg->arena);
    s->max_batch = cfg->max_batch;
    s->age_cap_ns = cfg->age_cap_us * 1000;
    s->express_work = cfg->express_work;
    s->launch_work = cfg->launch_work;
    s->alloc.reset(cfg->arena_bytes);
    s->slots.resize((size_t)cfg->n_slots);
    for (Slot &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            for (Slot &t : s->slots) {
                if (t.stream)
                    (void)hipStreamDestroy(t.stream);
                if (t.done)
                    (void)hipEventDestroy(t.done);
            }
            delete s;
            return ctp::set_error(CTP_EDEVICE, "stream or event creation failed");
        }
    }
    try {
        s->worker = std::thread([s] { s->run(); });
    } catch (...) {
        for (Slot &t : s->slots) {
            (void)hipStreamDestroy(t.stream);
            (void)hipEventDestroy(t.done);
        }
        delete s;
        return ctp::set_error(CTP_ENOMEM, "could not start the server thread");
    }
    *out = s;
    return CTP_OK;
}

ctp_status ctp_server_submit(ctp_server *srv, const ctp_plan *plan, ctp_direction dir,
                             const void *input, ctp_dtype in_dtype, ctp_dtype out_dtype,
                             hipStream_t ready, uint64_t *ticket)
{
    ctp::clear_error();
    if (srv == nullptr || plan == nullptr || input == nullptr || ticket == nullptr)
        return ctp::set_error(CTP_EINVAL, "NULL server, plan, input or ticket pointer");
    if (dir != CTP_FORWARD && dir != CTP_BACKWARD)
        return ctp::set_error(CTP_EINVAL, "unknown direction");
    if (!valid_dtype(in_dtype) || !valid_dtype(out_dtype))
        return ctp::set_error(CTP_EINVAL, "unknown dtype");
    if (ctp::plan_device(plan) != srv->device)
        return ctp::set_error(CTP_EINVAL, "plan belongs to another device");
    auto r = std::make_unique<Request>();
    r->plan = plan;
    r->dir = dir;
    r->input = input;
    r->in_dt = in_dtype;
    r->out_dt = out_dtype;
    size_t vb_in = 0, sb_in = 0, vb_out = 0, sb_out = 0;
    ctp_plan_bytes(plan, in_dtype, 1, &vb_in, &sb_in);
    ctp_plan_bytes(plan, out_dtype, 1, &vb_out, &sb_out);
    r->in_bytes = dir == CTP_FORWARD ? vb_in : sb_in;
    r->out_bytes = dir == CTP_FORWARD ? sb_out : vb_out;
    r->work = ctp::plan_work(plan);
    size_t ws = 0;
    if (call_workspace(r.get(), 1, &ws) != CTP_OK)
        return CTP_EINVAL;
    if (ctp::Arena::round_up(r->out_bytes) + ctp::Arena::round_up(ws) > srv->alloc.size())
        return ctp::set_error(CTP_ENOMEM, "request needs " +
                                              std::to_string(ctp::Arena::round_up(r->out_bytes) +
                                                             ctp::Arena::round_up(ws)) +
                                              " arena bytes, the arena has " +
                                              std::to_string(srv->alloc.size()));
    r->ready = srv->take_event();
    if (r->ready == nullptr)
        return ctp::set_error(CTP_EDEVICE, "event creation failed");
    if (hipEventRecord(r->ready, ready) != hipSuccess) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->event_pool.push_back(r->ready);
        return ctp::set_error(CTP_EDEVICE, "event record on the producer stream failed");
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop)
            return ctp::set_error(CTP_EINVAL, "server is stopping");
        r->id = srv->next_id++;
        r->t_submit = now_ns();
        *ticket = r->id;
        srv->queue.push_back(r.get());
        srv->reqs[r->id] = std::move(r);
        ++srv->stats.submitted;
    }
    srv->wake.notify_one();
    return CTP_OK;
}

ctp_status ctp_server_wait(ctp_server *srv, uint64_t ticket, int64_t timeout_us, void **result)
{
    ctp::clear_error();
    if (srv == nullptr)
        return ctp::set_error(CTP_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end())
        return ctp::set_error(CTP_EINVAL, "unknown or released ticket");
    Request *r = it->second.get();
    auto finished = [r] { return r->state == Request::kDone || r->state == Request::kFailed; };
    if (timeout_us < 0) {
        srv->done_cv.wait(lk, finished);
    } else if (!srv->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), finished)) {
        return ctp::set_error(CTP_ETIMEOUT, "timeout");
    }
    if (r->state == Request::kFailed)
        return ctp::set_error(r->err, r->msg);
    if (result)
        *result = srv->arena + r->batch->out_off + (size_t)r->index * r->batch->out_item;
    return CTP_OK;
}

ctp_status ctp_server_query(ctp_server *srv, uint64_t ticket, int *done, void **result)
{
    ctp::clear_error();
    if (srv == nullptr || done == nullptr)
        return ctp::set_error(CTP_EINVAL, "NULL server or output pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end())
        return ctp::set_error(CTP_EINVAL, "unknown or released ticket");
    Request *r = it->second.get();
    *done = r->state == Request::kDone || r->state == Request::kFailed;
    if (r->state == Request::kFailed)
        return ctp::set_error(r->err, r->msg);
    if (*done && result)
        *result = srv->arena + r->batch->out_off + (size_t)r->index * r->batch->out_item;
    return CTP_OK;
}

ctp_status ctp_server_info(ctp_server *srv, uint64_t ticket, ctp_request_info *info)
{
    ctp::clear_error();
    if (srv == nullptr || info == nullptr)
        return ctp::set_error(CTP_EINVAL, "NULL server or output pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end())
        return ctp::set_error(CTP_EINVAL, "unknown or released ticket");
    const Request *r = it->second.get();
    info->submit_ns = r->t_submit;
    info->admit_ns = r->t_admit;
    info->done_ns = r->t_done;
    info->batch = r->batch ? (int32_t)r->batch->items.size() : 0;
    info->slot = r->batch ? r->batch->slot : -1;
    return CTP_OK;
}

ctp_status ctp_server_release(ctp_server *srv, uint64_t ticket, hipStream_t consumer)
{
    ctp::clear_error();
    if (srv == nullptr)
        return ctp::set_error(CTP_EINVAL, "NULL server");
    hipEvent_t ev = srv->take_event();
    if (ev == nullptr)
        return ctp::set_error(CTP_EDEVICE, "event creation failed");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || it->second->state == Request::kQueued ||
        it->second->state == Request::kRunning) {
        srv->event_pool.push_back(ev);
        return ctp::set_error(CTP_EINVAL, it == srv->reqs.end() ? "unknown or released ticket"
                                                               : "request is not finished");
    }
    std::shared_ptr<Batch> b = it->second->batch;
    srv->reqs.erase(it);
    if (!b) {                       // failed before its call held memory
        srv->event_pool.push_back(ev);
        return CTP_OK;
    }
    if (hipEventRecord(ev, consumer) != hipSuccess) {
        // fall back to waiting for the whole device before reuse
        (void)hipDeviceSynchronize();
        srv->event_pool.push_back(ev);
    } else {
        b->release_events.push_back(ev);
    }
    if (--b->live == 0)
        srv->releasing.push_back(b);
    srv->wake.notify_one();
    return CTP_OK;
}

ctp_status ctp_server_cancel(ctp_server *srv, uint64_t ticket)
{
    ctp::clear_error();
    if (srv == nullptr)
        return ctp::set_error(CTP_EINVAL, "NULL server");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end())
            return ctp::set_error(CTP_EINVAL, "unknown or released ticket");
        Request *r = it->second.get();
        if (r->state != Request::kQueued)
            return ctp::set_error(CTP_EINVAL, r->state == Request::kRunning
                                                  ? "request is running: it can no longer be cancelled"
                                                  : "request has already finished");
        for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q)
            if (*q == r) {
                srv->queue.erase(q);
                break;
            }
        r->state = Request::kFailed;
        r->err = CTP_ECANCELED;
        r->msg = "request cancelled before it ran";
        r->t_done = now_ns();
        srv->event_pool.push_back(r->ready);
        r->ready = nullptr;
        ++srv->stats.cancelled;
        srv->done_cv.notify_all();
    }
    srv->wake.notify_one();      // a head that was waiting for memory may have gone
    return CTP_OK;
}

ctp_status ctp_server_get_stats(ctp_server *srv, ctp_server_stats *stats)
{
    ctp::clear_error();
    if (srv == nullptr || stats == nullptr)
        return ctp::set_error(CTP_EINVAL, "NULL server or output pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    *stats = srv->stats;
    stats->arena_peak = srv->alloc.peak();
    return CTP_OK;
}

ctp_status ctp_server_destroy(ctp_server *srv)
{
    ctp::clear_error();
    if (srv == nullptr)
        return CTP_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->wake.notify_one();
    if (srv->worker.joinable())
        srv->worker.join();
    for (Slot &s : srv->slots) {
        (void)hipStreamSynchronize(s.stream);
        (void)hipStreamDestroy(s.stream);
        (void)hipEventDestroy(s.done);
    }
    for (auto &b : srv->releasing)
        for (hipEvent_t e : b->release_events) {
            (void)hipEventSynchronize(e);
            (void)hipEventDestroy(e);
        }
    std::set<Batch *> held;          // batches with unreleased outputs (shared by their items)
    for (auto &kv : srv->reqs) {
        if (kv.second->ready)
            (void)hipEventDestroy(kv.second->ready);
        if (kv.second->batch)
            held.insert(kv.second->batch.get());
    }
    for (Batch *b : held)
        for (hipEvent_t e : b->release_events) {
            (void)hipEventSynchronize(e);
            (void)hipEventDestroy(e);
        }
    for (hipEvent_t e : srv->event_pool)
        (void)hipEventDestroy(e);
    delete srv;
    return CTP_OK;
}

}  // extern "C"
