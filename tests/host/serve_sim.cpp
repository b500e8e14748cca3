// CPU simulation of the serving engine: csrc/server.cpp compiled unchanged against a simulated
// device (tests/host/fakehip) on which every stream runs its work for a set duration of wall
// time, events complete when the work before them has run, and the projector calls are stubs
// that only check their workspace against the library's size formulas and occupy their stream.
// Scenarios: bursts of mixed requests (large calls first, then many small ones of several
// plans, directions and storage types) with outputs held until every request is done, as a
// client that reads its results in submission order would; every request must complete.
// Failure handling: calls that fail to launch and calls whose completion reports a device error
// (injected through plans marked to fail) fail their own requests only, while every other
// request in flight completes and all arena memory comes back; queued requests can be
// cancelled; small requests overtake a long queue of large ones until the age cap; with an
// express threshold long calls run one at a time, split into launches by launch_work.
// Prints "ok" and exits 0 on success.
#include "../../paper_2503_16741_amd/csrc/server.cpp"

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>

// ---- simulated device -------------------------------------------------------------------------
struct SimStream {
    std::mutex mu;
    double busy_until = 0.0;     // microseconds on the steady clock
    bool poisoned = false;       // the work enqueued since the last event record failed
};
struct SimEvent {
    std::atomic<double> ready_at{0.0};
    std::atomic<bool> failed{false};
};

static double now_us()
{
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

static double enqueue(hipStream_t s, double dur)
{
    if (s == nullptr)
        return now_us() + dur;
    std::lock_guard<std::mutex> lk(s->mu);
    s->busy_until = std::max(s->busy_until, now_us()) + dur;
    return s->busy_until;
}

hipError_t hipGetDevice(int *dev) { *dev = 0; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = new SimStream(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t s)
{
    const double t = enqueue(s, 0.0);
    while (now_us() < t)
        std::this_thread::yield();
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned)
{
    std::lock_guard<std::mutex> lk(s->mu);
    s->busy_until = std::max(s->busy_until, e->ready_at.load());
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = new SimEvent(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    e->ready_at = enqueue(s, 0.0);
    bool bad = false;
    if (s != nullptr) {
        std::lock_guard<std::mutex> lk(s->mu);
        bad = s->poisoned;
        s->poisoned = false;
    }
    e->failed = bad;
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e)
{
    if (now_us() < e->ready_at)
        return hipErrorNotReady;
    return e->failed ? hipErrorLaunchFailure : hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    while (hipEventQuery(e) == hipErrorNotReady)
        std::this_thread::yield();
    return hipEventQuery(e);
}
hipError_t hipMemcpyAsync(void *, const void *, size_t n, hipMemcpyKind, hipStream_t s)
{
    enqueue(s, 1.0 + n * 1e-6);
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "success" : "error"; }

// ---- simulated plans: the library's size formulas ---------------------------------------------
struct ctp_plan {
    int device = 0;
    bool two_d = false, recon = false, sf = true;
    size_t nvox = 0, ncell = 0, plane = 0;
    double us_per_item = 10.0;
    int n_views = 8;
    int fail = 0;                // 1: the call fails to launch; 2: it fails on the device
};

static size_t a256(size_t n) { return (n + 255) & ~(size_t)255; }
static size_t esz(ctp_dtype d) { return d == CTP_F32 ? 4 : 2; }

static thread_local std::string sim_err;
namespace ctp {
ctp_status set_error(ctp_status st, const std::string &msg) { sim_err = msg; return st; }
void clear_error() { sim_err.clear(); }
int plan_device(const ctp_plan *plan) { return plan->device; }
double plan_work(const ctp_plan *plan) { return plan->us_per_item; }
int plan_views(const ctp_plan *plan) { return plan->n_views; }
}  // namespace ctp
extern "C" const char *ctp_last_error(void) { return sim_err.c_str(); }

extern "C" ctp_status ctp_plan_bytes(const ctp_plan *p, ctp_dtype d, int64_t batch, size_t *vb,
                                     size_t *sb)
{
    if (vb)
        *vb = p->nvox * (size_t)batch * esz(d);
    if (sb)
        *sb = p->ncell * (size_t)batch * esz(d);
    return CTP_OK;
}

extern "C" ctp_status ctp_workspace_bytes(const ctp_plan *p, ctp_direction dir, ctp_dtype vd,
                                          ctp_dtype sd, int64_t batch, size_t *bytes)
{
    const size_t b = (size_t)batch;
    if (dir == CTP_FORWARD) {
        const size_t item = p->two_d ? p->plane : p->nvox;
        const size_t bpi = std::max<size_t>(1, std::min<size_t>((item + 8191) / 8192, 1024));
        size_t t = a256(8 * b) + a256(b * bpi * 4) + a256(b * p->nvox * 4);
        if (sd != CTP_F32)
            t += p->ncell * b * 4;
        *bytes = t;
    } else {
        const bool scaled = !(sd == CTP_F32 && (p->recon || (p->two_d && p->sf)));
        const size_t off = scaled ? a256(p->ncell * b * 4) : 0;
        *bytes = off + (vd == CTP_F32 ? 0 : p->nvox * b * 4);
    }
    return CTP_OK;
}

static std::atomic<int> bad_calls{0};
static std::atomic<int> launches{0};    // kernel launches of the projector calls

// One call: its work enqueued on the stream as ceil(n_views / views_per_launch) launches.
static ctp_status sim_call(const ctp_plan *p, ctp_direction dir, ctp_dtype vd, ctp_dtype sd,
                           int64_t batch, void *ws, size_t ws_bytes, int vpl, hipStream_t st)
{
    size_t need = 0;
    ctp_workspace_bytes(p, dir, vd, sd, batch, &need);
    if (need > 0 && (ws == nullptr || ws_bytes < need || ((uintptr_t)ws & 255u))) {
        ++bad_calls;
        return ctp::set_error(CTP_EINVAL, "workspace too small or misaligned");
    }
    if (vpl < 1) {
        ++bad_calls;
        return ctp::set_error(CTP_EINVAL, "views_per_launch must be >= 1");
    }
    if (p->fail == 1)
        return ctp::set_error(CTP_EDEVICE, "injected launch failure");
    for (int v0 = 0; v0 < p->n_views; v0 += vpl) {
        const int n = std::min(vpl, p->n_views - v0);
        enqueue(st, p->us_per_item * (double)batch * n / p->n_views);
        ++launches;
    }
    if (p->fail == 2) {
        std::lock_guard<std::mutex> lk(st->mu);
        st->poisoned = true;
    }
    return CTP_OK;
}

namespace ctp {
ctp_status project_sliced(const ctp_plan *p, const void *, ctp_dtype vd, void *, ctp_dtype sd,
                          int64_t batch, void *ws, size_t wsb, int vpl, hipStream_t st)
{
    return sim_call(p, CTP_FORWARD, vd, sd, batch, ws, wsb, vpl, st);
}

ctp_status backproject_sliced(const ctp_plan *p, const void *, ctp_dtype sd, void *, ctp_dtype vd,
                              int64_t batch, void *ws, size_t wsb, int vpl, hipStream_t st)
{
    return sim_call(p, CTP_BACKWARD, vd, sd, batch, ws, wsb, vpl, st);
}
}  // namespace ctp

#define CHECK(c)                                                                          \
    do {                                                                                  \
        if (!(c)) {                                                                       \
            std::fprintf(stderr, "%s:%d: CHECK(%s) failed\n", __FILE__, __LINE__, #c);    \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)

struct Req {
    ctp_plan *plan;
    ctp_direction dir;
    ctp_dtype in, out;
};

// One burst: n_big large forward calls, then n_small mixed requests; the client waits for every
// ticket in order and releases the outputs only at the end.
static void burst(unsigned seed, size_t arena_bytes, int slots, int max_batch, int n_big,
                  int n_small)
{
    ctp_plan big, fan, cone, recon;
    big.nvox = 128ull * 128 * 128; big.ncell = 300ull * 200 * 256; big.us_per_item = 1500;
    fan.two_d = true; fan.nvox = fan.plane = 40 * 36; fan.ncell = 24 * 96; fan.us_per_item = 40;
    cone.nvox = 28 * 26 * 18; cone.ncell = 20 * 40 * 64; cone.us_per_item = 60;
    recon = cone; recon.recon = true;
    ctp_plan *smalls[3] = {&fan, &cone, &recon};
    std::mt19937 rng(seed);
    std::vector<Req> reqs;
    for (int i = 0; i < n_big; ++i)
        reqs.push_back({&big, CTP_FORWARD, CTP_F32, CTP_F32});
    const ctp_dtype dts[3] = {CTP_F32, CTP_BF16, CTP_F16};
    for (int i = 0; i < n_small; ++i) {
        Req r;
        r.plan = smalls[rng() % 3];
        r.dir = rng() % 2 ? CTP_FORWARD : CTP_BACKWARD;
        r.in = dts[rng() % 3];
        r.out = rng() % 10 < 7 ? r.in : CTP_F32;
        reqs.push_back(r);
    }
    // odd seeds: strict arrival order; even: age cap 20 ms; every third seed with two or more
    // slots also reserves the last slot for the small plans
    const double express = (seed % 3 == 0 && slots >= 2) ? 100.0 : 0.0;   // plan_work: us per item
    // every fourth seed splits calls into launches of at most 150 us of work
    ctp_server_config cfg{reinterpret_cast<void *>((uintptr_t)1 << 40), arena_bytes, slots, max_batch,
                          seed % 2 ? 0 : 20000, express, seed % 4 == 0 ? 150.0 : 0.0};
    ctp_server *srv = nullptr;
    CHECK(ctp_server_create(&cfg, &srv) == CTP_OK);
    static char dummy_input[16];
    std::vector<uint64_t> tickets;
    for (const Req &r : reqs) {
        uint64_t t = 0;
        const ctp_status st = ctp_server_submit(srv, r.plan, r.dir, dummy_input, r.in, r.out,
                                                nullptr, &t);
        CHECK(st == CTP_OK);
        tickets.push_back(t);
    }
    for (size_t i = 0; i < tickets.size(); ++i) {
        void *res = nullptr;
        const ctp_status st = ctp_server_wait(srv, tickets[i], 20 * 1000 * 1000, &res);
        if (st != CTP_OK) {
            ctp_server_stats s{};
            ctp_server_get_stats(srv, &s);
            std::fprintf(stderr,
                         "seed %u arena %zu slots %d max_batch %d: request %zu of %zu: %s "
                         "(status %d); submitted %lld completed %lld failed %lld calls %lld\n",
                         seed, arena_bytes, slots, max_batch, i, tickets.size(), ctp_last_error(),
                         (int)st, (long long)s.submitted, (long long)s.completed,
                         (long long)s.failed, (long long)s.calls);
            std::exit(1);
        }
        CHECK(res != nullptr);
    }
    for (uint64_t t : tickets)
        CHECK(ctp_server_release(srv, t, nullptr) == CTP_OK);
    ctp_server_stats s{};
    ctp_server_get_stats(srv, &s);
    CHECK(s.completed == (int64_t)tickets.size() && s.failed == 0);
    CHECK(s.arena_peak <= arena_bytes);
    CHECK(ctp_server_destroy(srv) == CTP_OK);
}

static ctp_server *make_server(size_t arena_bytes, int slots, int max_batch, int64_t age_cap_us,
                               double express_work = 0.0, double launch_work = 0.0)
{
    ctp_server_config cfg{reinterpret_cast<void *>((uintptr_t)1 << 40), arena_bytes, slots, max_batch,
                          age_cap_us, express_work, launch_work};
    ctp_server *srv = nullptr;
    CHECK(ctp_server_create(&cfg, &srv) == CTP_OK);
    return srv;
}

// Release every ticket and wait (bounded) until the arena is empty again.
static void release_all_and_drain(ctp_server *srv, const std::vector<uint64_t> &tickets)
{
    for (uint64_t t : tickets)
        CHECK(ctp_server_release(srv, t, nullptr) == CTP_OK);
    for (int i = 0; i < 20000; ++i) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (srv->alloc.in_use() == 0 && srv->releasing.empty())
                return;
        }
        srv->wake.notify_one();
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    CHECK(!"arena memory did not come back");
}

// A mix in which some calls fail to launch and some fail on the device: exactly the requests of
// the failing plans fail, with the device status, and everything else completes.
static void failure_injection(unsigned seed)
{
    ctp_plan ok_a, ok_b, bad_launch, bad_device;
    ok_a.nvox = 20 * 20 * 20; ok_a.ncell = 16 * 30 * 30; ok_a.us_per_item = 80;
    ok_b.two_d = true; ok_b.nvox = ok_b.plane = 30 * 30; ok_b.ncell = 20 * 64; ok_b.us_per_item = 30;
    bad_launch = ok_a; bad_launch.fail = 1;
    bad_device = ok_b; bad_device.fail = 2;
    ctp_plan *plans[4] = {&ok_a, &ok_b, &bad_launch, &bad_device};
    std::mt19937 rng(seed);
    ctp_server *srv = make_server(64u << 20, 3, 4, seed % 2 ? 0 : 5000);
    static char dummy_input[16];
    std::vector<uint64_t> tickets;
    std::vector<int> which;
    for (int i = 0; i < 120; ++i) {
        const int k = (int)(rng() % 4);
        uint64_t t = 0;
        CHECK(ctp_server_submit(srv, plans[k], rng() % 2 ? CTP_FORWARD : CTP_BACKWARD, dummy_input,
                                CTP_F32, CTP_F32, nullptr, &t) == CTP_OK);
        tickets.push_back(t);
        which.push_back(k);
    }
    int n_fail = 0;
    for (size_t i = 0; i < tickets.size(); ++i) {
        void *res = nullptr;
        const ctp_status st = ctp_server_wait(srv, tickets[i], 20 * 1000 * 1000, &res);
        if (which[i] >= 2) {
            CHECK(st == CTP_EDEVICE);
            ++n_fail;
        } else {
            CHECK(st == CTP_OK && res != nullptr);
        }
    }
    ctp_server_stats s{};
    ctp_server_get_stats(srv, &s);
    CHECK(s.failed == n_fail && s.completed == (int64_t)tickets.size() - n_fail);
    release_all_and_drain(srv, tickets);
    CHECK(ctp_server_destroy(srv) == CTP_OK);
}

// Wait (bounded) until the request's call has been admitted: the server thread may start late
// on a loaded host, so a fixed sleep is not enough.
static void wait_running(ctp_server *srv, uint64_t ticket)
{
    for (int i = 0; i < 20000; ++i) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (srv->reqs.at(ticket)->state != Request::kQueued)
                return;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    CHECK(!"request was never admitted");
}

// Cancelling queued requests on a one-slot server held busy by a long call.
static void cancellation()
{
    ctp_plan slow, quick;
    slow.nvox = 32 * 32 * 32; slow.ncell = 20 * 40 * 40; slow.us_per_item = 50000;
    quick.nvox = 8 * 8 * 8; quick.ncell = 4 * 10 * 10; quick.us_per_item = 100;
    ctp_server *srv = make_server(64u << 20, 1, 1, 0);
    static char dummy_input[16];
    uint64_t busy = 0;
    CHECK(ctp_server_submit(srv, &slow, CTP_FORWARD, dummy_input, CTP_F32, CTP_F32, nullptr, &busy) == CTP_OK);
    std::vector<uint64_t> tickets;
    for (int i = 0; i < 10; ++i) {
        uint64_t t = 0;
        CHECK(ctp_server_submit(srv, &quick, CTP_FORWARD, dummy_input, CTP_F32, CTP_F32, nullptr, &t) == CTP_OK);
        tickets.push_back(t);
    }
    wait_running(srv, busy);
    CHECK(ctp_server_cancel(srv, busy) == CTP_EINVAL);             // running: not cancellable
    for (size_t i = 0; i < tickets.size(); i += 2)
        CHECK(ctp_server_cancel(srv, tickets[i]) == CTP_OK);
    CHECK(ctp_server_cancel(srv, tickets[0]) == CTP_EINVAL);       // already cancelled
    CHECK(ctp_server_cancel(srv, 987654321) == CTP_EINVAL);        // unknown ticket
    CHECK(ctp_server_wait(srv, busy, -1, nullptr) == CTP_OK);
    for (size_t i = 0; i < tickets.size(); ++i) {
        const ctp_status st = ctp_server_wait(srv, tickets[i], 20 * 1000 * 1000, nullptr);
        CHECK(st == (i % 2 == 0 ? CTP_ECANCELED : CTP_OK));
    }
    ctp_server_stats s{};
    ctp_server_get_stats(srv, &s);
    CHECK(s.cancelled == 5 && s.completed == 6 && s.calls == 6);
    tickets.push_back(busy);
    release_all_and_drain(srv, tickets);
    CHECK(ctp_server_destroy(srv) == CTP_OK);
}

// Order: behind a queue of long calls, short requests start first (smallest work first); once
// requests have waited past the age cap they run in arrival order.
static void ordering()
{
    ctp_plan big, small;
    big.nvox = 32 * 32 * 32; big.ncell = 20 * 40 * 40; big.us_per_item = 20000;
    small.nvox = 8 * 8 * 8; small.ncell = 4 * 10 * 10; small.us_per_item = 200;
    static char dummy_input[16];
    for (int64_t cap_us : {(int64_t)0, (int64_t)1000000, (int64_t)10000}) {
        ctp_server *srv = make_server(256u << 20, 1, 1, cap_us);
        std::vector<uint64_t> bigs, smalls;
        for (int i = 0; i < 4; ++i) {
            uint64_t t = 0;
            CHECK(ctp_server_submit(srv, &big, CTP_FORWARD, dummy_input, CTP_F32, CTP_F32, nullptr, &t) == CTP_OK);
            bigs.push_back(t);
            if (i == 0)   // the first big call is running before anything else is queued
                wait_running(srv, t);
        }
        for (int i = 0; i < 4; ++i) {
            uint64_t t = 0;
            CHECK(ctp_server_submit(srv, &small, CTP_FORWARD, dummy_input, CTP_F32, CTP_F32, nullptr, &t) == CTP_OK);
            smalls.push_back(t);
        }
        for (uint64_t t : bigs)
            CHECK(ctp_server_wait(srv, t, 20 * 1000 * 1000, nullptr) == CTP_OK);
        for (uint64_t t : smalls)
            CHECK(ctp_server_wait(srv, t, 20 * 1000 * 1000, nullptr) == CTP_OK);
        ctp_request_info b1{}, s_last{};
        CHECK(ctp_server_info(srv, bigs[1], &b1) == CTP_OK);
        CHECK(ctp_server_info(srv, smalls[3], &s_last) == CTP_OK);
        if (cap_us == 0)
            CHECK(s_last.admit_ns > b1.admit_ns);      // arrival order: the smalls wait
        else if (cap_us == 1000000)
            CHECK(s_last.admit_ns < b1.admit_ns);      // smallest first: they overtake
        else {
            // cap 10 ms: when the first big call ends (20 ms) every queued request has waited
            // ~17 ms, past the cap, so they run in arrival order: the smalls after the last big
            ctp_request_info b3{};
            CHECK(ctp_server_info(srv, bigs[3], &b3) == CTP_OK);
            CHECK(s_last.admit_ns > b3.admit_ns);
        }
        std::vector<uint64_t> all(bigs);
        all.insert(all.end(), smalls.begin(), smalls.end());
        release_all_and_drain(srv, all);
        CHECK(ctp_server_destroy(srv) == CTP_OK);
    }
}

// Express slot: with a two-slot server whose last slot takes only short requests, short requests
// that arrive behind a queue of long calls run at once on the express slot (they finish before
// the second long call starts), while the long calls keep the other slot; a long request never
// runs on the express slot.
static void express_slot()
{
    ctp_plan big, small;
    big.nvox = 32 * 32 * 32; big.ncell = 20 * 40 * 40; big.us_per_item = 20000;
    small.nvox = 8 * 8 * 8; small.ncell = 4 * 10 * 10; small.us_per_item = 200;
    static char dummy_input[16];
    const double small_work = ctp::plan_work(&small);
    ctp_server *srv = make_server(256u << 20, 2, 1, 0, small_work);
    std::vector<uint64_t> bigs, smalls;
    for (int i = 0; i < 3; ++i) {
        uint64_t t = 0;
        CHECK(ctp_server_submit(srv, &big, CTP_FORWARD, dummy_input, CTP_F32, CTP_F32, nullptr, &t) == CTP_OK);
        bigs.push_back(t);
    }
    wait_running(srv, bigs[0]);
    for (int i = 0; i < 4; ++i) {
        uint64_t t = 0;
        CHECK(ctp_server_submit(srv, &small, CTP_FORWARD, dummy_input, CTP_F32, CTP_F32, nullptr, &t) == CTP_OK);
        smalls.push_back(t);
    }
    for (uint64_t t : bigs)
        CHECK(ctp_server_wait(srv, t, 20 * 1000 * 1000, nullptr) == CTP_OK);
    for (uint64_t t : smalls)
        CHECK(ctp_server_wait(srv, t, 20 * 1000 * 1000, nullptr) == CTP_OK);
    ctp_request_info b1{}, b2{};
    CHECK(ctp_server_info(srv, bigs[1], &b1) == CTP_OK);
    CHECK(ctp_server_info(srv, bigs[2], &b2) == CTP_OK);
    CHECK(b1.slot == 0 && b2.slot == 0);                // long calls never take the express slot
    for (uint64_t t : smalls) {
        ctp_request_info si{};
        CHECK(ctp_server_info(srv, t, &si) == CTP_OK);
        CHECK(si.done_ns < b1.admit_ns || si.slot == 1);   // ran beside the first long call
        CHECK(si.done_ns < b2.admit_ns);
    }
    std::vector<uint64_t> all(bigs);
    all.insert(all.end(), smalls.begin(), smalls.end());
    release_all_and_drain(srv, all);
    CHECK(ctp_server_destroy(srv) == CTP_OK);
}

// With an express threshold, long calls run one at a time on the regular slots while short
// ones run beside them; launch_work splits each long call into launches of a quarter of it.
static void long_calls_one_at_a_time()
{
    ctp_plan big, small;
    big.nvox = 32 * 32 * 32; big.ncell = 20 * 40 * 40; big.us_per_item = 8000;
    small.nvox = 8 * 8 * 8; small.ncell = 4 * 10 * 10; small.us_per_item = 300;
    static char dummy_input[16];
    const double big_work = ctp::plan_work(&big);
    ctp_server *srv = make_server(256u << 20, 4, 1, 0, ctp::plan_work(&small), big_work / 4);
    const int launches0 = launches;
    std::vector<uint64_t> bigs, smalls;
    for (int i = 0; i < 4; ++i) {
        uint64_t t = 0;
        CHECK(ctp_server_submit(srv, &big, CTP_FORWARD, dummy_input, CTP_F32, CTP_F32, nullptr, &t) == CTP_OK);
        bigs.push_back(t);
    }
    wait_running(srv, bigs[0]);
    for (int i = 0; i < 6; ++i) {
        uint64_t t = 0;
        CHECK(ctp_server_submit(srv, &small, CTP_BACKWARD, dummy_input, CTP_F32, CTP_F32, nullptr, &t) == CTP_OK);
        smalls.push_back(t);
    }
    for (uint64_t t : bigs)
        CHECK(ctp_server_wait(srv, t, 20 * 1000 * 1000, nullptr) == CTP_OK);
    for (uint64_t t : smalls)
        CHECK(ctp_server_wait(srv, t, 20 * 1000 * 1000, nullptr) == CTP_OK);
    std::vector<ctp_request_info> bi(bigs.size());
    for (size_t i = 0; i < bigs.size(); ++i)
        CHECK(ctp_server_info(srv, bigs[i], &bi[i]) == CTP_OK);
    for (size_t i = 0; i < bi.size(); ++i)
        for (size_t j = i + 1; j < bi.size(); ++j)     // no two long calls overlap
            CHECK(bi[i].done_ns <= bi[j].admit_ns || bi[j].done_ns <= bi[i].admit_ns);
    int64_t last_admit = 0;
    for (const ctp_request_info &b : bi)
        last_admit = std::max(last_admit, b.admit_ns);
    for (uint64_t t : smalls) {
        ctp_request_info si{};
        CHECK(ctp_server_info(srv, t, &si) == CTP_OK);
        CHECK(si.done_ns < last_admit);                 // the short ones ran beside the long ones
    }
    // each long call in 4 launches (8 views, 2 per launch), each short one in 1
    CHECK(launches - launches0 == 4 * 4 + 6);
    std::vector<uint64_t> all(bigs);
    all.insert(all.end(), smalls.begin(), smalls.end());
    release_all_and_drain(srv, all);
    CHECK(ctp_server_destroy(srv) == CTP_OK);
}

int main()
{
    // the configuration of the GPU serving test, then tighter arenas and other slot counts
    for (unsigned seed = 1; seed <= 12; ++seed)
        burst(seed, 256u << 20, 2, 6, 4, 60);
    for (unsigned seed = 1; seed <= 6; ++seed) {
        burst(100 + seed, 200u << 20, 2, 6, 3, 60);
        burst(200 + seed, 256u << 20, 4, 8, 4, 60);
        burst(300 + seed, 64u << 20, 3, 4, 0, 200);
    }
    CHECK(bad_calls == 0);
    for (unsigned seed = 1; seed <= 4; ++seed)
        failure_injection(seed);
    cancellation();
    ordering();
    express_slot();
    long_calls_one_at_a_time();
    std::printf("ok\n");
    return 0;
}
