// Serving loop: continuous batching of partition tasks onto one GPU.
//
// Callers submit tasks at any time (sparkcl_submit stamps the arrival).  A
// host thread admits them in FIFO order as ring slots, HBM budget and tile-map
// room free up (admission.h), writes each admitted task's descriptor into a
// ring of host-coherent pinned memory and release-stores the ring's tail.  The
// resident executor (k_serve: one dispatcher block plus worker blocks) picks
// the new descriptors up without any launch, spreads each task's tiles over
// the workers while earlier tasks are still running, and each task's last
// tile writes the result and a completion word into host memory.  The thread
// reaps completions, frees the task's budget, slot and partials, and keeps the
// result until sparkcl_poll collects it.  An idle executor exits on its own
// and is relaunched when work arrives.
//
// A task whose inputs live in host memory (SPARKCL_TASK_HOST_INPUT, pinned
// arrays) is admitted against the budget with its staging block, its inputs
// are copied into the arena on the server's copy streams while earlier tasks
// run, and it takes a ring slot only once the copy is done, so the tasks
// admitted after it are never held up by its transfer.  Its latency includes
// the PCIe time, the main cost of offload that the paper names (sec. 3,
// design issue 1).
//
// The same machinery also runs the baseline the paper's workers use: one
// kernel launch per task (SPARKCL_FLAG_SERVE_PER_TASK), spread over a pool of
// streams, with the same admission, descriptors and completion words.
//
// Where the paper serialises accelerator tasks per worker to avoid contention
// (`--cores 1`, sec. 3.1.5), this loop shares the GPU between tasks and keeps
// them within the memory budget instead; memory management and data layout
// are the framework's job (sec. 3, issue 3).
#include "serve.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <unordered_set>

namespace sparkcl {

namespace {

constexpr uint32_t kTileCap = 1u << 20;     // tile map entries
constexpr uint32_t kPoolStreams = 4;        // per-task launch baseline
constexpr uint64_t kMaxPending = 1u << 22;  // queued tasks before EAGAIN
constexpr uint64_t kSpinNs = 2000000;       // busy-poll this long after activity

uint64_t task_bytes(const sparkcl_task &t, uint32_t ntiles)
{
    uint64_t in = 0;
    if (t.kernel_id == SPARKCL_POLY)
        in = 4 * t.n;
    else if (t.kernel_id == SPARKCL_FMUL)
        in = 8 * t.n;
    const uint64_t out = (t.out && t.kernel_id != SPARKCL_MC_PI) ? 4 * t.n : 0;
    return in + out + sizeof(Partial) * (uint64_t)ntiles;
}

// Arena bytes that stage a host-input task: each input at its host address
// modulo 16 (so the kernel cuts the same quads and tiles, and the result is
// bit-identical to the same data in device memory), in 256-byte units.
uint64_t staging_stride(const sparkcl_task &t)
{
    return (4 * t.n + 16 + 255) / 256 * 256;
}

uint64_t staging_bytes(const sparkcl_task &t)
{
    return staging_stride(t) * (t.kernel_id == SPARKCL_FMUL ? 2 : 1);
}

// Whether p lies in page-locked host memory (hipHostMalloc or torch's
// pin_memory), which an asynchronous copy needs: a copy from pageable memory
// would stall the serving thread, and every task behind it.
bool host_pinned(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError(); // an unknown pointer: clear the error it left
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

sparkcl_result failed_result(int code)
{
    sparkcl_result r;
    std::memset(&r, 0, sizeof(r));
    r.max = -__builtin_huge_valf();
    r.status = code;
    return r;
}

} // namespace

Server::Server(sparkcl_ctx *ctx)
    : ctx_(ctx), adm_(ctx->config.budget_bytes, ctx->config.ring_capacity, kTileCap)
{
}

int Server::create(sparkcl_ctx *ctx, std::unique_ptr<Server> *out)
{
    std::unique_ptr<Server> s(new Server(ctx));
    int rc = s->init();
    if (rc != SPARKCL_OK)
        return rc;
    *out = std::move(s);
    return SPARKCL_OK;
}

void Server::set_tuning(const sparkcl_tuning &t)
{
    std::lock_guard<std::mutex> g(mu_);
    tuning_ = t;
}

int Server::init()
{
    tuning_ = ctx_->tuning;
    cap_ = ctx_->config.ring_capacity;
    tile_cap_ = kTileCap;
    per_task_launch_ = (ctx_->config.flags & SPARKCL_FLAG_SERVE_PER_TASK) != 0;
    workers_ = 2u * (uint32_t)ctx_->cus;

    const size_t bytes = sizeof(ServeHost) + (size_t)cap_ * sizeof(TaskDev) +
                         (size_t)cap_ * sizeof(sparkcl_result) + (size_t)cap_ * sizeof(uint64_t);
    SPARKCL_HIP(hipHostMalloc((void **)&pinned_, bytes,
                              hipHostMallocCoherent | hipHostMallocMapped));
    std::memset(pinned_, 0, bytes);
    char *p = pinned_;
    host_ = reinterpret_cast<ServeHost *>(p);
    p += sizeof(ServeHost);
    ring_ = reinterpret_cast<TaskDev *>(p);
    p += (size_t)cap_ * sizeof(TaskDev);
    results_ = reinterpret_cast<sparkcl_result *>(p);
    p += (size_t)cap_ * sizeof(sparkcl_result);
    done_ = reinterpret_cast<uint64_t *>(p);

    auto take = [&](uint64_t n, void **out) -> int {
        const uint64_t off = ctx_->arena.alloc(n);
        if (off == Arena::kFail)
            return fail(SPARKCL_ENOMEM, "arena too small for the serving tables");
        blocks_.push_back(off);
        *out = ctx_->dev(off);
        return SPARKCL_OK;
    };
    int rc;
    void *m;
    if ((rc = take(sizeof(ServeDev), &m)) != SPARKCL_OK)
        return rc;
    dev_ = static_cast<ServeDev *>(m);
    if ((rc = take((uint64_t)cap_ * sizeof(TaskDev), &m)) != SPARKCL_OK)
        return rc;
    table_ = static_cast<TaskDev *>(m);
    if ((rc = take((uint64_t)tile_cap_ * sizeof(uint32_t), &m)) != SPARKCL_OK)
        return rc;
    tilemap_ = static_cast<uint32_t *>(m);
    if ((rc = take((uint64_t)cap_ * sizeof(TaskSync), &m)) != SPARKCL_OK)
        return rc;
    sync_ = static_cast<TaskSync *>(m);

    SPARKCL_HIP(hipStreamCreateWithFlags(&exec_stream_, hipStreamNonBlocking));
    for (hipStream_t &c : copy_stream_)
        SPARKCL_HIP(hipStreamCreateWithFlags(&c, hipStreamNonBlocking));
    if ((rc = launch_zero(dev_, sizeof(ServeDev), exec_stream_)) != SPARKCL_OK ||
        (rc = launch_zero(sync_, (uint64_t)cap_ * sizeof(TaskSync), exec_stream_)) != SPARKCL_OK)
        return fail(rc, "clearing the serving tables failed");
    SPARKCL_HIP(hipStreamSynchronize(exec_stream_));
    if (per_task_launch_) {
        pool_.resize(kPoolStreams);
        for (auto &s : pool_)
            SPARKCL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    }
    return SPARKCL_OK;
}

Server::~Server()
{
    shutdown();
}

int Server::start_thread_locked()
{
    if (started_)
        return SPARKCL_OK;
    started_ = true;
    thread_ = std::thread([this] { loop(); });
    return SPARKCL_OK;
}

int Server::submit(const sparkcl_task &task, uint64_t *ticket)
{
    uint32_t variant = 0;
    int rc = check_task(task, &variant);
    if (rc != SPARKCL_OK)
        return rc;
    const bool host = (task.flags & SPARKCL_TASK_HOST_INPUT) != 0;
    if (host && task.n > 0 &&
        (!host_pinned(task.in0) || (task.kernel_id == SPARKCL_FMUL && !host_pinned(task.in1))))
        return fail(SPARKCL_EINVAL, "served host-input arrays must be in pinned host memory");
    if (declined(ctx_, task))
        return fail(SPARKCL_EDECLINED, "offload cost " + std::to_string(offload_cost(task)) +
                                           " bytes is below the offload threshold");
    std::lock_guard<std::mutex> g(mu_);
    const uint32_t tile = tile_for(tuning_, TM_SERVE, task.kernel_id, task.n);
    const uint64_t nt64 = std::max<uint64_t>(1, (task.n + tile - 1) / tile);
    if (nt64 > tile_cap_)
        return fail(SPARKCL_ETOOBIG, "task needs more tiles than the tile map holds");
    const uint32_t ntiles = (uint32_t)nt64;
    // a host-input task is charged its staging block (the library's copy of
    // its inputs) and its partials
    const uint64_t bytes = host ? staging_bytes(task) + sizeof(Partial) * (uint64_t)ntiles
                                : task_bytes(task, ntiles);
    if (!adm_.fits_at_all(bytes, ntiles))
        return fail(SPARKCL_ETOOBIG, "task needs " + std::to_string(bytes) +
                                         " bytes, budget is " + std::to_string(adm_.budget()));
    // its staging block must fit the arena too, or it could never be admitted
    if (host && staging_bytes(task) + sizeof(Partial) * (uint64_t)ntiles > ctx_->arena.size())
        return fail(SPARKCL_ETOOBIG, "host-input task's staging exceeds the arena");
    if (quit_ || poisoned_)
        return fail(SPARKCL_ESTOPPED, poisoned_ ? "serving executor could not be stopped"
                                                : "serving is shutting down");
    if (adm_.pending() >= kMaxPending)
        return fail(SPARKCL_EAGAIN, "pending queue full");
    Pending p;
    p.ticket = next_ticket_++;
    p.bytes = bytes;
    p.ntiles = ntiles;
    p.t_arrive = host_ns();
    p.staged = host && task.n > 0;
    adm_.push(p);
    Waiting w;
    w.task = task;
    w.ntiles = ntiles;
    w.tile = tile;
    w.unroll = kernel_unroll(tuning_, task.kernel_id);
    w.variant = variant;
    waiting_[p.ticket] = w;
    ++submitted_;
    *ticket = p.ticket;
    start_thread_locked();
    cv_work_.notify_one();
    return SPARKCL_OK;
}

int Server::poll(uint64_t ticket, sparkcl_result *result)
{
    std::lock_guard<std::mutex> g(mu_);
    auto it = done_map_.find(ticket);
    if (it != done_map_.end()) {
        *result = it->second;
        done_map_.erase(it);
        return SPARKCL_OK;
    }
    if (waiting_.count(ticket))
        return SPARKCL_EAGAIN;
    return fail(SPARKCL_ENOTFOUND, "unknown or already collected ticket");
}

void Server::stats(sparkcl_serve_stats *s)
{
    std::lock_guard<std::mutex> g(mu_);
    s->submitted = submitted_;
    s->admitted = admitted_;
    s->completed = completed_;
    s->failed = failed_;
    s->pending = adm_.pending();
    s->in_flight = adm_.in_flight();
    s->budget_in_use = adm_.in_use();
    s->budget_peak = adm_.peak();
    s->admission_waits = waits_;
    s->executor_launches = launches_;
}

int Server::drain(uint32_t timeout_ms)
{
    std::unique_lock<std::mutex> lk(mu_);
    const bool ok = cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                                      [this] { return waiting_.empty(); });
    return ok ? SPARKCL_OK : fail(SPARKCL_ETIMEDOUT, "drain timed out");
}

// Admit work while it fits.  First, staged tasks whose inputs are on the
// device take ring slots, in the order they were admitted.  Then queued tasks
// are admitted in FIFO order while the head fits: a device-input task takes
// its slot at once (appended to the in-flight list and copied to *out), a
// host-input one gets its staging block and copy event and goes to the
// staging list (and *to_copy) until its copy is done.
void Server::admit_some(std::vector<Flight> *out, std::vector<Flight> *to_copy)
{
    std::lock_guard<std::mutex> g(mu_);
    while (!staging_.empty() && staging_.front().ready && adm_.slot_free()) {
        Flight f = staging_.front();
        staging_.pop_front();
        adm_.take_slot(f.a);
        flight_.push_back(f);
        out->push_back(f);
    }
    for (;;) {
        const AdmitBlock b = adm_.head_block();
        if (b == AdmitBlock::EMPTY)
            break;
        if (b != AdmitBlock::NONE) {
            ++waits_;
            break;
        }
        Admitted a = adm_.admit_head();
        const Waiting &w = waiting_[a.p.ticket];
        const uint64_t off = ctx_->arena.alloc(sizeof(Partial) * (uint64_t)w.ntiles);
        if (off == Arena::kFail) {
            adm_.unadmit(a);
            ++waits_;
            break;
        }
        Flight f;
        f.a = a;
        f.task = w.task;
        f.variant = w.variant;
        f.tile = w.tile;
        f.unroll = w.unroll;
        f.part_off = off;
        f.t_admit = host_ns();
        f.dx = w.task.in0;
        f.dy = w.task.in1;
        if (a.p.staged) {
            const uint64_t so = ctx_->arena.alloc(staging_bytes(w.task));
            if (so == Arena::kFail) {
                ctx_->arena.release(off);
                adm_.unadmit(a);
                ++waits_;
                break;
            }
            if (free_events_.empty()) {
                hipEvent_t e = nullptr;
                if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                    ctx_->arena.release(so);
                    ctx_->arena.release(off);
                    adm_.unadmit(a);
                    ++waits_;
                    break;
                }
                events_.push_back(e);
                free_events_.push_back((int)events_.size() - 1);
            }
            f.ev = free_events_.back();
            free_events_.pop_back();
            f.cs = copy_next_++ & 1u;
            f.stage_off = so;
            char *base = static_cast<char *>(ctx_->dev(so));
            f.dx = reinterpret_cast<const float *>(base + ((uintptr_t)w.task.in0 & 15u));
            if (w.task.kernel_id == SPARKCL_FMUL)
                f.dy = reinterpret_cast<const float *>(base + staging_stride(w.task) +
                                                       ((uintptr_t)w.task.in1 & 15u));
            staging_.push_back(f);
            to_copy->push_back(f);
        } else {
            flight_.push_back(f);
            out->push_back(f);
        }
        ++admitted_;
    }
}

// Queue the host-to-device copies of newly staged tasks, each task's inputs
// on one of the two copy streams in turn, followed by its event.
int Server::start_copies(const std::vector<Flight> &fl)
{
    for (const Flight &f : fl) {
        const hipStream_t s = copy_stream_[f.cs];
        SPARKCL_HIP(hipMemcpyAsync(const_cast<float *>(f.dx), f.task.in0, 4 * f.task.n,
                                   hipMemcpyHostToDevice, s));
        if (f.task.kernel_id == SPARKCL_FMUL)
            SPARKCL_HIP(hipMemcpyAsync(const_cast<float *>(f.dy), f.task.in1, 4 * f.task.n,
                                       hipMemcpyHostToDevice, s));
        SPARKCL_HIP(hipEventRecord(events_[f.ev], s));
    }
    return SPARKCL_OK;
}

// Mark staged tasks whose copies are done.  The copies on one stream finish
// in the order they were queued, so each stream's tasks are queried from the
// oldest until one is still copying.
void Server::poll_staging()
{
    std::vector<std::pair<int, uint32_t>> cand; // (event, copy stream), oldest first
    {
        std::lock_guard<std::mutex> g(mu_);
        for (const Flight &f : staging_)
            if (!f.ready)
                cand.emplace_back(f.ev, f.cs);
    }
    if (cand.empty())
        return;
    std::unordered_set<int> done;
    bool busy[2] = {false, false};
    for (const auto &c : cand) {
        if (busy[c.second])
            continue;
        if (hipEventQuery(events_[c.first]) == hipSuccess) {
            done.insert(c.first);
        } else {
            (void)hipGetLastError(); // not ready yet: clear the status it left
            busy[c.second] = true;
            if (busy[0] && busy[1])
                break;
        }
    }
    if (done.empty())
        return;
    std::lock_guard<std::mutex> g(mu_);
    for (Flight &f : staging_)
        if (!f.ready && done.count(f.ev))
            f.ready = true;
}

// A finished task's arena blocks and copy event go back (caller holds mu_).
void Server::release_flight(const Flight &f)
{
    ctx_->arena.release(f.part_off);
    if (f.stage_off != Arena::kFail)
        ctx_->arena.release(f.stage_off);
    if (f.ev >= 0)
        free_events_.push_back(f.ev);
}

// Fail every staged task that has no ring slot yet, once its copies are done
// (they write its staging block).  keep_memory: leave its blocks reserved.
void Server::fail_staging(int code, bool keep_memory)
{
    std::deque<Flight> st;
    {
        std::lock_guard<std::mutex> g(mu_);
        st.swap(staging_);
    }
    for (const Flight &f : st)
        (void)hipEventSynchronize(events_[f.ev]);
    std::lock_guard<std::mutex> g(mu_);
    for (const Flight &f : st) {
        sparkcl_result r = failed_result(code);
        r.n = f.task.n;
        r.t_arrive_ns = f.a.p.t_arrive;
        r.t_admit_ns = f.t_admit;
        r.t_done_ns = host_ns();
        if (!keep_memory) {
            release_flight(f);
            adm_.complete(f.a);
        }
        done_map_[f.a.p.ticket] = r;
        waiting_.erase(f.a.p.ticket);
        ++failed_;
    }
    cv_done_.notify_all();
}

// Write the descriptors of newly admitted tasks and hand them to the GPU.
int Server::publish(const std::vector<Flight> &fl)
{
    if (fl.empty())
        return SPARKCL_OK;
    for (const Flight &f : fl) {
        const sparkcl_task &t = f.task;
        TaskDev d;
        std::memset(&d, 0, sizeof(d));
        d.kid = (uint16_t)t.kernel_id;
        d.unroll = (uint16_t)f.unroll;
        d.ops = t.reduce_ops;
        d.n = t.n;
        d.in0 = f.dx; // a host-input task reads its staged copies
        d.in1 = f.dy;
        d.out = t.out;
        d.seed = t.seed;
        d.pid = t.partition_id;
        d.variant = f.variant;
        std::memcpy(d.coef, t.coef, sizeof(d.coef));
        d.c = t.c;
        d.tile_elems = f.tile;
        d.ntiles = f.a.p.ntiles;
        d.index = f.a.slot;
        d.partials = static_cast<Partial *>(ctx_->dev(f.part_off));
        d.seq = f.a.seq;
        d.tile_first = tiles_pub_host_;
        tiles_pub_host_ += d.ntiles;
        std::memcpy(ring_ + f.a.slot, &d, sizeof(d));
    }
    if (per_task_launch_) {
        LaunchOut L{};
        L.sync = sync_;
        L.results = results_;
        L.done = done_;
        L.ntasks = 0;
        L.ns_per_tick = ctx_->ns_per_tick;
        const uint32_t cap = (uint32_t)ctx_->cus * (uint32_t)ctx_->occ_batch;
        for (const Flight &f : fl) {
            hipStream_t s = pool_[pool_next_++ % pool_.size()];
            const uint32_t slot = f.a.slot;
            SPARKCL_HIP(hipMemcpyAsync(table_ + slot, ring_ + slot, sizeof(TaskDev),
                                       hipMemcpyHostToDevice, s));
            const uint32_t nt = f.a.p.ntiles;
            int rc = launch_task(table_ + slot, nt, std::min(nt, cap), L, s);
            if (rc != SPARKCL_OK)
                return fail(rc, "per-task launch failed");
        }
        std::lock_guard<std::mutex> g(mu_);
        launches_ += fl.size();
        return SPARKCL_OK;
    }
    __atomic_store_n(&host_->tail, fl.back().a.seq + 1, __ATOMIC_RELEASE);
    return SPARKCL_OK;
}

bool Server::executor_running()
{
    if (!exec_launched_)
        return false;
    if (hipStreamQuery(exec_stream_) == hipSuccess)
        exec_launched_ = false;
    return exec_launched_;
}

int Server::launch_executor()
{
    ServeArgs a{};
    a.host = host_;
    a.ring = ring_;
    a.dev = dev_;
    a.table = table_;
    a.tilemap = tilemap_;
    a.out.sync = sync_;
    a.out.results = results_;
    a.out.done = done_;
    a.out.ntasks = 0;
    a.out.ns_per_tick = ctx_->ns_per_tick;
    a.cap = cap_;
    a.tile_cap = tile_cap_;
    a.idle_ticks = (uint64_t)ctx_->config.idle_exit_ms * 1000000ull / ctx_->ns_per_tick;
    const int rc = launch_serve(a, workers_, exec_stream_);
    if (rc != SPARKCL_OK)
        return fail(rc, "resident executor launch failed");
    exec_launched_ = true;
    std::lock_guard<std::mutex> g(mu_);
    ++launches_;
    return SPARKCL_OK;
}

int Server::stop_executor(uint32_t timeout_ms, bool abort)
{
    int rc = SPARKCL_OK;
    const uint64_t t0 = host_ns();
    auto wait_stream = [&](hipStream_t s) {
        while (hipStreamQuery(s) == hipErrorNotReady) {
            if (host_ns() - t0 > (uint64_t)timeout_ms * 1000000ull) {
                rc = fail(SPARKCL_ETIMEDOUT, "executor did not stop");
                return;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
    };
    __atomic_store_n(&host_->stop, abort ? 2ull : 1ull, __ATOMIC_RELEASE);
    wait_stream(exec_stream_);
    for (hipStream_t s : pool_)
        wait_stream(s);
    if (rc == SPARKCL_OK) {
        __atomic_store_n(&host_->stop, 0ull, __ATOMIC_RELEASE);
        exec_launched_ = false;
    }
    return rc;
}

// Completes every in-flight task whose completion word is set.
bool Server::reap()
{
    bool any = false;
    std::lock_guard<std::mutex> g(mu_);
    for (size_t i = 0; i < flight_.size();) {
        Flight &f = flight_[i];
        const uint64_t d = __atomic_load_n(done_ + f.a.slot, __ATOMIC_ACQUIRE);
        if (d != f.a.seq + 1) {
            ++i;
            continue;
        }
        sparkcl_result r = results_[f.a.slot];
        r.t_arrive_ns = f.a.p.t_arrive;
        r.t_admit_ns = f.t_admit;
        r.t_done_ns = host_ns();
        release_flight(f);
        adm_.complete(f.a);
        done_map_[f.a.p.ticket] = r;
        waiting_.erase(f.a.p.ticket);
        ++completed_;
        flight_[i] = flight_.back();
        flight_.pop_back();
        any = true;
    }
    if (any)
        cv_done_.notify_all();
    return any;
}

void Server::fail_in_flight(int code)
{
    fail_staging(code, false);
    std::lock_guard<std::mutex> g(mu_);
    for (Flight &f : flight_) {
        sparkcl_result r = failed_result(code);
        r.n = f.task.n;
        r.t_arrive_ns = f.a.p.t_arrive;
        r.t_admit_ns = f.t_admit;
        r.t_done_ns = host_ns();
        release_flight(f);
        adm_.complete(f.a);
        done_map_[f.a.p.ticket] = r;
        waiting_.erase(f.a.p.ticket);
        ++failed_;
    }
    flight_.clear();
    cv_done_.notify_all();
}

// After a stop: bring the device control block in line with the host so the
// next launch starts from a clean state (nothing claimable, tickets cleared).
int Server::reset_device_state()
{
    ServeDev d;
    std::memset(&d, 0, sizeof(d));
    d.taken = __atomic_load_n(&host_->tail, __ATOMIC_ACQUIRE);
    d.tiles_pub = tiles_pub_host_; // stop bit clear
    d.claim = tiles_pub_host_;
    SPARKCL_HIP(hipMemcpyAsync(dev_, &d, sizeof(d), hipMemcpyHostToDevice, exec_stream_));
    int rc = launch_zero(sync_, (uint64_t)cap_ * sizeof(TaskSync), exec_stream_);
    if (rc != SPARKCL_OK)
        return fail(rc, "clearing serving tickets failed");
    SPARKCL_HIP(hipStreamSynchronize(exec_stream_));
    return SPARKCL_OK;
}

void Server::loop()
{
    (void)hipSetDevice(ctx_->device);
    const uint64_t watchdog_ns = (uint64_t)ctx_->config.watchdog_ms * 1000000ull;
    uint64_t last_activity = host_ns();
    uint64_t last_exec_check = 0;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu_);
            if (quit_)
                break;
            if (flight_.empty() && staging_.empty() && adm_.pending() == 0 &&
                host_ns() - last_activity > kSpinNs) {
                cv_work_.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        poll_staging();
        std::vector<Flight> adm, to_copy;
        admit_some(&adm, &to_copy);
        bool progress = !adm.empty() || !to_copy.empty();
        if (start_copies(to_copy) != SPARKCL_OK || publish(adm) != SPARKCL_OK) {
            fail_in_flight(SPARKCL_EHIP);
            continue;
        }
        bool have_flight;
        {
            std::lock_guard<std::mutex> g(mu_);
            have_flight = !flight_.empty();
        }
        if (have_flight && !per_task_launch_) {
            const uint64_t now = host_ns();
            if (!adm.empty() || now - last_exec_check > 50000) {
                last_exec_check = now;
                if (!executor_running() && launch_executor() != SPARKCL_OK)
                    fail_in_flight(SPARKCL_EHIP);
            }
        }
        if (reap())
            progress = true;
        // Watchdog: a task stuck past the limit fails every in-flight task
        // after the executor has been stopped and the device state reset.
        uint64_t oldest = ~0ull;
        {
            std::lock_guard<std::mutex> g(mu_);
            for (const Flight &f : flight_)
                oldest = std::min(oldest, f.t_admit);
        }
        if (oldest != ~0ull && host_ns() - oldest > watchdog_ns) {
            if (stop_executor(2000, true) == SPARKCL_OK) {
                reap();
                fail_in_flight(SPARKCL_ETIMEDOUT);
                reset_device_state();
            } else {
                poison(SPARKCL_ETIMEDOUT);
                break;
            }
        }
        if (progress)
            last_activity = host_ns();
        else
            std::this_thread::yield();
    }
    // Shutdown: staged tasks without a slot fail; let in-flight work finish
    // (bounded), then stop the executor.
    if (!poisoned_)
        fail_staging(SPARKCL_ESTOPPED, false);
    const uint64_t t0 = host_ns();
    for (;;) {
        reap();
        bool empty;
        {
            std::lock_guard<std::mutex> g(mu_);
            empty = flight_.empty();
        }
        if (empty || host_ns() - t0 > 10000000000ull)
            break;
        if (!per_task_launch_ && !executor_running())
            launch_executor();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    if (poisoned_)
        return;
    const int rc = stop_executor(10000, false);
    reap();
    if (rc == SPARKCL_OK)
        fail_in_flight(SPARKCL_ESTOPPED);
    else
        poison(SPARKCL_ETIMEDOUT);
}

// The executor did not stop in time: fail every in-flight task but keep its
// partials and slot reserved, and refuse further work.
void Server::poison(int code)
{
    fail_staging(code, true);
    std::lock_guard<std::mutex> g(mu_);
    poisoned_ = true;
    for (Flight &f : flight_) {
        sparkcl_result r = failed_result(code);
        r.n = f.task.n;
        r.t_arrive_ns = f.a.p.t_arrive;
        r.t_admit_ns = f.t_admit;
        r.t_done_ns = host_ns();
        done_map_[f.a.p.ticket] = r;
        waiting_.erase(f.a.p.ticket);
        ++failed_;
    }
    flight_.clear();
    cv_done_.notify_all();
}

int Server::shutdown()
{
    {
        std::lock_guard<std::mutex> g(mu_);
        if (quit_ && !thread_.joinable() && !pinned_)
            return SPARKCL_OK;
        quit_ = true;
        // tasks never admitted fail with ESTOPPED
        for (const Pending &p : adm_.take_queue()) {
            sparkcl_result r = failed_result(SPARKCL_ESTOPPED);
            r.t_arrive_ns = p.t_arrive;
            done_map_[p.ticket] = r;
            waiting_.erase(p.ticket);
            ++failed_;
        }
    }
    cv_work_.notify_all();
    if (thread_.joinable())
        thread_.join();
    const int rc = poisoned_ ? SPARKCL_ETIMEDOUT : stop_executor(10000, false);
    if (rc == SPARKCL_OK) {
        for (hipStream_t s : pool_)
            (void)hipStreamDestroy(s);
        pool_.clear();
        if (exec_stream_)
            (void)hipStreamDestroy(exec_stream_);
        exec_stream_ = nullptr;
        for (hipStream_t &c : copy_stream_) {
            if (c) {
                (void)hipStreamSynchronize(c);
                (void)hipStreamDestroy(c);
            }
            c = nullptr;
        }
        for (hipEvent_t e : events_)
            (void)hipEventDestroy(e);
        events_.clear();
        free_events_.clear();
        for (uint64_t off : blocks_)
            ctx_->arena.release(off);
        blocks_.clear();
        if (pinned_)
            (void)hipHostFree(pinned_);
        pinned_ = nullptr;
    }
    // On a timeout the pinned memory is left allocated: a kernel may still
    // be reading it.
    cv_done_.notify_all();
    return rc;
}

} // namespace sparkcl
