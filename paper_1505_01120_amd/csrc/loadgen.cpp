// Open-loop load generator for the serving path: replays a trace of tasks
// through the public C ABI (sparkcl_submit / sparkcl_poll) at scheduled
// arrival times, from native code, so that the client keeps up with arrival
// rates a Python loop cannot.  Latency is measured against the scheduled
// arrival, not the submit call, so a late submit (a full pending queue, a
// slow client) counts against the server, never hides from it.
//
// Built as its own library (libsparkcl_loadgen.so) on top of libsparkcl.so;
// it is a measurement tool, not part of the sparkcl API.
#include <chrono>
#include <cstdint>
#include <thread>
#include <vector>

#include "sparkcl.h"

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

} // namespace

extern "C" __attribute__((visibility("default"))) int
sparkcl_loadgen_run(sparkcl_ctx *ctx, const sparkcl_task *tasks, const int64_t *sched_ns,
                    uint64_t count, int64_t lead_ns, uint32_t stall_ms, int64_t *t0_ns,
                    int64_t *done_ns, int32_t *status, sparkcl_result *results)
{
    // tasks[i] is submitted at t0 + sched_ns[i] (sched_ns ascending, t0 = now +
    // lead_ns); done_ns[i] receives the server's completion stamp (steady
    // clock), status[i] the result status or the submit error, and, when
    // `results` is not NULL, results[i] the task's result as polled.  The
    // call fails with SPARKCL_ETIMEDOUT when nothing completes or gets
    // submitted for stall_ms while work is outstanding.
    if (!ctx || (count && (!tasks || !sched_ns || !done_ns || !status)) || !t0_ns)
        return SPARKCL_EINVAL;
    for (uint64_t i = 1; i < count; ++i)
        if (sched_ns[i] < sched_ns[i - 1])
            return SPARKCL_EINVAL;
    std::vector<uint64_t> ticket(count, 0);
    std::vector<uint64_t> open; // indices submitted and not yet collected
    open.reserve(4096);
    const int64_t t0 = now_ns() + lead_ns;
    *t0_ns = t0;
    uint64_t next = 0;
    size_t cursor = 0;
    int64_t last_progress = now_ns();
    constexpr size_t kPollsPerPass = 256;
    while (next < count || !open.empty()) {
        int64_t now = now_ns();
        bool progress = false;
        while (next < count && t0 + sched_ns[next] <= now) {
            uint64_t tk = 0;
            const int rc = sparkcl_submit(ctx, &tasks[next], &tk);
            if (rc == SPARKCL_EAGAIN)
                break; // pending queue full: retry on the next pass
            progress = true;
            if (rc != SPARKCL_OK) {
                done_ns[next] = now;
                status[next] = rc;
            } else {
                ticket[next] = tk;
                open.push_back(next);
            }
            ++next;
        }
        // poll a bounded round-robin window of the open tasks
        const size_t polls = open.size() < kPollsPerPass ? open.size() : kPollsPerPass;
        for (size_t k = 0; k < polls && !open.empty(); ++k) {
            if (cursor >= open.size())
                cursor = 0;
            const uint64_t j = open[cursor];
            sparkcl_result r;
            const int rc = sparkcl_poll(ctx, ticket[j], &r);
            if (rc == SPARKCL_EAGAIN) {
                ++cursor;
                continue;
            }
            progress = true;
            done_ns[j] = rc == SPARKCL_OK ? (int64_t)r.t_done_ns : now_ns();
            status[j] = rc == SPARKCL_OK ? r.status : rc;
            if (results && rc == SPARKCL_OK)
                results[j] = r;
            open[cursor] = open.back();
            open.pop_back();
        }
        now = now_ns();
        if (progress) {
            last_progress = now;
        } else if (!open.empty() || next < count) {
            if (next < count && t0 + sched_ns[next] > now && open.empty()) {
                last_progress = now; // idle until the next arrival
                if (t0 + sched_ns[next] - now > 200000)
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
            } else if (now - last_progress > (int64_t)stall_ms * 1000000) {
                return SPARKCL_ETIMEDOUT;
            } else {
                // nothing completed: back off briefly rather than contend for
                // the server's lock with back-to-back polls
                int64_t until = now + 2000;
                if (next < count && t0 + sched_ns[next] < until)
                    until = t0 + sched_ns[next]; // never delay an arrival
                while (now_ns() < until) {
                }
            }
        }
    }
    return SPARKCL_OK;
}
