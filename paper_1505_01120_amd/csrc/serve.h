// Serving loop of the SparkCL hot path: continuous batching of partition tasks
// onto one GPU (see serve.cpp).
#pragma once

#include <atomic>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.h"
#include "runtime.h"

namespace sparkcl {

class Server {
  public:
    static int create(sparkcl_ctx *ctx, std::unique_ptr<Server> *out);
    ~Server();

    int submit(const sparkcl_task &task, uint64_t *ticket);
    int poll(uint64_t ticket, sparkcl_result *result);
    void stats(sparkcl_serve_stats *s);
    int drain(uint32_t timeout_ms);
    int shutdown();
    // The serving tile sizes come from this copy of the tuning table, taken
    // under the server's own lock: a table change (sparkcl_set_tuning, the
    // end of sparkcl_autotune) applies to tasks submitted after it, and a
    // task keeps the tile chosen at submit until it completes.
    void set_tuning(const sparkcl_tuning &t);

  private:
    explicit Server(sparkcl_ctx *ctx);
    int init();
    void loop();
    int start_thread_locked();
    // serving-thread helpers (called without mu_ held unless noted)
    struct Flight;
    void admit_some(std::vector<Flight> *out, std::vector<Flight> *to_copy);
    int start_copies(const std::vector<Flight> &fl);
    void poll_staging();
    void release_flight(const Flight &f);
    void fail_staging(int code, bool keep_memory);
    int publish(const std::vector<Flight> &fl);
    bool reap();
    bool executor_running();
    int launch_executor();
    // abort: leave without running further tiles (watchdog); otherwise the
    // executor drains the tiles already published before it exits
    int stop_executor(uint32_t timeout_ms, bool abort);
    void fail_in_flight(int code);
    void poison(int code);
    int reset_device_state();

    struct Flight {
        Admitted a;
        sparkcl_task task;
        uint32_t variant = 0;
        uint32_t tile = 0;     // tile size fixed at submit
        uint32_t unroll = 4;   // loads in flight per thread, fixed at submit
        uint64_t part_off = 0; // arena block for the partials
        uint64_t t_admit = 0;
        // host-input task: its staging block in the arena, the device copies
        // of its inputs there, and the event that marks the copies done
        uint64_t stage_off = Arena::kFail;
        const float *dx = nullptr, *dy = nullptr;
        int ev = -1;
        uint32_t cs = 0; // copy stream
        bool ready = false;
    };
    struct Waiting {
        sparkcl_task task;
        uint32_t ntiles = 0, tile = 0, variant = 0, unroll = 4;
    };

    sparkcl_ctx *ctx_;
    bool per_task_launch_ = false;
    uint32_t cap_ = 0, tile_cap_ = 0;
    uint32_t workers_ = 0;

    // host-coherent (pinned) memory shared with the device
    char *pinned_ = nullptr;
    ServeHost *host_ = nullptr;
    TaskDev *ring_ = nullptr;
    sparkcl_result *results_ = nullptr;
    uint64_t *done_ = nullptr;
    // device memory (arena)
    std::vector<uint64_t> blocks_;
    ServeDev *dev_ = nullptr;
    TaskDev *table_ = nullptr;
    uint32_t *tilemap_ = nullptr;
    TaskSync *sync_ = nullptr;

    hipStream_t exec_stream_ = nullptr;
    hipStream_t copy_stream_[2] = {nullptr, nullptr}; // host-input staging copies
    uint32_t copy_next_ = 0;
    std::vector<hipEvent_t> events_;  // copy-done events, by index
    std::vector<int> free_events_;
    std::vector<hipStream_t> pool_; // per-task launch mode
    uint32_t pool_next_ = 0;
    bool exec_launched_ = false;
    uint64_t tiles_pub_host_ = 0; // tiles handed out so far (global index)

    std::mutex mu_; // queue, tables, counters below, tuning_
    sparkcl_tuning tuning_{};
    std::condition_variable cv_work_, cv_done_;
    Admission adm_;
    std::unordered_map<uint64_t, Waiting> waiting_;     // ticket -> task (queued)
    std::unordered_map<uint64_t, sparkcl_result> done_map_;
    std::vector<Flight> flight_; // admitted, not complete (serving thread)
    // admitted host-input tasks whose inputs are being copied to the device,
    // in admission order; they move to flight_ when they take a ring slot
    std::deque<Flight> staging_;
    uint64_t next_ticket_ = 1;
    uint64_t submitted_ = 0, admitted_ = 0, completed_ = 0, failed_ = 0, waits_ = 0;
    uint64_t launches_ = 0;
    bool quit_ = false, started_ = false;
    // set when the executor could not be stopped: in-flight memory stays
    // reserved (the GPU may still write it) and no new work is accepted
    bool poisoned_ = false;
    std::thread thread_;
};

} // namespace sparkcl
