// sh_server.h -- continuous-batching server for projector requests.
//
// Clients register atoms (device point sets, a centre, a radial table) once, then
// submit requests "projectors of atom A up to lmax L".  A scheduler thread
//   1. admits pending requests in arrival order while their output fits in the
//      HBM budget (an arena carved from one device allocation),
//   2. packs every admitted, not yet launched request into one batch and launches
//      it on a free stream slot, so batches that arrive while others run overlap
//      on the device (up to n_slots batches in flight),
//   3. detects finished batches (events), stamps each request's latency (submit to
//      completion seen by the host) and, for auto-release requests, returns their
//      memory to the arena so deferred requests can be admitted.
// The scheduling core is device-agnostic; an Executor runs batches (HIP streams
// and one batched kernel per batch, or a simulation that computes nothing and is
// used to test scheduling on a machine without a GPU).
#pragma once

#include <stdint.h>

#include <chrono>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

struct sh_radial;

namespace shs {

using Clock = std::chrono::steady_clock;

// A radial handle also keeps, for each L <= kCompactLmax below its own lmax, a copy
// of its tables with only the first L + 1 channels: a projector build at lmax L
// then reads each knot's pairs from a row of L + 1 pairs instead of a row of all
// of them (fewer cache lines per lookup, a smaller table to cache).
constexpr int kCompactLmax = 5;

// The device table one atom uses: table `table` of a radial handle, in the
// precision of dtype (SH_F64: double pairs, SH_F32: float pairs), and its copies
// with fewer channels (compact[L]: L + 1 channels, null where the handle has none).
struct RadialRef {
    const void* tab;
    int lmax;  // channels - 1
    int n_r;
    double h, r_max;
    const void* compact[kCompactLmax + 1];
};

// Looks a table up in a radial handle (defined with the handles); SH_EINVAL for a
// table or dtype out of range.
int radial_table(sh_radial* radial, int table, int dtype, RadialRef* out);

// A registered atom: its grid points stay on the device for the server's life.
struct Atom {
    int dtype;           // SH_F64 or SH_F32 (points and outputs)
    int64_t n;           // number of points
    const void* points;  // device [n][3]
    double c[3];         // centre
    const void* tab;     // device (y, M) table of this atom's channels (double2 for FP64 atoms, float2
                         // for FP32 ones), may be null (simulation)
    int tab_lmax;        // channels - 1
    const void* tab_compact[kCompactLmax + 1];  // the same with L + 1 channels, or null
    int n_r;
    double h, r_max;
};

// One request of a batch, as the executor sees it.
struct Item {
    Atom atom;
    int lmax;
    void* out;  // device [F][n]
};

class Executor {
public:
    virtual ~Executor() = default;
    virtual int n_slots() const = 0;
    virtual int64_t max_items() const = 0;  // requests per batch
    virtual int64_t max_tiles() const = 0;    // tiles per batch
    virtual int64_t tile_points() const = 0;  // points per tile (the smallest, if they differ)
    virtual void* arena_base() = 0;
    // Queue a batch on a free slot; returns an SH_* status.
    virtual int launch(int slot, const std::vector<Item>& items) = 0;
    // 1: the slot's batch finished; 0: still running; negative: it failed.
    virtual int query(int slot) = 0;
    // Items of the slot's batch (indices into the vector launch() was given) whose
    // results are complete and were not reported before are appended to `done`;
    // returns what query() returns.  The default reports no item early: every item
    // completes with its batch.
    virtual int progress(int slot, std::vector<int>& done)
    {
        (void)done;
        return query(slot);
    }
};

// First-fit allocator over [0, capacity) with coalescing, 256-byte granularity.
class Arena {
public:
    explicit Arena(uint64_t capacity);
    bool alloc(uint64_t bytes, uint64_t* offset);
    void release(uint64_t offset, uint64_t bytes);
    uint64_t capacity() const { return cap_; }
    uint64_t in_use() const { return used_; }
    static uint64_t round(uint64_t bytes) { return (bytes + 255) & ~uint64_t(255); }

private:
    uint64_t cap_, used_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> size
};

enum ReqState { kPending = 0, kQueued = 1, kRunning = 2, kDone = 3, kFailed = 4, kReleased = 5 };

struct Request {
    int atom;
    int lmax;
    int flags;
    uint64_t bytes;
    uint64_t offset;
    int state;
    int error;
    int64_t refusals_at_submit;  // budget refusals counted before this request arrived
    Clock::time_point t_submit, t_done;
};

struct Stats {
    int64_t submitted, completed, failed, deferred, batches;
    int64_t points_done;
    uint64_t bytes_in_use, peak_bytes;
    double first_submit_s, last_done_s;  // seconds since server creation
    double scheduler_cpu_s;              // CPU time the scheduler thread has used
};

class Server {
public:
    Server(std::unique_ptr<Executor> ex, uint64_t budget, int64_t max_pending);
    ~Server();

    int add_atom(const Atom& a, int* id);
    int submit(int atom, int lmax, int flags, int64_t* ticket);
    int poll(int64_t ticket, int* state);
    int wait(int64_t ticket, double timeout_s, int* state);
    int result(int64_t ticket, void** ptr);
    int release(int64_t ticket);
    void stats(Stats* s);
    // Latencies (ms) of completed requests, in completion order.
    int64_t latencies(double* out, int64_t cap);
    // Block until nothing is pending, queued or running (or timeout).
    int drain(double timeout_s);

private:
    void loop();
    bool reap(std::unique_lock<std::mutex>& lk);
    bool admit_locked();
    void finish_locked(int slot, int status);
    void finish_req_locked(int64_t ticket, int status, Clock::time_point now);
    bool apply_locked();

    std::unique_ptr<Executor> ex_;
    Arena arena_;
    int64_t max_pending_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::atomic<bool> stop_{false};
    std::vector<Atom> atoms_;
    std::vector<Request> reqs_;
    std::deque<int64_t> pending_;
    std::vector<int64_t> queued_;
    std::vector<std::vector<int64_t>> slot_reqs_;
    std::vector<int> free_slots_;
    int busy_slots_ = 0;
    int64_t refusals_ = 0;  // admission attempts refused for lack of budget
    std::atomic<uint64_t> gen_{0};  // bumped by every submit, release and shutdown
    // how long an idle scheduler watches gen_ before it sleeps on cv_work_
    static constexpr std::chrono::microseconds kIdleSpin{200};
    // while batches run: poll their completion back to back for kBusySpin, then
    // with naps between polls that double from kNapMin up to kNapMax
    static constexpr std::chrono::microseconds kBusySpin{200};
    static constexpr std::chrono::microseconds kNapMin{20};
    static constexpr std::chrono::microseconds kNapMax{200};
    std::vector<int> busy_, done_;  // scratch of reap(): busy slots and their progress() results
    std::vector<std::vector<int>> early_;    // scratch of reap(): items reported complete per busy slot
    std::vector<std::vector<char>> finished_;  // per slot: which of its requests are already finished
    std::vector<double> lat_ms_;
    Stats st_{};
    Clock::time_point t0_;
    std::thread thr_;
};

std::unique_ptr<Executor> make_sim_executor(int n_slots, double bytes_per_s, int fail_every, double launch_s);
std::unique_ptr<Executor> make_hip_executor(uint64_t budget, int n_slots, int* status);

}  // namespace shs
