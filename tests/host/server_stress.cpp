// server_stress.cpp -- drives the projector server's scheduler and C ABI from
// several threads with the simulated executor, for the sanitizer builds (thread;
// address + undefined behaviour).  Built with a plain C++ compiler from
// sh_server.cpp and sh_server_api.cpp; the HIP executor and the radial handles
// are stubbed out (this build has no device).
//
// Scenarios: concurrent clients submitting, polling, waiting on and releasing
// requests (half of them auto-release) under a budget small enough to defer;
// failing batches; back-pressure from max_pending; destroying a server with work
// still pending and running; the scheduler thread's CPU time while long batches
// run.  Exits 0 when every check holds and prints one line per scenario.
#include <stdint.h>
#include <stdio.h>
#include <time.h>

#include <atomic>
#include <chrono>
#include <memory>
#include <random>
#include <thread>
#include <vector>

#include "../../include/shmi.h"
#include "../../paper_2510_05282_amd/csrc/sh_server.h"

namespace shs {
std::unique_ptr<Executor> make_hip_executor(uint64_t, int, int* status)
{
    *status = SH_EHIP;
    return nullptr;
}
int radial_table(sh_radial*, int, int, RadialRef*) { return SH_EINVAL; }
}  // namespace shs

static int g_fail = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            g_fail = 1;                                                  \
        }                                                                \
    } while (0)

static double cpu_seconds()
{
    timespec ts;
    clock_gettime(CLOCK_PROCESS_CPUTIME_ID, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

// Atoms of 1e3 .. 3e5 points at fake (nonzero) device addresses.
static std::vector<int> add_atoms(sh_server_t s, int count, unsigned seed)
{
    std::mt19937 rng(seed);
    std::vector<int> ids;
    for (int k = 0; k < count; ++k) {
        const int64_t n = 1000 + int64_t(rng() % 300000);
        const double c[3] = {1.0, 2.0, 3.0};
        int id = -1;
        CHECK(sh_server_add_atom(s, k % 5 == 0 ? SH_F32 : SH_F64, n, reinterpret_cast<void*>(uintptr_t(4096 + k)), c,
                                 nullptr, 0, &id) == SH_OK);
        ids.push_back(id);
    }
    return ids;
}

static void clients(int fail_every)
{
    sh_server_t s = nullptr;
    // 256 MB budget, requests up to ~24 MB: admission has to wait for memory
    CHECK(sh_server_create_simulated(256ull << 20, 1 << 16, 3, 2e11, fail_every, 0.0, &s) == SH_OK);
    const std::vector<int> atoms = add_atoms(s, 64, 1);
    constexpr int kThreads = 4, kPer = 300;
    std::atomic<int64_t> done{0}, failed{0};
    std::vector<std::thread> th;
    for (int t = 0; t < kThreads; ++t) {
        th.emplace_back([&, t] {
            std::mt19937 rng(100 + t);
            std::vector<int64_t> mine;
            for (int k = 0; k < kPer; ++k) {
                const int a = atoms[rng() % atoms.size()];
                const int lmax = int(rng() % 10);
                const int flags = (k & 1) ? SH_REQ_AUTORELEASE : 0;
                int64_t tk = -1;
                int rc;
                while ((rc = sh_server_submit(s, a, lmax, flags, &tk)) == SH_EBUSY) std::this_thread::yield();
                CHECK(rc == SH_OK || rc == SH_EINVAL);
                if (rc != SH_OK) continue;
                int st = -1;
                CHECK(sh_server_poll(s, tk, &st) == SH_OK && st >= SH_REQ_PENDING && st <= SH_REQ_RELEASED);
                if (!flags) mine.push_back(tk);
                if (mine.size() >= 8 || k == kPer - 1) {
                    for (int64_t m : mine) {
                        int st2 = -1;
                        CHECK(sh_server_wait(s, m, 60.0, &st2) == SH_OK);
                        if (st2 == SH_REQ_DONE) {
                            void* p = nullptr;
                            CHECK(sh_server_result(s, m, &p) == SH_OK);
                            ++done;
                        } else {
                            CHECK(st2 == SH_REQ_FAILED);
                            ++failed;
                        }
                        CHECK(sh_server_release(s, m) == SH_OK);
                    }
                    mine.clear();
                }
            }
        });
    }
    // a reader of statistics and latencies while the clients run
    std::atomic<bool> stop{false};
    std::thread reader([&] {
        std::vector<double> lat(1024);
        while (!stop) {
            sh_server_stats_t st;
            CHECK(sh_server_stats(s, &st) == SH_OK);
            CHECK(st.bytes_in_use <= (256ull << 20));
            CHECK(sh_server_latencies(s, lat.data(), int64_t(lat.size())) >= 0);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });
    for (auto& x : th) x.join();
    CHECK(sh_server_drain(s, 60.0) == SH_OK);
    stop = true;
    reader.join();
    sh_server_stats_t st;
    CHECK(sh_server_stats(s, &st) == SH_OK);
    CHECK(st.completed + st.failed == st.submitted);
    CHECK(st.bytes_in_use == 0);
    CHECK(st.peak_bytes <= (256ull << 20));
    if (fail_every == 0) CHECK(st.failed == 0);
    else CHECK(st.failed > 0);
    printf("clients(fail_every=%d): submitted %lld completed %lld failed %lld deferred %lld batches %lld\n",
           fail_every, (long long)st.submitted, (long long)st.completed, (long long)st.failed,
           (long long)st.deferred, (long long)st.batches);
    CHECK(sh_server_destroy(s) == SH_OK);
}

static void back_pressure_and_shutdown()
{
    sh_server_t s = nullptr;
    // slow batches (2 GB/s), at most 16 waiting: submissions are refused, then the
    // server is destroyed with batches running and requests pending
    CHECK(sh_server_create_simulated(1ull << 30, 16, 2, 2e9, 0, 0.0, &s) == SH_OK);
    const std::vector<int> atoms = add_atoms(s, 8, 2);
    int busy = 0, ok = 0;
    for (int k = 0; k < 200; ++k) {
        int64_t tk;
        const int rc = sh_server_submit(s, atoms[k % atoms.size()], 9, SH_REQ_AUTORELEASE, &tk);
        if (rc == SH_EBUSY) ++busy;
        else if (rc == SH_OK) ++ok;
        else CHECK(false);
    }
    CHECK(busy > 0 && ok > 0);
    std::thread other([&] {
        sh_server_stats_t st;
        for (int k = 0; k < 50; ++k) CHECK(sh_server_stats(s, &st) == SH_OK);
    });
    other.join();
    printf("back pressure: %d accepted, %d refused; destroyed with work in flight\n", ok, busy);
    CHECK(sh_server_destroy(s) == SH_OK);
}

// CPU time the scheduler thread uses while three long simulated batches run and
// this thread sleeps: with completion notices from the executor it sleeps too.
static void scheduler_cpu()
{
    sh_server_t s = nullptr;
    CHECK(sh_server_create_simulated(64ull << 30, 1024, 3, 1e9, 0, 0.0, &s) == SH_OK);
    const double c[3] = {0, 0, 0};
    int a = -1;
    CHECK(sh_server_add_atom(s, SH_F64, 1000000, reinterpret_cast<void*>(uintptr_t(4096)), c, nullptr, 0, &a) ==
          SH_OK);
    int64_t t[3];
    for (int k = 0; k < 3; ++k) CHECK(sh_server_submit(s, a, 5, 0, &t[k]) == SH_OK);  // 288 MB each: ~0.29 s
    std::this_thread::sleep_for(std::chrono::milliseconds(20));
    sh_server_stats_t s0, s1;
    CHECK(sh_server_stats(s, &s0) == SH_OK);
    const double c0 = cpu_seconds();
    const auto w0 = std::chrono::steady_clock::now();
    std::this_thread::sleep_for(std::chrono::milliseconds(200));
    CHECK(sh_server_stats(s, &s1) == SH_OK);
    const double used = cpu_seconds() - c0;
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
    const double sched = (s1.scheduler_cpu_s - s0.scheduler_cpu_s) / wall;
    printf("cpu while batches run: scheduler thread %.3f, process %.3f of one core\n", sched, used / wall);
    CHECK(s0.scheduler_cpu_s >= 0.0 && sched < 0.25);
    for (int k = 0; k < 3; ++k) {
        int st;
        CHECK(sh_server_wait(s, t[k], 10.0, &st) == SH_OK && st == SH_REQ_DONE);
        CHECK(sh_server_release(s, t[k]) == SH_OK);
    }
    CHECK(sh_server_destroy(s) == SH_OK);
}

int main()
{
    clients(0);
    clients(7);
    back_pressure_and_shutdown();
    scheduler_cpu();
    printf(g_fail ? "FAILED\n" : "OK\n");
    return g_fail;
}
