// sh_server_api.cpp -- the C ABI of the projector server (sh_server_* in shmi.h).
//
// Host code only: the scheduler (sh_server.cpp) and these entry points build with
// a plain C++ compiler as well, which is how they are checked under the thread,
// address and undefined-behaviour sanitizers; the HIP executor and the radial
// handles come from the library's HIP sources.
#include <stdint.h>

#include <memory>
#include <new>

#include "../../include/shmi.h"
#include "sh_server.h"

struct sh_server {
    std::unique_ptr<shs::Server> srv;
    bool simulated;
};

extern "C" {

static int server_new(std::unique_ptr<shs::Executor> ex, uint64_t budget, int max_pending, bool sim,
                      sh_server_t *out)
{
    sh_server *h = new (std::nothrow) sh_server{};
    if (!h) return SH_ENOMEM;
    h->simulated = sim;
    h->srv.reset(new (std::nothrow) shs::Server(std::move(ex), budget, max_pending));
    if (!h->srv) {
        delete h;
        return SH_ENOMEM;
    }
    *out = h;
    return SH_OK;
}

int sh_server_create(uint64_t budget_bytes, int max_pending, int n_slots, sh_server_t *out)
{
    if (!out) return SH_EINVAL;
    *out = nullptr;
    if (budget_bytes < 256 || max_pending < 1 || n_slots < 1 || n_slots > 16) return SH_EINVAL;
    int st = SH_OK;
    std::unique_ptr<shs::Executor> ex = shs::make_hip_executor(budget_bytes, n_slots, &st);
    if (!ex) return st == SH_OK ? SH_EHIP : st;
    return server_new(std::move(ex), budget_bytes, max_pending, false, out);
}

int sh_server_create_simulated(uint64_t budget_bytes, int max_pending, int n_slots, double bytes_per_second,
                               int fail_every, double launch_seconds, sh_server_t *out)
{
    if (!out) return SH_EINVAL;
    *out = nullptr;
    if (budget_bytes < 256 || max_pending < 1 || n_slots < 1 || n_slots > 16 || !(bytes_per_second > 0.0) ||
        !(launch_seconds >= 0.0 && launch_seconds < 10.0))
        return SH_EINVAL;
    return server_new(shs::make_sim_executor(n_slots, bytes_per_second, fail_every, launch_seconds), budget_bytes,
                      max_pending, true, out);
}

int sh_server_destroy(sh_server_t srv)
{
    delete srv;
    return SH_OK;
}

int sh_server_add_atom(sh_server_t srv, int dtype, int64_t n, const void *points, const double *center,
                       sh_radial_t radial, int table, int *atom_id)
{
    if (!srv || !center || !atom_id || !points || n <= 0) return SH_EINVAL;
    if (dtype != SH_F64 && dtype != SH_F32) return SH_EINVAL;
    shs::Atom a{};
    a.dtype = dtype;
    a.n = n;
    a.points = points;
    for (int q = 0; q < 3; ++q) a.c[q] = center[q];
    if (radial) {
        shs::RadialRef t;
        const int rc = shs::radial_table(radial, table, dtype, &t);
        if (rc != SH_OK) return rc;
        a.tab = t.tab;
        a.tab_lmax = t.lmax;
        for (int L = 0; L <= shs::kCompactLmax; ++L) a.tab_compact[L] = t.compact[L];
        a.n_r = t.n_r;
        a.h = t.h;
        a.r_max = t.r_max;
    } else {
        if (!srv->simulated) return SH_EINVAL;
        a.tab_lmax = SH_LMAX;
    }
    return srv->srv->add_atom(a, atom_id);
}

int sh_server_submit(sh_server_t srv, int atom_id, int lmax, int flags, int64_t *ticket)
{
    if (!srv) return SH_EINVAL;
    return srv->srv->submit(atom_id, lmax, flags, ticket);
}

int sh_server_poll(sh_server_t srv, int64_t ticket, int *state)
{
    if (!srv) return SH_EINVAL;
    return srv->srv->poll(ticket, state);
}

int sh_server_wait(sh_server_t srv, int64_t ticket, double timeout_s, int *state)
{
    if (!srv || !(timeout_s >= 0.0)) return SH_EINVAL;
    return srv->srv->wait(ticket, timeout_s, state);
}

int sh_server_result(sh_server_t srv, int64_t ticket, void **out)
{
    if (!srv) return SH_EINVAL;
    return srv->srv->result(ticket, out);
}

int sh_server_release(sh_server_t srv, int64_t ticket)
{
    if (!srv) return SH_EINVAL;
    return srv->srv->release(ticket);
}

int sh_server_drain(sh_server_t srv, double timeout_s)
{
    if (!srv || !(timeout_s >= 0.0)) return SH_EINVAL;
    return srv->srv->drain(timeout_s);
}

int sh_server_stats(sh_server_t srv, sh_server_stats_t *out)
{
    if (!srv || !out) return SH_EINVAL;
    shs::Stats s;
    srv->srv->stats(&s);
    out->submitted = s.submitted;
    out->completed = s.completed;
    out->failed = s.failed;
    out->deferred = s.deferred;
    out->batches = s.batches;
    out->points_done = s.points_done;
    out->bytes_in_use = s.bytes_in_use;
    out->peak_bytes = s.peak_bytes;
    out->first_submit_s = s.first_submit_s;
    out->last_done_s = s.last_done_s;
    out->scheduler_cpu_s = s.scheduler_cpu_s;
    return SH_OK;
}

int64_t sh_server_latencies(sh_server_t srv, double *out_ms, int64_t cap)
{
    if (!srv || cap < 0) return -SH_EINVAL;
    return srv->srv->latencies(out_ms, cap);
}

}  // extern "C"
