// sh_server.cpp -- scheduling core of the projector server and its simulated
// executor (host code only; the HIP executor lives in sh_serve.hip).
#include "sh_server.h"

#include <pthread.h>
#include <sys/prctl.h>
#include <time.h>

#include <algorithm>

#include "../../include/shmi.h"

namespace shs {

// ---------------------------------------------------------------- arena

Arena::Arena(uint64_t capacity) : cap_(capacity & ~uint64_t(255))
{
    if (cap_) free_[0] = cap_;
}

bool Arena::alloc(uint64_t bytes, uint64_t* offset)
{
    bytes = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= bytes) {
            const uint64_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            *offset = off;
            return true;
        }
    }
    return false;
}

void Arena::release(uint64_t offset, uint64_t bytes)
{
    bytes = round(bytes ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(offset, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
        it->second += next->second;
        free_.erase(next);
    }
    if (it != free_.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            free_.erase(it);
        }
    }
}

// ---------------------------------------------------------------- server

static uint64_t out_bytes(const Atom& a, int lmax)
{
    return uint64_t(lmax + 1) * uint64_t(lmax + 1) * uint64_t(a.n) * (a.dtype == SH_F64 ? 8u : 4u);
}

static double secs(Clock::duration d) { return std::chrono::duration<double>(d).count(); }

static void* at(void* base, uint64_t offset)
{
    return reinterpret_cast<void*>(reinterpret_cast<uintptr_t>(base) + offset);
}

Server::Server(std::unique_ptr<Executor> ex, uint64_t budget, int64_t max_pending)
    : ex_(std::move(ex)), arena_(budget), max_pending_(max_pending), t0_(Clock::now())
{
    const int ns = ex_->n_slots();
    slot_reqs_.resize(ns);
    finished_.resize(ns);
    for (int s = ns - 1; s >= 0; --s) free_slots_.push_back(s);
    st_.first_submit_s = -1.0;
    thr_ = std::thread([this] { loop(); });
}

Server::~Server()
{
    {
        std::lock_guard<std::mutex> g(mu_);
        stop_ = true;
        gen_++;
    }
    cv_work_.notify_all();
    thr_.join();
}

int Server::add_atom(const Atom& a, int* id)
{
    if (!id || a.n <= 0 || !a.points || (a.dtype != SH_F64 && a.dtype != SH_F32)) return SH_EINVAL;
    const int64_t tp = ex_->tile_points();
    if ((a.n + tp - 1) / tp > ex_->max_tiles()) return SH_EINVAL;  // one batch could never hold it
    std::lock_guard<std::mutex> g(mu_);
    atoms_.push_back(a);
    *id = int(atoms_.size() - 1);
    return SH_OK;
}

int Server::submit(int atom, int lmax, int flags, int64_t* ticket)
{
    // a request's latency starts before any wait for the lock
    const Clock::time_point t_submit = Clock::now();
    if (!ticket || lmax < 0 || lmax > SH_LMAX) return SH_EINVAL;
    std::lock_guard<std::mutex> g(mu_);
    if (stop_) return SH_EBUSY;
    if (atom < 0 || atom >= int(atoms_.size())) return SH_EINVAL;
    const Atom& a = atoms_[atom];
    if (a.tab && lmax > a.tab_lmax) return SH_EINVAL;
    const uint64_t bytes = out_bytes(a, lmax);
    if (Arena::round(bytes) > arena_.capacity()) return SH_EINVAL;  // could never be admitted
    if (int64_t(pending_.size()) >= max_pending_) return SH_EBUSY;
    Request r{};
    r.atom = atom;
    r.lmax = lmax;
    r.flags = flags;
    r.bytes = bytes;
    r.state = kPending;
    r.t_submit = t_submit;
    r.refusals_at_submit = refusals_;
    *ticket = int64_t(reqs_.size());
    reqs_.push_back(r);
    pending_.push_back(*ticket);
    gen_++;
    st_.submitted++;
    if (st_.first_submit_s < 0) st_.first_submit_s = secs(r.t_submit - t0_);
    cv_work_.notify_one();
    return SH_OK;
}

bool Server::admit_locked()
{
    bool prog = false;
    while (!pending_.empty()) {
        Request& r = reqs_[pending_.front()];
        uint64_t off;
        if (!arena_.alloc(r.bytes, &off)) {
            refusals_++;
            break;
        }
        // deferred: a refusal for lack of budget happened while it was waiting
        if (refusals_ > r.refusals_at_submit) st_.deferred++;
        r.offset = off;
        r.state = kQueued;
        queued_.push_back(pending_.front());
        pending_.pop_front();
        st_.bytes_in_use = arena_.in_use();
        st_.peak_bytes = std::max(st_.peak_bytes, st_.bytes_in_use);
        prog = true;
    }
    return prog;
}

void Server::finish_req_locked(int64_t t, int status, Clock::time_point now)
{
    Request& r = reqs_[t];
    r.t_done = now;
    if (status == SH_OK) {
        r.state = kDone;
        st_.completed++;
        st_.points_done += atoms_[r.atom].n;
        lat_ms_.push_back(secs(r.t_done - r.t_submit) * 1e3);
        st_.last_done_s = secs(now - t0_);
        if (r.flags & SH_REQ_AUTORELEASE) {
            arena_.release(r.offset, r.bytes);
            r.state = kReleased;
        }
    } else {
        r.state = kFailed;
        r.error = status;
        st_.failed++;
        arena_.release(r.offset, r.bytes);
    }
}

void Server::finish_locked(int slot, int status)
{
    const Clock::time_point now = Clock::now();
    for (size_t i = 0; i < slot_reqs_[slot].size(); ++i)
        if (!finished_[slot][i]) finish_req_locked(slot_reqs_[slot][i], status, now);
    st_.bytes_in_use = arena_.in_use();
    slot_reqs_[slot].clear();
    finished_[slot].clear();
    free_slots_.push_back(slot);
    cv_done_.notify_all();
}

// Finishes what progress() reported for the busy slots (done_, early_): single
// requests whose results are complete, and whole batches that ended.  lk held.
bool Server::apply_locked()
{
    bool prog = false, early = false;
    const Clock::time_point now = Clock::now();
    for (size_t k = 0; k < busy_.size(); ++k) {
        const int slot = busy_[k];
        for (int i : early_[k]) {
            if (i < 0 || i >= int(finished_[slot].size()) || finished_[slot][i]) continue;
            finished_[slot][i] = 1;
            finish_req_locked(slot_reqs_[slot][i], SH_OK, now);
            early = true;
        }
        early_[k].clear();
        if (done_[k] != 0) {
            busy_slots_--;
            finish_locked(slot, done_[k] > 0 ? SH_OK : SH_EHIP);
            prog = true;
        }
    }
    if (early) {
        st_.bytes_in_use = arena_.in_use();
        cv_done_.notify_all();
    }
    return prog || early;
}

// Finishes the requests and batches that have completed.  Called with lk held;
// the completion queries (HIP runtime calls) run with it released, so submitters
// are not held up.
bool Server::reap(std::unique_lock<std::mutex>& lk)
{
    busy_.clear();
    for (int s = 0; s < int(slot_reqs_.size()); ++s)
        if (!slot_reqs_[s].empty()) busy_.push_back(s);
    if (busy_.empty()) return false;
    done_.assign(busy_.size(), 0);
    early_.resize(busy_.size());
    for (auto& e : early_) e.clear();
    lk.unlock();
    for (size_t k = 0; k < busy_.size(); ++k) done_[k] = ex_->progress(busy_[k], early_[k]);
    lk.lock();
    return apply_locked();
}

void Server::loop()
{
    // naps of a few microseconds need a small timer slack (the default adds ~50 us)
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        bool prog = reap(lk);
        if (stop_) {
            // refuse what has not started; let running batches finish
            for (int64_t t : pending_) {
                reqs_[t].state = kFailed;
                reqs_[t].error = SH_EBUSY;
            }
            for (int64_t t : queued_) {
                reqs_[t].state = kFailed;
                reqs_[t].error = SH_EBUSY;
                arena_.release(reqs_[t].offset, reqs_[t].bytes);
            }
            pending_.clear();
            queued_.clear();
            cv_done_.notify_all();
            if (busy_slots_ == 0) break;
        } else {
            prog |= admit_locked();
        }
        if (!queued_.empty() && !free_slots_.empty()) {
            const int slot = free_slots_.back();
            free_slots_.pop_back();
            std::vector<Item> items;
            int64_t tiles = 0;
            size_t k = 0;
            for (; k < queued_.size() && int64_t(items.size()) < ex_->max_items(); ++k) {
                Request& r = reqs_[queued_[k]];
                const Atom& a = atoms_[r.atom];
                const int64_t nt = (a.n + ex_->tile_points() - 1) / ex_->tile_points();
                if (!items.empty() && tiles + nt > ex_->max_tiles()) break;
                tiles += nt;
                items.push_back(Item{a, r.lmax, at(ex_->arena_base(), r.offset)});
                r.state = kRunning;
                slot_reqs_[slot].push_back(queued_[k]);
            }
            finished_[slot].assign(slot_reqs_[slot].size(), 0);
            queued_.erase(queued_.begin(), queued_.begin() + k);
            // the slot counts as busy before the lock is dropped, so drain() cannot
            // observe an empty server while this batch is being launched
            busy_slots_++;
            lk.unlock();
            const int rc = ex_->launch(slot, items);
            lk.lock();
            if (rc != SH_OK) {
                busy_slots_--;
                finish_locked(slot, rc);
            } else {
                st_.batches++;
            }
            prog = true;
        }
        if (!prog) {
            if (busy_slots_ > 0) {
                // Batches are running and nothing else can be done: poll their
                // completion with the lock free until one finishes, or until a
                // submit, release or shutdown bumps gen_ while a slot is free (with
                // every slot busy, new work waits for a completion anyway, so
                // submitters never contend with this thread for the lock).
                // busy_ and free_slots_ change only on this thread.  Short batches
                // are caught by back-to-back polls; after kBusySpin the thread naps
                // between polls (kNapMin doubling to kNapMax), which bounds the CPU
                // it takes while long batches run and delays noticing their end by
                // at most one nap.
                const uint64_t g = gen_;
                const bool slot_free = !free_slots_.empty();
                done_.assign(busy_.size(), 0);
                early_.resize(busy_.size());
                for (auto& e : early_) e.clear();
                lk.unlock();
                const Clock::time_point t_poll = Clock::now();
                std::chrono::microseconds nap = kNapMin;
                for (bool got = false; !got && !(gen_ != g && (slot_free || stop_));) {
                    if (Clock::now() - t_poll < kBusySpin) {
                        std::this_thread::yield();
                    } else {
                        std::this_thread::sleep_for(nap);
                        nap = std::min(nap * 2, kNapMax);
                    }
                    for (size_t k = 0; k < busy_.size(); ++k) {
                        if (done_[k] == 0) done_[k] = ex_->progress(busy_[k], early_[k]);
                        got = got || done_[k] != 0 || !early_[k].empty();
                    }
                }
                lk.lock();
                apply_locked();
            } else {
                // nothing runs and nothing can be admitted: watch for a submit, a
                // release or shutdown with the lock free for up to kIdleSpin (a
                // thread asleep on the condition variable takes microseconds to
                // wake, which a lightly loaded server would add to every request),
                // then sleep until one comes
                const uint64_t g = gen_;
                lk.unlock();
                const auto t0 = std::chrono::steady_clock::now();
                while (gen_ == g && !stop_ && std::chrono::steady_clock::now() - t0 < kIdleSpin)
                    std::this_thread::yield();
                lk.lock();
                cv_work_.wait(lk, [&] { return stop_ || gen_ != g; });
            }
        }
    }
}

int Server::poll(int64_t ticket, int* state)
{
    if (!state) return SH_EINVAL;
    std::lock_guard<std::mutex> g(mu_);
    if (ticket < 0 || ticket >= int64_t(reqs_.size())) return SH_EINVAL;
    *state = reqs_[ticket].state;
    return SH_OK;
}

int Server::wait(int64_t ticket, double timeout_s, int* state)
{
    std::unique_lock<std::mutex> lk(mu_);
    if (ticket < 0 || ticket >= int64_t(reqs_.size())) return SH_EINVAL;
    const bool ok = cv_done_.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                      [&] { return reqs_[ticket].state >= kDone; });
    if (state) *state = reqs_[ticket].state;
    return ok ? SH_OK : SH_EBUSY;
}

int Server::result(int64_t ticket, void** ptr)
{
    if (!ptr) return SH_EINVAL;
    std::lock_guard<std::mutex> g(mu_);
    if (ticket < 0 || ticket >= int64_t(reqs_.size())) return SH_EINVAL;
    const Request& r = reqs_[ticket];
    if (r.state < kDone) return SH_EBUSY;
    if (r.state != kDone) return r.state == kFailed ? r.error : SH_EINVAL;
    *ptr = at(ex_->arena_base(), r.offset);
    return SH_OK;
}

int Server::release(int64_t ticket)
{
    std::lock_guard<std::mutex> g(mu_);
    if (ticket < 0 || ticket >= int64_t(reqs_.size())) return SH_EINVAL;
    Request& r = reqs_[ticket];
    if (r.state < kDone) return SH_EBUSY;
    if (r.state == kDone) {
        arena_.release(r.offset, r.bytes);
        st_.bytes_in_use = arena_.in_use();
        gen_++;
        cv_work_.notify_one();
    }
    r.state = kReleased;
    return SH_OK;
}

int Server::drain(double timeout_s)
{
    std::unique_lock<std::mutex> lk(mu_);
    const bool ok = cv_done_.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] {
        return pending_.empty() && queued_.empty() && busy_slots_ == 0;
    });
    return ok ? SH_OK : SH_EBUSY;
}

void Server::stats(Stats* s)
{
    clockid_t cid;
    timespec ts{};
    double cpu = -1.0;
    if (pthread_getcpuclockid(thr_.native_handle(), &cid) == 0 && clock_gettime(cid, &ts) == 0)
        cpu = double(ts.tv_sec) + 1e-9 * double(ts.tv_nsec);
    std::lock_guard<std::mutex> g(mu_);
    *s = st_;
    s->scheduler_cpu_s = cpu;
}

int64_t Server::latencies(double* out, int64_t cap)
{
    std::lock_guard<std::mutex> g(mu_);
    const int64_t n = std::min<int64_t>(cap, int64_t(lat_ms_.size()));
    if (out)
        for (int64_t i = 0; i < n; ++i) out[i] = lat_ms_[i];
    return int64_t(lat_ms_.size());
}

// ---------------------------------------------------------------- simulation

namespace {

// Runs nothing: a launch takes launch_s of host time, a batch "finishes" after its
// output bytes at a fixed rate, and every fail_every-th launch reports a failure.
// Used to test scheduling without a GPU; its arena has no memory (base address 0,
// offsets only).
class SimExecutor final : public Executor {
public:
    SimExecutor(int n_slots, double bps, int fail_every, double launch_s)
        : item_done_(n_slots), next_(n_slots, 0), done_at_(n_slots), fail_(n_slots, false), bps_(bps),
          fail_every_(fail_every), launch_s_(launch_s)
    {
    }
    int n_slots() const override { return int(done_at_.size()); }
    int64_t max_items() const override { return 4096; }
    int64_t max_tiles() const override { return int64_t(1) << 22; }
    int64_t tile_points() const override { return 256; }
    void* arena_base() override { return nullptr; }
    // Items run one after another, smallest output first (as the HIP executor orders
    // its launches); each completes when its cumulative bytes have been written.
    int launch(int slot, const std::vector<Item>& items) override
    {
        if (launch_s_ > 0) std::this_thread::sleep_for(std::chrono::duration<double>(launch_s_));
        std::vector<int> idx(items.size());
        for (size_t k = 0; k < idx.size(); ++k) idx[k] = int(k);
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            return out_bytes(items[a].atom, items[a].lmax) < out_bytes(items[b].atom, items[b].lmax);
        });
        {
            std::lock_guard<std::mutex> g(mu_);
            const Clock::time_point t0 = Clock::now();
            auto& q = item_done_[slot];
            q.clear();
            double bytes = 0;
            for (int k : idx) {
                bytes += double(out_bytes(items[k].atom, items[k].lmax));
                q.push_back({t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(bytes / bps_)),
                             k});
            }
            done_at_[slot] =
                t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(bytes / bps_));
            next_[slot] = 0;
            ++launches_;
            fail_[slot] = fail_every_ > 0 && launches_ % fail_every_ == 0;
        }
        return SH_OK;
    }
    int query(int slot) override
    {
        std::lock_guard<std::mutex> g(mu_);
        return query_locked(slot);
    }
    // a failing batch reports nothing early: all its requests fail with it
    int progress(int slot, std::vector<int>& done) override
    {
        std::lock_guard<std::mutex> g(mu_);
        const Clock::time_point now = Clock::now();
        const auto& q = item_done_[slot];
        while (!fail_[slot] && next_[slot] < q.size() && q[next_[slot]].first <= now)
            done.push_back(q[next_[slot]++].second);
        return query_locked(slot);
    }
private:
    int query_locked(int slot) const
    {
        if (Clock::now() < done_at_[slot]) return 0;
        return fail_[slot] ? -1 : 1;
    }
    std::mutex mu_;  // guards everything below (launch, query and progress may come from any thread)
    std::vector<std::vector<std::pair<Clock::time_point, int>>> item_done_;  // per slot: (completion, item)
    std::vector<size_t> next_;  // per slot: first item not yet reported by progress()
    std::vector<Clock::time_point> done_at_;
    std::vector<bool> fail_;
    double bps_;
    int fail_every_;
    double launch_s_;  // host time one launch takes
    int64_t launches_ = 0;
};

}  // namespace

std::unique_ptr<Executor> make_sim_executor(int n_slots, double bytes_per_s, int fail_every, double launch_s)
{
    return std::unique_ptr<Executor>(new SimExecutor(n_slots, bytes_per_s, fail_every, launch_s));
}

}  // namespace shs
