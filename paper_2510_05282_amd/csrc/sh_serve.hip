// sh_serve.hip -- HIP executor of the projector server: the launches of a batch on
// one of n_slots streams.
//
// A batch is a list of requests of any lmax and either dtype.  The requests are
// grouped by (dtype, lmax); each request is cut into tiles of 256 lanes x PPL
// adjacent points, evaluated with the same projector code as sh_projectors (PPL as
// there: the vector width for a group of at least kServeVecPoints points, else 1).
// Each vector-width group gets one launch of the kernel built for it (registers and
// occupancy sized for that lmax, no per-point dispatch); the one-point groups share
// one launch of the mixed kernel when there are two or more of them (a block runs
// the code of its request's (dtype, lmax)), which saves the host a launch and an
// event per extra group.  The launches go smallest output first, each with its
// group's event as the launch's own completion event (hipExtLaunchKernel: no
// separate event record), and progress() reports a launch's requests as soon as
// its event completes.  A launch of at most kInlineItems requests takes their descriptors as
// kernel arguments; the descriptors of larger launches and their first-tile
// indices travel host -> device in one copy per batch through a pinned staging
// buffer per slot (the slot is reused only after its previous batch has completed,
// so the staging buffer is never overwritten in flight), and a batch with no
// larger launch makes no copy.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <utility>

#include "../../include/shmi.h"
#include "sh_core.h"
#include "sh_proj.h"
#include "sh_server.h"

namespace shk {

struct ServeDesc {
    const void* points;
    void* out;
    const void* tab;  // knot_t of the request's dtype
    double c[3];
    double h, inv_h, r_max, h2_over_6;
    int64_t n;
    int64_t tile0;  // first tile of this request within the batch
    int n_r;
    int ch;  // channels of the table (its lmax + 1)
    int lmax;
    int dtype;
};

constexpr int kServeBlock = 256;  // lanes per tile and block

// Descriptors of a small group, passed by value as kernel arguments: the launch
// needs no copy and a block finds its request among them in registers.
constexpr int kInlineItems = 4;
struct ServeInline {
    ServeDesc d[kInlineItems];
};

// The descriptor of a launch's tile: the last of the launch's n_items requests whose
// first tile is at most `tile`, one of the first n_items descriptors of `in` when
// descs is null (n_items <= kInlineItems), else found by a wave-wide search over
// their first-tile indices in tile0.
__device__ __forceinline__ void find_desc(const ServeInline& in, const ServeDesc* __restrict__ descs,
                                          const int64_t* __restrict__ tile0, int n_items, int64_t tile, ServeDesc& d)
{
    if (descs == nullptr) {
        // uniform selection without indexing the argument block by a variable
        d = in.d[0];
#pragma unroll
        for (int k = 1; k < kInlineItems; ++k)
            if (k < n_items && in.d[k].tile0 <= tile) d = in.d[k];
    } else {
        // tile0 is increasing with tile0[0] = 0 <= tile, so the search finds an item
        d = descs[wave_search(tile0, n_items, tile)];
    }
}

// Point j of request d, one point per lane.
template <int LMAX, typename TIO>
__device__ __forceinline__ void serve_point(const ServeDesc& d, int64_t j, const SplineGrid& g)
{
    const TIO* p = static_cast<const TIO*>(d.points) + 3 * j;
    proj_point<LMAX, TIO>(double(p[0]), double(p[1]), double(p[2]), d.c, static_cast<const knot_t<TIO>*>(d.tab),
                          d.ch, g, static_cast<TIO*>(d.out) + j, d.n);
}

// One launch per (lmax, dtype) group of a batch: block b handles tile
// xcd_tile(b) of the group (the tiles of one group cost the same, so
// XCD-contiguous ranges stay balanced and each XCD keeps few requests' tables in
// its L2) and evaluates P adjacent points per lane (the request's last lane
// repeats its last point in the slots past the end and stores only its own).
template <int LMAX, typename TIO, int P>
__global__ __launch_bounds__(kServeBlock) void serve_kernel(ServeInline in, const ServeDesc* __restrict__ descs,
                                                            const int64_t* __restrict__ tile0, int n_items)
{
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    // as find_desc, written out: through a reference to the argument block the
    // compiler allocated this kernel's registers differently (104 VGPRs and 56
    // SGPRs against 122 and 40 at lmax 9, FP64), and the serving closed loop ran
    // 1.2% slower
    ServeDesc d;
    if (descs == nullptr) {
        d = in.d[0];
#pragma unroll
        for (int k = 1; k < kInlineItems; ++k)
            if (k < n_items && in.d[k].tile0 <= tile) d = in.d[k];
    } else {
        d = descs[wave_search(tile0, n_items, tile)];
    }
    const int64_t j = (tile - d.tile0) * (kServeBlock * P) + threadIdx.x * P;
    if (j < 0 || j >= d.n) return;
    const SplineGrid g{d.n_r, d.h, d.inv_h, d.r_max, d.h2_over_6};
    if constexpr (P == 1) {
        serve_point<LMAX, TIO>(d, j, g);
    } else {
        const int nvalid = d.n - j < P ? int(d.n - j) : P;
        const TIO* p = static_cast<const TIO*>(d.points) + 3 * j;
        double px[P], py[P], pz[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int qq = q < nvalid ? q : nvalid - 1;
            px[q] = double(p[3 * qq]);
            py[q] = double(p[3 * qq + 1]);
            pz[q] = double(p[3 * qq + 2]);
        }
        proj_points<LMAX, TIO, P>(px, py, pz, d.c, static_cast<const knot_t<TIO>*>(d.tab), d.ch, g,
                                  static_cast<TIO*>(d.out) + j, d.n, nvalid);
    }
}

// The one-point-per-lane groups of a batch in one launch: requests of any lmax and
// either dtype, each block running the code of its request's (dtype, lmax) (the
// same code as serve_kernel<LMAX, TIO, 1>, so a value does not depend on which
// launch computed it).
__global__ __launch_bounds__(kServeBlock) void serve_mixed_kernel(ServeInline in,
                                                                   const ServeDesc* __restrict__ descs,
                                                                   const int64_t* __restrict__ tile0, int n_items)
{
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    ServeDesc d;
    find_desc(in, descs, tile0, n_items, tile, d);
    const int64_t j = (tile - d.tile0) * kServeBlock + threadIdx.x;
    if (j < 0 || j >= d.n) return;
    const SplineGrid g{d.n_r, d.h, d.inv_h, d.r_max, d.h2_over_6};
    static_for<0, SH_LMAX + 1>([&](auto lc) {
        constexpr int L = decltype(lc)::value;
        if (d.lmax == L) {
            if (d.dtype == SH_F64) serve_point<L, double>(d, j, g);
            else serve_point<L, float>(d, j, g);
        }
    });
}

static hipError_t launch_mixed(int64_t tiles, const ServeInline& in, const ServeDesc* descs, const int64_t* tile0,
                               int n, hipStream_t s, hipEvent_t done)
{
    if (descs == nullptr && (n < 1 || n > kInlineItems)) return hipErrorInvalidValue;
    hipExtLaunchKernelGGL(serve_mixed_kernel, dim3(unsigned(tiles)), dim3(kServeBlock), 0, s, nullptr, done, 0, in,
                          descs, tile0, n);
    return hipGetLastError();
}

// Lane width of the vector-lane serving launches: the projector build's, except FP64
// at lmax 2, which keeps four points per lane here (the build moved to two in
// proj_vec_kernel; serve_kernel, which loads each point's knots in turn, took 116 us
// per lmax 2 FP64 launch with two against 87 us with four, closed-loop kernel trace).
template <typename TIO, int LMAX>
constexpr int kServePpl = sizeof(TIO) == 8 && LMAX == 2 ? 4 : kProjPpl<TIO, LMAX>;

template <int LMAX, typename TIO>
static void launch_group_l(int ppl, int64_t tiles, const ServeInline& in, const ServeDesc* descs,
                           const int64_t* tile0, int n, hipStream_t s, hipEvent_t done)
{
    const dim3 grid = dim3(unsigned(tiles)), block = dim3(kServeBlock);
    if (ppl == 1)
        hipExtLaunchKernelGGL((serve_kernel<LMAX, TIO, 1>), grid, block, 0, s, nullptr, done, 0, in, descs, tile0, n);
    else
        hipExtLaunchKernelGGL((serve_kernel<LMAX, TIO, kServePpl<TIO, LMAX>>), grid, block,
                              uint32_t(kProjCapLds<TIO, LMAX>), s, nullptr, done, 0, in, descs, tile0, n);
}

// Groups of at least this many points take several points per lane.  Lower than
// the projector build's kProjVecPoints: a group is one launch of a batch, and in the
// Poisson stream (batches of a few requests) groups of 2^18 to 2^20 points are
// common.  Measured on the 10,000-request stream, two runs each, against 2^20: at
// 75k req/s p50 0.18-0.19 ms (0.25-0.29), p99 1.11-1.15 ms (1.74-1.76); at 63k req/s
// p50 0.10-0.105 ms (0.116-0.118), p99 0.67-0.71 ms (0.77-0.78); closed loop
// unchanged within its spread (2^19: in between).
constexpr int64_t kServeVecPoints = int64_t(1) << 18;

// Lane width of a group of n points of one (dtype, lmax): 1 or kServePpl.
template <typename TIO, int... L>
static int vec_ppl_of(int lmax, std::integer_sequence<int, L...>)
{
    constexpr int w[] = {kServePpl<TIO, L>...};
    return w[lmax];
}
static int group_ppl(int dtype, int lmax, int64_t n)
{
    if (n < kServeVecPoints) return 1;
    return dtype == SH_F32 ? vec_ppl_of<float>(lmax, std::make_integer_sequence<int, SH_LMAX + 1>{})
                           : vec_ppl_of<double>(lmax, std::make_integer_sequence<int, SH_LMAX + 1>{});
}

// ppl is 1 or kServePpl<TIO, lmax>; descs null: the n <= kInlineItems descriptors
// of `in`, else n descriptors at descs and their first tiles at tile0 (device)
template <typename TIO>
static hipError_t launch_group(int lmax, int ppl, int64_t tiles, const ServeInline& in, const ServeDesc* descs,
                               const int64_t* tile0, int n, hipStream_t s, hipEvent_t done)
{
    if (descs == nullptr && (n < 1 || n > kInlineItems)) return hipErrorInvalidValue;
    switch (lmax) {
    case 0: launch_group_l<0, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    case 1: launch_group_l<1, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    case 2: launch_group_l<2, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    case 3: launch_group_l<3, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    case 4: launch_group_l<4, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    case 5: launch_group_l<5, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    case 6: launch_group_l<6, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    case 7: launch_group_l<7, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    case 8: launch_group_l<8, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    case 9: launch_group_l<9, TIO>(ppl, tiles, in, descs, tile0, n, s, done); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace shk

namespace shs {

namespace {

class HipExecutor final : public Executor {
public:
    HipExecutor(uint64_t budget, int n_slots, int* status) : slots_(n_slots)
    {
        *status = SH_OK;
        if (hipMalloc(&arena_, budget ? budget : 256) != hipSuccess) {
            (void)hipGetLastError();
            arena_ = nullptr;
            *status = SH_ENOMEM;
            return;
        }
        for (Slot& s : slots_) {
            s.group_done.assign(kMaxGroups, nullptr);
            bool events_ok = true;
            for (hipEvent_t& ev : s.group_done)
                events_ok = events_ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
            if (!events_ok || hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipHostMalloc(reinterpret_cast<void**>(&s.host), kSlotBytes) != hipSuccess ||
                hipMalloc(&s.dev, kSlotBytes) != hipSuccess) {
                (void)hipGetLastError();
                *status = SH_EHIP;
                return;
            }
        }
        if (!slots_.empty() && warm_up(slots_[0]) != hipSuccess) {
            (void)hipGetLastError();
            *status = SH_EHIP;
        }
    }
    ~HipExecutor() override
    {
        for (Slot& s : slots_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.dev) (void)hipFree(s.dev);
            if (s.host) (void)hipHostFree(s.host);
            for (hipEvent_t ev : s.group_done)
                if (ev) (void)hipEventDestroy(ev);
            if (s.stream) (void)hipStreamDestroy(s.stream);
        }
        if (arena_) (void)hipFree(arena_);
    }
    int n_slots() const override { return int(slots_.size()); }
    int64_t max_items() const override { return kMaxItems; }
    // a dispatch counts its work-items in 32 bits: tiles * 256 < 2^32
    int64_t max_tiles() const override { return (int64_t(1) << 24) - 1; }
    // the smallest tile (one point per lane); longer tiles only lower the count, so
    // the max_tiles bound stays safe
    int64_t tile_points() const override { return shk::kServeBlock; }
    void* arena_base() override { return arena_; }

    int launch(int slot, const std::vector<Item>& items) override
    {
        if (items.empty()) return SH_OK;
        Slot& s = slots_[slot];
        const size_t n = items.size();
        // items grouped by (dtype, lmax), in arrival order within a group; each
        // group's lane width from its size (keys: dtype * 16 + lmax)
        auto key = [&](int k) { return items[k].atom.dtype * 16 + items[k].lmax; };
        int64_t points_of[32] = {};
        for (size_t k = 0; k < n; ++k) points_of[key(int(k))] += items[k].atom.n;
        int ppl_of[32];
        int n_small = 0;           // groups with one point per lane
        int64_t small_points = 0;  // and their points
        for (int c = 0; c < 32; ++c) {
            ppl_of[c] = points_of[c] ? shk::group_ppl(c / 16, c % 16, points_of[c]) : 0;
            n_small += ppl_of[c] == 1;
            small_points += ppl_of[c] == 1 ? points_of[c] : 0;
        }
        // the one-point groups first, then the vector-lane groups; two or more
        // one-point groups of fewer than kServeVecPoints points together form one
        // launch (the mixed kernel): one launch and one event on the host instead
        // of one per group.  Larger sets keep their own kernels, whose registers are
        // sized for their lmax (the mixed kernel's for the largest).
        const bool merge = n_small >= 2 && small_points < shk::kServeVecPoints;
        order_.resize(n);
        for (size_t k = 0; k < n; ++k) order_[k] = int(k);
        auto rank = [&](int k) { return (ppl_of[key(k)] > 1 ? 64 : 0) + key(k); };
        std::stable_sort(order_.begin(), order_.end(), [&](int a, int b) { return rank(a) < rank(b); });
        groups_.clear();  // the launches: runs of order_
        for (size_t k = 0; k < n; ++k) {
            const int c = key(order_[k]);
            const bool join = !groups_.empty() && (merge && ppl_of[c] == 1 ? groups_.back().mixed
                                                                          : key(order_[groups_.back().first]) == c);
            if (!join) groups_.push_back({int(k), int(k), 0, 0, ppl_of[c], merge && ppl_of[c] == 1});
            Group& g = groups_.back();
            g.end = int(k) + 1;
            const Item& it = items[order_[k]];
            g.bytes += it.atom.n * (it.lmax + 1) * (it.lmax + 1) * (it.atom.dtype == SH_F64 ? 8 : 4);
        }
        // descriptors, then their first-tile indices (relative to their launch), in one copy
        int64_t* tile0 = reinterpret_cast<int64_t*>(s.host + n);
        for (Group& g : groups_) {
            const int64_t tp = int64_t(shk::kServeBlock) * g.ppl;
            for (int k = g.first; k < g.end; ++k) {
                const Item& it = items[order_[k]];
                shk::ServeDesc& d = s.host[k];
                memset(&d, 0, sizeof(d));
                d.points = it.atom.points;
                d.out = it.out;
                // the table copy with the request's channels only, where the handle has one
                const bool cmp = it.lmax < it.atom.tab_lmax && it.lmax <= kCompactLmax &&
                                 it.atom.tab_compact[it.lmax] != nullptr;
                d.tab = cmp ? it.atom.tab_compact[it.lmax] : it.atom.tab;
                for (int q = 0; q < 3; ++q) d.c[q] = it.atom.c[q];
                d.h = it.atom.h;
                d.inv_h = 1.0 / it.atom.h;
                d.r_max = it.atom.r_max;
                d.h2_over_6 = it.atom.h * it.atom.h / 6.0;
                d.n = it.atom.n;
                d.tile0 = g.tiles;
                tile0[k] = g.tiles;
                d.n_r = it.atom.n_r;
                d.ch = cmp ? it.lmax + 1 : it.atom.tab_lmax + 1;
                d.lmax = it.lmax;
                d.dtype = it.atom.dtype;
                g.tiles += (it.atom.n + tp - 1) / tp;
            }
            if (g.tiles > max_tiles()) return SH_EINVAL;
        }
        // launches of at most kInlineItems requests take their descriptors as arguments
        bool copy = false;
        for (const Group& g : groups_) copy = copy || g.end - g.first > shk::kInlineItems;
        hipError_t e = copy ? hipMemcpyAsync(s.dev, s.host, (sizeof(shk::ServeDesc) + sizeof(int64_t)) * n,
                                             hipMemcpyHostToDevice, s.stream)
                            : hipSuccess;
        const int64_t* dev_tile0 = reinterpret_cast<const int64_t*>(s.dev + n);
        // smallest output first, each launch's completion recorded, so the requests of
        // small groups complete without waiting for the large ones of the batch
        launch_order_.resize(groups_.size());
        for (size_t gi = 0; gi < groups_.size(); ++gi) launch_order_[gi] = int(gi);
        std::stable_sort(launch_order_.begin(), launch_order_.end(),
                         [&](int a, int b) { return groups_[a].bytes < groups_[b].bytes; });
        s.group_items.clear();
        s.group_end.clear();
        s.next = 0;
        for (size_t q = 0; q < launch_order_.size() && e == hipSuccess; ++q) {
            const Group& g = groups_[size_t(launch_order_[q])];
            const int b = g.first, m = g.end - g.first;
            const shk::ServeDesc& d = s.host[b];
            shk::ServeInline in;
            memset(&in, 0, sizeof(in));
            const bool inl = m <= shk::kInlineItems;
            if (inl) memcpy(in.d, s.host + b, sizeof(shk::ServeDesc) * m);
            const shk::ServeDesc* descs = inl ? nullptr : s.dev + b;
            const int64_t* t0 = inl ? nullptr : dev_tile0 + b;
            hipEvent_t ev = s.group_done[q];
            if (g.mixed) e = shk::launch_mixed(g.tiles, in, descs, t0, m, s.stream, ev);
            else if (d.dtype == SH_F64) e = shk::launch_group<double>(d.lmax, g.ppl, g.tiles, in, descs, t0, m, s.stream, ev);
            else e = shk::launch_group<float>(d.lmax, g.ppl, g.tiles, in, descs, t0, m, s.stream, ev);
            for (int k = b; k < b + m; ++k) s.group_items.push_back(order_[k]);
            s.group_end.push_back(int(s.group_items.size()));
        }
        if (e != hipSuccess) {
            // groups launched before the failure may still be writing into outputs the
            // scheduler is about to release: let them finish first
            (void)hipStreamSynchronize(s.stream);
            return SH_EHIP;
        }
        return SH_OK;
    }

    // The batch's last launch is its last group's, which completes that group's
    // event: the batch is complete when that event is.
    int query(int slot) override
    {
        const Slot& s = slots_[slot];
        if (s.group_end.empty()) return 1;
        const hipError_t e = hipEventQuery(s.group_done[s.group_end.size() - 1]);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        return -1;
    }

    // the groups launched so far complete in launch order (one stream)
    int progress(int slot, std::vector<int>& done) override
    {
        Slot& s = slots_[slot];
        while (s.next < int(s.group_end.size())) {
            const hipError_t e = hipEventQuery(s.group_done[s.next]);
            if (e == hipErrorNotReady) return 0;
            if (e != hipSuccess) return -1;
            for (int i = s.next ? s.group_end[s.next - 1] : 0; i < s.group_end[s.next]; ++i)
                done.push_back(s.group_items[i]);
            ++s.next;
        }
        return 1;  // every group's event has completed, the last one included
    }

private:
    static constexpr int64_t kMaxItems = 8192;
    // per slot: up to kMaxItems descriptors followed by as many first-tile indices
    static constexpr size_t kSlotBytes = (sizeof(shk::ServeDesc) + sizeof(int64_t)) * kMaxItems;
    // one launch per (dtype, lmax) group
    static constexpr int kMaxGroups = 2 * (SH_LMAX + 1);
    struct Slot {
        hipStream_t stream = nullptr;
        std::vector<hipEvent_t> group_done;  // recorded after each launch of a batch, in launch order
        std::vector<int> group_items;        // the batch's item indices, group by group in launch order
        std::vector<int> group_end;          // end of each group's items in group_items
        int next = 0;                        // first group not yet reported complete
        shk::ServeDesc* host = nullptr;
        shk::ServeDesc* dev = nullptr;
    };
    std::vector<Slot> slots_;
    void* arena_ = nullptr;
    std::vector<int> order_;                      // launch() scratch: items sorted by group
    // One launch of every kernel variant against a single empty request (n = 0, so
    // each block returns at once), at creation: the first launch of a kernel costs
    // far more than later ones, and a variant first used in the middle of serving
    // would stall that batch and every request queued behind it.
    hipError_t warm_up(Slot& s)
    {
        memset(s.host, 0, sizeof(shk::ServeDesc) + sizeof(int64_t));  // desc.n = 0, tile0[0] = 0
        hipError_t e = hipMemcpyAsync(s.dev, s.host, sizeof(shk::ServeDesc) + sizeof(int64_t),
                                      hipMemcpyHostToDevice, s.stream);
        const int64_t* tile0 = reinterpret_cast<const int64_t*>(s.dev + 1);
        shk::ServeInline in;
        memset(&in, 0, sizeof(in));
        if (e == hipSuccess) e = shk::launch_mixed(1, in, s.dev, tile0, 1, s.stream, nullptr);
        for (int lmax = 0; lmax <= SH_LMAX && e == hipSuccess; ++lmax) {
            for (const int ppl : {1, shk::group_ppl(SH_F64, lmax, shk::kServeVecPoints)})
                if (e == hipSuccess) e = shk::launch_group<double>(lmax, ppl, 1, in, s.dev, tile0, 1, s.stream, nullptr);
            for (const int ppl : {1, shk::group_ppl(SH_F32, lmax, shk::kServeVecPoints)})
                if (e == hipSuccess) e = shk::launch_group<float>(lmax, ppl, 1, in, s.dev, tile0, 1, s.stream, nullptr);
        }
        const hipError_t w = hipStreamSynchronize(s.stream);
        return e != hipSuccess ? e : w;
    }

    // one launch of a batch: one (dtype, lmax) group, or every one-point group (mixed)
    struct Group {
        int first, end;  // its items: order_[first .. end)
        int64_t tiles;   // tiles of the launch
        int64_t bytes;   // output bytes
        int ppl;         // points per lane
        bool mixed;      // the mixed kernel
    };
    std::vector<int> launch_order_;  // launch() scratch: launches, smallest output first
    std::vector<Group> groups_;      // launch() scratch
};

}  // namespace

std::unique_ptr<Executor> make_hip_executor(uint64_t budget, int n_slots, int* status)
{
    std::unique_ptr<Executor> ex(new HipExecutor(budget, n_slots, status));
    if (*status != SH_OK) ex.reset();
    return ex;
}

}  // namespace shs
