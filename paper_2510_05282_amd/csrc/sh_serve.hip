// sh_serve.hip -- HIP executor of the projector server: one batched kernel per
// batch on one of n_slots streams.
//
// A batch is a list of requests of any lmax and either dtype.  Each request is cut
// into tiles of kTilePoints points; block b handles tile b of the batch, finds its request by
// a wave-wide search over the requests' first-tile indices, and runs the same
// per-point projector evaluation as sh_projectors, dispatching once per block on
// the request's (dtype, lmax).  Request descriptors travel host -> device through
// a pinned staging buffer per slot (the slot is reused only after its previous
// batch has completed, so the staging buffer is never overwritten in flight).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "../../include/shmi.h"
#include "sh_core.h"
#include "sh_proj.h"
#include "sh_server.h"

namespace shk {

struct ServeDesc {
    const void* points;
    void* out;
    const double2* tab;
    double c[3];
    double h, inv_h, r_max, h2_over_6;
    int64_t n;
    int64_t tile0;  // first tile of this request within the batch
    int n_r;
    int ch;  // channels of the table (its lmax + 1)
    int lmax;
    int dtype;
};

template <int LMAX, typename TIO>
__device__ __forceinline__ void serve_point(const ServeDesc& d, int64_t j)
{
    const SplineGrid g{d.n_r, d.h, d.inv_h, d.r_max, d.h2_over_6};
    const TIO* p = static_cast<const TIO*>(d.points) + 3 * j;
    proj_point<LMAX, TIO>(double(p[0]), double(p[1]), double(p[2]), d.c, d.tab, d.ch, g,
                          static_cast<TIO*>(d.out) + j, d.n);
}

template <typename TIO>
__device__ __forceinline__ void serve_dispatch(const ServeDesc& d, int64_t j)
{
    switch (d.lmax) {
    case 0: serve_point<0, TIO>(d, j); break;
    case 1: serve_point<1, TIO>(d, j); break;
    case 2: serve_point<2, TIO>(d, j); break;
    case 3: serve_point<3, TIO>(d, j); break;
    case 4: serve_point<4, TIO>(d, j); break;
    case 5: serve_point<5, TIO>(d, j); break;
    case 6: serve_point<6, TIO>(d, j); break;
    case 7: serve_point<7, TIO>(d, j); break;
    case 8: serve_point<8, TIO>(d, j); break;
    case 9: serve_point<9, TIO>(d, j); break;
    default: break;
    }
}

constexpr int kServeBlock = 256;
constexpr int kTilePoints = 256;  // points per tile and block (a multiple of kServeBlock)

__global__ __launch_bounds__(kServeBlock) void serve_kernel(const ServeDesc* __restrict__ descs,
                                                            const int64_t* __restrict__ tile0, int n_items)
{
    // Tiles are dealt round-robin to the XCDs (no XCD-contiguous remap): the cost of
    // a tile varies ~100x with its request's lmax, and interleaving keeps the XCDs'
    // shares of a mixed batch even.
    const int64_t tile = blockIdx.x;
    // tile0 is increasing with tile0[0] = 0 <= tile, so the search finds an item
    const ServeDesc& d = descs[wave_search(tile0, n_items, tile)];
    const int64_t j0 = (tile - d.tile0) * kTilePoints + threadIdx.x;
    for (int q = 0; q < kTilePoints / kServeBlock; ++q) {
        const int64_t j = j0 + q * kServeBlock;
        if (j < 0 || j >= d.n) break;
        if (d.dtype == SH_F64) serve_dispatch<double>(d, j);
        else serve_dispatch<float>(d, j);
    }
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
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc(reinterpret_cast<void**>(&s.host), kSlotBytes) != hipSuccess ||
                hipMalloc(&s.dev, kSlotBytes) != hipSuccess) {
                (void)hipGetLastError();
                *status = SH_EHIP;
                return;
            }
        }
    }
    ~HipExecutor() override
    {
        for (Slot& s : slots_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.dev) (void)hipFree(s.dev);
            if (s.host) (void)hipHostFree(s.host);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
        }
        if (arena_) (void)hipFree(arena_);
    }
    int n_slots() const override { return int(slots_.size()); }
    int64_t max_items() const override { return kMaxItems; }
    // a dispatch counts its work-items in 32 bits: tiles * 256 < 2^32
    int64_t max_tiles() const override { return (int64_t(1) << 24) - 1; }
    int64_t tile_points() const override { return shk::kTilePoints; }
    void* arena_base() override { return arena_; }

    int launch(int slot, const std::vector<Item>& items) override
    {
        Slot& s = slots_[slot];
        int64_t* tile0 = reinterpret_cast<int64_t*>(s.host + kMaxItems);
        int64_t tiles = 0;
        for (size_t k = 0; k < items.size(); ++k) {
            const Item& it = items[k];
            shk::ServeDesc& d = s.host[k];
            memset(&d, 0, sizeof(d));
            d.points = it.atom.points;
            d.out = it.out;
            d.tab = static_cast<const double2*>(it.atom.tab);
            for (int q = 0; q < 3; ++q) d.c[q] = it.atom.c[q];
            d.h = it.atom.h;
            d.inv_h = 1.0 / it.atom.h;
            d.r_max = it.atom.r_max;
            d.h2_over_6 = it.atom.h * it.atom.h / 6.0;
            d.n = it.atom.n;
            d.tile0 = tiles;
            tile0[k] = tiles;
            d.n_r = it.atom.n_r;
            d.ch = it.atom.tab_lmax + 1;
            d.lmax = it.lmax;
            d.dtype = it.atom.dtype;
            tiles += (it.atom.n + shk::kTilePoints - 1) / shk::kTilePoints;
        }
        if (items.empty()) return SH_OK;
        if (tiles > max_tiles()) return SH_EINVAL;
        // descriptors, then the first-tile index array at a fixed offset
        hipError_t e = hipMemcpyAsync(s.dev, s.host, sizeof(shk::ServeDesc) * items.size(),
                                      hipMemcpyHostToDevice, s.stream);
        int64_t* dev_tile0 = reinterpret_cast<int64_t*>(s.dev + kMaxItems);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dev_tile0, tile0, sizeof(int64_t) * items.size(), hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(shk::serve_kernel, dim3(unsigned(tiles)), dim3(shk::kServeBlock), 0, s.stream, s.dev,
                               dev_tile0, int(items.size()));
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        return e == hipSuccess ? SH_OK : SH_EHIP;
    }

    int query(int slot) override
    {
        const hipError_t e = hipEventQuery(slots_[slot].done);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        return -1;
    }

private:
    static constexpr int64_t kMaxItems = 8192;
    // per slot: kMaxItems descriptors followed by kMaxItems first-tile indices
    static constexpr size_t kSlotBytes = (sizeof(shk::ServeDesc) + sizeof(int64_t)) * kMaxItems;
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        shk::ServeDesc* host = nullptr;
        shk::ServeDesc* dev = nullptr;
    };
    std::vector<Slot> slots_;
    void* arena_ = nullptr;
};

}  // namespace

std::unique_ptr<Executor> make_hip_executor(uint64_t budget, int n_slots, int* status)
{
    std::unique_ptr<Executor> ex(new HipExecutor(budget, n_slots, status));
    if (*status != SH_OK) ex.reset();
    return ex;
}

}  // namespace shs
