// sh_probe.hip -- store-pattern probes for the bandwidth measurements (libshprobe.so).
//
// Not part of the library's interface: bench.py times these kernels beside the
// forward kernel so that its HBM rate can be compared with what the same store
// pattern reaches without the harmonics' arithmetic, and with a plain fill.
//
//  shp_fill  one 16-byte store per lane over a contiguous buffer (the highest
//            write rate of the device).
//  shp_rows  the forward kernel's store pattern with no harmonics: each lane
//            loads two FP64 points (48 bytes) and writes `rows` rows of 16 bytes
//            (row r at out[r * ld + i]), 256 lanes per workgroup.  The rows can be
//            split over `split` workgroups per tile (1, 2, 4 or 8: each writes a
//            contiguous range of rows and reloads the tile's points), mapped to
//            the XCDs as `order` says:
//              0  workgroups of one row range on 8/split XCDs, each XCD walking
//                 one contiguous range of tiles (split 1: the forward kernel's
//                 XCD-contiguous order);
//              1  hardware order (tile b / split, range b % split), i.e. every XCD
//                 works on the same tiles at the same time;
//              k >= 2 (split 1 only)  8 << (k - 1) contiguous ranges of tiles,
//                 2^(k-1) per XCD, taken in turn by its workgroups (smaller write
//                 windows per range, more ranges).
//            `cap` reserves LDS to allow at most 2 workgroups per CU (cap 1, as the
//            forward kernel does below lmax 8) or 1 (cap 2, as it does in FP64 at
//            lmax 8 and 9); `mode` picks the store instruction: 0 global
//            store, 1.. buffer stores with cache-policy bits (see kAux).
//  shp_fwd_split  the lmax 9 FP64 forward kernel with its rows split the same
//            way: a workgroup evaluates only the harmonics of its row range.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_core.h"
#include "sh_fwd.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// cache-policy bits of the buffer-store variants: sc0 = 1, nt = 2, sc1 = 16
constexpr int kAux[] = {0, 0, 2, 1, 16, 17, 18, 3, 19};
constexpr int kModes = int(sizeof(kAux) / sizeof(kAux[0]));
constexpr size_t kCapLds = 54 * 1024;   // cap 1: at most 2 resident workgroups per CU
constexpr size_t kCapLds1 = 84 * 1024;  // cap 2: 1
__host__ inline size_t cap_lds(int cap) { return cap == 2 ? kCapLds1 : (cap ? kCapLds : 0); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, int(bytes), 0x00020000);
}

template <int MODE>
__device__ __forceinline__ void store16(double* row, uint32_t row_bytes, uint32_t boff, shk::double2_t v)
{
    if constexpr (MODE == 0) {
        *reinterpret_cast<shk::double2_t*>(reinterpret_cast<char*>(row) + boff) = v;
    } else {
        constexpr int aux = kAux[MODE];
        v4i w;
        __builtin_memcpy(&w, &v, 16);
        __builtin_amdgcn_raw_buffer_store_b128(w, rsrc(row, row_bytes), boff, 0, aux);
    }
}

// tile and row range of hardware workgroup b (grid = split * tiles, tiles % 8 == 0;
// for order >= 2, split == 1 and tiles % (8 << (order - 1)) == 0)
__device__ __forceinline__ void tile_of(uint32_t b, uint32_t tiles, int split, int order, uint32_t& tile,
                                        int& range)
{
    if (order == 1) {
        tile = b / uint32_t(split);
        range = int(b % uint32_t(split));
        return;
    }
    if (order >= 2) {
        // 8 << (order - 1) contiguous regions of tiles, 2^(order-1) per XCD, which
        // alternates between its regions workgroup by workgroup
        const uint32_t per_xcd = 1u << (order - 1), regions = 8u * per_xcd, len = tiles / regions;
        const uint32_t xcd = b % 8, k = b / 8;
        range = 0;
        tile = (xcd + 8u * (k % per_xcd)) * len + k / per_xcd;
        return;
    }
    const uint32_t xcd = b % 8, k = b / 8;
    range = int(xcd % uint32_t(split));
    const uint32_t sub = xcd / uint32_t(split);       // XCD within the range's 8/split XCDs
    const uint32_t per = tiles / (8 / uint32_t(split));  // tiles per XCD
    tile = sub * per + k;
}

template <int MODE>
__global__ __launch_bounds__(256) void fill_kernel(double* out, uint32_t bytes)
{
    const uint32_t off = (blockIdx.x * 256u + threadIdx.x) * 16u;
    const double v = double(off);
    store16<MODE>(out, bytes, off, shk::double2_t{v, v + 1.0});
}

template <int MODE>
__global__ __launch_bounds__(256) void rows_kernel(const double* __restrict__ xyz, double* __restrict__ out,
                                                   uint32_t tiles, int64_t ld, int rows, int split, int order)
{
    uint32_t tile;
    int range;
    tile_of(blockIdx.x, tiles, split, order, tile, range);
    const uint32_t i0 = (tile * 256u + threadIdx.x) * 2u;
    const double* p = xyz + 3 * size_t(i0);
    const shk::double2_t x = {p[0], p[3]}, y = {p[1], p[4]}, z = {p[2], p[5]};
    const int r0 = rows * range / split, r1 = rows * (range + 1) / split;
    const uint32_t boff = i0 * 8u, row_bytes = uint32_t(ld * 8);
    for (int r = r0; r < r1; ++r) {
        const double fr = double(r);
        store16<MODE>(out + int64_t(r) * ld, row_bytes, boff, x * fr + y + z);
    }
}

// Forward values of rows [R0, R1) only; the other rows' arithmetic is dead code
// once the sink drops their stores.
template <int R0, int R1>
__device__ __forceinline__ void fwd_rows(shk::double2_t x, shk::double2_t y, shk::double2_t z, shk::double2_t k,
                                         double* out, int64_t ld, uint32_t boff)
{
    shk::eval_unit<9, shk::double2_t>(x, y, z, k, [&](int r, shk::double2_t v) {
        if (r >= R0 && r < R1)
            *reinterpret_cast<shk::double2_t*>(reinterpret_cast<char*>(out + int64_t(r) * ld) + boff) = v;
    });
}

template <int S>
__global__ __launch_bounds__(256) void fwd_split_kernel(const double* __restrict__ xyz, double* __restrict__ out,
                                                        uint32_t tiles, int64_t ld, int order)
{
    uint32_t tile;
    int range;
    tile_of(blockIdx.x, tiles, S, order, tile, range);
    const uint32_t i0 = (tile * 256u + threadIdx.x) * 2u;
    shk::double2_t x, y, z, k;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        double xb, yb, zb, kb;
        shk::load_unit<shk::In::kXyz, double>(xyz, nullptr, i0 + q, xb, yb, zb, kb);
        x[q] = xb;
        y[q] = yb;
        z[q] = zb;
        k[q] = kb;
    }
    const uint32_t boff = i0 * 8u;
    shk::static_for<0, S>([&](auto gc) {
        constexpr int G = decltype(gc)::value;
        if (range == G) fwd_rows<100 * G / S, 100 * (G + 1) / S>(x, y, z, k, out, ld, boff);
    });
}

template <typename F>
hipError_t with_mode(int mode, F&& f)
{
    switch (mode) {
    case 0: return f(std::integral_constant<int, 0>{});
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
    }
}

bool split_ok(int split) { return split == 1 || split == 2 || split == 4 || split == 8; }

// orders 0 and 1 for any split; k in 2..6 with split 1 and whole tiles in every range
bool order_ok(int order, int split, int64_t n)
{
    if (order == 0 || order == 1) return true;
    if (order < 2 || order > 6 || split != 1) return false;
    const int64_t regions = int64_t(8) << (order - 1);
    return (n / 512) % regions == 0;
}

}  // namespace

extern "C" {

int shp_modes(void) { return kModes; }

// out: nbytes of device memory, nbytes a positive multiple of 4096; launches of
// at most 2^31 bytes each.
int shp_fill(void* out, int64_t nbytes, int mode, hipStream_t s)
{
    if (!out || nbytes <= 0 || nbytes % 4096 || mode < 0 || mode >= kModes) return 1;
    constexpr int64_t kPart = int64_t(1) << 31;
    for (int64_t o = 0; o < nbytes; o += kPart) {
        const int64_t nb = nbytes - o < kPart ? nbytes - o : kPart;
        char* base = static_cast<char*>(out) + o;
        const dim3 grid(unsigned(nb / 4096)), block(256);
        const hipError_t e = with_mode(mode, [&](auto mc) {
            hipLaunchKernelGGL(fill_kernel<decltype(mc)::value>, grid, block, 0, s, reinterpret_cast<double*>(base),
                               uint32_t(nb));
            return hipGetLastError();
        });
        if (e != hipSuccess) return 2;
    }
    return 0;
}

// xyz [n][3] double, out [rows][ld] double with ld >= n; n a positive multiple of
// 4096 (whole tiles of 512 points, a multiple of 8 tiles), ld * 8 < 2^32.
int shp_rows(const double* xyz, double* out, int64_t n, int64_t ld, int rows, int split, int order, int cap,
             int mode, hipStream_t s)
{
    if (!xyz || !out || n <= 0 || n % 4096 || ld < n || ld * 8 >= (int64_t(1) << 32) || rows < 1 || rows > 400 ||
        !split_ok(split) || !order_ok(order, split, n) || mode < 0 || mode >= kModes)
        return 1;
    const uint32_t tiles = uint32_t(n / 512);
    const dim3 grid(tiles * unsigned(split)), block(256);
    const hipError_t e = with_mode(mode, [&](auto mc) {
        hipLaunchKernelGGL(rows_kernel<decltype(mc)::value>, grid, block, cap_lds(cap), s, xyz, out, tiles, ld,
                           rows, split, order);
        return hipGetLastError();
    });
    return e == hipSuccess ? 0 : 2;
}

// The lmax 9 FP64 forward values of xyz [n][3] into out [100][ld] (same values as
// sh_eval), rows split over `split` workgroups per tile; n as for shp_rows.
int shp_fwd_split(const double* xyz, double* out, int64_t n, int64_t ld, int split, int order, int cap, hipStream_t s)
{
    if (!xyz || !out || n <= 0 || n % 4096 || ld < n || ld * 8 >= (int64_t(1) << 32) || !split_ok(split) ||
        !order_ok(order, split, n))
        return 1;
    const uint32_t tiles = uint32_t(n / 512);
    const dim3 grid(tiles * unsigned(split)), block(256);
    const size_t lds = cap_lds(cap);
    switch (split) {
    case 1: hipLaunchKernelGGL(fwd_split_kernel<1>, grid, block, lds, s, xyz, out, tiles, ld, order); break;
    case 2: hipLaunchKernelGGL(fwd_split_kernel<2>, grid, block, lds, s, xyz, out, tiles, ld, order); break;
    case 4: hipLaunchKernelGGL(fwd_split_kernel<4>, grid, block, lds, s, xyz, out, tiles, ld, order); break;
    default: hipLaunchKernelGGL(fwd_split_kernel<8>, grid, block, lds, s, xyz, out, tiles, ld, order); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // extern "C"
