// Tile binning: the depth-ordered per-tile lists of the tile-based rasteriser.
//
// The lists must hold, for every tile, the visible entries whose cut-off
// square reaches the tile, in ascending (depth, entry) order. Instead of one
// radix sort over 64-bit (tile << 32 | depth) keys, the stage sorts the
// visible entries once by depth (a short array), emits their (tile, entry)
// pairs in that order, and then sorts the pairs stably by tile alone. A
// stable sort keeps the depth order inside each tile, so the lists are the
// same as those of the 64-bit sort while the long pair array is sorted on
// ceil(log2(tiles)) bits instead of 32 + that many.
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// ---- sources and sinks of the two device-wide scans ----
struct VisibleSrc {  // 1 for every visible entry
    const uint32_t* tiles;
    int64_t n;
    __device__ int64_t count() const { return n; }
    __device__ uint32_t operator()(int64_t e) const { return tiles[e] ? 1u : 0u; }
};
struct CompactSink {  // visible entries -> (depth bits, entry), in entry order
    const uint32_t* tiles;
    const float4* rec;
    uint32_t* dkey;
    uint32_t* dval;
    __device__ void operator()(int64_t e, uint32_t v, uint32_t pos) const {
        if (v) {
            dkey[pos] = __float_as_uint(rec[3 * e + 1].w);
            dval[pos] = (uint32_t)e;
        }
    }
};
struct PairCountSrc {  // tiles touched, in depth order
    const uint32_t* tiles;
    const uint32_t* sorted_entry;
    const uint32_t* n_dev;
    __device__ int64_t count() const { return *n_dev; }
    __device__ uint32_t operator()(int64_t k) const { return tiles[sorted_entry[k]]; }
};
struct OffsetSink {
    uint32_t* offsets;
    __device__ void operator()(int64_t k, uint32_t, uint32_t pos) const { offsets[k] = pos; }
};

template <class Src>
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(Src src, uint32_t* sums) {
    __shared__ uint32_t smem[kScanThreads / 64 + 1];
    const int64_t n = src.count();
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) s += src(base + j);
    uint32_t tot;
    block_excl_scan<kScanThreads>(s, smem, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of the block sums in place (one block); *total = grand total.
__global__ void __launch_bounds__(1024) scan_sums_kernel(uint32_t* sums, int nb, uint32_t* total) {
    __shared__ uint32_t smem[1024 / 64 + 1];
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<1024>(v, smem, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

template <class Src, class Sink>
__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(Src src, Sink sink,
                                                                 const uint32_t* sums) {
    __shared__ uint32_t smem[kScanThreads / 64 + 1];
    const int64_t n = src.count();
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < n) ? src(base + j) : 0u;
        s += v[j];
    }
    uint32_t tot;
    uint32_t pos = block_excl_scan<kScanThreads>(s, smem, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) sink(base + j, v[j], pos);
        pos += v[j];
    }
}

template <class Src, class Sink>
hipError_t device_scan(Src src, Sink sink, int64_t n_max, uint32_t* sums, uint32_t* total,
                       hipStream_t s) {
    const int nb = (int)((n_max + kScanTile - 1) / kScanTile);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(scan_reduce_kernel<Src>, dim3(nb), dim3(kScanThreads), 0, s, src, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, sums, nb, total);
    hipLaunchKernelGGL((scan_down_kernel<Src, Sink>), dim3(nb), dim3(kScanThreads), 0, s, src,
                       sink, sums);
    return hipGetLastError();
}

// pairs = counters[kPairs]; written = min(pairs, capacity); flag overflow.
__global__ void capacity_kernel(uint32_t* counters, int64_t capacity) {
    const uint32_t p = counters[kPairs];
    if ((int64_t)p > capacity) {
        counters[kStatus] |= SGS_STATUS_PAIR_OVERFLOW;
        counters[kPairsWritten] = (uint32_t)capacity;
    } else {
        counters[kPairsWritten] = p;
    }
}

__global__ void __launch_bounds__(256) emit_kernel(const uint32_t* __restrict__ sorted_entry,
                                                   const uint32_t* __restrict__ offsets,
                                                   const float4* __restrict__ rec,
                                                   const uint32_t* __restrict__ counters,
                                                   int64_t n, Views views, RasterDev rp,
                                                   int64_t capacity, uint32_t* __restrict__ ptile,
                                                   uint32_t* __restrict__ pentry) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)counters[kVisible]) return;
    const uint32_t e = sorted_entry[k];
    const ViewDev& V = views.v[(int)(e / n)];
    const float4 r0 = rec[3 * (int64_t)e], r1 = rec[3 * (int64_t)e + 1];
    int x0, x1, y0, y1;
    tile_rect(r0.x, r0.y, (int)r1.z, rp.tile_w, rp.tile_h, V.tiles_x, V.tiles_y, &x0, &x1, &y0, &y1);
    int64_t off = offsets[k];
    for (int ty = y0; ty < y1; ++ty) {
        const uint32_t row = (uint32_t)(V.tile_offset + ty * V.tiles_x);
        for (int tx = x0; tx < x1; ++tx, ++off) {
            if (off < capacity) {
                ptile[off] = row + (uint32_t)tx;
                pentry[off] = e;
            }
        }
    }
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) ranges_kernel(const uint32_t* __restrict__ ptile,
                                                     const uint32_t* __restrict__ counters,
                                                     uint32_t* __restrict__ ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t P = counters[kPairsWritten];
    if (i >= P) return;
    const uint32_t t = ptile[i];
    if (i == 0 || ptile[i - 1] != t) ranges[2 * (int64_t)t] = (uint32_t)i;
    if (i == P - 1 || ptile[i + 1] != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
}

}  // namespace

hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_bin(const Views& views, const RasterDev& rp, int64_t n, const Layout& L,
                      char* ws, hipStream_t s) {
    const int64_t E = L.entries;
    uint32_t* counters = reinterpret_cast<uint32_t*>(ws + L.counters);
    uint32_t* tiles = reinterpret_cast<uint32_t*>(ws + L.tiles);
    const float4* rec = reinterpret_cast<const float4*>(ws + L.records);
    uint32_t* dkey[2] = {reinterpret_cast<uint32_t*>(ws + L.dkey[0]),
                         reinterpret_cast<uint32_t*>(ws + L.dkey[1])};
    uint32_t* dval[2] = {reinterpret_cast<uint32_t*>(ws + L.dval[0]),
                         reinterpret_cast<uint32_t*>(ws + L.dval[1])};
    uint32_t* offsets = reinterpret_cast<uint32_t*>(ws + L.offsets);
    uint32_t* sums = reinterpret_cast<uint32_t*>(ws + L.scan_sums);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.sort_hist);
    uint32_t* totals = reinterpret_cast<uint32_t*>(ws + L.sort_totals);
    uint32_t* ptile[2] = {reinterpret_cast<uint32_t*>(ws + L.pair_tile[0]),
                          reinterpret_cast<uint32_t*>(ws + L.pair_tile[1])};
    uint32_t* pentry[2] = {reinterpret_cast<uint32_t*>(ws + L.pair_entry[0]),
                           reinterpret_cast<uint32_t*>(ws + L.pair_entry[1])};
    uint32_t* ranges = reinterpret_cast<uint32_t*>(ws + L.ranges);
    hipError_t err;

    // visible entries -> (depth, entry), entry order; count -> counters[kVisible]
    if ((err = fill_u32(counters + kVisible, kEvaluated + 2 - kVisible, 0u, s)) != hipSuccess)
        return err;
    if (E > 0) {
        err = device_scan(VisibleSrc{tiles, E}, CompactSink{tiles, rec, dkey[0], dval[0]}, E, sums,
                          counters + kVisible, s);
        if (err != hipSuccess) return err;
        // stable sort by depth: ties keep ascending entry order
        int res = 0;
        err = radix_sort(dkey, dval, counters + kVisible, E, 32, hist, totals, s, &res);
        if (err != hipSuccess) return err;
        // pair offsets in depth order; total -> counters[kPairs]
        err = device_scan(PairCountSrc{tiles, dval[res], counters + kVisible}, OffsetSink{offsets},
                          E, sums, counters + kPairs, s);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(capacity_kernel, dim3(1), dim3(1), 0, s, counters, L.capacity);
        hipLaunchKernelGGL(emit_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s,
                           dval[res], offsets, rec, counters, n, views, rp, L.capacity, ptile[0],
                           pentry[0]);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        // stable sort of the pairs by tile
        int tres = 0;
        err = radix_sort(ptile, pentry, counters + kPairsWritten, L.capacity, L.tile_bits, hist,
                         totals, s, &tres);
        if (err != hipSuccess) return err;
    }
    if ((err = fill_u32(ranges, 2 * L.total_tiles, 0u, s)) != hipSuccess) return err;
    if (E > 0 && L.capacity > 0) {
        hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)((L.capacity + 255) / 256)), dim3(256), 0,
                           s, ptile[L.tile_result], counters, ranges);
    }
    return hipGetLastError();
}

}  // namespace sgs
