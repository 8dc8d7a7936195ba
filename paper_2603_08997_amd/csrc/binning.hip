// Tile binning: the depth-ordered per-tile lists of the tile-based rasteriser.
//
// The lists must hold, for every tile, the visible entries whose overlap box
// reaches the tile and that can reach alpha_min at one of its pixel centres
// (the exact tile test below), in ascending (depth, entry) order. Instead of one
// radix sort over 64-bit (tile << 32 | depth) keys, the stage sorts the
// visible entries once by depth (a short array), emits their (tile, entry)
// pairs in that order, and then sorts the pairs stably by tile alone. A
// stable sort keeps the depth order inside each tile, so the lists are the
// same as those of the 64-bit sort while the long pair array is sorted on
// ceil(log2(tiles)) bits instead of 32 + that many (uint16 keys when a batch
// has fewer than 65535 tiles).
#include <algorithm>

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
    const uint32_t* depth;
    uint32_t* dkey;
    uint32_t* dval;
    __device__ void operator()(int64_t e, uint32_t v, uint32_t pos) const {
        if (v) {
            dkey[pos] = depth[e];
            dval[pos] = (uint32_t)e;
        }
    }
};
struct PairCountSrc {  // tiles touched, in depth order (gathered by the depth sort)
    const uint32_t* tiles_sorted;
    const uint32_t* n_dev;
    __device__ int64_t count() const { return *n_dev; }
    __device__ uint32_t operator()(int64_t k) const { return tiles_sorted[k]; }
};
// Pair offset of every Gaussian in depth order, and for every emission window
// (kEmitWindow consecutive emission units, windows 0 .. n_windows) the
// Gaussian whose units hold the window's first unit. Gaussian k owns units
// [pos + kEmitHead k, pos + kEmitHead (k + 1) + v).
struct OffsetSink {
    uint32_t* offsets;
    uint32_t* window_first;
    uint32_t n_windows;
    __device__ void operator()(int64_t k, uint32_t v, uint32_t pos) const {
        offsets[k] = pos;
        const uint64_t first = (uint64_t)pos + (uint64_t)kEmitHead * (uint64_t)k;
        const uint64_t end = first + (uint64_t)kEmitHead + v;
        for (uint64_t w = (first + kEmitWindow - 1) / kEmitWindow;
             w <= n_windows && w * kEmitWindow < end; ++w)
            window_first[w] = (uint32_t)k;
    }
};

// Block sums of the scan input. Block 0 also zeroes `clear[0..nclear)` (the
// counters a binning pass accumulates into), saving a launch.
template <class Src>
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(Src src, uint32_t* sums,
                                                                   uint32_t* clear, int nclear) {
    __shared__ uint32_t smem[kScanThreads / 64 + 1];
    if (blockIdx.x == 0 && (int)threadIdx.x < nclear) clear[threadIdx.x] = 0u;
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

// Second and last kernel of the scan: every block adds up the sums of the
// blocks before it (a few thousand L2-resident words), scans its own tile and
// feeds the sink; the last block writes the grand total.
template <class Src, class Sink>
__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(Src src, Sink sink,
                                                                 const uint32_t* sums,
                                                                 uint32_t* total) {
    __shared__ uint32_t smem[kScanThreads / 64 + 1];
    uint32_t before = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += kScanThreads) before += sums[i];
    uint32_t prefix;
    block_excl_scan<kScanThreads>(before, smem, &prefix);
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
    uint32_t pos = block_excl_scan<kScanThreads>(s, smem, &tot) + prefix;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) sink(base + j, v[j], pos);
        pos += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = prefix + tot;
}

template <class Src, class Sink>
hipError_t device_scan(Src src, Sink sink, int64_t n_max, uint32_t* sums, uint32_t* total,
                       hipStream_t s, uint32_t* clear = nullptr, int nclear = 0) {
    const int nb = (int)((n_max + kScanTile - 1) / kScanTile);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(scan_reduce_kernel<Src>, dim3(nb), dim3(kScanThreads), 0, s, src, sums, clear,
                       nclear);
    hipLaunchKernelGGL((scan_down_kernel<Src, Sink>), dim3(nb), dim3(kScanThreads), 0, s, src,
                       sink, sums, total);
    return hipGetLastError();
}

// Exact tile test of one (tile, Gaussian) pair: can alpha' = o exp(-q/2),
// q = a dx^2 + 2 b dx dy + c dy^2, reach alpha_min at a pixel centre of the
// tile inside the overlap box? The pixel-centre rectangle of the tile is
// clipped to the box (widened by 1e-3 px). If the Gaussian's centre lies
// outside it, the minimum of the convex q over the rectangle lies on an edge
// that faces the centre (moving from any other boundary point towards the
// centre enters the rectangle and lowers q), at the clamped stationary point
// of that edge: at most one vertical and one horizontal edge to evaluate. The
// pair is kept when that minimum, less a bound on its rounding error (8 ulp of
// the sum of the terms' magnitudes), is within `lim` = 2 ln(o / alpha_min)
// inflated by 1% + 0.01 (formed once per Gaussian): a culled pair cannot pass
// the compositing kernels' skip test at any pixel of the tile, so images and
// gradients are those of the uncut lists.
__device__ __forceinline__ float reach_limit(float o, const RasterDev& rp) {
    return rp.alpha_min > 0.f ? 2.f * logf(o / rp.alpha_min) * 1.01f + 0.01f : INFINITY;
}

__device__ __forceinline__ bool tile_reachable(float u, float v, float a, float b, float c,
                                               float lim, float rx, float ry, int tx, int ty,
                                               const RasterDev& rp) {
    // relative to the centre; the box widened by 1e-3 px
    const float m = 1e-3f;
    const float bx = (float)(tx * rp.tile_w) - u, by = (float)(ty * rp.tile_h) - v;
    const float x0 = fmaxf(bx + 0.5f, -rx - m), x1 = fminf(bx + ((float)rp.tile_w - 0.5f), rx + m);
    const float y0 = fmaxf(by + 0.5f, -ry - m), y1 = fminf(by + ((float)rp.tile_h - 0.5f), ry + m);
    if (x0 > x1 || y0 > y1) return false;   // no pixel centre of the tile in the box
    const bool in_x = x0 <= 0.f && 0.f <= x1, in_y = y0 <= 0.f && 0.f <= y1;
    if (in_x && in_y) return true;
    if (lim == INFINITY) return true;
    constexpr float kErr = 8.f * 5.96046448e-8f;
    float best = INFINITY;
    auto at = [&](float dx, float dy) {
        const float bxy = b * dx * dy;
        const float q = a * dx * dx + 2.f * bxy + c * dy * dy;
        const float mag = a * dx * dx + 2.f * fabsf(bxy) + c * dy * dy;
        best = fminf(best, q - kErr * mag);
    };
    if (!in_x) {   // the vertical edge facing the centre
        const float ex = x0 > 0.f ? x0 : x1;
        at(ex, fminf(fmaxf(-b * ex * __builtin_amdgcn_rcpf(c), y0), y1));
    }
    if (!in_y) {   // the horizontal edge facing the centre
        const float ey = y0 > 0.f ? y0 : y1;
        at(fminf(fmaxf(-b * ey * __builtin_amdgcn_rcpf(a), x0), x1), ey);
    }
    return best <= lim;
}

// Pair emission, load balanced over emission units (a few header units per
// Gaussian, then one per pair): each workgroup takes a fixed window of
// kEmitTile consecutive units. The Gaussians (in depth order) whose units meet
// the window run from the one holding the window's first unit to the one
// holding the next window's first unit (both recorded by the offset scan); the
// header units bound their number, and so the LDS a workgroup needs (more
// workgroups in flight hide the dependent loads of each). Their tile
// rectangles are staged in LDS, a max-scan of their start positions gives
// every window position its Gaussian, and every thread expands its pairs to
// (tile, entry) with coalesced stores. Pair q of a Gaussian is
// tile (x0 + q % w, y0 + q / w) of its rectangle, row-major; pairs that fail
// the exact tile test get the all-ones key (kCulledTile, or kCulledTile16
// when the batch keeps uint16 tile keys).
constexpr int kEmitThreads = 256;
constexpr int kEmitItems = 4;
constexpr int kEmitTile = kEmitThreads * kEmitItems;
static_assert(kEmitTile == kEmitWindow, "emission window size");
// Gaussians meeting one window: each owns at least kEmitHead + 1 units.
constexpr int kEmitMaxG = kEmitTile / (kEmitHead + 1) + 2;

template <typename K>
__global__ void __launch_bounds__(kEmitThreads) emit_kernel(
    const uint32_t* __restrict__ sorted_entry, const uint32_t* __restrict__ offsets,
    const uint32_t* __restrict__ window_first, const float4* __restrict__ rec,
    uint32_t* __restrict__ counters, int64_t n, Views views, RasterDev rp,
    int64_t capacity, K* __restrict__ ptile, uint32_t* __restrict__ pentry) {
    __shared__ uint32_t s_off[kEmitMaxG];
    __shared__ uint32_t s_ent[kEmitMaxG];
    __shared__ uint32_t s_base[kEmitMaxG];   // global tile of the rectangle's first tile
    __shared__ uint16_t s_w[kEmitMaxG];      // rectangle width in tiles
    __shared__ uint16_t s_tx[kEmitMaxG];     // tiles per row of the Gaussian's view
    __shared__ uint16_t s_x0[kEmitMaxG];     // first tile column and row of the rectangle
    __shared__ uint16_t s_y0[kEmitMaxG];
    __shared__ float s_lim[kEmitMaxG];       // reach limit of the exact tile test
    __shared__ uint32_t s_own[kEmitTile];    // window position -> owning Gaussian
    __shared__ uint32_t s_scan[kEmitThreads / 64 + 1];
    // pairs written = min(pairs needed, capacity); block 0 records it and
    // flags an overflow (the tile sort reads the count after this kernel)
    const uint32_t total = counters[kPairs];
    const uint32_t P = (int64_t)total > capacity ? (uint32_t)capacity : total;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counters[kPairsWritten] = P;
        if ((int64_t)total > capacity) counters[kStatus] |= SGS_STATUS_PAIR_OVERFLOW;
    }
    const uint32_t nvis = counters[kVisible];
    const int win = blockIdx.x;
    const uint64_t c0 = (uint64_t)win * kEmitTile;   // first unit of the window
    const uint64_t units = (uint64_t)total + (uint64_t)kEmitHead * nvis;
    if (c0 >= units) return;   // uniform across the workgroup
    const int tid = threadIdx.x;
    const uint32_t k0 = window_first[win];
    // the next window's first Gaussian exists whenever units continue past
    // this window; otherwise the window ends with the last visible Gaussian
    const uint32_t k1 = c0 + kEmitTile < units ? window_first[win + 1] : nvis - 1u;
    const uint32_t cnt = k1 - k0 + 1u;
    if (k1 < k0 || cnt > (uint32_t)kEmitMaxG) return;   // cannot happen: the header bound
#pragma unroll
    for (int it = 0; it < kEmitItems; ++it) s_own[it * kEmitThreads + tid] = 0u;
    __syncthreads();
    for (uint32_t j = tid; j < cnt; j += kEmitThreads) {
        const uint32_t k = k0 + j;
        const uint32_t e = sorted_entry[k];
        const ViewDev& V = views.v[(int)(e / n)];
        const float4 r0 = rec[3 * (int64_t)e], r1 = rec[3 * (int64_t)e + 1];
        int x0, x1, y0, y1;
        tile_rect(r0.x, r0.y, (int)r1.z, (int)r1.w, rp.tile_w, rp.tile_h, V.tiles_x, V.tiles_y,
                  &x0, &x1, &y0, &y1);
        const uint32_t off = offsets[k];
        s_off[j] = off;
        s_ent[j] = e;
        s_base[j] = (uint32_t)(V.tile_offset + y0 * V.tiles_x + x0);
        s_w[j] = (uint16_t)(x1 - x0);
        s_tx[j] = (uint16_t)V.tiles_x;
        s_x0[j] = (uint16_t)x0;
        s_y0[j] = (uint16_t)y0;
        s_lim[j] = reach_limit(r1.y, rp);
        // mark where this Gaussian's units start inside the window
        const uint64_t first = (uint64_t)off + (uint64_t)kEmitHead * k;
        if (j > 0 && first - c0 < (uint64_t)kEmitTile) s_own[first - c0] = j;
    }
    __syncthreads();
    // owner of every window position = the last Gaussian starting at or
    // before it: inclusive max-scan of the start marks (thread t scans
    // positions kEmitItems t .. kEmitItems (t + 1) - 1, then the block
    // combines the per-thread maxima)
    {
        uint32_t run[kEmitItems];
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < kEmitItems; ++i) {
            m = max(m, s_own[tid * kEmitItems + i]);
            run[i] = m;
        }
        const uint32_t before = block_excl_max_scan<kEmitThreads>(m, s_scan);
#pragma unroll
        for (int i = 0; i < kEmitItems; ++i) s_own[tid * kEmitItems + i] = max(before, run[i]);
    }
    __syncthreads();
    // gather every item's record first (one round of memory latency), then
    // test and store; header units and units past the written pairs do nothing
    uint32_t own[kEmitItems], qq[kEmitItems], pp[kEmitItems];
    bool pair[kEmitItems];
    float4 g0[kEmitItems], g1[kEmitItems];
#pragma unroll
    for (int it = 0; it < kEmitItems; ++it) {
        const uint64_t c = c0 + (uint64_t)(it * kEmitThreads + tid);
        const uint32_t j = s_own[it * kEmitThreads + tid];
        const uint64_t first = (uint64_t)s_off[j] + (uint64_t)kEmitHead * (k0 + j);
        const bool is_pair = c < units && c >= first + (uint64_t)kEmitHead;
        const uint32_t q = is_pair ? (uint32_t)(c - first - (uint64_t)kEmitHead) : 0u;
        const uint32_t p = s_off[j] + q;
        own[it] = j;
        qq[it] = q;
        pp[it] = p;
        pair[it] = is_pair && p < P;
        if (pair[it]) {
            const int64_t e = s_ent[j];
            g0[it] = rec[3 * e];
            g1[it] = rec[3 * e + 1];
        }
    }
#pragma unroll
    for (int it = 0; it < kEmitItems; ++it) {
        if (!pair[it]) continue;
        const uint32_t j = own[it];
        const uint32_t q = qq[it], p = pp[it];
        const uint32_t w = s_w[j];
        // q / w and q % w through a float reciprocal, corrected to exact
        uint32_t qy = (uint32_t)((float)q * __builtin_amdgcn_rcpf((float)w));
        int32_t qx = (int32_t)(q - qy * w);
        while (qx < 0) { --qy; qx += (int32_t)w; }
        while (qx >= (int32_t)w) { ++qy; qx -= (int32_t)w; }
        const bool keep = tile_reachable(g0[it].x, g0[it].y, g0[it].z, g0[it].w, g1[it].x,
                                         s_lim[j], g1[it].z, g1[it].w, (int)s_x0[j] + qx,
                                         (int)(s_y0[j] + qy), rp);
        ptile[p] = keep ? (K)(s_base[j] + qy * s_tx[j] + (uint32_t)qx) : (K)~(K)0;
        pentry[p] = s_ent[j];
    }
}

// [start, end) of every tile by binary search in the sorted tile keys
// (empty tiles: [0, 0)).
template <typename K>
__global__ void __launch_bounds__(256) ranges_kernel(const K* __restrict__ ptile,
                                                     const uint32_t* __restrict__ counters,
                                                     int64_t total_tiles,
                                                     uint32_t* __restrict__ ranges) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total_tiles) return;
    const uint32_t P = counters[kPairsKept];
    uint32_t lo = 0, hi = P;
    while (lo < hi) {  // first key >= t
        const uint32_t mid = (lo + hi) >> 1;
        if (ptile[mid] < (uint32_t)t) lo = mid + 1; else hi = mid;
    }
    const uint32_t a = lo;
    hi = P;
    while (lo < hi) {  // first key > t
        const uint32_t mid = (lo + hi) >> 1;
        if (ptile[mid] <= (uint32_t)t) lo = mid + 1; else hi = mid;
    }
    const bool empty = lo == a;
    ranges[2 * t] = empty ? 0u : a;
    ranges[2 * t + 1] = empty ? 0u : lo;
}

// Counting sort of the tiles by cost >> shift, largest first, in one
// workgroup: bucket counts in LDS, their exclusive scan, then every tile takes
// the next slot of its bucket.
constexpr int kOrderThreads = 1024;
__global__ void __launch_bounds__(kOrderThreads) order_tiles_kernel(
    const uint32_t* __restrict__ cost, int64_t tiles, int shift, uint32_t* __restrict__ order,
    const int32_t* __restrict__ gate) {
    if (gate != nullptr && gate_closed(gate)) return;
    __shared__ uint32_t slot[kOrderThreads];
    __shared__ uint32_t smem[kOrderThreads / 64 + 1];
    const int tid = threadIdx.x;
    auto bucket = [&](int64_t t) {
        return (uint32_t)(kOrderThreads - 1) - min(cost[t] >> shift, (uint32_t)(kOrderThreads - 1));
    };
    slot[tid] = 0;
    __syncthreads();
    for (int64_t t = tid; t < tiles; t += kOrderThreads) atomicAdd(&slot[bucket(t)], 1u);
    __syncthreads();
    const uint32_t c = slot[tid];
    uint32_t tot;
    const uint32_t first = block_excl_scan<kOrderThreads>(c, smem, &tot);
    __syncthreads();
    slot[tid] = first;
    __syncthreads();
    for (int64_t t = tid; t < tiles; t += kOrderThreads)
        order[atomicAdd(&slot[bucket(t)], 1u)] = (uint32_t)t;
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
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
    uint32_t* window_first = reinterpret_cast<uint32_t*>(ws + L.window_first);
    uint32_t* sums = reinterpret_cast<uint32_t*>(ws + L.scan_sums);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.sort_hist);
    uint32_t* totals = reinterpret_cast<uint32_t*>(ws + L.sort_totals);
    uint32_t* ptile[2] = {reinterpret_cast<uint32_t*>(ws + L.pair_tile[0]),
                          reinterpret_cast<uint32_t*>(ws + L.pair_tile[1])};
    uint16_t* ptile16[2] = {reinterpret_cast<uint16_t*>(ws + L.pair_tile[0]),
                            reinterpret_cast<uint16_t*>(ws + L.pair_tile[1])};
    const bool key16 = L.tile_key_bytes == 2;
    uint32_t* pentry[2] = {reinterpret_cast<uint32_t*>(ws + L.pair_entry[0]),
                           reinterpret_cast<uint32_t*>(ws + L.pair_entry[1])};
    uint32_t* ranges = reinterpret_cast<uint32_t*>(ws + L.ranges);
    hipError_t err;

    // visible entries -> (depth, entry), entry order; count -> counters[kVisible]
    // (the first scan kernel also clears the counters binning and compositing
    // accumulate into)
    if (E == 0 && (err = fill_u32(counters + kVisible, kPairsKept + 1 - kVisible, 0u, s)) != hipSuccess)
        return err;
    if (E > 0) {
        err = device_scan(VisibleSrc{tiles, E},
                          CompactSink{reinterpret_cast<const uint32_t*>(ws + L.depth), dkey[0],
                                      dval[0]},
                          E, sums, counters + kVisible, s, counters + kVisible,
                          kPairsKept + 1 - kVisible);
        if (err != hipSuccess) return err;
        // stable sort by depth (ties keep ascending entry order); the last
        // pass also gathers each entry's tile count into `offsets`, in depth
        // order, for the scan below to read linearly and overwrite in place
        int res = 0;
        err = radix_sort(dkey, dval, counters + kVisible, E, 32, hist, totals, s, &res, nullptr,
                         tiles, offsets);
        if (err != hipSuccess) return err;
        // pair offsets in depth order; total -> counters[kPairs]
        const uint32_t n_windows = (uint32_t)emit_windows(E, L.capacity);
        err = device_scan(PairCountSrc{offsets, counters + kVisible},
                          OffsetSink{offsets, window_first, n_windows}, E, sums,
                          counters + kPairs, s);
        if (err != hipSuccess) return err;
        // at least one workgroup: block 0 also records the written pair count
        const dim3 egrid((unsigned)std::max<int64_t>(1, emit_windows(E, L.capacity)));
        if (key16)
            hipLaunchKernelGGL(emit_kernel<uint16_t>, egrid, dim3(kEmitThreads), 0, s, dval[res],
                               offsets, window_first, rec, counters, n, views, rp, L.capacity,
                               ptile16[0], pentry[0]);
        else
            hipLaunchKernelGGL(emit_kernel<uint32_t>, egrid, dim3(kEmitThreads), 0, s, dval[res],
                               offsets, window_first, rec, counters, n, views, rp, L.capacity,
                               ptile[0], pentry[0]);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        // stable sort of the pairs by tile; the first pass drops culled pairs
        // and counts the rest into counters[kPairsKept]
        int tres = 0;
        err = key16 ? radix_sort(ptile16, pentry, counters + kPairsWritten, L.capacity, L.tile_bits,
                                 hist, totals, s, &tres, counters + kPairsKept)
                    : radix_sort(ptile, pentry, counters + kPairsWritten, L.capacity, L.tile_bits,
                                 hist, totals, s, &tres, counters + kPairsKept);
        if (err != hipSuccess) return err;
    }
    const dim3 rgrid((unsigned)((L.total_tiles + 255) / 256));
    if (L.total_tiles > 0 && key16)
        hipLaunchKernelGGL(ranges_kernel<uint16_t>, rgrid, dim3(256), 0, s, ptile16[L.tile_result],
                           counters, L.total_tiles, ranges);
    else if (L.total_tiles > 0)
        hipLaunchKernelGGL(ranges_kernel<uint32_t>, rgrid, dim3(256), 0, s, ptile[L.tile_result],
                           counters, L.total_tiles, ranges);
    return hipGetLastError();
}

hipError_t launch_order_tiles(const uint32_t* cost, int64_t tiles, int shift, uint32_t* order,
                              const int32_t* gate, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(order_tiles_kernel, dim3(1), dim3(kOrderThreads), 0, s, cost, tiles, shift,
                       order, gate);
    return hipGetLastError();
}

}  // namespace sgs
