// Binning: the depth-ordered tile lists the tile-based rasteriser composites.
//
// The lists are built in two levels. First at the granularity of super-tiles
// (squares of S x S tiles): the stage sorts the visible entries once by depth
// (a short array), emits their (super-tile, entry) pairs in that order, and
// sorts the pairs stably by super-tile alone; stability keeps the depth order
// inside each super-tile, as a sort of 64-bit (super-tile << 32 | depth) keys
// would, on the bits of the super-tile index (the entry's tile rectangle
// inside the super-tile rides along in the key's upper bits). A super-tile's
// list holds the visible entries whose overlap box reaches it and that can
// reach alpha_min at one of its pixel centres.
//
// Then every super-tile list is split into the lists of its S x S tiles, in
// list order: per segment of a super-tile list, each pair's tile mask (the
// tiles of its rectangle on which the entry can reach alpha_min), per-tile
// counts, one scan over all (super-tile, tile, segment) counts for the list
// positions, and a stable scatter of the entries. A tile's list is therefore
// its depth-ordered list of entries whose overlap box reaches it and that can
// reach alpha_min on it; the sort never sees the (far more numerous) tile
// pairs.
//
// A tile composites only the front of its list, so a long super-tile list is
// split only in a prefix of its segments before compositing (a tile's list is
// then a prefix of its whole list). The compositing marks the tiles whose
// prefix ran out while pixels were still live; the completing split then
// splits the whole lists of their super-tiles after the prefix lists and
// points those tiles' ranges there, and the compositing resumes them.
#include <algorithm>

#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// ---- sources and sinks of the two device-wide scans ----
// The scans add in uint32 with saturation at 2^32 - 1 (saturating addition is
// associative, so the block and grand totals are the saturated true sums): a
// batch whose pair count does not fit ends with the all-ones total, which no
// capacity (< 2^31) reaches, and every offset past the overflow saturates.
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
struct PairCountSrc {  // super-tiles touched, in depth order (gathered by the depth sort)
    const uint32_t* counts_sorted;
    const uint32_t* n_dev;
    __device__ int64_t count() const { return *n_dev; }
    __device__ uint32_t operator()(int64_t k) const { return counts_sorted[k]; }
};
// Pair offset of every Gaussian in depth order, and for every emission window
// (kEmitWindow consecutive emission units, windows 0 .. n_windows) the
// Gaussian whose units hold the window's first unit. Gaussian k owns units
// [pos + kEmitHead k, pos + kEmitHead (k + 1) + v). A saturated offset lies
// beyond every window.
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

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
    const uint32_t c = a + b;
    return c < a ? 0xffffffffu : c;
}

// Inclusive saturating prefix sum over the lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_sat_scan(uint32_t v) {
    const int l = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (l >= d) v = sat_add(v, o);
    }
    return v;
}

// Exclusive saturating scan over a block of NT threads; *total = block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_sat_scan(uint32_t v, uint32_t* smem,
                                                        uint32_t* total) {
    constexpr int NW = NT / 64;
    const int w = threadIdx.x / 64;
    const int l = __lane_id();
    const uint32_t inc = wave_incl_sat_scan(v);
    if (l == 63) smem[w] = inc;
    __syncthreads();
    if (w == 0) {
        const uint32_t x = (l < NW) ? smem[l] : 0u;
        const uint32_t xi = wave_incl_sat_scan(x);
        const uint32_t ex = __shfl_up(xi, 1, 64);
        if (l < NW) smem[l] = l == 0 ? 0u : ex;
        if (l == NW - 1) smem[NW] = xi;
    }
    __syncthreads();
    // exclusive prefix of this thread = block prefix of its wave + the wave's
    // exclusive prefix (lane l - 1's inclusive value)
    const uint32_t wex = __shfl_up(inc, 1, 64);
    const uint32_t r = sat_add(smem[w], l == 0 ? 0u : wex);
    *total = smem[NW];
    __syncthreads();
    return r;
}

// Block sums of the scan input. Block 0 also zeroes `clear[0..nclear)` (the
// counters a binning pass accumulates into), saving a launch.
template <class Src>
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(Src src, uint32_t* sums,
                                                                   uint32_t* clear, int nclear) {
    __shared__ uint32_t smem[kScanThreads / 64 + 1];
    if (blockIdx.x == 0 && (int)threadIdx.x < nclear) clear[threadIdx.x] = 0u;
    const int64_t n = src.count();
    // blocks past the count (the grid covers a bound) contribute 0
    if ((int64_t)blockIdx.x * kScanTile >= n) {
        if (threadIdx.x == 0) sums[blockIdx.x] = 0u;
        return;
    }
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) s = sat_add(s, src(base + j));
    uint32_t tot;
    block_excl_sat_scan<kScanThreads>(s, smem, &tot);
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
    const int64_t n = src.count();
    // blocks past the count have nothing to feed; the last one still writes
    // the total
    const bool last = blockIdx.x == gridDim.x - 1;
    if ((int64_t)blockIdx.x * kScanTile >= n && !last) return;
    uint32_t before = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += kScanThreads) before = sat_add(before, sums[i]);
    uint32_t prefix;
    block_excl_sat_scan<kScanThreads>(before, smem, &prefix);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < n) ? src(base + j) : 0u;
        s = sat_add(s, v[j]);
    }
    uint32_t tot;
    uint32_t pos = sat_add(block_excl_sat_scan<kScanThreads>(s, smem, &tot), prefix);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) sink(base + j, v[j], pos);
        pos = sat_add(pos, v[j]);
    }
    if (last && threadIdx.x == 0) *total = sat_add(prefix, tot);
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

// Reach limit of a super-tile: the tile test's limit (reach_limit) widened by
// 1e-3 (1 + lim), more than twice the rounding bound of either evaluation, so
// that an entry the compositing forward's tile test keeps on any tile of the
// super-tile is never dropped from the super-tile's list (the minimum over
// the super-tile's pixels is at most the minimum over one tile's).
__device__ __forceinline__ float super_limit(float lim) {
    return lim == INFINITY ? lim : lim + 1e-3f * (1.f + fabsf(lim));
}

// Pair emission, load balanced over emission units (a few header units per
// Gaussian, then one per pair): each workgroup takes a fixed window of
// kEmitTile consecutive units. The Gaussians (in depth order) whose units meet
// the window run from the one holding the window's first unit to the one
// holding the next window's first unit (both recorded by the offset scan); the
// header units bound their number, and so the LDS a workgroup needs (more
// workgroups in flight hide the dependent loads of each). Their super-tile
// rectangles are staged in LDS, a max-scan of their start positions gives
// every window position its Gaussian, and every thread expands its pairs to
// (key, entry) with coalesced stores. Pair q of a Gaussian is super-tile
// (x0 + q % w, y0 + q / w) of its super-tile rectangle, row-major; its key
// packs the super-tile index and the part of the Gaussian's tile rectangle
// inside that super-tile. With alpha_min > 0, pairs whose Gaussian cannot
// reach alpha_min on the super-tile's pixels in the image get the all-ones
// key (kCulledTile).
constexpr int kEmitThreads = 256;
constexpr int kEmitItems = 4;
constexpr int kEmitTile = kEmitThreads * kEmitItems;
static_assert(kEmitTile == kEmitWindow, "emission window size");
// Gaussians meeting one window: each owns at least kEmitHead + 1 units.
constexpr int kEmitMaxG = kEmitTile / (kEmitHead + 1) + 2;

__global__ void __launch_bounds__(kEmitThreads) emit_kernel(
    const uint32_t* __restrict__ sorted_entry, const uint32_t* __restrict__ offsets,
    const uint32_t* __restrict__ window_first, const float4* __restrict__ rec,
    uint32_t* __restrict__ counters, int64_t n, const Views* __restrict__ views, RasterDev rp,
    int64_t capacity, uint32_t* __restrict__ pkey, uint32_t* __restrict__ pentry) {
    __shared__ uint32_t s_off[kEmitMaxG];
    __shared__ uint32_t s_ent[kEmitMaxG];
    __shared__ uint32_t s_base[kEmitMaxG];   // global super-tile of the rectangle's first one
    __shared__ uint16_t s_w[kEmitMaxG];      // rectangle width in super-tiles
    __shared__ uint16_t s_tx[kEmitMaxG];     // super-tiles per row of the Gaussian's view
    __shared__ uint16_t s_x0[kEmitMaxG];     // first super-tile column and row of the rectangle
    __shared__ uint16_t s_y0[kEmitMaxG];
    __shared__ uint16_t s_iw[kEmitMaxG];     // image size of the Gaussian's view
    __shared__ uint16_t s_ih[kEmitMaxG];
    __shared__ uint16_t s_tr[kEmitMaxG][4];  // tile rectangle [x0, x1) x [y0, y1)
    __shared__ float s_lim[kEmitMaxG];       // reach limit on a super-tile
    __shared__ float4 s_r0[kEmitMaxG];       // record words u v a b, c o rx ry
    __shared__ float4 s_r1[kEmitMaxG];
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
        const ViewDev& V = views->v[(int)(e / n)];
        const float4 r0 = rec[3 * (int64_t)e], r1 = rec[3 * (int64_t)e + 1];
        int x0, x1, y0, y1, sx0, sx1, sy0, sy1;
        tile_rect(r0.x, r0.y, (int)r1.z, (int)r1.w, rp.tile_w, rp.tile_h, V.tiles_x, V.tiles_y,
                  &x0, &x1, &y0, &y1);
        super_rect(x0, x1, y0, y1, rp.super_tile, &sx0, &sx1, &sy0, &sy1);
        const uint32_t off = offsets[k];
        s_off[j] = off;
        s_ent[j] = e;
        s_base[j] = (uint32_t)(V.sup_offset + sy0 * V.sup_x + sx0);
        s_w[j] = (uint16_t)(sx1 - sx0);
        s_tx[j] = (uint16_t)V.sup_x;
        s_x0[j] = (uint16_t)sx0;
        s_y0[j] = (uint16_t)sy0;
        s_iw[j] = (uint16_t)V.width;
        s_ih[j] = (uint16_t)V.height;
        s_tr[j][0] = (uint16_t)x0;
        s_tr[j][1] = (uint16_t)x1;
        s_tr[j][2] = (uint16_t)y0;
        s_tr[j][3] = (uint16_t)y1;
        s_lim[j] = super_limit(reach_limit(r1.y, rp));
        s_r0[j] = r0;
        s_r1[j] = r1;
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
    // test and store every item (the records were staged in LDS once per
    // Gaussian); header units and units past the written pairs do nothing
#pragma unroll
    for (int it = 0; it < kEmitItems; ++it) {
        const uint64_t c = c0 + (uint64_t)(it * kEmitThreads + tid);
        const uint32_t j = s_own[it * kEmitThreads + tid];
        const uint64_t first = (uint64_t)s_off[j] + (uint64_t)kEmitHead * (k0 + j);
        const bool is_pair = c < units && c >= first + (uint64_t)kEmitHead;
        const uint32_t q = is_pair ? (uint32_t)(c - first - (uint64_t)kEmitHead) : 0u;
        const uint32_t p = s_off[j] + q;
        if (!is_pair || p >= P) continue;
        const float4 g0 = s_r0[j], g1 = s_r1[j];
        const uint32_t w = s_w[j];
        // q / w and q % w through a float reciprocal, corrected to exact
        uint32_t qy = (uint32_t)((float)q * __builtin_amdgcn_rcpf((float)w));
        int32_t qx = (int32_t)(q - qy * w);
        while (qx < 0) { --qy; qx += (int32_t)w; }
        while (qx >= (int32_t)w) { ++qy; qx -= (int32_t)w; }
        // the super-tile's pixels inside the image
        const int sw = rp.super_tile * rp.tile_w, sh = rp.super_tile * rp.tile_h;
        const int px0 = ((int)s_x0[j] + qx) * sw, py0 = ((int)s_y0[j] + (int)qy) * sh;
        const bool keep = s_lim[j] == INFINITY ||
                          rect_reachable(g0.x, g0.y, g0.z, g0.w, g1.x, s_lim[j], g1.z, g1.w, px0,
                                         py0, min(sw, (int)s_iw[j] - px0),
                                         min(sh, (int)s_ih[j] - py0));
        // the tile rectangle inside the super-tile, relative to its first tile
        const int S = rp.super_tile;
        const int ox = ((int)s_x0[j] + qx) * S, oy = ((int)s_y0[j] + (int)qy) * S;
        const uint32_t lx0 = (uint32_t)(max((int)s_tr[j][0], ox) - ox);
        const uint32_t lx1 = (uint32_t)(min((int)s_tr[j][1], ox + S) - 1 - ox);
        const uint32_t ly0 = (uint32_t)(max((int)s_tr[j][2], oy) - oy);
        const uint32_t ly1 = (uint32_t)(min((int)s_tr[j][3], oy + S) - 1 - oy);
        const int rb = rp.rect_bits;
        const uint32_t rect = lx0 | (lx1 << rb) | (ly0 << (2 * rb)) | (ly1 << (3 * rb));
        const uint32_t sup = s_base[j] + qy * s_tx[j] + (uint32_t)qx;
        pkey[p] = keep ? (sup | (rect << rp.key_bits)) : kCulledTile;
        pentry[p] = s_ent[j];
    }
}

// [start, end) of every super-tile by binary search in the sorted keys
// (the super-tile index is the low key_bits bits; empty super-tiles: [0, 0)).
__global__ void __launch_bounds__(256) ranges_kernel(const uint32_t* __restrict__ pkey,
                                                     const uint32_t* __restrict__ counters,
                                                     int64_t total_supers, int key_bits,
                                                     uint32_t* __restrict__ ranges) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total_supers) return;
    const uint32_t mask = (uint32_t)((1ull << key_bits) - 1ull);
    const uint32_t P = counters[kPairsKept];
    uint32_t lo = 0, hi = P;
    while (lo < hi) {  // first key >= t
        const uint32_t mid = (lo + hi) >> 1;
        if ((pkey[mid] & mask) < (uint32_t)t) lo = mid + 1; else hi = mid;
    }
    const uint32_t a = lo;
    hi = P;
    while (lo < hi) {  // first key > t
        const uint32_t mid = (lo + hi) >> 1;
        if ((pkey[mid] & mask) <= (uint32_t)t) lo = mid + 1; else hi = mid;
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

// The call's view table into the workspace, word by word: the views passed
// by value or, with a camera table, its entry *d_view (clamped into range) as
// view 0 of a one-view batch (table entries are stored for that position).
__global__ void __launch_bounds__(64) store_views_kernel(Views v, const ViewDev* __restrict__ table,
                                                         int n_table,
                                                         const int32_t* __restrict__ d_view,
                                                         Views* __restrict__ dst) {
    static_assert(sizeof(Views) % 4 == 0 && sizeof(ViewDev) % 4 == 0, "word copy");
    constexpr int kWords = (int)(sizeof(Views) / 4), kViewWords = (int)(sizeof(ViewDev) / 4);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&v);
    const uint32_t* sel = nullptr;
    if (table != nullptr) {
        const int i = min(max(*d_view, 0), n_table - 1);
        sel = reinterpret_cast<const uint32_t*>(table + i);
    }
    uint32_t* out = reinterpret_cast<uint32_t*>(dst);
    for (int w = threadIdx.x; w < kWords; w += 64)
        out[w] = (sel != nullptr && w < kViewWords) ? sel[w] : src[w];
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---- the split of the super-tile lists into tile lists ----

__device__ __forceinline__ uint32_t list_segments(const uint32_t* ranges, int64_t s) {
    const uint32_t len = ranges[2 * s + 1] - ranges[2 * s];
    return (uint32_t)((len + kSegPairs - 1) / kSegPairs);
}
// Segments of every super-tile's list split before compositing (the scan
// numbers them): all, or the first `prefix` of a long list.
struct SegCountSrc {
    const uint32_t* ranges;
    int64_t n;
    uint32_t prefix;   // 0: all
    __device__ int64_t count() const { return n; }
    __device__ uint32_t operator()(int64_t s) const {
        return split_segments(list_segments(ranges, s), prefix);
    }
};
// The completing split: every segment of the super-tiles flagged in
// sup_redo, none of the others; nothing unless *redo is set.
struct RestSegSrc {
    const uint32_t* ranges;
    const uint32_t* sup_redo;
    const uint32_t* redo;
    int64_t n;
    __device__ int64_t count() const { return *redo ? n : 0; }
    __device__ uint32_t operator()(int64_t s) const {
        return sup_redo[s] ? list_segments(ranges, s) : 0u;
    }
};
// (super-tile, tile, segment) counts, in that order, for the list positions.
struct ItemCountSrc {
    const uint32_t* cnt;
    const uint32_t* n_seg;
    int tt;
    __device__ int64_t count() const { return (int64_t)*n_seg * tt; }
    __device__ uint32_t operator()(int64_t i) const { return cnt[i]; }
};
struct ItemOffSink {
    uint32_t* off;
    const uint32_t* base;   // nullable: list positions start there (after the prefix lists)
    __device__ void operator()(int64_t k, uint32_t, uint32_t pos) const {
        off[k] = base != nullptr ? sat_add(pos, *base) : pos;
    }
};

// Tile-list entries of both splits (saturating).
__device__ __forceinline__ uint32_t items_total(const uint32_t* counters) {
    return sat_add(counters[kItems], counters[kItemsRest]);
}

// Exclusive saturating scan of the segment counts of all super-tiles in one
// workgroup (a few hundred to a few ten thousand counts): first[s] for every
// super-tile and the total in first[n].
constexpr int kSegScanThreads = 1024;
constexpr int kSegScanItems = 4;
template <class Src>
__global__ void __launch_bounds__(kSegScanThreads) seg_scan_kernel(Src src, uint32_t* first) {
    __shared__ uint32_t smem[kSegScanThreads / 64 + 1];
    const int64_t n = src.count();
    constexpr int64_t kChunk = (int64_t)kSegScanThreads * kSegScanItems;
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
        const int64_t base = c0 + (int64_t)threadIdx.x * kSegScanItems;
        uint32_t v[kSegScanItems], sum = 0;
#pragma unroll
        for (int j = 0; j < kSegScanItems; ++j) {
            v[j] = base + j < n ? src(base + j) : 0u;
            sum = sat_add(sum, v[j]);
        }
        uint32_t tot;
        uint32_t pos = sat_add(carry, block_excl_sat_scan<kSegScanThreads>(sum, smem, &tot));
#pragma unroll
        for (int j = 0; j < kSegScanItems; ++j) {
            if (base + j < n) first[base + j] = pos;
            pos = sat_add(pos, v[j]);
        }
        carry = sat_add(carry, tot);
    }
    if (threadIdx.x == 0) first[src.n] = carry;
}

// Segment g of the split: super-tile s (global index), segment k of nseg in
// its list, pairs [a, b), the super-tile's first tile (tx0, ty0) in its view.
struct Segment {
    int s;
    uint32_t k, nseg, a, b;
    int tx0, ty0;
    const ViewDev* V;
};

__device__ __forceinline__ bool locate_segment(const Views* views, const uint32_t* seg_first,
                                               const uint32_t* sup_ranges, int S, uint32_t g,
                                               Segment* out) {
    const int ns = views->total_supers;
    if (g >= seg_first[ns]) return false;
    int lo = 0, hi = ns;   // first super-tile whose first segment lies past g
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (seg_first[mid] <= g) lo = mid + 1; else hi = mid;
    }
    const int s = lo - 1;
    int vi = 0;
    while (vi + 1 < views->n && s >= views->v[vi + 1].sup_offset) ++vi;
    const ViewDev* V = &views->v[vi];
    const int ls = s - V->sup_offset;
    out->s = s;
    out->k = g - seg_first[s];
    out->nseg = seg_first[s + 1] - seg_first[s];
    out->a = sup_ranges[2 * s] + out->k * (uint32_t)kSegPairs;
    out->b = min(sup_ranges[2 * s + 1], out->a + (uint32_t)kSegPairs);
    out->tx0 = (ls % V->sup_x) * S;
    out->ty0 = (ls / V->sup_x) * S;
    out->V = V;
    return true;
}

// Orders this wave's LDS accesses before and after (the lanes of one wave
// exchange data through their own rows of the LDS arrays).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t m) {
    uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        lo |= (uint32_t)__shfl_xor((int)lo, d, 64);
        hi |= (uint32_t)__shfl_xor((int)hi, d, 64);
    }
    return (uint64_t)__builtin_amdgcn_readfirstlane(lo) |
           ((uint64_t)__builtin_amdgcn_readfirstlane(hi) << 32);
}

// Transpose of the 64 x 64 bit matrix whose row l is lane l's word: returns,
// in lane t, the word whose bit l is bit t of lane l's input. Six stages
// swap the off-diagonal blocks of size 32, 16, ..., 1: a lane in the upper
// half of a block pair keeps its bits of the left half and takes its
// partner's left-half bits into the right half, and the other way round.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x) {
    const int l = __lane_id();
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    {
        const uint32_t plo = (uint32_t)__shfl_xor((int)lo, 32, 64);
        const uint32_t phi = (uint32_t)__shfl_xor((int)hi, 32, 64);
        const bool up = (l & 32) != 0;
        lo = up ? phi : lo;
        hi = up ? hi : plo;
    }
    constexpr uint32_t kKeep[5] = {0x0000ffffu, 0x00ff00ffu, 0x0f0f0f0fu, 0x33333333u,
                                   0x55555555u};
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const int j = 16 >> i;
        const uint32_t M = kKeep[i];
        const bool up = (l & j) != 0;
        const uint32_t plo = (uint32_t)__shfl_xor((int)lo, j, 64);
        const uint32_t phi = (uint32_t)__shfl_xor((int)hi, j, 64);
        const uint32_t slo = up ? (plo >> j) : (plo << j), shi = up ? (phi >> j) : (phi << j);
        lo = up ? ((lo & ~M) | (slo & M)) : ((lo & M) | (slo & ~M));
        hi = up ? ((hi & ~M) | (shi & M)) : ((hi & M) | (shi & ~M));
    }
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

constexpr int kSplitWaves = 4;
constexpr int64_t kSplitBlocks = 2048;   // blocks of the split kernels' grid-stride loops

// Reach of one entry by rows: q = a dx^2 + 2 b dx dy + c dy^2 <= lim is, for
// dy fixed, the interval |dx - s dy| <= sqrt((lim - k dy^2) / a) (s = -b/a,
// k = det/a, det = ac - b^2), so over a band of rows its right end is largest
// at the band point nearest the dy of the ellipse's rightmost point,
// dy_r = -b sqrt(lim / (c det)) (the right end is concave in dy), and its left
// end smallest at -dy_r. Formed once per entry, in float, with margins that
// keep the test conservative: det by Kahan's fused form (error a few ulp of
// det); lim raised by a bound on the rounding of the compositing kernels' own
// float evaluation of q (16 ulp of its terms' magnitudes, at most
// 2 (a + c)^2 lim / det on the ellipse); every interval end widened by 1e-3 px
// plus the worst effect of the rounding of lim - k dy^2 near the ellipse's
// top or bottom, sqrt(4 eps lim / a), plus relative rounding.
struct Reach {
    float s, k, inv_a, lim, ym, dyr, slack;
    bool conic;   // false: no reach limit or a degenerate conic (box only)
};

// (The hardware reciprocal and square root, 1 ulp each, are covered by the
// relative margins.)
__device__ __forceinline__ Reach make_reach(float a, float b, float c, float lim) {
    Reach r;
    const float bb = b * b;
    const float det = fmaf(a, c, -bb) - fmaf(b, b, -bb);
    r.conic = lim != INFINITY && a > 0.f && c > 0.f && det > 0.f;
    const float inv_det = __builtin_amdgcn_rcpf(det);
    const float ac = a + c;
    r.lim = lim * (1.f + 2e-6f * (ac * ac * inv_det));
    r.conic = r.conic && r.lim < INFINITY;
    r.inv_a = __builtin_amdgcn_rcpf(a);
    r.s = -b * r.inv_a;
    r.k = det * r.inv_a;
    r.ym = __builtin_amdgcn_sqrtf(r.lim * a * inv_det) * (1.f + 1e-5f) + 1e-3f;
    r.dyr = -b * __builtin_amdgcn_sqrtf(r.lim * __builtin_amdgcn_rcpf(c) * inv_det);
    r.slack = 1e-3f + 2.f * __builtin_amdgcn_sqrtf(4.8e-7f * r.lim * r.inv_a);
    return r;
}

// Tile columns [*c0, *c1] (view tile indices; *c0 > *c1: none) of the tiles in
// the row band of pixel rows [py0, py0 + h) that hold a pixel centre inside
// the overlap box (widened by 1e-3 px) within the entry's reach; tile width
// 2^tw_log2.
__device__ __forceinline__ void band_columns(const Reach& R, float u, float v, float rx, float ry,
                                             int py0, int h, int tw_log2, int width, int* c0,
                                             int* c1) {
    const float m = 1e-3f;
    float lo = fmaxf((float)py0 + 0.5f - v, -ry - m);
    float hi = fminf((float)(py0 + h) - 0.5f - v, ry + m);
    float xl = -rx - m, xr = rx + m;
    if (R.conic) {
        lo = fmaxf(lo, -R.ym);
        hi = fminf(hi, R.ym);
        const float y1 = fminf(fmaxf(R.dyr, lo), hi), y2 = fminf(fmaxf(-R.dyr, lo), hi);
        const float h1 = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-R.k * y1, y1, R.lim), 0.f) * R.inv_a);
        const float h2 = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-R.k * y2, y2, R.lim), 0.f) * R.inv_a);
        const float t1 = R.s * y1, t2 = R.s * y2;
        const float rel = 1e-5f * (fabsf(t1) + fabsf(t2) + h1 + h2);
        xl = fmaxf(xl, t2 - h2 - R.slack - rel);
        xr = fminf(xr, t1 + h1 + R.slack + rel);
    }
    *c0 = 1;
    *c1 = 0;
    if (!(lo <= hi) || !(xl <= xr)) return;
    // pixel columns whose centre lies in [u + xl, u + xr] (the sums' rounding,
    // below an ulp of |u| + |x|, widened away)
    const float ru = 2.4e-7f * (fabsf(u) + fabsf(xl) + fabsf(xr));
    const float fl = fmaxf(ceilf(u + xl - 0.5f - ru), 0.f);
    const float fr = fminf(floorf(u + xr - 0.5f + ru), (float)(width - 1));
    if (!(fl <= fr)) return;
    *c0 = (int)fl >> tw_log2;
    *c1 = (int)fr >> tw_log2;
}

// Tile masks and per-tile counts of one segment per wave. A pair's mask has
// bit (y S + x) for tile (x, y) of its super-tile when the tile lies in the
// pair's tile rectangle and, with alpha_min > 0, the entry can reach alpha_min
// on the tile's pixels in the image (row by row of the rectangle: the tile
// columns of each row band the entry reaches).
//
// With `local` (at most kLocalSupers super-tiles) every workgroup first forms
// the segment index (the exclusive scan of src over the super-tiles) in LDS,
// and workgroup 0 also stores it for the kernels after this one, which saves
// the scan's own launch; otherwise seg_first holds it already.
constexpr int kLocalSupers = 1024;
template <class Src>
__global__ void __launch_bounds__(kSplitWaves * 64) split_count_kernel(
    const Views* __restrict__ views, RasterDev rp, Src src, bool local,
    uint32_t* __restrict__ seg_first_g, const uint32_t* __restrict__ sup_ranges,
    const uint32_t* __restrict__ skey, const uint32_t* __restrict__ sentry,
    const float4* __restrict__ rec, uint32_t entries, uint64_t* __restrict__ mask,
    uint32_t* __restrict__ seg_cnt) {
    constexpr int NT = kSplitWaves * 64;
    __shared__ uint32_t s_first[kLocalSupers + 1];
    __shared__ uint32_t s_scan[NT / 64 + 1];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int S = rp.super_tile, TT = S * S;
    const uint32_t* seg_first = seg_first_g;
    if (local) {   // uniform
        const int ns = views->total_supers;
        const bool on = src.count() > 0;
        uint32_t carry = 0;
        for (int s0 = 0; s0 < ns; s0 += NT) {
            const int s = s0 + (int)threadIdx.x;
            const uint32_t v = (on && s < ns) ? src(s) : 0u;
            uint32_t tot;
            const uint32_t ex = sat_add(carry, block_excl_sat_scan<NT>(v, s_scan, &tot));
            if (s < ns) s_first[s] = ex;
            carry = sat_add(carry, tot);
        }
        if (threadIdx.x == 0) s_first[ns] = carry;
        __syncthreads();
        if (blockIdx.x == 0)
            for (int s = threadIdx.x; s <= ns; s += NT) seg_first_g[s] = s_first[s];
        seg_first = s_first;
    }
    // segments in a grid-stride loop (the grid is sized for the machine, not
    // for the capacity's bound on the segment count)
    for (uint32_t g = blockIdx.x * kSplitWaves + w;; g += gridDim.x * kSplitWaves) {
        Segment sg;
        if (!locate_segment(views, seg_first, sup_ranges, S, g, &sg)) return;   // uniform
        const ViewDev& V = *sg.V;
        const int rb = rp.rect_bits;
        const uint32_t rmask = (1u << rb) - 1u;
        const bool reach = rp.alpha_min > 0.f;
        const int tw_log2 = __builtin_ctz((unsigned)rp.tile_w);
        const float inv_th = 1.f / (float)rp.tile_h;
        uint32_t cnt = 0;   // lane t: pairs of the segment on tile t
        for (uint32_t p0 = sg.a; p0 < sg.b; p0 += 64) {
            const uint32_t p = p0 + (uint32_t)lane;
            const bool valid = p < sg.b;
            const uint32_t r = valid ? skey[p] >> rp.key_bits : 0u;
            const int x0 = (int)(r & rmask), x1 = (int)((r >> rb) & rmask);
            const int y0 = (int)((r >> (2 * rb)) & rmask), y1 = (int)((r >> (3 * rb)) & rmask);
            uint64_t M = 0;
            if (valid && !reach) {
                const uint64_t row = ((1ull << (x1 - x0 + 1)) - 1ull) << x0;
                for (int y = y0; y <= y1; ++y) M |= row << (y * S);
            } else if (valid) {
                const int64_t e = min(sentry[p], entries - 1u);
                const float4 g0 = rec[3 * e], g1 = rec[3 * e + 1];
                const Reach R = make_reach(g0.z, g0.w, g1.x, reach_limit(g1.y, rp));
                // only the rows the ellipse's height reaches
                int ya = y0, yb = y1;
                if (R.conic) {
                    const float top = fmaxf(floorf((g0.y - R.ym) * inv_th), -1e6f);
                    const float bot = fminf(floorf((g0.y + R.ym) * inv_th), 1e6f);
                    ya = max(ya, (int)top - sg.ty0 - 1);
                    yb = min(yb, (int)bot - sg.ty0 + 1);
                }
                for (int y = ya; y <= yb; ++y) {
                    const int py0 = (sg.ty0 + y) * rp.tile_h;
                    int c0, c1;
                    band_columns(R, g0.x, g0.y, g1.z, g1.w, py0, min(rp.tile_h, V.height - py0),
                                 tw_log2, V.width, &c0, &c1);
                    c0 = max(c0 - sg.tx0, x0);
                    c1 = min(c1 - sg.tx0, x1);
                    if (c0 <= c1) M |= (((1ull << (c1 - c0 + 1)) - 1ull) << c0) << (y * S);
                }
            }
            if (valid) mask[p] = M;
            // lane t counts the pairs of this step whose mask has tile t
            cnt += (uint32_t)popc64(wave_transpose64(M));
        }
        if (lane < TT)
            seg_cnt[(size_t)seg_first[sg.s] * TT + (size_t)lane * sg.nseg + sg.k] = cnt;
    }
}

// Stable scatter of one segment per wave into the tile lists, 64 pairs per
// step. The transposed masks give lane t the set of the step's pairs on tile
// t; the step's entries and their list positions are grouped by tile in LDS
// (tile t's after those of the tiles before it, in pair order), and the wave
// then stores the group with consecutive lanes on consecutive items, so that
// stores of neighbouring lanes mostly share cache lines. A step of more than
// kStepItems items (a few pairs covering most of their super-tile) is stored
// directly by the tile lanes.
constexpr int kWriteWaves = 4;
constexpr int kStepItems = 1024;
__global__ void __launch_bounds__(kWriteWaves * 64) split_write_kernel(
    const Views* __restrict__ views, RasterDev rp, const uint32_t* __restrict__ seg_first,
    const uint32_t* __restrict__ sup_ranges, const uint32_t* __restrict__ sentry,
    const uint64_t* __restrict__ mask, const uint32_t* __restrict__ seg_off,
    const uint32_t* __restrict__ counters, int64_t capacity, uint32_t* __restrict__ tile_entry) {
    __shared__ uint32_t s_ent[kWriteWaves][64];
    __shared__ uint32_t s_item[kWriteWaves][kStepItems];
    __shared__ uint32_t s_pos[kWriteWaves][kStepItems];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int S = rp.super_tile, TT = S * S;
    if ((int64_t)items_total(counters) > capacity) return;   // overflow: the tile lists stay empty
    for (uint32_t g = blockIdx.x * kWriteWaves + w;; g += gridDim.x * kWriteWaves) {
        Segment sg;
        if (!locate_segment(views, seg_first, sup_ranges, S, g, &sg)) return;
        // lane t: next list position of tile t
        const size_t base = (size_t)seg_first[sg.s] * TT + sg.k;
        uint32_t run = lane < TT ? seg_off[base + (size_t)lane * sg.nseg] : 0u;
        for (uint32_t p0 = sg.a; p0 < sg.b; p0 += 64) {
            const uint32_t p = p0 + (uint32_t)lane;
            const bool valid = p < sg.b;
            const uint64_t M = valid ? mask[p] : 0ull;
            s_ent[w][lane] = valid ? sentry[p] : 0u;
            uint64_t T = wave_transpose64(M);
            const uint32_t cnt = (uint32_t)popc64(T);
            const uint32_t incl = wave_incl_scan(cnt);
            const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
            if (total > (uint32_t)kStepItems) {
                wave_lds_sync();
                for (; T != 0ull; T &= T - 1ull) tile_entry[run++] = s_ent[w][__builtin_ctzll(T)];
                wave_lds_sync();
                continue;
            }
            wave_lds_sync();
            // group the step's entries by tile, with their list positions
            for (uint32_t o = incl - cnt; T != 0ull; T &= T - 1ull, ++o) {
                s_item[w][o] = s_ent[w][__builtin_ctzll(T)];
                s_pos[w][o] = run++;
            }
            wave_lds_sync();
            for (uint32_t i = (uint32_t)lane; i < total; i += 64)
                tile_entry[s_pos[w][i]] = s_item[w][i];
            wave_lds_sync();
        }
    }
}

// [start, end) of tile lists. After the split of the list prefixes (rest =
// false): every tile's, with its state (whether its super-tile's list was
// cut by the prefix); it also clears the super-tile redo flags, flags a
// tile-list overflow (all lists empty then) and records the segment count.
// After the completing split (rest = true): only the tiles marked
// incomplete, which now take their whole lists (empty on overflow).
__global__ void __launch_bounds__(256) tile_ranges_kernel(
    const Views* __restrict__ views, RasterDev rp, const uint32_t* __restrict__ sup_ranges,
    const uint32_t* __restrict__ seg_first, const uint32_t* __restrict__ seg_cnt,
    const uint32_t* __restrict__ seg_off, uint32_t* __restrict__ counters, int64_t capacity,
    uint32_t* __restrict__ tile_ranges, uint32_t* __restrict__ tile_state,
    uint32_t* __restrict__ sup_redo, bool rest) {
    if (rest && counters[kRedo] == 0u) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool overflow = (int64_t)items_total(counters) > capacity;
    if (t == 0) {
        if (!rest) counters[kSegments] = seg_first[views->total_supers];
        if (overflow) atomicOr(&counters[kStatus], (uint32_t)SGS_STATUS_PAIR_OVERFLOW);
    }
    if (!rest && t < views->total_supers) sup_redo[t] = 0u;
    if (t >= views->total_tiles) return;
    if (rest && tile_state[t] != kTileIncomplete) return;
    int vi = 0;
    while (vi + 1 < views->n && t >= views->v[vi + 1].tile_offset) ++vi;
    const ViewDev& V = views->v[vi];
    const int local = (int)t - V.tile_offset;
    const int tx = local % V.tiles_x, ty = local / V.tiles_x;
    const int S = rp.super_tile, TT = S * S;
    const int s = V.sup_offset + (ty / S) * V.sup_x + tx / S;
    if (!rest)
        tile_state[t] = split_segments(list_segments(sup_ranges, s), (uint32_t)rp.prefix_segs) <
                                list_segments(sup_ranges, s)
                            ? kTileTruncated
                            : kTileWhole;
    const uint32_t nseg = seg_first[s + 1] - seg_first[s];
    uint32_t a = 0, b = 0;
    if (nseg > 0 && !overflow) {
        const size_t i0 = (size_t)seg_first[s] * TT + (size_t)((ty % S) * S + tx % S) * nseg;
        a = seg_off[i0];
        b = seg_off[i0 + nseg - 1] + seg_cnt[i0 + nseg - 1];
    }
    tile_ranges[2 * t] = a;
    tile_ranges[2 * t + 1] = b;
}

}  // namespace

hipError_t launch_store_views(const Views& views, const ViewDev* table, int n_table,
                              const int32_t* d_view, Views* dst, hipStream_t s) {
    hipLaunchKernelGGL(store_views_kernel, dim3(1), dim3(64), 0, s, views, table, n_table, d_view,
                       dst);
    return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// The split of the sorted super-tile lists into tile lists: of the first
// rp.prefix_segs segments of the long ones, the others whole, before
// compositing (rest = false), or
// of the whole lists of the super-tiles flagged by that compositing, placed
// after the prefix lists (rest = true; predicated on counters[kRedo]).
static hipError_t launch_split(const RasterDev& rp, const Layout& L, char* ws, hipStream_t s,
                               bool rest) {
    if (L.total_supers == 0 || L.total_tiles == 0) return hipSuccess;
    const Views* views = reinterpret_cast<const Views*>(ws + L.views);
    uint32_t* counters = reinterpret_cast<uint32_t*>(ws + L.counters);
    const uint32_t* ranges = reinterpret_cast<const uint32_t*>(ws + L.sup_ranges);
    const uint32_t* skey = reinterpret_cast<const uint32_t*>(ws + L.pair_key[L.key_result]);
    const uint32_t* sentry = reinterpret_cast<const uint32_t*>(ws + L.pair_entry[L.key_result]);
    const float4* rec = reinterpret_cast<const float4*>(ws + L.records);
    uint32_t* seg_first = reinterpret_cast<uint32_t*>(ws + L.seg_first);
    uint32_t* seg_cnt = reinterpret_cast<uint32_t*>(ws + L.seg_cnt);
    uint32_t* seg_off = reinterpret_cast<uint32_t*>(ws + L.seg_off);
    uint64_t* mask = reinterpret_cast<uint64_t*>(ws + L.pair_mask);
    uint32_t* tile_entry = reinterpret_cast<uint32_t*>(ws + L.tile_entry);
    uint32_t* tile_ranges = reinterpret_cast<uint32_t*>(ws + L.tile_ranges);
    uint32_t* tile_state = reinterpret_cast<uint32_t*>(ws + L.tile_state);
    uint32_t* sup_redo = reinterpret_cast<uint32_t*>(ws + L.sup_redo);
    uint32_t* sums = reinterpret_cast<uint32_t*>(ws + L.scan_sums);
    const int tt = rp.super_tile * rp.super_tile;
    hipError_t err;
    // segments to split; their total -> seg_first[total_supers] (formed by
    // the count kernel itself when the super-tiles are few)
    const RestSegSrc rsrc{ranges, sup_redo, counters + kRedo, L.total_supers};
    const SegCountSrc psrc{ranges, L.total_supers, (uint32_t)rp.prefix_segs};
    const bool local = L.total_supers <= kLocalSupers;
    if (!local) {
        if (rest)
            hipLaunchKernelGGL(seg_scan_kernel<RestSegSrc>, dim3(1), dim3(kSegScanThreads), 0, s,
                               rsrc, seg_first);
        else
            hipLaunchKernelGGL(seg_scan_kernel<SegCountSrc>, dim3(1), dim3(kSegScanThreads), 0, s,
                               psrc, seg_first);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    // grid-stride over the segments: at most a few resident waves per SIMD
    // (the completing split, usually idle and otherwise a few super-tiles,
    // on a quarter of the grid)
    const int64_t blocks = rest ? kSplitBlocks / 4 : kSplitBlocks;
    const dim3 sgrid((unsigned)std::min<int64_t>((L.seg_slots + kSplitWaves - 1) / kSplitWaves,
                                                 blocks));
    const uint32_t entries = (uint32_t)std::max<int64_t>(1, L.entries);
    if (rest)
        hipLaunchKernelGGL(split_count_kernel<RestSegSrc>, sgrid, dim3(kSplitWaves * 64), 0, s,
                           views, rp, rsrc, local, seg_first, ranges, skey, sentry, rec, entries,
                           mask, seg_cnt);
    else
        hipLaunchKernelGGL(split_count_kernel<SegCountSrc>, sgrid, dim3(kSplitWaves * 64), 0, s,
                           views, rp, psrc, local, seg_first, ranges, skey, sentry, rec, entries,
                           mask, seg_cnt);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    // list positions (the completing split's after the prefix lists); the
    // number of entries -> counters[kItems] or counters[kItemsRest]
    err = device_scan(ItemCountSrc{seg_cnt, seg_first + L.total_supers, tt},
                      ItemOffSink{seg_off, rest ? counters + kItems : nullptr}, L.seg_slots * tt,
                      sums, counters + (rest ? kItemsRest : kItems), s);
    if (err != hipSuccess) return err;
    const dim3 wgrid((unsigned)std::min<int64_t>((L.seg_slots + kWriteWaves - 1) / kWriteWaves,
                                                 blocks));
    hipLaunchKernelGGL(split_write_kernel, wgrid, dim3(kWriteWaves * 64), 0, s, views, rp,
                       seg_first, ranges, sentry, mask, seg_off, counters, L.capacity, tile_entry);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(tile_ranges_kernel, dim3((unsigned)((L.total_tiles + 255) / 256)), dim3(256),
                       0, s, views, rp, ranges, seg_first, seg_cnt, seg_off, counters, L.capacity,
                       tile_ranges, tile_state, sup_redo, rest);
    return hipGetLastError();
}

hipError_t launch_split_rest(const RasterDev& rp, const Layout& L, char* ws, hipStream_t s) {
    return launch_split(rp, L, ws, s, true);
}

hipError_t launch_bin(const RasterDev& rp, int64_t n, const Layout& L, char* ws, hipStream_t s) {
    const int64_t E = L.entries;
    const Views* views = reinterpret_cast<const Views*>(ws + L.views);
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
    uint32_t* pkey[2] = {reinterpret_cast<uint32_t*>(ws + L.pair_key[0]),
                         reinterpret_cast<uint32_t*>(ws + L.pair_key[1])};
    uint32_t* pentry[2] = {reinterpret_cast<uint32_t*>(ws + L.pair_entry[0]),
                           reinterpret_cast<uint32_t*>(ws + L.pair_entry[1])};
    uint32_t* ranges = reinterpret_cast<uint32_t*>(ws + L.sup_ranges);
    hipError_t err;
    // counters this stage and the compositing forward accumulate into
    constexpr int kClear = kRedo + 1 - kVisible;

    // visible entries -> (depth, entry), entry order; count -> counters[kVisible]
    // (the first scan kernel also clears the counters)
    if (E == 0 && (err = fill_u32(counters + kVisible, kClear, 0u, s)) != hipSuccess) return err;
    if (E > 0) {
        err = device_scan(VisibleSrc{tiles, E},
                          CompactSink{reinterpret_cast<const uint32_t*>(ws + L.depth), dkey[0],
                                      dval[0]},
                          E, sums, counters + kVisible, s, counters + kVisible, kClear);
        if (err != hipSuccess) return err;
        // stable sort by depth (ties keep ascending entry order); the last
        // pass also gathers each entry's super-tile count into `offsets`, in
        // depth order, for the scan below to read linearly and overwrite in place
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
        hipLaunchKernelGGL(emit_kernel, egrid, dim3(kEmitThreads), 0, s, dval[res], offsets,
                           window_first, rec, counters, n, views, rp, L.capacity, pkey[0],
                           pentry[0]);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        // stable sort of the pairs by super-tile; the first pass drops culled
        // pairs and counts the rest into counters[kPairsKept]; a one-pass sort
        // (at most 255 super-tiles) also writes the super-tile ranges
        int kres = 0;
        const bool one_pass = L.key_passes == 1 && L.total_supers > 0;
        err = radix_sort(pkey, pentry, counters + kPairsWritten, L.capacity, L.key_bits, hist,
                         totals, s, &kres, counters + kPairsKept, nullptr, nullptr,
                         one_pass ? ranges : nullptr, one_pass ? (int)L.total_supers : 0);
        if (err != hipSuccess) return err;
    }
    const dim3 rgrid((unsigned)((L.total_supers + 255) / 256));
    if (L.total_supers > 0 && (E == 0 || L.key_passes != 1))
        hipLaunchKernelGGL(ranges_kernel, rgrid, dim3(256), 0, s, pkey[L.key_result], counters,
                           L.total_supers, L.key_bits, ranges);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    return launch_split(rp, L, ws, s, false);
}

hipError_t launch_order_tiles(const uint32_t* cost, int64_t tiles, int shift, uint32_t* order,
                              const int32_t* gate, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(order_tiles_kernel, dim3(1), dim3(kOrderThreads), 0, s, cost, tiles, shift,
                       order, gate);
    return hipGetLastError();
}

}  // namespace sgs
