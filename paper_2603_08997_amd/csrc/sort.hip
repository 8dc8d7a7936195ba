// Stable least-significant-digit radix sort of (key, uint32 value) pairs over
// the low bits of uint32 keys (the kernels are templates over the key type),
// digits of at most 8 bits, reduce-then-scan:
//   hist:    per-block digit counts, stored digit-major [256][blocks];
//   scan:    one block per digit row scans the row and records its total;
//   scatter: each block ranks its keys stably (each wave ranks a contiguous
//            quarter of the block with ballots and its own digit counters;
//            per-wave counts give the order across waves), sorts them into
//            LDS, and writes digit runs out coalesced.
// Each block owns a contiguous range of kTile keys, so equal digits keep
// their input order and the sort is stable; no pass waits on another block.
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // keys per block
constexpr int kRadix = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kScanThreads = 1024;
constexpr int kHistCopies = 4;

__device__ __forceinline__ uint32_t digit_of(uint32_t k, int shift, uint32_t mask) {
    return (k >> shift) & mask;
}

// Mask of the lanes whose (valid) digit equals this lane's digit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, int bits) {
    uint64_t peers = ballot(valid);
    for (int b = 0; b < bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// Culled-pair sentinel of a key type (all bits set).
template <typename K>
__device__ __forceinline__ constexpr uint32_t culled_key() {
    return (uint32_t)(K)~(K)0;
}

// Digit counts of one block's keys. Counting does not depend on order, so the
// keys are read as uint4 (4 or 8 keys) and counted into several LDS histograms.
template <typename K>
__global__ void __launch_bounds__(kThreads) radix_hist_kernel(const K* __restrict__ keys,
                                                              const uint32_t* __restrict__ n_dev,
                                                              int shift, int bits,
                                                              uint32_t* __restrict__ hist,
                                                              int nblocks, bool skip_culled) {
    constexpr int VEC = 16 / (int)sizeof(K);
    static_assert(kItems % VEC == 0, "keys per thread");
    // kHistCopies counters per digit, lane l counting into copy l % kHistCopies,
    // so that fewer lanes of one atomic instruction hit the same address
    __shared__ uint32_t cnt[kHistCopies][kRadix];
    const int tid = threadIdx.x, w = tid % kHistCopies;
#pragma unroll
    for (int k = 0; k < kHistCopies; ++k) cnt[k][tid] = 0;
    __syncthreads();
    const uint32_t n = *n_dev;
    const uint32_t mask = (1u << bits) - 1u;
    // the grid covers the capacity; the first ceil(n / kTile) workgroups work
    const int active = (int)(((int64_t)n + kTile - 1) / kTile);
    const int blk = (int)blockIdx.x < active ? xcd_block(blockIdx.x, active) : (int)blockIdx.x;
    const int64_t base = (int64_t)blk * kTile;
    if (base < (int64_t)n) {
        const uint4* k4 = reinterpret_cast<const uint4*>(keys + base);
        const int64_t left = (int64_t)n - base;
        // all loads first, then the counts
        uint4 q[kItems / VEC];
#pragma unroll
        for (int it = 0; it < kItems / VEC; ++it) {
            const int64_t j = (int64_t)(it * kThreads + tid) * VEC;
            if (j + VEC - 1 < left) {
                q[it] = k4[it * kThreads + tid];
            } else {
                K kk[VEC];
#pragma unroll
                for (int c = 0; c < VEC; ++c)
                    kk[c] = j + c < left ? keys[base + j + c] : (K)culled_key<K>();
                __builtin_memcpy(&q[it], kk, sizeof(q[it]));
            }
        }
#pragma unroll
        for (int it = 0; it < kItems / VEC; ++it) {
            const int64_t j = (int64_t)(it * kThreads + tid) * VEC;
            K kk[VEC];
            __builtin_memcpy(kk, &q[it], sizeof(q[it]));
#pragma unroll
            for (int c = 0; c < VEC; ++c) {
                const uint32_t k = kk[c];
                if (j + c < left && !(skip_culled && k == culled_key<K>()))
                    atomicAdd(&cnt[w][digit_of(k, shift, mask)], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < kHistCopies; ++k) total += cnt[k][tid];
    // only the rows of digits this pass can produce (each write is a separate
    // cache line of the digit-major table)
    if (tid < (1 << bits)) hist[(int64_t)tid * nblocks + blk] = total;
}

// Exclusive scan of each digit row hist[d][0..nblocks) in place; totals[d] =
// row sum. Each thread takes a run of up to kScanItems consecutive entries
// (kept in registers), so a row of up to kScanThreads * kScanItems entries
// needs one block scan; longer rows go in chunks of that size.
constexpr int kScanItems = 16;
__global__ void __launch_bounds__(kScanThreads) radix_scan_kernel(uint32_t* __restrict__ hist,
                                                                  int nblocks,
                                                                  uint32_t* __restrict__ totals,
                                                                  uint32_t* __restrict__ kept) {
    __shared__ uint32_t smem[kScanThreads / 64 + 1];
    uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
    const int per = min(kScanItems, (nblocks + kScanThreads - 1) / kScanThreads);
    const int chunk = per * kScanThreads;
    uint32_t carry = 0;
    for (int base = 0; base < nblocks; base += chunk) {
        const int first = base + (int)threadIdx.x * per;
        uint32_t v[kScanItems];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int i = first + k;
            v[k] = (k < per && i < nblocks) ? row[i] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t run = carry + block_excl_scan<kScanThreads>(sum, smem, &tot);
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int i = first + k;
            if (k < per && i < nblocks) row[i] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        totals[blockIdx.x] = carry;
        // the first tile-sort pass: the kept pairs are the sum of the rows
        if (kept != nullptr) atomicAdd(kept, carry);
    }
}

// Scatter of one block's kTile keys. Wave w owns the contiguous key range
// [w kTile/kWaves, (w+1) kTile/kWaves) and ranks it in kItems rounds of 64
// consecutive keys with its own LDS digit counters, so ranking needs no
// block barrier: within a round, lanes with the same digit are found with
// ballots and ordered by lane; across rounds the wave's counter carries the
// count. One barrier later, the digit's start in the block plus the counts of
// the earlier waves give every key its block-local position; keys are sorted
// into LDS and written out in digit runs.
template <typename K>
__global__ void __launch_bounds__(kThreads) radix_scatter_kernel(
    const K* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    K* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ n_dev, int shift, int bits, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ totals, int nblocks, bool skip_culled,
    const uint32_t* __restrict__ gather_src, uint32_t* __restrict__ gather_dst,
    uint32_t* __restrict__ ranges_out, int n_ranges) {
    __shared__ K lkeys[kTile];
    __shared__ uint32_t lvals[kTile];
    __shared__ uint32_t gbase[kRadix];          // global start of this block's digit run
    __shared__ uint32_t wcnt[kWaves][kRadix];   // keys of each digit per wave
    __shared__ uint32_t smem[kThreads / 64 + 1];

    const uint32_t n = *n_dev;
    const int active = (int)(((int64_t)n + kTile - 1) / kTile);
    const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
    if (ranges_out != nullptr && blockIdx.x == 0) {
        // a one-pass sort: [start, end) of every digit's run in the output
        // (empty runs: [0, 0)), from the digit totals
        uint32_t tot;
        const bool used = tid < (1 << bits);
        const uint32_t c = used ? totals[tid] : 0u;
        const uint32_t ex = block_excl_scan<kThreads>(c, smem, &tot);
        if (tid < n_ranges) {
            ranges_out[2 * tid] = c ? ex : 0u;
            ranges_out[2 * tid + 1] = c ? ex + c : 0u;
        }
    }
    if ((int)blockIdx.x >= active) return;  // uniform across the block
    const int blk = xcd_block(blockIdx.x, active);
    const int64_t base = (int64_t)blk * kTile;
    const uint32_t mask = (1u << bits) - 1u;
    const int nvalid = (int)min((int64_t)kTile, (int64_t)n - base);
    constexpr int kPerWave = kTile / kWaves;

    // all loads first: wave w, round it, lane l holds key w*kPerWave + 64*it + l
    uint32_t key[kItems], val[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int li = w * kPerWave + it * 64 + lane;
        const bool valid = li < nvalid;
        key[it] = valid ? (uint32_t)keys_in[base + li] : culled_key<K>();
        val[it] = valid ? vals_in[base + li] : 0u;
    }
    {
        uint32_t tot;
        const bool used = tid < (1 << bits);   // rows beyond 2^bits are not written
        const uint32_t ex = block_excl_scan<kThreads>(used ? totals[tid] : 0u, smem, &tot);
        gbase[tid] = ex + (used ? hist[(int64_t)tid * nblocks + blk] : 0u);
    }
#pragma unroll
    for (int k = 0; k < kWaves; ++k) wcnt[k][tid] = 0;
    __syncthreads();

    // wave-private stable ranking (dropped keys take no position)
    uint32_t rank[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int li = w * kPerWave + it * 64 + lane;
        const bool valid = li < nvalid && !(skip_culled && key[it] == culled_key<K>());
        const uint32_t d = digit_of(key[it], shift, mask);
        const uint64_t peers = match_digit(d, valid, bits);
        const uint32_t before = (uint32_t)popc64(peers & lanemask_lt());
        uint32_t r = 0;
        if (valid) r = wcnt[w][d] + before;
        rank[it] = r;
        // every lane has read the counters before the leaders advance them
        __builtin_amdgcn_wave_barrier();
        if (valid && before == 0) wcnt[w][d] += (uint32_t)popc64(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit (thread tid): start in the block and the counts of earlier waves
    int nkept;
    {
        uint32_t c[kWaves], sum = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) { c[k] = wcnt[k][tid]; sum += c[k]; }
        uint32_t tot;
        uint32_t start = block_excl_scan<kThreads>(sum, smem, &tot);
#pragma unroll
        for (int k = 0; k < kWaves; ++k) { wcnt[k][tid] = start; start += c[k]; }
        nkept = (int)tot;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int li = w * kPerWave + it * 64 + lane;
        if (li < nvalid && !(skip_culled && key[it] == culled_key<K>())) {
            const uint32_t d = digit_of(key[it], shift, mask);
            const uint32_t pos = wcnt[w][d] + rank[it];
            lkeys[pos] = (K)key[it];
            lvals[pos] = val[it];
        }
    }
    __syncthreads();
    // wcnt[0][d] is now the block-local start of digit d
#pragma unroll 4
    for (int li = tid; li < nkept; li += kThreads) {
        const K k = lkeys[li];
        const uint32_t d = digit_of(k, shift, mask);
        const uint32_t out = gbase[d] + (uint32_t)li - wcnt[0][d];
        const uint32_t val = lvals[li];
        keys_out[out] = k;
        vals_out[out] = val;
        if (gather_dst != nullptr) gather_dst[out] = gather_src[val];
    }
}

}  // namespace

int64_t radix_blocks(int64_t n_max) { return n_max <= 0 ? 1 : (n_max + kTile - 1) / kTile; }

int radix_passes(int bits) { return bits <= 0 ? 0 : (bits + 7) / 8; }

// Bits of pass p when `bits` are sorted in radix_passes(bits) passes of
// near-equal width (13 bits: 7 + 6).
static int pass_bits(int bits, int p, int* shift) {
    const int passes = radix_passes(bits);
    const int base = bits / passes, extra = bits % passes;
    int sh = 0;
    for (int q = 0; q < p; ++q) sh += base + (q < extra ? 1 : 0);
    *shift = sh;
    return base + (p < extra ? 1 : 0);
}

template <typename K>
hipError_t radix_sort(K* keys[2], uint32_t* vals[2], const uint32_t* n_dev, int64_t n_max,
                      int bits, uint32_t* hist, uint32_t* totals, hipStream_t s, int* result,
                      uint32_t* kept_dev, const uint32_t* gather_src, uint32_t* gather_dst,
                      uint32_t* ranges_out, int n_ranges) {
    const int passes = radix_passes(bits);
    if (ranges_out != nullptr && (passes != 1 || n_ranges > (1 << bits)))
        return hipErrorInvalidValue;   // digit runs are the sorted runs of one pass only
    const int nb = (int)radix_blocks(n_max);
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        int shift;
        const int pb = pass_bits(bits, p, &shift);
        const bool skip = kept_dev != nullptr && p == 0;
        const uint32_t* n_p = (kept_dev != nullptr && p > 0) ? kept_dev : n_dev;
        hipLaunchKernelGGL(radix_hist_kernel<K>, dim3(nb), dim3(kThreads), 0, s, keys[cur], n_p,
                           shift, pb, hist, nb, skip);
        // rows and totals of digits >= 2^pb are never read for a key of this pass
        hipLaunchKernelGGL(radix_scan_kernel, dim3(1u << pb), dim3(kScanThreads), 0, s, hist, nb,
                           totals, skip ? kept_dev : nullptr);
        const bool last = p == passes - 1;
        hipLaunchKernelGGL(radix_scatter_kernel<K>, dim3(nb), dim3(kThreads), 0, s, keys[cur],
                           vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_p, shift, pb, hist, totals,
                           nb, skip, last ? gather_src : nullptr, last ? gather_dst : nullptr,
                           ranges_out, n_ranges);
        cur ^= 1;
    }
    if (kept_dev != nullptr && passes == 0)
        return hipErrorInvalidValue;  // a kept count needs at least one pass
    *result = cur;
    return hipGetLastError();
}

template hipError_t radix_sort<uint32_t>(uint32_t* keys[2], uint32_t* vals[2], const uint32_t*,
                                         int64_t, int, uint32_t*, uint32_t*, hipStream_t, int*,
                                         uint32_t*, const uint32_t*, uint32_t*, uint32_t*, int);

}  // namespace sgs
