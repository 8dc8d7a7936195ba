// Stable least-significant-digit radix sort of (uint32 key, uint32 value)
// pairs, 8-bit digits, reduce-then-scan:
//   hist:    per-block digit counts, stored digit-major [256][blocks];
//   scan:    one block per digit row scans the row and records its total;
//   scatter: each block ranks its keys stably (wave64 ballots find the lanes
//            sharing a digit; per-wave counts give the order across waves),
//            sorts them into LDS, and writes digit runs out coalesced.
// Each block owns a contiguous range of kTile keys, so equal digits keep
// their input order and the sort is stable; no pass waits on another block.
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // keys per block
constexpr int kRadix = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kScanThreads = 1024;

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

// Digit counts of one block's keys. Counting does not depend on order, so the
// keys are read as uint4 and counted into per-wave LDS histograms.
__global__ void __launch_bounds__(kThreads) radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                              const uint32_t* __restrict__ n_dev,
                                                              int shift, int bits,
                                                              uint32_t* __restrict__ hist,
                                                              int nblocks) {
    __shared__ uint32_t cnt[kWaves][kRadix];
    const int tid = threadIdx.x, w = tid / 64;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) cnt[k][tid] = 0;
    __syncthreads();
    const uint32_t n = *n_dev;
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base < (int64_t)n) {
        const uint4* k4 = reinterpret_cast<const uint4*>(keys + base);
        const int64_t left = (int64_t)n - base;
#pragma unroll
        for (int it = 0; it < kItems / 4; ++it) {
            const int64_t j = (int64_t)(it * kThreads + tid) * 4;
            if (j + 3 < left) {
                const uint4 q = k4[it * kThreads + tid];
                atomicAdd(&cnt[w][digit_of(q.x, shift, mask)], 1u);
                atomicAdd(&cnt[w][digit_of(q.y, shift, mask)], 1u);
                atomicAdd(&cnt[w][digit_of(q.z, shift, mask)], 1u);
                atomicAdd(&cnt[w][digit_of(q.w, shift, mask)], 1u);
            } else {
                for (int64_t t = j; t < left && t < j + 4; ++t)
                    atomicAdd(&cnt[w][digit_of(keys[base + t], shift, mask)], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) total += cnt[k][tid];
    hist[(int64_t)tid * nblocks + blockIdx.x] = total;
}

// Exclusive scan of each digit row hist[d][0..nblocks) in place; totals[d] = row sum.
__global__ void __launch_bounds__(kScanThreads) radix_scan_kernel(uint32_t* __restrict__ hist,
                                                                  int nblocks,
                                                                  uint32_t* __restrict__ totals) {
    __shared__ uint32_t smem[kScanThreads / 64 + 1];
    uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int base = 0; base < nblocks; base += kScanThreads) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < nblocks ? row[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kScanThreads>(v, smem, &tot);
        if (i < nblocks) row[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(kThreads) radix_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ n_dev, int shift, int bits, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ totals, int nblocks) {
    __shared__ uint32_t lkeys[kTile];
    __shared__ uint32_t lvals[kTile];
    __shared__ uint32_t gbase[kRadix];     // global output start of this block's digit run
    __shared__ uint32_t dstart[kRadix];    // block-local start of each digit
    __shared__ uint32_t run[2][kRadix];    // keys of each digit in earlier rounds
    __shared__ uint32_t wcnt[2][kWaves][kRadix];  // (round tag << 16) | count, per wave
    __shared__ uint32_t smem[kThreads / 64 + 1];

    const uint32_t n = *n_dev;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base >= (int64_t)n) return;  // uniform across the block
    const int tid = threadIdx.x, w = tid / 64;
    const uint32_t mask = (1u << bits) - 1u;
    const int nvalid = (int)min((int64_t)kTile, (int64_t)n - base);

    // global base of each digit for this block: exclusive scan of the row totals
    {
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kThreads>(totals[tid], smem, &tot);
        gbase[tid] = ex + hist[(int64_t)tid * nblocks + blockIdx.x];
    }
    run[0][tid] = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) { wcnt[0][k][tid] = 0; wcnt[1][k][tid] = 0; }
    __syncthreads();

    uint32_t key[kItems], val[kItems], rank[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int li = it * kThreads + tid;
        const bool valid = li < nvalid;
        key[it] = valid ? keys_in[base + li] : 0xffffffffu;
        val[it] = valid ? vals_in[base + li] : 0u;
        const uint32_t d = digit_of(key[it], shift, mask);
        const uint64_t peers = match_digit(d, valid, bits);
        const int buf = it & 1;
        const uint32_t tag = (uint32_t)(it + 1) << 16;
        if (valid && (peers & lanemask_lt()) == 0) wcnt[buf][w][d] = tag | (uint32_t)popc64(peers);
        __syncthreads();
        uint32_t r = 0;
        if (valid) {
            r = run[buf][d] + (uint32_t)popc64(peers & lanemask_lt());
            for (int k = 0; k < w; ++k) {
                const uint32_t c = wcnt[buf][k][d];
                if ((c & 0xffff0000u) == tag) r += c & 0xffffu;
            }
        }
        rank[it] = r;
        // digit thread: advance the running count for the next round
        {
            uint32_t add = 0;
#pragma unroll
            for (int k = 0; k < kWaves; ++k) {
                const uint32_t c = wcnt[buf][k][tid];
                if ((c & 0xffff0000u) == tag) add += c & 0xffffu;
            }
            run[buf ^ 1][tid] = run[buf][tid] + add;
        }
    }
    __syncthreads();
    // block-local digit starts
    {
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kThreads>(run[kItems & 1][tid], smem, &tot);
        dstart[tid] = ex;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int li = it * kThreads + tid;
        if (li < nvalid) {
            const uint32_t d = digit_of(key[it], shift, mask);
            const uint32_t pos = dstart[d] + rank[it];
            lkeys[pos] = key[it];
            lvals[pos] = val[it];
        }
    }
    __syncthreads();
    for (int li = tid; li < nvalid; li += kThreads) {
        const uint32_t k = lkeys[li];
        const uint32_t d = digit_of(k, shift, mask);
        const uint32_t out = gbase[d] + (uint32_t)li - dstart[d];
        keys_out[out] = k;
        vals_out[out] = lvals[li];
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

hipError_t radix_sort(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* n_dev, int64_t n_max,
                      int bits, uint32_t* hist, uint32_t* totals, hipStream_t s, int* result) {
    const int passes = radix_passes(bits);
    const int nb = (int)radix_blocks(n_max);
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        int shift;
        const int pb = pass_bits(bits, p, &shift);
        hipLaunchKernelGGL(radix_hist_kernel, dim3(nb), dim3(kThreads), 0, s, keys[cur], n_dev,
                           shift, pb, hist, nb);
        hipLaunchKernelGGL(radix_scan_kernel, dim3(kRadix), dim3(kScanThreads), 0, s, hist, nb,
                           totals);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(nb), dim3(kThreads), 0, s, keys[cur],
                           vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_dev, shift, pb, hist, totals,
                           nb);
        cur ^= 1;
    }
    *result = cur;
    return hipGetLastError();
}

}  // namespace sgs
