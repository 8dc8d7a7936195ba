// Device helpers for gfx950 (wave64): lane masks, wave-level scans and
// reductions on DPP, block scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sgs_internal.hpp"

namespace sgs {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// Sum over the 64 lanes of a wave, result valid in lane 63 only. DPP steps:
// xor 1, xor 2 (quad permutes), rotate 4 and 8 within rows of 16 (every lane
// then holds its row's sum), then lane 15 of each row added into the next
// row and lane 31 into rows 2 and 3 (gfx9 wave64 row broadcasts). The
// broadcasts run on every row, so rows 0-2 end with partial or repeated sums,
// but lane 63 receives R3 + R2 and then R1 + R0 from lane 31; with full row
// masks each step is one fused add.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xb1, 0xf, 0xf, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4e, 0xf, 0xf, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xf, 0xf, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xf, 0xf, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xf, 0xf, false));
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to_lane63(v)), 63));
}

// Inclusive prefix sum over the lanes of a wave (Hillis-Steele on shuffles).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int l = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (l >= d) v += o;
    }
    return v;
}

// Exclusive scan over the threads of a block of NT threads (NT multiple of
// 64, <= 1024). Returns the exclusive prefix; *total gets the block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* smem /* >= NT/64 + 1 */,
                                                    uint32_t* total) {
    constexpr int NW = NT / 64;
    const int w = threadIdx.x / 64;
    const int l = __lane_id();
    uint32_t inc = wave_incl_scan(v);
    if (l == 63) smem[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t s = (l < NW) ? smem[l] : 0u;
        uint32_t si = wave_incl_scan(s);
        if (l < NW) smem[l] = si - s;
        if (l == NW - 1) smem[NW] = si;
    }
    __syncthreads();
    uint32_t r = smem[w] + inc - v;
    *total = smem[NW];
    __syncthreads();
    return r;
}

// Exclusive max-scan over the threads of a block (identity 0).
template <int NT>
__device__ __forceinline__ uint32_t block_excl_max_scan(uint32_t v, uint32_t* smem) {
    const int w = threadIdx.x / 64;
    const int l = __lane_id();
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d, 64);
        if (l >= d) inc = max(inc, o);
    }
    if (l == 63) smem[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before = max(before, smem[k]);
    uint32_t ex = __shfl_up(inc, 1, 64);
    if (l == 0) ex = 0;
    __syncthreads();
    return max(before, ex);
}

// One plane array of the [F][stride] layout seen through buffer descriptors:
// plane j is a descriptor built in scalar registers from base + j * stride,
// and lane i addresses it with the 32-bit offset 4 i, so a thread that reads
// and writes many planes holds one offset register instead of a 64-bit
// address per plane. Requires stride * 4 < 2^31; accesses past the plane
// read 0 and are dropped on write.
// Cache policy of the plane loads and stores: non-temporal (the nt bit of the
// gfx950 cache-policy field). Each plane element is touched once per pass, so
// the lines are streamed rather than kept in L2 and the last-level cache.
#ifndef SGS_PLANE_CPOL
#define SGS_PLANE_CPOL 2
#endif
struct PlaneBuf {
    float* base;
    int64_t stride;
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int j) const {
        // the empty asm makes the compiler rebuild the descriptor at each use
        // (a few scalar instructions) instead of keeping one per plane live
        float* b = base;
        asm volatile("" : "+s"(b));
        return __builtin_amdgcn_make_buffer_rsrc(b + (int64_t)j * stride, (short)0,
                                                 (int)(stride * 4), 0x00020000);
    }
    // CP: cache policy of the access (the streaming default, or 0 where the
    // lanes of a wave touch a line only in part and the line is best merged
    // in L2)
    template <int CP = SGS_PLANE_CPOL>
    __device__ __forceinline__ float load(int j, uint32_t lane_off) const {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc(j), (int)lane_off, 0, CP));
    }
    template <int CP = SGS_PLANE_CPOL>
    __device__ __forceinline__ void store(int j, uint32_t lane_off, float x) const {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), rsrc(j), (int)lane_off, 0, CP);
    }
};

// Logical block index that gives each XCD a contiguous range of blocks. The
// gfx950 dispatcher hands workgroups to its 8 XCDs round-robin (workgroup w to
// XCD w % 8); with this mapping, blocks that write neighbouring addresses (the
// columns of a digit-major histogram, adjacent digit runs of a radix scatter)
// run on the same XCD, so partial cache lines merge in one L2 instead of being
// written back by several. A bijection of [0, nblocks) whatever the dispatch.
__device__ __forceinline__ int xcd_block(int wg, int nblocks) {
    constexpr int kXcds = 8;
    const int q = nblocks / kXcds, r = nblocks % kXcds;
    const int x = wg % kXcds, k = wg / kXcds;
    return x * q + min(x, r) + k;
}

__device__ __forceinline__ int floordiv(int a, int b) {
    const int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Tile rectangle [x0, x1) x [y0, y1) of the box |x - u| <= rx, |y - v| <= ry.
// With rx, ry and the tile size integers, floor((u - rx)/tw) =
// floor((floor(u) - rx)/tw), so the rectangle is exact in integer arithmetic
// on floor(u) (|u| < 2^24).
__device__ __forceinline__ void tile_rect(float u, float v, int rx, int ry, int tw, int th,
                                          int tx_n, int ty_n, int* x0, int* x1, int* y0,
                                          int* y1) {
    const int fu = (int)floorf(u), fv = (int)floorf(v);
    *x0 = min(max(floordiv(fu - rx, tw), 0), tx_n);
    *x1 = min(max(floordiv(fu + rx, tw) + 1, 0), tx_n);
    *y0 = min(max(floordiv(fv - ry, th), 0), ty_n);
    *y1 = min(max(floordiv(fv + ry, th) + 1, 0), ty_n);
}

// Super-tiles [sx0, sx1) x [sy0, sy1) (edge S tiles) holding the non-empty
// tile rectangle [x0, x1) x [y0, y1), and their number.
__device__ __forceinline__ void super_rect(int x0, int x1, int y0, int y1, int S, int* sx0,
                                           int* sx1, int* sy0, int* sy1) {
    *sx0 = x0 / S;
    *sx1 = (x1 - 1) / S + 1;
    *sy0 = y0 / S;
    *sy1 = (y1 - 1) / S + 1;
}
__device__ __forceinline__ uint32_t super_count(int x0, int x1, int y0, int y1, int S) {
    int a, b, c, d;
    super_rect(x0, x1, y0, y1, S, &a, &b, &c, &d);
    return (uint32_t)((b - a) * (d - c));
}

// Reach test of one Gaussian on a rectangle of pixels: can alpha' = o exp(-q/2),
// q = a dx^2 + 2 b dx dy + c dy^2, reach alpha_min at a pixel centre of the w x h
// pixels starting at (px0, py0) that lies inside the overlap box? The
// pixel-centre rectangle is clipped to the box (widened by 1e-3 px). If the
// Gaussian's centre lies outside it, the minimum of the convex q over the
// rectangle lies on an edge that faces the centre (moving from any other
// boundary point towards the centre enters the rectangle and lowers q), at the
// clamped stationary point of that edge: at most one vertical and one
// horizontal edge to evaluate. The test passes when that minimum, less a bound
// on its rounding error (8 ulp of the sum of the terms' magnitudes), is within
// `lim`. With lim = 2 ln(o / alpha_min) (inflated, see reach_limit) a Gaussian
// that fails cannot pass the compositing kernels' skip test at any pixel of
// the rectangle. The limit 2 ln(o / alpha_min) = 2 ln 2 (log2 o - log2 alpha_min)
// is formed with the hardware log2 and inflated by 1% + 0.01, far more than
// the rounding of either; +inf for alpha_min = 0 (log2 alpha_min = -inf).
__device__ __forceinline__ float reach_limit(float o, const RasterDev& rp) {
    constexpr float kTwoLn2 = 1.38629436111989061883f;
    return (kTwoLn2 * 1.01f) * (__builtin_amdgcn_logf(o) - rp.log2_alpha_min) + 0.01f;
}

__device__ __forceinline__ bool rect_reachable(float u, float v, float a, float b, float c,
                                               float lim, float rx, float ry, int px0, int py0,
                                               int w, int h) {
    // relative to the centre; the box widened by 1e-3 px
    const float m = 1e-3f;
    const float bx = (float)px0 - u, by = (float)py0 - v;
    const float x0 = fmaxf(bx + 0.5f, -rx - m), x1 = fminf(bx + ((float)w - 0.5f), rx + m);
    const float y0 = fmaxf(by + 0.5f, -ry - m), y1 = fminf(by + ((float)h - 0.5f), ry + m);
    if (x0 > x1 || y0 > y1) return false;   // no pixel centre of the rectangle in the box
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

// Adam element update, shared by the plain step and the fused backward step
// so both give identical results. The bias corrections enter as reciprocals
// formed once per step; the square root and the final reciprocal use the
// hardware's single-instruction forms (about 1 ulp each).
__device__ __forceinline__ AdamStep adam_bias_correction(const AdamDev& a, int k) {
    AdamStep s;
    s.ibc1 = (float)(1.0 / (1.0 - pow(a.beta1, (double)k)));
    s.ibc2 = (float)(1.0 / (1.0 - pow(a.beta2, (double)k)));
    return s;
}

__device__ __forceinline__ void adam_update(float g, float& p, float& m, float& v, float lr,
                                            const AdamDev& a, const AdamStep& s) {
    m = a.b1 * m + a.c1 * g;
    v = a.b2 * v + a.c2 * g * g;
    const float mh = m * s.ibc1, vh = v * s.ibc2;
    p = p - lr * mh * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vh) + a.eps);
}

__device__ __forceinline__ bool gate_closed(const int32_t* gate) {
    return gate != nullptr && *gate == 0;
}

}  // namespace sgs
