// Front-to-back compositing (paper Sec. 3, Eqs. 4-5) over the per-tile
// depth-ordered lists, and its reverse-order adjoint.
//
// One wavefront (64 lanes) per tile; lane l owns column l % TW of the tile
// and the rows l / TW + k * 64 / TW, k < TW*TH/64 (pixel k of lane l is
// tile-local index l + 64 k, so every per-pixel load or store of the wave is a
// run of contiguous row segments). The tile's list is staged through LDS B
// records at a time (B = lds_batch); while staging, each lane turns records
// into the coefficients the inner loop needs. Every lane then walks the batch
// with broadcast LDS reads.
//
// The exponent of Eq. 5 is evaluated in base 2 with the opacity folded in,
// E = log2(o) + A dx^2 + B dx dy + C dy^2 (A = -a log2(e)/2, B = -b log2(e),
// C = -c log2(e)/2), so that o exp(P) = 2^E. The part that depends on dx only
// is formed once per lane and Gaussian (the lane's pixels share a column);
// each pixel then costs two fused multiply-adds. A pixel takes part when it
// lies in the overlap box (bit masks over the tile's columns and rows, formed
// exactly in binary64 at staging), E >= log2(alpha_min) (alpha' >= alpha_min;
// alpha_min <= alpha_max) and E <= log2(o) (P <= 0); only then is 2^E
// evaluated. Forward and backward share these functions, so their skip
// decisions agree bit for bit.
//
// The forward keeps, per pixel, only the final transmittance and the list
// position of the last blended Gaussian. The backward walks the list again
// from that position towards the front, recovering T_i = T_{i+1} / (1 -
// alpha'_i) and, per pixel, G.S = sum over channels of dL/dC times the colour
// accumulated behind the Gaussian, so no per-pixel blend list is stored. A
// Gaussian's gradient is gathered per lane as moments of dL/dP over its
// pixels, turned into the 9 parameter gradients per lane, summed over the 64
// lanes reduce-scatter style (lane k ends with gradient k), and added with one
// hardware float atomic instruction over 9 lanes for that (tile, Gaussian)
// pair; Gaussians that touch no pixel of the tile skip both.
//
// All tiles of a launch are resident at once, so a launch lasts as long as
// its busiest SIMD. The forward records each tile's work for the backward
// (the longest prefix of the list any pixel blends), and the backward takes
// the tiles in decreasing order of it: consecutive workgroups land on
// different SIMDs, so every SIMD gets a mix of long and short tiles.
#include <algorithm>

#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

constexpr int kLanes = 64;
constexpr float kNegHalfLog2e = -0.721347520444481703680f;  // -log2(e) / 2
constexpr float kNegLog2e = -1.44269504088896340736f;       // -log2(e)

// Bit q set iff the pixel origin + q (centre origin + q + 0.5) of an n-pixel
// tile span lies in the overlap box |p - centre| <= r (r an integer). With
// f = floor(centre) and t = centre - f (both exact in FP32, |centre| < 2^24),
// the first such pixel is f - r + [t > 1/2] and the last f + r - [t < 1/2]:
// the box test of the reals in integer arithmetic.
__device__ __forceinline__ uint32_t box_mask(float centre, float r, int origin, int n) {
    const float f = floorf(centre);
    const float t = centre - f;
    const int fi = (int)f, ri = (int)r;
    const int lo = fi - ri + (t > 0.5f ? 1 : 0) - origin;
    const int hi = fi + ri - (t < 0.5f ? 1 : 0) - origin;
    const int l = max(lo, 0), h = min(hi, n - 1);
    if (l > h) return 0u;
    return (0xffffffffu >> (31 - h)) & (0xffffffffu << l);
}

// Staged record of one list entry for one tile: geo = (u, v, A, B), aux = (C,
// log2 o, column mask bits, row mask bits).
__device__ __forceinline__ void stage_entry(const float4& r0, const float4& r1, int x0, int y0,
                                            int tw, int th, float4& geo, float4& aux) {
    geo = make_float4(r0.x, r0.y, r0.z * kNegHalfLog2e, r0.w * kNegLog2e);
    aux = make_float4(r1.x * kNegHalfLog2e, __builtin_amdgcn_logf(r1.y),
                      __uint_as_float(box_mask(r0.x, r1.z, x0, tw)),
                      __uint_as_float(box_mask(r0.y, r1.w, y0, th)));
}

// Per lane and Gaussian: the dx-only part of E and the box bits of the
// lane's pixels (bit RS*k for pixel k).
struct LaneTerms {
    float dx, bx, base;
    uint32_t m;
};

__device__ __forceinline__ LaneTerms lane_terms(const float4& geo, const float4& aux, float px,
                                                int col, int row0) {
    LaneTerms t;
    t.dx = px - geo.x;
    t.base = fmaf(geo.z * t.dx, t.dx, aux.y);
    t.bx = geo.w * t.dx;
    const uint32_t inx = (__float_as_uint(aux.z) >> col) & 1u;
    t.m = inx ? (__float_as_uint(aux.w) >> row0) : 0u;
    return t;
}

// E at the pixel row offset dy = py - v.
__device__ __forceinline__ float exponent2(const LaneTerms& t, const float4& aux, float dy) {
    return fmaf(dy, fmaf(aux.x, dy, t.bx), t.base);
}

__device__ __forceinline__ bool takes_part(bool in_box, float e, const float4& aux, float lmin) {
    return in_box & (e >= lmin) & (e <= aux.y);
}

template <int kCtrl>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xf, 0xf, false));
}

// One exchange step of the reduce-scatter: lanes with `hi` set keep b and
// send a, the others keep a and send b; the kept value adds what the partner
// lane (the DPP source, which differs in that bit) sent, the sum of the same
// value over both lanes.
template <int kCtrl>
__device__ __forceinline__ float rs_step(float a, float b, bool hi) {
    const float keep = hi ? b : a, send = hi ? a : b;
    return keep + dpp_f<kCtrl>(send);
}

// x + x of the lane 16 (permlane16 swap) or 32 (permlane32 swap) apart.
__device__ __forceinline__ float xrow16(float x) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xrow32(float x) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sums of x[0..8] over the 64 lanes of a (fully active) wave. Returns, in
// lane l, the total of x[l % 8]; *t8 gets the total of x[8] in every lane.
// Bits 0, 1, 2 of the lane pick, in three halving exchanges (xor 1, xor 2,
// rotate by 4 within the row), which of the eight values the lane keeps; a
// rotate by 8 completes the row sums and two permlane swaps add the rows.
__device__ __forceinline__ float wave_sum9_scatter(const float (&x)[9], int lane, float* t8) {
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    float y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = rs_step<0xb1>(x[2 * k], x[2 * k + 1], b0);   // xor 1
    float s = x[8] + dpp_f<0xb1>(x[8]);
    const float z0 = rs_step<0x4e>(y[0], y[1], b1), z1 = rs_step<0x4e>(y[2], y[3], b1);  // xor 2
    s += dpp_f<0x4e>(s);
    float w = rs_step<0x124>(z0, z1, b2);   // row rotate 4: the source lane differs in bit 2
    s += dpp_f<0x124>(s);
    w += dpp_f<0x128>(w);                   // row rotate 8: same bits 0-2, the other half-row
    s += dpp_f<0x128>(s);
    w = xrow32(xrow16(w));
    *t8 = xrow32(xrow16(s));
    return w;
}

__device__ __forceinline__ int view_of_tile(const Views* views, int tile) {
    int vi = 0;
    while (vi + 1 < views->n && tile >= views->v[vi + 1].tile_offset) ++vi;
    return vi;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_add_u32(uint32_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += (uint32_t)__shfl_xor((int)v, d, 64);
    return v;
}

// Forward of one tile: the wave composites its tile list front to back in
// batches of B entries (records gathered and staged in LDS per batch) and
// stops when every pixel of the tile has terminated.
template <int TW, int TH, int B>
__global__ void __launch_bounds__(kLanes) raster_forward_kernel(
    const Views* __restrict__ views, RasterDev rp, const uint32_t* __restrict__ tile_ranges,
    const uint32_t* __restrict__ tile_entry, const float4* __restrict__ rec,
    float* __restrict__ out_rgb, float* __restrict__ t_final, uint32_t* __restrict__ n_last,
    uint32_t* __restrict__ tile_stats, uint32_t* __restrict__ tile_cost, uint32_t entries,
    uint32_t* __restrict__ tile_state, uint32_t* __restrict__ tile_resume,
    uint32_t* __restrict__ sup_redo, uint32_t* __restrict__ counters, bool redo) {
    constexpr int PIX = TW * TH / kLanes;
    constexpr int RS = kLanes / TW;   // row step between a lane's pixels
    static_assert(B % 32 == 0 && B >= 32 && B <= 256, "batch size");
    __shared__ float4 s_geo[B];
    __shared__ float4 s_aux[B];
    __shared__ float4 s_col[B];   // r, g, b, -

    const int tile = blockIdx.x;
    // the second pass goes on with the tiles the first left incomplete
    if (redo && tile_state[tile] != kTileIncomplete) return;
    const ViewDev& V = views->v[view_of_tile(views, tile)];
    const int local = tile - V.tile_offset;
    const int tx = local % V.tiles_x, ty = local / V.tiles_x;
    const int tid = threadIdx.x;
    const int col = tid % TW, row0 = tid / TW;
    const uint32_t start = tile_ranges[2 * tile], end = tile_ranges[2 * tile + 1];
    const float lmin = rp.log2_alpha_min, amax = rp.alpha_max, tmin = rp.t_min;
    const int px0 = tx * TW, py0 = ty * TH;

    const float px = (float)(px0 + col) + 0.5f;
    const int64_t plane = (int64_t)V.width * V.height;
    float* img = out_rgb + 3 * V.px_offset;
    float py[PIX], T[PIX], C0[PIX], C1[PIX], C2[PIX];
    uint32_t last[PIX];
    uint32_t live = 0;   // bit RS*k: pixel k is in the view and has not stopped
    // the second pass resumes each pixel where the first stopped, at the end
    // of the tile's list prefix (which begins its whole list): transmittance,
    // colour sums (stored without the background), last blended position and
    // whether the pixel is still live (bit 31 of that position)
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
        const int y = py0 + row0 + RS * k;
        py[k] = (float)y + 0.5f;
        T[k] = 1.f;
        C0[k] = C1[k] = C2[k] = 0.f;
        last[k] = 0;
        if (px0 + col < V.width && y < V.height) {
            if (redo) {
                const int64_t pix = (int64_t)y * V.width + px0 + col;
                T[k] = t_final[V.px_offset + pix];
                C0[k] = img[pix];
                C1[k] = img[plane + pix];
                C2[k] = img[2 * plane + pix];
                const uint32_t nl = n_last[V.px_offset + pix];
                last[k] = nl & 0x7fffffffu;
                if (nl >> 31) live |= 1u << (RS * k);
            } else {
                live |= 1u << (RS * k);
            }
        }
    }
    const uint32_t begin = redo ? min(start + tile_resume[tile], end) : start;
    uint32_t n_blend = 0, n_eval = 0;
    if (redo && tid == 0) {
        n_blend = tile_stats[2 * tile];
        n_eval = tile_stats[2 * tile + 1];
    }
    // Software pipeline over the batches: the entry indices are loaded two
    // batches ahead and (one entry per lane, B <= 64) the records one batch
    // ahead, so the gathers of a batch run while the previous one composites
    // (a tile whose pixels stay live walks its whole list, and its time is
    // otherwise a chain of two memory round trips per batch).
    constexpr int NE = (B + kLanes - 1) / kLanes;   // entries per lane per batch
    auto entry_at = [&](uint32_t b, int i) -> uint32_t {
        const uint32_t k = b + (uint32_t)(i * kLanes + tid);
        return k < end ? min(tile_entry[k], entries - 1u) : 0u;
    };
    uint32_t e_cur[NE], e_next[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        e_cur[i] = entry_at(begin, i);
        e_next[i] = entry_at(begin + (uint32_t)B, i);
    }
    float4 q0, q1, q2;   // records of the lane's entry of the current batch (NE == 1)
    if constexpr (NE == 1) {
        q0 = rec[3 * (int64_t)e_cur[0]];
        q1 = rec[3 * (int64_t)e_cur[0] + 1];
        q2 = rec[3 * (int64_t)e_cur[0] + 2];
    }
    for (uint32_t b0 = begin; b0 < end; b0 += (uint32_t)B) {
        if (ballot(live != 0u) == 0) break;
        __syncthreads();
        const int cnt = (int)min((uint32_t)B, end - b0);
        if constexpr (NE == 1) {
            if (tid < cnt) {
                stage_entry(q0, q1, px0, py0, TW, TH, s_geo[tid], s_aux[tid]);
                s_col[tid] = q2;
            }
            const uint32_t e2 = entry_at(b0 + 2u * (uint32_t)B, 0);
            q0 = rec[3 * (int64_t)e_next[0]];
            q1 = rec[3 * (int64_t)e_next[0] + 1];
            q2 = rec[3 * (int64_t)e_next[0] + 2];
            e_next[0] = e2;
        } else {
#pragma unroll
            for (int i = 0; i < NE; ++i) {
                const int j = i * kLanes + tid;
                if (j < cnt) {
                    const int64_t e = e_cur[i];
                    const float4 r0 = rec[3 * e], r1 = rec[3 * e + 1];
                    stage_entry(r0, r1, px0, py0, TW, TH, s_geo[j], s_aux[j]);
                    s_col[j] = rec[3 * e + 2];
                }
                e_cur[i] = e_next[i];
                e_next[i] = entry_at(b0 + 2u * (uint32_t)B, i);
            }
        }
        __syncthreads();
        // the next entry's LDS reads are issued before the current entry is
        // processed, so a wave running alone does not wait on them
        float4 Gn = s_geo[0], Xn = s_aux[0], Cn = s_col[0];
        // unrolled twice: the prefetched records alternate between two
        // register sets instead of being copied at the end of every step
#pragma unroll 2
        for (int j = 0; j < cnt && live != 0u; ++j) {
            const float4 G = Gn, X = Xn, c = Cn;
            const int jn = min(j + 1, cnt - 1);
            Gn = s_geo[jn];
            Xn = s_aux[jn];
            Cn = s_col[jn];
            const LaneTerms L = lane_terms(G, X, px, col, row0);
            const uint32_t m = L.m & live;
            const uint32_t pos = b0 - start + (uint32_t)j + 1u;
            n_eval += (uint32_t)__builtin_popcount(live);
#pragma unroll
            for (int k = 0; k < PIX; ++k) {
                const float e = exponent2(L, X, py[k] - G.y);
                if (takes_part(((m >> (RS * k)) & 1u) != 0u, e, X, lmin)) {
                    // a pixel whose transmittance would fall below t_min stops
                    // before this Gaussian; otherwise the Gaussian is blended
                    const float alpha = fminf(__builtin_amdgcn_exp2f(e), amax);
                    const float wgt = alpha * T[k];
                    const float tn = T[k] - wgt;
                    const bool stop = tn < tmin;
                    const float wv = stop ? 0.f : wgt;
                    C0[k] = fmaf(c.x, wv, C0[k]);
                    C1[k] = fmaf(c.y, wv, C1[k]);
                    C2[k] = fmaf(c.z, wv, C2[k]);
                    T[k] = stop ? T[k] : tn;
                    last[k] = stop ? last[k] : pos;
                    n_blend += stop ? 0u : 1u;
                    live &= stop ? ~(1u << (RS * k)) : ~0u;
                }
            }
        }
    }

    // a pixel still live at the end of a list cut by the split prefix: the
    // tile is resumed by the second pass over its whole list, after the whole
    // lists of its super-tile have been split; until then its pixels hold the
    // state to resume from
    const bool suspend = !redo && tile_state != nullptr && ballot(live != 0u) != 0 &&
                         tile_state[tile] == kTileTruncated;
    const int x = px0 + col;
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
        const int y = py0 + row0 + RS * k;
        if (x >= V.width || y >= V.height) continue;
        const int64_t pix = (int64_t)y * V.width + x;
        const bool lk = (live >> (RS * k)) & 1u;
        img[pix] = suspend ? C0[k] : fmaf(T[k], rp.bg[0], C0[k]);
        img[plane + pix] = suspend ? C1[k] : fmaf(T[k], rp.bg[1], C1[k]);
        img[2 * plane + pix] = suspend ? C2[k] : fmaf(T[k], rp.bg[2], C2[k]);
        t_final[V.px_offset + pix] = T[k];
        n_last[V.px_offset + pix] = suspend && lk ? last[k] | 0x80000000u : last[k];
    }
    // the backward walks every pixel's list up to its last blended Gaussian:
    // the tile's longest such prefix is its work
    uint32_t my_last = 0;
#pragma unroll
    for (int k = 0; k < PIX; ++k) my_last = max(my_last, last[k]);
    const uint32_t tile_last = wave_max_u32(my_last);
    // work counters per tile, summed by a small kernel after the launch
    // (atomics of every tile on the one counters line serialise across the
    // chip and would lengthen the launch by a fifth)
    const uint32_t nb = wave_add_u32(n_blend), ne2 = wave_add_u32(n_eval);
    if (tid == 0) {
        tile_cost[tile] = tile_last;
        tile_stats[2 * tile] = nb;
        tile_stats[2 * tile + 1] = ne2;
        if (redo) {
            tile_state[tile] = kTileWhole;
        } else if (suspend) {
            const int S = rp.super_tile;
            tile_state[tile] = kTileIncomplete;
            tile_resume[tile] = end - start;
            sup_redo[V.sup_offset + (ty / S) * V.sup_x + tx / S] = 1u;
            counters[kRedo] = 1u;
        }
    }
}

// counters[kBlended], [kEvaluated] (uint64) and [kUsed] (saturating uint32)
// from the per-tile work of the last compositing forward.
constexpr int kStatThreads = 1024;
__global__ void __launch_bounds__(kStatThreads) sum_tile_stats_kernel(
    const uint32_t* __restrict__ tile_stats, const uint32_t* __restrict__ tile_cost,
    int64_t tiles, uint32_t* __restrict__ counters) {
    __shared__ unsigned long long s_sum[3][kStatThreads / 64];
    unsigned long long b = 0, e = 0, u = 0;
    for (int64_t t = threadIdx.x; t < tiles; t += kStatThreads) {
        b += tile_stats[2 * t];
        e += tile_stats[2 * t + 1];
        u += tile_cost[t];
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        b += __shfl_xor(b, d, 64);
        e += __shfl_xor(e, d, 64);
        u += __shfl_xor(u, d, 64);
    }
    const int w = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) {
        s_sum[0][w] = b;
        s_sum[1][w] = e;
        s_sum[2][w] = u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        b = e = u = 0;
        for (int k = 0; k < kStatThreads / 64; ++k) {
            b += s_sum[0][k];
            e += s_sum[1][k];
            u += s_sum[2][k];
        }
        reinterpret_cast<unsigned long long*>(counters + kBlended)[0] = b;
        reinterpret_cast<unsigned long long*>(counters + kEvaluated)[0] = e;
        counters[kUsed] = (uint32_t)min(u, 0xffffffffull);
    }
}

// At most 72 VGPRs (batches of 64), so that 7 waves fit on each SIMD: the
// 6700 tiles of a 1600x1060 view (16x16 tiles) then all run at once on the
// 1024 SIMDs of the chip instead of leaving a second round for the last tiles.
//
// Gradient of one (tile, Gaussian) pair from per-lane moments of dL/dP over
// the lane's pixels (dP = dL/dP, dy per pixel, dx per lane): with
// P = -(a dx^2 + c dy^2)/2 - b dx dy, dx = px - u, dy = py - v,
//   dL/du = a M1 + b M2,  dL/dv = b M1 + c M2,  dL/da = -M3/2,
//   dL/db = -M4,  dL/dc = -M5/2,  dL/do = M6 / o  (unclamped alpha' = o e^P),
// M1 = sum dP dx, M2 = sum dP dy, M3 = sum dP dx^2, M4 = sum dP dx dy,
// M5 = sum dP dy^2, M6 = sum dP.
// Waves per SIMD the LDS of a batch allows (64 B per staged entry).
constexpr int backward_waves(int batch) { return batch <= 64 ? 7 : (batch == 128 ? 5 : 3); }

template <int TW, int TH, int B>
__global__ void __launch_bounds__(kLanes, backward_waves(B)) raster_backward_kernel(
    const Views* __restrict__ views, RasterDev rp, const uint32_t* __restrict__ tile_ranges,
    const uint32_t* __restrict__ tile_entry, const float4* __restrict__ rec,
    const float* __restrict__ t_final, const uint32_t* __restrict__ n_last,
    const float* __restrict__ dl_drgb, const int32_t* __restrict__ gate,
    float* __restrict__ accum, const uint32_t* __restrict__ order, int total_tiles,
    uint32_t entries) {
    constexpr int PIX = TW * TH / kLanes;
    constexpr int RS = kLanes / TW;
    __shared__ float4 s_geo[B];
    __shared__ float4 s_aux[B];
    __shared__ float4 s_col[B];   // r, g, b, entry (bits)
    __shared__ float4 s_con[B];   // a, b, c, 1 / o
    if (gate_closed(gate)) return;

    const int tile = (int)order[blockIdx.x];
    if (tile >= total_tiles) return;   // order is a permutation of the tiles
    const ViewDev& V = views->v[view_of_tile(views, tile)];
    const int local = tile - V.tile_offset;
    const int tx = local % V.tiles_x, ty = local / V.tiles_x;
    const int tid = threadIdx.x;
    const int col = tid % TW, row0 = tid / TW;
    const float lmin = rp.log2_alpha_min, amax = rp.alpha_max;

    const int64_t plane = (int64_t)V.width * V.height;
    const float* dl = dl_drgb + 3 * V.px_offset;
    const int x = tx * TW + col;
    const float px = (float)x + 0.5f;
    float py[PIX], T[PIX], G0[PIX], G1[PIX], G2[PIX], GS[PIX];
    uint32_t last[PIX];
    uint32_t my_max = 0;
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
        const int y = ty * TH + row0 + RS * k;
        py[k] = (float)y + 0.5f;
        T[k] = 1.f;
        G0[k] = G1[k] = G2[k] = 0.f;
        last[k] = 0;
        if (x < V.width && y < V.height) {
            const int64_t pix = (int64_t)y * V.width + x;
            G0[k] = dl[pix];
            G1[k] = dl[plane + pix];
            G2[k] = dl[2 * plane + pix];
            T[k] = t_final[V.px_offset + pix];
            last[k] = n_last[V.px_offset + pix];
        }
        // dL/dC . (colour composited behind the current Gaussian), background included
        GS[k] = fmaf(G0[k], rp.bg[0], fmaf(G1[k], rp.bg[1], G2[k] * rp.bg[2])) * T[k];
        my_max = max(my_max, last[k]);
    }
    const uint32_t start = tile_ranges[2 * tile], end = tile_ranges[2 * tile + 1];
    const uint32_t stop = min(wave_max_u32(my_max), end - start);

    // the list from the last blended position towards the front, B entries
    // at a time (list positions [b0, b_end), staged last first)
    for (uint32_t b_end = stop; b_end > 0u;) {
        const uint32_t b0 = b_end > (uint32_t)B ? b_end - (uint32_t)B : 0u;
        const int cnt = (int)(b_end - b0);
        __syncthreads();
        for (int k = tid; k < cnt; k += kLanes) {
            const uint32_t e = min(tile_entry[start + b_end - 1u - (uint32_t)k], entries - 1u);
            const float4 r0 = rec[3 * (int64_t)e], r1 = rec[3 * (int64_t)e + 1],
                         r2 = rec[3 * (int64_t)e + 2];
            stage_entry(r0, r1, tx * TW, ty * TH, TW, TH, s_geo[k], s_aux[k]);
            s_col[k] = make_float4(r2.x, r2.y, r2.z, __uint_as_float(e));
            // 1/o capped at FLT_MAX: an opacity that underflowed to 0 can only
            // take part with alpha' = 0 (alpha_min = 0), where M6 = 0
            s_con[k] = make_float4(r0.z, r0.w, r1.x, fminf(1.f / r1.y, 3.402823466e38f));
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const uint32_t rel = b_end - 1u - (uint32_t)j;   // list position
            const float4 G = s_geo[j];
            const float4 X = s_aux[j];
            // read once per Gaussian with the coefficients (the compiler would
            // otherwise re-read it inside each pixel's branch)
            const float4 c = s_col[j];
            asm volatile("" ::"v"(c.x), "v"(c.y), "v"(c.z));
            const LaneTerms L = lane_terms(G, X, px, col, row0);
            // -0 is the additive identity for every float, so the first
            // accumulation into each sum folds away
            float sdp = -0.f, sdy = -0.f, sdy2 = -0.f, d_r = -0.f, d_g = -0.f, d_bl = -0.f;
            bool contrib = false;
#pragma unroll
            for (int k = 0; k < PIX; ++k) {
                const float dy = py[k] - G.y;
                const float e = exponent2(L, X, dy);
                if ((rel < last[k]) & takes_part(((L.m >> (RS * k)) & 1u) != 0u, e, X, lmin)) {
                    const float raw = __builtin_amdgcn_exp2f(e);
                    const bool clamped = raw > amax;
                    const float alpha = fminf(raw, amax);
                    // 1 - alpha' >= 1 - alpha_max > 0: one hardware reciprocal
                    // (1 ulp) serves the transmittance recovery and dC/dalpha'
                    const float inv_om = __builtin_amdgcn_rcpf(1.f - alpha);
                    const float Ti = T[k] * inv_om;
                    const float w = alpha * Ti;
                    d_r = fmaf(G0[k], w, d_r);
                    d_g = fmaf(G1[k], w, d_g);
                    d_bl = fmaf(G2[k], w, d_bl);
                    // dL/dalpha' = T_i (dL/dC . c_i) - (dL/dC . S_i) / (1 - alpha'_i)
                    const float gc = fmaf(G0[k], c.x, fmaf(G1[k], c.y, G2[k] * c.z));
                    const float d_alpha = fmaf(Ti, gc, -(inv_om * GS[k]));
                    GS[k] = fmaf(w, gc, GS[k]);
                    T[k] = Ti;
                    // alpha' = o exp(P) unless clamped at alpha_max (then it
                    // depends on neither o nor the geometry); dalpha'/dP = alpha'
                    const float dP = clamped ? 0.f : d_alpha * alpha;
                    sdp += dP;
                    const float t = dP * dy;
                    sdy += t;
                    sdy2 = fmaf(t, dy, sdy2);
                    contrib = true;
                }
            }
            if (ballot(contrib) == 0) continue;
            // per-lane parameter gradients (the moments scaled by the
            // Gaussian's a, b, c, 1/o), summed over the wave reduce-scatter
            // style: lane k < 8 ends with the total of gradient k, every lane
            // with the total of gradient 8; one atomic instruction adds all 9
            const float4 Q = s_con[j];
            const float m1 = L.dx * sdp;
            float x[9];
            x[0] = fmaf(Q.x, m1, Q.y * sdy);   // dL/du
            x[1] = fmaf(Q.y, m1, Q.z * sdy);   // dL/dv
            x[2] = (-0.5f * L.dx) * m1;        // dL/da
            x[3] = -(L.dx * sdy);              // dL/db
            x[4] = -0.5f * sdy2;               // dL/dc
            x[5] = Q.w * sdp;                  // dL/do
            x[6] = d_r;
            x[7] = d_g;
            x[8] = d_bl;
            float t8;
            const float t = wave_sum9_scatter(x, tid, &t8);
            if (tid < 9)
                unsafeAtomicAdd(accum + (int64_t)kAccumFloats * __float_as_uint(s_col[j].w) + tid,
                                tid == 8 ? t8 : t);
        }
        b_end = b0;
    }
}

// Clears the accumulators in a grid-stride loop over a grid sized for the
// machine (a closed gate then costs a launch of a few thousand blocks, not
// one block per 256 float4).
constexpr int kZeroBlocks = 2048;
__global__ void zero_f32_gated_kernel(float4* p, int64_t n4, const int32_t* gate) {
    if (gate_closed(gate)) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

// Kernel instantiations: tile shapes 16x16, 8x8, 32x8 and batches 32, 64,
// 128, 256 (the shapes and batches the raster parameters accept).
#define SGS_RASTER_DISPATCH(KERNEL, ...)                                              \
    do {                                                                             \
        const int tw_ = rp.tile_w, b_ = rp.batch;                                    \
        if (tw_ == 16) {                                                             \
            if (b_ == 32) SGS_LAUNCH((KERNEL<16, 16, 32>), __VA_ARGS__);               \
            else if (b_ == 128) SGS_LAUNCH((KERNEL<16, 16, 128>), __VA_ARGS__);        \
            else if (b_ == 256) SGS_LAUNCH((KERNEL<16, 16, 256>), __VA_ARGS__);        \
            else SGS_LAUNCH((KERNEL<16, 16, 64>), __VA_ARGS__);                        \
        } else if (tw_ == 8) {                                                       \
            if (b_ == 32) SGS_LAUNCH((KERNEL<8, 8, 32>), __VA_ARGS__);                 \
            else if (b_ == 128) SGS_LAUNCH((KERNEL<8, 8, 128>), __VA_ARGS__);          \
            else if (b_ == 256) SGS_LAUNCH((KERNEL<8, 8, 256>), __VA_ARGS__);          \
            else SGS_LAUNCH((KERNEL<8, 8, 64>), __VA_ARGS__);                          \
        } else {                                                                     \
            if (b_ == 32) SGS_LAUNCH((KERNEL<32, 8, 32>), __VA_ARGS__);                \
            else if (b_ == 128) SGS_LAUNCH((KERNEL<32, 8, 128>), __VA_ARGS__);         \
            else if (b_ == 256) SGS_LAUNCH((KERNEL<32, 8, 256>), __VA_ARGS__);         \
            else SGS_LAUNCH((KERNEL<32, 8, 64>), __VA_ARGS__);                         \
        }                                                                            \
    } while (0)
#define SGS_LAUNCH(K, ...) hipLaunchKernelGGL((K), grid, block, 0, s, __VA_ARGS__)

hipError_t launch_rasterize(const RasterDev& rp, const Layout& L, char* ws, float* out_rgb,
                            hipStream_t s) {
    if (L.total_tiles == 0) return hipSuccess;
    const Views* views = reinterpret_cast<const Views*>(ws + L.views);
    const uint32_t* ranges = reinterpret_cast<const uint32_t*>(ws + L.tile_ranges);
    const uint32_t* entry = reinterpret_cast<const uint32_t*>(ws + L.tile_entry);
    const float4* rec = reinterpret_cast<const float4*>(ws + L.records);
    float* tf = reinterpret_cast<float*>(ws + L.t_final);
    uint32_t* nl = reinterpret_cast<uint32_t*>(ws + L.n_last);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(ws + L.counters);
    uint32_t* cost = reinterpret_cast<uint32_t*>(ws + L.tile_cost);
    uint32_t* stats = reinterpret_cast<uint32_t*>(ws + L.tile_stats);
    const uint32_t entries = (uint32_t)std::max<int64_t>(1, L.entries);
    uint32_t* state = rp.prefix_segs > 0 ? reinterpret_cast<uint32_t*>(ws + L.tile_state) : nullptr;
    uint32_t* sup_redo = reinterpret_cast<uint32_t*>(ws + L.sup_redo);
    uint32_t* resume = reinterpret_cast<uint32_t*>(ws + L.tile_resume);
    const dim3 grid((unsigned)L.total_tiles), block(kLanes);
    SGS_RASTER_DISPATCH(raster_forward_kernel, views, rp, ranges, entry, rec, out_rgb, tf, nl,
                        stats, cost, entries, state, resume, sup_redo, cnt, false);
    if (hipError_t err = hipGetLastError(); err != hipSuccess) return err;
    if (state != nullptr) {
        // tiles whose list prefix ran out with live pixels: the whole lists of
        // their super-tiles, then their compositing resumed
        if (hipError_t err = launch_split_rest(rp, L, ws, s); err != hipSuccess) return err;
        SGS_RASTER_DISPATCH(raster_forward_kernel, views, rp, ranges, entry, rec, out_rgb, tf, nl,
                            stats, cost, entries, state, resume, sup_redo, cnt, true);
        if (hipError_t err = hipGetLastError(); err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(sum_tile_stats_kernel, dim3(1), dim3(kStatThreads), 0, s, stats, cost,
                       L.total_tiles, cnt);
    return hipGetLastError();
}

hipError_t launch_rasterize_backward(const RasterDev& rp, const Layout& L, char* ws,
                                     const float* dl_drgb, const int32_t* gate, hipStream_t s) {
    float* acc = reinterpret_cast<float*>(ws + L.accum);
    const int64_t n4 = L.entries * kAccumFloats / 4;
    if (n4 > 0)
        hipLaunchKernelGGL(zero_f32_gated_kernel,
                           dim3((unsigned)std::min<int64_t>((n4 + 255) / 256, kZeroBlocks)),
                           dim3(256), 0, s, reinterpret_cast<float4*>(acc), n4, gate);
    if (L.total_tiles == 0 || L.entries == 0) return hipGetLastError();
    const Views* views = reinterpret_cast<const Views*>(ws + L.views);
    const uint32_t* ranges = reinterpret_cast<const uint32_t*>(ws + L.tile_ranges);
    const uint32_t* entry = reinterpret_cast<const uint32_t*>(ws + L.tile_entry);
    const float4* rec = reinterpret_cast<const float4*>(ws + L.records);
    const float* tf = reinterpret_cast<const float*>(ws + L.t_final);
    const uint32_t* nl = reinterpret_cast<const uint32_t*>(ws + L.n_last);
    // the tiles in order of the forward's measured work, largest first, so
    // that every SIMD gets a mix of long and short tiles
    uint32_t* order = reinterpret_cast<uint32_t*>(ws + L.tile_order);
    if (hipError_t err = launch_order_tiles(reinterpret_cast<const uint32_t*>(ws + L.tile_cost),
                                            L.total_tiles, 0, order, gate, s);
        err != hipSuccess)
        return err;
    const int tiles = (int)L.total_tiles;
    const dim3 grid((unsigned)L.total_tiles), block(kLanes);
    SGS_RASTER_DISPATCH(raster_backward_kernel, views, rp, ranges, entry, rec, tf, nl, dl_drgb,
                        gate, acc, order, tiles, (uint32_t)L.entries);
    return hipGetLastError();
}

#undef SGS_LAUNCH
#undef SGS_RASTER_DISPATCH

}  // namespace sgs
