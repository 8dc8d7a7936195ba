// Front-to-back compositing (paper Sec. 3, Eqs. 4-5) over the per-tile
// depth-ordered lists, and its reverse-order adjoint.
//
// One wavefront (64 lanes) per tile; each lane owns TW*TH/64 pixels of the
// tile (pixel k of lane l is tile-local index l + 64 k, so every per-pixel
// load or store of the wave is a run of contiguous row segments). The tile's
// list is staged through LDS 64 records at a time; every lane then walks the
// batch with broadcast LDS reads, reusing each record for all its pixels.
//
// The forward keeps, per pixel, only the final transmittance and the list
// position of the last blended Gaussian. The backward walks the list again
// from that position towards the front, recovering T_i = T_{i+1} / (1 -
// alpha'_i) and the colour accumulated behind each Gaussian, so no per-pixel
// blend list is stored. A Gaussian's gradient is summed over the lane's
// pixels in registers, then over the 64 lanes with one DPP reduction, and one
// lane issues the 9 hardware float atomics of that (tile, Gaussian) pair;
// Gaussians that touch no pixel of the tile skip both.
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

constexpr int kLanes = 64;

struct Splat {
    float alpha;           // alpha' after the clamp
    float ex;              // exp(P)
    float dx, dy;          // pixel centre - mean
    float dx2, dy2, dxy;   // dx^2, dy^2, dx dy
    bool clamped;          // o exp(P) > alpha_max
};

// Overlap test, Gaussian falloff and alpha' of one (pixel, Gaussian) pair.
// Forward and backward call this same function, so their skip decisions agree
// bit for bit. Branch-free: every quantity is computed and the return value
// says whether the Gaussian contributes. P = -(a dx^2 + c dy^2)/2 - b dx dy
// with explicit fused multiply-adds; exp(P) is the hardware 2^x of P log2(e)
// (about 2 ulp over the range where alpha' can reach alpha_min).
__device__ __forceinline__ bool splat_alpha(float px, float py, float u, float v, float rx,
                                            float ry, float o, float a, float b, float c,
                                            const RasterDev& rp, Splat& s) {
    // overlap box |p - mean| <= (rx, ry); p +- r is exact for half-integer p, integer r
    const bool inbox = (px - rx <= u) & (u <= px + rx) & (py - ry <= v) & (v <= py + ry);
    s.dx = px - u;
    s.dy = py - v;
    s.dx2 = s.dx * s.dx;
    s.dy2 = s.dy * s.dy;
    s.dxy = s.dx * s.dy;
    const float power = fmaf(-0.5f, fmaf(a, s.dx2, c * s.dy2), -b * s.dxy);
    s.ex = __builtin_amdgcn_exp2f(power * 1.44269504088896341f);
    const float raw = o * s.ex;
    s.clamped = raw > rp.alpha_max;
    s.alpha = s.clamped ? rp.alpha_max : raw;
    return inbox & (power <= 0.f) & (s.alpha >= rp.alpha_min);
}

__device__ __forceinline__ int view_of_tile(const Views& views, int tile) {
    int vi = 0;
    while (vi + 1 < views.n && tile >= views.v[vi + 1].tile_offset) ++vi;
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

template <int TW, int TH>
__global__ void __launch_bounds__(kLanes) raster_forward_kernel(
    Views views, RasterDev rp, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ pentry, const float4* __restrict__ rec,
    float* __restrict__ out_rgb, float* __restrict__ t_final, uint32_t* __restrict__ n_last,
    uint32_t* __restrict__ counters) {
    constexpr int PIX = TW * TH / kLanes;
    __shared__ float4 s_pos[kLanes];   // u, v, rx, ry
    __shared__ float4 s_con[kLanes];   // a, b, c, opacity
    __shared__ float4 s_col[kLanes];   // r, g, b, -

    const int tile = blockIdx.x;
    const ViewDev& V = views.v[view_of_tile(views, tile)];
    const int local = tile - V.tile_offset;
    const int tx = local % V.tiles_x, ty = local / V.tiles_x;
    const int tid = threadIdx.x;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

    float px[PIX], py[PIX], T[PIX], C0[PIX], C1[PIX], C2[PIX];
    uint32_t last[PIX];
    bool done[PIX], inside[PIX];
    bool lane_done = true;
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
        const int li = tid + kLanes * k;
        const int x = tx * TW + li % TW, y = ty * TH + li / TW;
        inside[k] = x < V.width && y < V.height;
        px[k] = (float)x + 0.5f;
        py[k] = (float)y + 0.5f;
        T[k] = 1.f;
        C0[k] = C1[k] = C2[k] = 0.f;
        last[k] = 0;
        done[k] = !inside[k];
        lane_done = lane_done && done[k];
    }
    uint32_t n_blend = 0, n_eval = 0;
    for (uint32_t b0 = start; b0 < end; b0 += kLanes) {
        if (ballot(!lane_done) == 0) break;
        __syncthreads();
        const uint32_t idx = b0 + tid;
        if (idx < end) {
            const int64_t e = pentry[idx];
            const float4 r0 = rec[3 * e], r1 = rec[3 * e + 1], r2 = rec[3 * e + 2];
            s_pos[tid] = make_float4(r0.x, r0.y, r1.z, r1.w);
            s_con[tid] = make_float4(r0.z, r0.w, r1.x, r1.y);
            s_col[tid] = r2;
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)kLanes, end - b0);
        for (int j = 0; j < cnt && !lane_done; ++j) {
            const float4 P = s_pos[j];
            const float4 Q = s_con[j];
            lane_done = true;
            const uint32_t pos = b0 + (uint32_t)j + 1u - start;
#pragma unroll
            for (int k = 0; k < PIX; ++k) {
                n_eval += done[k] ? 0u : 1u;
                Splat s;
                const bool hit =
                    !done[k] & splat_alpha(px[k], py[k], P.x, P.y, P.z, P.w, Q.w, Q.x, Q.y, Q.z, rp, s);
                if (hit) {
                    // a pixel whose transmittance would fall below t_min stops
                    // before this Gaussian; otherwise the Gaussian is blended
                    const float test = T[k] * (1.f - s.alpha);
                    const bool stop = test < rp.t_min;
                    const float4 col = s_col[j];
                    const float w = stop ? 0.f : s.alpha * T[k];
                    C0[k] = fmaf(col.x, w, C0[k]);
                    C1[k] = fmaf(col.y, w, C1[k]);
                    C2[k] = fmaf(col.z, w, C2[k]);
                    T[k] = stop ? T[k] : test;
                    last[k] = stop ? last[k] : pos;
                    n_blend += stop ? 0u : 1u;
                    done[k] = stop;
                }
                lane_done = lane_done & done[k];
            }
        }
    }
    const int64_t plane = (int64_t)V.width * V.height;
    float* img = out_rgb + 3 * V.px_offset;
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
        if (!inside[k]) continue;
        const int li = tid + kLanes * k;
        const int64_t pix = (int64_t)(ty * TH + li / TW) * V.width + (tx * TW + li % TW);
        img[pix] = fmaf(T[k], rp.bg[0], C0[k]);
        img[plane + pix] = fmaf(T[k], rp.bg[1], C1[k]);
        img[2 * plane + pix] = fmaf(T[k], rp.bg[2], C2[k]);
        t_final[V.px_offset + pix] = T[k];
        n_last[V.px_offset + pix] = last[k];
    }
    // work counters: one 64-bit atomic each per tile
    const uint32_t nb = wave_add_u32(n_blend), ne = wave_add_u32(n_eval);
    if (tid == 0) {
        atomicAdd(reinterpret_cast<unsigned long long*>(counters + kBlended),
                  (unsigned long long)nb);
        atomicAdd(reinterpret_cast<unsigned long long*>(counters + kEvaluated),
                  (unsigned long long)ne);
    }
}

// At most 72 VGPRs, so that 7 waves fit on each SIMD: the 6700 tiles of a
// 1600x1060 view (16x16 tiles) then all run at once on the 1024 SIMDs of the
// chip instead of leaving a second round for the last tiles.
template <int TW, int TH>
__global__ void __launch_bounds__(kLanes, 7) raster_backward_kernel(
    Views views, RasterDev rp, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ pentry, const float4* __restrict__ rec,
    const float* __restrict__ t_final, const uint32_t* __restrict__ n_last,
    const float* __restrict__ dl_drgb, const int32_t* __restrict__ gate,
    float* __restrict__ accum) {
    constexpr int PIX = TW * TH / kLanes;
    __shared__ float4 s_pos[kLanes];   // u, v, rx, ry
    __shared__ float4 s_con[kLanes];   // a, b, c, opacity
    __shared__ float4 s_col[kLanes];   // r, g, b, entry (bits)
    if (gate_closed(gate)) return;

    const int tile = blockIdx.x;
    const ViewDev& V = views.v[view_of_tile(views, tile)];
    const int local = tile - V.tile_offset;
    const int tx = local % V.tiles_x, ty = local / V.tiles_x;
    const int tid = threadIdx.x;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

    const int64_t plane = (int64_t)V.width * V.height;
    const float* dl = dl_drgb + 3 * V.px_offset;
    float px[PIX], py[PIX], T[PIX], G0[PIX], G1[PIX], G2[PIX], S0[PIX], S1[PIX], S2[PIX];
    uint32_t last[PIX];
    uint32_t my_max = 0;
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
        const int li = tid + kLanes * k;
        const int x = tx * TW + li % TW, y = ty * TH + li / TW;
        px[k] = (float)x + 0.5f;
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
        // colour composited behind the current Gaussian, background included
        S0[k] = rp.bg[0] * T[k];
        S1[k] = rp.bg[1] * T[k];
        S2[k] = rp.bg[2] * T[k];
        my_max = max(my_max, last[k]);
    }
    const uint32_t stop = start + min(wave_max_u32(my_max), end - start);

    for (uint32_t b_end = stop; b_end > start;) {
        const uint32_t b0 = (b_end - start > (uint32_t)kLanes) ? b_end - kLanes : start;
        const int cnt = (int)(b_end - b0);
        __syncthreads();
        if (tid < cnt) {
            const uint32_t idx = b_end - 1u - tid;
            const uint32_t e = pentry[idx];
            const float4 r0 = rec[3 * (int64_t)e], r1 = rec[3 * (int64_t)e + 1],
                         r2 = rec[3 * (int64_t)e + 2];
            s_pos[tid] = make_float4(r0.x, r0.y, r1.z, r1.w);
            s_con[tid] = make_float4(r0.z, r0.w, r1.x, r1.y);
            s_col[tid] = make_float4(r2.x, r2.y, r2.z, __uint_as_float(e));
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const uint32_t rel = b_end - 1u - (uint32_t)j - start;   // list position
            // -0 is the additive identity for every float, so the first
            // accumulation into each sum folds away
            float d_u = -0.f, d_v = -0.f, d_a = -0.f, d_b = -0.f, d_c = -0.f, d_o = -0.f;
            float d_r = -0.f, d_g = -0.f, d_bl = -0.f;
            bool contrib = false;
            const float4 P = s_pos[j];
            const float4 Q = s_con[j];
#pragma unroll
            for (int k = 0; k < PIX; ++k) {
                Splat s;
                const bool hit = (rel < last[k]) &
                                 splat_alpha(px[k], py[k], P.x, P.y, P.z, P.w, Q.w, Q.x, Q.y, Q.z, rp, s);
                if (hit) {
                    const float4 col = s_col[j];
                    // 1 - alpha' >= 1 - alpha_max > 0: one hardware reciprocal
                    // (1 ulp) serves the transmittance recovery and dC/dalpha'
                    const float inv_om = __builtin_amdgcn_rcpf(1.f - s.alpha);
                    const float Ti = T[k] * inv_om;
                    const float w = s.alpha * Ti;
                    d_r = fmaf(G0[k], w, d_r);
                    d_g = fmaf(G1[k], w, d_g);
                    d_bl = fmaf(G2[k], w, d_bl);
                    // dC/dalpha' = T_i c_i - S_i / (1 - alpha'_i), per channel
                    const float d_alpha =
                        fmaf(G0[k], fmaf(col.x, Ti, -S0[k] * inv_om),
                             fmaf(G1[k], fmaf(col.y, Ti, -S1[k] * inv_om),
                                  G2[k] * fmaf(col.z, Ti, -S2[k] * inv_om)));
                    S0[k] = fmaf(col.x, w, S0[k]);
                    S1[k] = fmaf(col.y, w, S1[k]);
                    S2[k] = fmaf(col.z, w, S2[k]);
                    T[k] = Ti;
                    // alpha' = o exp(P) unless clamped at alpha_max (then it
                    // depends on neither o nor the geometry); dalpha'/dP = alpha'
                    const float dA = s.clamped ? 0.f : d_alpha;
                    const float dP = dA * s.alpha;
                    const float hP = -0.5f * dP;
                    d_o = fmaf(dA, s.ex, d_o);
                    d_a = fmaf(hP, s.dx2, d_a);
                    d_b = fmaf(-dP, s.dxy, d_b);
                    d_c = fmaf(hP, s.dy2, d_c);
                    // dP/du = a dx + b dy, dP/dv = b dx + c dy
                    d_u = fmaf(dP, fmaf(Q.x, s.dx, Q.y * s.dy), d_u);
                    d_v = fmaf(dP, fmaf(Q.y, s.dx, Q.z * s.dy), d_v);
                    contrib = true;
                }
            }
            if (ballot(contrib) == 0) continue;
            d_u = wave_sum_to_lane63(d_u);
            d_v = wave_sum_to_lane63(d_v);
            d_a = wave_sum_to_lane63(d_a);
            d_b = wave_sum_to_lane63(d_b);
            d_c = wave_sum_to_lane63(d_c);
            d_o = wave_sum_to_lane63(d_o);
            d_r = wave_sum_to_lane63(d_r);
            d_g = wave_sum_to_lane63(d_g);
            d_bl = wave_sum_to_lane63(d_bl);
            if (tid == 63) {
                float* acc = accum + (int64_t)kAccumFloats * __float_as_uint(s_col[j].w);
                unsafeAtomicAdd(acc + 0, d_u);
                unsafeAtomicAdd(acc + 1, d_v);
                unsafeAtomicAdd(acc + 2, d_a);
                unsafeAtomicAdd(acc + 3, d_b);
                unsafeAtomicAdd(acc + 4, d_c);
                unsafeAtomicAdd(acc + 5, d_o);
                unsafeAtomicAdd(acc + 6, d_r);
                unsafeAtomicAdd(acc + 7, d_g);
                unsafeAtomicAdd(acc + 8, d_bl);
            }
        }
        b_end = b0;
    }
}

__global__ void zero_f32_gated_kernel(float4* p, int64_t n4, const int32_t* gate) {
    if (gate_closed(gate)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

hipError_t launch_rasterize(const Views& views, const RasterDev& rp, const Layout& L, char* ws,
                            float* out_rgb, hipStream_t s) {
    if (L.total_tiles == 0) return hipSuccess;
    const uint32_t* ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
    const uint32_t* pentry = reinterpret_cast<const uint32_t*>(ws + L.pair_entry[L.tile_result]);
    const float4* rec = reinterpret_cast<const float4*>(ws + L.records);
    float* tf = reinterpret_cast<float*>(ws + L.t_final);
    uint32_t* nl = reinterpret_cast<uint32_t*>(ws + L.n_last);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(ws + L.counters);
    const dim3 grid((unsigned)L.total_tiles), block(kLanes);
    if (rp.tile_w == 16 && rp.tile_h == 16)
        hipLaunchKernelGGL((raster_forward_kernel<16, 16>), grid, block, 0, s, views, rp, ranges,
                           pentry, rec, out_rgb, tf, nl, cnt);
    else if (rp.tile_w == 8 && rp.tile_h == 8)
        hipLaunchKernelGGL((raster_forward_kernel<8, 8>), grid, block, 0, s, views, rp, ranges,
                           pentry, rec, out_rgb, tf, nl, cnt);
    else
        hipLaunchKernelGGL((raster_forward_kernel<32, 8>), grid, block, 0, s, views, rp, ranges,
                           pentry, rec, out_rgb, tf, nl, cnt);
    return hipGetLastError();
}

hipError_t launch_rasterize_backward(const Views& views, const RasterDev& rp, const Layout& L,
                                     char* ws, const float* dl_drgb, const int32_t* gate,
                                     hipStream_t s) {
    float* acc = reinterpret_cast<float*>(ws + L.accum);
    const int64_t n4 = L.entries * kAccumFloats / 4;
    if (n4 > 0)
        hipLaunchKernelGGL(zero_f32_gated_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0,
                           s, reinterpret_cast<float4*>(acc), n4, gate);
    if (L.total_tiles == 0) return hipGetLastError();
    const uint32_t* ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
    const uint32_t* pentry = reinterpret_cast<const uint32_t*>(ws + L.pair_entry[L.tile_result]);
    const float4* rec = reinterpret_cast<const float4*>(ws + L.records);
    const float* tf = reinterpret_cast<const float*>(ws + L.t_final);
    const uint32_t* nl = reinterpret_cast<const uint32_t*>(ws + L.n_last);
    const dim3 grid((unsigned)L.total_tiles), block(kLanes);
    if (rp.tile_w == 16 && rp.tile_h == 16)
        hipLaunchKernelGGL((raster_backward_kernel<16, 16>), grid, block, 0, s, views, rp, ranges,
                           pentry, rec, tf, nl, dl_drgb, gate, acc);
    else if (rp.tile_w == 8 && rp.tile_h == 8)
        hipLaunchKernelGGL((raster_backward_kernel<8, 8>), grid, block, 0, s, views, rp, ranges,
                           pentry, rec, tf, nl, dl_drgb, gate, acc);
    else
        hipLaunchKernelGGL((raster_backward_kernel<32, 8>), grid, block, 0, s, views, rp, ranges,
                           pentry, rec, tf, nl, dl_drgb, gate, acc);
    return hipGetLastError();
}

}  // namespace sgs
