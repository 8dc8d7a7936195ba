// Front-to-back compositing (paper Sec. 3, Eqs. 4-5) over the per-tile
// depth-ordered lists, and its reverse-order adjoint.
//
// One workgroup per tile, one thread per pixel. The tile's list is staged
// through LDS in batches of one record per thread; every thread then walks the
// batch (LDS broadcast reads). The forward keeps, per pixel, only the final
// transmittance and the list position of the last blended Gaussian; the
// backward walks the list again from that position towards the front,
// recovering T_i = T_{i+1} / (1 - alpha'_i) and the colour accumulated behind
// each Gaussian, so no per-pixel blend list is ever stored.
//
// Per-Gaussian gradients are summed over the 64 pixels of a wavefront with
// DPP before one lane issues the hardware float atomics, and waves with no
// contribution for a Gaussian skip both.
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

struct Splat {
    float alpha;   // alpha' after the clamp
    float ex;      // exp(P)
    float dx, dy;  // pixel centre - mean
    bool clamped;  // o exp(P) > alpha_max
};

// Overlap test, Gaussian falloff and alpha' of one (pixel, Gaussian) pair.
// Forward and backward call this same function, so their skip decisions agree
// bit for bit. Returns false when the Gaussian does not contribute.
__device__ __forceinline__ bool splat_alpha(float px, float py, float u, float v, float r,
                                            float o, float a, float b, float c,
                                            const RasterDev& rp, Splat& s) {
    // |p - mean| <= r per axis; p +- r is exact for half-integer p, integer r
    if (!(px - r <= u && u <= px + r && py - r <= v && v <= py + r)) return false;
    s.dx = px - u;
    s.dy = py - v;
    const float power = -0.5f * fmaf(a, s.dx * s.dx, c * (s.dy * s.dy)) - b * (s.dx * s.dy);
    if (power > 0.f) return false;
    s.ex = expf(power);
    const float raw = o * s.ex;
    s.clamped = raw > rp.alpha_max;
    s.alpha = s.clamped ? rp.alpha_max : raw;
    return s.alpha >= rp.alpha_min;
}

__device__ __forceinline__ int view_of_tile(const Views& views, int tile) {
    int vi = 0;
    while (vi + 1 < views.n && tile >= views.v[vi + 1].tile_offset) ++vi;
    return vi;
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW* TH) raster_forward_kernel(
    Views views, RasterDev rp, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ pentry, const float4* __restrict__ rec,
    float* __restrict__ out_rgb, float* __restrict__ t_final, uint32_t* __restrict__ n_last,
    uint32_t* __restrict__ counters) {
    constexpr int NT = TW * TH;
    __shared__ float4 s_pos[NT];   // u, v, radius, opacity
    __shared__ float4 s_con[NT];   // a, b, c, -
    __shared__ float4 s_col[NT];   // r, g, b, -
    __shared__ uint32_t s_cnt[2];

    const int tile = blockIdx.x;
    const ViewDev& V = views.v[view_of_tile(views, tile)];
    const int local = tile - V.tile_offset;
    const int tx = local % V.tiles_x, ty = local / V.tiles_x;
    const int tid = threadIdx.x;
    const int x = tx * TW + tid % TW, y = ty * TH + tid / TW;
    const bool inside = x < V.width && y < V.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    uint32_t last = 0, n_blend = 0, n_eval = 0;
    bool done = !inside;
    if (tid < 2) s_cnt[tid] = 0;
    for (uint32_t b0 = start; b0 < end; b0 += NT) {
        if (__syncthreads_and(done)) break;
        const uint32_t idx = b0 + tid;
        if (idx < end) {
            const int64_t e = pentry[idx];
            const float4 r0 = rec[3 * e], r1 = rec[3 * e + 1], r2 = rec[3 * e + 2];
            s_pos[tid] = make_float4(r0.x, r0.y, r1.z, r1.y);
            s_con[tid] = make_float4(r0.z, r0.w, r1.x, 0.f);
            s_col[tid] = r2;
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)NT, end - b0);
        if (!done) {
            for (int j = 0; j < cnt; ++j) {
                const float4 P = s_pos[j];
                const float4 Q = s_con[j];
                Splat s;
                ++n_eval;
                if (!splat_alpha(px, py, P.x, P.y, P.z, P.w, Q.x, Q.y, Q.z, rp, s)) continue;
                const float test = T * (1.f - s.alpha);
                if (test < rp.t_min) { done = true; break; }
                ++n_blend;
                const float4 col = s_col[j];
                const float w = s.alpha * T;
                C0 = fmaf(col.x, w, C0);
                C1 = fmaf(col.y, w, C1);
                C2 = fmaf(col.z, w, C2);
                T = test;
                last = b0 + (uint32_t)j + 1u - start;
            }
        }
    }
    if (inside) {
        const int64_t plane = (int64_t)V.width * V.height;
        const int64_t pix = (int64_t)y * V.width + x;
        float* img = out_rgb + 3 * V.px_offset;
        img[pix] = fmaf(T, rp.bg[0], C0);
        img[plane + pix] = fmaf(T, rp.bg[1], C1);
        img[2 * plane + pix] = fmaf(T, rp.bg[2], C2);
        t_final[V.px_offset + pix] = T;
        n_last[V.px_offset + pix] = last;
    }
    // work counters: one 64-bit atomic per workgroup
    __syncthreads();
    if (n_blend) atomicAdd(&s_cnt[0], n_blend);
    if (n_eval) atomicAdd(&s_cnt[1], n_eval);
    __syncthreads();
    if (tid == 0) {
        atomicAdd(reinterpret_cast<unsigned long long*>(counters + kBlended),
                  (unsigned long long)s_cnt[0]);
        atomicAdd(reinterpret_cast<unsigned long long*>(counters + kEvaluated),
                  (unsigned long long)s_cnt[1]);
    }
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW* TH) raster_backward_kernel(
    Views views, RasterDev rp, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ pentry, const float4* __restrict__ rec,
    const float* __restrict__ t_final, const uint32_t* __restrict__ n_last,
    const float* __restrict__ dl_drgb, const int32_t* __restrict__ gate,
    float* __restrict__ accum) {
    constexpr int NT = TW * TH;
    __shared__ float4 s_pos[NT];   // u, v, radius, opacity
    __shared__ float4 s_con[NT];   // a, b, c, entry (bits)
    __shared__ float4 s_col[NT];   // r, g, b, -
    __shared__ uint32_t s_max;
    if (gate_closed(gate)) return;

    const int tile = blockIdx.x;
    const ViewDev& V = views.v[view_of_tile(views, tile)];
    const int local = tile - V.tile_offset;
    const int tx = local % V.tiles_x, ty = local / V.tiles_x;
    const int tid = threadIdx.x;
    const int x = tx * TW + tid % TW, y = ty * TH + tid / TW;
    const bool inside = x < V.width && y < V.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

    float T = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    uint32_t last = 0;
    if (inside) {
        const int64_t plane = (int64_t)V.width * V.height;
        const int64_t pix = (int64_t)y * V.width + x;
        const float* dl = dl_drgb + 3 * V.px_offset;
        g0 = dl[pix];
        g1 = dl[plane + pix];
        g2 = dl[2 * plane + pix];
        T = t_final[V.px_offset + pix];
        last = n_last[V.px_offset + pix];
    }
    // colour composited behind the current Gaussian, background included
    float S0 = rp.bg[0] * T, S1 = rp.bg[1] * T, S2 = rp.bg[2] * T;
    if (tid == 0) s_max = 0;
    __syncthreads();
    if (last) atomicMax(&s_max, last);
    __syncthreads();
    const uint32_t stop = start + min(s_max, end - start);

    for (uint32_t b_end = stop; b_end > start;) {
        const uint32_t b0 = (b_end - start > (uint32_t)NT) ? b_end - NT : start;
        const int cnt = (int)(b_end - b0);
        __syncthreads();
        if (tid < cnt) {
            const uint32_t idx = b_end - 1u - tid;
            const uint32_t e = pentry[idx];
            const float4 r0 = rec[3 * (int64_t)e], r1 = rec[3 * (int64_t)e + 1],
                         r2 = rec[3 * (int64_t)e + 2];
            s_pos[tid] = make_float4(r0.x, r0.y, r1.z, r1.y);
            s_con[tid] = make_float4(r0.z, r0.w, r1.x, __uint_as_float(e));
            s_col[tid] = r2;
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const uint32_t rel = b_end - 1u - (uint32_t)j - start;   // list position
            float d_u = 0.f, d_v = 0.f, d_a = 0.f, d_b = 0.f, d_c = 0.f, d_o = 0.f;
            float d_r = 0.f, d_g = 0.f, d_bl = 0.f;
            bool contrib = false;
            const float4 P = s_pos[j];
            const float4 Q = s_con[j];
            Splat s;
            if (rel < last && splat_alpha(px, py, P.x, P.y, P.z, P.w, Q.x, Q.y, Q.z, rp, s)) {
                const float4 col = s_col[j];
                const float om = 1.f - s.alpha;
                const float Ti = T / om;
                const float w = s.alpha * Ti;
                d_r = g0 * w;
                d_g = g1 * w;
                d_bl = g2 * w;
                const float d_alpha = g0 * (col.x * Ti - S0 / om) + g1 * (col.y * Ti - S1 / om) +
                                      g2 * (col.z * Ti - S2 / om);
                S0 = fmaf(col.x, w, S0);
                S1 = fmaf(col.y, w, S1);
                S2 = fmaf(col.z, w, S2);
                T = Ti;
                if (!s.clamped) {
                    const float dP = d_alpha * s.alpha;
                    d_o = d_alpha * s.ex;
                    d_a = -0.5f * dP * s.dx * s.dx;
                    d_b = -dP * s.dx * s.dy;
                    d_c = -0.5f * dP * s.dy * s.dy;
                    d_u = dP * (Q.x * s.dx + Q.y * s.dy);
                    d_v = dP * (Q.y * s.dx + Q.z * s.dy);
                }
                contrib = true;
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
            if (lane_id() == 63) {
                float* acc = accum + (int64_t)kAccumFloats * __float_as_uint(Q.w);
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
    const dim3 grid((unsigned)L.total_tiles);
    if (rp.tile_w == 16 && rp.tile_h == 16)
        hipLaunchKernelGGL((raster_forward_kernel<16, 16>), grid, dim3(256), 0, s, views, rp,
                           ranges, pentry, rec, out_rgb, tf, nl, cnt);
    else if (rp.tile_w == 8 && rp.tile_h == 8)
        hipLaunchKernelGGL((raster_forward_kernel<8, 8>), grid, dim3(64), 0, s, views, rp, ranges,
                           pentry, rec, out_rgb, tf, nl, cnt);
    else
        hipLaunchKernelGGL((raster_forward_kernel<32, 8>), grid, dim3(256), 0, s, views, rp,
                           ranges, pentry, rec, out_rgb, tf, nl, cnt);
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
    const dim3 grid((unsigned)L.total_tiles);
    if (rp.tile_w == 16 && rp.tile_h == 16)
        hipLaunchKernelGGL((raster_backward_kernel<16, 16>), grid, dim3(256), 0, s, views, rp,
                           ranges, pentry, rec, tf, nl, dl_drgb, gate, acc);
    else if (rp.tile_w == 8 && rp.tile_h == 8)
        hipLaunchKernelGGL((raster_backward_kernel<8, 8>), grid, dim3(64), 0, s, views, rp, ranges,
                           pentry, rec, tf, nl, dl_drgb, gate, acc);
    else
        hipLaunchKernelGGL((raster_backward_kernel<32, 8>), grid, dim3(256), 0, s, views, rp,
                           ranges, pentry, rec, tf, nl, dl_drgb, gate, acc);
    return hipGetLastError();
}

}  // namespace sgs
