// Photometric loss (paper Eq. 6): L = (1 - lambda) L1 + lambda (1 - SSIM),
// SSIM with an 11x11 Gaussian window (sigma 1.5), zero-padded same-size
// filtering, both terms averaged over the 3 H W values.
//
// One 16x16 output tile per workgroup: the tile plus a 5-pixel halo is
// staged in LDS, the five local moments (mu_x, mu_y, E[x^2], E[y^2], E[xy])
// are filtered separably, and the per-tile sums are reduced across tiles in a
// fixed order by the last workgroup to finish, so the loss is bit-reproducible.
//
// Backward: per pixel p the SSIM value S(p) depends on x through mu_x(p),
// E[x^2](p) and E[xy](p); the map derivatives dS/dmu_x, dS/dE[x^2],
// dS/dE[xy] are written once and filtered again (the window is symmetric):
//   dSSIM/dx(q) = F[dS/dmu_x](q) + 2 x(q) F[dS/dE[x^2]](q) + y(q) F[dS/dE[xy]](q).
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

constexpr int kT = 16;               // output tile edge
constexpr int kR = 5;                // window radius
constexpr int kE = kT + 2 * kR;      // staged edge (26)
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Window {
    float g[11];
};

Window make_window() {
    Window w;
    double s = 0.0, v[11];
    for (int k = 0; k < 11; ++k) {
        const double d = k - 5;
        v[k] = std::exp(-(d * d) / (2.0 * 1.5 * 1.5));
        s += v[k];
    }
    for (int k = 0; k < 11; ++k) w.g[k] = (float)(v[k] / s);
    return w;
}

// Loss workspace: [partials: 2 * blocks floats][counter: 64 B][maps: 9 * H * W floats]
struct LossLayout {
    int64_t blocks;
    size_t partials, counter, maps, total;
};

LossLayout loss_layout(int w, int h) {
    LossLayout L;
    L.blocks = (int64_t)((w + kT - 1) / kT) * ((h + kT - 1) / kT);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    L.partials = 0;
    L.counter = al(L.partials + sizeof(float) * 2 * L.blocks);
    L.maps = al(L.counter + 64);
    L.total = al(L.maps + sizeof(float) * 9 * (size_t)w * h);
    return L;
}

// Filters the staged 26x26 fields (k of them) to the 16x16 tile: horizontal
// pass into hbuf[k][26][16], then vertical.
template <int K>
__device__ __forceinline__ void separable(const float (*src)[kE][kE], float (*hbuf)[kE][kT],
                                          const Window& W, int tid, float out[K]) {
    for (int i = tid; i < kE * kT; i += 256) {
        const int r = i / kT, c = i % kT;
#pragma unroll
        for (int f = 0; f < K; ++f) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < 11; ++k) s = fmaf(W.g[k], src[f][r][c + k], s);
            hbuf[f][r][c] = s;
        }
    }
    __syncthreads();
    const int r = tid / kT, c = tid % kT;
#pragma unroll
    for (int f = 0; f < K; ++f) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < 11; ++k) s = fmaf(W.g[k], hbuf[f][r + k][c], s);
        out[f] = s;
    }
    __syncthreads();
}

// Forward tile: sums of |x - y| and of S over the tile's 3 x 256 values.
// With MAPS, also writes dS/dmu_x, dS/dE[x^2], dS/dE[xy] per pixel and channel.
template <bool MAPS>
__global__ void __launch_bounds__(256) ssim_forward_kernel(const float* __restrict__ x,
                                                           const float* __restrict__ y, int w,
                                                           int h, float lambda, Window W,
                                                           float* __restrict__ partials,
                                                           uint32_t* __restrict__ counter,
                                                           float* __restrict__ maps,
                                                           float* __restrict__ d_loss,
                                                           const int32_t* __restrict__ gate) {
    if (MAPS && gate_closed(gate)) return;
    __shared__ float src[5][kE][kE];
    __shared__ float hbuf[5][kE][kT];
    __shared__ float red[2][4];
    __shared__ bool last_block;
    const int tid = threadIdx.x;
    const int bx = blockIdx.x, by = blockIdx.y;
    const int x0 = bx * kT - kR, y0 = by * kT - kR;
    const int ox = bx * kT + tid % kT, oy = by * kT + tid / kT;
    const bool inside = ox < w && oy < h;
    const int64_t plane = (int64_t)w * h;
    float s_l1 = 0.f, s_ssim = 0.f;
    for (int ch = 0; ch < 3; ++ch) {
        const float* xc = x + ch * plane;
        const float* yc = y + ch * plane;
        for (int i = tid; i < kE * kE; i += 256) {
            const int r = i / kE, c = i % kE;
            const int gx = x0 + c, gy = y0 + r;
            float a = 0.f, b = 0.f;
            if (gx >= 0 && gx < w && gy >= 0 && gy < h) {
                a = xc[(int64_t)gy * w + gx];
                b = yc[(int64_t)gy * w + gx];
            }
            src[0][r][c] = a;
            src[1][r][c] = b;
            src[2][r][c] = a * a;
            src[3][r][c] = b * b;
            src[4][r][c] = a * b;
        }
        __syncthreads();
        float m[5];
        separable<5>(src, hbuf, W, tid, m);
        if (inside) {
            const float mx = m[0], my = m[1];
            const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
            const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
            const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
            const float D = B1 * B2;
            const float S = (A1 * A2) / D;
            const float a = src[0][tid / kT + kR][tid % kT + kR];
            const float b = src[1][tid / kT + kR][tid % kT + kR];
            s_l1 += fabsf(a - b);
            s_ssim += S;
            if (MAPS) {
                const int64_t pix = (int64_t)oy * w + ox;
                maps[(0 * 3 + ch) * plane + pix] =
                    2.f * my * (A2 - A1) / D - 2.f * mx * S * (1.f / B1 - 1.f / B2);
                maps[(1 * 3 + ch) * plane + pix] = -S / B2;
                maps[(2 * 3 + ch) * plane + pix] = 2.f * A1 / D;
            }
        }
        __syncthreads();
    }
    if (MAPS) return;
    // fixed-order block reduction
    s_l1 = wave_sum(s_l1);
    s_ssim = wave_sum(s_ssim);
    if (lane_id() == 0) {
        red[0][tid / 64] = s_l1;
        red[1][tid / 64] = s_ssim;
    }
    __syncthreads();
    const int64_t blk = (int64_t)by * gridDim.x + bx;
    if (tid == 0) {
        partials[2 * blk] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        partials[2 * blk + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        __threadfence();
        const uint32_t ticket = atomicAdd(counter, 1u);
        last_block = ticket == gridDim.x * gridDim.y - 1;
    }
    __syncthreads();
    if (!last_block) return;
    __threadfence();
    // the last block sums every tile's partials in index order, in binary64
    const int64_t nb = (int64_t)gridDim.x * gridDim.y;
    __shared__ double dred[2][256];
    double a = 0.0, b = 0.0;
    for (int64_t i = tid; i < nb; i += 256) {
        a += (double)__hip_atomic_load(&partials[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        b += (double)__hip_atomic_load(&partials[2 * i + 1], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    }
    dred[0][tid] = a;
    dred[1][tid] = b;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            dred[0][tid] += dred[0][tid + st];
            dred[1][tid] += dred[1][tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double cnt = 3.0 * (double)w * (double)h;
        const double l1 = dred[0][0] / cnt, ssim = dred[1][0] / cnt;
        *d_loss = (float)((1.0 - (double)lambda) * l1 + (double)lambda * (1.0 - ssim));
        *counter = 0u;
    }
}

__global__ void __launch_bounds__(256) ssim_backward_kernel(const float* __restrict__ x,
                                                            const float* __restrict__ y, int w,
                                                            int h, float lambda, Window W,
                                                            const float* __restrict__ maps,
                                                            const int32_t* __restrict__ gate,
                                                            float* __restrict__ dl) {
    if (gate_closed(gate)) return;
    __shared__ float src[3][kE][kE];
    __shared__ float hbuf[3][kE][kT];
    const int tid = threadIdx.x;
    const int bx = blockIdx.x, by = blockIdx.y;
    const int x0 = bx * kT - kR, y0 = by * kT - kR;
    const int ox = bx * kT + tid % kT, oy = by * kT + tid / kT;
    const bool inside = ox < w && oy < h;
    const int64_t plane = (int64_t)w * h;
    const float inv = 1.f / (3.f * (float)w * (float)h);
    for (int ch = 0; ch < 3; ++ch) {
        for (int i = tid; i < kE * kE; i += 256) {
            const int r = i / kE, c = i % kE;
            const int gx = x0 + c, gy = y0 + r;
            const bool in = gx >= 0 && gx < w && gy >= 0 && gy < h;
            const int64_t pix = (int64_t)gy * w + gx;
#pragma unroll
            for (int f = 0; f < 3; ++f) src[f][r][c] = in ? maps[(f * 3 + ch) * plane + pix] : 0.f;
        }
        __syncthreads();
        float F[3];
        separable<3>(src, hbuf, W, tid, F);
        if (inside) {
            const int64_t pix = (int64_t)oy * w + ox;
            const float a = x[ch * plane + pix], b = y[ch * plane + pix];
            const float d_ssim = F[0] + 2.f * a * F[1] + b * F[2];
            const float sgn = a > b ? 1.f : (a < b ? -1.f : 0.f);
            dl[ch * plane + pix] = (1.f - lambda) * sgn * inv - lambda * d_ssim * inv;
        }
    }
}

}  // namespace

size_t loss_workspace_bytes(int w, int h) { return loss_layout(w, h).total; }

hipError_t launch_loss_forward(const float* rgb, const float* target, int w, int h, float lambda,
                               char* ws, float* d_loss, hipStream_t s) {
    const LossLayout L = loss_layout(w, h);
    const dim3 grid((unsigned)((w + kT - 1) / kT), (unsigned)((h + kT - 1) / kT));
    hipLaunchKernelGGL(ssim_forward_kernel<false>, grid, dim3(256), 0, s, rgb, target, w, h, lambda,
                       make_window(), reinterpret_cast<float*>(ws + L.partials),
                       reinterpret_cast<uint32_t*>(ws + L.counter), (float*)nullptr, d_loss,
                       (const int32_t*)nullptr);
    return hipGetLastError();
}

hipError_t launch_loss_backward(const float* rgb, const float* target, int w, int h, float lambda,
                                char* ws, const int32_t* gate, float* dl, hipStream_t s) {
    const LossLayout L = loss_layout(w, h);
    const dim3 grid((unsigned)((w + kT - 1) / kT), (unsigned)((h + kT - 1) / kT));
    float* maps = reinterpret_cast<float*>(ws + L.maps);
    hipLaunchKernelGGL(ssim_forward_kernel<true>, grid, dim3(256), 0, s, rgb, target, w, h, lambda,
                       make_window(), (float*)nullptr, (uint32_t*)nullptr, maps, (float*)nullptr,
                       gate);
    hipLaunchKernelGGL(ssim_backward_kernel, grid, dim3(256), 0, s, rgb, target, w, h, lambda,
                       make_window(), maps, gate, dl);
    return hipGetLastError();
}

}  // namespace sgs
