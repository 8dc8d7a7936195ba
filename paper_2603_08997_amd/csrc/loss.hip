// Photometric loss (paper Eq. 6): L = (1 - lambda) L1 + lambda (1 - SSIM),
// SSIM with an 11x11 Gaussian window (sigma 1.5), zero-padded same-size
// filtering, both terms averaged over the 3 H W values.
//
// One 16x16 output tile per workgroup. The tile plus a 5-pixel halo of all
// three channels of both images is staged in LDS once; per channel the five
// local moments (mu_x, mu_y, E[x^2], E[y^2], E[xy]) are filtered separably,
// the horizontal pass forming the products from x and y as it reads them.
// Per-tile sums go to a partials array that a one-workgroup kernel reduces in
// index order in binary64, so the loss is bit-reproducible.
//
// Backward: per pixel p the SSIM value S(p) depends on x through mu_x(p),
// E[x^2](p) and E[xy](p); the map derivatives dS/dmu_x, dS/dE[x^2],
// dS/dE[xy] are written by the forward (when a workspace holds them) and
// filtered again by the backward (the window is symmetric):
//   dSSIM/dx(q) = F[dS/dmu_x](q) + 2 x(q) F[dS/dE[x^2]](q) + y(q) F[dS/dE[xy]](q).
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

constexpr int kT = 16;               // output tile edge
constexpr int kR = 5;                // window radius
constexpr int kE = kT + 2 * kR;      // staged edge (26)
constexpr int kThreads = kT * kT;
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

// Loss workspace: [partials: 2 * blocks floats][maps: 9 * H * W floats]
struct LossLayout {
    int64_t blocks;
    size_t partials, maps, total;
};

LossLayout loss_layout(int w, int h) {
    LossLayout L;
    L.blocks = (int64_t)((w + kT - 1) / kT) * ((h + kT - 1) / kT);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    L.partials = 0;
    L.maps = al(L.partials + sizeof(float) * 2 * L.blocks);
    L.total = al(L.maps + sizeof(float) * 9 * (size_t)w * h);
    return L;
}

// The reference image of a call: the given one, or image *d_view (clamped)
// of an array of n_targets images of 3 H W floats.
__device__ __forceinline__ const float* target_of(const TargetRef& t, int64_t image_floats) {
    if (t.d_view == nullptr) return t.base;
    const int i = min(max(*t.d_view, 0), t.n_targets - 1);
    return t.base + (int64_t)i * image_floats;
}

// Stages field f of channels 0..2 of an image (plane stride `plane`) around
// the tile into dst[ch][26][26], zero outside the image.
__device__ __forceinline__ void stage3(const float* __restrict__ img, int64_t plane, int w, int h,
                                       int x0, int y0, float (*dst)[kE][kE]) {
    for (int i = threadIdx.x; i < 3 * kE * kE; i += kThreads) {
        const int ch = i / (kE * kE), rc = i % (kE * kE);
        const int r = rc / kE, c = rc % kE;
        const int gx = x0 + c, gy = y0 + r;
        dst[ch][r][c] = (gx >= 0 && gx < w && gy >= 0 && gy < h)
                            ? img[ch * plane + (int64_t)gy * w + gx] : 0.f;
    }
}

// The five filtered moments of channel ch at this thread's output pixel.
__device__ __forceinline__ void moments(const float (*X)[kE], const float (*Y)[kE],
                                        float (*hb)[kE][kT], const Window& W, float m[5]) {
    const int tid = threadIdx.x;
    for (int i = tid; i < kE * kT; i += kThreads) {
        const int r = i / kT, c = i % kT;
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            const float a = X[r][c + k], b = Y[r][c + k], g = W.g[k];
            s0 = fmaf(g, a, s0);
            s1 = fmaf(g, b, s1);
            s2 = fmaf(g, a * a, s2);
            s3 = fmaf(g, b * b, s3);
            s4 = fmaf(g, a * b, s4);
        }
        hb[0][r][c] = s0;
        hb[1][r][c] = s1;
        hb[2][r][c] = s2;
        hb[3][r][c] = s3;
        hb[4][r][c] = s4;
    }
    __syncthreads();
    const int r = tid / kT, c = tid % kT;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < 11; ++k) s = fmaf(W.g[k], hb[f][r + k][c], s);
        m[f] = s;
    }
    __syncthreads();
}

// Forward tile: sums of |x - y| and of S over the tile's 3 x 256 values into
// partials[2 blk] and, with kMaps, the maps dS/dmu_x, dS/dE[x^2], dS/dE[xy]
// the backward filters. The maps are written on every forward: forming them
// again in the backward would repeat the whole moment pass, which costs more
// than the writes it saves on iterations whose backward is skipped.
template <bool kMaps>
__global__ void __launch_bounds__(kThreads) ssim_forward_kernel(
    const float* __restrict__ x, TargetRef target, int w, int h, Window W,
    float* __restrict__ partials, float* __restrict__ maps) {
    __shared__ float sx[3][kE][kE];
    __shared__ float sy[3][kE][kE];
    __shared__ float hb[5][kE][kT];
    __shared__ float red[2][kThreads / 64];
    const int tid = threadIdx.x;
    const int bx = blockIdx.x, by = blockIdx.y;
    const int x0 = bx * kT - kR, y0 = by * kT - kR;
    const int ox = bx * kT + tid % kT, oy = by * kT + tid / kT;
    const bool inside = ox < w && oy < h;
    const int64_t plane = (int64_t)w * h;
    const float* __restrict__ y = target_of(target, 3 * plane);
    stage3(x, plane, w, h, x0, y0, sx);
    stage3(y, plane, w, h, x0, y0, sy);
    __syncthreads();
    float s_l1 = 0.f, s_ssim = 0.f;
    for (int ch = 0; ch < 3; ++ch) {
        float m[5];
        moments(sx[ch], sy[ch], hb, W, m);
        if (inside) {
            const float mx = m[0], my = m[1];
            const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
            const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
            const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
            const float D = B1 * B2;
            const float S = (A1 * A2) / D;
            const float a = sx[ch][tid / kT + kR][tid % kT + kR];
            const float b = sy[ch][tid / kT + kR][tid % kT + kR];
            s_l1 += fabsf(a - b);
            s_ssim += S;
            if (kMaps) {
                const int64_t pix = (int64_t)oy * w + ox;
                maps[(0 * 3 + ch) * plane + pix] =
                    2.f * my * (A2 - A1) / D - 2.f * mx * S * (1.f / B1 - 1.f / B2);
                maps[(1 * 3 + ch) * plane + pix] = -S / B2;
                maps[(2 * 3 + ch) * plane + pix] = 2.f * A1 / D;
            }
        }
    }
    // fixed-order workgroup sum
    s_l1 = wave_sum(s_l1);
    s_ssim = wave_sum(s_ssim);
    if (lane_id() == 0) {
        red[0][tid / 64] = s_l1;
        red[1][tid / 64] = s_ssim;
    }
    __syncthreads();
    if (tid == 0) {
        const int64_t blk = (int64_t)by * gridDim.x + bx;
        partials[2 * blk] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        partials[2 * blk + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// Sum of the per-tile partials in index order (binary64), then Eq. 6.
__global__ void __launch_bounds__(1024) loss_reduce_kernel(const float* __restrict__ partials,
                                                           int64_t nb, double count, float lambda,
                                                           float* __restrict__ d_loss) {
    __shared__ double dred[2][1024];
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t i = tid; i < nb; i += 1024) {
        a += (double)partials[2 * i];
        b += (double)partials[2 * i + 1];
    }
    dred[0][tid] = a;
    dred[1][tid] = b;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (tid < st) {
            dred[0][tid] += dred[0][tid + st];
            dred[1][tid] += dred[1][tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double l1 = dred[0][0] / count, ssim = dred[1][0] / count;
        *d_loss = (float)((1.0 - (double)lambda) * l1 + (double)lambda * (1.0 - ssim));
    }
}

__global__ void __launch_bounds__(kThreads) ssim_backward_kernel(
    const float* __restrict__ x, TargetRef target, int w, int h, float lambda,
    Window W, const float* __restrict__ maps, const int32_t* __restrict__ gate,
    float* __restrict__ dl) {
    if (gate_closed(gate)) return;
    __shared__ float sm[3][kE][kE];   // the three maps of one channel
    __shared__ float hb[3][kE][kT];
    const int tid = threadIdx.x;
    const int bx = blockIdx.x, by = blockIdx.y;
    const int x0 = bx * kT - kR, y0 = by * kT - kR;
    const int ox = bx * kT + tid % kT, oy = by * kT + tid / kT;
    const bool inside = ox < w && oy < h;
    const int64_t plane = (int64_t)w * h;
    const float* __restrict__ y = target_of(target, 3 * plane);
    const float inv = 1.f / (3.f * (float)w * (float)h);
    for (int ch = 0; ch < 3; ++ch) {
        for (int i = tid; i < 3 * kE * kE; i += kThreads) {
            const int f = i / (kE * kE), rc = i % (kE * kE);
            const int r = rc / kE, c = rc % kE;
            const int gx = x0 + c, gy = y0 + r;
            sm[f][r][c] = (gx >= 0 && gx < w && gy >= 0 && gy < h)
                              ? maps[(f * 3 + ch) * plane + (int64_t)gy * w + gx] : 0.f;
        }
        __syncthreads();
        // horizontal pass: two neighbouring outputs per thread share 10 of
        // their 12 inputs (kE rows x kT / 2 pairs: one round of the workgroup)
        for (int i = tid; i < kE * (kT / 2); i += kThreads) {
            const int r = i / (kT / 2), c = 2 * (i % (kT / 2));
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                float v[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) v[k] = sm[f][r][c + k];
                float s0 = 0.f, s1 = 0.f;
#pragma unroll
                for (int k = 0; k < 11; ++k) {
                    s0 = fmaf(W.g[k], v[k], s0);
                    s1 = fmaf(W.g[k], v[k + 1], s1);
                }
                hb[f][r][c] = s0;
                hb[f][r][c + 1] = s1;
            }
        }
        __syncthreads();
        const int r = tid / kT, c = tid % kT;
        float F0 = 0.f, F1 = 0.f, F2 = 0.f;
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            F0 = fmaf(W.g[k], hb[0][r + k][c], F0);
            F1 = fmaf(W.g[k], hb[1][r + k][c], F1);
            F2 = fmaf(W.g[k], hb[2][r + k][c], F2);
        }
        if (inside) {
            const int64_t pix = (int64_t)oy * w + ox;
            const float a = x[ch * plane + pix], b = y[ch * plane + pix];
            const float d_ssim = F0 + 2.f * a * F1 + b * F2;
            const float sgn = a > b ? 1.f : (a < b ? -1.f : 0.f);
            dl[ch * plane + pix] = (1.f - lambda) * sgn * inv - lambda * d_ssim * inv;
        }
        __syncthreads();
    }
}

}  // namespace

size_t loss_workspace_bytes(int w, int h) { return loss_layout(w, h).total; }

int64_t loss_partial_floats(int w, int h) { return 2 * loss_layout(w, h).blocks; }

hipError_t launch_loss_partials(const float* rgb, TargetRef target, int w, int h, float lambda,
                                float* partials, float* d_loss, hipStream_t s) {
    const LossLayout L = loss_layout(w, h);
    const dim3 grid((unsigned)((w + kT - 1) / kT), (unsigned)((h + kT - 1) / kT));
    hipLaunchKernelGGL((ssim_forward_kernel<false>), grid, dim3(kThreads), 0, s, rgb, target, w, h,
                       make_window(), partials, nullptr);
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(1024), 0, s, partials, L.blocks,
                       3.0 * (double)w * (double)h, lambda, d_loss);
    return hipGetLastError();
}

hipError_t launch_loss_forward(const float* rgb, TargetRef target, int w, int h, float lambda,
                               char* ws, float* d_loss, hipStream_t s) {
    const LossLayout L = loss_layout(w, h);
    const dim3 grid((unsigned)((w + kT - 1) / kT), (unsigned)((h + kT - 1) / kT));
    float* partials = reinterpret_cast<float*>(ws + L.partials);
    float* maps = reinterpret_cast<float*>(ws + L.maps);
    hipLaunchKernelGGL((ssim_forward_kernel<true>), grid, dim3(kThreads), 0, s, rgb, target, w, h,
                       make_window(), partials, maps);
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(1024), 0, s, partials, L.blocks,
                       3.0 * (double)w * (double)h, lambda, d_loss);
    return hipGetLastError();
}

hipError_t launch_loss_backward(const float* rgb, TargetRef target, int w, int h, float lambda,
                                char* ws, const int32_t* gate, float* dl, hipStream_t s) {
    const LossLayout L = loss_layout(w, h);
    const dim3 grid((unsigned)((w + kT - 1) / kT), (unsigned)((h + kT - 1) / kT));
    const float* maps = reinterpret_cast<const float*>(ws + L.maps);
    hipLaunchKernelGGL(ssim_backward_kernel, grid, dim3(kThreads), 0, s, rgb, target, w, h, lambda,
                       make_window(), maps, gate, dl);
    return hipGetLastError();
}

}  // namespace sgs
