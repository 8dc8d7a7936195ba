// Projection of 3D Gaussians (paper Sec. 3, Eqs. 2-3, SH colour) and its
// adjoint. One thread per (view, Gaussian) entry; parameters are read as
// coalesced planes of the [F][stride] layout.
#include <algorithm>

#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

// Real SH normalisation constants with the Condon-Shortley phase (index
// k = l^2 + l + m), evaluated at a unit direction.
constexpr float kY0 = 0.28209479177387814f;
constexpr float kY1 = 0.4886025119029199f;
constexpr float kY2a = 1.0925484305920792f;
constexpr float kY2b = 0.31539156525252005f;
constexpr float kY2c = 0.5462742152960396f;
constexpr float kY3a = 0.5900435899266435f;
constexpr float kY3b = 2.890611442640554f;
constexpr float kY3c = 0.4570457994644658f;
constexpr float kY3d = 0.3731763325901154f;
constexpr float kY3e = 1.445305721320277f;

__device__ __forceinline__ void sh_eval(int deg, float x, float y, float z, float* Y) {
    Y[0] = kY0;
    if (deg < 1) return;
    Y[1] = -kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = -kY1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kY2a * x * y;
    Y[5] = -kY2a * y * z;
    Y[6] = kY2b * (2.f * zz - xx - yy);
    Y[7] = -kY2a * x * z;
    Y[8] = kY2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = -kY3a * y * (3.f * xx - yy);
    Y[10] = kY3b * x * y * z;
    Y[11] = -kY3c * y * (4.f * zz - xx - yy);
    Y[12] = kY3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -kY3c * x * (4.f * zz - xx - yy);
    Y[14] = kY3e * z * (xx - yy);
    Y[15] = -kY3a * x * (xx - 3.f * yy);
}

// d/d(x, y, z) of sum_k w_k Y_k(x, y, z), accumulated into g.
__device__ __forceinline__ void sh_grad_dir(int deg, float x, float y, float z, const float* w,
                                            float g[3]) {
    g[0] = g[1] = g[2] = 0.f;
    if (deg < 1) return;
    g[0] += -kY1 * w[3];
    g[1] += -kY1 * w[1];
    g[2] += kY1 * w[2];
    if (deg < 2) return;
    g[0] += kY2a * y * w[4] - kY2a * z * w[7] - 2.f * kY2b * x * w[6] + 2.f * kY2c * x * w[8];
    g[1] += kY2a * x * w[4] - kY2a * z * w[5] - 2.f * kY2b * y * w[6] - 2.f * kY2c * y * w[8];
    g[2] += -kY2a * y * w[5] + 4.f * kY2b * z * w[6] - kY2a * x * w[7];
    if (deg < 3) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    g[0] += -kY3a * 6.f * x * y * w[9] + kY3b * y * z * w[10] + kY3c * 2.f * x * y * w[11]
            - kY3d * 6.f * x * z * w[12] - kY3c * (4.f * zz - 3.f * xx - yy) * w[13]
            + kY3e * 2.f * x * z * w[14] - kY3a * (3.f * xx - 3.f * yy) * w[15];
    g[1] += -kY3a * (3.f * xx - 3.f * yy) * w[9] + kY3b * x * z * w[10]
            - kY3c * (4.f * zz - xx - 3.f * yy) * w[11] - kY3d * 6.f * y * z * w[12]
            + kY3c * 2.f * x * y * w[13] - kY3e * 2.f * y * z * w[14] + kY3a * 6.f * x * y * w[15];
    g[2] += kY3b * x * y * w[10] - kY3c * 8.f * y * z * w[11]
            + kY3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12] - kY3c * 8.f * x * z * w[13]
            + kY3e * (xx - yy) * w[14];
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.f / (1.f + expf(-x)); }

struct Geometry {
    float tx, ty, tz;          // camera-space centre
    float xr, yr;              // tx/tz, ty/tz after the clamp
    bool clx, cly;             // clamp active
    float qn[4], qnorm;        // normalised quaternion and |q|
    float s[3];                // scales
    float Rq[9];               // rotation of qn
    float Sig[6];              // 3D covariance xx xy xz yy yz zz
    float T[6];                // J W (2x3, row-major)
    float sxx, sxy, syy;       // 2D covariance incl. dilation
};

__device__ __forceinline__ bool compute_geometry(const float mu[3], const float ls[3],
                                                 const float q[4], const ViewDev& V,
                                                 const RasterDev& rp, Geometry& G) {
    G.tx = V.R[0] * mu[0] + V.R[1] * mu[1] + V.R[2] * mu[2] + V.t[0];
    G.ty = V.R[3] * mu[0] + V.R[4] * mu[1] + V.R[5] * mu[2] + V.t[1];
    G.tz = V.R[6] * mu[0] + V.R[7] * mu[1] + V.R[8] * mu[2] + V.t[2];
    if (!(G.tz > rp.near_z)) return false;
    const float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    G.qnorm = sqrtf(qq);
    if (!(G.qnorm > 0.f) || !isfinite(G.qnorm)) return false;
    const float w = q[0] / G.qnorm, x = q[1] / G.qnorm, y = q[2] / G.qnorm, z = q[3] / G.qnorm;
    G.qn[0] = w; G.qn[1] = x; G.qn[2] = y; G.qn[3] = z;
    float* R = G.Rq;
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
    G.s[0] = expf(ls[0]); G.s[1] = expf(ls[1]); G.s[2] = expf(ls[2]);
    float M[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[3 * i + j] = R[3 * i + j] * G.s[j];
    // Sigma = M M^T (Eq. 2)
    G.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    G.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    G.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    G.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    G.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    G.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
    // EWA Jacobian at the centre (Eq. 3), clamped ray direction.
    const float xr = G.tx / G.tz, yr = G.ty / G.tz;
    G.clx = !(xr >= -V.lim_x && xr <= V.lim_x);
    G.cly = !(yr >= -V.lim_y && yr <= V.lim_y);
    G.xr = fminf(fmaxf(xr, -V.lim_x), V.lim_x);
    G.yr = fminf(fmaxf(yr, -V.lim_y), V.lim_y);
    const float j00 = V.fx / G.tz, j02 = -V.fx * G.xr / G.tz;
    const float j11 = V.fy / G.tz, j12 = -V.fy * G.yr / G.tz;
    // T = J W, W = camera rotation
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        G.T[c] = j00 * V.R[c] + j02 * V.R[6 + c];
        G.T[3 + c] = j11 * V.R[3 + c] + j12 * V.R[6 + c];
    }
    // Sigma2D = T Sigma T^T
    const float* S = G.Sig;
    float a0 = G.T[0] * S[0] + G.T[1] * S[1] + G.T[2] * S[2];
    float a1 = G.T[0] * S[1] + G.T[1] * S[3] + G.T[2] * S[4];
    float a2 = G.T[0] * S[2] + G.T[1] * S[4] + G.T[2] * S[5];
    float b0 = G.T[3] * S[0] + G.T[4] * S[1] + G.T[5] * S[2];
    float b1 = G.T[3] * S[1] + G.T[4] * S[3] + G.T[5] * S[4];
    float b2 = G.T[3] * S[2] + G.T[4] * S[4] + G.T[5] * S[5];
    G.sxx = a0 * G.T[0] + a1 * G.T[1] + a2 * G.T[2] + rp.dilation;
    G.sxy = a0 * G.T[3] + a1 * G.T[4] + a2 * G.T[5];
    G.syy = b0 * G.T[3] + b1 * G.T[4] + b2 * G.T[5] + rp.dilation;
    return true;
}

__device__ __forceinline__ int find_view(int64_t e, int64_t n, int64_t* i) {
    const int v = (int)(e / n);
    *i = e - (int64_t)v * n;
    return v;
}

template <int sh_degree>
__global__ void __launch_bounds__(256) project_kernel(const float* __restrict__ planes, int64_t n,
                                                      int64_t stride, const Views* __restrict__ views,
                                                      RasterDev rp, float4* __restrict__ rec,
                                                      uint32_t* __restrict__ tiles,
                                                      uint32_t* __restrict__ dkey) {
    const int64_t entries = n * views->n;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= entries) return;
    int64_t i;
    const int vi = find_view(e, n, &i);
    const ViewDev& V = views->v[vi];
    const PlaneBuf P{const_cast<float*>(planes), stride};
    const uint32_t off = (uint32_t)i * 4u;
    float mu[3], ls[3], q[4];
#pragma unroll
    for (int k = 0; k < 3; ++k) mu[k] = P.load(k, off);
#pragma unroll
    for (int k = 0; k < 3; ++k) ls[k] = P.load(3 + k, off);
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = P.load(6 + k, off);
    const float logit = P.load(10, off);

    uint32_t ntiles = 0;
    float depth = 0.f;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    Geometry G;
    if (compute_geometry(mu, ls, q, V, rp, G)) {
        const float det = G.sxx * G.syy - G.sxy * G.sxy;
        const float u = V.fx * G.tx / G.tz + V.cx;
        const float v = V.fy * G.ty / G.tz + V.cy;
        const float mid = 0.5f * (G.sxx + G.syy);
        const float lam = mid + sqrtf(fmaxf(mid * mid - det, 0.f));
        const float rf = ceilf(3.f * sqrtf(fmaxf(lam, 0.f)));
        // colour: SH at the view direction, + 0.5, clamped at 0
        constexpr int K = (sh_degree + 1) * (sh_degree + 1);
        float dx = mu[0] - V.C[0], dy = mu[1] - V.C[1], dz = mu[2] - V.C[2];
        const float dn = sqrtf(dx * dx + dy * dy + dz * dz);
        dx /= dn; dy /= dn; dz /= dn;
        float Y[16];
        sh_eval(sh_degree, dx, dy, dz, Y);
        float col[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) col[c] += P.load(11 + 3 * k + c, off) * Y[k];
        }
        const float o = sigmoidf(logit);
        const float ca = G.syy / det, cb = -G.sxy / det, cc = G.sxx / det;
        // overlap box: where o exp(P) can reach alpha_min, within the square r
        float ex = rf, ey = rf;
        bool reach = true;
        if (rp.alpha_min > 0.f) {
            const float tau = logf(o / rp.alpha_min);
            reach = tau >= 0.f;
            ex = fminf(rf, ceilf(sqrtf(2.f * fmaxf(tau, 0.f) * G.sxx)));
            ey = fminf(rf, ceilf(sqrtf(2.f * fmaxf(tau, 0.f) * G.syy)));
        }
        bool ok = det > 0.f && reach && isfinite(u) && isfinite(v) &&
                  fabsf(u) < (float)kMaxExtent && fabsf(v) < (float)kMaxExtent &&
                  rf < (float)kMaxExtent && isfinite(ca) && isfinite(cb) && isfinite(cc) &&
                  isfinite(o) && isfinite(col[0]) && isfinite(col[1]) && isfinite(col[2]);
        if (ok) {
            int x0, x1, y0, y1;
            tile_rect(u, v, (int)ex, (int)ey, rp.tile_w, rp.tile_h, V.tiles_x, V.tiles_y, &x0, &x1,
                      &y0, &y1);
            if (x1 > x0 && y1 > y0) {
                ntiles = super_count(x0, x1, y0, y1, rp.super_tile);
                const uint32_t mask = (col[0] >= 0.f ? 1u : 0u) | (col[1] >= 0.f ? 2u : 0u) |
                                      (col[2] >= 0.f ? 4u : 0u);
                r0 = make_float4(u, v, ca, cb);
                r1 = make_float4(cc, o, ex, ey);
                r2 = make_float4(fmaxf(col[0], 0.f), fmaxf(col[1], 0.f), fmaxf(col[2], 0.f),
                                 __uint_as_float(mask));
                depth = G.tz;
            }
        }
    }
    rec[3 * e + 0] = r0;
    rec[3 * e + 1] = r1;
    rec[3 * e + 2] = r2;
    tiles[e] = ntiles;
    dkey[e] = __float_as_uint(depth);
}

__global__ void __launch_bounds__(256) load_records_kernel(
    int64_t entries, int64_t n, const float* __restrict__ u, const float* __restrict__ v,
    const float* __restrict__ depth, const int32_t* __restrict__ extent,
    const float* __restrict__ conic, const float* __restrict__ opacity,
    const float* __restrict__ rgb, const Views* __restrict__ views, RasterDev rp,
    float4* __restrict__ rec,
    uint32_t* __restrict__ tiles, uint32_t* __restrict__ dkey) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= entries) return;
    int64_t i;
    const ViewDev& V = views->v[find_view(e, n, &i)];
    const int rx = extent[2 * e], ry = extent[2 * e + 1];
    uint32_t ntiles = 0;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    if (rx >= 0 && ry >= 0 && rx < (int)kMaxExtent && ry < (int)kMaxExtent &&
        fabsf(u[e]) < (float)kMaxExtent && fabsf(v[e]) < (float)kMaxExtent) {
        int x0, x1, y0, y1;
        tile_rect(u[e], v[e], rx, ry, rp.tile_w, rp.tile_h, V.tiles_x, V.tiles_y, &x0, &x1, &y0,
                  &y1);
        if (x1 > x0 && y1 > y0) {
            ntiles = super_count(x0, x1, y0, y1, rp.super_tile);
            r0 = make_float4(u[e], v[e], conic[3 * e], conic[3 * e + 1]);
            r1 = make_float4(conic[3 * e + 2], opacity[e], (float)rx, (float)ry);
            r2 = make_float4(rgb[3 * e], rgb[3 * e + 1], rgb[3 * e + 2], __uint_as_float(7u));
        }
    }
    rec[3 * e + 0] = r0;
    rec[3 * e + 1] = r1;
    rec[3 * e + 2] = r2;
    tiles[e] = ntiles;
    dkey[e] = __float_as_uint(ntiles ? depth[e] : 0.f);
}

// Per-view quantities of one visible entry that the SH part of the backward
// needs: unit view direction d, |mu - C|, and dL/d(raw colour) (zero on
// channels the forward clamped at 0).
struct ViewSH {
    float d[3], dn, draw[3];
};

__device__ __forceinline__ void view_sh(const float mu[3], const ViewDev& V, float4 a1, float4 a2,
                                        float4 r2, ViewSH& o) {
    const float dir[3] = {mu[0] - V.C[0], mu[1] - V.C[1], mu[2] - V.C[2]};
    o.dn = sqrtf(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) o.d[c] = dir[c] / o.dn;
    const uint32_t mask = __float_as_uint(r2.w);
    o.draw[0] = (mask & 1u) ? a1.z : 0.f;
    o.draw[1] = (mask & 2u) ? a1.w : 0.f;
    o.draw[2] = (mask & 4u) ? a2.x : 0.f;
}

// Gradient of the non-SH raw parameters of one visible entry (mean through
// the projection, log-scale, quaternion, opacity logit), ADDED to the outputs.
// Returns false if the geometry is culled (never for a visible entry).
__device__ __forceinline__ bool geom_grads(const float mu[3], const float ls[3], const float q[4],
                                           float logit, const ViewDev& V, const RasterDev& rp,
                                           float4 a0, float4 a1, float g_mu[3], float g_ls[3],
                                           float g_q[4], float* g_logit) {
    const float d_u = a0.x, d_v = a0.y, d_ca = a0.z, d_cb = a0.w, d_cc = a1.x, d_o = a1.y;
    Geometry G;
    if (!compute_geometry(mu, ls, q, V, rp, G)) return false;
    // opacity = sigmoid(logit)
    const float o = sigmoidf(logit);
    *g_logit += d_o * o * (1.f - o);
    // conic = inverse of Sigma2D': dSigma' = -Q G Q with G the symmetric
    // gradient [[da, db/2], [db/2, dc]].
    const float det = G.sxx * G.syy - G.sxy * G.sxy;
    const float A = G.syy / det, B = -G.sxy / det, C = G.sxx / det;
    const float g00 = d_ca, g01 = 0.5f * d_cb, g11 = d_cc;
    const float p00 = A * g00 + B * g01, p01 = A * g01 + B * g11;
    const float p10 = B * g00 + C * g01, p11 = B * g01 + C * g11;
    const float d_sxx = -(p00 * A + p01 * B);
    const float d_sxy = -2.f * (p00 * B + p01 * C);   // symmetric entry counted twice
    const float d_syy = -(p10 * B + p11 * C);
    // Sigma2D = T Sigma T^T: dSigma = T^T H T, dT = 2 H T Sigma, H = [[dxx, dxy/2],[dxy/2, dyy]]
    const float h00 = d_sxx, h01 = 0.5f * d_sxy, h11 = d_syy;
    const float* T = G.T;
    float HT[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        HT[c] = h00 * T[c] + h01 * T[3 + c];
        HT[3 + c] = h01 * T[c] + h11 * T[3 + c];
    }
    float dS[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) dS[3 * r + c] = T[r] * HT[c] + T[3 + r] * HT[3 + c];
    const float* S = G.Sig;
    const float Sm[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
    float dT[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            dT[3 * r + c] = 2.f * (HT[3 * r] * Sm[c] + HT[3 * r + 1] * Sm[3 + c] +
                                   HT[3 * r + 2] * Sm[6 + c]);
    // T = J W: dJ = dT W^T (only J00, J02, J11, J12 vary)
    const float dJ00 = dT[0] * V.R[0] + dT[1] * V.R[1] + dT[2] * V.R[2];
    const float dJ02 = dT[0] * V.R[6] + dT[1] * V.R[7] + dT[2] * V.R[8];
    const float dJ11 = dT[3] * V.R[3] + dT[4] * V.R[4] + dT[5] * V.R[5];
    const float dJ12 = dT[3] * V.R[6] + dT[4] * V.R[7] + dT[5] * V.R[8];
    const float tz = G.tz, tz2 = tz * tz;
    float d_tx = 0.f, d_ty = 0.f, d_tz = 0.f;
    d_tz += -dJ00 * V.fx / tz2 + dJ02 * V.fx * G.xr / tz2 - dJ11 * V.fy / tz2 +
            dJ12 * V.fy * G.yr / tz2;
    const float d_xr = -dJ02 * V.fx / tz, d_yr = -dJ12 * V.fy / tz;
    if (!G.clx) { d_tx += d_xr / tz; d_tz += -d_xr * G.tx / tz2; }
    if (!G.cly) { d_ty += d_yr / tz; d_tz += -d_yr * G.ty / tz2; }
    // pixel centre u = fx tx/tz + cx, v = fy ty/tz + cy
    d_tx += d_u * V.fx / tz;
    d_ty += d_v * V.fy / tz;
    d_tz += -d_u * V.fx * G.tx / tz2 - d_v * V.fy * G.ty / tz2;
    // t = R mu + t0
#pragma unroll
    for (int c = 0; c < 3; ++c) g_mu[c] += V.R[c] * d_tx + V.R[3 + c] * d_ty + V.R[6 + c] * d_tz;
    // Sigma = M M^T, M = Rq diag(s): dM = 2 dSigma M; dRq = dM diag(s); ds_j = sum_i dM_ij Rq_ij
    float M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) M[3 * r + c] = G.Rq[3 * r + c] * G.s[c];
    float dM[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            dM[3 * r + c] = 2.f * (dS[3 * r] * M[c] + dS[3 * r + 1] * M[3 + c] +
                                   dS[3 * r + 2] * M[6 + c]);
    float dR[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float ds = 0.f;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            dR[3 * r + c] = dM[3 * r + c] * G.s[c];
            ds += dM[3 * r + c] * G.Rq[3 * r + c];
        }
        g_ls[c] += ds * G.s[c];
    }
    // Rq(qn): derivative of the unit-quaternion rotation matrix
    const float w = G.qn[0], x = G.qn[1], y = G.qn[2], z = G.qn[3];
    float dqn[4];
    dqn[0] = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dqn[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] +
                    z * dR[6] + w * dR[7] - 2.f * x * dR[8]);
    dqn[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] -
                    w * dR[6] + z * dR[7] - 2.f * y * dR[8]);
    dqn[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] +
                    y * dR[5] + x * dR[6] + y * dR[7]);
    // qn = q/|q|
    const float dot = dqn[0] * w + dqn[1] * x + dqn[2] * y + dqn[3] * z;
#pragma unroll
    for (int c = 0; c < 4; ++c) g_q[c] += (dqn[c] - G.qn[c] * dot) / G.qnorm;
    return true;
}

// Threads per workgroup of the per-Gaussian backward kernels, and planes per
// batch of the update loop.
#ifndef SGS_BACKWARD_THREADS
#define SGS_BACKWARD_THREADS 256
#endif
#ifndef SGS_UPDATE_BATCH
#define SGS_UPDATE_BATCH 8
#endif
constexpr int kBackwardThreads = SGS_BACKWARD_THREADS;
constexpr int64_t kAdamBlocks = 2048;   // grid of the fused backward + Adam step
constexpr int kUpdateBatch = SGS_UPDATE_BATCH;

// dL/d(mean) through the view direction of one view: with w_k = sum_c
// d_raw[c] f_{k,c}, the gradient of sum_k w_k Y_k(d) projected orthogonally to
// d and divided by |mu - C|. Added to g_mu.
template <int sh_degree>
__device__ __forceinline__ void sh_mean_grad(const ViewSH& o, const float* f, float g_mu[3]) {
    constexpr int K = (sh_degree + 1) * (sh_degree + 1);
    if constexpr (sh_degree > 0) {
        float w[16];
#pragma unroll
        for (int k = 0; k < K; ++k)
            w[k] = o.draw[0] * f[3 * k] + o.draw[1] * f[3 * k + 1] + o.draw[2] * f[3 * k + 2];
        float gd[3];
        sh_grad_dir(sh_degree, o.d[0], o.d[1], o.d[2], w, gd);
        const float dot = gd[0] * o.d[0] + gd[1] * o.d[1] + gd[2] * o.d[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) g_mu[c] += (gd[c] - o.d[c] * dot) / o.dn;
    }
}

// dL/d f_{k,c} of one view: d_raw[c] Y_k(d).
template <int sh_degree>
__device__ __forceinline__ void sh_coef_grad(const ViewSH& o, float* g_sh) {
    constexpr int K = (sh_degree + 1) * (sh_degree + 1);
    float Y[16];
    sh_eval(sh_degree, o.d[0], o.d[1], o.d[2], Y);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) g_sh[3 * k + c] += o.draw[c] * Y[k];
}

// The per-Gaussian backward. All parameters of the Gaussian are loaded at
// once; the gradient stays in registers, and the update (kFused: Adam on every
// plane, dense as in the paper's optimiser, also for Gaussians visible in no
// view; otherwise: gradient ADDED to grads, visible Gaussians only) runs over
// the planes in batches whose moment (or gradient) loads are issued one batch
// ahead, so that each thread keeps several memory requests in flight.
template <int sh_degree, bool kFused, bool kMulti, bool kSparse = false>
__device__ __forceinline__ void gaussian_backward(float* __restrict__ planes, int64_t n,
                                                  int64_t stride, int64_t i,
                                                  const Views* __restrict__ views,
                                                  const RasterDev& rp,
                                                  const float4* __restrict__ rec,
                                                  const uint32_t* __restrict__ tiles,
                                                  const float4* __restrict__ acc,
                                                  float* __restrict__ grads, const AdamDev* ad,
                                                  const AdamStep* as, float* __restrict__ m,
                                                  float* __restrict__ v) {
    constexpr int K = (sh_degree + 1) * (sh_degree + 1);
    constexpr int NP = 11 + 3 * K;
    // the visible-only step updates a scattered subset of each wave's lines:
    // its accesses go through L2, where the partly written lines meet the
    // full lines its loads brought in; the dense step streams every line
    constexpr int kPlaneCP = kSparse ? 0 : SGS_PLANE_CPOL;
    const PlaneBuf P{planes, stride}, M{m, stride}, Vb{v, stride}, G{grads, stride};
    const uint32_t off = (uint32_t)i * 4u;
    float p[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) p[j] = P.template load<kPlaneCP>(j, off);
    const float* mu = p;
    const float* ls = p + 3;
    const float* q = p + 6;
    const float* f = p + 11;
    float g[11];
#pragma unroll
    for (int j = 0; j < 11; ++j) g[j] = 0.f;
    // SH coefficient gradients: kept per plane for several views, recomputed
    // from the one view's direction otherwise
    float g_sh[kMulti ? 3 * K : 1];
    if constexpr (kMulti) {
#pragma unroll
        for (int j = 0; j < 3 * K; ++j) g_sh[j] = 0.f;
    }
    bool any = false;
    ViewSH one;
    for (int vi = 0; vi < views->n; ++vi) {
        const int64_t e = (int64_t)vi * n + i;
        if (tiles[e] == 0) continue;
        const float4 a0 = acc[3 * e], a1 = acc[3 * e + 1];
        if (geom_grads(mu, ls, q, p[10], views->v[vi], rp, a0, a1, g, g + 3, g + 6, g + 10)) {
            any = true;
            ViewSH o;
            view_sh(mu, views->v[vi], a1, acc[3 * e + 2], rec[3 * e + 2], o);
            sh_mean_grad<sh_degree>(o, f, g);
            if constexpr (kMulti) sh_coef_grad<sh_degree>(o, g_sh);
            else one = o;
        }
    }
    // without a visible entry: nothing to add (gradient accumulation), or,
    // for the visible-only (sparse) Adam step, nothing to update
    if ((!kFused || kSparse) && !any) return;
    float Y[16];
    if constexpr (!kMulti) {
        if (any) sh_eval(sh_degree, one.d[0], one.d[1], one.d[2], Y);
    }
    auto grad_of = [&](int j) -> float {
        if (j < 11) return g[j];
        if constexpr (kMulti) {
            return g_sh[j - 11];
        } else {
            return any ? one.draw[(j - 11) % 3] * Y[(j - 11) / 3] : 0.f;
        }
    };
    constexpr int B = kUpdateBatch;
    constexpr int NB = (NP + B - 1) / B;
    float ma[2][B], va[2][B];
    auto load = [&](int b, int buf) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const int j = b * B + t;
            if (j < NP) {
                if constexpr (kFused) {
                    ma[buf][t] = M.template load<kPlaneCP>(j, off);
                    va[buf][t] = Vb.template load<kPlaneCP>(j, off);
                } else {
                    ma[buf][t] = G.load(j, off);
                }
            }
        }
    };
    load(0, 0);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b + 1 < NB) load(b + 1, (b + 1) & 1);
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const int j = b * B + t;
            if (j < NP) {
                const float gj = grad_of(j);
                if constexpr (kFused) {
                    float pj = p[j], mm = ma[b & 1][t], vv = va[b & 1][t];
                    adam_update(gj, pj, mm, vv, ad->lr[j], *ad, *as);
                    P.template store<kPlaneCP>(j, off, pj);
                    M.template store<kPlaneCP>(j, off, mm);
                    Vb.template store<kPlaneCP>(j, off, vv);
                } else {
                    G.store(j, off, ma[b & 1][t] + gj);
                }
            }
        }
    }
}

// Adjoint of the projection: one thread per Gaussian, gradient ADDED to grads.
template <int sh_degree, bool kMulti>
__global__ void __launch_bounds__(kBackwardThreads) project_backward_kernel(
    const float* __restrict__ planes, int64_t n, int64_t stride, const Views* __restrict__ views,
    RasterDev rp,
    const float4* __restrict__ rec, const uint32_t* __restrict__ tiles,
    const float4* __restrict__ acc, const int32_t* __restrict__ gate, float* __restrict__ grads) {
    if (gate_closed(gate)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    gaussian_backward<sh_degree, false, kMulti>(const_cast<float*>(planes), n, stride, i, views,
                                                rp, rec, tiles, acc, grads, nullptr, nullptr,
                                                nullptr, nullptr);
}

// Adjoint of the projection fused with the Adam step: every Gaussian (dense
// Adam: visible or not) or only the Gaussians visible in a view of the batch
// (kSparse) gets its gradient computed in registers and its parameters, first
// and second moments updated in place; no gradient array is written or read.
template <int sh_degree, bool kMulti, bool kSparse>
__global__ void __launch_bounds__(kBackwardThreads) project_backward_adam_kernel(
    float* __restrict__ planes, int64_t n, int64_t stride, const Views* __restrict__ views,
    RasterDev rp, const float4* __restrict__ rec, const uint32_t* __restrict__ tiles,
    const float4* __restrict__ acc, AdamDev ad, float* __restrict__ m, float* __restrict__ v,
    const int32_t* __restrict__ step, const int32_t* __restrict__ gate) {
    if (gate_closed(gate)) return;
    __shared__ AdamStep s_as;
    if (threadIdx.x == 0) s_as = adam_bias_correction(ad, *step);
    __syncthreads();
    const AdamStep as = s_as;
    // grid-stride over the Gaussians on a grid sized for the machine, so that
    // a closed gate costs a launch of a few thousand workgroups, not one per
    // 256 Gaussians
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        gaussian_backward<sh_degree, true, kMulti, kSparse>(planes, n, stride, i, views, rp, rec,
                                                            tiles, acc, nullptr, &ad, &as, m, v);
}

}  // namespace

hipError_t launch_project(const float* planes, int64_t n, int64_t stride, int sh_degree,
                          const RasterDev& rp, const Layout& L, char* ws, hipStream_t s) {
    const int64_t entries = L.entries;
    if (entries == 0) return hipSuccess;
    const int nt = 256;
    const int64_t nb = (entries + nt - 1) / nt;
    const Views* views = reinterpret_cast<const Views*>(ws + L.views);
    float4* rec = reinterpret_cast<float4*>(ws + L.records);
    uint32_t* tiles = reinterpret_cast<uint32_t*>(ws + L.tiles);
    uint32_t* dkey = reinterpret_cast<uint32_t*>(ws + L.depth);
#define SGS_PK(D)                                                                          \
    hipLaunchKernelGGL(project_kernel<D>, dim3((unsigned)nb), dim3(nt), 0, s, planes, n, stride, \
                       views, rp, rec, tiles, dkey)
    switch (sh_degree) {
        case 0: SGS_PK(0); break;
        case 1: SGS_PK(1); break;
        case 2: SGS_PK(2); break;
        default: SGS_PK(3); break;
    }
#undef SGS_PK
    return hipGetLastError();
}

hipError_t launch_load_records(const float* u, const float* v, const float* depth,
                               const int32_t* extent, const float* conic, const float* opacity,
                               const float* rgb, int64_t n, const RasterDev& rp, const Layout& L,
                               char* ws, hipStream_t s) {
    const int64_t entries = L.entries;
    if (entries == 0) return hipSuccess;
    const int nt = 256;
    const int64_t nb = (entries + nt - 1) / nt;
    hipLaunchKernelGGL(load_records_kernel, dim3((unsigned)nb), dim3(nt), 0, s, entries, n, u, v,
                       depth, extent, conic, opacity, rgb,
                       reinterpret_cast<const Views*>(ws + L.views), rp,
                       reinterpret_cast<float4*>(ws + L.records),
                       reinterpret_cast<uint32_t*>(ws + L.tiles),
                       reinterpret_cast<uint32_t*>(ws + L.depth));
    return hipGetLastError();
}

#define SGS_DISPATCH_DEG(MACRO, multi)                                      \
    switch (sh_degree) {                                                    \
        case 0: if (multi) MACRO(0, true); else MACRO(0, false); break;    \
        case 1: if (multi) MACRO(1, true); else MACRO(1, false); break;    \
        case 2: if (multi) MACRO(2, true); else MACRO(2, false); break;    \
        default: if (multi) MACRO(3, true); else MACRO(3, false); break;   \
    }

hipError_t launch_project_backward(const float* planes, int64_t n, int64_t stride,
                                   int sh_degree, const RasterDev& rp, const Layout& L, char* ws,
                                   const int32_t* gate, float* grads, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int nt = kBackwardThreads;
    const int64_t nb = (n + nt - 1) / nt;
    const Views* views = reinterpret_cast<const Views*>(ws + L.views);
    const float4* rec = reinterpret_cast<const float4*>(ws + L.records);
    const uint32_t* tl = reinterpret_cast<const uint32_t*>(ws + L.tiles);
    const float4* acc = reinterpret_cast<const float4*>(ws + L.accum);
#define SGS_PB(D, M)                                                                              \
    hipLaunchKernelGGL((project_backward_kernel<D, M>), dim3((unsigned)nb), dim3(nt), 0, s, planes, \
                       n, stride, views, rp, rec, tl, acc, gate, grads)
    SGS_DISPATCH_DEG(SGS_PB, L.n_views > 1)
#undef SGS_PB
    return hipGetLastError();
}

hipError_t launch_project_backward_adam(float* planes, int64_t n, int64_t stride, int sh_degree,
                                        const RasterDev& rp, const Layout& L, char* ws,
                                        const sgs_adam_params* prm, bool sparse, float* m,
                                        float* v, int32_t* step, const int32_t* gate,
                                        hipStream_t s) {
    hipError_t err = launch_adam_count(step, gate, s);
    if (err != hipSuccess || n == 0) return err;
    const AdamDev ad = make_adam(prm);
    const int nt = kBackwardThreads;
    const int64_t nb = std::min<int64_t>((n + nt - 1) / nt, kAdamBlocks);
    const Views* views = reinterpret_cast<const Views*>(ws + L.views);
    const float4* rec = reinterpret_cast<const float4*>(ws + L.records);
    const uint32_t* tl = reinterpret_cast<const uint32_t*>(ws + L.tiles);
    const float4* acc = reinterpret_cast<const float4*>(ws + L.accum);
#define SGS_PBA_S(D, M, SP)                                                                     \
    hipLaunchKernelGGL((project_backward_adam_kernel<D, M, SP>), dim3((unsigned)nb), dim3(nt), 0, \
                       s, planes, n, stride, views, rp, rec, tl, acc, ad, m, v, step, gate)
#define SGS_PBA(D, M) \
    if (sparse) SGS_PBA_S(D, M, true); else SGS_PBA_S(D, M, false)
    SGS_DISPATCH_DEG(SGS_PBA, L.n_views > 1)
#undef SGS_PBA
#undef SGS_PBA_S
    return hipGetLastError();
}

}  // namespace sgs
