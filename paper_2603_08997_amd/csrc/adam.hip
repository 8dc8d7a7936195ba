// Adam on the planar parameter array, applied only when the gate opens the
// backward (Algorithm 1: the optimiser step is coupled to the backward).
// Streaming kernel: float4 loads and stores of p, g, m, v; g is cleared after
// use so the next backward can accumulate into it.
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

struct AdamArgs {
    float b1, b2, c1, c2, eps;  // beta, 1 - beta (formed in binary64), eps
    double beta1, beta2;        // for the bias corrections
    float lr[SGS_MAX_PLANES];
};

__global__ void adam_count_kernel(int32_t* step, const int32_t* gate) {
    if (gate_closed(gate)) return;
    *step += 1;
}

__global__ void __launch_bounds__(256) adam_kernel(AdamArgs a, float4* __restrict__ p,
                                                   float4* __restrict__ g, float4* __restrict__ m,
                                                   float4* __restrict__ v, int64_t stride4,
                                                   const int32_t* __restrict__ step,
                                                   const int32_t* __restrict__ gate) {
    if (gate_closed(gate)) return;
    const int plane = blockIdx.y;
    const int k = *step;
    const float bc1 = (float)(1.0 - pow(a.beta1, (double)k));
    const float bc2 = (float)(1.0 - pow(a.beta2, (double)k));
    const float lr = a.lr[plane];
    const float b1 = a.b1, b2 = a.b2, c1 = a.c1, c2 = a.c2;
    const int64_t base = (int64_t)plane * stride4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < stride4;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = base + i;
        float4 gg = g[j], mm = m[j], vv = v[j], pp = p[j];
        float* gf = &gg.x;
        float* mf = &mm.x;
        float* vf = &vv.x;
        float* pf = &pp.x;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            mf[c] = b1 * mf[c] + c1 * gf[c];
            vf[c] = b2 * vf[c] + c2 * gf[c] * gf[c];
            const float mh = mf[c] / bc1, vh = vf[c] / bc2;
            pf[c] = pf[c] - lr * mh / (sqrtf(vh) + a.eps);
        }
        p[j] = pp;
        m[j] = mm;
        v[j] = vv;
        g[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

}  // namespace

hipError_t launch_adam(const sgs_adam_params* prm, float* params, float* grads, float* m, float* v,
                       int64_t n, int64_t stride, int n_planes, int32_t* step,
                       const int32_t* gate, hipStream_t s) {
    (void)n;
    AdamArgs a;
    a.beta1 = prm->beta1;
    a.beta2 = prm->beta2;
    a.b1 = (float)prm->beta1;
    a.b2 = (float)prm->beta2;
    a.c1 = (float)(1.0 - prm->beta1);
    a.c2 = (float)(1.0 - prm->beta2);
    a.eps = (float)prm->eps;
    for (int i = 0; i < SGS_MAX_PLANES; ++i) a.lr[i] = prm->lr[i];
    hipLaunchKernelGGL(adam_count_kernel, dim3(1), dim3(1), 0, s, step, gate);
    const int64_t stride4 = stride / 4;
    const int64_t want = (stride4 + 255) / 256;
    const unsigned bx = (unsigned)(want < 2048 ? want : 2048);
    hipLaunchKernelGGL(adam_kernel, dim3(bx, (unsigned)n_planes), dim3(256), 0, s, a,
                       reinterpret_cast<float4*>(params), reinterpret_cast<float4*>(grads),
                       reinterpret_cast<float4*>(m), reinterpret_cast<float4*>(v), stride4, step,
                       gate);
    return hipGetLastError();
}

}  // namespace sgs
