// Adam on the planar parameter array, applied only when the gate opens the
// backward (Algorithm 1: the optimiser step is coupled to the backward).
// Streaming kernel: float4 loads and stores of p, g, m, v; g is cleared after
// use so the next backward can accumulate into it. The element update is the
// one the fused backward step uses.
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

__global__ void adam_count_kernel(int32_t* step, const int32_t* gate) {
    if (gate_closed(gate)) return;
    *step += 1;
}

__global__ void __launch_bounds__(256) adam_kernel(AdamDev a, float4* __restrict__ p,
                                                   float4* __restrict__ g, float4* __restrict__ m,
                                                   float4* __restrict__ v, int64_t stride4,
                                                   const int32_t* __restrict__ step,
                                                   const int32_t* __restrict__ gate) {
    if (gate_closed(gate)) return;
    const int plane = blockIdx.y;
    __shared__ AdamStep s_as;
    if (threadIdx.x == 0) s_as = adam_bias_correction(a, *step);
    __syncthreads();
    const AdamStep as = s_as;
    const float lr = a.lr[plane];
    const int64_t base = (int64_t)plane * stride4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < stride4;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = base + i;
        float4 gg = g[j], mm = m[j], vv = v[j], pp = p[j];
        adam_update(gg.x, pp.x, mm.x, vv.x, lr, a, as);
        adam_update(gg.y, pp.y, mm.y, vv.y, lr, a, as);
        adam_update(gg.z, pp.z, mm.z, vv.z, lr, a, as);
        adam_update(gg.w, pp.w, mm.w, vv.w, lr, a, as);
        p[j] = pp;
        m[j] = mm;
        v[j] = vv;
        g[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

}  // namespace

AdamDev make_adam(const sgs_adam_params* prm) {
    AdamDev a;
    a.beta1 = prm->beta1;
    a.beta2 = prm->beta2;
    a.b1 = (float)prm->beta1;
    a.b2 = (float)prm->beta2;
    a.c1 = (float)(1.0 - prm->beta1);
    a.c2 = (float)(1.0 - prm->beta2);
    a.eps = (float)prm->eps;
    for (int i = 0; i < SGS_MAX_PLANES; ++i) a.lr[i] = prm->lr[i];
    return a;
}

hipError_t launch_adam_count(int32_t* step, const int32_t* gate, hipStream_t s) {
    hipLaunchKernelGGL(adam_count_kernel, dim3(1), dim3(1), 0, s, step, gate);
    return hipGetLastError();
}

hipError_t launch_adam(const sgs_adam_params* prm, float* params, float* grads, float* m, float* v,
                       int64_t n, int64_t stride, int n_planes, int32_t* step,
                       const int32_t* gate, hipStream_t s) {
    (void)n;
    const AdamDev a = make_adam(prm);
    hipError_t err = launch_adam_count(step, gate, s);
    if (err != hipSuccess) return err;
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
