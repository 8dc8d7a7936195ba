// Adaptive density control of the densification phase (Sec. 3): the
// view-space positional gradient statistic gathered after each backward, and
// one clone / split / prune step over all Gaussians.
//
// Statistic: for every Gaussian visible in a view of the last render, the
// norm of dL/d(u, v) in normalised device units (the image spans [-1, 1] on
// each axis), || (dL/du W / 2, dL/dv H / 2) ||, added to a running sum and
// the view counted; dL/du and dL/dv are the first two floats of the entry's
// record-gradient accumulator the compositing backward left.
//
// Step: a Gaussian whose opacity is below min_opacity produces nothing; one
// whose mean statistic reaches grad_threshold is cloned (exact copy added)
// when its largest scale is at most percent_dense * scene_extent and split
// otherwise (replaced by two children centred at mu + R(q) diag(s) z_j, z_j
// drawn by the caller, with scales s / split_scale); every other Gaussian is
// kept. The new set is written as the kept Gaussians in index order, then the
// clones, then the children (two per split Gaussian), into separate output
// planes; kept Gaussians keep their Adam moments, new ones start at zero. The
// decisions compare the float32 log-scale and opacity logit with float32
// thresholds formed in binary64 on the host, and the statistic's sum with
// threshold * count in binary64, so they are exact for the given inputs.
//
// Three launches: per-block counts of the three outcomes (packed in one word
// per thread), a one-workgroup scan of the block counts that also records the
// size of the new set, and the write, which repeats the decisions, scans them
// within the block and streams every plane of every output Gaussian; all
// outputs of one segment from one block are consecutive, so the stores
// coalesce. An output set larger than the output planes' stride is reported
// and nothing is written.
#include <algorithm>

#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

constexpr int kDensifyThreads = 256;
constexpr int kDensifyScanThreads = 1024;
// outcome counts packed in one word: keep in bits 0-9, clone 10-19, split 20-29
constexpr int kClonePos = 10, kSplitPos = 20;
constexpr uint32_t kField = (1u << 10) - 1u;

__global__ void __launch_bounds__(256) densify_stats_kernel(
    const Views* __restrict__ views, int64_t n, const uint32_t* __restrict__ tiles,
    const float* __restrict__ accum, const int32_t* __restrict__ gate, float* __restrict__ grad_sum,
    int32_t* __restrict__ count) {
    if (gate_closed(gate)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    int c = 0;
    for (int v = 0; v < views->n; ++v) {
        const int64_t e = (int64_t)v * n + i;
        if (tiles[e] == 0u) continue;
        const float du = accum[kAccumFloats * e] * (0.5f * (float)views->v[v].width);
        const float dv = accum[kAccumFloats * e + 1] * (0.5f * (float)views->v[v].height);
        s += sqrtf(fmaf(du, du, dv * dv));
        ++c;
    }
    if (c > 0) {
        grad_sum[i] += s;
        count[i] += c;
    }
}

// Output stores through L2 with the default policy: the outputs of a wave
// start at arbitrary positions, so their cache lines are filled by several
// waves and are best merged in L2 before they go to HBM.
__device__ __forceinline__ void put(const PlaneBuf& B, int j, uint32_t lane_off, float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), B.rsrc(j), (int)lane_off, 0, 0);
}

__device__ __forceinline__ uint32_t outcome(const PlaneBuf& P, uint32_t off, float g, int32_t c,
                                            const DensifyDev& d) {
    const float logit = P.load(10, off);
    const float ls = fmaxf(fmaxf(P.load(3, off), P.load(4, off)), P.load(5, off));
    if (logit < d.logit_min) return 0u;
    const bool cand = c > 0 && (double)g >= (double)d.grad_threshold * (double)c;
    if (!cand) return 1u;                       // keep
    return ls > d.log_size ? (1u << kSplitPos)  // split
                           : (1u | (1u << kClonePos));   // keep and clone
}

__global__ void __launch_bounds__(kDensifyThreads) densify_count_kernel(
    PlaneBuf P, int64_t n, const float* __restrict__ grad_sum, const int32_t* __restrict__ count,
    DensifyDev d, uint32_t* __restrict__ block_counts) {
    __shared__ uint32_t smem[kDensifyThreads / 64 + 1];
    const int64_t i = (int64_t)blockIdx.x * kDensifyThreads + threadIdx.x;
    const uint32_t o = i < n ? outcome(P, (uint32_t)i * 4u, grad_sum[i], count[i], d) : 0u;
    uint32_t tot;
    block_excl_scan<kDensifyThreads>(o, smem, &tot);
    if (threadIdx.x == 0) block_counts[blockIdx.x] = tot;
}

// block_off[3 b + k]: outputs of segment k (kept, clones, split Gaussians)
// before block b; meta[0..2]: the totals; *n_out: the size of the new set.
__global__ void __launch_bounds__(kDensifyScanThreads) densify_scan_kernel(
    const uint32_t* __restrict__ block_counts, int64_t nblocks, uint32_t* __restrict__ block_off,
    uint32_t* __restrict__ meta, int64_t* __restrict__ n_out) {
    __shared__ uint32_t smem[kDensifyScanThreads / 64 + 1];
    uint32_t carry[3] = {0u, 0u, 0u};
    for (int64_t b0 = 0; b0 < nblocks; b0 += kDensifyScanThreads) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t w = b < nblocks ? block_counts[b] : 0u;
        const uint32_t v[3] = {w & kField, (w >> kClonePos) & kField, (w >> kSplitPos) & kField};
        uint32_t ex[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint32_t tot;
            ex[k] = carry[k] + block_excl_scan<kDensifyScanThreads>(v[k], smem, &tot);
            carry[k] += tot;
        }
        if (b < nblocks) {
            block_off[3 * b] = ex[0];
            block_off[3 * b + 1] = ex[1];
            block_off[3 * b + 2] = ex[2];
        }
    }
    if (threadIdx.x == 0) {
        meta[0] = carry[0];
        meta[1] = carry[1];
        meta[2] = carry[2];
        *n_out = (int64_t)carry[0] + (int64_t)carry[1] + 2 * (int64_t)carry[2];
    }
}

__global__ void __launch_bounds__(kDensifyThreads) densify_write_kernel(
    PlaneBuf P, PlaneBuf M, PlaneBuf V, int64_t n, int F, const float* __restrict__ grad_sum,
    const int32_t* __restrict__ count, const float* __restrict__ normals, DensifyDev d,
    const uint32_t* __restrict__ block_off, const uint32_t* __restrict__ meta,
    const int64_t* __restrict__ n_out, int64_t out_stride, PlaneBuf PO, PlaneBuf MO, PlaneBuf VO) {
    __shared__ uint32_t smem[kDensifyThreads / 64 + 1];
    if (*n_out > out_stride) return;   // the caller provides larger planes and calls again
    const int64_t i = (int64_t)blockIdx.x * kDensifyThreads + threadIdx.x;
    const uint32_t off = (uint32_t)i * 4u;
    const uint32_t o = i < n ? outcome(P, off, grad_sum[i], count[i], d) : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<kDensifyThreads>(o, smem, &tot);
    if (o == 0u) return;
    const uint32_t K = meta[0], Cn = meta[1];
    const uint32_t* bo = block_off + 3 * (int64_t)blockIdx.x;
    const bool keep = (o & kField) != 0u, clone = ((o >> kClonePos) & kField) != 0u;
    const bool split = ((o >> kSplitPos) & kField) != 0u;
    const uint32_t pk = bo[0] + (ex & kField);
    const uint32_t pc = K + bo[1] + ((ex >> kClonePos) & kField);
    const uint32_t ps = K + Cn + 2u * (bo[2] + ((ex >> kSplitPos) & kField));
    if (keep || clone) {
        // planes in groups of kGroup, every load of a group issued before its
        // stores, so that each lane keeps many loads in flight
        constexpr int kGroup = 8;
        for (int f0 = 0; f0 < F; f0 += kGroup) {
            float x[kGroup], mm[kGroup], vv[kGroup];
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                const int f = min(f0 + k, F - 1);
                x[k] = P.load(f, off);
                mm[k] = keep ? M.load(f, off) : 0.f;
                vv[k] = keep ? V.load(f, off) : 0.f;
            }
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                const int f = f0 + k;
                if (f >= F) break;
                if (keep) {
                    put(PO, f, pk * 4u, x[k]);
                    put(MO, f, pk * 4u, mm[k]);
                    put(VO, f, pk * 4u, vv[k]);
                }
                if (clone) {
                    put(PO, f, pc * 4u, x[k]);
                    put(MO, f, pc * 4u, 0.f);
                    put(VO, f, pc * 4u, 0.f);
                }
            }
        }
    }
    if (split) {
        float mu[3], s[3], q[4];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mu[k] = P.load(k, off);
            s[k] = expf(P.load(3 + k, off));
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = P.load(6 + k, off);
        const float qn = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
        const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                            2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                            2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
        for (int j = 0; j < 2; ++j) {
            const uint32_t po = (ps + (uint32_t)j) * 4u;
            const float* zj = normals + 6 * i + 3 * j;
            const float t[3] = {s[0] * zj[0], s[1] * zj[1], s[2] * zj[2]};
#pragma unroll
            for (int r = 0; r < 3; ++r)
                put(PO, r, po, mu[r] + (R[3 * r] * t[0] + R[3 * r + 1] * t[1] + R[3 * r + 2] * t[2]));
#pragma unroll
            for (int k = 0; k < 3; ++k) put(PO, 3 + k, po, P.load(3 + k, off) - d.log_split);
            for (int f = 6; f < F; ++f) put(PO, f, po, P.load(f, off));
            for (int f = 0; f < F; ++f) {
                put(MO, f, po, 0.f);
                put(VO, f, po, 0.f);
            }
        }
    }
}

}  // namespace

int64_t densify_blocks(int64_t n) { return (n + kDensifyThreads - 1) / kDensifyThreads; }

hipError_t launch_densify_stats(const Layout& L, char* ws, int64_t n, const int32_t* gate,
                                float* grad_sum, int32_t* count, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const Views* views = reinterpret_cast<const Views*>(ws + L.views);
    const uint32_t* tiles = reinterpret_cast<const uint32_t*>(ws + L.tiles);
    const float* acc = reinterpret_cast<const float*>(ws + L.accum);
    hipLaunchKernelGGL(densify_stats_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       views, n, tiles, acc, gate, grad_sum, count);
    return hipGetLastError();
}

hipError_t launch_densify(const DensifyDev& d, float* params, float* m, float* v, int64_t n,
                          int64_t stride, int F, const float* grad_sum, const int32_t* count,
                          const float* normals, float* out_params, float* out_m, float* out_v,
                          int64_t out_stride, uint32_t* scratch, int64_t* n_out, hipStream_t s) {
    const int64_t nb = densify_blocks(n);
    uint32_t* block_counts = scratch;
    uint32_t* block_off = scratch + nb;
    uint32_t* meta = scratch + 4 * nb;
    const PlaneBuf P{params, stride}, M{m, stride}, V{v, stride};
    const PlaneBuf PO{out_params, out_stride}, MO{out_m, out_stride}, VO{out_v, out_stride};
    if (nb > 0)
        hipLaunchKernelGGL(densify_count_kernel, dim3((unsigned)nb), dim3(kDensifyThreads), 0, s, P,
                           n, grad_sum, count, d, block_counts);
    hipLaunchKernelGGL(densify_scan_kernel, dim3(1), dim3(kDensifyScanThreads), 0, s, block_counts,
                       nb, block_off, meta, n_out);
    if (nb > 0)
        hipLaunchKernelGGL(densify_write_kernel, dim3((unsigned)nb), dim3(kDensifyThreads), 0, s, P,
                           M, V, n, F, grad_sum, count, normals, d, block_off, meta, n_out,
                           out_stride, PO, MO, VO);
    return hipGetLastError();
}

}  // namespace sgs
