// SkipGS backward gate (paper Sec. 4, Algorithm 1, Eqs. 7-13) on the device.
// One thread updates the state in binary64, so the decision never leaves the
// GPU: the backward and Adam kernels read the flag it writes, and the view
// index itself is read from device memory, so a captured iteration can be
// replayed over a device-side view sequence. The library is built without
// floating-point contraction, so every operation rounds once, in the order
// written.
//
// The kernel separates what the gate observes (the score of Eq. 8 and the
// ratio of Eq. 10, both against the state before this iteration), what it
// decides (a pure function of the proposal of Eq. 9, the phase and the budget
// test of Eq. 11) and how its state moves (warmup statistic and calibration,
// Eqs. 12-13; the backward count; the EMA of Eq. 7, on every iteration).
#include "sgs_internal.hpp"
#include "sgs_device.hpp"

namespace sgs {

namespace {

// Device state: this header, then double ema[n_views], then uint8 has_ema[n_views].
static_assert(sizeof(sgs_gate_snapshot) % 8 == 0, "header must keep the EMA array aligned");

struct GateArgs {
    double beta, eps, delta, rho_lo;
    int32_t warmup, window, calibrate, budget, n_views;
};

struct GateView {
    sgs_gate_snapshot* h;
    double* ema;
    uint8_t* has;
    __device__ GateView(char* state, int n_views)
        : h(reinterpret_cast<sgs_gate_snapshot*>(state)),
          ema(reinterpret_cast<double*>(state + sizeof(sgs_gate_snapshot))),
          has(reinterpret_cast<uint8_t*>(state + sizeof(sgs_gate_snapshot) +
                                         sizeof(double) * (size_t)n_views)) {}
};

// g of one iteration (Eqs. 9 and 11): warmup iterations always run the
// backward; afterwards the proposal stands unless the budget floor is
// enforced and the backward ratio is below it.
__device__ __forceinline__ int gate_decision(int proposal, bool in_warmup, bool budget, double rho,
                                             double rho_min) {
    if (in_warmup) return 1;
    if (budget && rho < rho_min) return 1;
    return proposal;
}

// Eqs. 12-13: the floor from the warmup statistic, once, after the warmup;
// with no scored warmup iteration the floor stays at rho_lo.
__device__ __forceinline__ void calibrate_floor(const GateArgs& p, sgs_gate_snapshot* h) {
    if (h->calibrated || !p.calibrate || p.warmup <= 0) return;
    if (h->warm_count > 0)
        h->rho_min = p.rho_lo + (1.0 - p.rho_lo) * ((double)h->warm_hits / (double)h->warm_count);
    h->calibrated = 1;
}

__global__ void gate_init_kernel(GateArgs p, char* state) {
    GateView S(state, p.n_views);
    for (int i = threadIdx.x; i < p.n_views; i += blockDim.x) {
        S.ema[i] = 0.0;
        S.has[i] = 0;
    }
    if (threadIdx.x == 0) {
        sgs_gate_snapshot* h = S.h;
        h->t = h->b = h->t_w = h->b_w = h->warm_hits = h->warm_count = 0;
        h->rho_min = p.rho_lo;
        h->last_s = 0.0;
        h->last_rho = 0.0;
        h->calibrated = 0;
        h->flags = 0;
        h->last_g = h->last_proposed = h->last_forced = 0;
        h->last_view = -1;
    }
}

__global__ void gate_update_kernel(GateArgs p, char* state, const int32_t* d_view,
                                   const float* d_loss, int32_t* d_gate) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    GateView S(state, p.n_views);
    sgs_gate_snapshot* h = S.h;
    const int view = *d_view;
    if (view < 0 || view >= p.n_views) {
        // not an iteration: the state keeps its clock, counts and EMAs
        h->flags |= (int32_t)SGS_STATUS_BAD_VIEW;
        h->last_g = h->last_proposed = h->last_forced = 0;
        h->last_view = view;
        *d_gate = 0;
        return;
    }
    const double L = (double)*d_loss;
    // the clock (and the tumbling window) advance on every iteration
    h->t += 1;
    if (p.window > 0 && (h->t - 1) % p.window == 0) {
        h->t_w = 0;
        h->b_w = 0;
    }
    h->t_w += 1;
    h->last_view = view;
    if (!isfinite(L)) {
        h->flags |= (int32_t)SGS_STATUS_NONFINITE_LOSS;
        h->last_g = h->last_proposed = h->last_forced = 0;
        h->last_s = __builtin_nan("");
        h->last_rho = __builtin_nan("");
        *d_gate = 0;
        return;
    }
    // observation: score (Eq. 8; +inf for a view with no EMA yet, which
    // always proposes) and ratio (Eq. 10) against the state before this
    // iteration
    const bool scored = S.has[view] != 0;
    const double s = scored ? L / (S.ema[view] + p.eps) : __builtin_inf();
    const int proposal = s > 1.0 + p.delta ? 1 : 0;
    const double rho = p.window > 0 ? (double)h->b_w / (double)max(h->t_w - 1, (int64_t)1)
                                    : (double)h->b / (double)max(h->t - 1, (int64_t)1);
    const bool in_warmup = h->t <= p.warmup;
    if (in_warmup) {
        if (scored) {
            h->warm_count += 1;
            h->warm_hits += proposal;
        }
    } else {
        calibrate_floor(p, h);
    }
    const int g = gate_decision(proposal, in_warmup, p.budget != 0, rho, h->rho_min);
    h->b += g;
    h->b_w += g;
    S.ema[view] = scored ? p.beta * S.ema[view] + (1.0 - p.beta) * L : L;
    S.has[view] = 1;
    h->last_g = g;
    h->last_proposed = proposal;
    h->last_forced = (g == 1 && proposal == 0) ? 1 : 0;
    h->last_s = s;
    h->last_rho = rho;
    *d_gate = g;
}

__global__ void sequence_next_kernel(const int32_t* seq, int64_t len, int64_t* iter,
                                     int32_t* view) {
    if (threadIdx.x != 0) return;
    const int64_t k = *iter;
    *view = seq[k % len];
    *iter = k + 1;
}

GateArgs args_of(const sgs_gate_params* p) {
    return GateArgs{p->beta, p->eps, p->delta, p->rho_lo, p->warmup, p->window, p->calibrate,
                    p->budget, p->n_views};
}

}  // namespace

size_t gate_state_bytes(const sgs_gate_params* p) {
    return sizeof(sgs_gate_snapshot) + sizeof(double) * (size_t)p->n_views + (size_t)p->n_views;
}

hipError_t launch_gate_init(const sgs_gate_params* p, void* state, hipStream_t s) {
    hipLaunchKernelGGL(gate_init_kernel, dim3(1), dim3(256), 0, s, args_of(p),
                       static_cast<char*>(state));
    return hipGetLastError();
}

hipError_t launch_sequence_next(const int32_t* seq, int64_t len, int64_t* d_iter, int32_t* d_view,
                                hipStream_t s) {
    hipLaunchKernelGGL(sequence_next_kernel, dim3(1), dim3(64), 0, s, seq, len, d_iter, d_view);
    return hipGetLastError();
}

hipError_t launch_gate_update(const sgs_gate_params* p, void* state, const int32_t* view,
                              const float* loss, int32_t* gate, hipStream_t s) {
    hipLaunchKernelGGL(gate_update_kernel, dim3(1), dim3(64), 0, s, args_of(p),
                       static_cast<char*>(state), view, loss, gate);
    return hipGetLastError();
}

}  // namespace sgs
