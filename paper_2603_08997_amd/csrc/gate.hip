// SkipGS backward gate (paper Sec. 4, Algorithm 1, Eqs. 7-13) on the device.
// One thread updates the state in binary64, so the decision never leaves the
// GPU: the backward and Adam kernels read the flag it writes. The library is
// built without floating-point contraction, so every operation rounds once,
// in the order written.
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

__global__ void gate_init_kernel(GateArgs p, char* state) {
    sgs_gate_snapshot* h = reinterpret_cast<sgs_gate_snapshot*>(state);
    double* ema = reinterpret_cast<double*>(state + sizeof(sgs_gate_snapshot));
    uint8_t* has = reinterpret_cast<uint8_t*>(ema + p.n_views);
    for (int i = threadIdx.x; i < p.n_views; i += blockDim.x) {
        ema[i] = 0.0;
        has[i] = 0;
    }
    if (threadIdx.x == 0) {
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

__global__ void gate_update_kernel(GateArgs p, char* state, int view, const float* d_loss,
                                   int32_t* d_gate) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sgs_gate_snapshot* h = reinterpret_cast<sgs_gate_snapshot*>(state);
    double* ema = reinterpret_cast<double*>(state + sizeof(sgs_gate_snapshot));
    uint8_t* has = reinterpret_cast<uint8_t*>(ema + p.n_views);

    const double L = (double)*d_loss;
    h->t += 1;
    const int64_t t = h->t;
    if (p.window > 0 && (t - 1) % p.window == 0) {
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
    // deviation score against the EMA before this iteration (Eq. 8) and the
    // skip test (Eq. 9)
    const bool had = has[view] != 0;
    double s;
    int g;
    if (had) {
        s = L / (ema[view] + p.eps);
        g = s > 1.0 + p.delta ? 1 : 0;
    } else {
        s = __builtin_inf();
        g = 1;
    }
    const int proposed = g;
    // backward ratio before this iteration (Eq. 10)
    const double rho = p.window > 0 ? (double)h->b_w / (double)max(h->t_w - 1, (int64_t)1)
                                    : (double)h->b / (double)max(t - 1, (int64_t)1);
    if (t <= p.warmup) {
        if (had) {
            h->warm_count += 1;
            h->warm_hits += g;
        }
        g = 1;
    } else {
        // calibration of the budget, once, after warmup (Eqs. 12-13)
        if (p.calibrate && p.warmup > 0 && !h->calibrated) {
            if (h->warm_count > 0) {
                const double rho_hat = (double)h->warm_hits / (double)h->warm_count;
                h->rho_min = p.rho_lo + (1.0 - p.rho_lo) * rho_hat;
            }
            h->calibrated = 1;
        }
        // budget override (Eq. 11)
        if (p.budget && rho < h->rho_min) g = 1;
    }
    if (g) {
        h->b += 1;
        h->b_w += 1;
    }
    // EMA update, unconditional (Eq. 7)
    if (had) {
        ema[view] = p.beta * ema[view] + (1.0 - p.beta) * L;
    } else {
        ema[view] = L;
        has[view] = 1;
    }
    h->last_g = g;
    h->last_proposed = proposed;
    h->last_forced = (g && !proposed) ? 1 : 0;
    h->last_s = s;
    h->last_rho = rho;
    *d_gate = g;
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

hipError_t launch_gate_update(const sgs_gate_params* p, void* state, int view, const float* loss,
                              int32_t* gate, hipStream_t s) {
    hipLaunchKernelGGL(gate_update_kernel, dim3(1), dim3(64), 0, s, args_of(p),
                       static_cast<char*>(state), view, loss, gate);
    return hipGetLastError();
}

}  // namespace sgs
