/*
 * skipgs.h - C ABI of the MI355X (gfx950) hot path of SkipGS-style 3DGS training.
 *
 * The library renders views of N 3D Gaussians with a tile-based rasteriser
 * (paper Sec. 3, Eqs. 1-5), computes the photometric loss (Eq. 6), decides per
 * post-densification iteration whether to run the backward pass (Sec. 4,
 * Algorithm 1, Eqs. 7-13), and applies the Adam update when it does.
 *
 * Conventions shared by every entry point
 *  - Memory: every pointer argument is DEVICE memory unless its comment says
 *    host. The caller owns all memory, including workspaces; the library
 *    allocates nothing and keeps no state between calls.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream). Every call only enqueues work on it and returns without waiting,
 *    except the ones documented as synchronising.
 *  - Errors: every call returns an sgs_status. Arguments are validated on the
 *    host before anything is enqueued; on an error nothing is enqueued and
 *    sgs_last_error() describes it (thread-local string). Conditions only the
 *    device can see (pair capacity exceeded, non-finite loss) set bits in a
 *    device status word read back by sgs_read_status().
 *  - Predicates: `d_gate` arguments are nullable device int32 flags. When
 *    non-null and *d_gate == 0 at execution time, every kernel of the call
 *    returns without touching memory. This is how a skipped backward costs no
 *    host synchronisation.
 *
 * Gaussian parameter layout (float32, planar, [F][stride], F = 11 + 3 (D+1)^2):
 *   planes 0-2 mean xyz | 3-5 log-scale xyz | 6-9 quaternion wxyz (any norm)
 *   | 10 opacity logit | 11 + 3k + c: SH coefficient k, colour channel c.
 *   Gradients and Adam moments use the identical layout and stride.
 *   stride >= n, a multiple of 64 and < 2^29; data 256-byte aligned.
 *
 * Images: planar float32 [3][H][W] per view; a multi-view call concatenates
 * the views in order (view v starts at 3 * sum_{u<v} H_u W_u floats).
 */
#ifndef SKIPGS_H
#define SKIPGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGS_OK = 0,
    SGS_ERR_INVALID_ARG = 1,  /* null pointer, bad size, alignment or value */
    SGS_ERR_UNSUPPORTED = 2,  /* valid but not implemented (e.g. tile shape) */
    SGS_ERR_CAPACITY = 3,     /* workspace or pair capacity too small        */
    SGS_ERR_HIP = 4,          /* a HIP runtime call failed                  */
    SGS_ERR_NONFINITE = 5     /* reserved for host-side non-finite values   */
} sgs_status;

/* Device status word bits (sgs_read_status). */
#define SGS_STATUS_PAIR_OVERFLOW 0x1u  /* more tile/Gaussian pairs than pair_capacity */
#define SGS_STATUS_NONFINITE_LOSS 0x2u /* the gate saw a non-finite loss              */

#define SGS_MAX_VIEWS 16
#define SGS_MAX_PLANES 59

/* Human-readable description of the last non-OK status on this thread. */
const char* sgs_last_error(void);
/* Library version, e.g. 100 for 0.1.0. */
int32_t sgs_version(void);

/* ---------------------------------------------------------------------------
 * Inputs
 * ------------------------------------------------------------------------- */
typedef struct {
    float* data;        /* device, [F][stride] float32, planes as above        */
    int64_t n;          /* number of Gaussians, >= 0                           */
    int64_t stride;     /* plane stride in elements, >= n, multiple of 64, < 2^29 */
    int32_t sh_degree;  /* D in {0, 1, 2, 3}                                    */
} sgs_gaussians;

/* Pinhole camera, OpenCV axes (x right, y down, z forward); host struct.
 * x_cam = R x_world + t; pixel (u, v) = (fx x/z + cx, fy y/z + cy); the centre
 * of pixel (i, j) is (i + 0.5, j + 0.5). W of Eq. 3 is R. */
typedef struct {
    float R[9];          /* row-major world-to-camera rotation */
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
} sgs_camera;

/* Rasteriser readings of points the paper leaves open (Sec. 3 gives only the
 * equations). Defaults: 16x16 tiles, black background, near 0.2, dilation 0.3,
 * alpha_min 1/255, alpha_max 0.99, t_min 1e-4, jac_clamp 1.3. */
typedef struct {
    int32_t tile_w, tile_h;  /* 8x8, 16x16 or 32x8                                  */
    float bg[3];             /* background colour, added with weight T_final        */
    float near_z;            /* camera depth <= near_z culls                        */
    float dilation;          /* Sigma2D += dilation * I (pixels^2)                  */
    float alpha_min;         /* alpha' below this skips the Gaussian for the pixel; */
                             /* 0 <= alpha_min <= alpha_max                         */
    float alpha_max;         /* alpha' = min(alpha_max, o exp(P))                   */
    float t_min;             /* stop before transmittance would fall below t_min   */
    float jac_clamp;         /* EWA Jacobian evaluated with tx/tz, ty/tz clamped to */
                             /* +-jac_clamp * half-extent / focal; 0 disables       */
} sgs_raster_params;

/* Fills *rp with the defaults above. */
void sgs_default_raster_params(sgs_raster_params* rp);

/* ---------------------------------------------------------------------------
 * Forward rendering (Sec. 3, Eqs. 1-5)
 *
 * One call renders n_views (1..SGS_MAX_VIEWS) views of the same Gaussians in
 * one batch of launches: projection of every (view, Gaussian) entry, a
 * depth-ordered tile binning of all views together, and compositing of every
 * tile of every view. Each pixel composites, front to back in (depth,
 * Gaussian index) order, the Gaussians whose overlap box contains the pixel
 * centre (C(p) = sum c_i alpha'_i T_i + bg T_final).
 *
 * The workspace holds everything the backward needs (projected records, the
 * per-tile sorted lists, per-pixel final transmittance and last contributor).
 * It is valid for sgs_render_backward until it is reused; the backward must
 * see the same Gaussians, cameras and parameters. The status word (sticky,
 * see sgs_read_status) of a newly allocated workspace is undefined: clear it
 * once with sgs_clear_status before the first forward.
 *
 * pair_capacity bounds the number of (tile, Gaussian) pairs of the whole
 * batch. If exceeded, the device sets SGS_STATUS_PAIR_OVERFLOW, records the
 * required count (sgs_read_status) and the image is incomplete.
 * ------------------------------------------------------------------------- */
sgs_status sgs_forward_workspace_size(const sgs_raster_params* rp, int64_t n,
                                      const sgs_camera* cams /* host */, int32_t n_views,
                                      int64_t pair_capacity, size_t* bytes_out /* host */);

sgs_status sgs_render_forward(const sgs_gaussians* g /* host struct */,
                              const sgs_camera* cams /* host */, int32_t n_views,
                              const sgs_raster_params* rp /* host */,
                              void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                              float* out_rgb /* planar images of all views */,
                              void* stream);

/* Synchronises `stream`, then reads the workspace's device status word, the
 * number of visible (view, Gaussian) entries and of (tile, Gaussian) pairs of
 * the last forward. Any output pointer may be NULL. */
sgs_status sgs_read_status(const void* workspace, uint32_t* flags_out, int64_t* visible_out,
                           int64_t* pairs_out, void* stream);

/* Clears the device status word. */
sgs_status sgs_clear_status(void* workspace, void* stream);

/* ---------------------------------------------------------------------------
 * Backward of the forward (exact derivative of the forward with every
 * discrete decision fixed: culling, overlap, skip and stop rules, clamps).
 *
 * dl_drgb has the layout of out_rgb. Gradients w.r.t. the raw parameters
 * (means, log-scales, unnormalised quaternion, opacity logit, SH) are ADDED
 * to `grads` ([F][stride], same layout as the parameters), summed over the
 * views of the batch. Per-pixel blend lists are recomputed from the tile
 * lists in reverse order, not stored.
 * ------------------------------------------------------------------------- */
sgs_status sgs_render_backward(const sgs_gaussians* g, const sgs_camera* cams, int32_t n_views,
                               const sgs_raster_params* rp,
                               void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                               const float* dl_drgb, const int32_t* d_gate /* nullable */,
                               float* grads, void* stream);

/* ---------------------------------------------------------------------------
 * Stage entry points (the forward and backward are these in order). They
 * share the workspace of sgs_render_forward and exist so each stage can be
 * checked and timed on its own.
 * ------------------------------------------------------------------------- */
/* Projection (Eqs. 2-3, SH colour, culling, tile rectangles) of every entry. */
sgs_status sgs_project(const sgs_gaussians* g, const sgs_camera* cams, int32_t n_views,
                       const sgs_raster_params* rp, void* workspace, size_t workspace_bytes,
                       int64_t pair_capacity, void* stream);

/* Writes projected records directly (bypassing sgs_project) for n_views x n
 * entries: entry e = v n + i. Device arrays of n_views * n elements: u, v
 * (pixel coords), depth (> 0), extent (int32, 2 per entry: half-sizes r_x,
 * r_y of the overlap box; negative = not visible), conic (3 per entry: a, b, c
 * of the inverse screen covariance), opacity, rgb (3 per entry, used as the
 * colour with no clamp). */
sgs_status sgs_load_records(const sgs_camera* cams, int32_t n_views, int64_t n,
                            const sgs_raster_params* rp, void* workspace, size_t workspace_bytes,
                            int64_t pair_capacity, const float* u, const float* v,
                            const float* depth, const int32_t* extent, const float* conic,
                            const float* opacity, const float* rgb, void* stream);

/* Tile binning: depth-ordered, per-tile lists of the visible entries whose
 * overlap box reaches the tile and that can reach alpha_min at one of its pixel
 * centres, ties in depth broken by ascending entry index. */
sgs_status sgs_bin(const sgs_camera* cams, int32_t n_views, int64_t n, const sgs_raster_params* rp,
                   void* workspace, size_t workspace_bytes, int64_t pair_capacity, void* stream);

/* Compositing forward of every tile (Eqs. 4-5). */
sgs_status sgs_rasterize(const sgs_camera* cams, int32_t n_views, int64_t n,
                         const sgs_raster_params* rp, void* workspace, size_t workspace_bytes,
                         int64_t pair_capacity, float* out_rgb, void* stream);

/* Compositing backward: per-entry gradients w.r.t. the projected record
 * (u, v, conic a, b, c, opacity, r, g, b) into the workspace's accumulators,
 * which it clears first. */
sgs_status sgs_rasterize_backward(const sgs_camera* cams, int32_t n_views, int64_t n,
                                  const sgs_raster_params* rp, void* workspace,
                                  size_t workspace_bytes, int64_t pair_capacity,
                                  const float* dl_drgb, const int32_t* d_gate, void* stream);

/* Projection backward: chain rule from the accumulators to the raw
 * parameters, summed over views and ADDED to grads. */
sgs_status sgs_project_backward(const sgs_gaussians* g, const sgs_camera* cams, int32_t n_views,
                                const sgs_raster_params* rp, void* workspace,
                                size_t workspace_bytes, int64_t pair_capacity,
                                const int32_t* d_gate, float* grads, void* stream);

/* Byte offsets of the workspace regions, for inspection (host struct).
 * records:    float32 [entries][12]  u v a b | c o rx ry | r g b clamp-mask(bits)
 * tiles:      uint32  [entries]      tiles touched (0 = not visible)
 * depth:      float32 [entries]      camera depth (the sort key) of visible entries
 * pair_tile:  uint16 or uint32 (pair_tile_bytes: 2 when total_tiles < 65535)
 *             [pair_capacity] sorted global tile index per pair
 * pair_entry: uint32  [pair_capacity] entry index per pair (sorted with tiles)
 * ranges:     uint32  [total_tiles][2] [start, end) into the pair arrays
 * t_final:    float32 [total_pixels]  final transmittance per pixel
 * n_last:     uint32  [total_pixels]  1 + list position of the last blended pair (0: none)
 * accum:      float32 [entries][12]   du dv da db | dc do dr dg | db 0 0 0
 * counters:   uint32  [16]            status, visible, pairs needed, pairs written,
 *                                     blended (u64), examined (u64), pairs kept, ... */
typedef struct {
    size_t records, tiles, depth, pair_tile, pair_entry, ranges, t_final, n_last, accum, counters;
    int64_t entries, total_tiles, total_pixels;
    int32_t pair_tile_bytes;  /* 2 or 4 */
} sgs_workspace_layout;

sgs_status sgs_get_workspace_layout(const sgs_raster_params* rp, int64_t n, const sgs_camera* cams,
                                    int32_t n_views, int64_t pair_capacity,
                                    sgs_workspace_layout* out);

/* ---------------------------------------------------------------------------
 * Photometric loss (Eq. 6): L = (1 - lambda) L1 + lambda (1 - SSIM), mean over
 * the 3 H W values; SSIM with an 11x11 Gaussian window (sigma 1.5), C1 = 1e-4,
 * C2 = 9e-4, zero-padded same-size filtering. The reduction order is fixed, so
 * the loss is bit-reproducible.
 * ------------------------------------------------------------------------- */
sgs_status sgs_loss_workspace_size(int32_t width, int32_t height, size_t* bytes_out);

/* Writes the loss to *d_loss (device float). Runs unconditionally: the gate
 * needs the forward loss on every iteration. */
sgs_status sgs_photometric_loss(const float* rgb, const float* target, int32_t width,
                                int32_t height, float lambda, void* workspace,
                                size_t workspace_bytes, float* d_loss, void* stream);

/* dL/d rgb (planar [3][H][W]) of the loss above; predicated on d_gate. It
 * reads per-pixel SSIM derivative maps that sgs_photometric_loss leaves in the
 * workspace: call it after sgs_photometric_loss with the same rgb, target,
 * size and workspace (the training step always does). */
sgs_status sgs_photometric_loss_backward(const float* rgb, const float* target, int32_t width,
                                         int32_t height, float lambda, void* workspace,
                                         size_t workspace_bytes, const int32_t* d_gate,
                                         float* dl_drgb, void* stream);

/* ---------------------------------------------------------------------------
 * SkipGS backward gate (Algorithm 1, Eqs. 7-13), one update per iteration,
 * executed on the device by a single thread in binary64.
 *   s = L / (EMA_v + eps) if view v has an EMA, else +inf          (Eq. 8)
 *   proposal g = 1[s > 1 + delta]                                   (Eq. 9)
 *   rho = b / max(t - 1, 1) (or over the current tumbling window)  (Eq. 10)
 *   t <= warmup: record the proposal when v had an EMA, force g = 1
 *   t  > warmup: calibrate rho_min once (Eqs. 12-13); force g = 1 if
 *                rho < rho_min and budget != 0                      (Eq. 11)
 *   g = 1: b += 1; always: EMA_v <- beta EMA_v + (1 - beta) L      (Eq. 7)
 * The first observation of a view sets its EMA to L. A non-finite loss leaves
 * the EMA alone, gives g = 0 and sets SGS_STATUS_NONFINITE_LOSS in the state.
 * ------------------------------------------------------------------------- */
typedef struct {
    double beta;       /* EMA decay (paper: 0.95)                               */
    double eps;        /* stability constant (1e-8)                             */
    double delta;      /* threshold offset: backward iff s > 1 + delta (0)      */
    double rho_lo;     /* budget floor (0.5)                                    */
    int32_t warmup;    /* W (500)                                               */
    int32_t window;    /* 0: cumulative ratio; > 0: tumbling window length      */
    int32_t calibrate; /* 1: rho_min from warmup statistics (Eqs. 12-13)        */
    int32_t budget;    /* 0: no override (the "w/o budget" ablation)           */
    int32_t n_views;   /* number of training views                              */
} sgs_gate_params;

/* Host view of the gate's device state header. */
typedef struct {
    int64_t t, b, t_w, b_w, warm_hits, warm_count;
    double rho_min, last_s, last_rho;
    int32_t calibrated, flags, last_g, last_proposed, last_forced, last_view;
} sgs_gate_snapshot;

sgs_status sgs_gate_state_size(const sgs_gate_params* p, size_t* bytes_out);
/* Resets the state (no EMA, t = b = 0, rho_min = rho_lo). */
sgs_status sgs_gate_init(const sgs_gate_params* p, void* d_state, void* stream);
/* One iteration: reads *d_loss (device float), writes *d_gate (device int32). */
sgs_status sgs_gate_update(const sgs_gate_params* p, void* d_state, int32_t view,
                           const float* d_loss, int32_t* d_gate, void* stream);
/* Synchronises `stream`; copies the header and, if non-null, the per-view
 * EMA (host double[n_views]) and has-EMA flags (host uint8[n_views]). */
sgs_status sgs_gate_read(const sgs_gate_params* p, const void* d_state,
                         sgs_gate_snapshot* out, double* ema_out, uint8_t* has_ema_out,
                         void* stream);

/* ---------------------------------------------------------------------------
 * Adam (the update applied when the backward runs), per element of the
 * [n_planes][stride] parameter array, one learning rate per plane:
 *   k <- k + 1; m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 *   p <- p - lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps); g <- 0.
 * Predicated on d_gate; *d_step (device int32) is the executed-step count k.
 * ------------------------------------------------------------------------- */
typedef struct {
    double beta1, beta2, eps;  /* 1 - beta is formed in binary64 before rounding */
    float lr[SGS_MAX_PLANES];  /* per plane; planes beyond n_planes ignored     */
} sgs_adam_params;

sgs_status sgs_adam_step(const sgs_adam_params* p, float* params, float* grads, float* m,
                         float* v, int64_t n, int64_t stride, int32_t n_planes,
                         int32_t* d_step, const int32_t* d_gate, void* stream);

/* ---------------------------------------------------------------------------
 * Fused training step: the projection backward and the Adam update in one
 * pass over all Gaussians (dense Adam: Gaussians visible in no view get a
 * zero gradient and are still updated). Each Gaussian's gradient stays in
 * registers; no gradient array is read or written. Gives the same result as
 * sgs_project_backward into a zeroed gradient array followed by
 * sgs_adam_step. g->data is updated in place; m, v have its layout.
 * ------------------------------------------------------------------------- */
sgs_status sgs_project_backward_adam(const sgs_gaussians* g, const sgs_camera* cams,
                                     int32_t n_views, const sgs_raster_params* rp,
                                     void* workspace, size_t workspace_bytes,
                                     int64_t pair_capacity, const sgs_adam_params* adam,
                                     float* m, float* v, int32_t* d_step,
                                     const int32_t* d_gate, void* stream);

/* sgs_rasterize_backward followed by sgs_project_backward_adam. */
sgs_status sgs_render_backward_adam(const sgs_gaussians* g, const sgs_camera* cams,
                                    int32_t n_views, const sgs_raster_params* rp, void* workspace,
                                    size_t workspace_bytes, int64_t pair_capacity,
                                    const float* dl_drgb, const sgs_adam_params* adam, float* m,
                                    float* v, int32_t* d_step, const int32_t* d_gate,
                                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SKIPGS_H */
