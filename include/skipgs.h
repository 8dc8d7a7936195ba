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
 *  - Versioned structs: the parameter structs start with `struct_size`, which
 *    the caller sets to sizeof(the struct) as compiled against this header;
 *    a call that sees another value returns SGS_ERR_INVALID_ARG.
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
#define SGS_STATUS_BAD_VIEW 0x4u       /* the gate read a view index out of range     */

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
    uint32_t struct_size; /* sizeof(sgs_gaussians)                             */
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
 * equations), and the launch shape. Defaults: 16x16 tiles, super-tiles of 8x8
 * tiles, batches of 64 list entries, black background, near 0.2, dilation
 * 0.3, alpha_min 1/255, alpha_max 0.99, t_min 1e-4, jac_clamp 1.3. The tile
 * shape, super-tile edge and batch change how the work is laid out, never the
 * image or the gradients. */
typedef struct {
    uint32_t struct_size;    /* sizeof(sgs_raster_params)                           */
    int32_t tile_w, tile_h;  /* 8x8, 16x16 or 32x8                                  */
    int32_t super_tile;      /* binning granularity: squares of super_tile tiles,   */
                             /* 1..8 (0: 8)                                         */
    int32_t lds_batch;       /* list entries per compositing batch staged in LDS:   */
                             /* 32, 64, 128 or 256 (0: 64)                          */
    int32_t split_prefix;    /* pairs of a long super-tile list split into tile     */
                             /* lists before compositing (rounded up to 512-pair    */
                             /* segments), 0 <= split_prefix <= 2^30, 0: all; see   */
                             /* sgs_render_forward (default 8192)                   */
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

/* Fills *rp with the defaults above (struct_size included). */
void sgs_default_raster_params(sgs_raster_params* rp);

/* ---------------------------------------------------------------------------
 * Forward rendering (Sec. 3, Eqs. 1-5)
 *
 * One call renders n_views (1..SGS_MAX_VIEWS) views of the same Gaussians in
 * one batch of launches: projection of every (view, Gaussian) entry, a
 * depth-ordered binning of all views together, and compositing of every tile
 * of every view. Each pixel composites, front to back in (float32 depth,
 * Gaussian index) order, the Gaussians whose overlap box contains the pixel
 * centre (C(p) = sum c_i alpha'_i T_i + bg T_final).
 *
 * Binning works on super-tiles (squares of super_tile tiles): their
 * depth-ordered lists are sorted once and then split into the depth-ordered
 * lists of their tiles, keeping on each tile the entries that can reach
 * alpha_min there. The compositing of each tile walks its list in batches of
 * lds_batch entries and stops when every pixel has terminated.
 *
 * A tile rarely composites more than the front of its list, so with
 * split_prefix > 0 binning splits a super-tile list of more than
 * 4 x split_prefix pairs (both counted in whole 512-pair segments) only in its
 * first split_prefix pairs (shorter lists whole): a tile's list is then the prefix of its whole list made of the
 * entries from those pairs. A tile whose pixels are not all terminated when
 * its prefix runs out is marked, the whole lists of the marked tiles'
 * super-tiles are split (after the prefix lists, in the same pair capacity)
 * and the marked tiles resume their compositing over their whole lists, all
 * on the device within the compositing call. The image, the per-pixel state
 * and the gradients equal those of split_prefix = 0; only the tile lists a
 * caller reads after sgs_bin alone differ (prefixes).
 *
 * The workspace holds everything the backward needs (projected records, the
 * tile lists, per-pixel final transmittance and last contributor).
 * It is valid for sgs_render_backward until it is reused; the backward must
 * see the same Gaussians, cameras and parameters. The status word (sticky,
 * see sgs_read_status) of a newly allocated workspace is undefined: clear it
 * once with sgs_clear_status before the first forward.
 *
 * pair_capacity bounds both the (super-tile, Gaussian) pairs of the batch and
 * the entries of its tile lists. If either is exceeded, the device sets
 * SGS_STATUS_PAIR_OVERFLOW and records the required capacity
 * (sgs_read_status); the image and the gradients are then incomplete.
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
 * number of visible (view, Gaussian) entries and the pair capacity the last
 * forward needed (the larger of its super-tile pairs and its recorded list
 * entries). Any output pointer may be NULL. */
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

/* Binning: the depth-ordered list of every tile (ties in depth broken by
 * ascending entry index): the visible entries whose overlap box reaches the
 * tile and that can reach alpha_min at one of its pixel centres. Built from
 * per-super-tile lists (S x S tiles, S = super_tile) that are sorted once and
 * then split into the lists of their tiles. pair_capacity bounds both the
 * super-tile pairs and the tile-list entries (sgs_read_status reports the
 * larger need). With split_prefix > 0 the list of a tile in a long
 * super-tile list holds only the entries from the list's first split_prefix
 * pairs; sgs_rasterize completes the lists its tiles need. Also clears the counters the
 * compositing forward accumulates into: every sgs_rasterize follows an
 * sgs_bin. */
sgs_status sgs_bin(const sgs_camera* cams, int32_t n_views, int64_t n, const sgs_raster_params* rp,
                   void* workspace, size_t workspace_bytes, int64_t pair_capacity, void* stream);

/* Compositing forward of every tile (Eqs. 4-5) over its list; with
 * split_prefix > 0 it also splits the whole lists of the super-tiles of the
 * tiles that reach the end of their prefix with live pixels, and composites
 * those tiles again over their whole lists. */
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
 * tiles:      uint32  [entries]      super-tiles touched (0 = not visible)
 * depth:      float32 [entries]      camera depth (the sort key) of visible entries
 * sup_key:    uint32  [pair_capacity] per pair, sorted by the global super-tile
 *             index in the low key_bits bits; above them the pair's tile
 *             rectangle inside the super-tile (first and last column, first
 *             and last row relative to it, rect_bits bits each)
 * sup_entry:  uint32  [pair_capacity] entry index per pair (sorted with the keys)
 * sup_ranges: uint32  [total_supers][2] [start, end) into the pair arrays
 * tile_entry: uint32  [pair_capacity] entry indices of the tile lists
 * tile_ranges: uint32 [total_tiles][2] [start, end) of each tile's list in tile_entry
 * t_final:    float32 [total_pixels]  final transmittance per pixel
 * n_last:     uint32  [total_pixels]  1 + list position of the last blended entry (0: none)
 * accum:      float32 [entries][12]   du dv da db | dc do dr dg | db 0 0 0
 * counters:   uint32  [16]            status, visible, pairs needed, pairs written,
 *                                     blended (u64), examined (u64), pairs kept,
 *                                     tile-list entries needed, list segments,
 *                                     tile-list entries up to the last blend */
typedef struct {
    size_t records, tiles, depth, sup_key, sup_entry, sup_ranges, tile_entry, tile_ranges,
        t_final, n_last, accum, counters;
    int64_t entries, total_tiles, total_pixels, total_supers;
    int32_t key_bits;    /* bits of the super-tile index in sup_key */
    int32_t rect_bits;   /* bits per tile-rectangle coordinate in sup_key */
    int32_t batch;       /* list entries per compositing batch (lds_batch) */
    int32_t super_tile;  /* super-tile edge in tiles */
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

/* For callers that cannot allocate device memory (code under graph capture,
 * serving loops, harnesses that forbid allocation): sgs_photometric_loss
 * without a workspace: the same loss value, bit for bit (it leaves no SSIM maps
 * for a backward: use it where only the loss is wanted). The per-tile partial
 * sums live in a file-scope device array of the library (one per GPU, 512 KiB,
 * held until the process ends), so images are limited to 65536 tiles of 16x16 pixels
 * (e.g. 4096x4096); larger ones fail with SGS_ERR_CAPACITY before anything is
 * enqueued. Allocates nothing. All calls on one GPU share that array: calls
 * that overlap in time on one GPU (different streams, or threads) race and
 * must be serialised by the caller. */
sgs_status sgs_photometric_loss_static(const float* rgb, const float* target, int32_t width,
                                       int32_t height, float lambda, float* d_loss,
                                       void* stream);

/* ---------------------------------------------------------------------------
 * SkipGS backward gate (Sec. 4: Algorithm 1, Eqs. 7-13), one update per
 * post-densification iteration, executed on the device by a single thread in
 * binary64. It scores the iteration's loss against the view's loss EMA
 * (Eq. 8), proposes the backward pass when the score exceeds 1 + delta
 * (Eq. 9; delta = 0 is the paper's test), and overrides a skip when the
 * fraction of iterations that ran the backward falls below the budget floor
 * (Eqs. 10-11), a floor calibrated once from the warmup (Eqs. 12-13). The
 * EMA moves on every iteration (Eq. 7).
 * Readings where the paper is silent: the first observation of a view sets
 * its EMA to the loss (and runs the backward); only views that already had an
 * EMA count towards the warmup statistic, and with none the floor stays at
 * rho_lo; `window` > 0 takes the ratio over tumbling windows aligned at
 * t = 1, window + 1, ...; `budget` = 0 drops the override (the "w/o budget"
 * ablation of Table 4). A non-finite loss leaves the EMA alone, gives g = 0
 * and sets SGS_STATUS_NONFINITE_LOSS in the state's flags.
 * ------------------------------------------------------------------------- */
typedef struct {
    uint32_t struct_size; /* sizeof(sgs_gate_params)                              */
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
/* One iteration: reads the view index *d_view (device int32) and the loss
 * *d_loss (device float), writes *d_gate (device int32). A view index outside
 * [0, n_views) is not an iteration: the state is left as it was apart from
 * SGS_STATUS_BAD_VIEW in its flags, and *d_gate = 0. Everything stays on the
 * device, so a training iteration can be captured once and replayed over a
 * device-side view sequence. */
sgs_status sgs_gate_update(const sgs_gate_params* p, void* d_state, const int32_t* d_view,
                           const float* d_loss, int32_t* d_gate, void* stream);
/* Synchronises `stream`; copies the header and, if non-null, the per-view
 * EMA (host double[n_views]) and has-EMA flags (host uint8[n_views]). */
sgs_status sgs_gate_read(const sgs_gate_params* p, const void* d_state,
                         sgs_gate_snapshot* out, double* ema_out, uint8_t* has_ema_out,
                         void* stream);

/* ---------------------------------------------------------------------------
 * Adaptive density control of the densification phase (Sec. 3): until T_d,
 * every few iterations, a Gaussian whose screen position receives a large
 * gradient is copied when it is small and replaced by two smaller ones when it
 * is large, and one that is nearly transparent is removed; after T_d the set
 * stays fixed and the gate of Algorithm 1 decides every backward pass.
 *
 * Statistic (sgs_densify_stats, after a render backward): for every
 * Gaussian visible in a view of the batch, || (dL/du W/2, dL/dv H/2) || (the
 * gradient of its screen position in normalised device units, the image
 * spanning [-1, 1] on each axis) is added to grad_sum[i] and the view counted
 * in count[i] (device float / int32 arrays of n, accumulated by the caller's
 * schedule and reset after each step).
 *
 * Step (sgs_densify): Gaussian i produces nothing when its opacity is below
 * min_opacity; otherwise, when grad_sum[i] >= grad_threshold * count[i]
 * (count > 0), it is kept and cloned when its largest scale is at most
 * percent_dense * scene_extent, and replaced by two children when larger:
 * centres mu + R(q) diag(s) z_j with z_j = normals[6 i + 3 j .. + 3]
 * (standard-normal draws supplied by the caller, n x 2 x 3 floats), scales
 * s / split_scale, all other parameters copied; every other Gaussian is kept.
 * The new set is written to out_params / out_m / out_v ([F][out_stride],
 * the parameter layout) as the kept Gaussians in index order, then the
 * clones, then the children (two per split Gaussian); kept Gaussians keep
 * their Adam moments, new ones get zeros. The size of the new set goes to
 * *d_n_out (device int64); when it exceeds out_stride nothing is written and
 * the caller calls again with larger planes. The decisions compare float32
 * log-scales and opacity logits with float32 thresholds formed in binary64
 * (log(percent_dense * scene_extent), logit(min_opacity)) and the gradient
 * sum with threshold * count in binary64. Inputs and outputs must not
 * overlap. workspace: sgs_densify_workspace_size(n) bytes of device memory.
 * ------------------------------------------------------------------------- */
typedef struct {
    uint32_t struct_size;    /* sizeof(sgs_densify_params)                       */
    float grad_threshold;    /* mean view-space gradient that densifies (2e-4)  */
    float percent_dense;     /* clone / split boundary as a fraction of the     */
                             /* scene extent (0.01)                             */
    float scene_extent;      /* world-space extent of the scene (> 0)           */
    float min_opacity;       /* opacity below this prunes (0.005), in [0, 1)    */
    float split_scale;       /* children's scales = parent's / split_scale (1.6)*/
} sgs_densify_params;

void sgs_default_densify_params(sgs_densify_params* p);

/* Adds the statistic of the last render backward in `workspace` (the views
 * and visibility its forward stored, the record gradients its backward
 * left); cams / n_views / rp / pair_capacity describe that workspace.
 * Predicated on d_gate (nullable). */
sgs_status sgs_densify_stats(const sgs_camera* cams, int32_t n_views, int64_t n,
                             const sgs_raster_params* rp, const void* workspace,
                             size_t workspace_bytes, int64_t pair_capacity, const int32_t* d_gate,
                             float* grad_sum, int32_t* count, void* stream);

sgs_status sgs_densify_workspace_size(int64_t n, size_t* bytes_out);

sgs_status sgs_densify(const sgs_densify_params* p, const sgs_gaussians* g, const float* m,
                       const float* v, const float* grad_sum, const int32_t* count,
                       const float* normals, float* out_params, float* out_m, float* out_v,
                       int64_t out_stride, void* workspace, size_t workspace_bytes,
                       int64_t* d_n_out, void* stream);

/* ---------------------------------------------------------------------------
 * Adam (Kingma & Ba, with bias correction): the optimiser the 3DGS parameters
 * are trained with (Sec. 3) and the standard update SkipGS applies whenever
 * the gate runs the backward (Sec. 4, Algorithm 1; Sec. 5.1), per element of
 * the [n_planes][stride] parameter array, one learning rate per plane:
 *   k <- k + 1; m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 *   p <- p - lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps); g <- 0.
 * Predicated on d_gate; *d_step (device int32) is the executed-step count k.
 * ------------------------------------------------------------------------- */
typedef struct {
    uint32_t struct_size;      /* sizeof(sgs_adam_params)                       */
    double beta1, beta2, eps;  /* 1 - beta is formed in binary64 before rounding */
    float lr[SGS_MAX_PLANES];  /* per plane; planes beyond n_planes ignored     */
    int32_t visible_only;      /* fused step only: 1 updates only the Gaussians  */
                               /* visible in a view of the batch (the others    */
                               /* keep parameters and moments; the step count k */
                               /* is the shared executed-step count); 0: dense  */
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

/* ---------------------------------------------------------------------------
 * One post-densification training iteration (Sec. 4, Algorithm 1) with the
 * view chosen on the device, so that an iteration can be captured once (HIP
 * graph) and replayed over a device-side view sequence.
 *
 * A camera table holds n_cams cameras of one resolution, prepared for the
 * device. sgs_camera_table_init validates them on the host and copies the
 * table to device memory; it synchronises `stream` (set-up, not for capture).
 * ------------------------------------------------------------------------- */
sgs_status sgs_camera_table_size(int32_t n_cams, size_t* bytes_out);
sgs_status sgs_camera_table_init(const sgs_camera* cams /* host, n_cams */, int32_t n_cams,
                                 const sgs_raster_params* rp, void* d_table, size_t table_bytes,
                                 void* stream);

/* *d_view = d_sequence[*d_iter % sequence_len]; *d_iter += 1 (device int64).
 * The first launch of a captured iteration, so that each replay takes the
 * next view of the sequence. */
sgs_status sgs_view_sequence_next(const int32_t* d_sequence, int64_t sequence_len,
                                  int64_t* d_iter, int32_t* d_view, void* stream);

/* One iteration for view v = *d_view of the table (all cameras of the table
 * share cams[0]'s size; cams is the host array the table was built from):
 * render view v (sgs_render_forward), the loss against targets[v] (planar
 * [n_cams][3][H][W]) into *d_loss, the gate decision into *d_gate
 * (sgs_gate_update; with gate_state NULL the backward always runs: *d_gate =
 * 1), and, predicated on *d_gate, the loss backward into dl_drgb, the
 * compositing backward and the fused projection backward + Adam step
 * (sgs_render_backward_adam). No host synchronisation; rgb and dl_drgb are
 * [3][H][W] device buffers; the view index is clamped into the table for the
 * render and the loss (the gate flags an out-of-range index). */
sgs_status sgs_train_iteration(const sgs_gaussians* g, const sgs_camera* cams /* host */,
                               const void* d_table, int32_t n_cams, const int32_t* d_view,
                               const sgs_raster_params* rp, void* workspace,
                               size_t workspace_bytes, int64_t pair_capacity,
                               const float* targets, float lambda, void* loss_workspace,
                               size_t loss_workspace_bytes, float* rgb, float* dl_drgb,
                               float* d_loss, const sgs_gate_params* gp, void* gate_state,
                               int32_t* d_gate, const sgs_adam_params* adam, float* m, float* v,
                               int32_t* d_step, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SKIPGS_H */
