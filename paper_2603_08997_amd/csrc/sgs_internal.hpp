// Internal declarations of the gfx950 hot path: device-side view table,
// workspace layout, launch wrappers. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/skipgs.h"

namespace sgs {

constexpr int kWave = 64;
constexpr uint32_t kMaxExtent = 1u << 24;   // |u|, |v|, radius beyond this: degenerate, culled
constexpr int kRecordFloats = 12;           // u v a b | c o rx ry | r g b clamp-mask
constexpr int kAccumFloats = 12;            // du dv da db | dc do dr dg | db - - -
constexpr int kDefaultSuperTile = 8;        // super-tile edge in tiles
constexpr int kDefaultBatch = 64;           // list entries per compositing batch
constexpr int kDefaultSplitPrefix = 8192;   // super-tile list pairs split before compositing

// Per-view constants. A call's views live in device memory (the workspace's
// view table): a one-thread kernel stores them there at the start of every
// call, from its arguments or from a camera table picked by a device-side
// view index, and every other kernel reads them through a pointer.
struct ViewDev {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float C[3];          // camera centre in world coordinates, -R^T t
    float lim_x, lim_y;  // clamp of tx/tz, ty/tz in the EWA Jacobian (inf: off)
    int32_t width, height, tiles_x, tiles_y;
    int32_t tile_offset; // first global tile index of the view
    int32_t sup_x, sup_y;   // super-tiles per row and column
    int32_t sup_offset;     // first global super-tile index of the view
    int64_t px_offset;   // first global pixel index of the view
};

struct Views {
    ViewDev v[SGS_MAX_VIEWS];
    int32_t n;
    int32_t total_tiles;
    int64_t total_pixels;
    int32_t total_supers;
    int32_t pad;
};

struct RasterDev {
    int32_t tile_w, tile_h;
    int32_t super_tile;    // super-tile edge in tiles
    int32_t batch;         // list entries per compositing batch (and per list chunk)
    int32_t key_bits;      // low bits of a pair key: the super-tile index
    int32_t rect_bits;     // bits per coordinate of the tile rectangle above them
    int32_t prefix_segs;   // segments of a long super-tile list split before compositing (0: all)
    float bg[3];
    float near_z, dilation, alpha_min, alpha_max, t_min;
    float log2_alpha_min;  // log2(alpha_min), rounded from binary64 (-inf for 0)
};

// Adam constants: beta and 1 - beta formed in binary64, then rounded.
struct AdamDev {
    float b1, b2, c1, c2, eps;
    double beta1, beta2;  // for the bias corrections
    float lr[SGS_MAX_PLANES];
};
struct AdamStep {
    float ibc1, ibc2;  // 1 / (1 - beta^k), formed in binary64
};
AdamDev make_adam(const sgs_adam_params* p);

// Counters region of the workspace (uint32 words).
enum Counter : int {
    kStatus = 0,        // SGS_STATUS_* bits
    kVisible = 1,       // visible entries of the last forward
    kPairs = 2,         // (super-tile, entry) pairs needed by the last forward (saturating)
    kPairsWritten = 3,  // min(pairs, capacity)
    kBlended = 4,       // uint64 at words 4-5: blended (pixel, Gaussian) pairs of the last rasterize
    kEvaluated = 6,     // uint64 at words 6-7: (pixel, list entry) pairs the forward examined
    kPairsKept = 8,     // super-tile pairs left after the reach test (length of the sorted lists)
    kItems = 9,         // tile-list entries needed (saturating)
    kSegments = 10,     // super-tile list segments of the tile-list split
    kUsed = 11,         // tile-list entries up to each tile's last blended one (summed)
    kItemsRest = 12,    // tile-list entries of the completing split (saturating)
    kRedo = 13,         // 1: a tile reached the end of its list prefix with live pixels
    kNumCounters = 16
};

// Pair key (uint32): the super-tile index in the low key_bits bits (a value
// below 2^key_bits - 1, so that no key has all bits set), and above them the
// entry's tile rectangle inside the super-tile, four coordinates of
// rect_bits bits (first column, last column, first row, last row, relative to
// the super-tile). Only the index is sorted on; the rectangle rides along to
// the split of the super-tile lists into tile lists. The key of an emitted
// pair whose Gaussian cannot reach alpha_min on the super-tile has all bits
// set; the first pass of the super-tile sort drops such pairs.
constexpr uint32_t kCulledTile = 0xffffffffu;
constexpr int kMaxSuperTile = 8;   // S x S tiles of a super-tile fit a 64-bit tile mask

// Emission units: each visible Gaussian (in depth order) owns kEmitHead
// header units followed by one unit per pair; a workgroup of the emission
// kernel covers a window of kEmitWindow consecutive units, so it meets at
// most kEmitWindow / (kEmitHead + 1) + 2 Gaussians.
constexpr int64_t kEmitWindow = 1024;
constexpr int64_t kEmitHead = 2;
// Windows of an emission over `entries` entries and `capacity` pairs.
constexpr int64_t emit_windows(int64_t entries, int64_t capacity) {
    return (capacity + kEmitHead * entries + kEmitWindow - 1) / kEmitWindow;
}

// The split of the super-tile lists into tile lists works on segments of
// kSegPairs consecutive pairs of one super-tile's list (a super-tile of L
// pairs has ceil(L / kSegPairs) segments). Segment slots: an upper bound on
// the number of segments of any batch with `capacity` pairs.
constexpr int64_t kSegPairs = 512;
constexpr int64_t segment_slots(int64_t capacity, int64_t supers) {
    return (capacity + kSegPairs - 1) / kSegPairs + supers;
}

// With a split prefix, a super-tile list longer than kCutFactor prefixes is
// split only in its first prefix_segs segments before compositing (the tiles
// that composite a whole short list, often into the background, never wait
// for a second split; long lists are where the split's work is).
constexpr uint32_t kCutFactor = 4;
__host__ __device__ constexpr uint32_t split_segments(uint32_t segs, uint32_t prefix_segs) {
    return prefix_segs > 0 && segs > kCutFactor * prefix_segs ? prefix_segs : segs;
}
// Per tile (tile_state):
enum TileState : uint32_t {
    kTileWhole = 0,       // the tile's list is whole
    kTileTruncated = 1,   // its super-tile's list is longer than the prefix
    kTileIncomplete = 2,  // truncated, and a pixel was still live at the end of the list
};

struct Layout {
    int64_t entries, total_tiles, total_pixels, total_supers, capacity, seg_slots;
    int n_views;
    int64_t scan_blocks, sort_blocks;
    int key_bits, rect_bits, key_passes, key_result;  // result buffer (0/1) of the super-tile sort
    int batch;
    size_t views, records, tiles, depth, dkey[2], dval[2], offsets, window_first, scan_sums,
        pair_key[2], pair_entry[2], sort_hist, sort_totals, sup_ranges, seg_first, seg_cnt,
        seg_off, pair_mask, tile_entry, tile_ranges, tile_state, tile_resume, sup_redo, tile_cost,
        tile_stats, tile_order, t_final, n_last, accum, counters, total;
};

bool make_views(const sgs_camera* cams, int n_views, const sgs_raster_params* rp, Views* out,
                const char** err);
void make_layout(const Views& views, const RasterDev& rp, int64_t n, int64_t capacity, Layout* L);
RasterDev make_raster(const sgs_raster_params* rp);

// The call's views into the workspace's view table: from the host (by value)
// or, when `table` is non-null, view `*d_view` of a device camera table
// (clamped into [0, n_table)) as the batch's single view.
hipError_t launch_store_views(const Views& views, const ViewDev* table, int n_table,
                              const int32_t* d_view, Views* dst, hipStream_t s);

// ---- launch wrappers (all asynchronous on `s`). Kernels read the views from
// the workspace's view table (ws + L.views); L carries the sizes. ----
hipError_t launch_project(const float* planes, int64_t n, int64_t stride, int sh_degree,
                          const RasterDev& rp, const Layout& L, char* ws, hipStream_t s);
hipError_t launch_load_records(const float* u, const float* v, const float* depth,
                               const int32_t* extent, const float* conic, const float* opacity,
                               const float* rgb, int64_t n, const RasterDev& rp, const Layout& L,
                               char* ws, hipStream_t s);
hipError_t launch_bin(const RasterDev& rp, int64_t n, const Layout& L, char* ws, hipStream_t s);
// After a compositing forward over list prefixes: the whole lists of the
// super-tiles that have a tile marked incomplete (tile_state 2), appended
// after the prefix lists, and the new ranges of the incomplete tiles. Every
// kernel returns at once unless counters[kRedo] is set.
hipError_t launch_split_rest(const RasterDev& rp, const Layout& L, char* ws, hipStream_t s);
hipError_t launch_rasterize(const RasterDev& rp, const Layout& L, char* ws, float* out_rgb,
                            hipStream_t s);
hipError_t launch_rasterize_backward(const RasterDev& rp, const Layout& L, char* ws,
                                     const float* dl_drgb, const int32_t* gate, hipStream_t s);
hipError_t launch_project_backward(const float* planes, int64_t n, int64_t stride,
                                   int sh_degree, const RasterDev& rp, const Layout& L, char* ws,
                                   const int32_t* gate, float* grads, hipStream_t s);

// p[0..n) = v on stream s (a kernel, so that callers can be captured).
hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
// order = the tiles sorted by cost >> shift, largest first (ties in any
// order); a permutation of [0, tiles). Skipped when the gate is closed.
hipError_t launch_order_tiles(const uint32_t* cost, int64_t tiles, int shift, uint32_t* order,
                              const int32_t* gate, hipStream_t s);

// Stable LSD radix sort of (key, uint32 value) pairs over key bits [0, bits).
// n is read on the device from *n_dev; n_max bounds it for the grid size.
// Returns the index (0/1) of the buffer holding the result.
int radix_passes(int bits);
// K is uint32_t. kept_dev (nullable, must hold 0): the first
// pass drops keys with all bits set (kCulledTile) and adds the number of
// remaining pairs there; later passes sort that many.
// gather_dst (nullable): the last pass also writes gather_src[value] at each
// sorted position.
// ranges_out (nullable; one-pass sorts only): [start, end) of the run of each
// digit d < n_ranges in the sorted output ([0, 0) when empty).
template <typename K>
hipError_t radix_sort(K* keys[2], uint32_t* vals[2], const uint32_t* n_dev, int64_t n_max,
                      int bits, uint32_t* hist, uint32_t* totals, hipStream_t s, int* result,
                      uint32_t* kept_dev = nullptr, const uint32_t* gather_src = nullptr,
                      uint32_t* gather_dst = nullptr, uint32_t* ranges_out = nullptr,
                      int n_ranges = 0);
int64_t radix_blocks(int64_t n_max);

// Adaptive density control. Thresholds as the kernels compare them (float32
// values formed in binary64 on the host).
struct DensifyDev {
    float grad_threshold;   // the statistic's mean at or above which a Gaussian densifies
    float log_size;         // log(percent_dense * scene_extent): larger max log-scale splits
    float logit_min;        // logit(min_opacity): a smaller opacity logit prunes
    float log_split;        // log(split_scale), subtracted from the children's log-scales
};
int64_t densify_blocks(int64_t n);
// Scratch words of a step over n Gaussians.
constexpr int64_t densify_scratch_words(int64_t blocks) { return 4 * blocks + 3; }
hipError_t launch_densify_stats(const Layout& L, char* ws, int64_t n, const int32_t* gate,
                                float* grad_sum, int32_t* count, hipStream_t s);
hipError_t launch_densify(const DensifyDev& d, float* params, float* m, float* v, int64_t n,
                          int64_t stride, int F, const float* grad_sum, const int32_t* count,
                          const float* normals, float* out_params, float* out_m, float* out_v,
                          int64_t out_stride, uint32_t* scratch, int64_t* n_out, hipStream_t s);

// Loss / gate / Adam
// target: the reference image, or with d_view non-null the image
// *d_view (clamped into [0, n_targets)) of an array of n_targets images.
struct TargetRef {
    const float* base;
    const int32_t* d_view;
    int32_t n_targets;
};
hipError_t launch_loss_forward(const float* rgb, TargetRef target, int w, int h, float lambda,
                               char* ws, float* d_loss, hipStream_t s);
hipError_t launch_loss_backward(const float* rgb, TargetRef target, int w, int h, float lambda,
                                char* ws, const int32_t* gate, float* dl, hipStream_t s);
size_t loss_workspace_bytes(int w, int h);
// The loss forward with the per-tile partial sums (loss_partial_floats(w, h)
// floats) in caller-provided device memory.
int64_t loss_partial_floats(int w, int h);
hipError_t launch_loss_partials(const float* rgb, TargetRef target, int w, int h, float lambda,
                                float* partials, float* d_loss, hipStream_t s);

hipError_t launch_gate_init(const sgs_gate_params* p, void* state, hipStream_t s);
hipError_t launch_gate_update(const sgs_gate_params* p, void* state, const int32_t* view,
                              const float* loss, int32_t* gate, hipStream_t s);
size_t gate_state_bytes(const sgs_gate_params* p);
// *d_view = seq[*d_iter % len]; *d_iter += 1.
hipError_t launch_sequence_next(const int32_t* seq, int64_t len, int64_t* d_iter, int32_t* d_view,
                                hipStream_t s);

hipError_t launch_adam(const sgs_adam_params* p, float* params, float* grads, float* m, float* v,
                       int64_t n, int64_t stride, int n_planes, int32_t* step,
                       const int32_t* gate, hipStream_t s);
hipError_t launch_adam_count(int32_t* step, const int32_t* gate, hipStream_t s);
// sparse: update only the Gaussians visible in a view of the batch (the
// others keep their parameters and moments); dense otherwise.
hipError_t launch_project_backward_adam(float* planes, int64_t n, int64_t stride, int sh_degree,
                                        const RasterDev& rp, const Layout& L, char* ws,
                                        const sgs_adam_params* prm, bool sparse, float* m,
                                        float* v, int32_t* step, const int32_t* gate,
                                        hipStream_t s);

}  // namespace sgs
