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

// Per-view constants, passed by value to every kernel of a multi-view batch.
struct ViewDev {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float C[3];          // camera centre in world coordinates, -R^T t
    float lim_x, lim_y;  // clamp of tx/tz, ty/tz in the EWA Jacobian (inf: off)
    int32_t width, height, tiles_x, tiles_y;
    int32_t tile_offset; // first global tile index of the view
    int32_t pad;
    int64_t px_offset;   // first global pixel index of the view
};

struct Views {
    ViewDev v[SGS_MAX_VIEWS];
    int32_t n;
    int32_t total_tiles;
    int64_t total_pixels;
};

struct RasterDev {
    int32_t tile_w, tile_h;
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
    kPairs = 2,         // (tile, entry) pairs needed by the last forward
    kPairsWritten = 3,  // min(pairs, capacity)
    kBlended = 4,       // uint64 at words 4-5: blended (pixel, Gaussian) pairs of the last rasterize
    kEvaluated = 6,     // uint64 at words 6-7: (pixel, list entry) pairs the forward examined
    kPairsKept = 8,     // pairs left after the exact tile test (length of the sorted lists)
    kNumCounters = 16
};

// Tile key of an emitted pair whose Gaussian cannot reach alpha_min at any
// pixel centre of the tile; the first pass of the tile sort drops such pairs.
// Batches of fewer than 65535 tiles keep tile keys in uint16 (kCulledTile16).
constexpr uint32_t kCulledTile = 0xffffffffu;
constexpr uint16_t kCulledTile16 = 0xffffu;
constexpr int64_t kMaxTiles16 = 0xffff;

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

struct Layout {
    int64_t entries, total_tiles, total_pixels, capacity;
    int64_t scan_blocks, sort_blocks;
    int tile_bits, tile_passes, tile_result;  // result buffer index (0/1) of the tile sort
    int tile_key_bytes;                        // 2 (total_tiles < kMaxTiles16) or 4
    size_t records, tiles, depth, dkey[2], dval[2], offsets, window_first, scan_sums, pair_tile[2],
        pair_entry[2],
        sort_hist, sort_totals, ranges, tile_cost, tile_order, t_final, n_last, accum, counters,
        total;
};

bool make_views(const sgs_camera* cams, int n_views, const sgs_raster_params* rp, Views* out,
                const char** err);
void make_layout(const Views& views, int64_t n, int64_t capacity, Layout* L);
RasterDev make_raster(const sgs_raster_params* rp);

// ---- launch wrappers (all asynchronous on `s`) ----
hipError_t launch_project(const float* planes, int64_t n, int64_t stride, int sh_degree,
                          const Views& views, const RasterDev& rp, float* records,
                          uint32_t* tiles, uint32_t* dkey, hipStream_t s);
hipError_t launch_load_records(int64_t entries, const float* u, const float* v,
                               const float* depth, const int32_t* extent, const float* conic,
                               const float* opacity, const float* rgb, int64_t n,
                               const Views& views, const RasterDev& rp, float* records,
                               uint32_t* tiles, uint32_t* dkey, hipStream_t s);
hipError_t launch_bin(const Views& views, const RasterDev& rp, int64_t n, const Layout& L,
                      char* ws, hipStream_t s);
hipError_t launch_rasterize(const Views& views, const RasterDev& rp, const Layout& L, char* ws,
                            float* out_rgb, hipStream_t s);
hipError_t launch_rasterize_backward(const Views& views, const RasterDev& rp, const Layout& L,
                                     char* ws, const float* dl_drgb, const int32_t* gate,
                                     hipStream_t s);
hipError_t launch_project_backward(const float* planes, int64_t n, int64_t stride,
                                   int sh_degree, const Views& views, const RasterDev& rp,
                                   const Layout& L, char* ws, const int32_t* gate, float* grads,
                                   hipStream_t s);

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
// K is uint32_t or uint16_t. kept_dev (nullable, must hold 0): the first
// pass drops keys with all bits set (kCulledTile, or kCulledTile16 for uint16
// keys) and adds the number of remaining pairs there; later passes sort that
// many.
// gather_dst (nullable): the last pass also writes gather_src[value] at each
// sorted position.
template <typename K>
hipError_t radix_sort(K* keys[2], uint32_t* vals[2], const uint32_t* n_dev, int64_t n_max,
                      int bits, uint32_t* hist, uint32_t* totals, hipStream_t s, int* result,
                      uint32_t* kept_dev = nullptr, const uint32_t* gather_src = nullptr,
                      uint32_t* gather_dst = nullptr);
int64_t radix_blocks(int64_t n_max);

// Loss / gate / Adam
hipError_t launch_loss_forward(const float* rgb, const float* target, int w, int h, float lambda,
                               char* ws, float* d_loss, hipStream_t s);
hipError_t launch_loss_backward(const float* rgb, const float* target, int w, int h, float lambda,
                                char* ws, const int32_t* gate, float* dl, hipStream_t s);
size_t loss_workspace_bytes(int w, int h);

hipError_t launch_gate_init(const sgs_gate_params* p, void* state, hipStream_t s);
hipError_t launch_gate_update(const sgs_gate_params* p, void* state, int view, const float* loss,
                              int32_t* gate, hipStream_t s);
size_t gate_state_bytes(const sgs_gate_params* p);

hipError_t launch_adam(const sgs_adam_params* p, float* params, float* grads, float* m, float* v,
                       int64_t n, int64_t stride, int n_planes, int32_t* step,
                       const int32_t* gate, hipStream_t s);
hipError_t launch_adam_count(int32_t* step, const int32_t* gate, hipStream_t s);
hipError_t launch_project_backward_adam(float* planes, int64_t n, int64_t stride, int sh_degree,
                                        const Views& views, const RasterDev& rp, const Layout& L,
                                        char* ws, const sgs_adam_params* prm, float* m, float* v,
                                        int32_t* step, const int32_t* gate, hipStream_t s);

}  // namespace sgs
