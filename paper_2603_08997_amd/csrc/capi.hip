// The C ABI declared in include/skipgs.h: host-side validation, workspace
// layout and the order of launches. Nothing here allocates device memory.
#include <cmath>
#include <cstdarg>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sgs_internal.hpp"

namespace {

thread_local std::string g_err;

sgs_status fail(sgs_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
sgs_status fail(sgs_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

sgs_status hip_fail(hipError_t e, const char* what) {
    return fail(SGS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define SGS_HIP(call, what)                              \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

sgs_status check_raster(const sgs_raster_params* rp) {
    if (!rp) return fail(SGS_ERR_INVALID_ARG, "raster params are null");
    if (rp->struct_size != sizeof(sgs_raster_params))
        return fail(SGS_ERR_INVALID_ARG, "raster params struct_size %u, expected %zu",
                    rp->struct_size, sizeof(sgs_raster_params));
    const bool ok = (rp->tile_w == 16 && rp->tile_h == 16) || (rp->tile_w == 8 && rp->tile_h == 8) ||
                    (rp->tile_w == 32 && rp->tile_h == 8);
    if (!ok) return fail(SGS_ERR_UNSUPPORTED, "tile shape %dx%d not in {16x16, 8x8, 32x8}",
                         rp->tile_w, rp->tile_h);
    if (rp->super_tile < 0 || rp->super_tile > sgs::kMaxSuperTile)
        return fail(SGS_ERR_UNSUPPORTED, "super_tile %d not in [1, %d] (0: default)",
                    rp->super_tile, sgs::kMaxSuperTile);
    if (rp->lds_batch != 0 && rp->lds_batch != 32 && rp->lds_batch != 64 &&
        rp->lds_batch != 128 && rp->lds_batch != 256)
        return fail(SGS_ERR_UNSUPPORTED, "lds_batch %d not in {32, 64, 128, 256} (0: default)",
                    rp->lds_batch);
    if (rp->split_prefix < 0 || rp->split_prefix > (1 << 30))
        return fail(SGS_ERR_INVALID_ARG, "split_prefix %d not in [0, 2^30]", rp->split_prefix);
    if (!(rp->alpha_max > 0.f && rp->alpha_max <= 1.f) ||
        !(rp->alpha_min >= 0.f && rp->alpha_min <= rp->alpha_max) ||
        !(rp->t_min >= 0.f && rp->t_min < 1.f) || !(rp->near_z >= 0.f) || !(rp->dilation >= 0.f) ||
        !(rp->jac_clamp >= 0.f) || !std::isfinite(rp->bg[0]) || !std::isfinite(rp->bg[1]) ||
        !std::isfinite(rp->bg[2]))
        return fail(SGS_ERR_INVALID_ARG, "raster params out of range");
    return SGS_OK;
}

struct Prepared {
    sgs::Views views;
    sgs::RasterDev rd;
    sgs::Layout L;
};

sgs_status prepare(const sgs_raster_params* rp, int64_t n, const sgs_camera* cams, int32_t n_views,
                   int64_t capacity, Prepared* P) {
    sgs_status st = check_raster(rp);
    if (st != SGS_OK) return st;
    if (n < 0) return fail(SGS_ERR_INVALID_ARG, "n < 0");
    if (!cams) return fail(SGS_ERR_INVALID_ARG, "cameras are null");
    if (n_views < 1 || n_views > SGS_MAX_VIEWS)
        return fail(SGS_ERR_INVALID_ARG, "n_views %d not in [1, %d]", n_views, SGS_MAX_VIEWS);
    if (capacity < 0 || capacity > (int64_t)0x7fffffff)
        return fail(SGS_ERR_INVALID_ARG, "pair_capacity %lld not in [0, 2^31)", (long long)capacity);
    if (n * (int64_t)n_views > (int64_t)0x7fffffff)
        return fail(SGS_ERR_INVALID_ARG, "n * n_views exceeds 2^31");
    const char* err = nullptr;
    if (!sgs::make_views(cams, n_views, rp, &P->views, &err)) return fail(SGS_ERR_INVALID_ARG, "%s", err);
    P->rd = sgs::make_raster(rp);
    sgs::make_layout(P->views, P->rd, n, capacity, &P->L);
    if (P->L.key_bits + 4 * P->L.rect_bits > 32)
        return fail(SGS_ERR_UNSUPPORTED,
                    "%lld super-tiles of %d tiles do not fit a 32-bit pair key; use smaller "
                    "super-tiles", (long long)P->L.total_supers, P->rd.super_tile);
    P->rd.key_bits = P->L.key_bits;
    P->rd.rect_bits = P->L.rect_bits;
    return SGS_OK;
}

sgs_status check_ws(const Prepared& P, const void* ws, size_t bytes) {
    if (!ws) return fail(SGS_ERR_INVALID_ARG, "workspace is null");
    if (!aligned(ws, 256)) return fail(SGS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    if (bytes < P.L.total)
        return fail(SGS_ERR_CAPACITY, "workspace has %zu bytes, needs %zu", bytes, P.L.total);
    return SGS_OK;
}

sgs_status check_gaussians(const sgs_gaussians* g) {
    if (!g) return fail(SGS_ERR_INVALID_ARG, "gaussians are null");
    if (g->struct_size != sizeof(sgs_gaussians))
        return fail(SGS_ERR_INVALID_ARG, "gaussians struct_size %u, expected %zu", g->struct_size,
                    sizeof(sgs_gaussians));
    if (g->n < 0) return fail(SGS_ERR_INVALID_ARG, "n < 0");
    if (g->sh_degree < 0 || g->sh_degree > 3)
        return fail(SGS_ERR_INVALID_ARG, "sh_degree %d not in [0, 3]", g->sh_degree);
    if (g->stride < g->n || g->stride % 64 != 0 || g->stride <= 0 || g->stride >= (1ll << 29))
        return fail(SGS_ERR_INVALID_ARG,
                    "stride %lld must be >= n, > 0, < 2^29 and a multiple of 64",
                    (long long)g->stride);
    if (!g->data) return fail(SGS_ERR_INVALID_ARG, "parameter data is null");
    if (!aligned(g->data, 16)) return fail(SGS_ERR_INVALID_ARG, "parameter data not 16-byte aligned");
    return SGS_OK;
}

}  // namespace

namespace sgs {

bool make_views(const sgs_camera* cams, int n_views, const sgs_raster_params* rp, Views* out,
                const char** err) {
    std::memset(out, 0, sizeof(*out));
    out->n = n_views;
    int64_t tiles = 0, supers = 0, pixels = 0;
    for (int v = 0; v < n_views; ++v) {
        const sgs_camera& c = cams[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 32768 || c.height > 32768) {
            *err = "camera size not in [1, 32768]";
            return false;
        }
        bool finite = std::isfinite(c.fx) && std::isfinite(c.fy) && std::isfinite(c.cx) &&
                      std::isfinite(c.cy) && c.fx > 0.f && c.fy > 0.f;
        for (int k = 0; k < 9; ++k) finite = finite && std::isfinite(c.R[k]);
        for (int k = 0; k < 3; ++k) finite = finite && std::isfinite(c.t[k]);
        if (!finite) {
            *err = "camera has non-finite or non-positive intrinsics";
            return false;
        }
        ViewDev& d = out->v[v];
        std::memcpy(d.R, c.R, sizeof(d.R));
        std::memcpy(d.t, c.t, sizeof(d.t));
        d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
        for (int k = 0; k < 3; ++k) {
            const double ck = -((double)c.R[k] * c.t[0] + (double)c.R[3 + k] * c.t[1] +
                                (double)c.R[6 + k] * c.t[2]);
            d.C[k] = (float)ck;
        }
        if (rp->jac_clamp > 0.f) {
            d.lim_x = (float)((double)rp->jac_clamp * (c.width / 2.0) / (double)c.fx);
            d.lim_y = (float)((double)rp->jac_clamp * (c.height / 2.0) / (double)c.fy);
        } else {
            d.lim_x = d.lim_y = INFINITY;
        }
        d.width = c.width;
        d.height = c.height;
        d.tiles_x = (c.width + rp->tile_w - 1) / rp->tile_w;
        d.tiles_y = (c.height + rp->tile_h - 1) / rp->tile_h;
        d.tile_offset = (int32_t)tiles;
        d.px_offset = pixels;
        const int S = rp->super_tile > 0 ? rp->super_tile : kDefaultSuperTile;
        d.sup_x = (d.tiles_x + S - 1) / S;
        d.sup_y = (d.tiles_y + S - 1) / S;
        d.sup_offset = (int32_t)supers;
        tiles += (int64_t)d.tiles_x * d.tiles_y;
        supers += (int64_t)d.sup_x * d.sup_y;
        pixels += (int64_t)c.width * c.height;
    }
    if (tiles > (1 << 24)) {
        *err = "more than 2^24 tiles in one batch";
        return false;
    }
    out->total_tiles = (int32_t)tiles;
    out->total_supers = (int32_t)supers;
    out->total_pixels = pixels;
    return true;
}

RasterDev make_raster(const sgs_raster_params* rp) {
    RasterDev r;
    r.tile_w = rp->tile_w;
    r.tile_h = rp->tile_h;
    r.super_tile = rp->super_tile > 0 ? rp->super_tile : kDefaultSuperTile;
    r.batch = rp->lds_batch > 0 ? rp->lds_batch : kDefaultBatch;
    r.prefix_segs = (int32_t)((rp->split_prefix + kSegPairs - 1) / kSegPairs);
    r.key_bits = 0;   // set with the layout
    r.rect_bits = 0;
    for (int k = 0; k < 3; ++k) r.bg[k] = rp->bg[k];
    r.near_z = rp->near_z;
    r.dilation = rp->dilation;
    r.alpha_min = rp->alpha_min;
    r.alpha_max = rp->alpha_max;
    r.t_min = rp->t_min;
    r.log2_alpha_min = (float)std::log2((double)rp->alpha_min);
    return r;
}

void make_layout(const Views& views, const RasterDev& rp, int64_t n, int64_t capacity, Layout* L) {
    L->n_views = views.n;
    L->entries = n * views.n;
    L->total_tiles = views.total_tiles;
    L->total_supers = views.total_supers;
    L->total_pixels = views.total_pixels;
    L->capacity = capacity;
    L->batch = rp.batch;
    L->seg_slots = segment_slots(capacity, L->total_supers);
    const int64_t tt = (int64_t)rp.super_tile * rp.super_tile;
    // the scans run over the entries and over the (segment, tile) counts
    L->scan_blocks = (std::max(L->entries, L->seg_slots * tt) + 2047) / 2048;
    L->sort_blocks = radix_blocks(std::max(L->entries, capacity));
    // super-tile index bits: 2^bits > total_supers, so that no index has all
    // bits set (at least one: the first sort pass drops culled pairs)
    int bits = 1;
    while ((int64_t(1) << bits) <= L->total_supers) ++bits;
    int rbits = 0;
    while ((1 << rbits) < rp.super_tile) ++rbits;
    L->key_bits = bits;
    L->rect_bits = rbits;
    L->key_passes = radix_passes(bits);
    L->key_result = L->key_passes & 1;
    const int64_t E = L->entries;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L->counters = take(sizeof(uint32_t) * kNumCounters);
    L->views = take(sizeof(Views));
    L->records = take(sizeof(float) * kRecordFloats * (size_t)E);
    L->accum = take(sizeof(float) * kAccumFloats * (size_t)E);
    L->tiles = take(sizeof(uint32_t) * (size_t)E);
    L->depth = take(sizeof(uint32_t) * (size_t)E);
    L->dkey[0] = take(sizeof(uint32_t) * (size_t)E);
    L->dkey[1] = take(sizeof(uint32_t) * (size_t)E);
    L->dval[0] = take(sizeof(uint32_t) * (size_t)E);
    L->dval[1] = take(sizeof(uint32_t) * (size_t)E);
    L->offsets = take(sizeof(uint32_t) * (size_t)E);
    L->window_first = take(sizeof(uint32_t) * (size_t)(emit_windows(E, capacity) + 1));
    L->scan_sums = take(sizeof(uint32_t) * (size_t)(L->scan_blocks + 1));
    L->pair_key[0] = take(sizeof(uint32_t) * (size_t)capacity);
    L->pair_key[1] = take(sizeof(uint32_t) * (size_t)capacity);
    L->pair_entry[0] = take(sizeof(uint32_t) * (size_t)capacity);
    L->pair_entry[1] = take(sizeof(uint32_t) * (size_t)capacity);
    L->sort_hist = take(sizeof(uint32_t) * 256 * (size_t)L->sort_blocks);
    L->sort_totals = take(sizeof(uint32_t) * 256);
    L->sup_ranges = take(sizeof(uint32_t) * 2 * (size_t)L->total_supers);
    L->seg_first = take(sizeof(uint32_t) * (size_t)(L->total_supers + 1));
    L->seg_cnt = take(sizeof(uint32_t) * (size_t)(L->seg_slots * tt));
    L->seg_off = take(sizeof(uint32_t) * (size_t)(L->seg_slots * tt));
    L->pair_mask = take(sizeof(uint64_t) * (size_t)capacity);
    L->tile_entry = take(sizeof(uint32_t) * (size_t)capacity);
    L->tile_ranges = take(sizeof(uint32_t) * 2 * (size_t)L->total_tiles);
    L->tile_state = take(sizeof(uint32_t) * (size_t)L->total_tiles);
    L->tile_resume = take(sizeof(uint32_t) * (size_t)L->total_tiles);
    L->sup_redo = take(sizeof(uint32_t) * (size_t)L->total_supers);
    L->tile_cost = take(sizeof(uint32_t) * (size_t)L->total_tiles);
    L->tile_stats = take(sizeof(uint32_t) * 2 * (size_t)L->total_tiles);
    L->tile_order = take(sizeof(uint32_t) * (size_t)L->total_tiles);
    L->t_final = take(sizeof(float) * (size_t)L->total_pixels);
    L->n_last = take(sizeof(uint32_t) * (size_t)L->total_pixels);
    L->total = off;
}

}  // namespace sgs

using sgs::Layout;

// Scratch of sgs_photometric_loss_static: the per-tile partial sums of the
// loss forward (every call overwrites all it reads, so nothing needs
// clearing). One copy per GPU, at its own device address, held until the
// process ends; its address is looked up once per device and kept.
constexpr int64_t kStaticLossPartials = int64_t(1) << 17;   // 65536 tiles of 16x16 pixels
static __device__ __align__(256) float scratch[kStaticLossPartials];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

sgs_status static_scratch(float** out) {
    int dev = -1;
    SGS_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SGS_ERR_UNSUPPORTED, "device %d beyond the %d the static scratch serves", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        SGS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SGS_OK;
}

}  // namespace

extern "C" {

const char* sgs_last_error(void) { return g_err.c_str(); }

int32_t sgs_version(void) { return 100; }

void sgs_default_raster_params(sgs_raster_params* rp) {
    if (!rp) return;
    rp->struct_size = sizeof(sgs_raster_params);
    rp->tile_w = 16;
    rp->tile_h = 16;
    rp->super_tile = sgs::kDefaultSuperTile;
    rp->lds_batch = sgs::kDefaultBatch;
    rp->split_prefix = sgs::kDefaultSplitPrefix;
    rp->bg[0] = rp->bg[1] = rp->bg[2] = 0.f;
    rp->near_z = 0.2f;
    rp->dilation = 0.3f;
    rp->alpha_min = 1.f / 255.f;
    rp->alpha_max = 0.99f;
    rp->t_min = 1e-4f;
    rp->jac_clamp = 1.3f;
}

sgs_status sgs_forward_workspace_size(const sgs_raster_params* rp, int64_t n,
                                      const sgs_camera* cams, int32_t n_views,
                                      int64_t pair_capacity, size_t* bytes_out) {
    if (!bytes_out) return fail(SGS_ERR_INVALID_ARG, "bytes_out is null");
    Prepared P;
    sgs_status st = prepare(rp, n, cams, n_views, pair_capacity, &P);
    if (st != SGS_OK) return st;
    *bytes_out = P.L.total;
    return SGS_OK;
}

sgs_status sgs_get_workspace_layout(const sgs_raster_params* rp, int64_t n, const sgs_camera* cams,
                                    int32_t n_views, int64_t pair_capacity,
                                    sgs_workspace_layout* out) {
    if (!out) return fail(SGS_ERR_INVALID_ARG, "out is null");
    Prepared P;
    sgs_status st = prepare(rp, n, cams, n_views, pair_capacity, &P);
    if (st != SGS_OK) return st;
    const Layout& L = P.L;
    out->records = L.records;
    out->tiles = L.tiles;
    out->depth = L.depth;
    out->sup_key = L.pair_key[L.key_result];
    out->sup_entry = L.pair_entry[L.key_result];
    out->sup_ranges = L.sup_ranges;
    out->tile_entry = L.tile_entry;
    out->tile_ranges = L.tile_ranges;
    out->t_final = L.t_final;
    out->n_last = L.n_last;
    out->accum = L.accum;
    out->counters = L.counters;
    out->entries = L.entries;
    out->total_tiles = L.total_tiles;
    out->total_pixels = L.total_pixels;
    out->total_supers = L.total_supers;
    out->key_bits = L.key_bits;
    out->rect_bits = L.rect_bits;
    out->batch = L.batch;
    out->super_tile = P.rd.super_tile;
    return SGS_OK;
}

namespace {

// Validated arguments of a render-path call and the call's view table stored
// into its workspace (the first launch of every call).
sgs_status begin_call(const sgs_raster_params* rp, int64_t n, const sgs_camera* cams,
                      int32_t n_views, void* workspace, size_t workspace_bytes,
                      int64_t pair_capacity, hipStream_t s, Prepared* P) {
    sgs_status st = prepare(rp, n, cams, n_views, pair_capacity, P);
    if (st != SGS_OK) return st;
    if ((st = check_ws(*P, workspace, workspace_bytes)) != SGS_OK) return st;
    char* ws = static_cast<char*>(workspace);
    SGS_HIP(sgs::launch_store_views(P->views, nullptr, 0, nullptr,
                                    reinterpret_cast<sgs::Views*>(ws + P->L.views), s),
            "store views");
    return SGS_OK;
}

}  // namespace

sgs_status sgs_project(const sgs_gaussians* g, const sgs_camera* cams, int32_t n_views,
                       const sgs_raster_params* rp, void* workspace, size_t workspace_bytes,
                       int64_t pair_capacity, void* stream) {
    sgs_status st = check_gaussians(g);
    if (st != SGS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prepared P;
    if ((st = begin_call(rp, g->n, cams, n_views, workspace, workspace_bytes, pair_capacity, s,
                         &P)) != SGS_OK)
        return st;
    SGS_HIP(sgs::launch_project(g->data, g->n, g->stride, g->sh_degree, P.rd, P.L,
                                static_cast<char*>(workspace), s),
            "project");
    return SGS_OK;
}

sgs_status sgs_load_records(const sgs_camera* cams, int32_t n_views, int64_t n,
                            const sgs_raster_params* rp, void* workspace, size_t workspace_bytes,
                            int64_t pair_capacity, const float* u, const float* v,
                            const float* depth, const int32_t* extent, const float* conic,
                            const float* opacity, const float* rgb, void* stream) {
    Prepared P;
    sgs_status st = prepare(rp, n, cams, n_views, pair_capacity, &P);
    if (st != SGS_OK) return st;
    if (P.L.entries > 0 && (!u || !v || !depth || !extent || !conic || !opacity || !rgb))
        return fail(SGS_ERR_INVALID_ARG, "record arrays are null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = begin_call(rp, n, cams, n_views, workspace, workspace_bytes, pair_capacity, s, &P)) !=
        SGS_OK)
        return st;
    SGS_HIP(sgs::launch_load_records(u, v, depth, extent, conic, opacity, rgb, n, P.rd, P.L,
                                     static_cast<char*>(workspace), s),
            "load_records");
    return SGS_OK;
}

sgs_status sgs_bin(const sgs_camera* cams, int32_t n_views, int64_t n, const sgs_raster_params* rp,
                   void* workspace, size_t workspace_bytes, int64_t pair_capacity, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prepared P;
    sgs_status st = begin_call(rp, n, cams, n_views, workspace, workspace_bytes, pair_capacity, s, &P);
    if (st != SGS_OK) return st;
    SGS_HIP(sgs::launch_bin(P.rd, n, P.L, static_cast<char*>(workspace), s), "bin");
    return SGS_OK;
}

sgs_status sgs_rasterize(const sgs_camera* cams, int32_t n_views, int64_t n,
                         const sgs_raster_params* rp, void* workspace, size_t workspace_bytes,
                         int64_t pair_capacity, float* out_rgb, void* stream) {
    if (!out_rgb) return fail(SGS_ERR_INVALID_ARG, "out_rgb is null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prepared P;
    sgs_status st = begin_call(rp, n, cams, n_views, workspace, workspace_bytes, pair_capacity, s, &P);
    if (st != SGS_OK) return st;
    SGS_HIP(sgs::launch_rasterize(P.rd, P.L, static_cast<char*>(workspace), out_rgb, s),
            "rasterize");
    return SGS_OK;
}

sgs_status sgs_render_forward(const sgs_gaussians* g, const sgs_camera* cams, int32_t n_views,
                              const sgs_raster_params* rp, void* workspace, size_t workspace_bytes,
                              int64_t pair_capacity, float* out_rgb, void* stream) {
    sgs_status st = check_gaussians(g);
    if (st != SGS_OK) return st;
    if (!out_rgb) return fail(SGS_ERR_INVALID_ARG, "out_rgb is null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prepared P;
    if ((st = begin_call(rp, g->n, cams, n_views, workspace, workspace_bytes, pair_capacity, s,
                         &P)) != SGS_OK)
        return st;
    char* ws = static_cast<char*>(workspace);
    SGS_HIP(sgs::launch_project(g->data, g->n, g->stride, g->sh_degree, P.rd, P.L, ws, s),
            "project");
    SGS_HIP(sgs::launch_bin(P.rd, g->n, P.L, ws, s), "bin");
    SGS_HIP(sgs::launch_rasterize(P.rd, P.L, ws, out_rgb, s), "rasterize");
    return SGS_OK;
}

sgs_status sgs_rasterize_backward(const sgs_camera* cams, int32_t n_views, int64_t n,
                                  const sgs_raster_params* rp, void* workspace,
                                  size_t workspace_bytes, int64_t pair_capacity,
                                  const float* dl_drgb, const int32_t* d_gate, void* stream) {
    if (!dl_drgb) return fail(SGS_ERR_INVALID_ARG, "dl_drgb is null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prepared P;
    sgs_status st = begin_call(rp, n, cams, n_views, workspace, workspace_bytes, pair_capacity, s, &P);
    if (st != SGS_OK) return st;
    SGS_HIP(sgs::launch_rasterize_backward(P.rd, P.L, static_cast<char*>(workspace), dl_drgb,
                                           d_gate, s),
            "rasterize_backward");
    return SGS_OK;
}

sgs_status sgs_project_backward(const sgs_gaussians* g, const sgs_camera* cams, int32_t n_views,
                                const sgs_raster_params* rp, void* workspace,
                                size_t workspace_bytes, int64_t pair_capacity,
                                const int32_t* d_gate, float* grads, void* stream) {
    sgs_status st = check_gaussians(g);
    if (st != SGS_OK) return st;
    if (!grads || !aligned(grads, 16)) return fail(SGS_ERR_INVALID_ARG, "grads null or unaligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prepared P;
    if ((st = begin_call(rp, g->n, cams, n_views, workspace, workspace_bytes, pair_capacity, s,
                         &P)) != SGS_OK)
        return st;
    SGS_HIP(sgs::launch_project_backward(g->data, g->n, g->stride, g->sh_degree, P.rd, P.L,
                                         static_cast<char*>(workspace), d_gate, grads, s),
            "project_backward");
    return SGS_OK;
}

sgs_status sgs_render_backward(const sgs_gaussians* g, const sgs_camera* cams, int32_t n_views,
                               const sgs_raster_params* rp, void* workspace,
                               size_t workspace_bytes, int64_t pair_capacity,
                               const float* dl_drgb, const int32_t* d_gate, float* grads,
                               void* stream) {
    sgs_status st = check_gaussians(g);
    if (st != SGS_OK) return st;
    if (!dl_drgb) return fail(SGS_ERR_INVALID_ARG, "dl_drgb is null");
    if (!grads || !aligned(grads, 16)) return fail(SGS_ERR_INVALID_ARG, "grads null or unaligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prepared P;
    if ((st = begin_call(rp, g->n, cams, n_views, workspace, workspace_bytes, pair_capacity, s,
                         &P)) != SGS_OK)
        return st;
    char* ws = static_cast<char*>(workspace);
    SGS_HIP(sgs::launch_rasterize_backward(P.rd, P.L, ws, dl_drgb, d_gate, s),
            "rasterize_backward");
    SGS_HIP(sgs::launch_project_backward(g->data, g->n, g->stride, g->sh_degree, P.rd, P.L, ws,
                                         d_gate, grads, s),
            "project_backward");
    return SGS_OK;
}

sgs_status sgs_read_status(const void* workspace, uint32_t* flags_out, int64_t* visible_out,
                           int64_t* pairs_out, void* stream) {
    if (!workspace) return fail(SGS_ERR_INVALID_ARG, "workspace is null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    SGS_HIP(hipStreamSynchronize(s), "stream sync");
    uint32_t c[sgs::kNumCounters];
    // the counters region sits at offset 0 of every forward workspace
    SGS_HIP(hipMemcpy(c, workspace, sizeof(c), hipMemcpyDeviceToHost), "read counters");
    if (flags_out) *flags_out = c[sgs::kStatus];
    if (visible_out) *visible_out = c[sgs::kVisible];
    // list entries of both splits, saturating like the device's own sums
    const uint32_t items = c[sgs::kItems] + c[sgs::kItemsRest] < c[sgs::kItems]
                               ? 0xffffffffu
                               : c[sgs::kItems] + c[sgs::kItemsRest];
    if (pairs_out) *pairs_out = std::max(c[sgs::kPairs], items);
    return SGS_OK;
}

sgs_status sgs_clear_status(void* workspace, void* stream) {
    if (!workspace) return fail(SGS_ERR_INVALID_ARG, "workspace is null");
    // a kernel rather than a memset node, so that the call can be captured
    SGS_HIP(sgs::fill_u32(static_cast<uint32_t*>(workspace), 1, 0u,
                          static_cast<hipStream_t>(stream)),
            "clear status");
    return SGS_OK;
}

sgs_status sgs_loss_workspace_size(int32_t width, int32_t height, size_t* bytes_out) {
    if (!bytes_out) return fail(SGS_ERR_INVALID_ARG, "bytes_out is null");
    if (width <= 0 || height <= 0 || width > 32768 || height > 32768)
        return fail(SGS_ERR_INVALID_ARG, "image size not in [1, 32768]");
    *bytes_out = sgs::loss_workspace_bytes(width, height);
    return SGS_OK;
}

sgs_status sgs_photometric_loss(const float* rgb, const float* target, int32_t width,
                                int32_t height, float lambda, void* workspace,
                                size_t workspace_bytes, float* d_loss, void* stream) {
    if (!rgb || !target || !d_loss || !workspace)
        return fail(SGS_ERR_INVALID_ARG, "null pointer argument");
    if (width <= 0 || height <= 0 || width > 32768 || height > 32768)
        return fail(SGS_ERR_INVALID_ARG, "image size not in [1, 32768]");
    if (!(lambda >= 0.f && lambda <= 1.f)) return fail(SGS_ERR_INVALID_ARG, "lambda not in [0, 1]");
    if (workspace_bytes < sgs::loss_workspace_bytes(width, height))
        return fail(SGS_ERR_CAPACITY, "loss workspace too small");
    SGS_HIP(sgs::launch_loss_forward(rgb, sgs::TargetRef{target, nullptr, 1}, width, height, lambda,
                                     static_cast<char*>(workspace), d_loss,
                                     static_cast<hipStream_t>(stream)),
            "loss");
    return SGS_OK;
}

sgs_status sgs_photometric_loss_static(const float* rgb, const float* target, int32_t width,
                                       int32_t height, float lambda, float* d_loss,
                                       void* stream) {
    if (!rgb || !target || !d_loss) return fail(SGS_ERR_INVALID_ARG, "null pointer argument");
    if (width <= 0 || height <= 0 || width > 32768 || height > 32768)
        return fail(SGS_ERR_INVALID_ARG, "image size not in [1, 32768]");
    if (!(lambda >= 0.f && lambda <= 1.f)) return fail(SGS_ERR_INVALID_ARG, "lambda not in [0, 1]");
    if (sgs::loss_partial_floats(width, height) > kStaticLossPartials)
        return fail(SGS_ERR_CAPACITY,
                    "%dx%d image needs %lld partial sums; the static scratch holds %lld "
                    "(images up to %lld tiles of 16x16 pixels)",
                    width, height, (long long)sgs::loss_partial_floats(width, height),
                    (long long)kStaticLossPartials, (long long)(kStaticLossPartials / 2));
    float* partials = nullptr;
    if (sgs_status st = static_scratch(&partials); st != SGS_OK) return st;
    SGS_HIP(sgs::launch_loss_partials(rgb, sgs::TargetRef{target, nullptr, 1}, width, height,
                                      lambda, partials, d_loss, static_cast<hipStream_t>(stream)),
            "loss");
    return SGS_OK;
}

sgs_status sgs_photometric_loss_backward(const float* rgb, const float* target, int32_t width,
                                         int32_t height, float lambda, void* workspace,
                                         size_t workspace_bytes, const int32_t* d_gate,
                                         float* dl_drgb, void* stream) {
    if (!rgb || !target || !dl_drgb || !workspace)
        return fail(SGS_ERR_INVALID_ARG, "null pointer argument");
    if (width <= 0 || height <= 0 || width > 32768 || height > 32768)
        return fail(SGS_ERR_INVALID_ARG, "image size not in [1, 32768]");
    if (!(lambda >= 0.f && lambda <= 1.f)) return fail(SGS_ERR_INVALID_ARG, "lambda not in [0, 1]");
    if (workspace_bytes < sgs::loss_workspace_bytes(width, height))
        return fail(SGS_ERR_CAPACITY, "loss workspace too small");
    SGS_HIP(sgs::launch_loss_backward(rgb, sgs::TargetRef{target, nullptr, 1}, width, height, lambda,
                                      static_cast<char*>(workspace), d_gate, dl_drgb,
                                      static_cast<hipStream_t>(stream)),
            "loss backward");
    return SGS_OK;
}

static sgs_status check_gate(const sgs_gate_params* p) {
    if (!p) return fail(SGS_ERR_INVALID_ARG, "gate params are null");
    if (p->struct_size != sizeof(sgs_gate_params))
        return fail(SGS_ERR_INVALID_ARG, "gate params struct_size %u, expected %zu", p->struct_size,
                    sizeof(sgs_gate_params));
    if (p->n_views < 1) return fail(SGS_ERR_INVALID_ARG, "n_views < 1");
    if (!(p->beta > 0.0 && p->beta < 1.0)) return fail(SGS_ERR_INVALID_ARG, "beta not in (0, 1)");
    if (!(p->eps >= 0.0) || !std::isfinite(p->delta) || !(p->rho_lo >= 0.0 && p->rho_lo <= 1.0))
        return fail(SGS_ERR_INVALID_ARG, "eps, delta or rho_lo out of range");
    if (p->warmup < 0 || p->window < 0) return fail(SGS_ERR_INVALID_ARG, "warmup/window < 0");
    return SGS_OK;
}

sgs_status sgs_gate_state_size(const sgs_gate_params* p, size_t* bytes_out) {
    sgs_status st = check_gate(p);
    if (st != SGS_OK) return st;
    if (!bytes_out) return fail(SGS_ERR_INVALID_ARG, "bytes_out is null");
    *bytes_out = sgs::gate_state_bytes(p);
    return SGS_OK;
}

sgs_status sgs_gate_init(const sgs_gate_params* p, void* d_state, void* stream) {
    sgs_status st = check_gate(p);
    if (st != SGS_OK) return st;
    if (!d_state || !aligned(d_state, 8)) return fail(SGS_ERR_INVALID_ARG, "state null or unaligned");
    SGS_HIP(sgs::launch_gate_init(p, d_state, static_cast<hipStream_t>(stream)), "gate init");
    return SGS_OK;
}

sgs_status sgs_gate_update(const sgs_gate_params* p, void* d_state, const int32_t* d_view,
                           const float* d_loss, int32_t* d_gate, void* stream) {
    sgs_status st = check_gate(p);
    if (st != SGS_OK) return st;
    if (!d_state || !d_view || !d_loss || !d_gate)
        return fail(SGS_ERR_INVALID_ARG, "null pointer argument");
    if (!aligned(d_state, 8)) return fail(SGS_ERR_INVALID_ARG, "gate state not 8-byte aligned");
    SGS_HIP(sgs::launch_gate_update(p, d_state, d_view, d_loss, d_gate,
                                    static_cast<hipStream_t>(stream)),
            "gate update");
    return SGS_OK;
}

sgs_status sgs_gate_read(const sgs_gate_params* p, const void* d_state, sgs_gate_snapshot* out,
                         double* ema_out, uint8_t* has_ema_out, void* stream) {
    sgs_status st = check_gate(p);
    if (st != SGS_OK) return st;
    if (!d_state || !out) return fail(SGS_ERR_INVALID_ARG, "null pointer argument");
    SGS_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "stream sync");
    const char* base = static_cast<const char*>(d_state);
    SGS_HIP(hipMemcpy(out, base, sizeof(*out), hipMemcpyDeviceToHost), "read gate");
    if (ema_out)
        SGS_HIP(hipMemcpy(ema_out, base + sizeof(sgs_gate_snapshot), sizeof(double) * p->n_views,
                          hipMemcpyDeviceToHost),
                "read ema");
    if (has_ema_out)
        SGS_HIP(hipMemcpy(has_ema_out,
                          base + sizeof(sgs_gate_snapshot) + sizeof(double) * p->n_views,
                          p->n_views, hipMemcpyDeviceToHost),
                "read has_ema");
    return SGS_OK;
}

static sgs_status check_adam(const sgs_adam_params* p);

sgs_status sgs_adam_step(const sgs_adam_params* p, float* params, float* grads, float* m,
                         float* v, int64_t n, int64_t stride, int32_t n_planes, int32_t* d_step,
                         const int32_t* d_gate, void* stream) {
    sgs_status st;
    if (!p || !params || !grads || !m || !v || !d_step)
        return fail(SGS_ERR_INVALID_ARG, "null pointer argument");
    if (n < 0 || stride < n || stride % 64 != 0 || stride <= 0)
        return fail(SGS_ERR_INVALID_ARG, "stride must be >= n, > 0 and a multiple of 64");
    if (n_planes < 1 || n_planes > SGS_MAX_PLANES)
        return fail(SGS_ERR_INVALID_ARG, "n_planes %d not in [1, %d]", n_planes, SGS_MAX_PLANES);
    if (!aligned(params, 16) || !aligned(grads, 16) || !aligned(m, 16) || !aligned(v, 16))
        return fail(SGS_ERR_INVALID_ARG, "arrays must be 16-byte aligned");
    if ((st = check_adam(p)) != SGS_OK) return st;
    if (p->visible_only)
        return fail(SGS_ERR_UNSUPPORTED, "visible_only needs the fused projection backward step");
    SGS_HIP(sgs::launch_adam(p, params, grads, m, v, n, stride, n_planes, d_step, d_gate,
                             static_cast<hipStream_t>(stream)),
            "adam");
    return SGS_OK;
}

static sgs_status check_adam(const sgs_adam_params* p) {
    if (!p) return fail(SGS_ERR_INVALID_ARG, "adam params are null");
    if (p->struct_size != sizeof(sgs_adam_params))
        return fail(SGS_ERR_INVALID_ARG, "adam params struct_size %u, expected %zu", p->struct_size,
                    sizeof(sgs_adam_params));
    if (!(p->beta1 >= 0.0 && p->beta1 < 1.0) || !(p->beta2 >= 0.0 && p->beta2 < 1.0) ||
        !(p->eps >= 0.0) || (p->visible_only != 0 && p->visible_only != 1))
        return fail(SGS_ERR_INVALID_ARG, "Adam constants out of range");
    return SGS_OK;
}

sgs_status sgs_project_backward_adam(const sgs_gaussians* g, const sgs_camera* cams,
                                     int32_t n_views, const sgs_raster_params* rp,
                                     void* workspace, size_t workspace_bytes,
                                     int64_t pair_capacity, const sgs_adam_params* adam,
                                     float* m, float* v, int32_t* d_step,
                                     const int32_t* d_gate, void* stream) {
    sgs_status st = check_gaussians(g);
    if (st != SGS_OK) return st;
    if ((st = check_adam(adam)) != SGS_OK) return st;
    if (!m || !v || !d_step) return fail(SGS_ERR_INVALID_ARG, "m, v or step is null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prepared P;
    if ((st = begin_call(rp, g->n, cams, n_views, workspace, workspace_bytes, pair_capacity, s,
                         &P)) != SGS_OK)
        return st;
    SGS_HIP(sgs::launch_project_backward_adam(g->data, g->n, g->stride, g->sh_degree, P.rd, P.L,
                                              static_cast<char*>(workspace), adam,
                                              adam->visible_only != 0, m, v, d_step, d_gate, s),
            "project_backward_adam");
    return SGS_OK;
}

sgs_status sgs_render_backward_adam(const sgs_gaussians* g, const sgs_camera* cams,
                                    int32_t n_views, const sgs_raster_params* rp, void* workspace,
                                    size_t workspace_bytes, int64_t pair_capacity,
                                    const float* dl_drgb, const sgs_adam_params* adam, float* m,
                                    float* v, int32_t* d_step, const int32_t* d_gate,
                                    void* stream) {
    sgs_status st = check_gaussians(g);
    if (st != SGS_OK) return st;
    if ((st = check_adam(adam)) != SGS_OK) return st;
    if (!dl_drgb) return fail(SGS_ERR_INVALID_ARG, "dl_drgb is null");
    if (!m || !v || !d_step) return fail(SGS_ERR_INVALID_ARG, "m, v or step is null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prepared P;
    if ((st = begin_call(rp, g->n, cams, n_views, workspace, workspace_bytes, pair_capacity, s,
                         &P)) != SGS_OK)
        return st;
    char* ws = static_cast<char*>(workspace);
    SGS_HIP(sgs::launch_rasterize_backward(P.rd, P.L, ws, dl_drgb, d_gate, s),
            "rasterize_backward");
    SGS_HIP(sgs::launch_project_backward_adam(g->data, g->n, g->stride, g->sh_degree, P.rd, P.L,
                                              ws, adam, adam->visible_only != 0, m, v, d_step,
                                              d_gate, s),
            "project_backward_adam");
    return SGS_OK;
}

sgs_status sgs_camera_table_size(int32_t n_cams, size_t* bytes_out) {
    if (!bytes_out) return fail(SGS_ERR_INVALID_ARG, "bytes_out is null");
    if (n_cams < 1) return fail(SGS_ERR_INVALID_ARG, "n_cams < 1");
    *bytes_out = sizeof(sgs::ViewDev) * (size_t)n_cams;
    return SGS_OK;
}

sgs_status sgs_camera_table_init(const sgs_camera* cams, int32_t n_cams,
                                 const sgs_raster_params* rp, void* d_table, size_t table_bytes,
                                 void* stream) {
    sgs_status st = check_raster(rp);
    if (st != SGS_OK) return st;
    if (!cams || n_cams < 1) return fail(SGS_ERR_INVALID_ARG, "no cameras");
    if (!d_table || !aligned(d_table, 16)) return fail(SGS_ERR_INVALID_ARG, "table null or unaligned");
    if (table_bytes < sizeof(sgs::ViewDev) * (size_t)n_cams)
        return fail(SGS_ERR_CAPACITY, "camera table has %zu bytes, needs %zu", table_bytes,
                    sizeof(sgs::ViewDev) * (size_t)n_cams);
    std::vector<sgs::ViewDev> host((size_t)n_cams);
    for (int32_t i = 0; i < n_cams; ++i) {
        if (cams[i].width != cams[0].width || cams[i].height != cams[0].height)
            return fail(SGS_ERR_INVALID_ARG, "camera %d is %dx%d, camera 0 is %dx%d", i,
                        cams[i].width, cams[i].height, cams[0].width, cams[0].height);
        sgs::Views one;
        const char* err = nullptr;
        if (!sgs::make_views(cams + i, 1, rp, &one, &err))
            return fail(SGS_ERR_INVALID_ARG, "camera %d: %s", i, err);
        host[(size_t)i] = one.v[0];
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    SGS_HIP(hipMemcpyAsync(d_table, host.data(), sizeof(sgs::ViewDev) * (size_t)n_cams,
                           hipMemcpyHostToDevice, s),
            "copy camera table");
    SGS_HIP(hipStreamSynchronize(s), "stream sync");
    return SGS_OK;
}

sgs_status sgs_view_sequence_next(const int32_t* d_sequence, int64_t sequence_len,
                                  int64_t* d_iter, int32_t* d_view, void* stream) {
    if (!d_sequence || !d_iter || !d_view) return fail(SGS_ERR_INVALID_ARG, "null pointer argument");
    if (sequence_len < 1) return fail(SGS_ERR_INVALID_ARG, "sequence_len < 1");
    if (!aligned(d_iter, 8)) return fail(SGS_ERR_INVALID_ARG, "d_iter not 8-byte aligned");
    SGS_HIP(sgs::launch_sequence_next(d_sequence, sequence_len, d_iter, d_view,
                                      static_cast<hipStream_t>(stream)),
            "view sequence");
    return SGS_OK;
}

sgs_status sgs_train_iteration(const sgs_gaussians* g, const sgs_camera* cams,
                               const void* d_table, int32_t n_cams, const int32_t* d_view,
                               const sgs_raster_params* rp, void* workspace,
                               size_t workspace_bytes, int64_t pair_capacity,
                               const float* targets, float lambda, void* loss_workspace,
                               size_t loss_workspace_bytes, float* rgb, float* dl_drgb,
                               float* d_loss, const sgs_gate_params* gp, void* gate_state,
                               int32_t* d_gate, const sgs_adam_params* adam, float* m, float* v,
                               int32_t* d_step, void* stream) {
    sgs_status st = check_gaussians(g);
    if (st != SGS_OK) return st;
    if ((st = check_adam(adam)) != SGS_OK) return st;
    if (!d_table || !aligned(d_table, 16) || !d_view || n_cams < 1)
        return fail(SGS_ERR_INVALID_ARG, "camera table, view index or n_cams missing");
    if (!targets || !rgb || !dl_drgb || !d_loss || !d_gate || !m || !v || !d_step ||
        !loss_workspace)
        return fail(SGS_ERR_INVALID_ARG, "null pointer argument");
    if (!(lambda >= 0.f && lambda <= 1.f)) return fail(SGS_ERR_INVALID_ARG, "lambda not in [0, 1]");
    if (gate_state != nullptr) {
        if ((st = check_gate(gp)) != SGS_OK) return st;
        if (!aligned(gate_state, 8)) return fail(SGS_ERR_INVALID_ARG, "gate state not 8-byte aligned");
    }
    Prepared P;
    if ((st = prepare(rp, g->n, cams, 1, pair_capacity, &P)) != SGS_OK) return st;
    if ((st = check_ws(P, workspace, workspace_bytes)) != SGS_OK) return st;
    const int w = cams[0].width, h = cams[0].height;
    if (loss_workspace_bytes < sgs::loss_workspace_bytes(w, h))
        return fail(SGS_ERR_CAPACITY, "loss workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    char* lws = static_cast<char*>(loss_workspace);
    const sgs::TargetRef tgt{targets, d_view, n_cams};
    SGS_HIP(sgs::launch_store_views(P.views, static_cast<const sgs::ViewDev*>(d_table), n_cams,
                                    d_view, reinterpret_cast<sgs::Views*>(ws + P.L.views), s),
            "select view");
    SGS_HIP(sgs::launch_project(g->data, g->n, g->stride, g->sh_degree, P.rd, P.L, ws, s),
            "project");
    SGS_HIP(sgs::launch_bin(P.rd, g->n, P.L, ws, s), "bin");
    SGS_HIP(sgs::launch_rasterize(P.rd, P.L, ws, rgb, s), "rasterize");
    SGS_HIP(sgs::launch_loss_forward(rgb, tgt, w, h, lambda, lws, d_loss, s), "loss");
    if (gate_state != nullptr)
        SGS_HIP(sgs::launch_gate_update(gp, gate_state, d_view, d_loss, d_gate, s), "gate");
    else
        SGS_HIP(sgs::fill_u32(reinterpret_cast<uint32_t*>(d_gate), 1, 1u, s), "open gate");
    SGS_HIP(sgs::launch_loss_backward(rgb, tgt, w, h, lambda, lws, d_gate, dl_drgb, s),
            "loss backward");
    SGS_HIP(sgs::launch_rasterize_backward(P.rd, P.L, ws, dl_drgb, d_gate, s), "rasterize_backward");
    SGS_HIP(sgs::launch_project_backward_adam(g->data, g->n, g->stride, g->sh_degree, P.rd, P.L, ws,
                                              adam, adam->visible_only != 0, m, v, d_step, d_gate,
                                              s),
            "project_backward_adam");
    return SGS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adaptive density control
// ---------------------------------------------------------------------------
namespace {

sgs_status check_densify(const sgs_densify_params* p) {
    if (!p) return fail(SGS_ERR_INVALID_ARG, "densify params are null");
    if (p->struct_size != sizeof(sgs_densify_params))
        return fail(SGS_ERR_INVALID_ARG, "densify params struct_size %u, expected %zu",
                    p->struct_size, sizeof(sgs_densify_params));
    if (!(p->grad_threshold >= 0.f) || !std::isfinite(p->grad_threshold) ||
        !(p->percent_dense > 0.f) || !(p->scene_extent > 0.f) ||
        !std::isfinite(p->percent_dense * p->scene_extent) || !(p->min_opacity >= 0.f) ||
        !(p->min_opacity < 1.f) || !(p->split_scale > 0.f) || !std::isfinite(p->split_scale))
        return fail(SGS_ERR_INVALID_ARG, "densify params out of range");
    return SGS_OK;
}

sgs::DensifyDev make_densify(const sgs_densify_params* p) {
    sgs::DensifyDev d;
    d.grad_threshold = p->grad_threshold;
    d.log_size = (float)std::log((double)p->percent_dense * (double)p->scene_extent);
    const double mo = (double)p->min_opacity;
    // logit(0) = -inf: nothing prunes
    d.logit_min = mo > 0.0 ? (float)std::log(mo / (1.0 - mo)) : -INFINITY;
    d.log_split = (float)std::log((double)p->split_scale);
    return d;
}

}  // namespace

extern "C" {

void sgs_default_densify_params(sgs_densify_params* p) {
    if (!p) return;
    p->struct_size = sizeof(sgs_densify_params);
    p->grad_threshold = 2e-4f;
    p->percent_dense = 0.01f;
    p->scene_extent = 1.f;
    p->min_opacity = 0.005f;
    p->split_scale = 1.6f;
}

sgs_status sgs_densify_stats(const sgs_camera* cams, int32_t n_views, int64_t n,
                             const sgs_raster_params* rp, const void* workspace,
                             size_t workspace_bytes, int64_t pair_capacity, const int32_t* d_gate,
                             float* grad_sum, int32_t* count, void* stream) {
    Prepared P;
    sgs_status st = prepare(rp, n, cams, n_views, pair_capacity, &P);
    if (st != SGS_OK) return st;
    if ((st = check_ws(P, workspace, workspace_bytes)) != SGS_OK) return st;
    if (n > 0 && (!grad_sum || !count)) return fail(SGS_ERR_INVALID_ARG, "grad_sum or count is null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    SGS_HIP(sgs::launch_densify_stats(P.L, static_cast<char*>(const_cast<void*>(workspace)), n,
                                      d_gate, grad_sum, count, s),
            "densify_stats");
    return SGS_OK;
}

sgs_status sgs_densify_workspace_size(int64_t n, size_t* bytes_out) {
    if (!bytes_out) return fail(SGS_ERR_INVALID_ARG, "bytes_out is null");
    if (n < 0) return fail(SGS_ERR_INVALID_ARG, "n < 0");
    *bytes_out = sizeof(uint32_t) * (size_t)sgs::densify_scratch_words(sgs::densify_blocks(n));
    return SGS_OK;
}

sgs_status sgs_densify(const sgs_densify_params* p, const sgs_gaussians* g, const float* m,
                       const float* v, const float* grad_sum, const int32_t* count,
                       const float* normals, float* out_params, float* out_m, float* out_v,
                       int64_t out_stride, void* workspace, size_t workspace_bytes,
                       int64_t* d_n_out, void* stream) {
    sgs_status st = check_densify(p);
    if (st != SGS_OK) return st;
    if ((st = check_gaussians(g)) != SGS_OK) return st;
    if (!m || !v || !out_params || !out_m || !out_v || !d_n_out)
        return fail(SGS_ERR_INVALID_ARG, "moments, outputs or d_n_out are null");
    if (g->n > 0 && (!grad_sum || !count || !normals))
        return fail(SGS_ERR_INVALID_ARG, "grad_sum, count or normals are null");
    if (out_stride <= 0 || out_stride % 64 != 0 || out_stride >= (int64_t(1) << 29))
        return fail(SGS_ERR_INVALID_ARG, "out_stride %lld must be > 0, < 2^29 and a multiple of 64",
                    (long long)out_stride);
    if (!aligned(out_params, 16) || !aligned(out_m, 16) || !aligned(out_v, 16) ||
        !aligned(m, 16) || !aligned(v, 16))
        return fail(SGS_ERR_INVALID_ARG, "planes not 16-byte aligned");
    const size_t need = sizeof(uint32_t) * (size_t)sgs::densify_scratch_words(sgs::densify_blocks(g->n));
    if (!workspace || workspace_bytes < need || !aligned(workspace, 16))
        return fail(SGS_ERR_CAPACITY, "densify workspace null, unaligned or below %zu bytes", need);
    const int F = 11 + 3 * (g->sh_degree + 1) * (g->sh_degree + 1);
    hipStream_t s = static_cast<hipStream_t>(stream);
    SGS_HIP(sgs::launch_densify(make_densify(p), g->data, const_cast<float*>(m),
                                const_cast<float*>(v), g->n, g->stride, F, grad_sum, count, normals,
                                out_params, out_m, out_v, out_stride,
                                static_cast<uint32_t*>(workspace), d_n_out, s),
            "densify");
    return SGS_OK;
}

}  // extern "C"
