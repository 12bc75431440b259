// bp_api.cpp -- the C ABI declared in include/bp.h: argument validation,
// per-context scratch, the choice of path / views per pass / z-unroll, and
// the launch sequence of one call.
#include "../../include/bp.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "bp_internal.h"

struct bp_ctx_s {
    bp_config cfg;
    std::string last_error;
    // scratch, grown on demand, freed by bp_destroy
    bp::ViewConst* d_views = nullptr;
    size_t views_cap = 0;  // records
    void* d_pad = nullptr;
    size_t pad_cap = 0;  // bytes
    void* d_cull = nullptr;
    size_t cull_cap = 0;  // bytes
    void* d_scale = nullptr;  // compact staging: per-view max |pixel| bits, then 2^-e scales
    size_t scale_cap = 0;
    void* d_fp = nullptr;  // LDS-staged taps: footprint tables of two passes
    size_t fp_cap = 0;
    // Staging of pass p + 1 runs on a side stream while pass p back-projects on the caller's
    // stream; the staging scratch holds two passes (halves 0 and 1).  Default priority.
    hipStream_t side = nullptr;
    hipEvent_t ev_start = nullptr, ev_staged[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
    int options = 0;      // BP_OPT_* flags
    // overrides set by bp_set_tuning (0 = tuned)
    bp_path path_override = BP_PATH_AUTO;
    int k_override = 0;
    int zu_override = 0;
    int tx_override = 0;
    int tap_split = -1;  // views of every 8 of a staged pass that read directly; -1 = tuned
    // kernel timing (bp_enable_timing): event pairs per kernel kind
    bool timing = false;
    struct Pair {
        hipEvent_t start, stop;
    };
    std::vector<Pair> pending[3];
    double total_ms[3] = {0, 0, 0};
    long long launches[3] = {0, 0, 0};
    std::vector<hipEvent_t> event_pool;
    // device address of the allocation-free entry point's static scratch on the context's device
    void* noalloc = nullptr;
};

namespace {

const char* const kVersion = "0.1.0";
// XCD-private region split of each z-layer: ax regions along x, 8 / ax along y (measured at L = 512).
const int kDefaultRegionAx = 8;

bp_status fail(bp_ctx ctx, bp_status st, const std::string& msg)
{
    if (ctx) ctx->last_error = msg;
    return st;
}

// Switch to the context's device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
    }
    ~DeviceGuard()
    {
        if (ok && prev >= 0) (void)hipSetDevice(prev);
    }
};

bool valid_zu(int zu) { return zu == 1 || zu == 2 || zu == 4 || zu == 8; }

// The side stream and its events, created on first use.
bp_status ensure_side(bp_ctx ctx)
{
    if (ctx->side) return BP_OK;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return BP_ERR_DEVICE;
    }
    hipEvent_t* evs[5] = {&ctx->ev_start, &ctx->ev_staged[0], &ctx->ev_staged[1], &ctx->ev_done[0], &ctx->ev_done[1]};
    for (hipEvent_t* e : evs) {
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            for (hipEvent_t* f : evs)
                if (*f) {
                    (void)hipEventDestroy(*f);
                    *f = nullptr;
                }
            (void)hipStreamDestroy(st);
            return BP_ERR_DEVICE;
        }
    }
    ctx->side = st;
    return BP_OK;
}
bool valid_tx(int tx) { return tx == 8 || tx == 16 || tx == 32 || tx == 64; }

bool fault_injected(const char* what)
{
    const char* v = std::getenv("BP_FAULT_INJECT");
    return v && std::strcmp(v, what) == 0;
}

bp_status ensure(bp_ctx ctx, void** ptr, size_t* cap, size_t need, const char* what)
{
    if (need <= *cap) return BP_OK;
    if (*ptr) {
        // Work already enqueued may still read the old buffer.
        if (hipDeviceSynchronize() != hipSuccess || hipFree(*ptr) != hipSuccess)
            return fail(ctx, BP_ERR_DEVICE, std::string("freeing scratch for ") + what + " failed");
        *ptr = nullptr;
        *cap = 0;
    }
    if (fault_injected("alloc") || hipMalloc(ptr, need) != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(ctx, BP_ERR_OUT_OF_MEMORY,
                    std::string("cannot allocate ") + std::to_string(need) + " bytes of scratch for " + what);
    }
    *cap = need;
    return BP_OK;
}

hipEvent_t take_event(bp_ctx ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Bracket one launch with events when timing is on.
template <class F>
hipError_t timed(bp_ctx ctx, int kind, hipStream_t s, F&& launch)
{
    if (!ctx->timing) return launch();
    bp_ctx_s::Pair p{take_event(ctx), take_event(ctx)};
    if (!p.start || !p.stop) return hipErrorOutOfMemory;
    (void)hipEventRecord(p.start, s);
    const hipError_t e = launch();
    (void)hipEventRecord(p.stop, s);
    ctx->pending[kind].push_back(p);
    return e;
}

// Fold finished event pairs into the totals (synchronises on each stop event).
bp_status drain_timing(bp_ctx ctx)
{
    bp_status st = BP_OK;
    for (int k = 0; k < 3; ++k) {
        for (auto& p : ctx->pending[k]) {
            float ms = 0.0f;
            if (hipEventSynchronize(p.stop) != hipSuccess || hipEventElapsedTime(&ms, p.start, p.stop) != hipSuccess)
                st = BP_ERR_DEVICE;
            ctx->total_ms[k] += ms;
            ctx->launches[k] += 1;
            ctx->event_pool.push_back(p.start);
            ctx->event_pool.push_back(p.stop);
        }
        ctx->pending[k].clear();
    }
    return st;
}

// Does the fused path stage its taps through LDS?  (The footprint table packs padded rows
// and columns into 16 bits.)
// 16-bit projections staged as compact FP16 records (on request; by default they are staged like
// FP32 projections, their pixels widened exactly).
bool compact_records(const bp_ctx_s* ctx)
{
    return ctx->cfg.proj_dtype != BP_F32 && (ctx->options & BP_OPT_COMPACT_STAGING) &&
           !(ctx->options & BP_OPT_WIDE_STAGING);
}

bool staged_taps(const bp_ctx_s* ctx, bp::Layout layout, int W, int H)
{
    return layout != bp::Layout::Checked && !(ctx->options & BP_OPT_DIRECT_TAPS) && W + 2 < 65536 && H + 2 < 65536;
}

struct Plan {
    bp_path path;
    int k;
    int zu;
    int tx;
    bool direct_taps = false;  // fused path: every tap through L1, no LDS stage
};

// Tuned defaults (measured on MI355X at L = 512, 496 views); BP_PATH_AUTO
// resolves here unless bp_set_tuning or the context's config fixes a choice.
Plan plan_for(const bp_ctx_s* ctx, int nx, int ny, int nz, int n_views)
{
    Plan p;
    p.path = ctx->path_override != BP_PATH_AUTO ? ctx->path_override : ctx->cfg.path;
    if (p.path == BP_PATH_AUTO) {
        // Coarse voxels (few per detector pixel, so a tile's footprint overflows the LDS stage and
        // no two voxels share a pixel) favour reading the caller's images directly.  Measured at
        // 1248 x 960 pixels, 496 views, 256 mm field: FP32 (pixel-pair taps) direct at L = 384
        // (1030 GUPS against 627 staged), staged at L = 448 (1762 against 1129); BF16 (pixel-pair
        // taps) direct at L = 320 (788 against 660), staged at L = 384 (890 against 819).
        const double voxels = (double)nx * (double)ny * (double)nz;
        const double pixels = (double)ctx->cfg.det_width * (double)ctx->cfg.det_height;
        const double crossover = ctx->cfg.proj_dtype == BP_F32 ? 64.0 : 40.0;
        p.path = voxels < crossover * pixels ? BP_PATH_FUSED_DIRECT : BP_PATH_FUSED;
    }
    // Staged or direct taps for the fused pass.  FP32 records staged as records, on a fine grid
    // (many voxels per detector pixel), reuse the L1 well enough that the direct loads win:
    // measured at 1248 x 960 pixels and a 256 mm field of view, that split is ahead at L = 512
    // and behind from L = 640 up.  Compact records, and FP32 footprints staged as pixels, favour
    // the split at every size measured (pixels at L = 1024: 2675 GUPS against 2396 direct).
    const bool compact = compact_records(ctx);
    const bool pixels = !compact && !(ctx->options & BP_OPT_STAGE_RECORDS);
    const double voxels = (double)nx * (double)ny * (double)nz;
    p.direct_taps = p.path == BP_PATH_FUSED &&
                    ((ctx->options & BP_OPT_DIRECT_TAPS) ||
                     (!compact && !pixels && ctx->tap_split < 0 && voxels >= 2.0e8));
    p.k = ctx->k_override > 0 ? ctx->k_override : ctx->cfg.views_per_pass;
    if (p.k <= 0) {
        if (p.path == BP_PATH_FUSED_DIRECT) p.k = 64;
        else if (p.direct_taps) p.k = compact || voxels >= 2.0e8 ? 64 : 32;
        // LDS-staged taps, measured at 496 views of 1248 x 960: pixel stages of 16-bit input and
        // of large volumes take every view in one pass, up to 512 (against K = 128: BF16 at
        // L = 512 +3.2%, FP32 and BF16 at L = 1024 +7.3% and +5.8%: the volume is read and written
        // once); FP32 pixel stages below 2e8 voxels take K = 64, level in time with one pass and
        // with K = 128 at L = 512 and with the least HBM traffic per update (the footprint bands
        // of fewer views stay in L2); compact records K = 128
        else if (pixels && (ctx->cfg.proj_dtype != BP_F32 || voxels >= 2.0e8)) p.k = std::min(n_views, 512);
        else p.k = pixels ? 64 : 128;
    }
    if (p.path == BP_PATH_PLAIN) p.k = 1;
    if (p.k > n_views) p.k = n_views;
    p.zu = ctx->zu_override > 0 ? ctx->zu_override : ctx->cfg.z_unroll;
    if (p.zu <= 0) p.zu = 8;
    while (p.zu > 1 && p.zu > nz) p.zu >>= 1;
    p.tx = ctx->tx_override > 0 ? ctx->tx_override : ctx->cfg.tile_x;
    if (p.tx <= 0) p.tx = 16;
    // the caller's-image taps come in 16- and 64-wide tiles
    if ((p.path == BP_PATH_PLAIN || p.path == BP_PATH_FUSED_DIRECT) && p.tx != 16) p.tx = 64;

    (void)nx;
    (void)ny;
    return p;
}

bp::Dtype to_dt(bp_dtype d) { return static_cast<bp::Dtype>(static_cast<int>(d)); }

size_t elem_bytes(bp_dtype d);

// What one call of a given shape enqueues and the scratch it needs (bytes per buffer).
struct CallShape {
    Plan plan;
    bp::Layout layout;
    bool lds, culled, staged, raw_stage, overlap;
    int split, words, halves;
    long tiles;
    size_t pad_half, fp_half, scale_half;
    size_t views_bytes, pad_bytes, scale_bytes, cull_bytes, fp_bytes;
    size_t total() const { return views_bytes + pad_bytes + scale_bytes + cull_bytes + fp_bytes; }
};

CallShape call_shape(const bp_ctx_s* ctx, int nx, int ny, int nz, int n_views)
{
    CallShape c;
    const int W = ctx->cfg.det_width, H = ctx->cfg.det_height;
    c.plan = plan_for(ctx, nx, ny, nz, n_views);
    c.layout = c.plan.path == BP_PATH_FUSED ? bp::Layout::Patch : bp::Layout::Checked;
    if (c.layout == bp::Layout::Patch && compact_records(ctx))
        c.layout = bp::Layout::Patch16;
    // LDS-staged taps: the footprint table packs padded rows and columns into 16 bits
    c.lds = !c.plan.direct_taps && staged_taps(ctx, c.layout, W, H);
    // clipping mask for every pass that does not stage footprints (which carry their own skip entries)
    c.culled = !c.lds && !(ctx->options & BP_OPT_NO_CULL);
    c.tiles = bp::n_tiles(nx, ny, nz, c.plan.zu, c.plan.tx);
    c.words = bp::cull_words(n_views);
    // Staging of the next pass overlaps the current pass when there are two or more passes.  Tuned:
    // compact records only (L = 512, 496 views: BF16 2068 -> 2151 GUPS); the FP32 staging kernel
    // contends with the pass for the vector memory path, and the pass slows by what the overlap hides.
    c.staged = c.layout != bp::Layout::Checked;
    // FP32 records (FP32 input, or 16-bit input with wide staging): the LDS stage holds the caller's
    // pixels as FP32 (a quarter of the bytes of the records)
    c.raw_stage = c.lds && c.layout == bp::Layout::Patch && !(ctx->options & BP_OPT_STAGE_RECORDS);
    // share of the views of each 8 that read directly while the others are staged (tuned at L = 512,
    // 496 views, K = 128: pixel stages 0 -- every view staged; BF16 24.55 ms against 25.05 at 1 of 8,
    // FP32 26.57 against 26.49; FP32 record stages 4; compact records 3)
    c.split = ctx->tap_split >= 0 ? ctx->tap_split : (c.raw_stage ? 0 : c.layout == bp::Layout::Patch ? 4 : 3);
    c.overlap = c.staged && n_views > c.plan.k && !(ctx->options & BP_OPT_SERIAL_STAGING) &&
                (c.layout == bp::Layout::Patch16 || (ctx->options & BP_OPT_OVERLAP_STAGING));
    c.halves = c.overlap ? 2 : 1;
    c.pad_half = bp::staged_view_bytes(c.layout, W, H) * (size_t)c.plan.k;
    c.fp_half = (size_t)c.tiles * (size_t)c.plan.k;  // uint2 entries
    c.scale_half = 8u * (size_t)c.plan.k;            // bytes: max |pixel| bits, then 2^-e scales
    c.views_bytes = sizeof(bp::ViewConst) * (size_t)n_views;
    c.pad_bytes = c.staged ? c.pad_half * c.halves : 0;
    c.scale_bytes = c.staged && (c.layout == bp::Layout::Patch16 || c.raw_stage) ? c.scale_half * c.halves : 0;
    c.cull_bytes = c.culled ? (size_t)c.tiles * (size_t)c.words * 4u : 0;
    c.fp_bytes = c.lds ? c.fp_half * c.halves * sizeof(uint2) : 0;
    return c;
}

size_t elem_bytes(bp_dtype d) { return d == BP_F32 ? 4 : 2; }

// Argument checks shared by the entry points (nothing is enqueued when one fails).
bp_status check_call(bp_ctx ctx, const float* volume, int nx, int ny, int nz, const void* projections,
                     const float* matrices, int n_views, float voxel_size, const float origin[3])
{
    if (!volume || !projections || !matrices || !origin)
        return fail(ctx, BP_ERR_INVALID_ARG, "null pointer argument");
    if (nx < 1 || ny < 1 || nz < 1) return fail(ctx, BP_ERR_INVALID_ARG, "volume dimensions must be >= 1");
    if ((uint64_t)nx * (uint64_t)ny * (uint64_t)nz >= ((uint64_t)1 << 40))
        return fail(ctx, BP_ERR_INVALID_ARG, "volume too large");
    if (nx > (1 << 24) || ny > (1 << 24) || nz > (1 << 24))
        return fail(ctx, BP_ERR_INVALID_ARG, "volume edge beyond 2^24 voxels");
    if (n_views < 1) return fail(ctx, BP_ERR_INVALID_ARG, "n_views must be >= 1");
    if (!std::isfinite(voxel_size) || !(voxel_size > 0.0f))
        return fail(ctx, BP_ERR_INVALID_ARG, "voxel_size must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(origin[a])) return fail(ctx, BP_ERR_INVALID_ARG, "origin must be finite");
    if (reinterpret_cast<uintptr_t>(volume) % 4 != 0 || reinterpret_cast<uintptr_t>(matrices) % 4 != 0 ||
        reinterpret_cast<uintptr_t>(projections) % elem_bytes(ctx->cfg.proj_dtype) != 0)
        return fail(ctx, BP_ERR_INVALID_ARG, "misaligned device pointer");
    return BP_OK;
}

// tile order: XCD z-slices (opt-in), plain (opt-in), else XCD-private regions of each z-layer
int tile_order(const bp_ctx_s* ctx)
{
    int xcd_order = 2 * kDefaultRegionAx;
    if (const int r = (ctx->options & BP_OPT_XCD_REGION_MASK) >> BP_OPT_XCD_REGION_SHIFT) xcd_order = 2 * r;
    if (ctx->options & BP_OPT_PLAIN_ORDER) xcd_order = 0;
    if (ctx->options & BP_OPT_XCD_ORDER) xcd_order = 1;
    return xcd_order;
}

}  // namespace

extern "C" {

void bp_config_default(bp_config* cfg)
{
    if (!cfg) return;
    cfg->device = 0;
    cfg->det_width = 1248;
    cfg->det_height = 960;
    cfg->proj_dtype = BP_F32;
    cfg->path = BP_PATH_AUTO;
    cfg->views_per_pass = 0;
    cfg->z_unroll = 0;
    cfg->tile_x = 0;
}

const char* bp_version(void) { return kVersion; }

const char* bp_status_string(bp_status s)
{
    switch (s) {
    case BP_OK: return "ok";
    case BP_ERR_INVALID_ARG: return "invalid argument";
    case BP_ERR_UNSUPPORTED: return "unsupported";
    case BP_ERR_OUT_OF_MEMORY: return "out of device memory";
    case BP_ERR_DEVICE: return "device error";
    case BP_ERR_LAUNCH: return "kernel launch failed";
    }
    return "unknown status";
}

const char* bp_last_error(bp_ctx ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

bp_status bp_create(const bp_config* cfg, bp_ctx* out)
{
    if (!out) return BP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!cfg) return BP_ERR_INVALID_ARG;
    if (cfg->det_width < 1 || cfg->det_height < 1 || cfg->det_width > (1 << 20) ||
        cfg->det_height > (1 << 20))
        return BP_ERR_INVALID_ARG;
    if ((size_t)(cfg->det_width + 3) * (size_t)(cfg->det_height + 3) * 4u >= (size_t)1 << 31)
        return BP_ERR_UNSUPPORTED;  // one view must fit a 32-bit buffer offset
    if (cfg->proj_dtype != BP_F32 && cfg->proj_dtype != BP_F16 && cfg->proj_dtype != BP_BF16)
        return BP_ERR_INVALID_ARG;
    if (cfg->path != BP_PATH_AUTO && cfg->path != BP_PATH_PLAIN && cfg->path != BP_PATH_FUSED &&
        cfg->path != BP_PATH_FUSED_DIRECT)
        return BP_ERR_INVALID_ARG;
    if (cfg->views_per_pass < 0 || (cfg->z_unroll != 0 && !valid_zu(cfg->z_unroll)) ||
        (cfg->tile_x != 0 && !valid_tx(cfg->tile_x)))
        return BP_ERR_INVALID_ARG;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev < 1) {
        (void)hipGetLastError();
        return BP_ERR_DEVICE;
    }
    if (cfg->device < 0 || cfg->device >= n_dev) return BP_ERR_INVALID_ARG;
    bp_ctx ctx = new (std::nothrow) bp_ctx_s();
    if (!ctx) return BP_ERR_OUT_OF_MEMORY;
    ctx->cfg = *cfg;
    {
        // set-up of the allocation-free entry point: the scratch array's address on this device
        DeviceGuard g(cfg->device);
        if (!g.ok || bp::noalloc_scratch(cfg->device, &ctx->noalloc) != hipSuccess) {
            (void)hipGetLastError();
            ctx->noalloc = nullptr;  // looked up again at that entry point's first call
        }
    }
    *out = ctx;
    return BP_OK;
}

bp_status bp_destroy(bp_ctx ctx)
{
    if (!ctx) return BP_OK;
    bp_status st = BP_OK;
    {
        DeviceGuard g(ctx->cfg.device);
        if (drain_timing(ctx) != BP_OK) st = BP_ERR_DEVICE;
        for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
        ctx->event_pool.clear();
        if (ctx->d_views || ctx->d_pad || ctx->d_cull || ctx->d_scale || ctx->d_fp || ctx->side) {
            if (hipDeviceSynchronize() != hipSuccess) st = BP_ERR_DEVICE;
            if (ctx->d_views && hipFree(ctx->d_views) != hipSuccess) st = BP_ERR_DEVICE;
            if (ctx->d_pad && hipFree(ctx->d_pad) != hipSuccess) st = BP_ERR_DEVICE;
            if (ctx->d_cull && hipFree(ctx->d_cull) != hipSuccess) st = BP_ERR_DEVICE;
            if (ctx->d_scale && hipFree(ctx->d_scale) != hipSuccess) st = BP_ERR_DEVICE;
            if (ctx->d_fp && hipFree(ctx->d_fp) != hipSuccess) st = BP_ERR_DEVICE;
            if (ctx->side) {
                for (hipEvent_t e : {ctx->ev_start, ctx->ev_staged[0], ctx->ev_staged[1], ctx->ev_done[0],
                                     ctx->ev_done[1]})
                    (void)hipEventDestroy(e);
                if (hipStreamDestroy(ctx->side) != hipSuccess) st = BP_ERR_DEVICE;
            }
        }
    }
    delete ctx;
    return st;
}

bp_status bp_set_tuning(bp_ctx ctx, bp_path path, int views_per_pass, int z_unroll, int tile_x)
{
    if (!ctx) return BP_ERR_INVALID_ARG;
    if (path != BP_PATH_AUTO && path != BP_PATH_PLAIN && path != BP_PATH_FUSED && path != BP_PATH_FUSED_DIRECT)
        return fail(ctx, BP_ERR_INVALID_ARG, "unknown path");
    if (views_per_pass < 0) return fail(ctx, BP_ERR_INVALID_ARG, "views_per_pass < 0");
    if (z_unroll != 0 && !valid_zu(z_unroll)) return fail(ctx, BP_ERR_INVALID_ARG, "z_unroll not in {1,2,4,8}");
    if (tile_x != 0 && !valid_tx(tile_x)) return fail(ctx, BP_ERR_INVALID_ARG, "tile_x not in {8,16,32,64}");
    ctx->path_override = path;
    ctx->k_override = views_per_pass;
    ctx->zu_override = z_unroll;
    ctx->tx_override = tile_x;
    return BP_OK;
}

bp_status bp_set_tap_split(bp_ctx ctx, int direct_eighths)
{
    if (!ctx) return BP_ERR_INVALID_ARG;
    if (direct_eighths < -1 || direct_eighths > 8) return fail(ctx, BP_ERR_INVALID_ARG, "tap split not in -1..8");
    ctx->tap_split = direct_eighths;
    return BP_OK;
}

bp_status bp_query_plan(bp_ctx ctx, int nx, int ny, int nz, int n_views, bp_path* path, int* views_per_pass,
                        int* z_unroll, int* tile_x, int* direct_taps)
{
    if (!ctx || nx < 1 || ny < 1 || nz < 1 || n_views < 1) return BP_ERR_INVALID_ARG;
    const Plan p = plan_for(ctx, nx, ny, nz, n_views);
    if (path) *path = p.path;
    if (views_per_pass) *views_per_pass = p.k;
    if (z_unroll) *z_unroll = p.zu;
    if (tile_x) *tile_x = p.tx;
    if (direct_taps) *direct_taps = p.direct_taps ? 1 : 0;
    return BP_OK;
}

bp_status bp_query_scratch(bp_ctx ctx, int nx, int ny, int nz, int n_views, size_t* bytes)
{
    if (!ctx || !bytes || nx < 1 || ny < 1 || nz < 1 || n_views < 1) return BP_ERR_INVALID_ARG;
    *bytes = call_shape(ctx, nx, ny, nz, n_views).total();
    return BP_OK;
}

bp_status bp_set_options(bp_ctx ctx, int options)
{
    if (!ctx) return BP_ERR_INVALID_ARG;
    if (options & ~(BP_OPT_NO_CULL | BP_OPT_NO_COLUMN | BP_OPT_XCD_ORDER | BP_OPT_WIDE_STAGING | BP_OPT_PLAIN_ORDER |
                    BP_OPT_XCD_REGION_MASK | BP_OPT_DIRECT_TAPS | BP_OPT_SERIAL_STAGING | BP_OPT_OVERLAP_STAGING |
                    BP_OPT_STAGE_RECORDS | BP_OPT_POISON_STAGING | BP_OPT_SINGLE_TAPS | BP_OPT_COMPACT_STAGING))
        return fail(ctx, BP_ERR_INVALID_ARG, "unknown option bits");
    const int ax = (options & BP_OPT_XCD_REGION_MASK) >> BP_OPT_XCD_REGION_SHIFT;
    if (ax != 0 && ax != 1 && ax != 2 && ax != 4 && ax != 8)
        return fail(ctx, BP_ERR_INVALID_ARG, "XCD region split must be 1, 2, 4 or 8 along x");
    if ((options & BP_OPT_SERIAL_STAGING) && (options & BP_OPT_OVERLAP_STAGING))
        return fail(ctx, BP_ERR_INVALID_ARG, "staging cannot be both serial and overlapped");
    if ((options & BP_OPT_COMPACT_STAGING) && (options & BP_OPT_WIDE_STAGING))
        return fail(ctx, BP_ERR_INVALID_ARG, "staging cannot be both compact and wide");
    ctx->options = options;
    return BP_OK;
}

bp_status bp_enable_timing(bp_ctx ctx, int enable)
{
    if (!ctx) return BP_ERR_INVALID_ARG;
    DeviceGuard g(ctx->cfg.device);
    const bp_status st = drain_timing(ctx);
    for (int k = 0; k < 3; ++k) {
        ctx->total_ms[k] = 0.0;
        ctx->launches[k] = 0;
    }
    ctx->timing = enable != 0;
    return st;
}

bp_status bp_kernel_timing(bp_ctx ctx, int kind, double* total_ms, long long* launches)
{
    if (!ctx || kind < 0 || kind > 2) return BP_ERR_INVALID_ARG;
    DeviceGuard g(ctx->cfg.device);
    const bp_status st = drain_timing(ctx);
    if (total_ms) *total_ms = ctx->total_ms[kind];
    if (launches) *launches = ctx->launches[kind];
    return st != BP_OK ? fail(ctx, st, "timing events failed") : BP_OK;
}

bp_status bp_backproject_box(bp_ctx ctx, float* volume, int nx, int ny, int nz, const void* projections,
                             const float* matrices, int n_views, float voxel_size, const float origin[3],
                             void* stream)
{
    if (!ctx) return BP_ERR_INVALID_ARG;
    if (const bp_status st = check_call(ctx, volume, nx, ny, nz, projections, matrices, n_views, voxel_size, origin))
        return st;

    const int W = ctx->cfg.det_width, H = ctx->cfg.det_height;
    const CallShape cs = call_shape(ctx, nx, ny, nz, n_views);
    const Plan& plan = cs.plan;
    const bp::Box box{nx, ny, nz, voxel_size, origin[0], origin[1], origin[2]};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const bp::Dtype dt = to_dt(ctx->cfg.proj_dtype);

    DeviceGuard g(ctx->cfg.device);
    if (!g.ok) return fail(ctx, BP_ERR_DEVICE, "cannot select the context's device");

    const bp::Layout layout = cs.layout;
    const bool lds = cs.lds, culled = cs.culled, staged = cs.staged, raw_stage = cs.raw_stage, overlap = cs.overlap;
    const int split = cs.split, words = cs.words;
    const size_t pad_half = cs.pad_half, fp_half = cs.fp_half, scale_half = cs.scale_half;
    const bool poison = (ctx->options & BP_OPT_POISON_STAGING) != 0;
    if (poison && lds && plan.zu != 8)
        return fail(ctx, BP_ERR_UNSUPPORTED, "poisoned staging runs the LDS pass with z_unroll 8 only");

    // all scratch first: a call that fails here has enqueued nothing
    bp_status st = ensure(ctx, reinterpret_cast<void**>(&ctx->d_views), &ctx->views_cap, cs.views_bytes,
                          "view constants");
    if (st != BP_OK) return st;
    if (cs.pad_bytes) {
        st = ensure(ctx, &ctx->d_pad, &ctx->pad_cap, cs.pad_bytes, "staged projections");
        if (st != BP_OK) return st;
    }
    if (cs.scale_bytes) {
        st = ensure(ctx, &ctx->d_scale, &ctx->scale_cap, cs.scale_bytes, "staging scales");
        if (st != BP_OK) return st;
    }
    if (cs.cull_bytes) {
        st = ensure(ctx, &ctx->d_cull, &ctx->cull_cap, cs.cull_bytes, "clipping mask");
        if (st != BP_OK) return st;
    }
    if (cs.fp_bytes) {
        st = ensure(ctx, &ctx->d_fp, &ctx->fp_cap, cs.fp_bytes, "footprints");
        if (st != BP_OK) return st;
    }
    if (overlap && ensure_side(ctx) != BP_OK) return fail(ctx, BP_ERR_DEVICE, "cannot create the staging stream");

    const bool column_ok = !(ctx->options & BP_OPT_NO_COLUMN);
    if (timed(ctx, 2, s, [&] { return bp::launch_prep_views(matrices, n_views, box, column_ok, ctx->d_views, s); }) !=
        hipSuccess)
        return fail(ctx, BP_ERR_LAUNCH, "view-constant kernel launch failed");

    // Clipping mask for the fused path: skip bits per (tile, view).
    bp::Cull cull{nullptr, 0, 0};
    if (culled) {
        if (timed(ctx, 2, s, [&] {
                return bp::launch_cull(ctx->d_views, n_views, box, plan.zu, plan.tx, W, H, (uint32_t*)ctx->d_cull, s);
            }) != hipSuccess)
            return fail(ctx, BP_ERR_LAUNCH, "clipping-mask kernel launch failed");
        cull.bits = (const uint32_t*)ctx->d_cull;
        cull.words = words;
    }

    const size_t img_bytes = (size_t)W * (size_t)H * elem_bytes(ctx->cfg.proj_dtype);
    const int xcd_order = tile_order(ctx);
    // the side stream starts after the view constants (and everything before this call on s)
    const hipStream_t ss = overlap ? ctx->side : s;
    if (overlap && (hipEventRecord(ctx->ev_start, s) != hipSuccess || hipStreamWaitEvent(ss, ctx->ev_start, 0) != hipSuccess))
        return fail(ctx, BP_ERR_LAUNCH, "cannot order the staging stream after the caller's stream");
    for (int k0 = 0, pass = 0; k0 < n_views; k0 += plan.k, ++pass) {
        const int kc = n_views - k0 < plan.k ? n_views - k0 : plan.k;
        const int half = overlap ? (pass & 1) : 0;
        const void* src_views = static_cast<const uint8_t*>(projections) + (size_t)k0 * img_bytes;
        cull.kbase = k0;
        hipError_t e;
        if (staged) {
            void* pad = static_cast<uint8_t*>(ctx->d_pad) + (size_t)half * pad_half;
            uint32_t* maxabs = ctx->d_scale ? (uint32_t*)(static_cast<uint8_t*>(ctx->d_scale) + half * scale_half) : nullptr;
            float* inv_scale = maxabs ? (float*)maxabs + plan.k : nullptr;
            uint2* fp = lds ? static_cast<uint2*>(ctx->d_fp) + (size_t)half * fp_half : nullptr;
            // this half was last read by the pass two before
            if (overlap && pass >= 2 && hipStreamWaitEvent(ss, ctx->ev_done[half], 0) != hipSuccess)
                return fail(ctx, BP_ERR_LAUNCH, "cannot order the staging stream");
            if (poison) {  // testing aid: records no view of the pass writes stay NaN
                e = bp::launch_fill(pad, pad_half, bp::kPoisonPattern, ss);
                if (e != hipSuccess) return fail(ctx, BP_ERR_LAUNCH, std::string("fill kernel: ") + hipGetErrorString(e));
            }
            // Footprints first: with pixel stages they flag the views whose records are read at all
            // (the scale scratch holds the pass's flags), and only those are staged as records.
            bp::ViewNeed need;
            if (raw_stage) {
                need.vc = ctx->d_views + k0;
                need.big = maxabs;
                need.direct_eighths = split;
                e = timed(ctx, 2, ss, [&] { return bp::launch_zero(maxabs, kc, ss); });
                if (e != hipSuccess) return fail(ctx, BP_ERR_LAUNCH, std::string("fill kernel: ") + hipGetErrorString(e));
            }
            if (lds) {
                e = timed(ctx, 2, ss, [&] {
                    return bp::launch_footprint(ctx->d_views + k0, kc, box, plan.zu, plan.tx, W, H, raw_stage,
                                                split, fp, raw_stage ? maxabs : nullptr, ss);
                });
                if (e != hipSuccess)
                    return fail(ctx, BP_ERR_LAUNCH, std::string("footprint kernel: ") + hipGetErrorString(e));
            }
            e = timed(ctx, 1, ss, [&] {
                return layout == bp::Layout::Patch16
                           ? bp::launch_patch16(dt, src_views, W, H, kc, pad, maxabs, inv_scale, ss)
                           : bp::launch_patch(dt, src_views, W, H, kc, pad, need, ss);
            });
            if (e != hipSuccess) return fail(ctx, BP_ERR_LAUNCH, std::string("staging kernel: ") + hipGetErrorString(e));
            if (overlap && (hipEventRecord(ctx->ev_staged[half], ss) != hipSuccess ||
                            hipStreamWaitEvent(s, ctx->ev_staged[half], 0) != hipSuccess))
                return fail(ctx, BP_ERR_LAUNCH, "cannot order the pass after its staging");
            e = timed(ctx, 0, s, [&] {
                return bp::launch_backproject(dt, layout, plan.zu, plan.tx, volume, box, ctx->d_views + k0, kc,
                                              pad, W, H, cull, xcd_order, inv_scale, fp,
                                              raw_stage ? src_views : nullptr, s, poison && lds);
            });
            if (e == hipSuccess && overlap && hipEventRecord(ctx->ev_done[half], s) != hipSuccess)
                return fail(ctx, BP_ERR_LAUNCH, "cannot record the end of a pass");
        } else {
            e = timed(ctx, 0, s, [&] {
                return bp::launch_backproject(dt, layout, plan.zu, plan.tx, volume, box, ctx->d_views + k0, kc,
                                              src_views, W, H, cull, xcd_order, nullptr, nullptr, nullptr, s, false,
                                              (ctx->options & BP_OPT_SINGLE_TAPS) != 0);
            });
        }
        if (e != hipSuccess)
            return fail(ctx, BP_ERR_LAUNCH, std::string("back-projection kernel: ") + hipGetErrorString(e));
    }
    return BP_OK;
}

bp_status bp_backproject_noalloc(bp_ctx ctx, float* volume, int nx, int ny, int nz, const void* projections,
                                 const float* matrices, int n_views, float voxel_size, const float origin[3],
                                 void* stream)
{
    if (!ctx) return BP_ERR_INVALID_ARG;
    if (const bp_status st = check_call(ctx, volume, nx, ny, nz, projections, matrices, n_views, voxel_size, origin))
        return st;
    const size_t views_bytes = sizeof(bp::ViewConst) * (size_t)n_views;
    if (views_bytes > bp::kNoAllocScratchBytes)
        return fail(ctx, BP_ERR_UNSUPPORTED, "n_views beyond the allocation-free limit of 65536");
    // The caller's images only: plain passes stay plain, every other choice runs the fused pass on
    // the caller's images (no staging copy, so no scratch beyond the view constants and the mask).
    Plan plan = plan_for(ctx, nx, ny, nz, n_views);
    if (plan.path != BP_PATH_PLAIN) {
        plan.path = BP_PATH_FUSED_DIRECT;
        if (plan.tx != 16) plan.tx = 64;
        const int k_set = ctx->k_override > 0 ? ctx->k_override : ctx->cfg.views_per_pass;
        plan.k = k_set > 0 ? (k_set < n_views ? k_set : n_views) : (64 < n_views ? 64 : n_views);
    }
    const int W = ctx->cfg.det_width, H = ctx->cfg.det_height;
    const bp::Box box{nx, ny, nz, voxel_size, origin[0], origin[1], origin[2]};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard g(ctx->cfg.device);
    if (!g.ok) return fail(ctx, BP_ERR_DEVICE, "cannot select the context's device");
    if (!ctx->noalloc && bp::noalloc_scratch(ctx->cfg.device, &ctx->noalloc) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, BP_ERR_DEVICE, "cannot look up the static scratch of this device");
    }
    // scratch: view constants, then (256-byte aligned) the clipping mask when it fits beside them;
    // without it every (tile, view) is computed, which gives the same bits (skipped pairs add 0)
    const size_t mask_off = (views_bytes + 255) & ~size_t(255);
    const int words = bp::cull_words(n_views);
    const size_t mask_bytes = (size_t)bp::n_tiles(nx, ny, nz, plan.zu, plan.tx) * (size_t)words * 4u;
    const bool culled = !(ctx->options & BP_OPT_NO_CULL) && mask_off + mask_bytes <= bp::kNoAllocScratchBytes;
    bp::ViewConst* vc = static_cast<bp::ViewConst*>(ctx->noalloc);
    uint32_t* mask = reinterpret_cast<uint32_t*>(static_cast<unsigned char*>(ctx->noalloc) + mask_off);
    const bool column_ok = !(ctx->options & BP_OPT_NO_COLUMN);
    if (bp::launch_prep_views(matrices, n_views, box, column_ok, vc, s) != hipSuccess)
        return fail(ctx, BP_ERR_LAUNCH, "view-constant kernel launch failed");
    bp::Cull cull{nullptr, 0, 0};
    if (culled) {
        if (bp::launch_cull(vc, n_views, box, plan.zu, plan.tx, W, H, mask, s) != hipSuccess)
            return fail(ctx, BP_ERR_LAUNCH, "clipping-mask kernel launch failed");
        cull.bits = mask;
        cull.words = words;
    }
    const size_t img_bytes = (size_t)W * (size_t)H * elem_bytes(ctx->cfg.proj_dtype);
    const int xcd_order = tile_order(ctx);
    const bp::Dtype dt = to_dt(ctx->cfg.proj_dtype);
    for (int k0 = 0; k0 < n_views; k0 += plan.k) {
        const int kc = n_views - k0 < plan.k ? n_views - k0 : plan.k;
        cull.kbase = k0;
        const void* src = static_cast<const uint8_t*>(projections) + (size_t)k0 * img_bytes;
        const hipError_t e = bp::launch_backproject(dt, bp::Layout::Checked, plan.zu, plan.tx, volume, box, vc + k0, kc,
                                                    src, W, H, cull, xcd_order, nullptr, nullptr, nullptr, s, false,
                                                    (ctx->options & BP_OPT_SINGLE_TAPS) != 0);
        if (e != hipSuccess)
            return fail(ctx, BP_ERR_LAUNCH, std::string("back-projection kernel: ") + hipGetErrorString(e));
    }
    return BP_OK;
}

bp_status bp_backproject(bp_ctx ctx, float* volume, const void* projections, const float* matrices, int n_views,
                         int L, float voxel_size, const float origin[3], void* stream)
{
    if (!ctx) return BP_ERR_INVALID_ARG;
    if (L < 1) return fail(ctx, BP_ERR_INVALID_ARG, "L must be >= 1");
    if ((uint64_t)L * L * L >= ((uint64_t)1 << 31)) return fail(ctx, BP_ERR_INVALID_ARG, "L^3 must be < 2^31");
    return bp_backproject_box(ctx, volume, L, L, L, projections, matrices, n_views, voxel_size, origin, stream);
}

}  // extern "C"
