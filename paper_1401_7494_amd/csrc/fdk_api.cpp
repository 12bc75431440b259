// fdk_api.cpp -- the C ABI of the FDK pre-processing (include/bp.h, bp_fdk_*):
// argument validation, the per-handle tables and the launch.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/bp.h"
#include "fdk_internal.h"

struct bp_fdk_s {
    bp_fdk_config cfg;
    std::string last_error;
    double tau = 0.0;           // pixel pitch at the isocentre
    double2* d_tw = nullptr;    // twiddle table, kTransform entries
    double* d_spec = nullptr;   // ramp spectrum, kTransform entries
};

namespace {

bp_status fdk_fail(bp_fdk f, bp_status st, const std::string& msg)
{
    if (f) f->last_error = msg;
    return st;
}

struct FdkDeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit FdkDeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
    }
    ~FdkDeviceGuard()
    {
        if (ok && prev >= 0) (void)hipSetDevice(prev);
    }
};

bool positive_finite(double x) { return std::isfinite(x) && x > 0.0; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace

extern "C" {

void bp_fdk_config_default(bp_fdk_config* cfg)
{
    if (!cfg) return;
    cfg->device = 0;
    cfg->det_width = 1248;
    cfg->det_height = 960;
    cfg->pitch = 0.32;
    cfg->sid = 800.0;
    cfg->sdd = 1200.0;
}

bp_status bp_fdk_create(const bp_fdk_config* cfg, bp_fdk* out)
{
    if (!out) return BP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!cfg) return BP_ERR_INVALID_ARG;
    if (cfg->det_width < 1 || cfg->det_height < 1) return BP_ERR_INVALID_ARG;
    if (!positive_finite(cfg->pitch) || !positive_finite(cfg->sid) || !positive_finite(cfg->sdd))
        return BP_ERR_INVALID_ARG;
    if (cfg->det_width > bp::fdk::kMaxWidth) return BP_ERR_UNSUPPORTED;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || cfg->device < 0 || cfg->device >= n_dev) {
        (void)hipGetLastError();
        return BP_ERR_DEVICE;
    }
    FdkDeviceGuard g(cfg->device);
    if (!g.ok) return BP_ERR_DEVICE;
    bp_fdk f = new bp_fdk_s;
    f->cfg = *cfg;
    f->tau = cfg->pitch * cfg->sid / cfg->sdd;
    const size_t n = bp::fdk::kTransform;
    if (hipMalloc((void**)&f->d_tw, n * sizeof(double2)) != hipSuccess ||
        hipMalloc((void**)&f->d_spec, n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        bp_fdk_destroy(f);
        return BP_ERR_OUT_OF_MEMORY;
    }
    // The tables are built once, on the null stream, and are ready when this returns.
    if (bp::fdk::launch_setup(f->d_tw, f->d_spec, cfg->det_width, f->tau, nullptr) != hipSuccess ||
        hipStreamSynchronize(nullptr) != hipSuccess) {
        (void)hipGetLastError();
        bp_fdk_destroy(f);
        return BP_ERR_LAUNCH;
    }
    *out = f;
    return BP_OK;
}

bp_status bp_fdk_destroy(bp_fdk f)
{
    if (!f) return BP_OK;
    bp_status st = BP_OK;
    {
        FdkDeviceGuard g(f->cfg.device);
        if (f->d_tw || f->d_spec) {
            // Filter calls still in flight read the tables.
            if (hipDeviceSynchronize() != hipSuccess) st = BP_ERR_DEVICE;
            if (f->d_tw && hipFree(f->d_tw) != hipSuccess) st = BP_ERR_DEVICE;
            if (f->d_spec && hipFree(f->d_spec) != hipSuccess) st = BP_ERR_DEVICE;
        }
    }
    delete f;
    return st;
}

const char* bp_fdk_last_error(bp_fdk f) { return f ? f->last_error.c_str() : "null handle"; }

bp_status bp_fdk_filter(bp_fdk f, const float* raw, void* filtered, bp_dtype out_dtype, int n_views, void* stream)
{
    if (!f) return BP_ERR_INVALID_ARG;
    if (!raw || !filtered) return fdk_fail(f, BP_ERR_INVALID_ARG, "null raw or filtered pointer");
    if (n_views < 1) return fdk_fail(f, BP_ERR_INVALID_ARG, "n_views must be >= 1");
    if (out_dtype != BP_F32 && out_dtype != BP_F16 && out_dtype != BP_BF16)
        return fdk_fail(f, BP_ERR_INVALID_ARG, "unknown output dtype");
    const int W = f->cfg.det_width, H = f->cfg.det_height;
    const long long rows = (long long)n_views * H;
    if (rows > ((long long)1 << 32)) return fdk_fail(f, BP_ERR_UNSUPPORTED, "more than 2^32 detector rows");
    const size_t pixels = (size_t)rows * (size_t)W;
    const size_t in_bytes = pixels * 4, out_bytes = pixels * (out_dtype == BP_F32 ? 4 : 2);
    if ((uintptr_t)raw % 4 != 0 || (uintptr_t)filtered % (out_dtype == BP_F32 ? 4 : 2) != 0)
        return fdk_fail(f, BP_ERR_INVALID_ARG, "misaligned raw or filtered pointer");
    const bool in_place = (const void*)raw == filtered && out_dtype == BP_F32;
    if (!in_place && overlaps(raw, in_bytes, filtered, out_bytes))
        return fdk_fail(f, BP_ERR_INVALID_ARG, "filtered overlaps raw (only an FP32 in-place call may alias)");
    FdkDeviceGuard g(f->cfg.device);
    if (!g.ok) return fdk_fail(f, BP_ERR_DEVICE, "cannot select the handle's device");
    bp::fdk::Geometry geo;
    geo.half_w = (W - 1) / 2.0;
    geo.half_h = (H - 1) / 2.0;
    geo.pitch = f->cfg.pitch;
    geo.sdd = f->cfg.sdd;
    geo.sdd2 = f->cfg.sdd * f->cfg.sdd;
    const hipError_t e = bp::fdk::launch_filter(raw, filtered, (int)out_dtype, (long)rows, W, H, geo, f->d_tw,
                                                f->d_spec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fdk_fail(f, BP_ERR_LAUNCH, std::string("FDK filter kernel: ") + hipGetErrorString(e));
    }
    return BP_OK;
}

}  // extern "C"
