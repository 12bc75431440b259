// bp_internal.h -- launchers shared between the C ABI (bp_api.cpp) and the
// HIP kernels (bp_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace bp {

// Per-view constants, one 64-byte record per view, read with scalar loads.
struct ViewConst {
    float p[12];  // P_k row-major
    int safe;     // 1: every voxel of the box has w >= 1e-4 * max w > 0
    int pad[3];
};
static_assert(sizeof(ViewConst) == 64, "ViewConst must be 64 bytes");

enum class Dtype : int { F32 = 0, F16 = 1, BF16 = 2 };

// Where a back-projection pass reads its taps from.
enum class Layout : int {
    Checked = 0,  // the caller's images, per-tap detector bounds (plain path)
    Pairs = 1,    // zero-padded staging copy, 4-byte elements (FP32 pixel or 16-bit pair)
    Patch = 2     // bilinear-patch staging copy, 16-byte FP32 coefficients per element
};

struct Box {
    int nx, ny, nz;
    float vs;            // voxel size
    float ox, oy, oz;    // centre of voxel (0,0,0)
};

// Bytes of one staging image of the given layout.
inline size_t staged_view_bytes(Layout l, int W, int H)
{
    if (l == Layout::Patch) return (size_t)(W + 2) * (size_t)(H + 2) * 16u;
    if (l == Layout::Pairs) return (size_t)(W + 3) * (size_t)(H + 3) * 4u;
    return 0;
}

hipError_t launch_prep_views(const float* mats, int n_views, const Box& box, ViewConst* out,
                             hipStream_t s);

// Copy views [0, n) of `proj` (dtype dt, H x W each) into the zero-padded
// staging layout: FP32 -> float per element; FP16/BF16 -> packed pairs
// (pixel i, pixel i+1) per element.
hipError_t launch_pad(Dtype dt, const void* proj, int W, int H, int n, void* padded,
                      hipStream_t s);

// Bilinear-patch staging copy of views [0, n) of `proj`.
hipError_t launch_patch(Dtype dt, const void* proj, int W, int H, int n, void* out, hipStream_t s);

// One volume pass over views [0, n) of the given view constants; `src` is the
// caller's images (Layout::Checked) or the staging copy of that layout.
hipError_t launch_backproject(Dtype dt, Layout layout, int z_unroll, float* vol, const Box& box,
                              const ViewConst* vc, int n, const void* src, int W, int H,
                              hipStream_t s);

}  // namespace bp
