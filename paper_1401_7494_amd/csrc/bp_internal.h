// bp_internal.h -- launchers shared between the C ABI (bp_api.cpp) and the
// HIP kernels (bp_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace bp {

// Per-view constants, one 64-byte record per view, read with scalar loads.
struct ViewConst {
    float p[12];  // P_k row-major
    int mode;     // kModeGuarded, kModeSafe or kModeColumn
    int pad[3];
};
static_assert(sizeof(ViewConst) == 64, "ViewConst must be 64 bytes");

// Branch of a view: guarded (some voxel of the box at w < 1e-4 max w, i.e. at
// or behind the source), safe (every voxel in front: clamped, no tests), or
// column (safe, and u and w do not depend on z).
constexpr int kModeGuarded = 0, kModeSafe = 1, kModeColumn = 2;

// Per-(tile, view) skip bits of a pass (null bits = no culling).
struct Cull {
    const uint32_t* bits;
    int words;  // words per tile row
    int kbase;  // bit index of the pass's first view
};

inline int cull_words(int n_views) { return (n_views + 31) / 32; }

enum class Dtype : int { F32 = 0, F16 = 1, BF16 = 2 };

// Where a back-projection pass reads its taps from.
enum class Layout : int {
    Checked = 0,  // the caller's images, per-tap detector bounds (plain path)
    Patch = 2,    // bilinear-patch staging copy, 16-byte FP32 coefficients per element
    Patch16 = 3   // bilinear-patch staging copy, 8-byte scaled FP16 coefficients per element
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
    if (l == Layout::Patch16) return (size_t)(W + 2) * (size_t)(H + 2) * 8u;
    return 0;
}

// column_ok = false keeps every safe view on the general (per-voxel) branch.
hipError_t launch_prep_views(const float* mats, int n_views, const Box& box, bool column_ok, ViewConst* out,
                             hipStream_t s);

// Bilinear-patch staging copy of views [0, n) of `proj`.
// Which views of a pass need their patch records when the staged footprints hold
// pixels: the views the tap split sends to L1 (k % 8 < direct_eighths), guarded
// views (vc[k].mode), and views with a footprint too large for the stage
// (big[k] != 0, set by launch_footprint).  vc == null: every view.
struct ViewNeed {
    const ViewConst* vc = nullptr;
    const uint32_t* big = nullptr;
    int direct_eighths = 8;
};

hipError_t launch_patch(Dtype dt, const void* proj, int W, int H, int n, void* out, const ViewNeed& need,
                        hipStream_t s);

// Fill n words with 0 (a kernel, so that a captured graph holds no memset node).
hipError_t launch_zero(uint32_t* p, int n, hipStream_t s);

// Compact (FP16, scaled) bilinear-patch staging of views [0, n): per-view
// max |pixel| into maxabs[n] (scratch), 2^-e scale into inv_scale[n].
hipError_t launch_patch16(Dtype dt, const void* proj, int W, int H, int n, void* out, uint32_t* maxabs,
                          float* inv_scale, hipStream_t s);

// One volume pass over views [0, n) of the given view constants; `src` is the
// caller's images (Layout::Checked) or the staging copy of that layout.
// tile_x: columns along x per block (64, 32, 16 or 8; the plain path takes
// 16 or 64); a block covers tile_x x (256 / tile_x)
// columns.  xcd_order: deal contiguous z-ranges of tiles to the 8 XCDs.
// footprints (patch layouts only; null = read the taps directly): the pass's
// footprint table from launch_footprint, [tile][view] -- the taps are then
// staged through LDS.  raw (Layout::Patch with footprints only; else null): the
// caller's images of the pass (of type dt), [n][H][W] -- staged footprints are then
// copied into LDS as FP32 pixels (footprint table made with raw = true).  poison (LDS-staged passes
// with z_unroll 8 only): fill the LDS stage with NaN before each staged footprint (testing aid).
// single_taps (caller's FP32 images): one dword load per tap instead of one 8-byte load per
// pixel pair.
hipError_t launch_backproject(Dtype dt, Layout layout, int z_unroll, int tile_x, float* vol, const Box& box,
                              const ViewConst* vc, int n, const void* src, int W, int H,
                              const Cull& cull, int xcd_order, const float* inv_scale, const uint2* footprints,
                              const void* raw, hipStream_t s, bool poison = false, bool single_taps = false);

// Fill `bytes` (a multiple of 4) with copies of a 32-bit word (a kernel, not a memset node).
hipError_t launch_fill(void* p, size_t bytes, uint32_t word, hipStream_t s);
// The NaN pattern of the poisoned staging (a quiet NaN as FP32 and as each FP16 half).
constexpr uint32_t kPoisonPattern = 0x7FC07FC0u;

// Patch records a block of the staged pass holds one view's footprint in (LDS):
// footprints of up to 64 columns by 32 rows.
constexpr int kStageRecords = 2048;
// Footprint table entries {x, y}: y == kFootprintSkip -> the tile misses the
// detector in that view; y == kFootprintDirect -> read that view's taps
// directly (patch records); y == kFootprintPixels (pixel stages only) -> the
// footprint is too large for the stage, read the four pixels of each patch from
// the caller's image; otherwise x = cmin | rmin << 16, y = fw | fh << 16,
// with the kFootprintInner bit set in y when no position needs clamping into
// the footprint (fw < 2^15).
constexpr uint32_t kFootprintSkip = 0u, kFootprintDirect = 0xffffffffu, kFootprintPixels = 0xfffffffeu;
constexpr uint32_t kFootprintInner = 0x8000u, kFootprintWidthMask = 0x7fffu;


// Footprint table of one pass: n views (view constants vc[0, n)), every tile;
// views with k % 8 < direct_eighths are marked to read their taps directly.
// raw: footprints sized for staging FP32 pixels (fw < 64, fh < 36) rather
// than patch records (fw <= 64, fh <= 32, fw fh <= kStageRecords); a larger
// footprint is then marked kFootprintPixels.
// big (may be null; record stages): big[k] = 1 for a view with a footprint too
// large for the stage, whose records are then read directly (big zeroed beforehand).
hipError_t launch_footprint(const ViewConst* vc, int n, const Box& box, int z_unroll, int tile_x, int W, int H,
                            bool raw, int direct_eighths, uint2* out, uint32_t* big, hipStream_t s);

// Tiles of a pass: tile_x x (256 / tile_x) x z_unroll voxels each.
inline long n_tiles(int nx, int ny, int nz, int z_unroll, int tile_x)
{
    const int ty = 256 / tile_x;
    return (long)((nx + tile_x - 1) / tile_x) * ((ny + ty - 1) / ty) * ((nz + z_unroll - 1) / z_unroll);
}

// Device scratch of the allocation-free entry point: a file-scope static array in the kernel
// source, one copy per device, held until the process ends.  Its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and kept; host code passes
// that address, never the array's name.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
constexpr int kNoAllocMaxDevices = 64;
// The device address of the scratch array on the current device (`device` is its ordinal).
hipError_t noalloc_scratch(int device, void** ptr);

// Skip bits for every (tile, view) of a call, cull_words(n_views) words per tile.
hipError_t launch_cull(const ViewConst* vc, int n_views, const Box& box, int z_unroll, int tile_x, int W, int H,
                       uint32_t* out, hipStream_t s);

}  // namespace bp
