// bp_kernels.hip -- gfx950 kernels of the voxel-driven cone-beam back projector.
//
// The computation (Hofmann et al., WPMVP'14, Sec. 4.1, Listing 1), per voxel
// and view: Part 1 maps the voxel centre through the view's 3x4 matrix and
// de-homogenises; Part 2 fetches the four neighbouring pixels, zero off the
// detector; Part 3 blends them bilinearly, weights by 1/w^2 and accumulates.
//
// GPU mapping
//   * One thread owns ZU voxels of one (x, y) column at consecutive z; a
//     wavefront spans 64 consecutive x, so every volume load/store is one
//     coalesced 256-byte row segment.  Voxels stay in registers for all the
//     views of a pass; the volume is read and written once per pass (the
//     8 bytes per voxel update of Sec. 4.2 divided by the views per pass).
//   * View constants are wave-uniform: scalar loads, no VGPRs.
//   * Part 1 hoists the (x, y) terms out of the z loop: u, v, w cost one FMA
//     each per voxel; 1/w is the hardware reciprocal (Sec. 5.1 makes the same
//     substitution on the CPUs).
//   * Part 2 uses buffer loads: 32-bit offsets, and hardware range checks
//     that return 0 past the end of a view instead of faulting.  With the
//     zero-padded staging copy (Sec. 5.1.1) the tap position is clamped into
//     the padded frame and the four taps need no tests; horizontally adjacent
//     taps are fetched together (the pairwise loads of Sec. 6.1).
//   * A view whose matrix puts some voxel of the box behind (or too near) the
//     source plane takes a guarded branch that zeroes such contributions; the
//     branch is uniform per view, decided once per call.

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "bp_internal.h"

namespace bp {

namespace {

constexpr int kWaveX = 64;  // lanes along x
constexpr int kRowsY = 4;   // waves per block, one y row each

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    // raw buffer (stride 0): offsets >= bytes read as 0.  Word 3 = 0x00020000 on gfx9.
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ float u32_as_f32(uint32_t v) { return __builtin_bit_cast(float, v); }

__device__ __forceinline__ float f16_lo(uint32_t v)
{
    return __half2float(__builtin_bit_cast(__half, (unsigned short)(v & 0xffffu)));
}
__device__ __forceinline__ float f16_hi(uint32_t v)
{
    return __half2float(__builtin_bit_cast(__half, (unsigned short)(v >> 16)));
}
__device__ __forceinline__ float bf16_lo(uint32_t v) { return u32_as_f32(v << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t v) { return u32_as_f32(v & 0xffff0000u); }

// ---------------------------------------------------------------------------
// Tap sources.  Each provides, for one view, the four taps around a position.
// ---------------------------------------------------------------------------

// Plain path: the caller's W x H image of T.  Positions are raw detector
// coordinates; a tap off the detector reads 0 (column test in VALU, row test
// by the buffer range check: rows -1 and H fall outside the view's bytes).
template <typename T>
struct CheckedSource {
    static constexpr uint32_t kElem = sizeof(T);
    const uint8_t* base;
    int W, H;

    struct View {
        __amdgpu_buffer_rsrc_t rs;
    };

    __device__ __forceinline__ View view(int k) const
    {
        const uint32_t bytes = (uint32_t)W * (uint32_t)H * kElem;
        return View{make_rsrc(base + (size_t)k * bytes, bytes)};
    }

    __device__ __forceinline__ float tap(const View& v, int idx) const
    {
        const uint32_t off = (uint32_t)idx * kElem;  // negative idx wraps past the end -> 0
        if constexpr (sizeof(T) == 4) {
            return u32_as_f32(__builtin_amdgcn_raw_buffer_load_b32(v.rs, off, 0, 0));
        } else {
            const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(v.rs, off, 0, 0);
            if constexpr (__is_same(T, __half)) return f16_lo(h);
            else return bf16_lo(h);
        }
    }

    // Contribution of one view at (u, v, w); 0 unless w > 0 and the position
    // lies strictly inside (-1, W) x (-1, H).
    __device__ __forceinline__ float contrib(const View& vw, float u, float v, float w) const
    {
        const float r = __builtin_amdgcn_rcpf(w);
        float s = u * r, t = v * r;
        const bool ok = (w > 0.0f) & (s > -1.0f) & (s < (float)W) & (t > -1.0f) & (t < (float)H);
        s = ok ? s : 0.0f;
        t = ok ? t : 0.0f;
        const float fs = floorf(s), ft = floorf(t);
        const int i0 = (int)fs, j0 = (int)ft;
        const float fx = s - fs, fy = t - ft;
        const bool c0 = i0 >= 0, c1 = i0 + 1 < W;
        const int idx = j0 * W + i0;
        const float a = c0 ? tap(vw, idx) : 0.0f;
        const float b = c1 ? tap(vw, idx + 1) : 0.0f;
        const float c = c0 ? tap(vw, idx + W) : 0.0f;
        const float d = c1 ? tap(vw, idx + W + 1) : 0.0f;
        const float top = fmaf(fx, b - a, a);
        const float bot = fmaf(fx, d - c, c);
        const float val = fmaf(fy, bot - top, top);
        return ok ? val * (r * r) : 0.0f;
    }
};

// Fused path: zero-padded staging copy, (W + 3) x (H + 3) elements of 4 bytes;
// pixel (i, j) sits at element (j + 1) * pitch + (i + 1).  Element types:
//   Dtype::F32  -> one float per element; a dword pair load fetches two columns.
//   Dtype::F16/BF16 -> a packed pair (pixel i, pixel i+1) per element.
template <Dtype DT>
struct PaddedSource {
    const uint8_t* base;
    int W, H;

    struct View {
        __amdgpu_buffer_rsrc_t rs;
    };

    __device__ __forceinline__ int pitch() const { return W + 3; }

    __device__ __forceinline__ View view(int k) const
    {
        const uint32_t bytes = (uint32_t)(W + 3) * (uint32_t)(H + 3) * 4u;
        return View{make_rsrc(base + (size_t)k * bytes, bytes)};
    }

    __device__ __forceinline__ void taps(const View& vw, int i0, int j0, float& a, float& b,
                                         float& c, float& d) const
    {
        const uint32_t pitch_b = (uint32_t)pitch() * 4u;
        const uint32_t off = (__umul24((uint32_t)j0, (uint32_t)pitch()) + (uint32_t)i0) * 4u;
        if constexpr (DT == Dtype::F32) {
            const auto r0 = __builtin_amdgcn_raw_buffer_load_b64(vw.rs, off, 0, 0);
            const auto r1 = __builtin_amdgcn_raw_buffer_load_b64(vw.rs, off, pitch_b, 0);
            a = u32_as_f32(r0[0]);
            b = u32_as_f32(r0[1]);
            c = u32_as_f32(r1[0]);
            d = u32_as_f32(r1[1]);
        } else {
            const uint32_t p0 = __builtin_amdgcn_raw_buffer_load_b32(vw.rs, off, 0, 0);
            const uint32_t p1 = __builtin_amdgcn_raw_buffer_load_b32(vw.rs, off, pitch_b, 0);
            if constexpr (DT == Dtype::F16) {
                a = f16_lo(p0); b = f16_hi(p0); c = f16_lo(p1); d = f16_hi(p1);
            } else {
                a = bf16_lo(p0); b = bf16_hi(p0); c = bf16_lo(p1); d = bf16_hi(p1);
            }
        }
    }

    // Every voxel of the box has w >= 1e-4 * max w > 0: clamp the padded
    // position into [0, W+1] x [0, H+1]; clamped positions see only pad zeros
    // (or carry zero weight), exactly as the unbounded image would.
    __device__ __forceinline__ float contrib_safe(const View& vw, float u, float v, float w) const
    {
        const float r = __builtin_amdgcn_rcpf(w);
        const float s = __builtin_amdgcn_fmed3f(fmaf(u, r, 1.0f), 0.0f, (float)(W + 1));
        const float t = __builtin_amdgcn_fmed3f(fmaf(v, r, 1.0f), 0.0f, (float)(H + 1));
        const int i0 = (int)s, j0 = (int)t;  // s, t >= 0: truncation is floor
        const float fx = __builtin_amdgcn_fractf(s);
        const float fy = __builtin_amdgcn_fractf(t);
        float a, b, c, d;
        taps(vw, i0, j0, a, b, c, d);
        const float top = fmaf(fx, b - a, a);
        const float bot = fmaf(fx, d - c, c);
        const float val = fmaf(fy, bot - top, top);
        return val * (r * r);
    }

    // General view: contributions are 0 unless w > 0 and the position is
    // strictly inside (-1, W) x (-1, H), i.e. (0, W+1) x (0, H+1) padded.
    __device__ __forceinline__ float contrib_guarded(const View& vw, float u, float v, float w) const
    {
        const float r = __builtin_amdgcn_rcpf(w);
        float s = fmaf(u, r, 1.0f), t = fmaf(v, r, 1.0f);
        const bool ok = (w > 0.0f) & (s > 0.0f) & (s < (float)(W + 1)) & (t > 0.0f) &
                        (t < (float)(H + 1));
        s = ok ? s : 0.0f;
        t = ok ? t : 0.0f;
        const int i0 = (int)s, j0 = (int)t;
        const float fx = __builtin_amdgcn_fractf(s);
        const float fy = __builtin_amdgcn_fractf(t);
        float a, b, c, d;
        taps(vw, i0, j0, a, b, c, d);
        const float top = fmaf(fx, b - a, a);
        const float bot = fmaf(fx, d - c, c);
        const float val = fmaf(fy, bot - top, top);
        return ok ? val * (r * r) : 0.0f;
    }
};

// Fused path, bilinear-patch layout: element (r, c) of a (H + 2) x (W + 2) grid
// holds the four coefficients of the bilinear patch whose corners are the
// zero-padded pixels (r, c), (r, c+1), (r+1, c), (r+1, c+1) -- padded pixel
// (r, c) is detector pixel (c - 1, r - 1):
//     a = P(r,c), dx = P(r,c+1) - a, dy = P(r+1,c) - a, dxy = P(r+1,c+1) - P(r+1,c) - dx
// so B = a + fx dx + fy (dy + fx dxy): one 16-byte load and three FMAs per
// voxel update instead of four taps and three lerps.  The coefficients are
// FP32 whatever the storage type of the projections.
typedef int i32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Indexed buffer load: address = base + vindex * stride; vindex >= num_records reads 0.
__device__ f32x4_t struct_buffer_load_f32x4(i32x4_t rsrc, int vindex, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.buffer.load.v4f32");

struct PatchSource {
    const uint8_t* base;
    int W, H;

    struct View {
        i32x4_t rs;
    };

    __device__ __forceinline__ int cols() const { return W + 2; }

    __device__ __forceinline__ View view(int k) const
    {
        const uint32_t n = (uint32_t)(W + 2) * (uint32_t)(H + 2);
        const uint64_t a = (uint64_t)(base + (size_t)k * n * 16u);
        View v;
        v.rs.x = (int)(uint32_t)a;
        v.rs.y = (int)((uint32_t)(a >> 32) & 0xffffu) | (16 << 16);  // stride 16 bytes
        v.rs.z = (int)n;                                             // records
        v.rs.w = 0x00020000;
        return v;
    }

    __device__ __forceinline__ float patch(const View& vw, float s, float t) const
    {
        const int c0 = (int)s, r0 = (int)t;  // s, t >= 0 here: truncation is floor
        const float fx = __builtin_amdgcn_fractf(s);
        const float fy = __builtin_amdgcn_fractf(t);
        const f32x4_t q = struct_buffer_load_f32x4(vw.rs, __mul24(r0, cols()) + c0, 0, 0, 0);
        return fmaf(fx, q.y, fmaf(fy, fmaf(fx, q.w, q.z), q.x));
    }

    // See PaddedSource::contrib_safe: positions clamped into [0, W+1] x [0, H+1].
    __device__ __forceinline__ float contrib_safe(const View& vw, float u, float v, float w) const
    {
        const float r = __builtin_amdgcn_rcpf(w);
        const float s = __builtin_amdgcn_fmed3f(fmaf(u, r, 1.0f), 0.0f, (float)(W + 1));
        const float t = __builtin_amdgcn_fmed3f(fmaf(v, r, 1.0f), 0.0f, (float)(H + 1));
        return patch(vw, s, t) * (r * r);
    }

    __device__ __forceinline__ float contrib_guarded(const View& vw, float u, float v, float w) const
    {
        const float r = __builtin_amdgcn_rcpf(w);
        float s = fmaf(u, r, 1.0f), t = fmaf(v, r, 1.0f);
        const bool ok = (w > 0.0f) & (s > 0.0f) & (s < (float)(W + 1)) & (t > 0.0f) &
                        (t < (float)(H + 1));
        s = ok ? s : 0.0f;
        t = ok ? t : 0.0f;
        const float val = patch(vw, s, t);
        return ok ? val * (r * r) : 0.0f;
    }
};

// ---------------------------------------------------------------------------
// The back-projection pass.
// ---------------------------------------------------------------------------

template <class Src, int ZU, bool PADDED>
__global__ __launch_bounds__(kWaveX* kRowsY) void backproject_kernel(
    float* __restrict__ vol, Box box, const ViewConst* __restrict__ vc, int n_views, Src src)
{
    int x = (int)blockIdx.x * kWaveX + (int)threadIdx.x;
    int y = (int)blockIdx.y * kRowsY + (int)threadIdx.y;
    const int z0 = (int)blockIdx.z * ZU;
    const bool in_xy = (x < box.nx) & (y < box.ny);
    // Lanes past a ragged edge compute a valid voxel of the box and store nothing.
    x = min(x, box.nx - 1);
    y = min(y, box.ny - 1);
    const float X = fmaf(box.vs, (float)x, box.ox);
    const float Y = fmaf(box.vs, (float)y, box.oy);
    float Z[ZU], acc[ZU];
#pragma unroll
    for (int i = 0; i < ZU; ++i) {
        Z[i] = fmaf(box.vs, (float)min(z0 + i, box.nz - 1), box.oz);
        acc[i] = 0.0f;
    }

    for (int k = 0; k < n_views; ++k) {
        const ViewConst& c = vc[k];
        const auto view = src.view(k);
        const float uxy = fmaf(c.p[1], Y, fmaf(c.p[0], X, c.p[3]));
        const float vxy = fmaf(c.p[5], Y, fmaf(c.p[4], X, c.p[7]));
        const float wxy = fmaf(c.p[9], Y, fmaf(c.p[8], X, c.p[11]));
        if constexpr (PADDED) {
            if (c.safe) {
#pragma unroll
                for (int i = 0; i < ZU; ++i)
                    acc[i] += src.contrib_safe(view, fmaf(c.p[2], Z[i], uxy),
                                               fmaf(c.p[6], Z[i], vxy), fmaf(c.p[10], Z[i], wxy));
            } else {
#pragma unroll
                for (int i = 0; i < ZU; ++i)
                    acc[i] += src.contrib_guarded(view, fmaf(c.p[2], Z[i], uxy),
                                                  fmaf(c.p[6], Z[i], vxy), fmaf(c.p[10], Z[i], wxy));
            }
        } else {
#pragma unroll
            for (int i = 0; i < ZU; ++i)
                acc[i] += src.contrib(view, fmaf(c.p[2], Z[i], uxy), fmaf(c.p[6], Z[i], vxy),
                                      fmaf(c.p[10], Z[i], wxy));
        }
    }

    if (in_xy) {
        const size_t plane = (size_t)box.nx * (size_t)box.ny;
        const size_t col = (size_t)y * box.nx + x;
#pragma unroll
        for (int i = 0; i < ZU; ++i) {
            if (z0 + i < box.nz) {
                float* p = vol + (size_t)(z0 + i) * plane + col;
                *p += acc[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Per-view constants: copy P_k and decide whether the view is "safe" (every
// voxel centre of the box in front of the source by a margin).  w is affine,
// so its extremes over the box are at the 8 corner voxels; evaluated in FP64.
// ---------------------------------------------------------------------------
__global__ void prep_views_kernel(const float* __restrict__ mats, int n_views, Box box,
                                  ViewConst* __restrict__ out)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n_views) return;
    ViewConst c;
#pragma unroll
    for (int i = 0; i < 12; ++i) c.p[i] = mats[12 * k + i];
    const double lo[3] = {box.ox, box.oy, box.oz};
    const double hi[3] = {box.ox + (double)box.vs * (box.nx - 1), box.oy + (double)box.vs * (box.ny - 1),
                          box.oz + (double)box.vs * (box.nz - 1)};
    double wmin = 0.0, wmax = 0.0;
    for (int q = 0; q < 8; ++q) {
        const double X = (q & 1) ? hi[0] : lo[0];
        const double Y = (q & 2) ? hi[1] : lo[1];
        const double Z = (q & 4) ? hi[2] : lo[2];
        const double w = (double)c.p[8] * X + (double)c.p[9] * Y + (double)c.p[10] * Z + (double)c.p[11];
        wmin = q ? fmin(wmin, w) : w;
        wmax = q ? fmax(wmax, w) : w;
    }
    c.safe = (wmin > 0.0 && wmin >= 1e-4 * wmax) ? 1 : 0;  // false for NaN
    c.pad[0] = c.pad[1] = c.pad[2] = 0;
    out[k] = c;
}

// ---------------------------------------------------------------------------
// Zero-padded staging copy (Sec. 5.1.1): one thread per padded element.
// ---------------------------------------------------------------------------
template <Dtype DT>
__global__ __launch_bounds__(256) void pad_kernel(const void* __restrict__ proj, int W, int H,
                                                  uint32_t* __restrict__ out)
{
    const int Wp = W + 3, Hp = H + 3;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int r = (int)blockIdx.y;
    const int k = (int)blockIdx.z;
    if (c >= Wp || r >= Hp) return;
    const int i = c - 1, j = r - 1;
    const bool row_ok = (j >= 0) & (j < H);
    uint32_t v = 0;
    if constexpr (DT == Dtype::F32) {
        const float* img = (const float*)proj + (size_t)k * W * H;
        if (row_ok && i >= 0 && i < W) v = __builtin_bit_cast(uint32_t, img[(size_t)j * W + i]);
    } else {
        const uint16_t* img = (const uint16_t*)proj + (size_t)k * W * H;
        uint32_t lo = 0, hi = 0;
        if (row_ok && i >= 0 && i < W) lo = img[(size_t)j * W + i];
        if (row_ok && i + 1 >= 0 && i + 1 < W) hi = img[(size_t)j * W + i + 1];
        v = lo | (hi << 16);
    }
    out[((size_t)k * Hp + r) * Wp + c] = v;
}

template <typename T>
__device__ __forceinline__ float pixel_f32(const T* img, int W, int H, int i, int j)
{
    if (i < 0 || i >= W || j < 0 || j >= H) return 0.0f;
    const T v = img[(size_t)j * W + i];
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(float, v);
    else if constexpr (__is_same(T, __half)) return __half2float(v);
    else return __builtin_bit_cast(float, (uint32_t)v << 16);
}

// Bilinear-patch staging copy: one thread per patch (r, c) of a (H+2) x (W+2) grid.
template <typename T>
__global__ __launch_bounds__(256) void patch_kernel(const T* __restrict__ proj, int W, int H,
                                                    f32x4_t* __restrict__ out)
{
    const int Wq = W + 2, Hq = H + 2;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int r = (int)blockIdx.y;
    const int k = (int)blockIdx.z;
    if (c >= Wq || r >= Hq) return;
    const T* img = proj + (size_t)k * W * H;
    const int i = c - 1, j = r - 1;  // detector pixel of the patch's first corner
    const float a = pixel_f32(img, W, H, i, j);
    const float b = pixel_f32(img, W, H, i + 1, j);
    const float cc = pixel_f32(img, W, H, i, j + 1);
    const float d = pixel_f32(img, W, H, i + 1, j + 1);
    const float dx = b - a;
    f32x4_t q;
    q.x = a;
    q.y = dx;
    q.z = cc - a;
    q.w = (d - cc) - dx;
    out[((size_t)k * Hq + r) * Wq + c] = q;
}

template <class Src, bool PADDED>
hipError_t launch_zu(int zu, float* vol, const Box& box, const ViewConst* vc, int n, const Src& src,
                     hipStream_t s)
{
    const dim3 block(kWaveX, kRowsY, 1);
    auto grid = [&](int z) {
        return dim3((unsigned)((box.nx + kWaveX - 1) / kWaveX), (unsigned)((box.ny + kRowsY - 1) / kRowsY),
                    (unsigned)((box.nz + z - 1) / z));
    };
    switch (zu) {
    case 1: hipLaunchKernelGGL((backproject_kernel<Src, 1, PADDED>), grid(1), block, 0, s, vol, box, vc, n, src); break;
    case 2: hipLaunchKernelGGL((backproject_kernel<Src, 2, PADDED>), grid(2), block, 0, s, vol, box, vc, n, src); break;
    case 4: hipLaunchKernelGGL((backproject_kernel<Src, 4, PADDED>), grid(4), block, 0, s, vol, box, vc, n, src); break;
    case 8: hipLaunchKernelGGL((backproject_kernel<Src, 8, PADDED>), grid(8), block, 0, s, vol, box, vc, n, src); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_prep_views(const float* mats, int n_views, const Box& box, ViewConst* out, hipStream_t s)
{
    const int threads = 64;
    hipLaunchKernelGGL(prep_views_kernel, dim3((unsigned)((n_views + threads - 1) / threads)), dim3(threads), 0,
                       s, mats, n_views, box, out);
    return hipGetLastError();
}

hipError_t launch_pad(Dtype dt, const void* proj, int W, int H, int n, void* padded, hipStream_t s)
{
    const dim3 block(256, 1, 1);
    const dim3 grid((unsigned)((W + 3 + 255) / 256), (unsigned)(H + 3), (unsigned)n);
    uint32_t* out = (uint32_t*)padded;
    switch (dt) {
    case Dtype::F32: hipLaunchKernelGGL(pad_kernel<Dtype::F32>, grid, block, 0, s, proj, W, H, out); break;
    case Dtype::F16: hipLaunchKernelGGL(pad_kernel<Dtype::F16>, grid, block, 0, s, proj, W, H, out); break;
    case Dtype::BF16: hipLaunchKernelGGL(pad_kernel<Dtype::BF16>, grid, block, 0, s, proj, W, H, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_patch(Dtype dt, const void* proj, int W, int H, int n, void* out, hipStream_t s)
{
    const dim3 block(256, 1, 1);
    const dim3 grid((unsigned)((W + 2 + 255) / 256), (unsigned)(H + 2), (unsigned)n);
    f32x4_t* q = (f32x4_t*)out;
    switch (dt) {
    case Dtype::F32: hipLaunchKernelGGL(patch_kernel<float>, grid, block, 0, s, (const float*)proj, W, H, q); break;
    case Dtype::F16: hipLaunchKernelGGL(patch_kernel<__half>, grid, block, 0, s, (const __half*)proj, W, H, q); break;
    case Dtype::BF16: hipLaunchKernelGGL(patch_kernel<uint16_t>, grid, block, 0, s, (const uint16_t*)proj, W, H, q); break;
    }
    return hipGetLastError();
}

hipError_t launch_backproject(Dtype dt, Layout layout, int zu, float* vol, const Box& box, const ViewConst* vc,
                              int n, const void* src, int W, int H, hipStream_t s)
{
    const uint8_t* base = (const uint8_t*)src;
    if (layout == Layout::Patch) return launch_zu<PatchSource, true>(zu, vol, box, vc, n, {base, W, H}, s);
    if (layout == Layout::Pairs) {
        switch (dt) {
        case Dtype::F32: return launch_zu<PaddedSource<Dtype::F32>, true>(zu, vol, box, vc, n, {base, W, H}, s);
        case Dtype::F16: return launch_zu<PaddedSource<Dtype::F16>, true>(zu, vol, box, vc, n, {base, W, H}, s);
        case Dtype::BF16: return launch_zu<PaddedSource<Dtype::BF16>, true>(zu, vol, box, vc, n, {base, W, H}, s);
        }
    } else {
        switch (dt) {
        case Dtype::F32: return launch_zu<CheckedSource<float>, false>(zu, vol, box, vc, n, {base, W, H}, s);
        case Dtype::F16: return launch_zu<CheckedSource<__half>, false>(zu, vol, box, vc, n, {base, W, H}, s);
        case Dtype::BF16: return launch_zu<CheckedSource<uint16_t>, false>(zu, vol, box, vc, n, {base, W, H}, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace bp
