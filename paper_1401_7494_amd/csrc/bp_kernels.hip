// bp_kernels.hip -- gfx950 kernels of the voxel-driven cone-beam back projector.
//
// The computation (Hofmann et al., WPMVP'14, Sec. 4.1, Listing 1), per voxel
// and view: Part 1 maps the voxel centre through the view's 3x4 matrix and
// de-homogenises; Part 2 fetches the four neighbouring pixels, zero off the
// detector; Part 3 blends them bilinearly, weights by 1/w^2 and accumulates.
//
// GPU mapping
//   * One thread owns ZU voxels of one (x, y) column at consecutive z; a
//     256-thread block covers TX x (256 / TX) columns (16 x 16 by default), a
//     wavefront TX x (64 / TX) in the passes on the caller's images (so volume
//     loads and stores are whole row segments) and an 8 x 8 quadrant of a
//     16 x 16 tile in the LDS-staged pass (whose volume traffic is 8/K bytes
//     per update).  Voxels stay in registers for all the views of a pass; the
//     volume is read and written once per pass (the 8 bytes per voxel update
//     of Sec. 4.2 divided by the views per pass).
//   * View constants are wave-uniform: scalar loads, no VGPRs.
//   * Part 1 hoists the (x, y) terms out of the z loop: u, v, w cost one FMA
//     each per voxel; 1/w is the hardware reciprocal (Sec. 5.1 makes the same
//     substitution on the CPUs).  For views whose u and w do not depend on z
//     (circular orbits) the column, 1/w and 1/w^2 are formed once per column.
//   * Part 2: the fused pass reads a staging copy of the views in which every
//     pixel carries the four coefficients of its bilinear patch and the
//     detector has a one-pixel zero border (the zero-padded copy of Sec.
//     5.1.1): the position is clamped into the bordered frame, so the taps
//     need no tests, and one 16-byte (8-byte for 16-bit data) record replaces
//     the four taps.  The record comes either from L1 (an indexed buffer
//     load) or from the block tile's footprint staged in LDS -- for FP32
//     input the footprint's pixels, from which an update forms the record;
//     the default pass
//     mixes the two by view.  Footprints with a record of margin inside the
//     detector on every side ("interior") need no clamp at all.  The plain
//     and direct-fused passes read the caller's images with per-tap bounds
//     tests instead (FP32: each row's pixel pair as one 8-byte load).
//   * A view whose matrix puts some voxel of the box behind (or too near) the
//     source plane takes a guarded branch that zeroes such contributions; the
//     branch is uniform per view, decided once per call.

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "bp_internal.h"

namespace bp {

namespace {

constexpr int kBlock = 256;  // threads per block: 4 wavefronts
constexpr int kXcds = 8;     // MI355X: 8 XCDs, consecutive workgroups go to consecutive XCDs
// LDS-staged taps: one footprint row per wave and slot, one column per lane
constexpr int kStageSlots = 8;
constexpr int kStageMaxWidth = 64, kStageMaxHeight = 4 * kStageSlots;
// Slots of a pixel stage: 36 rows, so that footprints of the benchmark geometry never exceed them.
constexpr int kRawSlots = kStageSlots + 1, kRawRows = 4 * kRawSlots;
// FP32 pixels staged for the footprint of fw x fh patches: (fw + 1) x (fh + 1) pixels, at most 64 x 36,
// column-major with an odd column stride: a patch's four pixels are two ds_read2_b32 with immediate
// offsets (0/1 down a column, 37/38 in the next), a wave's row of 64 lanes writes 64 distinct banks,
// and a wave's reads spread over the banks better than with 68-float rows (measured: BF16 +2%, FP32
// +0-1.4%; strides 39, 41, 45, 53 slower).
constexpr int kRawColStride = kRawRows + 1;

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
__device__ __forceinline__ float bf16_lo(uint32_t v) { return u32_as_f32(v << 16); }

// ---------------------------------------------------------------------------
// Tap sources.  Each provides, for one view, the four taps around a position.
// ---------------------------------------------------------------------------

typedef int i32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
// Byte-offset buffer load of two FP32 values (the intrinsic itself: the b64 builtin with its
// elements bit-cast to float compiles to a single dword load here, element 0 used twice).
__device__ f32x2_t raw_buffer_load_f32x2(i32x4_t rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.v2f32");
// Byte-offset buffer load of one dword, at any 2-byte boundary (two 16-bit pixels).
__device__ uint32_t raw_buffer_load_u32(i32x4_t rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.i32");

// Plain path: the caller's W x H image of T.  Positions are raw detector
// coordinates; a tap off the detector reads 0 (row and column tests in VALU;
// every load stays inside the view).  PAIRS: the two taps of one row as one
// load, 8 bytes of FP32 or 4 bytes of FP16/BF16 (W >= 2).
template <typename T, bool PAIRS = false>
struct CheckedSource {
    static constexpr uint32_t kElem = sizeof(T);
    const uint8_t* base;
    int W, H;

    struct View {
        __amdgpu_buffer_rsrc_t rs;  // single taps
        i32x4_t pair_rs;            // pair taps: the same raw buffer
    };

    __device__ __forceinline__ View view(int k) const
    {
        const uint32_t bytes = (uint32_t)W * (uint32_t)H * kElem;
        View v;
        if constexpr (PAIRS) {
            const uint64_t a = (uint64_t)(base + (size_t)k * bytes);
            v.pair_rs.x = (int)(uint32_t)a;
            v.pair_rs.y = (int)((uint32_t)(a >> 32) & 0xffffu);  // stride 0: byte-addressed
            v.pair_rs.z = (int)bytes;
            v.pair_rs.w = 0x00020000;
        } else {
            v.rs = make_rsrc(base + (size_t)k * bytes, bytes);
        }
        return v;
    }

    // the FP32 values of the low and high 16-bit pixels of a dword
    static __device__ __forceinline__ float widen_lo(uint32_t b)
    {
        if constexpr (__is_same(T, __half)) return f16_lo(b);
        else return bf16_lo(b);
    }
    static __device__ __forceinline__ float widen_hi(uint32_t b)
    {
        if constexpr (__is_same(T, __half)) return f16_lo(b >> 16);
        else return u32_as_f32(b & 0xffff0000u);
    }

    __device__ __forceinline__ float tap(const View& v, int idx) const
    {
        const uint32_t off = (uint32_t)idx * kElem;
        if constexpr (sizeof(T) == 4) {
            return u32_as_f32(__builtin_amdgcn_raw_buffer_load_b32(v.rs, off, 0, 0));
        } else {
            const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(v.rs, off, 0, 0);
            if constexpr (__is_same(T, __half)) return f16_lo(h);
            else return bf16_lo(h);
        }
    }

    // The horizontal part of Part 3 at column position i0 + fx: a row's value is
    // (1 - fx) P[i0] + fx P[i0 + 1], pixels off the detector 0.
    //   single taps: the two pixels loaded one each at clamped, in-bounds
    //     indices, zeroed by explicit row and column tests;
    //   PAIRS (W >= 2): the pair at columns c, c + 1, c = i0 clamped into
    //     [0, W - 2], as one load, with per-column weights (w0, w1) of its two
    //     pixels that put (1 - fx) and fx on the right ones and 0 on any other
    //     (column -1 or W, or a pixel of the pair that is not a tap).  A row off the
    //     detector is read at a byte offset outside [0, W H e) -- negative rows as
    //     offsets of 2^32 - k, rows below as offsets past the end, and a pair never
    //     straddles either boundary -- which the buffer's range check returns as 0.
    // Both give fmaf(fx, P[i0 + 1], (1 - fx) P[i0]) with the same roundings.
    struct Col {
        int i0;
        float fx;
        int c_bytes;  // pairs: byte offset of column c in a row
        float w0, w1;
    };

    __device__ __forceinline__ Col col(int i0, float fx) const
    {
        Col k;
        k.i0 = i0;
        k.fx = fx;
        if constexpr (PAIRS) {
            const int c = min(max(i0, 0), W - 2);
            const float g = 1.0f - fx;
            k.c_bytes = c * (int)kElem;
            k.w0 = c == i0 ? g : (c == i0 + 1 ? fx : 0.0f);
            k.w1 = c + 1 == i0 ? g : (c + 1 == i0 + 1 ? fx : 0.0f);
        } else {
            k.c_bytes = 0;
            k.w0 = k.w1 = 0.0f;
        }
        return k;
    }

    // Value of the bilinear interpolant at column k and row position j0 + fy (j0 in [-1, H]).
    __device__ __forceinline__ float value(const View& v, const Col& k, int j0, float fy) const
    {
        float top, bot;
        if constexpr (PAIRS) {
            // both rows' offsets in the VGPR operand: the range check covers that operand only (an
            // SGPR offset is added after it), so a row off the detector must be off in the VGPR
            const int row_b = W * (int)kElem;
            const int off = __mul24(j0, row_b) + k.c_bytes;
            if constexpr (sizeof(T) == 4) {
                const f32x2_t q0 = raw_buffer_load_f32x2(v.pair_rs, off, 0, 0);
                const f32x2_t q1 = raw_buffer_load_f32x2(v.pair_rs, off + row_b, 0, 0);
                top = fmaf(k.w1, q0.y, k.w0 * q0.x);
                bot = fmaf(k.w1, q1.y, k.w0 * q1.x);
            } else {
                // 16-bit pixels: the pair as one dword at a 2-byte boundary, each half widened exactly
                const uint32_t h0 = raw_buffer_load_u32(v.pair_rs, off, 0, 0);
                const uint32_t h1 = raw_buffer_load_u32(v.pair_rs, off + row_b, 0, 0);
                top = fmaf(k.w1, widen_hi(h0), k.w0 * widen_lo(h0));
                bot = fmaf(k.w1, widen_hi(h1), k.w0 * widen_lo(h1));
            }
        } else {
            // i0 in [-1, W] (a clamped column position reaches W)
            const bool c0 = (k.i0 >= 0) & (k.i0 < W), c1 = k.i0 + 1 < W;
            const int ia = min(max(k.i0, 0), W - 1), ib = min(k.i0 + 1, W - 1);
            float p[2][2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = j0 + r;
                const bool rj = (j >= 0) & (j < H);
                const int row = min(max(j, 0), H - 1) * W;
                const float ta = tap(v, row + ia), tb = tap(v, row + ib);
                p[r][0] = (rj & c0) ? ta : 0.0f;
                p[r][1] = (rj & c1) ? tb : 0.0f;
            }
            top = fmaf(k.fx, p[0][1], (1.0f - k.fx) * p[0][0]);
            bot = fmaf(k.fx, p[1][1], (1.0f - k.fx) * p[1][0]);
        }
        return fmaf(fy, bot, (1.0f - fy) * top);
    }

    // Contribution of one view at (u, v, w); 0 unless w > 0 and the position
    // lies strictly inside (-1, W) x (-1, H), each tap 0 off the detector.
    __device__ __forceinline__ float contrib(const View& vw, float u, float v, float w) const
    {
        const float r = __builtin_amdgcn_rcpf(w);
        float s = u * r, t = v * r;
        const bool ok = (w > 0.0f) & (s > -1.0f) & (s < (float)W) & (t > -1.0f) & (t < (float)H);
        s = ok ? s : 0.0f;
        t = ok ? t : 0.0f;
        const float fs = floorf(s), ft = floorf(t);
        const float val = value(vw, col((int)fs, s - fs), (int)ft, t - ft);
        return ok ? val * (r * r) : 0.0f;
    }

    // Column view (u and w do not depend on z, as for a circular orbit about z; w > 0 on the
    // whole box): 1/w and the column are formed once for the thread's ZU voxels, per voxel only
    // the row t(Z) = (v_xy + P[1][2] Z) / w.  Positions are clamped into [-1, W] x [-1, H]: a
    // position at or beyond an edge weighs only pixels off the detector, as the zero-extended
    // image gives (the interpolant is 0 there and continuous across the clamp).
    template <int ZU>
    __device__ __forceinline__ void column(const View& vw, float uxy, float vxy, float wxy, float p12,
                                           const float (&Z)[ZU], float (&acc)[ZU]) const
    {
        const float r = __builtin_amdgcn_rcpf(wxy);
        const float s = __builtin_amdgcn_fmed3f(uxy * r, -1.0f, (float)W);
        const float fs = floorf(s);
        const Col k = col((int)fs, s - fs);
        const float r2 = r * r, dt = p12 * r, tb = vxy * r;
#pragma unroll
        for (int i = 0; i < ZU; ++i) {
            const float t = __builtin_amdgcn_fmed3f(fmaf(Z[i], dt, tb), -1.0f, (float)H);
            const float ft = floorf(t);
            acc[i] = fmaf(value(vw, k, (int)ft, t - ft), r2, acc[i]);
        }
    }
};

// Fused path, bilinear-patch layout: element (r, c) of a (H + 2) x (W + 2) grid
// holds the four coefficients of the bilinear patch whose corners are the
// zero-padded pixels (r, c), (r, c+1), (r+1, c), (r+1, c+1) -- padded pixel
// (r, c) is detector pixel (c - 1, r - 1): the left pixel of each of the two
// rows and its difference to the right one,
//     a = P(r,c), dx = P(r,c+1) - a, c = P(r+1,c), dx' = P(r+1,c+1) - c,
// so the two rows' lerps along x are one FMA each, top = a + fx dx and
// bot = c + fx dx', and B = top + fy (bot - top): one 16-byte load instead of
// four taps, and the same two subtractions and three FMAs whether an update
// forms the coefficients from four pixels or reads them.  The coefficients are
// FP32 whatever the storage type of the projections.
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Indexed buffer load: address = base + vindex * stride; vindex >= num_records reads 0.
__device__ f32x4_t struct_buffer_load_f32x4(i32x4_t rsrc, int vindex, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.buffer.load.v4f32");
// Byte-offset buffer load of one FP32 value; offsets >= num_records read 0.
__device__ float raw_buffer_load_f32(i32x4_t rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.f32");

// med3 clamp of a position into [lo, hi], or the position itself where it is known to lie there.
template <bool CLAMP>
__device__ __forceinline__ float clamp_to(float x, float lo, float hi)
{
    if constexpr (CLAMP) return __builtin_amdgcn_fmed3f(x, lo, hi);
    else return x;
}

struct PatchSource {
    const uint8_t* base;
    int W, H;
    static constexpr bool kRawStage = false;  // staged footprints copy patch records

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

    using Rec = f32x4_t;

    __device__ __forceinline__ Rec load(const View& vw, int idx) const
    {
        return struct_buffer_load_f32x4(vw.rs, idx, 0, 0, 0);
    }

    // Part 3 on one patch: the lerps of the two rows along x, then the lerp between them along y.
    static __device__ __forceinline__ float eval(const Rec& q, float fx, float fy)
    {
        const float top = fmaf(fx, q.y, q.x), bot = fmaf(fx, q.w, q.z);
        return fmaf(fy, bot - top, top);
    }

    // 1/w^2 from r = 1/w: as the column branch and the per-voxel branch form it.
    __device__ __forceinline__ float weight_column(const View&, float r) const { return r * r; }
    __device__ __forceinline__ float weight_voxel(const View&, float r) const { return r * r; }

    // Patch value at padded column c0 + fx, padded row t (t >= 0, so truncation is floor).
    __device__ __forceinline__ float patch_at(const View& vw, int c0, float fx, float t) const
    {
        const int r0 = (int)t;
        const float fy = __builtin_amdgcn_fractf(t);
        return eval(load(vw, __mul24(r0, cols()) + c0), fx, fy);
    }

    __device__ __forceinline__ float patch(const View& vw, float s, float t) const
    {
        return patch_at(vw, (int)s, __builtin_amdgcn_fractf(s), t);
    }

    // Column view (u and w do not depend on z): everything but the row is
    // shared by the ZU voxels of the thread's column.  t(Z) = (v_xy + P[1][2] Z) / w + 1.
    // CLAMP = false: the caller knows every position lies inside the bordered frame (an interior
    // footprint), so the clamps are left out.
    template <int ZU, bool CLAMP = true>
    __device__ __forceinline__ void column(const View& vw, float uxy, float vxy, float wxy, float p12,
                                           const float (&Z)[ZU], float (&acc)[ZU]) const
    {
        const float r = __builtin_amdgcn_rcpf(wxy);
        const float s = clamp_to<CLAMP>(fmaf(uxy, r, 1.0f), 0.0f, (float)(W + 1));
        const int c0 = (int)s;
        const float fx = __builtin_amdgcn_fractf(s);
        const float r2 = r * r;
        const float dt = p12 * r;
        const float tb = fmaf(vxy, r, 1.0f);
#pragma unroll
        for (int i = 0; i < ZU; ++i) {
            const float t = clamp_to<CLAMP>(fmaf(Z[i], dt, tb), 0.0f, (float)(H + 1));
            acc[i] = fmaf(patch_at(vw, c0, fx, t), r2, acc[i]);
        }
    }

    // Safe view (every voxel of the box has w >= 1e-4 * max w > 0): the
    // position is clamped into the bordered frame [0, W+1] x [0, H+1]; a
    // clamped position lands on border patches whose value there is exactly 0,
    // as the zero-extended image would give.
    template <bool CLAMP = true>
    __device__ __forceinline__ float contrib_safe(const View& vw, float u, float v, float w) const
    {
        const float r = __builtin_amdgcn_rcpf(w);
        const float s = clamp_to<CLAMP>(fmaf(u, r, 1.0f), 0.0f, (float)(W + 1));
        const float t = clamp_to<CLAMP>(fmaf(v, r, 1.0f), 0.0f, (float)(H + 1));
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

// Pixel stages: directly read views take FP32 patch records as PatchSource
// does; a staged footprint is copied into LDS as the caller's pixels, in FP32
// (a quarter of the bytes of its records; 16-bit pixels convert exactly), and
// each update forms its patch's coefficients from the four pixels with the
// same FP32 operations as patch_kernel, so both paths give the same bits.
__device__ short raw_buffer_load_i16(i32x4_t rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.i16");

template <typename T>
struct RawPatchSource : PatchSource {
    const T* raw;  // the caller's images of the pass, [n][H][W]
    static constexpr bool kRawStage = true;
    static constexpr uint32_t kElem = sizeof(T);

    // View k's pixels as a byte-addressed buffer of W H values: offsets past the end read 0
    // (the buffer's range check; no memory access).
    __device__ __forceinline__ i32x4_t raw_view(int k) const
    {
        const uint64_t a = (uint64_t)(raw + (size_t)k * W * H);
        i32x4_t rs;
        rs.x = (int)(uint32_t)a;
        rs.y = (int)((uint32_t)(a >> 32) & 0xffffu);
        rs.z = (int)((uint32_t)W * (uint32_t)H * kElem);
        rs.w = 0x00020000;
        return rs;
    }

    // The bits of the pixel at byte offset `off` of a view (0 past the view's end), and their FP32
    // value.  The prefetch keeps the bits, so that no conversion waits on a load in flight.
    static __device__ __forceinline__ uint32_t raw_bits(const i32x4_t& rs, int off)
    {
        if constexpr (sizeof(T) == 4) return __builtin_bit_cast(uint32_t, raw_buffer_load_f32(rs, off, 0, 0));
        else return (uint16_t)raw_buffer_load_i16(rs, off, 0, 0);
    }
    static __device__ __forceinline__ float from_bits(uint32_t b)
    {
        if constexpr (sizeof(T) == 4) return u32_as_f32(b);
        else if constexpr (__is_same(T, __half)) return f16_lo(b);
        else return bf16_lo(b);
    }
    static __device__ __forceinline__ float raw_tap(const i32x4_t& rs, int off) { return from_bits(raw_bits(rs, off)); }

    __device__ __forceinline__ Rec raw_rec(const i32x4_t& rs, int c0, int r0) const
    {
        const int i = c0 - 1, j = r0 - 1;
        const bool ca = (unsigned)i < (unsigned)W, cb = (unsigned)(i + 1) < (unsigned)W;
        const bool ra = (unsigned)j < (unsigned)H, rb = (unsigned)(j + 1) < (unsigned)H;
        const int ia = min(max(i, 0), W - 1), ib = min(i + 1, W - 1);
        const int ja = min(max(j, 0), H - 1) * W, jb = min(j + 1, H - 1) * W;
        const int e = (int)kElem;
        const float a0 = raw_tap(rs, (ja + ia) * e), b0 = raw_tap(rs, (ja + ib) * e);
        const float c1 = raw_tap(rs, (jb + ia) * e), d1 = raw_tap(rs, (jb + ib) * e);
        const float a = (ra & ca) ? a0 : 0.0f, b = (ra & cb) ? b0 : 0.0f;
        const float cc = (rb & ca) ? c1 : 0.0f, d = (rb & cb) ? d1 : 0.0f;
        Rec q;
        q.x = a;
        q.y = b - a;
        q.z = cc;
        q.w = d - cc;
        return q;
    }
};

// Compact bilinear-patch layout for 16-bit projections: the four coefficients
//     a = P(r,c), dx = P(r,c+1) - a, dy = P(r+1,c) - a, dxy = P(r+1,c+1) - P(r+1,c) - dx
// of the patch, B = a + fx dx + fy (dy + fx dxy), stored as FP16 (8 bytes per record) after
// scaling view k by a power of two, 2^e_k, chosen from the view's largest
// |pixel| so that no coefficient can overflow FP16 (|dxy| <= 4 max|p| <=
// 2^13).  v_fma_mix_f32 evaluates FP16 coefficients with FP32 weights and
// FP32 results, so Part 3 still costs three instructions; the scale is undone
// in the 1/w^2 weight (exact: a power of two).
typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));
__device__ f16x4_t struct_buffer_load_f16x4(i32x4_t rsrc, int vindex, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.buffer.load.v4f16");

struct Patch16Source {
    const uint8_t* base;
    int W, H;
    const float* inv_scale;  // 2^-e_k per view of the pass
    static constexpr bool kRawStage = false;

    struct View {
        i32x4_t rs;
        float inv;
    };

    __device__ __forceinline__ int cols() const { return W + 2; }

    __device__ __forceinline__ View view(int k) const
    {
        const uint32_t n = (uint32_t)(W + 2) * (uint32_t)(H + 2);
        const uint64_t a = (uint64_t)(base + (size_t)k * n * 8u);
        View v;
        v.rs.x = (int)(uint32_t)a;
        v.rs.y = (int)((uint32_t)(a >> 32) & 0xffffu) | (8 << 16);  // stride 8 bytes
        v.rs.z = (int)n;
        v.rs.w = 0x00020000;
        v.inv = inv_scale[k];
        return v;
    }

    using Rec = f16x4_t;

    __device__ __forceinline__ Rec load(const View& vw, int idx) const
    {
        return struct_buffer_load_f16x4(vw.rs, idx, 0, 0, 0);
    }

    static __device__ __forceinline__ float eval(const Rec& q, float fx, float fy)
    {
        return fmaf(fx, (float)q.y, fmaf(fy, fmaf(fx, (float)q.w, (float)q.z), (float)q.x));
    }

    __device__ __forceinline__ float weight_column(const View& vw, float r) const { return r * r * vw.inv; }
    __device__ __forceinline__ float weight_voxel(const View& vw, float r) const { return r * (r * vw.inv); }

    __device__ __forceinline__ float patch_at(const View& vw, int c0, float fx, float t) const
    {
        const int r0 = (int)t;
        const float fy = __builtin_amdgcn_fractf(t);
        return eval(load(vw, __mul24(r0, cols()) + c0), fx, fy);
    }

    __device__ __forceinline__ float patch(const View& vw, float s, float t) const
    {
        return patch_at(vw, (int)s, __builtin_amdgcn_fractf(s), t);
    }

    // CLAMP = false: the caller knows every position lies inside the bordered frame (an interior
    // footprint), so the clamps are left out.
    template <int ZU, bool CLAMP = true>
    __device__ __forceinline__ void column(const View& vw, float uxy, float vxy, float wxy, float p12,
                                           const float (&Z)[ZU], float (&acc)[ZU]) const
    {
        const float r = __builtin_amdgcn_rcpf(wxy);
        const float s = clamp_to<CLAMP>(fmaf(uxy, r, 1.0f), 0.0f, (float)(W + 1));
        const int c0 = (int)s;
        const float fx = __builtin_amdgcn_fractf(s);
        const float r2 = weight_column(vw, r);
        const float dt = p12 * r;
        const float tb = fmaf(vxy, r, 1.0f);
#pragma unroll
        for (int i = 0; i < ZU; ++i) {
            const float t = clamp_to<CLAMP>(fmaf(Z[i], dt, tb), 0.0f, (float)(H + 1));
            acc[i] = fmaf(patch_at(vw, c0, fx, t), r2, acc[i]);
        }
    }

    template <bool CLAMP = true>
    __device__ __forceinline__ float contrib_safe(const View& vw, float u, float v, float w) const
    {
        const float r = __builtin_amdgcn_rcpf(w);
        const float s = clamp_to<CLAMP>(fmaf(u, r, 1.0f), 0.0f, (float)(W + 1));
        const float t = clamp_to<CLAMP>(fmaf(v, r, 1.0f), 0.0f, (float)(H + 1));
        return patch(vw, s, t) * weight_voxel(vw, r);
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
        return ok ? val * (r * (r * vw.inv)) : 0.0f;
    }
};

// ---------------------------------------------------------------------------
// The back-projection pass.
// ---------------------------------------------------------------------------
template <bool B>
struct bool_tag {
    static constexpr bool value = B;
};

template <class Src>
struct has_column {
    static constexpr bool value = false;
};
template <>
struct has_column<PatchSource> {
    static constexpr bool value = true;
};
template <>
struct has_column<Patch16Source> {
    static constexpr bool value = true;
};
template <typename T, bool PAIRS>
struct has_column<CheckedSource<T, PAIRS>> {
    static constexpr bool value = true;
};

// One block = 256 threads covering a TX x (256/TX) tile of (x, y) columns and
// ZU voxels along z; a wavefront covers TX x (64/TX) columns.  Narrow tiles
// keep the detector footprint of one wavefront's 64 loads small.
//
// Tiles are numbered x fastest, then y, then z, and by default block b takes
// tile b: the blocks resident at any moment cover a thin z-band of the whole
// xy-plane, whose projection is a band of detector rows shared by all XCDs in
// MALL.  With xcd_order, block b takes tile (b % 8) * ceil(T / 8) + b / 8, so
// each XCD (blocks are dealt to the 8 XCDs round-robin) works through its own
// contiguous z-range; on MI355X that is slower (8 bands compete for MALL).
// With xcd_order = 2 ax (ax in 1, 2, 4, 8) the XCDs share the z-layer but
// each takes its own region of ax x (8 / ax) regions of the layer, so its L2
// holds only the part of the band that region projects to (measured +16% at
// L = 512 for ax = 8).
//
// cull: optional per-(tile, view) skip bits, `cull_words` words per tile,
// bit (kbase + k) set when the whole tile projects off the detector in view k
// of this pass.  Skipped views contribute exact zeros.
__device__ __forceinline__ int tile_of_block(int b, int gx, int gy, int n_tiles, int xcd_order)
{
    int tile = b;
    if (xcd_order == 1) {
        const int per = (n_tiles + kXcds - 1) / kXcds;
        tile = (tile % kXcds) * per + tile / kXcds;
    } else if (xcd_order >= 2) {
        // Shared z-layer, XCD-private xy-region: block b runs on XCD b % 8; the layer's
        // tiles are split into an ax x ay grid of regions (ax * ay = 8, ax = xcd_order / 2
        // ... encoded as xcd_order = 2 * ax) and that XCD takes its region, row by row.
        // (Launched only when gx % ax == 0 and gy % ay == 0.)
        const int ax = xcd_order >> 1, ay = kXcds / ax;
        const int xcd = tile % kXcds, j = tile / kXcds;
        const int rx = gx / ax, ry = gy / ay, per_layer = rx * ry;
        const int layer = j / per_layer, r = j % per_layer;
        const int bx_ = (xcd % ax) * rx + r % rx, by_ = (xcd / ax) * ry + r / rx;
        tile = (layer * gy + by_) * gx + bx_;
    }
    return tile;
}

// Passes on the caller's images (plain and direct-fused) are compiled for 8 waves per SIMD: they
// stream the volume, and occupancy keeps more of its loads in flight (L = 512, one view per pass:
// 419 -> 456 GUPS with 64-wide tiles, 417 -> 470 with 16-wide tiles).
// NT (passes on the caller's images, 64-wide tiles): the volume's read-modify-write as
// nontemporal loads and stores, for volumes that stream through HBM and leave the caches to the
// taps (plain pass at L = 512: 455 -> 481 GUPS; with 16-wide tiles, whose rows are half cache
// lines, and with volumes that fit in the caches it is slower, so the host takes it only for
// volumes of 256 MiB or more).  A compile-time choice: the compiler merges a nontemporal and a
// plain load of one address into one plain load.
template <class Src, int ZU, bool PADDED, int TX, bool NT = false>
__global__ __launch_bounds__(kBlock, PADDED ? 1 : 8) void backproject_kernel(
    float* __restrict__ vol, Box box, const ViewConst* __restrict__ vc, int n_views, Src src,
    const uint32_t* __restrict__ cull, int cull_words, int kbase, int xcd_order)
{
    constexpr int TY = kBlock / TX;
    const int gx = (box.nx + TX - 1) / TX, gy = (box.ny + TY - 1) / TY, gz = (box.nz + ZU - 1) / ZU;
    const int n_tiles = gx * gy * gz;
    const int tile = tile_of_block((int)blockIdx.x, gx, gy, n_tiles, xcd_order);
    if (tile >= n_tiles) return;  // padding blocks of the XCD order (no barriers in this kernel)
    const int bx = tile % gx, by = (tile / gx) % gy, bz = tile / (gx * gy);
    int x = bx * TX + (int)threadIdx.x % TX;
    int y = by * TY + (int)threadIdx.x / TX;
    const int z0 = bz * ZU;
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
    const uint32_t* cull_row = cull ? cull + (size_t)tile * cull_words : nullptr;
    // Passes on the caller's images (the plain pass reads one view per pass): load the volume's
    // old values before the taps, so that the read overlaps them (x, y are clamped: in bounds).
    // A tile that every view of the pass misses keeps its values: neither read nor written.
    float old[ZU];
    if constexpr (!PADDED) {
        if (cull_row) {
            bool missed = true;
            for (int k = 0; k < n_views && missed; ++k) {
                const int kk = kbase + k;
                missed = (cull_row[kk >> 5] >> (kk & 31)) & 1u;
            }
            if (missed) return;  // uniform over the block (no barriers in this kernel)
        }
        const size_t plane = (size_t)box.nx * (size_t)box.ny;
        const size_t col = (size_t)y * box.nx + x;
#pragma unroll
        for (int i = 0; i < ZU; ++i) {
            const float* p = vol + (size_t)(z0 + i) * plane + col;
            if constexpr (NT) old[i] = z0 + i < box.nz ? __builtin_nontemporal_load(p) : 0.0f;
            else old[i] = z0 + i < box.nz ? *p : 0.0f;
        }
    }

    for (int k = 0; k < n_views; ++k) {
        if (cull_row) {
            const int kk = kbase + k;
            if ((cull_row[kk >> 5] >> (kk & 31)) & 1u) continue;
        }
        const ViewConst& c = vc[k];
        const auto view = src.view(k);
        const float uxy = fmaf(c.p[1], Y, fmaf(c.p[0], X, c.p[3]));
        const float vxy = fmaf(c.p[5], Y, fmaf(c.p[4], X, c.p[7]));
        const float wxy = fmaf(c.p[9], Y, fmaf(c.p[8], X, c.p[11]));
        if constexpr (PADDED) {
            if constexpr (has_column<Src>::value) {
                if (c.mode == kModeColumn) {
                    src.column(view, uxy, vxy, wxy, c.p[6], Z, acc);
                    continue;
                }
            }
            if (c.mode != kModeGuarded) {
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
            if constexpr (has_column<Src>::value) {
                if (c.mode == kModeColumn) {
                    src.column(view, uxy, vxy, wxy, c.p[6], Z, acc);
                    continue;
                }
            }
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
                if constexpr (!PADDED) {  // the same sum as += (no other writer)
                    if constexpr (NT) __builtin_nontemporal_store(old[i] + acc[i], p);
                    else *p = old[i] + acc[i];
                } else {
                    *p += acc[i];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The fused pass with the taps staged through LDS.  For each staged view of
// the pass the block first copies its tile's footprint -- the rectangle of
// patches that any voxel of the tile can read, from the footprint table --
// into LDS with coalesced row loads: the patch records themselves (records
// sources), or the caller's FP32 pixels at the patches' corners (pixel
// sources), from which each update forms its patch with the record's own
// FP32 operations.  Every voxel then reads its patch from LDS.  The positions
// are clamped to the footprint instead of the bordered frame; the footprint
// holds every position the tile's voxels reach with a margin (see
// footprint_kernel), so the clamp only ever acts at the detector border,
// exactly as in the direct pass, and the results are bit-identical to it.
// The tap split's direct views, views whose footprint does not fit the
// stage, and guarded views read their patch records directly.
// ---------------------------------------------------------------------------
template <class Src, bool RAW = Src::kRawStage>
struct StageOf {
    using type = typename Src::Rec;  // what the stage holds: records
    using pre = type;
};
template <class Src>
struct StageOf<Src, true> {
    using type = float;     // the stage: the footprint's pixels
    using pre = uint32_t;   // their bits as loaded
};


// POISON (a testing aid, instantiated for ZU = 8 only): before each staged footprint is written,
// every word of the LDS stage is set to a NaN pattern, so that any read of a stage element the
// footprint did not write would turn the voxel's sum into NaN.
// The pixel-stage pass is compiled for 8 waves per SIMD (at most 64 VGPRs): its LDS reads and
// their arithmetic hide latency by occupancy (at L = 512: 32.4 -> 29.3 ms for a reconstruction
// with every view staged, against 5 waves at 94 VGPRs).  Record stages keep the compiler's
// choice: their directly read records need the registers to stay in flight.
template <class Src>
constexpr int kLdsWavesPerSimd = Src::kRawStage ? 8 : 1;

template <class Src, int ZU, int TX, bool POISON = false>
__global__ __launch_bounds__(kBlock, kLdsWavesPerSimd<Src>) void backproject_lds_kernel(
    float* __restrict__ vol, Box box, const ViewConst* __restrict__ vc, int n_views, Src src,
    const uint2* __restrict__ fp, int xcd_order)
{
    using Rec = typename Src::Rec;
    constexpr bool kRaw = Src::kRawStage;
    static_assert(kStageMaxWidth * kStageMaxHeight == kStageRecords, "LDS stage shape");
    using StageT = typename StageOf<Src>::type;  // patch records, or FP32 pixels
    using PreT = typename StageOf<Src>::pre;     // what a lane prefetches: records, or pixel bits
    __shared__ StageT lds[kRaw ? kRawColStride * kStageMaxWidth : kStageRecords];
    constexpr int TY = kBlock / TX;
    const int gx = (box.nx + TX - 1) / TX, gy = (box.ny + TY - 1) / TY, gz = (box.nz + ZU - 1) / ZU;
    const int n_tiles = gx * gy * gz;
    const int tile = tile_of_block((int)blockIdx.x, gx, gy, n_tiles, xcd_order);
    if (tile >= n_tiles) return;  // whole block: before any barrier
    const int bx = tile % gx, by = (tile / gx) % gy, bz = tile / (gx * gy);
    // A 16 x 16 tile's waves are its 8 x 8 quadrants (other widths: rows of the tile): with the
    // column-major pixel stage their LDS reads conflict less (measured: FP32 +2%, BF16 +3.7%).
    const int wv = (int)threadIdx.x >> 6, ln = (int)threadIdx.x & 63;
    int x = TX == 16 ? bx * TX + 8 * (wv & 1) + (ln & 7) : bx * TX + (int)threadIdx.x % TX;
    int y = TX == 16 ? by * TY + 8 * (wv >> 1) + (ln >> 3) : by * TY + (int)threadIdx.x / TX;
    const int z0 = bz * ZU;
    const bool in_xy = (x < box.nx) & (y < box.ny);
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
    const uint2* fp_row = fp + (size_t)tile * n_views;
    // The next staged footprint, loaded while the current view is computed: footprint row
    // wave + 4 j is slot j of that wave, one column per lane.  Records: fw <= 64 and fh <= 4
    // kStageSlots; FP32 pixels: the fw + 1 columns and fh + 1 rows of the patches' corners,
    // fw < 64 and fh < 4 kRawSlots (the footprint table keeps to these bounds).
    constexpr int kSlots = kRaw ? kRawSlots : kStageSlots;
    PreT pre[kSlots];
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int lane = (int)threadIdx.x & 63;
    // a pixel stage's byte offset of the lane's column in a row, kept in a register (so that a
    // row's offset is one add to a uniform sum, not refolded into a shift of the column)
    uint32_t lane_b = (uint32_t)lane * 4u;
    if constexpr (kRaw) lane_b = (uint32_t)lane * Src::kElem;
    asm("" : "+v"(lane_b));
    auto prefetch = [&](int k, uint2 f) {
        const int cmin = (int)(f.x & 0xffffu), rmin = (int)(f.x >> 16);
        const int fw = (int)(f.y & kFootprintWidthMask), fh = (int)(f.y >> 16);
        if constexpr (kRaw) {
            // Padded pixel (r, c) is detector pixel (c - 1, r - 1), at byte offset ((r - 1) W + c - 1) e
            // of the view (e bytes per pixel).  A pixel off the detector is read at an offset at or past
            // the view's W H e < 2^31 bytes, which the buffer's range check returns as 0 without a
            // memory access: columns off the detector at kFar and beyond (kFar less four rows for slot
            // 0, still past 2^31), rows below it past the end by themselves, and the row above it (slot
            // 0 of wave 0 when rmin = 0) at (c - 1) e - W e < 0, which wraps to 2^32 - W e or more
            // (W <= 2^20).  Each lane loads one pixel per slot (no two of its loads are adjacent, so
            // none is merged into a wider load).
            constexpr uint32_t kFar = 0xC0000000u;
            constexpr uint32_t e = Src::kElem;
            // lane l holds padded column cmin + l, a detector column when 1 <= cmin + l <= W (l <= fw):
            // the bounds are uniform, the lane's byte offset within a row one add
            const bool col_ok = (lane >= 1 - cmin) & (lane <= min(fw, src.W - cmin));
            const uint32_t row_bytes = (uint32_t)src.W * e;
            // slot 1's row, rmin + 3 + wave >= 3, is never above the detector (the sum is exact modulo
            // 2^32, the column term wrapping for cmin = 0)
            const uint32_t off1 =
                col_ok ? (uint32_t)(rmin + 3 + wave) * row_bytes + (uint32_t)(cmin - 1) * e + lane_b : kFar;
            const i32x4_t rs = src.raw_view(k);
            if (wave <= fh) pre[0] = Src::raw_bits(rs, (int)(off1 - 4u * row_bytes));
#pragma unroll
            for (int j = 1; j < kSlots; ++j)
                if (wave + 4 * j <= fh)
                    pre[j] = Src::raw_bits(rs, (int)(off1 + (uint32_t)(4 * (j - 1)) * row_bytes));
        } else {
            const auto vw = src.view(k);
            const int cols = src.cols();
            const int g = (rmin + wave) * cols + cmin + lane;  // record index in the staging view
            if (lane < fw) {
#pragma unroll
                for (int j = 0; j < kSlots; ++j)
                    if (wave + 4 * j < fh) pre[j] = src.load(vw, g + 4 * j * cols);
            }
        }
    };
    auto staged = [](uint2 f) { return f.y != kFootprintSkip && f.y != kFootprintDirect && f.y != kFootprintPixels; };
    auto stage = [&](StageT* buf, uint2 f) {  // the prefetched records or pixels into LDS
        const int fw = (int)(f.y & kFootprintWidthMask), fh = (int)(f.y >> 16);
        if constexpr (kRaw) {
            if (lane <= fw) {
                StageT* dst = buf + lane * kRawColStride + wave;  // column lane, row wave + 4 j
#pragma unroll
                for (int j = 0; j < kSlots; ++j)
                    if (wave + 4 * j <= fh) dst[4 * j] = Src::from_bits(pre[j]);
            }
        } else {
            if (lane < fw) {
                StageT* dst = buf + wave * fw + lane;
#pragma unroll
                for (int j = 0; j < kSlots; ++j)
                    if (wave + 4 * j < fh) dst[4 * j * fw] = pre[j];
            }
        }
    };
    // Patch (r0, c0) of the staged footprint, as a record.  Records: row stride fw; pixels: the
    // four corners, column-major at a fixed column stride.  `off` is the byte offset of (r0, c0).
    auto staged_rec = [&](uint32_t off) -> Rec {
        const char* lds_b = reinterpret_cast<const char*>(lds);
        if constexpr (kRaw) {
            // the record (a, b - a, c, d - c) of the four pixels with the roundings of patch_kernel
            const float* q = static_cast<const float*>(__builtin_assume_aligned(lds_b + off, 4));
            const float a = q[0], cc = q[1], b = q[kRawColStride], d = q[kRawColStride + 1];
            Rec r;
            r.x = a;
            r.y = b - a;
            r.z = cc;
            r.w = d - cc;
            return r;
        } else {
            return *static_cast<const Rec*>(__builtin_assume_aligned(lds_b + off, sizeof(Rec)));
        }
    };
    uint2 f_next = fp_row[0];
    if (staged(f_next)) prefetch(0, f_next);

    // One LDS buffer, two barriers per staged view.  (Two buffers and one barrier per view
    // measured slower for 8-byte records: fewer blocks fit a CU.)
    for (int k = 0; k < n_views; ++k) {
        const uint2 f = f_next;  // the same for the whole block
        if (staged(f)) {
            __syncthreads();  // every wave is done with the previous footprint
            if constexpr (POISON) {
                uint32_t* words = reinterpret_cast<uint32_t*>(lds);
                for (int i = (int)threadIdx.x; i < (int)(sizeof(lds) / 4); i += kBlock) words[i] = kPoisonPattern;
                __syncthreads();
            }
            stage(lds, f);
            __syncthreads();
        }
        if (k + 1 < n_views) {
            f_next = fp_row[k + 1];
            if (staged(f_next)) prefetch(k + 1, f_next);
        }
        if (f.y == kFootprintSkip) continue;
        const ViewConst& c = vc[k];
        const auto view = src.view(k);
        const float uxy = fmaf(c.p[1], Y, fmaf(c.p[0], X, c.p[3]));
        const float vxy = fmaf(c.p[5], Y, fmaf(c.p[4], X, c.p[7]));
        const float wxy = fmaf(c.p[9], Y, fmaf(c.p[8], X, c.p[11]));
        if (f.y == kFootprintDirect) {
            // directly read views keep the clamp into the bordered frame (without it the compiler
            // keeps all ZU record loads in flight at once: 114 VGPRs instead of 94, measured)
            if (c.mode == kModeColumn) {
                src.column(view, uxy, vxy, wxy, c.p[6], Z, acc);
            } else if (c.mode == kModeSafe) {
#pragma unroll
                for (int i = 0; i < ZU; ++i)
                    acc[i] += src.contrib_safe(view, fmaf(c.p[2], Z[i], uxy), fmaf(c.p[6], Z[i], vxy),
                                               fmaf(c.p[10], Z[i], wxy));
            } else {
#pragma unroll
                for (int i = 0; i < ZU; ++i)
                    acc[i] += src.contrib_guarded(view, fmaf(c.p[2], Z[i], uxy), fmaf(c.p[6], Z[i], vxy),
                                                  fmaf(c.p[10], Z[i], wxy));
            }
            continue;
        }
        if constexpr (kRaw) {
            if (f.y == kFootprintPixels) {
                // a footprint too large for the stage: the patches' pixels from the caller's image,
                // positions clamped into the bordered frame as the directly read views do
                const i32x4_t rs = src.raw_view(k);
                const float sw = (float)(src.W + 1), sh = (float)(src.H + 1);
                if (c.mode == kModeColumn) {
                    const float r = __builtin_amdgcn_rcpf(wxy);
                    const float sc = __builtin_amdgcn_fmed3f(fmaf(uxy, r, 1.0f), 0.0f, sw);
                    const int c0 = (int)sc;
                    const float fx = __builtin_amdgcn_fractf(sc);
                    const float r2 = src.weight_column(view, r);
                    const float dt = c.p[6] * r;
                    const float tb = fmaf(vxy, r, 1.0f);
#pragma unroll
                    for (int i = 0; i < ZU; ++i) {
                        const float t = __builtin_amdgcn_fmed3f(fmaf(Z[i], dt, tb), 0.0f, sh);
                        const Rec q = src.raw_rec(rs, c0, (int)t);
                        acc[i] = fmaf(Src::eval(q, fx, __builtin_amdgcn_fractf(t)), r2, acc[i]);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < ZU; ++i) {
                        const float w = fmaf(c.p[10], Z[i], wxy);
                        const float r = __builtin_amdgcn_rcpf(w);
                        const float sv = __builtin_amdgcn_fmed3f(fmaf(fmaf(c.p[2], Z[i], uxy), r, 1.0f), 0.0f, sw);
                        const float tv = __builtin_amdgcn_fmed3f(fmaf(fmaf(c.p[6], Z[i], vxy), r, 1.0f), 0.0f, sh);
                        const Rec q = src.raw_rec(rs, (int)sv, (int)tv);
                        acc[i] += Src::eval(q, __builtin_amdgcn_fractf(sv), __builtin_amdgcn_fractf(tv)) *
                                  src.weight_voxel(view, r);
                    }
                }
                continue;
            }
        }
        const int cmin = (int)(f.x & 0xffffu), rmin = (int)(f.x >> 16);
        const int fw = (int)(f.y & kFootprintWidthMask), fh = (int)(f.y >> 16);
        // byte offsets of the stage, so that a row's address is one multiply-add:
        // patch (r0, c0) at r0 * row_b + (c0 cstride - rmin stride - cmin cstride) * elem, with
        // stride / cstride the elements between rows / columns (pixels: column-major; records:
        // row-major, the footprint's width apart)
        const int stride = kRaw ? 1 : fw;
        const int cstride = kRaw ? kRawColStride : 1;
        const uint32_t elem = (uint32_t)sizeof(StageT);
        const uint32_t row_b = (uint32_t)stride * elem;
        const int base = -(rmin * stride + cmin * cstride);
        // row r0's offset: pixels one element apart (a shift), records a footprint width apart
        auto row_off = [&](int r0) -> uint32_t {
            if constexpr (kRaw) return (uint32_t)r0 * row_b;
            else return __umul24((uint32_t)r0, row_b);
        };
        // positions are clamped into [cmin, cmin + fw) x [rmin, rmin + fh) (the upper bounds the
        // largest floats below them): a position inside keeps its fraction, and the patch stays in
        // the footprint.  An interior footprint (kFootprintInner) has a record of margin on every
        // side of every position of the tile and needs no clamp.
        auto staged_view = [&](auto clamp_tag) {
            constexpr bool CLAMP = decltype(clamp_tag)::value;
            float s_lo = 0.0f, s_hi = 0.0f, t_lo = 0.0f, t_hi = 0.0f;
            if constexpr (CLAMP) {
                s_lo = (float)cmin;
                s_hi = __int_as_float(__float_as_int((float)(cmin + fw)) - 1);
                t_lo = (float)rmin;
                t_hi = __int_as_float(__float_as_int((float)(rmin + fh)) - 1);
            }
            if (c.mode == kModeColumn) {
                const float r = __builtin_amdgcn_rcpf(wxy);
                const float sc = clamp_to<CLAMP>(fmaf(uxy, r, 1.0f), s_lo, s_hi);
                const int c0 = (int)sc;
                const float fx = __builtin_amdgcn_fractf(sc);
                const float r2 = src.weight_column(view, r);
                const float dt = c.p[6] * r;
                const float tb = fmaf(vxy, r, 1.0f);
                // pixels: the column's first element as one 24-bit multiply-add (0 <= c0 < 2^24)
                const uint32_t cb_b = (uint32_t)(kRaw ? base + (int)__umul24((uint32_t)c0, (uint32_t)kRawColStride)
                                                      : base + c0) * elem;
#pragma unroll
                for (int i = 0; i < ZU; ++i) {
                    const float t = clamp_to<CLAMP>(fmaf(Z[i], dt, tb), t_lo, t_hi);
                    const int r0 = (int)t;
                    const float fy = __builtin_amdgcn_fractf(t);
                    const Rec q = staged_rec(row_off(r0) + cb_b);
                    acc[i] = fmaf(Src::eval(q, fx, fy), r2, acc[i]);
                }
            } else {  // safe
                uint32_t base_b = (uint32_t)base * elem;
                asm("" : "+s"(base_b));
#pragma unroll
                for (int i = 0; i < ZU; ++i) {
                    const float u = fmaf(c.p[2], Z[i], uxy), v = fmaf(c.p[6], Z[i], vxy),
                                w = fmaf(c.p[10], Z[i], wxy);
                    const float r = __builtin_amdgcn_rcpf(w);
                    const float sv = clamp_to<CLAMP>(fmaf(u, r, 1.0f), s_lo, s_hi);
                    const float tv = clamp_to<CLAMP>(fmaf(v, r, 1.0f), t_lo, t_hi);
                    const int c0 = (int)sv, r0 = (int)tv;
                    // pixels: (c0 * column stride + r0) as one 24-bit multiply-add (c0 and r0 are at
                    // least 0 and below 2^24), then one shift-add of the footprint's origin (an opaque
                    // uniform, so that the compiler does not fold it into the sum before the shift)
                    const uint32_t off = kRaw ? (__umul24((uint32_t)c0, (uint32_t)kRawColStride) + (uint32_t)r0) * elem +
                                                    base_b
                                              : row_off(r0) + (uint32_t)(base + c0) * elem;
                    const Rec q = staged_rec(off);
                    const float val = Src::eval(q, __builtin_amdgcn_fractf(sv), __builtin_amdgcn_fractf(tv));
                    acc[i] += val * src.weight_voxel(view, r);
                }
            }
        };
        if (f.y & kFootprintInner) staged_view(bool_tag<false>{});
        else staged_view(bool_tag<true>{});
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
// Footprints of a pass: for tile t and view k of the pass, the rectangle of
// patch records [cmin, cmin + fw) x [rmin, rmin + fh) that the tile's voxels
// can read.  The corners' positions (FP64, padded coordinates s = u/w + 1,
// t = v/w + 1) bound every voxel's position (w > 0 on the box, so the image
// of the tile is the convex hull of the corners' images); the rectangle adds
// one record below and one above the corners' range on each axis, far more
// than the FP32 rounding of the pass, and is cut to the bordered frame
// [0, W+1] x [0, H+1].  Entry {0, kFootprintSkip}: the tile projects off the
// detector (the test of cull_kernel, exact zeros); {0, kFootprintDirect}: a
// guarded view, a footprint (of a record stage) wider than max_w records,
// taller than max_h or of more than `cap` records, or one of the views k with
// k % 8 < direct_eighths -- those read their taps directly, so that the
// pass draws on the L1 path and the LDS path at once; {0, kFootprintPixels}:
// a pixel stage's footprint beyond those bounds (its pixels are read directly).
// The kFootprintInner bit of a staged entry's width field marks an interior
// footprint, whose positions need no clamp.
// ---------------------------------------------------------------------------
// The footprint table entry of one (tile, view) from the range of its corners' padded positions and
// the bound on the FP32 error of the pass's positions.
__device__ uint2 footprint_entry(bool skip, double smin, double smax, double tmin, double tmax, double err, int k,
                                 int W, int H, int cap, int max_w, int max_h, int direct_eighths, bool raw,
                                 uint32_t* __restrict__ big)
{
    if (skip) return make_uint2(0u, kFootprintSkip);
    // Interior: the rectangle below (one record of margin on each side of the corners' range) lies
    // inside the bordered frame without cutting, and the FP32 position error of the pass is far
    // below that margin, so no position of the tile needs clamping.  (NaN compares false.)
    const bool inner = err < 0.25 && floor(smin) - 1.0 >= 0.0 && floor(smax) + 1.0 <= (double)(W + 1) &&
                       floor(tmin) - 1.0 >= 0.0 && floor(tmax) + 1.0 <= (double)(H + 1);
    // this share of the views reads its taps directly (through L1)
    if ((k & 7) < direct_eighths) return make_uint2(0u, kFootprintDirect);
    // fmin / fmax also map a NaN to the frame
    const int c0 = (int)fmin(fmax(floor(smin) - 1.0, 0.0), (double)(W + 1));
    const int c1 = (int)fmin(fmax(floor(smax) + 1.0, 0.0), (double)(W + 1));
    const int r0 = (int)fmin(fmax(floor(tmin) - 1.0, 0.0), (double)(H + 1));
    const int r1 = (int)fmin(fmax(floor(tmax) + 1.0, 0.0), (double)(H + 1));
    const int fw = max(c1 - c0 + 1, 1), fh = max(r1 - r0 + 1, 1);
    if (fw > max_w || fh > max_h || (long)fw * fh > cap) {
        if (raw) return make_uint2(0u, kFootprintPixels);  // the tile reads the caller's pixels
        if (big) big[k] = 1u;  // this view's records are read after all (every writer stores 1)
        return make_uint2(0u, kFootprintDirect);
    }
    return make_uint2((uint32_t)c0 | ((uint32_t)r0 << 16),
                      (uint32_t)fw | (inner ? kFootprintInner : 0u) | ((uint32_t)fh << 16));
}

// First-order bound on the FP32 error of a padded position p = n / w + 1 as the pass forms it (each
// FP32 operation rounds by at most 2^-24 of its result, the reciprocal by 2^-23): 8 roundings on the
// magnitudes an (of the terms of the numerator) and aw (of w), plus the +1.
__device__ __forceinline__ double position_error(double p, double an, double aw, double arw)
{
    return 8.0 * 0x1p-24 * (an + fabs(p - 1.0) * aw) * arw + 0x1p-23 * (2.0 * fabs(p) + 2.0);
}

// One thread per (column of tiles (bx, by), view): the entries of every z-layer of tiles.  For a
// column view (u and w do not depend on z) the reciprocals of w and the column positions are formed
// once, at the 4 (x, y) corners, and each z-layer only adds its rows; other views take all 8 corners
// of each tile.
__global__ void footprint_kernel(const ViewConst* __restrict__ vc, int n_views, Box box, int tx, int ty, int tz,
                                 int gx, int gy, int gz, int W, int H, int cap, int max_w, int max_h,
                                 int direct_eighths, bool raw, uint2* __restrict__ out, uint32_t* __restrict__ big)
{
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long)gx * gy * n_views) return;
    const int xy = (int)(id / n_views), k = (int)(id % n_views);
    const long layer = (long)gx * gy * n_views;  // entries of one z-layer of tiles
    uint2* o = out + id;                           // tile (bx, by, bz), view k: o[bz * layer]
    const ViewConst& c = vc[k];
    if (c.mode == kModeGuarded) {
        for (int bz = 0; bz < gz; ++bz) o[bz * layer] = make_uint2(0u, kFootprintDirect);
        return;
    }
    const int bx = xy % gx, by = xy / gx;
    const int xs[2] = {bx * tx, min(bx * tx + tx - 1, box.nx - 1)};
    const int ys[2] = {by * ty, min(by * ty + ty - 1, box.ny - 1)};
    // per axis and corner coordinate: the terms of u, v, w and their magnitudes
    double tu[2][2], tv[2][2], tw[2][2], au[2][2], av[2][2], aw[2][2];
    for (int e = 0; e < 2; ++e) {
        const double X = (double)box.ox + (double)box.vs * xs[e];
        const double Y = (double)box.oy + (double)box.vs * ys[e];
        tu[0][e] = (double)c.p[0] * X;
        tv[0][e] = (double)c.p[4] * X;
        tw[0][e] = (double)c.p[8] * X;
        tu[1][e] = (double)c.p[1] * Y;
        tv[1][e] = (double)c.p[5] * Y;
        tw[1][e] = (double)c.p[9] * Y;
        for (int a = 0; a < 2; ++a) {
            au[a][e] = fabs(tu[a][e]);
            av[a][e] = fabs(tv[a][e]);
            aw[a][e] = fabs(tw[a][e]);
        }
    }
    if (c.mode == kModeColumn) {
        // P[0][2] = P[2][2] = 0: u, w and the column positions at the 4 (x, y) corners
        double rw[4], vxy[4], avxy[4], wq[4], awq[4];
        bool left = true, right = true;
        double smin = 0.0, smax = 0.0, es = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ex = q & 1, ey = q >> 1;
            const double u = tu[0][ex] + tu[1][ey] + (double)c.p[3];
            const double w = tw[0][ex] + tw[1][ey] + (double)c.p[11];
            left &= u <= -2.0 * w;
            right &= u >= (W + 1.0) * w;
            rw[q] = 1.0 / w;
            wq[q] = w;
            vxy[q] = tv[0][ex] + tv[1][ey];
            avxy[q] = av[0][ex] + av[1][ey] + fabs((double)c.p[7]);
            awq[q] = aw[0][ex] + aw[1][ey] + fabs((double)c.p[11]);
            const double sq = fma(u, rw[q], 1.0);
            smin = q ? fmin(smin, sq) : sq;
            smax = q ? fmax(smax, sq) : sq;
            es = fmax(es, position_error(sq, au[0][ex] + au[1][ey] + fabs((double)c.p[3]), awq[q], fabs(rw[q])));
        }
        for (int bz = 0; bz < gz; ++bz) {
            const int zs[2] = {bz * tz, min(bz * tz + tz - 1, box.nz - 1)};
            bool top = true, bottom = true;
            double tmin = 0.0, tmax = 0.0, err = es;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int ez = q >> 2, cq = q & 3;
                const double pz = (double)c.p[6] * ((double)box.oz + (double)box.vs * zs[ez]);
                const double v = vxy[cq] + pz + (double)c.p[7];
                top &= v <= -2.0 * wq[cq];
                bottom &= v >= (H + 1.0) * wq[cq];
                const double t = fma(v, rw[cq], 1.0);
                tmin = q ? fmin(tmin, t) : t;
                tmax = q ? fmax(tmax, t) : t;
                err = fmax(err, position_error(t, avxy[cq] + fabs(pz), awq[cq], fabs(rw[cq])));
            }
            o[bz * layer] = footprint_entry(left | right | top | bottom, smin, smax, tmin, tmax, err, k, W, H, cap,
                                            max_w, max_h, direct_eighths, raw, big);
        }
        return;
    }
    for (int bz = 0; bz < gz; ++bz) {
        const int zs[2] = {bz * tz, min(bz * tz + tz - 1, box.nz - 1)};
        double tu2[2], tv2[2], tw2[2], au2[2], av2[2], aw2[2];  // z terms with the constant column
        for (int e = 0; e < 2; ++e) {
            const double Z = (double)box.oz + (double)box.vs * zs[e];
            tu2[e] = (double)c.p[2] * Z + (double)c.p[3];
            tv2[e] = (double)c.p[6] * Z + (double)c.p[7];
            tw2[e] = (double)c.p[10] * Z + (double)c.p[11];
            au2[e] = fabs((double)c.p[2] * Z) + fabs((double)c.p[3]);
            av2[e] = fabs((double)c.p[6] * Z) + fabs((double)c.p[7]);
            aw2[e] = fabs((double)c.p[10] * Z) + fabs((double)c.p[11]);
        }
        bool left = true, right = true, top = true, bottom = true;
        double smin = 0.0, smax = 0.0, tmin = 0.0, tmax = 0.0, err = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int ex = q & 1, ey = (q >> 1) & 1, ez = q >> 2;
            const double u = tu[0][ex] + tu[1][ey] + tu2[ez];
            const double v = tv[0][ex] + tv[1][ey] + tv2[ez];
            const double w = tw[0][ex] + tw[1][ey] + tw2[ez];
            left &= u <= -2.0 * w;
            right &= u >= (W + 1.0) * w;
            top &= v <= -2.0 * w;
            bottom &= v >= (H + 1.0) * w;
            const double rw = 1.0 / w;
            const double s = fma(u, rw, 1.0), t = fma(v, rw, 1.0);
            smin = q ? fmin(smin, s) : s;
            smax = q ? fmax(smax, s) : s;
            tmin = q ? fmin(tmin, t) : t;
            tmax = q ? fmax(tmax, t) : t;
            const double awq = aw[0][ex] + aw[1][ey] + aw2[ez], arw = fabs(rw);
            err = fmax(err, fmax(position_error(s, au[0][ex] + au[1][ey] + au2[ez], awq, arw),
                                 position_error(t, av[0][ex] + av[1][ey] + av2[ez], awq, arw)));
        }
        o[bz * layer] = footprint_entry(left | right | top | bottom, smin, smax, tmin, tmax, err, k, W, H, cap, max_w,
                                        max_h, direct_eighths, raw, big);
    }
}

__global__ void zero_u32_kernel(uint32_t* __restrict__ p, int n)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0u;
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t word)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = word;
}

// ---------------------------------------------------------------------------
// Per-view constants: copy P_k and pick the view's branch.  w is affine, so
// its extremes over the box are at the 8 corner voxels (evaluated in FP64).
//   guarded  some voxel may have w < 1e-4 * max w (at or behind the source)
//   safe     every voxel is in front of the source: clamp, no tests
//   column   safe, and P[0][2] = P[2][2] = 0: u and w do not vary along z,
//            as for any circular orbit about the z axis
// ---------------------------------------------------------------------------
__global__ void prep_views_kernel(const float* __restrict__ mats, int n_views, Box box, int column_ok,
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
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 12; ++i) finite &= isfinite(c.p[i]);
    // false for NaN; a non-finite matrix or a vanishing w also takes the guarded branch
    const bool safe = finite && wmin > 0.0 && wmin >= 1e-4 * wmax && wmin > 1e-30;
    c.mode = !safe                                                  ? kModeGuarded
             : (column_ok && c.p[2] == 0.0f && c.p[10] == 0.0f) ? kModeColumn
                                                                : kModeSafe;
    c.pad[0] = c.pad[1] = c.pad[2] = 0;
    out[k] = c;
}

// ---------------------------------------------------------------------------
// Clipping mask (the per-line start/stop of Sec. 5, here per block tile and
// view): bit k of a tile's row is set when all 8 corner voxels of the tile
// project at least one pixel beyond the same detector edge (s <= -2, s >= W+1,
// t <= -2 or t >= H+1; FP64, no division).  For a safe view w > 0 on the whole
// box, so the tile's image is the convex hull of the corners' images and
// every voxel of the tile clamps into the zero border: its contribution is
// exactly 0.  Guarded views are never skipped.  One thread per (tile, word).
// ---------------------------------------------------------------------------
__global__ void cull_kernel(const ViewConst* __restrict__ vc, int n_views, Box box, int tx, int ty, int tz,
                            int gx, int gy, int n_tiles, int words, int W, int H, uint32_t* __restrict__ out)
{
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long)n_tiles * words) return;
    const int tile = (int)(id / words), word = (int)(id % words);
    const int bx = tile % gx, by = (tile / gx) % gy, bz = tile / (gx * gy);
    const int xs[2] = {bx * tx, min(bx * tx + tx - 1, box.nx - 1)};
    const int ys[2] = {by * ty, min(by * ty + ty - 1, box.ny - 1)};
    const int zs[2] = {bz * tz, min(bz * tz + tz - 1, box.nz - 1)};
    double cx[2], cy[2], cz[2];
    for (int i = 0; i < 2; ++i) {
        cx[i] = (double)box.ox + (double)box.vs * xs[i];
        cy[i] = (double)box.oy + (double)box.vs * ys[i];
        cz[i] = (double)box.oz + (double)box.vs * zs[i];
    }
    uint32_t bits = 0;
    const int k_end = min(n_views, (word + 1) * 32);
    for (int k = word * 32; k < k_end; ++k) {
        const ViewConst& c = vc[k];
        if (c.mode == kModeGuarded) continue;
        bool left = true, right = true, top = true, bottom = true;
        for (int q = 0; q < 8; ++q) {
            const double X = cx[q & 1], Y = cy[(q >> 1) & 1], Z = cz[q >> 2];
            const double u = (double)c.p[0] * X + (double)c.p[1] * Y + (double)c.p[2] * Z + (double)c.p[3];
            const double v = (double)c.p[4] * X + (double)c.p[5] * Y + (double)c.p[6] * Z + (double)c.p[7];
            const double w = (double)c.p[8] * X + (double)c.p[9] * Y + (double)c.p[10] * Z + (double)c.p[11];
            left &= u <= -2.0 * w;
            right &= u >= (W + 1.0) * w;
            top &= v <= -2.0 * w;
            bottom &= v >= (H + 1.0) * w;
        }
        if (left | right | top | bottom) bits |= 1u << (k & 31);
    }
    out[id] = bits;
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

// Bilinear-patch staging copy: a block covers 256 columns by kPatchRows rows of the (H+2) x (W+2)
// grid of patches, a thread one column of them, top to bottom, so that it loads each pixel row once
// (the lower corners of one patch are the upper corners of the next).
constexpr int kPatchRows = 16;

template <typename T>
__global__ __launch_bounds__(256) void patch_kernel(const T* __restrict__ proj, int W, int H,
                                                    f32x4_t* __restrict__ out, ViewNeed need)
{
    const int Wq = W + 2, Hq = H + 2;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int k = (int)blockIdx.z;
    if (need.vc && (k & 7) >= need.direct_eighths && need.vc[k].mode != kModeGuarded && need.big[k] == 0u)
        return;  // whole block: no tile reads this view's records
    if (c >= Wq) return;
    const int r_begin = (int)blockIdx.y * kPatchRows, r_end = min(r_begin + kPatchRows, Hq);
    const T* img = proj + (size_t)k * W * H;
    const int i = c - 1;  // detector column of the patches' first corners
    f32x4_t* dst = out + ((size_t)k * Hq + r_begin) * Wq + c;
    float a = pixel_f32(img, W, H, i, r_begin - 1), b = pixel_f32(img, W, H, i + 1, r_begin - 1);
    for (int r = r_begin; r < r_end; ++r, dst += Wq) {
        const float cc = pixel_f32(img, W, H, i, r), d = pixel_f32(img, W, H, i + 1, r);
        f32x4_t q;
        q.x = a;
        q.y = b - a;
        q.z = cc;
        q.w = d - cc;
        *dst = q;
        a = cc;
        b = d;
    }
}

// Largest |pixel| of each view (as the bits of a non-negative float, which
// order like unsigned integers): block reduction, then one atomic per block.
template <typename T>
__global__ __launch_bounds__(256) void maxabs_kernel(const T* __restrict__ proj, int W, int H,
                                                     uint32_t* __restrict__ out)
{
    const int k = (int)blockIdx.y;
    const size_t n = (size_t)W * H;
    const T* img = proj + (size_t)k * n;
    float m = 0.0f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(pixel_f32(img, W, H, (int)(i % W), (int)(i / W))));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
        atomicMax(&out[k], __float_as_uint(m));
    }
}

// 2^e with 4 * maxabs * 2^e <= 2^15 (so |coefficient| <= 2^15 < 65504); 1 for a zero view.
__device__ __forceinline__ float patch16_scale(uint32_t maxabs_bits)
{
    const float m = __uint_as_float(maxabs_bits);
    if (!(m > 0.0f) || !(m < 3.0e38f)) return 1.0f;
    int e;
    frexpf(m, &e);  // m < 2^e
    return ldexpf(1.0f, 13 - e);
}

template <typename T>
__global__ __launch_bounds__(256) void patch16_kernel(const T* __restrict__ proj, int W, int H,
                                                      const uint32_t* __restrict__ maxabs,
                                                      f16x4_t* __restrict__ out, float* __restrict__ inv_scale)
{
    const int Wq = W + 2, Hq = H + 2;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int k = (int)blockIdx.z;
    const float sc = patch16_scale(maxabs[k]);
    if (c == 0 && blockIdx.y == 0) inv_scale[k] = 1.0f / sc;
    if (c >= Wq) return;
    const int r_begin = (int)blockIdx.y * kPatchRows, r_end = min(r_begin + kPatchRows, Hq);
    const T* img = proj + (size_t)k * W * H;
    const int i = c - 1;
    f16x4_t* dst = out + ((size_t)k * Hq + r_begin) * Wq + c;
    float a = pixel_f32(img, W, H, i, r_begin - 1) * sc, b = pixel_f32(img, W, H, i + 1, r_begin - 1) * sc;
    for (int r = r_begin; r < r_end; ++r, dst += Wq) {
        const float cc = pixel_f32(img, W, H, i, r) * sc, d = pixel_f32(img, W, H, i + 1, r) * sc;
        const float dx = b - a;
        f16x4_t q;
        q.x = (_Float16)a;
        q.y = (_Float16)dx;
        q.z = (_Float16)(cc - a);
        q.w = (_Float16)((d - cc) - dx);
        *dst = q;
        a = cc;
        b = d;
    }
}

template <class Src, bool PADDED, int TX>
hipError_t launch_zu(int zu, float* vol, const Box& box, const ViewConst* vc, int n, const Src& src,
                     const Cull& cl, int xcd_order, hipStream_t s)
{
    if (xcd_order >= 2) {  // the region split needs gx % ax == 0 and gy % ay == 0
        const int ax = xcd_order >> 1, ay = kXcds / ax;
        const int gx = (box.nx + TX - 1) / TX, gy = (box.ny + (kBlock / TX) - 1) / (kBlock / TX);
        if (gx % ax != 0 || gy % ay != 0) xcd_order = 0;
    }
    const dim3 block(kBlock, 1, 1);
    auto grid = [&](int z) {
        const long t = n_tiles(box.nx, box.ny, box.nz, z, TX);
        return dim3((unsigned)(xcd_order == 1 ? (t + kXcds - 1) / kXcds * kXcds : t));
    };
    const bool nt = !PADDED && TX == 64 && (double)box.nx * (double)box.ny * (double)box.nz * 4.0 >= (double)(1u << 28);
#define BP_LAUNCH(Z)                                                                                             \
    do {                                                                                                         \
        if constexpr (!PADDED && TX == 64) {                                                                     \
            if (nt) {                                                                                            \
                hipLaunchKernelGGL((backproject_kernel<Src, Z, PADDED, TX, true>), grid(Z), block, 0, s, vol, box, \
                                   vc, n, src, cl.bits, cl.words, cl.kbase, xcd_order);                          \
                break;                                                                                           \
            }                                                                                                    \
        }                                                                                                        \
        hipLaunchKernelGGL((backproject_kernel<Src, Z, PADDED, TX>), grid(Z), block, 0, s, vol, box, vc, n, src, \
                           cl.bits, cl.words, cl.kbase, xcd_order);                                              \
    } while (0)
    switch (zu) {
    case 1: BP_LAUNCH(1); break;
    case 2: BP_LAUNCH(2); break;
    case 4: BP_LAUNCH(4); break;
    case 8: BP_LAUNCH(8); break;
    default: return hipErrorInvalidValue;
    }
#undef BP_LAUNCH
    return hipGetLastError();
}

template <class Src, int TX>
hipError_t launch_zu_lds(int zu, float* vol, const Box& box, const ViewConst* vc, int n, const Src& src,
                         const uint2* fp, int xcd_order, bool poison, hipStream_t s)
{
    if (xcd_order >= 2) {
        const int ax = xcd_order >> 1, ay = kXcds / ax;
        const int gx = (box.nx + TX - 1) / TX, gy = (box.ny + (kBlock / TX) - 1) / (kBlock / TX);
        if (gx % ax != 0 || gy % ay != 0) xcd_order = 0;
    }
    const dim3 block(kBlock, 1, 1);
    auto grid = [&](int z) {
        const long t = n_tiles(box.nx, box.ny, box.nz, z, TX);
        return dim3((unsigned)(xcd_order == 1 ? (t + kXcds - 1) / kXcds * kXcds : t));
    };
#define BP_LAUNCH(Z)                                                                                     \
    hipLaunchKernelGGL((backproject_lds_kernel<Src, Z, TX>), grid(Z), block, 0, s, vol, box, vc, n, src, fp, \
                       xcd_order)
    if (poison) {
        if (zu != 8) return hipErrorInvalidValue;
        hipLaunchKernelGGL((backproject_lds_kernel<Src, 8, TX, true>), grid(8), block, 0, s, vol, box, vc, n, src, fp,
                           xcd_order);
        return hipGetLastError();
    }
    switch (zu) {
    case 1: BP_LAUNCH(1); break;
    case 2: BP_LAUNCH(2); break;
    case 4: BP_LAUNCH(4); break;
    case 8: BP_LAUNCH(8); break;
    default: return hipErrorInvalidValue;
    }
#undef BP_LAUNCH
    return hipGetLastError();
}

// Scratch of the allocation-free entry point (per-view constants and the clipping mask of a
// call).  Every call on a device shares that device's copy; calls that overlap on one device race.
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr)
{
    static std::mutex mu;
    static void* addr[kNoAllocMaxDevices] = {};
    if (device < 0 || device >= kNoAllocMaxDevices || !ptr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_prep_views(const float* mats, int n_views, const Box& box, bool column_ok, ViewConst* out,
                             hipStream_t s)
{
    const int threads = 64;
    hipLaunchKernelGGL(prep_views_kernel, dim3((unsigned)((n_views + threads - 1) / threads)), dim3(threads), 0,
                       s, mats, n_views, box, column_ok ? 1 : 0, out);
    return hipGetLastError();
}

hipError_t launch_patch(Dtype dt, const void* proj, int W, int H, int n, void* out, const ViewNeed& need,
                        hipStream_t s)
{
    const dim3 block(256, 1, 1);
    const dim3 grid((unsigned)((W + 2 + 255) / 256), (unsigned)((H + 2 + kPatchRows - 1) / kPatchRows), (unsigned)n);
    f32x4_t* q = (f32x4_t*)out;
    switch (dt) {
    case Dtype::F32:
        hipLaunchKernelGGL(patch_kernel<float>, grid, block, 0, s, (const float*)proj, W, H, q, need);
        break;
    case Dtype::F16:
        hipLaunchKernelGGL(patch_kernel<__half>, grid, block, 0, s, (const __half*)proj, W, H, q, need);
        break;
    case Dtype::BF16:
        hipLaunchKernelGGL(patch_kernel<uint16_t>, grid, block, 0, s, (const uint16_t*)proj, W, H, q, need);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_fill(void* p, size_t bytes, uint32_t word, hipStream_t s)
{
    const size_t n = bytes / 4;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
    if (n) hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, n, word);
    return hipGetLastError();
}

hipError_t launch_zero(uint32_t* p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_cull(const ViewConst* vc, int n_views, const Box& box, int z_unroll, int tile_x, int W, int H,
                       uint32_t* out, hipStream_t s)
{
    const int tx = tile_x, ty = kBlock / tile_x;
    const int gx = (box.nx + tx - 1) / tx, gy = (box.ny + ty - 1) / ty;
    const long tiles = n_tiles(box.nx, box.ny, box.nz, z_unroll, tile_x);
    const int words = cull_words(n_views);
    const long total = tiles * words;
    const int threads = 256;
    hipLaunchKernelGGL(cull_kernel, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s, vc,
                       n_views, box, tx, ty, z_unroll, gx, gy, (int)tiles, words, W, H, out);
    return hipGetLastError();
}

hipError_t launch_footprint(const ViewConst* vc, int n, const Box& box, int z_unroll, int tile_x, int W, int H,
                            bool raw, int direct_eighths, uint2* out, uint32_t* big, hipStream_t s)
{
    const int tx = tile_x, ty = kBlock / tile_x;
    const int gx = (box.nx + tx - 1) / tx, gy = (box.ny + ty - 1) / ty;
    const int gz = (box.nz + z_unroll - 1) / z_unroll;
    const long total = (long)gx * gy * n;
    const int threads = 256;
    hipLaunchKernelGGL(footprint_kernel, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s, vc,
                       n, box, tx, ty, z_unroll, gx, gy, gz, W, H, raw ? kStageMaxWidth * kRawRows : kStageRecords,
                       raw ? kStageMaxWidth - 1 : kStageMaxWidth, raw ? kRawRows - 1 : kStageMaxHeight,
                       direct_eighths, raw, out, big);
    return hipGetLastError();
}

hipError_t launch_patch16(Dtype dt, const void* proj, int W, int H, int n, void* out, uint32_t* maxabs,
                          float* inv_scale, hipStream_t s)
{
    // a fill kernel rather than a memset node, so that the call can be captured in a graph
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, maxabs, n);
    const dim3 rgrid(64, (unsigned)n), block(256, 1, 1);
    const dim3 grid((unsigned)((W + 2 + 255) / 256), (unsigned)((H + 2 + kPatchRows - 1) / kPatchRows), (unsigned)n);
    f16x4_t* q = (f16x4_t*)out;
    switch (dt) {
    case Dtype::F32:
        hipLaunchKernelGGL(maxabs_kernel<float>, rgrid, block, 0, s, (const float*)proj, W, H, maxabs);
        hipLaunchKernelGGL(patch16_kernel<float>, grid, block, 0, s, (const float*)proj, W, H, maxabs, q, inv_scale);
        break;
    case Dtype::F16:
        hipLaunchKernelGGL(maxabs_kernel<__half>, rgrid, block, 0, s, (const __half*)proj, W, H, maxabs);
        hipLaunchKernelGGL(patch16_kernel<__half>, grid, block, 0, s, (const __half*)proj, W, H, maxabs, q, inv_scale);
        break;
    case Dtype::BF16:
        hipLaunchKernelGGL(maxabs_kernel<uint16_t>, rgrid, block, 0, s, (const uint16_t*)proj, W, H, maxabs);
        hipLaunchKernelGGL(patch16_kernel<uint16_t>, grid, block, 0, s, (const uint16_t*)proj, W, H, maxabs, q,
                           inv_scale);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_backproject(Dtype dt, Layout layout, int zu, int tile_x, float* vol, const Box& box,
                              const ViewConst* vc, int n, const void* src, int W, int H, const Cull& cl,
                              int xcd_order, const float* inv_scale, const uint2* fp, const void* raw,
                              hipStream_t s, bool poison, bool single_taps)
{
    const uint8_t* base = (const uint8_t*)src;
    if (fp && raw && layout == Layout::Patch) {
        auto go = [&](auto tag) -> hipError_t {
            using T = decltype(tag);
            RawPatchSource<T> ps;
            ps.base = base;
            ps.W = W;
            ps.H = H;
            ps.raw = static_cast<const T*>(raw);
            switch (tile_x) {
            case 64: return launch_zu_lds<RawPatchSource<T>, 64>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
            case 32: return launch_zu_lds<RawPatchSource<T>, 32>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
            case 16: return launch_zu_lds<RawPatchSource<T>, 16>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
            case 8: return launch_zu_lds<RawPatchSource<T>, 8>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
            default: return hipErrorInvalidValue;
            }
        };
        switch (dt) {
        case Dtype::F32: return go(float{});
        case Dtype::F16: return go(__half{});
        case Dtype::BF16: return go(uint16_t{});
        }
        return hipErrorInvalidValue;
    }
    if (raw) return hipErrorInvalidValue;  // pixels are staged for FP32 records only
    if (fp && layout == Layout::Patch16) {
        const Patch16Source ps{base, W, H, inv_scale};
        switch (tile_x) {
        case 64: return launch_zu_lds<Patch16Source, 64>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
        case 32: return launch_zu_lds<Patch16Source, 32>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
        case 16: return launch_zu_lds<Patch16Source, 16>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
        case 8: return launch_zu_lds<Patch16Source, 8>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (fp && layout == Layout::Patch) {
        const PatchSource ps{base, W, H};
        switch (tile_x) {
        case 64: return launch_zu_lds<PatchSource, 64>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
        case 32: return launch_zu_lds<PatchSource, 32>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
        case 16: return launch_zu_lds<PatchSource, 16>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
        case 8: return launch_zu_lds<PatchSource, 8>(zu, vol, box, vc, n, ps, fp, xcd_order, poison, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (fp) return hipErrorInvalidValue;  // the plain path reads the caller's images
    if (layout == Layout::Patch16) {
        const Patch16Source ps{base, W, H, inv_scale};
        switch (tile_x) {
        case 64: return launch_zu<Patch16Source, true, 64>(zu, vol, box, vc, n, ps, cl, xcd_order, s);
        case 32: return launch_zu<Patch16Source, true, 32>(zu, vol, box, vc, n, ps, cl, xcd_order, s);
        case 16: return launch_zu<Patch16Source, true, 16>(zu, vol, box, vc, n, ps, cl, xcd_order, s);
        case 8: return launch_zu<Patch16Source, true, 8>(zu, vol, box, vc, n, ps, cl, xcd_order, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (layout == Layout::Patch) {
        const PatchSource ps{base, W, H};
        switch (tile_x) {
        case 64: return launch_zu<PatchSource, true, 64>(zu, vol, box, vc, n, ps, cl, xcd_order, s);
        case 32: return launch_zu<PatchSource, true, 32>(zu, vol, box, vc, n, ps, cl, xcd_order, s);
        case 16: return launch_zu<PatchSource, true, 16>(zu, vol, box, vc, n, ps, cl, xcd_order, s);
        case 8: return launch_zu<PatchSource, true, 8>(zu, vol, box, vc, n, ps, cl, xcd_order, s);
        default: return hipErrorInvalidValue;
        }
    }
    {
#define BP_CHECKED(...)                                                                                         \
    (tile_x == 16 ? launch_zu<CheckedSource<__VA_ARGS__>, false, 16>(zu, vol, box, vc, n, {base, W, H}, cl, xcd_order, s) \
                  : launch_zu<CheckedSource<__VA_ARGS__>, false, 64>(zu, vol, box, vc, n, {base, W, H}, cl, xcd_order, s))
        if (tile_x != 16 && tile_x != 64) return hipErrorInvalidValue;
        switch (dt) {
        case Dtype::F32: return single_taps || W < 2 ? BP_CHECKED(float, false) : BP_CHECKED(float, true);
        case Dtype::F16: return single_taps || W < 2 ? BP_CHECKED(__half, false) : BP_CHECKED(__half, true);
        case Dtype::BF16: return single_taps || W < 2 ? BP_CHECKED(uint16_t, false) : BP_CHECKED(uint16_t, true);
        }
#undef BP_CHECKED
    }
    return hipErrorInvalidValue;
}

}  // namespace bp
