// fdk_kernels.hip -- FDK pre-processing of raw cone-beam projections: cosine
// weighting and row-wise Ram-Lak filtering, the step that turns detector data
// into the filtered, weighted projections that the back projection consumes
// (Sec. 4 describes its input that way).  FP64 arithmetic, FP32 input, output
// rounded once to FP32 (then to FP16 / BF16 if asked).
//
// One workgroup filters two detector rows at once: row A as the real part and
// row B as the imaginary part of one complex sequence.  The ramp kernel is real
// and even, so its spectrum G is real and
//     IDFT(DFT(a + i b) * G) = (a (*) g) + i (b (*) g),
// which needs no separation step.  The convolution is linear: a row of W <= 2048
// samples is zero-padded to N = 4096 >= 2W - 1, so the circular convolution of
// length N equals the linear one on the W output samples.
//
// The length-4096 DFT runs as three radix-16 passes (4096 = 16^3), 16 points per
// thread in registers, with the exchanges between passes through a padded LDS
// buffer:
//   n = 256 a + b,  k = k1 + 16 (c1 + 16 c2)
//   pass 1 (thread b):         DFT16 over a, twiddle w4096^(b k1)
//   pass 2 (thread (k1, d)):   DFT16 over c of element 16 c + d, twiddle w256^(d c1)
//   pass 3 (thread k1 + 16 c1): DFT16 over d -> X[k1 + 16 c1 + 256 c2]
// After pass 3 thread t holds X[t + 256 c2], c2 = 0..15, which is exactly the
// input layout of pass 1 (thread b holds x[256 a + b]); so the inverse transform
// starts in registers, and it leaves thread t with output sample t + 256 c2:
// coalesced loads and stores at both ends.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdk_internal.h"

namespace bp {
namespace fdk {

namespace {

constexpr int kN = kTransform;
constexpr int kThreads = 256;
constexpr int kStride = 257;  // complex values per LDS row: consecutive k1 rows shift by 4 banks

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}

// In-place 4-point DFT; Dir = -1 forward (w4 = -i), +1 inverse (w4 = +i).
template <int Dir>
__device__ __forceinline__ void dft4(double2& x0, double2& x1, double2& x2, double2& x3)
{
    const double2 a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = csub(x1, x3);
    const double2 jd = Dir < 0 ? make_double2(d.y, -d.x) : make_double2(-d.y, d.x);  // (Dir i) d
    x0 = cadd(a, c);
    x2 = csub(a, c);
    x1 = cadd(b, jd);
    x3 = csub(b, jd);
}

// cos and sin of 2 pi m / 16 for m = 0..9
__device__ __forceinline__ double2 w16(int m, int dir)
{
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;  // pi/8
    constexpr double r2 = 0.70710678118654752440;
    double c = 1.0, s = 0.0;
    switch (m) {
    case 1: c = c1; s = s1; break;
    case 2: c = r2; s = r2; break;
    case 3: c = s1; s = c1; break;
    case 4: c = 0.0; s = 1.0; break;
    case 6: c = -r2; s = r2; break;
    case 9: c = -c1; s = -s1; break;
    default: break;
    }
    return make_double2(c, dir * s);
}

// 16-point DFT of v[a], a = a0 + 4 a1.  Output V[k] lands in v[perm16(k)].
__device__ __forceinline__ constexpr int perm16(int k) { return 4 * (k & 3) + (k >> 2); }

template <int Dir>
__device__ __forceinline__ void dft16(double2 (&v)[16])
{
#pragma unroll
    for (int a0 = 0; a0 < 4; ++a0) dft4<Dir>(v[a0], v[a0 + 4], v[a0 + 8], v[a0 + 12]);
    // now v[a0 + 4 k1] = sum_a1 x[a0 + 4 a1] w4^(a1 k1); twiddle by w16^(a0 k1)
#pragma unroll
    for (int a0 = 1; a0 < 4; ++a0)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) v[a0 + 4 * k1] = cmul(v[a0 + 4 * k1], w16(a0 * k1, Dir));
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<Dir>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] = V[k1 + 4 k2]
}

// twiddle w^m (forward: exp(-2 pi i m / N), inverse: its conjugate)
template <int Dir>
__device__ __forceinline__ double2 twiddle(double2 v, const double2* __restrict__ tw, int m)
{
    const double2 w = tw[m];
    return Dir < 0 ? cmul(v, w) : cmulc(v, w);
}

// Passes 2 and 3 and the exchanges before them; pass 1 output is in v (V[k1] at perm16(k1)),
// already twiddled.  On return thread t holds X[t + 256 c2] at v[perm16(c2)].
template <int Dir>
__device__ __forceinline__ void passes_23(double2 (&v)[16], double2* buf, const double2* __restrict__ tw)
{
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) buf[k1 * kStride + t] = v[perm16(k1)];
    __syncthreads();
    {
        const int k1 = t >> 4, d = t & 15;
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = buf[k1 * kStride + 16 * c + d];
        dft16<Dir>(v);
#pragma unroll
        for (int c1 = 1; c1 < 16; ++c1) v[perm16(c1)] = twiddle<Dir>(v[perm16(c1)], tw, 16 * d * c1);
        __syncthreads();  // every pass-2 read is done before the buffer is overwritten
#pragma unroll
        for (int c1 = 0; c1 < 16; ++c1) buf[k1 * kStride + 16 * c1 + d] = v[perm16(c1)];
    }
    __syncthreads();
    {
        const int k1 = t & 15, c1 = t >> 4;
#pragma unroll
        for (int d = 0; d < 16; ++d) v[d] = buf[k1 * kStride + 16 * c1 + d];
        dft16<Dir>(v);
    }
}

// Pass 1 on registers that hold x[256 a + t] in v[a]; output twiddled, V[k1] at v[perm16(k1)].
template <int Dir>
__device__ __forceinline__ void pass_1(double2 (&v)[16], const double2* __restrict__ tw)
{
    const int t = (int)threadIdx.x;
    dft16<Dir>(v);
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) v[perm16(k1)] = twiddle<Dir>(v[perm16(k1)], tw, t * k1);
}

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf / nan
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <typename T>
__device__ __forceinline__ void store(void* out, size_t idx, double x);
template <>
__device__ __forceinline__ void store<float>(void* out, size_t idx, double x)
{
    static_cast<float*>(out)[idx] = (float)x;
}
template <>
__device__ __forceinline__ void store<_Float16>(void* out, size_t idx, double x)
{
    static_cast<_Float16*>(out)[idx] = (_Float16)(float)x;
}
template <>
__device__ __forceinline__ void store<uint16_t>(void* out, size_t idx, double x)
{
    static_cast<uint16_t*>(out)[idx] = bf16_rne((float)x);
}

// Rows r = view * H + j of the stack, two per workgroup (the last one alone if the count is odd).
template <typename T>
__global__ __launch_bounds__(kThreads) void fdk_kernel(const float* raw, void* out,
                                                       long n_rows, int W, int H, Geometry g,
                                                       const double2* __restrict__ tw,
                                                       const double* __restrict__ spectrum)
{
    __shared__ double2 buf[16 * kStride];
    const int t = (int)threadIdx.x;
    const long r0 = 2 * (long)blockIdx.x;
    const bool two = r0 + 1 < n_rows;
    const float* a = raw + (size_t)r0 * W;
    const float* b = a + W;
    const double va = ((double)(int)(r0 % H) - g.half_h) * g.pitch;
    const double vb = ((double)(int)((r0 + 1) % H) - g.half_h) * g.pitch;
    const double sa = fma(va, va, g.sdd2), sb = fma(vb, vb, g.sdd2);

    double2 v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < kN / 2 / kThreads; ++i) {  // W <= N / 2: only a < 8 can be inside the row
        const int n = kThreads * i + t;
        if (n < W) {
            const double u = ((double)n - g.half_w) * g.pitch;
            const double ca = g.sdd / sqrt(fma(u, u, sa));
            const double cb = g.sdd / sqrt(fma(u, u, sb));
            v[i].x = (double)a[n] * ca;
            if (two) v[i].y = (double)b[n] * cb;
        }
    }
    // forward transform
    pass_1<-1>(v, tw);
    passes_23<-1>(v, buf, tw);
    // thread t holds X[t + 256 c2]: apply the ramp (with tau and 1 / N folded in)
#pragma unroll
    for (int c2 = 0; c2 < 16; ++c2) {
        const double s = spectrum[t + kThreads * c2];
        v[perm16(c2)].x *= s;
        v[perm16(c2)].y *= s;
    }
    // inverse transform: v[a] must hold element 256 a + t
    double2 x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = v[perm16(i)];
    pass_1<1>(x, tw);
    __syncthreads();  // the forward pass-3 reads are done before the buffer is reused
    passes_23<1>(x, buf, tw);
#pragma unroll
    for (int c2 = 0; c2 < kN / 2 / kThreads; ++c2) {
        const int n = t + kThreads * c2;
        if (n < W) {
            const double2 y = x[perm16(c2)];
            store<T>(out, (size_t)r0 * W + n, y.x);
            if (two) store<T>(out, (size_t)(r0 + 1) * W + n, y.y);
        }
    }
}

__global__ void twiddle_kernel(double2* __restrict__ tw)
{
    const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m >= kN) return;
    double s, c;
    sincospi(2.0 * (double)m / (double)kN, &s, &c);
    tw[m] = make_double2(c, -s);
}

// G[k] = (tau / N) * sum_{|n| < W} h(n) cos(2 pi n k / N), h the discrete Ram-Lak kernel:
// h(0) = 1 / (4 tau^2), h(odd n) = -1 / (pi n tau)^2, h(even n) = 0.
__global__ void spectrum_kernel(double* __restrict__ G, int W, double tau)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= kN) return;
    constexpr double kPi = 3.14159265358979323846;
    double odd = 0.0;
    for (int n = W - 1 - ((W - 1) % 2 == 0 ? 1 : 0); n >= 1; n -= 2) {  // largest odd n < W first (small terms first)
        const int m = (int)(((long long)n * k) % kN);
        odd += cospi(2.0 * (double)m / (double)kN) / ((double)n * (double)n);
    }
    const double hc = 0.25 / (tau * tau) - 2.0 * odd / (kPi * kPi * tau * tau);
    G[k] = hc * tau / (double)kN;
}

}  // namespace

hipError_t launch_setup(double2* tw, double* spectrum, int W, double tau, hipStream_t s)
{
    hipLaunchKernelGGL(twiddle_kernel, dim3(kN / 256), dim3(256), 0, s, tw);
    hipLaunchKernelGGL(spectrum_kernel, dim3(kN / 256), dim3(256), 0, s, spectrum, W, tau);
    return hipGetLastError();
}

hipError_t launch_filter(const float* raw, void* out, int out_dtype, long n_rows, int W, int H, const Geometry& g,
                         const double2* tw, const double* spectrum, hipStream_t s)
{
    const dim3 grid((unsigned)((n_rows + 1) / 2)), block(kThreads);
    switch (out_dtype) {
    case 0: hipLaunchKernelGGL(fdk_kernel<float>, grid, block, 0, s, raw, out, n_rows, W, H, g, tw, spectrum); break;
    case 1: hipLaunchKernelGGL(fdk_kernel<_Float16>, grid, block, 0, s, raw, out, n_rows, W, H, g, tw, spectrum); break;
    case 2: hipLaunchKernelGGL(fdk_kernel<uint16_t>, grid, block, 0, s, raw, out, n_rows, W, H, g, tw, spectrum); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdk
}  // namespace bp
