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
// The length-4096 DFT runs as four radix-8 passes (4096 = 8^4), 8 points per
// thread of a 512-thread workgroup, with the exchanges between passes through
// an LDS buffer laid out so that every access of a wavefront spreads over all
// banks:
//   n = 512 a + b,  k = k1 + 8 (c1 + 8 (l1 + 8 l2))
//   pass 1 (thread b):                 DFT8 over a, twiddle w4096^(b k1)
//   pass 2 (thread (k1, d)):           DFT8 over c of element 64 c + d, twiddle w512^(d c1)
//   pass 3 (thread (k1, c1, f)):       DFT8 over e of element 8 e + f, twiddle w64^(f l1)
//   pass 4 (thread k1 + 8 c1 + 64 l1): DFT8 over f -> X[k1 + 8 c1 + 64 l1 + 512 l2]
// After pass 4 thread t holds X[t + 512 l2], l2 = 0..7, which is exactly the
// input layout of pass 1 (thread b holds x[512 a + b]); so the inverse transform
// starts in registers, and it leaves thread t with output sample t + 512 l2:
// coalesced loads and stores at both ends.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdk_internal.h"

namespace bp {
namespace fdk {

namespace {

constexpr int kN = kTransform;
constexpr int kThreads = 512;
constexpr int kIn = kN / 2 / kThreads;  // W <= N / 2: only elements 512 a + t with a < 4 can be inside a row
// LDS layouts of the three exchanges (complex values)
__device__ __forceinline__ int lds_y(int k1, int b) { return k1 * 512 + b; }
__device__ __forceinline__ int lds_z(int k1, int c1, int d) { return k1 * 576 + c1 * 72 + d; }
__device__ __forceinline__ int lds_q(int k1, int c1, int l1, int f) { return f * 513 + l1 * 64 + c1 * 8 + k1; }
constexpr int kLds = 4600;  // largest index of the three layouts + 1

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
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

// In-place 8-point DFT, natural order in and out: DFT4 of the even and of the odd
// elements, then V[k] = E[k] + w8^k O[k] and V[k + 4] = E[k] - w8^k O[k].
template <int Dir>
__device__ __forceinline__ void dft8(double2 (&v)[8])
{
    constexpr double r2 = 0.70710678118654752440;
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<Dir>(e0, e1, e2, e3);
    dft4<Dir>(o0, o1, o2, o3);
    // w8^1 = (r2, Dir r2), w8^2 = Dir i, w8^3 = (-r2, Dir r2)
    const double2 t1 = make_double2(r2 * (o1.x - Dir * o1.y), r2 * (o1.y + Dir * o1.x));
    const double2 t2 = Dir < 0 ? make_double2(o2.y, -o2.x) : make_double2(-o2.y, o2.x);
    const double2 t3 = make_double2(-r2 * (o3.x + Dir * o3.y), r2 * (Dir * o3.x - o3.y));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, t1);
    v[5] = csub(e1, t1);
    v[2] = cadd(e2, t2);
    v[6] = csub(e2, t2);
    v[3] = cadd(e3, t3);
    v[7] = csub(e3, t3);
}

// v[k] *= w^(m k) for k = 1..7, w = exp(Dir 2 pi i / N).  One entry of the table
// tw[j] = exp(-2 pi i j / N) gives w^m and its powers are formed by products (at most
// three roundings each, FP64): one table load per pass instead of seven, which halved
// the kernel's time (the seven-load form streamed the 64 KB table through L2 per pass).
template <int Dir>
__device__ __forceinline__ void twiddle(double2 (&v)[8], const double2* __restrict__ tw, int m)
{
    double2 p1 = tw[m];
    if (Dir > 0) p1.y = -p1.y;
    const double2 p2 = cmul(p1, p1), p3 = cmul(p2, p1), p4 = cmul(p2, p2);
    v[1] = cmul(v[1], p1);
    v[2] = cmul(v[2], p2);
    v[3] = cmul(v[3], p3);
    v[4] = cmul(v[4], p4);
    v[5] = cmul(v[5], cmul(p4, p1));
    v[6] = cmul(v[6], cmul(p3, p3));
    v[7] = cmul(v[7], cmul(p4, p3));
}

// One transform: v[a] holds element 512 a + t on entry; X[t + 512 l2] in v[l2] on return.
// The caller separates uses of buf by a barrier.
template <int Dir>
__device__ __forceinline__ void fft4096(double2 (&v)[8], double2* buf, const double2* __restrict__ tw)
{
    const int t = (int)threadIdx.x;
    dft8<Dir>(v);  // pass 1: over a
    twiddle<Dir>(v, tw, t);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) buf[lds_y(k1, t)] = v[k1];
    __syncthreads();
    {
        const int k1 = t >> 6, d = t & 63;  // pass 2: over c of element 64 c + d
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = buf[lds_y(k1, 64 * c + d)];
        dft8<Dir>(v);
        twiddle<Dir>(v, tw, 8 * d);
        __syncthreads();
#pragma unroll
        for (int c1 = 0; c1 < 8; ++c1) buf[lds_z(k1, c1, d)] = v[c1];
    }
    __syncthreads();
    {
        const int f = t & 7, c1 = (t >> 3) & 7, k1 = t >> 6;  // pass 3: over e of element 8 e + f
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = buf[lds_z(k1, c1, 8 * e + f)];
        dft8<Dir>(v);
        twiddle<Dir>(v, tw, 64 * f);
        __syncthreads();
#pragma unroll
        for (int l1 = 0; l1 < 8; ++l1) buf[lds_q(k1, c1, l1, f)] = v[l1];
    }
    __syncthreads();
    {
        const int k1 = t & 7, c1 = (t >> 3) & 7, l1 = t >> 6;  // pass 4: over f
#pragma unroll
        for (int f = 0; f < 8; ++f) v[f] = buf[lds_q(k1, c1, l1, f)];
        dft8<Dir>(v);
    }
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
__global__ __launch_bounds__(kThreads) void fdk_kernel(const float* raw, void* out, long n_rows, int W, int H,
                                                       Geometry g, const double2* __restrict__ tw,
                                                       const double* __restrict__ spectrum)
{
    __shared__ double2 buf[kLds];
    const int t = (int)threadIdx.x;
    const long r0 = 2 * (long)blockIdx.x;
    const bool two = r0 + 1 < n_rows;
    const float* a = raw + (size_t)r0 * W;
    const float* b = a + W;
    const double va = ((double)(int)(r0 % H) - g.half_h) * g.pitch;
    const double vb = ((double)(int)((r0 + 1) % H) - g.half_h) * g.pitch;
    const double sa = fma(va, va, g.sdd2), sb = fma(vb, vb, g.sdd2);

    double2 v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < kIn; ++i) {
        const int n = kThreads * i + t;
        if (n < W) {
            const double u = ((double)n - g.half_w) * g.pitch;
            v[i].x = (double)a[n] * (g.sdd / sqrt(fma(u, u, sa)));
            if (two) v[i].y = (double)b[n] * (g.sdd / sqrt(fma(u, u, sb)));
        }
    }
    fft4096<-1>(v, buf, tw);
    // thread t holds X[t + 512 l2]: apply the ramp (with tau and 1 / N folded in)
#pragma unroll
    for (int l2 = 0; l2 < 8; ++l2) {
        const double s = spectrum[t + kThreads * l2];
        v[l2].x *= s;
        v[l2].y *= s;
    }
    __syncthreads();  // the forward pass-4 reads are done before the buffer is reused
    fft4096<1>(v, buf, tw);  // v[a] holds element 512 a + t, as pass 1 wants
#pragma unroll
    for (int l2 = 0; l2 < kIn; ++l2) {
        const int n = t + kThreads * l2;
        if (n < W) {
            store<T>(out, (size_t)r0 * W + n, v[l2].x);
            if (two) store<T>(out, (size_t)(r0 + 1) * W + n, v[l2].y);
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
