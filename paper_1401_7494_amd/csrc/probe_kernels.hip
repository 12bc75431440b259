// probe_kernels.hip -- measured roofs for the back projector on gfx950 (libbpprobe.so).
//
// The paper measures the limits its kernels run against with microbenchmarks
// (Table 1: the "Node Update" streaming read-modify-write bandwidth; Sec. 6:
// instruction counts and cycles).  These kernels measure the same limits on
// MI355X:
//   probe_update  a[i] += c over a large FP32 array: the 8 bytes per voxel
//                 update of the plain form (one read and one write per element),
//                 with 16-byte vector accesses, grid-stride
//   probe_copy    b[i] = a[i]: a plain copy of known size (the yardstick of the
//                 HBM traffic counters)
//   probe_valu    a long run of one VALU instruction class per lane (inline
//                 assembly: exactly that instruction, on 8 independent registers
//                 per lane), so that instructions per second per class follow
//                 from the time: the FP32 FMA, multiply, add and subtract, the
//                 reciprocal of w, the conversions, floor and fraction of Part 2,
//                 the clamp (med3), the integer address arithmetic, selects and
//                 the mixed-precision FMA of the 16-bit records
// Every access is in bounds by construction (grid-stride loops bounded by n;
// the VALU probe writes one value per launched thread into an array the caller
// sizes from probe_valu_threads).  Launch-only: the caller times them with
// events on the same stream.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__global__ __launch_bounds__(256) void update_kernel(float* __restrict__ a, long n, float c)
{
    const long n4 = n / 4;
    float4* a4 = reinterpret_cast<float4*>(a);
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        float4 v = a4[i];
        v.x += c;
        v.y += c;
        v.z += c;
        v.w += c;
        a4[i] = v;
    }
    for (long i = 4 * n4 + (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] += c;
}

__global__ __launch_bounds__(256) void copy_kernel(const float* __restrict__ a, float* __restrict__ b, long n)
{
    const long n4 = n / 4;
    const float4* a4 = reinterpret_cast<const float4*>(a);
    float4* b4 = reinterpret_cast<float4*>(b);
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) b4[i] = a4[i];
    for (long i = 4 * n4 + (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// One instruction of the class on register r (operands 1.0001 and 0.5 where it takes more).
#define PROBE_OP(OP, r) asm volatile(OP : "+v"(r) : "v"(k1), "v"(k2))

template <int CLASS>
__global__ __launch_bounds__(256) void valu_kernel(float* __restrict__ out, int iters)
{
    float r0 = threadIdx.x * 1e-3f, r1 = r0 + 1.0f, r2 = r0 + 2.0f, r3 = r0 + 3.0f;
    float r4 = r0 + 4.0f, r5 = r0 + 5.0f, r6 = r0 + 6.0f, r7 = r0 + 7.0f;
    const float k1 = 1.0001f, k2 = 0.5f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#define EIGHT(OP)                                                                                   \
    PROBE_OP(OP, r0); PROBE_OP(OP, r1); PROBE_OP(OP, r2); PROBE_OP(OP, r3);                         \
    PROBE_OP(OP, r4); PROBE_OP(OP, r5); PROBE_OP(OP, r6); PROBE_OP(OP, r7)
            if constexpr (CLASS == 0) { EIGHT("v_fma_f32 %0, %0, %1, %2"); }
            else if constexpr (CLASS == 1) { EIGHT("v_mul_f32 %0, %0, %1"); }
            else if constexpr (CLASS == 2) { EIGHT("v_add_f32 %0, %0, %1"); }
            else if constexpr (CLASS == 3) { EIGHT("v_rcp_f32 %0, %0"); }
            else if constexpr (CLASS == 4) { EIGHT("v_cvt_flr_i32_f32 %0, %0"); }
            else if constexpr (CLASS == 5) { EIGHT("v_fract_f32 %0, %0"); }
            else if constexpr (CLASS == 6) { EIGHT("v_med3_f32 %0, %0, %1, %2"); }
            else if constexpr (CLASS == 7) { EIGHT("v_mad_u32_u24 %0, %0, %1, %2"); }
            else if constexpr (CLASS == 8) { EIGHT("v_floor_f32 %0, %0"); }
            else if constexpr (CLASS == 9) { EIGHT("v_cvt_i32_f32 %0, %0"); }
            else if constexpr (CLASS == 10) { EIGHT("v_cvt_f32_i32 %0, %0"); }
            else if constexpr (CLASS == 11) { EIGHT("v_add_u32 %0, %0, %1"); }
            else if constexpr (CLASS == 12) { EIGHT("v_and_b32 %0, %0, %1"); }
            else if constexpr (CLASS == 13) { EIGHT("v_lshl_add_u32 %0, %0, 2, %1"); }
            else if constexpr (CLASS == 14) { EIGHT("v_mul_u32_u24 %0, %0, %1"); }
            else if constexpr (CLASS == 15) { EIGHT("v_max_f32 %0, %0, %1"); }
            else if constexpr (CLASS == 16) { EIGHT("v_sub_f32 %0, %0, %1"); }
            else if constexpr (CLASS == 17) { EIGHT("v_fma_mix_f32 %0, %0, %1, %2 op_sel_hi:[1,0,0]"); }
            else if constexpr (CLASS == 18) { EIGHT("v_cndmask_b32 %0, %0, %1, vcc"); }
            else if constexpr (CLASS == 19) { EIGHT("v_fmac_f32 %0, %1, %2"); }
            else if constexpr (CLASS == 20) { EIGHT("v_add_lshl_u32 %0, %0, %1, 2"); }
#undef EIGHT
        }
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = r0 + r1 + r2 + r3 + r4 + r5 + r6 + r7;
}
#undef PROBE_OP

}  // namespace

extern "C" {

// Instructions of the class per launched lane: iters x 16.
long long probe_valu_per_lane(int iters) { return 16LL * iters; }

// Threads a probe_valu launch runs (the size of `out`, in floats).
long long probe_valu_threads(int blocks) { return 256LL * blocks; }

int probe_update(float* a, long n, float c, int blocks, void* stream)
{
    if (!a || n < 0 || blocks < 1 || (reinterpret_cast<uintptr_t>(a) & 15u)) return 1;
    hipLaunchKernelGGL(update_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), a, n, c);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

int probe_copy(const float* a, float* b, long n, int blocks, void* stream)
{
    if (!a || !b || n < 0 || blocks < 1 || ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15u))
        return 1;
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), a, b, n);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

// klass: 0 fma, 1 mul, 2 add, 3 rcp, 4 cvt_flr_i32, 5 fract, 6 med3, 7 mad_u32_u24, 8 floor,
// 9 cvt_i32_f32, 10 cvt_f32_i32, 11 add_u32, 12 and_b32, 13 lshl_add_u32, 14 mul_u32_u24, 15 max_f32,
// 16 sub_f32, 17 fma_mix_f32, 18 cndmask_b32, 19 fmac_f32, 20 add_lshl_u32.
// out: probe_valu_threads(blocks) floats (device).
int probe_valu(int klass, float* out, int blocks, int iters, void* stream)
{
    if (!out || blocks < 1 || iters < 1) return 1;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 g(blocks), b(256);
    switch (klass) {
    case 0: hipLaunchKernelGGL(valu_kernel<0>, g, b, 0, s, out, iters); break;
    case 1: hipLaunchKernelGGL(valu_kernel<1>, g, b, 0, s, out, iters); break;
    case 2: hipLaunchKernelGGL(valu_kernel<2>, g, b, 0, s, out, iters); break;
    case 3: hipLaunchKernelGGL(valu_kernel<3>, g, b, 0, s, out, iters); break;
    case 4: hipLaunchKernelGGL(valu_kernel<4>, g, b, 0, s, out, iters); break;
    case 5: hipLaunchKernelGGL(valu_kernel<5>, g, b, 0, s, out, iters); break;
    case 6: hipLaunchKernelGGL(valu_kernel<6>, g, b, 0, s, out, iters); break;
    case 7: hipLaunchKernelGGL(valu_kernel<7>, g, b, 0, s, out, iters); break;
    case 8: hipLaunchKernelGGL(valu_kernel<8>, g, b, 0, s, out, iters); break;
    case 9: hipLaunchKernelGGL(valu_kernel<9>, g, b, 0, s, out, iters); break;
    case 10: hipLaunchKernelGGL(valu_kernel<10>, g, b, 0, s, out, iters); break;
    case 11: hipLaunchKernelGGL(valu_kernel<11>, g, b, 0, s, out, iters); break;
    case 12: hipLaunchKernelGGL(valu_kernel<12>, g, b, 0, s, out, iters); break;
    case 13: hipLaunchKernelGGL(valu_kernel<13>, g, b, 0, s, out, iters); break;
    case 14: hipLaunchKernelGGL(valu_kernel<14>, g, b, 0, s, out, iters); break;
    case 15: hipLaunchKernelGGL(valu_kernel<15>, g, b, 0, s, out, iters); break;
    case 16: hipLaunchKernelGGL(valu_kernel<16>, g, b, 0, s, out, iters); break;
    case 17: hipLaunchKernelGGL(valu_kernel<17>, g, b, 0, s, out, iters); break;
    case 18: hipLaunchKernelGGL(valu_kernel<18>, g, b, 0, s, out, iters); break;
    case 19: hipLaunchKernelGGL(valu_kernel<19>, g, b, 0, s, out, iters); break;
    case 20: hipLaunchKernelGGL(valu_kernel<20>, g, b, 0, s, out, iters); break;
    default: return 1;
    }
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // extern "C"
