// synth_kernels.hip -- seeded synthetic input generation on the GPU (not part
// of the back projector; libbpsynth.so is loaded only by the input generator).
//
// Analytic line integrals of a phantom of ellipsoids along source -> pixel
// rays of a circular cone-beam scan: for an ellipsoid (x - c)^T M (x - c) = 1
// and a unit ray x = S + lam d, the chord is 2 sqrt(B^2 - A C) / A with
// A = d^T M d, B = d^T M (S - c), C = (S - c)^T M (S - c) - 1; densities add.
#include <hip/hip_runtime.h>

namespace {

__global__ __launch_bounds__(256) void line_integrals_kernel(double* __restrict__ out,
                                                             const double* __restrict__ frames, int W, int H,
                                                             double pitch, const double* __restrict__ ell,
                                                             int n_ell)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int j = (int)blockIdx.y;
    const int k = (int)blockIdx.z;
    if (i >= W) return;
    const double* f = frames + 12 * (size_t)k;  // S, D, e_u, e_v
    const double du = (i - 0.5 * (W - 1)) * pitch, dv = (j - 0.5 * (H - 1)) * pitch;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = f[3 + a] + du * f[6 + a] + dv * f[9 + a] - f[a];
    const double inv = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) d[a] *= inv;
    double sum = 0.0;
    for (int e = 0; e < n_ell; ++e) {
        const double* p = ell + 13 * (size_t)e;  // c(3), M(9) row-major, density
        const double q[3] = {f[0] - p[0], f[1] - p[1], f[2] - p[2]};
        double Md[3], Mq[3];
        for (int r = 0; r < 3; ++r) {
            Md[r] = p[3 + 3 * r] * d[0] + p[4 + 3 * r] * d[1] + p[5 + 3 * r] * d[2];
            Mq[r] = p[3 + 3 * r] * q[0] + p[4 + 3 * r] * q[1] + p[5 + 3 * r] * q[2];
        }
        const double A = d[0] * Md[0] + d[1] * Md[1] + d[2] * Md[2];
        const double B = d[0] * Mq[0] + d[1] * Mq[1] + d[2] * Mq[2];
        const double C = q[0] * Mq[0] + q[1] * Mq[1] + q[2] * Mq[2] - 1.0;
        const double disc = B * B - A * C;
        if (disc > 0.0) sum += p[12] * 2.0 * sqrt(disc) / A;
    }
    out[((size_t)k * H + j) * W + i] = sum;
}

}  // namespace

// out: device, n_views*H*W doubles; frames: device, n_views*12 doubles (S, D,
// e_u, e_v per view); ell: device, n_ell*13 doubles (centre, M row-major,
// density).  Enqueued on `stream`; returns a hipError_t code.
extern "C" int bpsynth_line_integrals(double* out, const double* frames, int n_views, int W, int H, double pitch,
                                      const double* ell, int n_ell, void* stream)
{
    if (!out || !frames || !ell || n_views < 1 || W < 1 || H < 1 || n_ell < 0) return (int)hipErrorInvalidValue;
    const dim3 block(256, 1, 1), grid((unsigned)((W + 255) / 256), (unsigned)H, (unsigned)n_views);
    hipLaunchKernelGGL(line_integrals_kernel, grid, block, 0, (hipStream_t)stream, out, frames, W, H, pitch, ell,
                       n_ell);
    return (int)hipGetLastError();
}
