// fdk_internal.h -- launch interface of the FDK pre-processing kernels
// (fdk_kernels.hip), used by the C ABI in fdk_api.cpp.
#pragma once

#include <hip/hip_runtime.h>

namespace bp {
namespace fdk {

// Transform length of the row convolution: rows of up to kTransform / 2 samples.
constexpr int kTransform = 4096;
constexpr int kMaxWidth = kTransform / 2;

// Detector geometry of the cosine weight SDD / sqrt(SDD^2 + u^2 + v^2), with
// u = (i - half_w) * pitch and v = (j - half_h) * pitch.
struct Geometry {
    double half_w, half_h, pitch, sdd, sdd2;
};

// Fill the twiddle table tw[m] = exp(-2 pi i m / N) and the real ramp spectrum
// (tau and 1 / N folded in) of the Ram-Lak kernel truncated to |n| < W.
hipError_t launch_setup(double2* tw, double* spectrum, int W, double tau, hipStream_t s);

// Weight and filter n_rows rows of W samples (row r belongs to detector row r % H).
// out_dtype: 0 FP32, 1 FP16, 2 BF16.  out may equal raw for FP32 output.
hipError_t launch_filter(const float* raw, void* out, int out_dtype, long n_rows, int W, int H, const Geometry& g,
                         const double2* tw, const double* spectrum, hipStream_t s);

}  // namespace fdk
}  // namespace bp
