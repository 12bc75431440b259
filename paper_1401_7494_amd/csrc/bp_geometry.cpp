// bp_geometry.cpp -- host FP64 composition of circular-orbit projection
// matrices (the per-view 3x4 A_i of Hofmann et al., WPMVP'14, Sec. 4).
//
// A view is a pinhole camera P = K [R | -R S] / SID with
//   R = rows (e_u, e_v, n): detector column axis, row axis, principal ray
//   S = source position
//   K = [[f, 0, c_u], [0, f, c_v], [0, 0, 1]], f = SDD / pitch (pixels),
//       principal point (c_u, c_v) = ((W-1)/2, (H-1)/2)
// Dividing by SID makes w = n.(X - S) / SID, 1 at the isocentre.
#include "../../include/bp.h"

#include <cmath>

extern "C" bp_status bp_circular_matrices(const double* angles, int n_views, double sid, double sdd,
                                          double pitch, int det_width, int det_height, double* out_f64,
                                          float* out_f32)
{
    if (!angles || n_views < 1 || (!out_f64 && !out_f32)) return BP_ERR_INVALID_ARG;
    if (!std::isfinite(sid) || !std::isfinite(sdd) || !std::isfinite(pitch) || !(sid > 0.0) ||
        !(sdd > 0.0) || !(pitch > 0.0) || det_width < 1 || det_height < 1)
        return BP_ERR_INVALID_ARG;
    const double f = sdd / pitch;
    const double cu = 0.5 * (det_width - 1), cv = 0.5 * (det_height - 1);
    for (int k = 0; k < n_views; ++k) {
        const double th = angles[k];
        if (!std::isfinite(th)) return BP_ERR_INVALID_ARG;
        const double c = std::cos(th), s = std::sin(th);
        const double S[3] = {sid * c, sid * s, 0.0};
        const double R[3][3] = {{-s, c, 0.0}, {0.0, 0.0, 1.0}, {-c, -s, 0.0}};
        double t[3];  // t = -R S
        for (int r = 0; r < 3; ++r) t[r] = -(R[r][0] * S[0] + R[r][1] * S[1] + R[r][2] * S[2]);
        const double K[3][3] = {{f, 0.0, cu}, {0.0, f, cv}, {0.0, 0.0, 1.0}};
        double P[3][4];
        for (int r = 0; r < 3; ++r) {
            for (int col = 0; col < 4; ++col) {
                double acc = 0.0;
                for (int m = 0; m < 3; ++m) acc += K[r][m] * (col < 3 ? R[m][col] : t[m]);
                P[r][col] = acc / sid;
            }
        }
        for (int r = 0; r < 3; ++r)
            for (int col = 0; col < 4; ++col) {
                if (out_f64) out_f64[12 * k + 4 * r + col] = P[r][col];
                if (out_f32) out_f32[12 * k + 4 * r + col] = static_cast<float>(P[r][col]);
            }
    }
    return BP_OK;
}
