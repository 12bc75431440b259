// Sanitizer driver of the library's host-only matrix composition (bp_circular_matrices) --
// TEST INFRASTRUCTURE.  Built with AddressSanitizer + UndefinedBehaviorSanitizer; composes the
// matrices of orbits of several sizes into exactly sized buffers, checks the isocentre maps to
// the detector centre with w = 1, and that invalid arguments are rejected.  Exit 0 on success.
#include <cmath>
#include <cstdio>
#include <vector>

#include "bp.h"

int main()
{
    for (int n : {1, 2, 7, 496}) {
        std::vector<double> ang(n), p64(12 * (size_t)n);
        std::vector<float> p32(12 * (size_t)n);
        for (int k = 0; k < n; ++k) ang[k] = 3.4906585 * k / n;
        if (bp_circular_matrices(ang.data(), n, 800.0, 1200.0, 0.32, 1248, 960, p64.data(), p32.data()) != BP_OK)
            return 1;
        for (int k = 0; k < n; ++k) {
            const double* P = &p64[12 * (size_t)k];
            const double w = P[11], s = P[3] / w, t = P[7] / w;  // the isocentre (0, 0, 0)
            if (std::fabs(w - 1.0) > 1e-12 || std::fabs(s - 623.5) > 1e-9 || std::fabs(t - 479.5) > 1e-9) return 2;
            for (int i = 0; i < 12; ++i)
                if (p32[12 * (size_t)k + i] != (float)P[i]) return 3;
        }
        // either output alone
        if (bp_circular_matrices(ang.data(), n, 800.0, 1200.0, 0.32, 1248, 960, nullptr, p32.data()) != BP_OK) return 4;
        if (bp_circular_matrices(ang.data(), n, 800.0, 1200.0, 0.32, 1248, 960, p64.data(), nullptr) != BP_OK) return 5;
    }
    double a = 0.0, out[12];
    if (bp_circular_matrices(&a, 1, -1.0, 1200.0, 0.32, 8, 8, out, nullptr) != BP_ERR_INVALID_ARG) return 6;
    if (bp_circular_matrices(&a, 1, 800.0, NAN, 0.32, 8, 8, out, nullptr) != BP_ERR_INVALID_ARG) return 7;
    if (bp_circular_matrices(&a, 0, 800.0, 1200.0, 0.32, 8, 8, out, nullptr) != BP_ERR_INVALID_ARG) return 8;
    if (bp_circular_matrices(nullptr, 1, 800.0, 1200.0, 0.32, 8, 8, out, nullptr) != BP_ERR_INVALID_ARG) return 9;
    std::printf("geometry driver ok\n");
    return 0;
}
