/*
 * Sanitizer driver of the FP64 oracle (bp_oracle.c) -- TEST INFRASTRUCTURE.
 *
 * Built with AddressSanitizer + UndefinedBehaviorSanitizer and, separately, with
 * ThreadSanitizer; runs the block and voxel-list entries (plain and magnitude mode) with
 * several threads on a small random problem, including voxels behind the source and positions
 * off the detector, and checks that the voxel-list entry reproduces the block entry bit for
 * bit and that the magnitude is never below |V|.  Exit status 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_backproject(double *vol, int x0, int y0, int z0, int nx, int ny, int nz, const float *proj, int W,
                       int H, int n_views, const double *P, double MM, const double *O, int n_threads);
int oracle_backproject_abs(double *vol, int x0, int y0, int z0, int nx, int ny, int nz, const float *proj, int W,
                           int H, int n_views, const double *P, double MM, const double *O, int n_threads);
int oracle_backproject_points(double *out, const int *xyz, long n, const float *proj, int W, int H, int n_views,
                              const double *P, double MM, const double *O, int n_threads);

static unsigned long long rng_state = 88172645463325252ULL;
static double uniform(void) /* xorshift64, in [0, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0;
}

int main(void)
{
    enum { W = 23, H = 17, N = 5, L = 11 };
    float *proj = malloc(sizeof(float) * W * H * N);
    double P[12 * N];
    for (int i = 0; i < W * H * N; ++i) proj[i] = (float)(2.0 * uniform() - 1.0);
    for (int k = 0; k < N; ++k) {
        const double a = 0.7 * k;
        /* a pinhole looking at the origin from distance 30 (voxels span +-25: some lie behind it) */
        const double c = cos(a), s = sin(a);
        const double row0[4] = {-s * 20.0, c * 20.0, 0.0, 11.0 * 30.0};
        const double row1[4] = {0.0, 0.0, 20.0, 8.0 * 30.0};
        const double row2[4] = {-c, -s, 0.0, 30.0};
        for (int j = 0; j < 4; ++j) {
            P[12 * k + j] = row0[j] / 30.0 + 0.1 * row2[j] * (k == 3);
            P[12 * k + 4 + j] = row1[j] / 30.0;
            P[12 * k + 8 + j] = row2[j] / 30.0;
        }
    }
    const double MM = 5.0, O[3] = {-25.0, -25.0, -25.0};
    double *V = calloc(L * L * L, sizeof(double)), *A = calloc(L * L * L, sizeof(double));
    if (oracle_backproject(V, 0, 0, 0, L, L, L, proj, W, H, N, P, MM, O, 4) != 0) return 1;
    if (oracle_backproject_abs(A, 0, 0, 0, L, L, L, proj, W, H, N, P, MM, O, 3) != 0) return 2;
    int xyz[3 * 64];
    double pts[64];
    memset(pts, 0, sizeof pts);
    for (int m = 0; m < 64; ++m)
        for (int a = 0; a < 3; ++a) xyz[3 * m + a] = (int)(uniform() * L);
    if (oracle_backproject_points(pts, xyz, 64, proj, W, H, N, P, MM, O, 5) != 0) return 3;
    int nonzero = 0;
    for (int m = 0; m < 64; ++m) {
        const double v = V[((long)xyz[3 * m + 2] * L + xyz[3 * m + 1]) * L + xyz[3 * m]];
        if (pts[m] != v) return 4;
    }
    for (int i = 0; i < L * L * L; ++i) {
        if (A[i] < fabs(V[i])) return 5;
        nonzero += V[i] != 0.0;
    }
    if (nonzero == 0) return 6;
    /* invalid arguments are rejected */
    if (oracle_backproject(NULL, 0, 0, 0, L, L, L, proj, W, H, N, P, MM, O, 2) != -1) return 7;
    printf("oracle driver ok: %d non-zero voxels\n", nonzero);
    free(proj);
    free(V);
    free(A);
    return 0;
}
