/*
 * bp_oracle.c -- FP64 reference back projector.  TEST INFRASTRUCTURE ONLY.
 *
 * This file is the oracle the GPU path is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * The product library never links, includes or calls it, and the two share
 * no code.  It is deliberately plain: one voxel at a time, views in order,
 * double precision, no blocking, no fusion, no reordering.
 *
 * What it computes -- voxel-driven cone-beam back projection as defined by the
 * RabbitCT reference module (Hofmann, Treibig, Hager, Wellein, WPMVP'14,
 * Sec. 4.1 "Algorithm"), one projection image per view:
 *
 *   for every voxel of the block and every view k = 0 .. N-1:
 *     X          = origin + MM * (x, y, z)            voxel centre, world coords
 *     (u, v, w)  = P_k (X, 1)                         homogeneous detector coords
 *     (s, t)     = (u / w, v / w)                     position on the detector
 *     B_k(s, t)  = sum over pixels (i, j) of I_k[j][i] tent(s - i) tent(t - j),
 *                  tent(r) = max(0, 1 - |r|), pixels off the detector 0
 *                  (the bilinear interpolant of the zero-extended image; only
 *                  the 2 x 2 pixels around (s, t) have a non-zero weight)
 *     V[x, y, z] += B_k(s, t) / w^2                   inverse-square weight
 *
 * A second mode sums |B_k(s, t) / w^2| instead: the magnitude of what the
 * back projection adds up, which sets how much any finite-precision
 * evaluation of the sum can be off (the sum's conditioning).
 *
 * Readings where the printed listing is silent or slips (each is also listed
 * in the design notes of the repository):
 *   - the integer pixel index is floor(), not truncation toward zero, so the
 *     interpolant is continuous at the left/top detector edge;
 *   - the column bound is the image width W (the row stride) and the row
 *     bound is the height H;
 *   - A_k is given row-major, P[r][c] at 12k + 4r + c;
 *   - the origin is given per axis (voxel (0,0,0) centre);
 *   - a view contributes 0 to a voxel unless w > 0 (voxel in front of the
 *     source);
 *   - positions with s <= -1, s >= W, t <= -1 or t >= H contribute 0
 *     exactly (every pixel with a weight is off the detector), which is tested
 *     before the float-to-integer conversion so huge positions cannot overflow it.
 *
 * Threads split the block into independent z-planes, the task decomposition
 * of the paper's Sec. 5; each voxel is owned by exactly one thread.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <unistd.h>

/* one pixel of the zero-extended image */
static double pixel(const float *img, int W, int H, long i, long j)
{
    if (i < 0 || i >= W || j < 0 || j >= H)
        return 0.0;
    return (double)img[j * (long)W + i];
}

/* hat function of unit half-width */
static double tent(double r)
{
    r = fabs(r);
    return r < 1.0 ? 1.0 - r : 0.0;
}

/* Bilinear interpolant of the zero-extended image at detector position (s, t): each pixel
 * weighted by tent(s - i) tent(t - j).  The weights vanish outside the 2 x 2 pixels
 * i = floor(s), floor(s) + 1 and j = floor(t), floor(t) + 1, so only those are summed;
 * positions with s <= -1, s >= W, t <= -1 or t >= H weigh only pixels off the detector and
 * give 0 (tested first, so that huge positions never reach the integer conversion). */
static double interpolate(const float *img, int W, int H, double s, double t)
{
    if (!(s > -1.0 && s < (double)W && t > -1.0 && t < (double)H))
        return 0.0;
    const long c0 = (long)floor(s), r0 = (long)floor(t);
    double sum = 0.0;
    for (long j = r0; j <= r0 + 1; ++j) {
        const double wt = tent(t - (double)j);
        for (long i = c0; i <= c0 + 1; ++i)
            sum += pixel(img, W, H, i, j) * tent(s - (double)i) * wt;
    }
    return sum;
}

/* contribution of view k to the voxel centred at world position (wx, wy, wz) */
static double contribution(const float *img, int W, int H, const double *A,
                           double wx, double wy, double wz)
{
    double u = A[0] * wx + A[1] * wy + A[2] * wz + A[3];
    double v = A[4] * wx + A[5] * wy + A[6] * wz + A[7];
    double w = A[8] * wx + A[9] * wy + A[10] * wz + A[11];
    if (!(w > 0.0))
        return 0.0;
    double val = interpolate(img, W, H, u / w, v / w);
    return val / (w * w);
}

typedef struct {
    double *vol;
    int x0, y0, z0, nx, ny, nz;
    const float *proj;
    int W, H, n_views;
    const double *P;
    double MM;
    double O[3];
    int absolute;  /* sum |contribution| instead of the contribution */
    int first_plane, plane_step;
} job_t;

static void *run_planes(void *arg)
{
    const job_t *jb = (const job_t *)arg;
    const long img_size = (long)jb->W * jb->H;
    for (int iz = jb->first_plane; iz < jb->nz; iz += jb->plane_step) {
        double wz = jb->O[2] + jb->MM * (double)(jb->z0 + iz);
        for (int iy = 0; iy < jb->ny; ++iy) {
            double wy = jb->O[1] + jb->MM * (double)(jb->y0 + iy);
            for (int ix = 0; ix < jb->nx; ++ix) {
                double wx = jb->O[0] + jb->MM * (double)(jb->x0 + ix);
                double *voxel = &jb->vol[((long)iz * jb->ny + iy) * jb->nx + ix];
                double sum = *voxel;
                for (int k = 0; k < jb->n_views; ++k) {
                    const double c = contribution(jb->proj + k * img_size, jb->W, jb->H,
                                                  jb->P + 12 * (long)k, wx, wy, wz);
                    sum += jb->absolute ? fabs(c) : c;
                }
                *voxel = sum;
            }
        }
    }
    return NULL;
}

/*
 * Accumulate the back projection of n_views images into a block of the volume.
 *
 *   vol      nx*ny*nz doubles, index (iz*ny + iy)*nx + ix, holds voxel
 *            (x0+ix, y0+iy, z0+iz); the result is ADDED to what it holds.
 *   proj     n_views images of H rows by W columns, FP32, pixel (i, j) of
 *            view k at (k*H + j)*W + i.
 *   P        n_views row-major 3x4 matrices, FP64.
 *   MM       voxel size; O[3] world position of the centre of voxel (0,0,0).
 *   n_threads  <= 0 picks the number of online CPUs.
 * Returns 0, or -1 for an invalid argument.
 */
static int backproject_block(double *vol, int x0, int y0, int z0, int nx, int ny, int nz,
                             const float *proj, int W, int H, int n_views,
                             const double *P, double MM, const double *O, int n_threads, int absolute)
{
    if (!vol || !proj || !P || !O || nx < 0 || ny < 0 || nz < 0 || W < 1 || H < 1 ||
        n_views < 0)
        return -1;
    if (n_threads <= 0)
        n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > nz)
        n_threads = nz > 0 ? nz : 1;

    job_t *jobs = (job_t *)calloc((size_t)n_threads, sizeof(job_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return -1;
    }
    for (int t = 0; t < n_threads; ++t) {
        job_t *jb = &jobs[t];
        jb->vol = vol;
        jb->x0 = x0; jb->y0 = y0; jb->z0 = z0;
        jb->nx = nx; jb->ny = ny; jb->nz = nz;
        jb->proj = proj; jb->W = W; jb->H = H; jb->n_views = n_views;
        jb->P = P; jb->MM = MM;
        jb->O[0] = O[0]; jb->O[1] = O[1]; jb->O[2] = O[2];
        jb->absolute = absolute;
        jb->first_plane = t;
        jb->plane_step = n_threads;
    }
    int started = 0;
    for (int t = 1; t < n_threads; ++t) {
        if (pthread_create(&tid[t], NULL, run_planes, &jobs[t]) != 0)
            break;
        started = t;
    }
    /* planes of threads that failed to start are done here, in order */
    for (int t = started + 1; t < n_threads; ++t)
        run_planes(&jobs[t]);
    run_planes(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tid[t], NULL);
    free(jobs);
    free(tid);
    return 0;
}

int oracle_backproject(double *vol, int x0, int y0, int z0, int nx, int ny, int nz,
                       const float *proj, int W, int H, int n_views,
                       const double *P, double MM, const double *O, int n_threads)
{
    return backproject_block(vol, x0, y0, z0, nx, ny, nz, proj, W, H, n_views, P, MM, O, n_threads, 0);
}

/* As oracle_backproject, adding |contribution| of every view (the sum's magnitude). */
int oracle_backproject_abs(double *vol, int x0, int y0, int z0, int nx, int ny, int nz,
                           const float *proj, int W, int H, int n_views,
                           const double *P, double MM, const double *O, int n_threads)
{
    return backproject_block(vol, x0, y0, z0, nx, ny, nz, proj, W, H, n_views, P, MM, O, n_threads, 1);
}

typedef struct {
    double *out;
    const int *xyz;
    long n;
    const float *proj;
    int W, H, n_views;
    const double *P;
    double MM;
    double O[3];
    int absolute;
    long first, step;
} points_job_t;

static void *run_points(void *arg)
{
    const points_job_t *jb = (const points_job_t *)arg;
    const long img_size = (long)jb->W * jb->H;
    for (long m = jb->first; m < jb->n; m += jb->step) {
        double wx = jb->O[0] + jb->MM * (double)jb->xyz[3 * m];
        double wy = jb->O[1] + jb->MM * (double)jb->xyz[3 * m + 1];
        double wz = jb->O[2] + jb->MM * (double)jb->xyz[3 * m + 2];
        double sum = jb->out[m];
        for (int k = 0; k < jb->n_views; ++k) {
            const double c = contribution(jb->proj + k * img_size, jb->W, jb->H, jb->P + 12 * (long)k, wx, wy, wz);
            sum += jb->absolute ? fabs(c) : c;
        }
        jb->out[m] = sum;
    }
    return NULL;
}

/*
 * The same back projection for an arbitrary list of voxels: out[m] += sum over
 * views for voxel (xyz[3m], xyz[3m+1], xyz[3m+2]).  Used to sample a large
 * volume uniformly.  Returns 0, or -1 for an invalid argument.
 */
static int backproject_list(double *out, const int *xyz, long n, const float *proj, int W, int H,
                            int n_views, const double *P, double MM, const double *O, int n_threads,
                            int absolute)
{
    if (!out || !xyz || !proj || !P || !O || n < 0 || W < 1 || H < 1 || n_views < 0)
        return -1;
    if (n_threads <= 0)
        n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > n)
        n_threads = n > 0 ? (int)n : 1;
    points_job_t *jobs = (points_job_t *)calloc((size_t)n_threads, sizeof(points_job_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return -1;
    }
    for (int t = 0; t < n_threads; ++t) {
        points_job_t *jb = &jobs[t];
        jb->out = out; jb->xyz = xyz; jb->n = n;
        jb->proj = proj; jb->W = W; jb->H = H; jb->n_views = n_views;
        jb->P = P; jb->MM = MM;
        jb->O[0] = O[0]; jb->O[1] = O[1]; jb->O[2] = O[2];
        jb->absolute = absolute;
        jb->first = t; jb->step = n_threads;
    }
    int started = 0;
    for (int t = 1; t < n_threads; ++t) {
        if (pthread_create(&tid[t], NULL, run_points, &jobs[t]) != 0)
            break;
        started = t;
    }
    for (int t = started + 1; t < n_threads; ++t)
        run_points(&jobs[t]);
    run_points(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tid[t], NULL);
    free(jobs);
    free(tid);
    return 0;
}

int oracle_backproject_points(double *out, const int *xyz, long n, const float *proj, int W, int H,
                              int n_views, const double *P, double MM, const double *O, int n_threads)
{
    return backproject_list(out, xyz, n, proj, W, H, n_views, P, MM, O, n_threads, 0);
}

/* As oracle_backproject_points, adding |contribution| of every view. */
int oracle_backproject_points_abs(double *out, const int *xyz, long n, const float *proj, int W, int H,
                                  int n_views, const double *P, double MM, const double *O, int n_threads)
{
    return backproject_list(out, xyz, n, proj, W, H, n_views, P, MM, O, n_threads, 1);
}

/* Bilinear interpolant of one zero-extended image at one position (exported for pins). */
double oracle_interpolate(const float *img, int W, int H, double s, double t)
{
    return interpolate(img, W, H, s, t);
}
