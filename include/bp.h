/*
 * bp.h -- C ABI of the MI355X (gfx950) voxel-driven cone-beam back projector.
 *
 * The operation is the back projection of filtered, weighted projection
 * images into a voxel volume that RabbitCT benchmarks (Hofmann, Treibig,
 * Hager, Wellein, "Comparing the Performance of Different x86 SIMD
 * Instruction Sets for a Medical Imaging Application on Modern Multi- and
 * Manycore Chips", WPMVP'14, Sec. 4 and Sec. 4.1, Listing 1):
 *
 *   for every voxel (x, y, z) and every view k:
 *     X       = origin + voxel_size * (x, y, z)         voxel centre (world, mm)
 *     (u,v,w) = P_k (X, 1)                              3x4 projection matrix
 *     if w > 0:
 *       volume[x,y,z] += B_k(u/w, v/w) / w^2
 *
 * where B_k is the bilinear interpolant of image k with every pixel off the
 * detector taken as 0 (the zero-padded buffer of Sec. 5.1.1) and integer
 * pixel indices are floor(u/w), floor(v/w).  Arithmetic is FP32 (the
 * reciprocal of w uses the hardware reciprocal, as Sec. 5.1 does on the
 * CPUs); projections may be stored as FP32, FP16 or BF16 and are always
 * interpolated and accumulated in FP32.
 *
 * Memory layouts (all arrays dense, no padding):
 *   volume       FP32, voxel (x, y, z) at (z * ny + y) * nx + x  (x fastest,
 *                the VOL[z*L*L + y*L + x] layout of Listing 1 when nx=ny=nz=L).
 *   projections  n_views images of det_height rows by det_width columns of
 *                the context's dtype; pixel (i, j) of view k at
 *                (k * det_height + j) * det_width + i  (i = column, fast axis).
 *   matrices     n_views row-major 3x4 FP32 matrices; P_k[r][c] at 12 k + 4 r + c.
 *                (Listing 1 indexes its A column-major: A[3c + r] == P[r][c].)
 *
 * Ownership and concurrency: the caller owns every array.  volume,
 * projections and matrices are DEVICE pointers on the context's device; they
 * must stay valid and unmodified until the work enqueued on `stream` has
 * completed.  A context owns device scratch that every call reuses: per-view
 * constants, the staging copy of a pass of views (up to K (W+2)(H+2) x 16
 * bytes, 8 for compact 16-bit records: 1.2 GB at K = 64 and 1248 x 960; with
 * the default pixel stages only the views read directly get records; a call
 * of two or more passes staged ahead holds two such copies, see
 * BP_OPT_OVERLAP_STAGING), the footprint tables or clipping mask of the block
 * tiles, and a side stream with its events for the staging.  It grows on
 * demand (a growth waits for the device) and is freed by bp_destroy, so
 * calls on one context must not overlap: use one context per stream that
 * runs concurrently.  Creating a context allocates nothing.
 *
 * Errors: argument checks and scratch growth run on the host before anything
 * is enqueued, and a call they reject has enqueued nothing.  A launch failure
 * (BP_ERR_LAUNCH) can come after earlier passes were enqueued; the volume
 * then holds a partial sum.  Device faults surface at the caller's next
 * synchronisation of `stream`.
 * bp_last_error(ctx) describes the last failure of a call on that context.
 */
#ifndef BP_H
#define BP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bp_ctx_s *bp_ctx;

typedef enum {
    BP_OK = 0,
    BP_ERR_INVALID_ARG = 1,   /* null pointer, bad size, non-finite geometry, ... */
    BP_ERR_UNSUPPORTED = 2,   /* valid request the library cannot serve */
    BP_ERR_OUT_OF_MEMORY = 3, /* device scratch could not be allocated */
    BP_ERR_DEVICE = 4,        /* HIP runtime error outside a launch */
    BP_ERR_LAUNCH = 5         /* a kernel launch was rejected */
} bp_status;

typedef enum { BP_F32 = 0, BP_F16 = 1, BP_BF16 = 2 } bp_dtype;

/* How the views of a call reach the volume. */
typedef enum {
    BP_PATH_AUTO = 0,   /* the tuned choice for (dtype, volume size) */
    BP_PATH_PLAIN = 1,  /* one volume pass per view, taps read from the caller's images
                           with the per-tap detector bounds of Listing 1 (Sec. 4.1) */
    BP_PATH_FUSED = 2,  /* views_per_pass views per volume pass, accumulated in
                           registers; taps read from a zero-padded staging copy
                           (Sec. 5.1.1), so no per-tap bounds tests */
    BP_PATH_FUSED_DIRECT = 3 /* views_per_pass views per volume pass, taps read from
                           the caller's images with per-tap bounds (no staging copy):
                           for volumes small next to the projections, where writing
                           the staging copy would cost more than the taps save.
                           BP_PATH_AUTO takes it when the box has fewer than 64 x W x H
                           voxels for FP32 projections (40 x W x H for 16-bit ones) */
} bp_path;

typedef struct {
    int device;           /* HIP device ordinal */
    int det_width;        /* W, detector columns (1248 for the RabbitCT data) */
    int det_height;       /* H, detector rows (960) */
    bp_dtype proj_dtype;  /* storage type of the projections */
    bp_path path;         /* BP_PATH_AUTO picks a path per call */
    int views_per_pass;   /* K for the fused paths; 0 = tuned */
    int z_unroll;         /* voxels per thread along z (1, 2, 4 or 8); 0 = tuned */
    int tile_x;           /* columns along x per 256-thread block (8, 16, 32 or 64; the block is
                             tile_x x 256/tile_x columns); 0 = tuned.  The caller's-image
                             paths (PLAIN, FUSED_DIRECT) take 16 or 64 (others give 64). */
} bp_config;

/* Fill *cfg with defaults: device 0, 1248 x 960, FP32, AUTO, tuned K, z_unroll and tile_x. */
void bp_config_default(bp_config *cfg);

/* Create a context on cfg->device.  Validates cfg; allocates nothing on the device yet. */
bp_status bp_create(const bp_config *cfg, bp_ctx *out);

/* Destroy a context and free its scratch.  Synchronises the context's device
   first (its scratch may be in use by enqueued work).  NULL is a no-op. */
bp_status bp_destroy(bp_ctx ctx);

/*
 * Accumulate the back projection of n_views images into an L x L x L volume
 * (the cubic form of the Listing 1 interface; equivalent to bp_backproject_box with
 * nx = ny = nz = L).
 *
 *   volume      device FP32, L^3, ACCUMULATED (+=): zero it first for a fresh
 *               reconstruction; calls over consecutive chunks of views add up
 *               (view streaming and resume).  Must be 4-byte aligned.
 *   projections device, n_views images of the context's dtype and size.
 *   matrices    device FP32, n_views * 12.
 *   n_views     >= 1.
 *   L           >= 1, L^3 < 2^31.
 *   voxel_size  MM of Listing 1, > 0 and finite.
 *   origin      HOST pointer to 3 floats: world position of the centre of
 *               voxel (0, 0, 0).  The centred volume of Listing 1 has
 *               origin = -(L - 1) / 2 * voxel_size on each axis.
 *   stream      hipStream_t to enqueue on; NULL = the null stream.
 */
bp_status bp_backproject(bp_ctx ctx, float *volume, const void *projections,
                         const float *matrices, int n_views, int L, float voxel_size,
                         const float origin[3], void *stream);

/* As bp_backproject for an nx x ny x nz box of voxels (e.g. a z-slab of a
   larger volume, whose origin is the world centre of the box's first voxel). */
bp_status bp_backproject_box(bp_ctx ctx, float *volume, int nx, int ny, int nz,
                             const void *projections, const float *matrices, int n_views,
                             float voxel_size, const float origin[3], void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): bp_backproject_box with no allocation at all.  The
 * arguments, layouts, accumulation and checks are those of bp_backproject_box; the taps are read
 * from the caller's images (PLAIN when the context's path is PLAIN, else FUSED_DIRECT with the
 * context's K, z_unroll and tile width, K = 64 when not set), which gives the same bits as
 * bp_backproject_box on those paths.  Scratch (per-view constants and, when it fits beside
 * them, the clipping mask) lives in a static device array of 4 MiB that each device the library
 * runs on holds until the process ends; its address is looked up once per device (at
 * bp_create, else at this entry's first call on the device).  Limits: n_views <= 65536
 * (BP_ERR_UNSUPPORTED beyond); a call whose clipping mask does not fit computes every
 * (tile, view) instead (same bits).  Every call on a device shares that device's array:
 * calls that overlap on one device race -- serialise them (one stream, or events).  No
 * hipMalloc, hipFree or allocating library routine is called; timing events
 * (bp_enable_timing) are not recorded.
 */
bp_status bp_backproject_noalloc(bp_ctx ctx, float *volume, int nx, int ny, int nz,
                                 const void *projections, const float *matrices, int n_views,
                                 float voxel_size, const float origin[3], void *stream);

/* Override the per-call choices of a context (path, K, z_unroll, tile_x); 0 keeps the tuned value. */
bp_status bp_set_tuning(bp_ctx ctx, bp_path path, int views_per_pass, int z_unroll, int tile_x);

/*
 * Options (bit flags, default 0; results are equal whatever the flags, up to
 * FP32 rounding for BP_OPT_NO_COLUMN and FP16 rounding for BP_OPT_COMPACT_STAGING):
 *   BP_OPT_NO_CULL    do not skip (tile, view) pairs whose whole tile projects
 *                     off the detector (the clipping mask of Sec. 5)
 *   BP_OPT_NO_COLUMN  do not specialise views whose matrix has P[0][2] = P[2][2] = 0
 *                     (u and w constant along z, as for a circular orbit about z)
 *   BP_OPT_COMPACT_STAGING  FP16/BF16 projections: stage them as compact FP16
 *                     bilinear-patch coefficients (8 bytes per pixel, scaled per
 *                     view by a power of two; adds the rounding of the pixel
 *                     differences to FP16, ~2^-11 relative) instead of the
 *                     default, which treats them as FP32 projections: their
 *                     pixels (exactly widened) staged in LDS and FP32
 *                     coefficients for the views read directly
 *   BP_OPT_WIDE_STAGING  FP16/BF16 projections: the default FP32 staging, named
 *                     (with BP_OPT_COMPACT_STAGING: an error)
 *   BP_OPT_DIRECT_TAPS  fused path: read every tap directly through the vector
 *                     L1 cache.  By default the fused path copies, for every
 *                     (block tile, view), the tile's footprint of the staging
 *                     buffer into LDS with coalesced row loads and reads the
 *                     taps from there, for all views but a share of them
 *                     (bp_set_tap_split) that still read directly, so that the
 *                     pass draws on both paths at once.  Results are
 *                     bit-identical either way.
 *   BP_OPT_SERIAL_STAGING   fused path: stage each pass's views on the caller's
 *                     stream just before the pass.
 *   BP_OPT_OVERLAP_STAGING  fused path, calls of two or more passes: stage pass
 *                     p + 1 on a side stream of the context (default priority,
 *                     ordered after the caller's stream by events) while pass p
 *                     runs, into the other half of a two-pass staging buffer.
 *                     Neither flag: overlapped for compact 16-bit records,
 *                     serial for FP32 records (whose staging contends with the
 *                     pass for the vector memory path).  Both flags: an error.
 *                     Results are bit-identical in every case.
 *   BP_OPT_STAGE_RECORDS  fused path, FP32 staging: copy the LDS footprints
 *                     as 16-byte patch records rather than as the caller's
 *                     pixels in FP32 (from which each update then forms its
 *                     patch with the staging copy's own FP32 operations).
 *                     Bit-identical.
 *   BP_OPT_POISON_STAGING  testing aid, fused path: fill each pass's staging copy
 *                     with NaN before the views are staged into it, and (LDS
 *                     stage, z_unroll 8 only; other z-unrolls: BP_ERR_UNSUPPORTED)
 *                     the LDS stage before each footprint is copied in, so that
 *                     any read of an element the staging did not write shows as
 *                     NaN in the result.  Results are bit-identical otherwise.
 *   BP_OPT_SINGLE_TAPS  paths on the caller's images (PLAIN, FUSED_DIRECT): load
 *                     each tap on its own instead of each row's pixel pair as one
 *                     load (8 bytes of FP32, 4 bytes of FP16/BF16).  Bit-identical.
 *
 *   Tile order (which blocks run together; results are identical in every order):
 *   default           XCD-private regions: all XCDs work through the same z-layer of
 *                     tiles, each on its own ax x (8/ax) region of it (ax = 8 unless set
 *                     below; plain order if the tile grid does not divide)
 *   BP_OPT_XCD_REGION(ax)  choose ax in {1, 2, 4, 8}
 *   BP_OPT_PLAIN_ORDER     tiles in plain order, x fastest
 *   BP_OPT_XCD_ORDER  deal contiguous z-ranges of tiles to the 8 XCDs (measured slowest)
 */
#define BP_OPT_NO_CULL 1
#define BP_OPT_NO_COLUMN 2
#define BP_OPT_XCD_ORDER 4
#define BP_OPT_WIDE_STAGING 8
#define BP_OPT_PLAIN_ORDER 16
#define BP_OPT_XCD_REGION_SHIFT 5
#define BP_OPT_XCD_REGION_MASK (15 << BP_OPT_XCD_REGION_SHIFT)
#define BP_OPT_XCD_REGION(ax) ((ax) << BP_OPT_XCD_REGION_SHIFT)
#define BP_OPT_DIRECT_TAPS (1 << 9)
#define BP_OPT_SERIAL_STAGING (1 << 10)
#define BP_OPT_OVERLAP_STAGING (1 << 11)
#define BP_OPT_STAGE_RECORDS (1 << 12)
#define BP_OPT_POISON_STAGING (1 << 13)
#define BP_OPT_SINGLE_TAPS (1 << 14)
#define BP_OPT_COMPACT_STAGING (1 << 15)
bp_status bp_set_options(bp_ctx ctx, int options);

/* Fused path with LDS staging: of every 8 consecutive views of a pass, how many
 * read their taps directly through L1 instead of from the LDS stage (0..8);
 * -1 restores the tuned share (0 for pixel stages, 4 for FP32 record stages, 3 for compact records).
 * Results are bit-identical for every share. */
bp_status bp_set_tap_split(bp_ctx ctx, int direct_eighths);

/* The choices the next call of size nx*ny*nz with n_views views will use; any output may be NULL.
 * direct_taps: 1 if the fused pass reads every tap through L1 (no LDS stage) -- set by
 * BP_OPT_DIRECT_TAPS, or chosen on boxes of 2e8 voxels or more for FP32 staging as records
 * (BP_OPT_STAGE_RECORDS) unless a tap split is set.  Pixel stages (the default) and compact
 * records keep the stage: K = 64 for FP32 pixel stages of fewer than 2e8 voxels, every view in
 * one pass (at most 512) for the other pixel stages, K = 128 for records. */
bp_status bp_query_plan(bp_ctx ctx, int nx, int ny, int nz, int n_views,
                        bp_path *path, int *views_per_pass, int *z_unroll, int *tile_x, int *direct_taps);

/* Bytes of device scratch that the next call of size nx*ny*nz with n_views views on this context
 * needs with its current settings: per-view constants, the staging copy of a pass (two when the
 * next pass is staged while one runs), staging scales, the footprint tables or the clipping
 * mask.  A context keeps the largest scratch of its calls until bp_destroy, so a caller that
 * admits work by device memory (a server) counts max(held, this) per context.
 * BP_ERR_INVALID_ARG for a null ctx or bytes, or a size below 1. */
bp_status bp_query_scratch(bp_ctx ctx, int nx, int ny, int nz, int n_views, size_t *bytes);

/*
 * Compose the projection matrices of a circular cone-beam orbit on the host
 * in FP64 and round them once to FP32 (the per-view A_i of Sec. 4, which
 * RabbitCT ships with its data).  Convention: source at
 * SID (cos t, sin t, 0), detector centre at -(SDD - SID)(cos t, sin t, 0),
 * detector columns along (-sin t, cos t, 0), rows along (0, 0, 1), pixel
 * (i, j) centred at ((W-1)/2, (H-1)/2) + (i, j) * pitch on the detector.
 * Normalised so that w = depth along the principal ray / SID (w = 1 at the
 * isocentre; 1/w^2 is then the FDK distance weight).
 *
 *   angles   host, n_views angles t_k in radians.
 *   out_f64  host, n_views * 12 doubles, or NULL.
 *   out_f32  host, n_views * 12 floats (rounded to nearest), or NULL.
 * Returns BP_ERR_INVALID_ARG for non-positive or non-finite distances, pitch
 * or detector size, or SDD <= 0.
 */
bp_status bp_circular_matrices(const double *angles, int n_views, double sid, double sdd,
                               double pitch, int det_width, int det_height,
                               double *out_f64, float *out_f32);

/*
 * Kernel timing for measurement.  When enabled, every kernel launch of the
 * context is bracketed by two HIP events on the call's stream (the events add
 * a few microseconds per launch).  bp_kernel_timing synchronises on those
 * events and returns, for one kernel kind, the summed elapsed time in
 * milliseconds and the number of launches since timing was last enabled or
 * reset.  Kinds: 0 = back-projection pass, 1 = zero-padded staging copy,
 * 2 = per-view constants.
 */
bp_status bp_enable_timing(bp_ctx ctx, int enable);
bp_status bp_kernel_timing(bp_ctx ctx, int kind, double *total_ms, long long *launches);

const char *bp_status_string(bp_status s);
const char *bp_last_error(bp_ctx ctx);

/* Library version, "major.minor.patch". */
const char *bp_version(void);

/* ------------------------------------------------------------------------
 * FDK pre-processing: raw projections -> the filtered, weighted projections
 * that bp_backproject consumes (Sec. 4 describes the benchmark input as
 * filtered and weighted; the paper does not spell the two steps out, so
 * this library uses the Feldkamp-Davis-Kress pre-processing):
 *
 *   c[j][i]    = SDD / sqrt(SDD^2 + u_i^2 + v_j^2)        cosine weight,
 *                u_i = (i - (W-1)/2) pitch, v_j = (j - (H-1)/2) pitch (mm)
 *   q[k][j][i] = tau * sum_{m=0}^{W-1} h(i - m) c[j][m] p[k][j][m]
 *                (linear convolution along each detector row: no samples
 *                beyond the row), tau = pitch * SID / SDD, and h the discrete
 *                Ram-Lak kernel of Kak and Slaney: h(0) = 1/(4 tau^2),
 *                h(odd n) = -1/(pi n tau)^2, h(even n != 0) = 0.
 *
 * Arithmetic is FP64 (by FFT of length 4096, so det_width <= 2048); each
 * output is rounded once to FP32, and from there to FP16 or BF16 (round to
 * nearest even) if asked.
 *
 * Layouts: raw and filtered are n_views x det_height x det_width, pixel (i, j)
 * of view k at (k * det_height + j) * det_width + i, DEVICE pointers on the
 * handle's device; raw is FP32, filtered is out_dtype.  The caller owns both;
 * they must stay valid until the work on `stream` has completed.  filtered
 * may be the same pointer as raw for FP32 output (in place); any other
 * overlap is an error.  A handle owns two small read-only device tables
 * (96 KiB), so concurrent calls on one handle are safe.
 *
 * Errors as above: checks run before anything is enqueued; a call that
 * returns anything but BP_OK has enqueued nothing.
 * ------------------------------------------------------------------------ */
typedef struct bp_fdk_s *bp_fdk;

typedef struct {
    int device;     /* HIP device index */
    int det_width;  /* W: columns per row, 1 <= W <= 2048 (else BP_ERR_UNSUPPORTED) */
    int det_height; /* H: rows per view, >= 1 */
    double pitch;   /* detector pixel pitch, mm, > 0 */
    double sid;     /* source to isocentre distance, mm, > 0 */
    double sdd;     /* source to detector distance, mm, > 0 */
} bp_fdk_config;

/* RabbitCT-like defaults: device 0, 1248 x 960 pixels of 0.32 mm, SID 800, SDD 1200. */
void bp_fdk_config_default(bp_fdk_config *cfg);

/* Allocate the handle and build its tables (synchronously).  On failure
 * *out is NULL: BP_ERR_INVALID_ARG (bad config), BP_ERR_UNSUPPORTED (width),
 * BP_ERR_DEVICE, BP_ERR_OUT_OF_MEMORY or BP_ERR_LAUNCH. */
bp_status bp_fdk_create(const bp_fdk_config *cfg, bp_fdk *out);

/* Weight and filter n_views raw views into `filtered`, asynchronously on
 * `stream` (a hipStream_t; NULL = the null stream).  out_dtype: BP_F32,
 * BP_F16 or BP_BF16. */
bp_status bp_fdk_filter(bp_fdk f, const float *raw, void *filtered, bp_dtype out_dtype, int n_views,
                        void *stream);

/* Waits for the device, then frees the handle.  bp_fdk_destroy(NULL) is a no-op. */
bp_status bp_fdk_destroy(bp_fdk f);

/* Description of the last failed call on the handle. */
const char *bp_fdk_last_error(bp_fdk f);


#ifdef __cplusplus
}
#endif

#endif /* BP_H */
