/*
 * cbct.h -- C ABI of libcbct.so: the circular-orbit cone-beam projector pair
 * on AMD Instinct MI355X (gfx950).
 *
 * Operators (arXiv 2512.21180, Sec. 2.2, definition of the cone-beam
 * transform and of the backprojection as its adjoint; Alg. 1 applies both to
 * multi-channel stacks and at several resolutions):
 *
 *   A   (forward projector)  line integrals of a voxel volume along the rays
 *                            from the source to every detector pixel;
 *   A^T (adjoint)            the exact Euclidean transpose of A, computed as
 *                            a gather (every voxel written once, no atomics).
 *
 * Geometry (Sec. 2.2): isocenter at the origin, rotation axis z.  For source
 * angle th the source is S = sid (cos th, sin th, 0); the panel is the plane
 * at distance sdd from the source, perpendicular to the central ray, with
 * columns along e_u = (-sin th, cos th, 0) (the direction of source motion)
 * and rows along +z; its centre sits at -(sdd - sid)(cos th, sin th, 0) +
 * off_u e_u + off_v e_z.  Pixel (iu, iv) is centred (iu - (nu-1)/2) du along
 * e_u and (iv - (nv-1)/2) dv along z from the panel centre.  Voxel (i,j,k) is
 * centred at origin + ((i-(nx-1)/2) vx, (j-(ny-1)/2) vy, (k-(nz-1)/2) vz).
 *
 * Discretisation: a ray whose direction d has |d_x| >= |d_y| is sampled on
 * every voxel-centre plane x = const (else on the planes y = const); each
 * sample is the bilinear interpolant, in the two remaining axes, of the
 * zero-padded volume on that plane; the ray value is the sum of its samples
 * times vox_major |d| / |d_major|, the ray length per plane spacing.
 * Attenuation in mm^-1 gives dimensionless line integrals.
 *
 * Layouts (all dense, C order):
 *   volume    [C][nz][ny][nx]          x fastest
 *   sinogram  [C][n_angles][nv][nu]    u fastest
 * where C = n_channels; all channels share the geometry.
 *
 * Ownership: every data pointer is a device pointer owned by the caller; the
 * library never frees or keeps it after the call returns.  A geometry handle
 * owns its device tables and is immutable after creation; one handle may be
 * used from several streams at once.
 *
 * Execution: compute calls only enqueue work on `stream` (a hipStream_t; NULL
 * selects the null stream) and return; outputs are overwritten, never
 * accumulated.  Results are bitwise reproducible run to run and identical
 * between the single-case and the batched entry points.
 *
 * Errors: every call returns a status; nothing aborts.  Validation happens on
 * the host before any device work is enqueued, so a failed call leaves the
 * outputs untouched.
 */
#ifndef CBCT_H
#define CBCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage type of a volume or sinogram buffer.  Arithmetic is always FP32;
 * BF16/FP16 buffers are widened on load and rounded to nearest-even on
 * store. */
typedef enum { CBCT_F32 = 0, CBCT_BF16 = 1, CBCT_F16 = 2 } cbct_dtype;

typedef enum {
    CBCT_OK = 0,
    CBCT_E_NULL = -1,   /* a required pointer is NULL */
    CBCT_E_GEOM = -2,   /* geometry rejected (see cbct_geom_create) */
    CBCT_E_DTYPE = -3,  /* unknown storage type */
    CBCT_E_SHAPE = -4,  /* sizes out of range (channels, batch count, index range) */
    CBCT_E_HIP = -5,    /* a HIP runtime call failed; see cbct_last_hip_error */
    CBCT_E_ALLOC = -6,  /* host or device allocation failed */
    CBCT_E_ARG = -7     /* any other invalid argument */
} cbct_status;

/* Acquisition and volume geometry (Sec. 2.2).  Distances in mm, angles in
 * radians. */
typedef struct {
    double sid_mm;              /* source to isocenter, > 0 (paper: 1000) */
    double sdd_mm;              /* source to panel, > sid_mm (paper: 1000 + 536) */
    int n_angles;               /* number of source positions, > 0 */
    const double *angles_rad;   /* host array of n_angles angles, or NULL for
                                   2 pi a / n_angles (a = 0..n_angles-1); copied */
    int nu, nv;                 /* panel columns (along e_u) and rows (along z) */
    double du_mm, dv_mm;        /* pixel pitch, > 0 */
    double off_u_mm, off_v_mm;  /* panel-centre offset along e_u and z (paper: 115 lateral) */
    int nx, ny, nz;             /* voxel counts, > 0 */
    double vx_mm, vy_mm, vz_mm; /* voxel pitch, > 0 */
    double origin_mm[3];        /* volume centre relative to the isocenter */
} cbct_geom_desc;

typedef struct cbct_geom cbct_geom;   /* opaque, immutable after creation */

/*
 * Validate `desc`, build the per-angle and per-column tables in FP64 on the
 * host, round them to FP32 and upload them to the current HIP device.
 * CBCT_E_GEOM is returned when: a size or pitch is not positive, sdd <= sid,
 * an angle is not finite, the volume's support (the voxel box widened by one
 * voxel in x and y) is not strictly inside the cylinder of radius
 * min(sid, sdd - sid) about z (so some sample would not lie strictly between
 * source and panel), a ray is steeper in z than in x and y
 * (|d_z| >= max(|d_x|, |d_y|)), the columns of one angle change sampling axis
 * more than once, a size exceeds 2^31 elements, or one of nu, nv, nx, ny, nz
 * exceeds 65536.  On success *out
 * receives a handle to release with cbct_geom_destroy.
 */
cbct_status cbct_geom_create(const cbct_geom_desc *desc, cbct_geom **out);

/* Release a handle and its device tables (NULL is accepted).  The caller
 * must ensure no enqueued work still uses it. */
cbct_status cbct_geom_destroy(cbct_geom *g);

/* Number of samples one application of A (or A^T) performs: the (ray, plane)
 * pairs whose bilinear support meets the volume.  This is the unit of the
 * Gsamples/s throughput figures.  Computed on the host in FP64, once. */
cbct_status cbct_sample_count(const cbct_geom *g, uint64_t *samples);

/* Sizes of one channel: voxels (nx*ny*nz) and sinogram elements
 * (n_angles*nv*nu). */
cbct_status cbct_geom_sizes(const cbct_geom *g, uint64_t *n_vox, uint64_t *n_sino);

/*
 * sino = A vol for n_channels >= 1 stacked channels.  vol (storage vt) is
 * [C][nz][ny][nx]; sino (storage st) is [C][n_angles][nv][nu].  Geometries
 * whose ray tiles spread over more voxels than the tiled kernel stages, or
 * whose volume channel with 64 more z planes reaches 4 GiB in FP32, run a
 * one-thread-per-ray
 * kernel with the same arithmetic (slower; cbct_geom_plan_info tells which).
 * The tiled kernel first writes the volume with x and y swapped (C x
 * nx*ny*nz elements of storage vt) into the device buffer the library owns
 * (the one cbct_adjoint uses: the first call on a device, or a larger one,
 * allocates; calls on different streams are ordered on it): tiles that
 * sweep x planes stage their boxes from it.  Multichannel FP32 stacks pack
 * their channels there instead.
 */
cbct_status cbct_forward(const cbct_geom *g, const void *vol, cbct_dtype vt,
                         void *sino, cbct_dtype st, int n_channels, void *stream);

/*
 * vol = A^T sino for n_channels >= 1 stacked channels (layouts as above).
 * The weights are the ones cbct_forward applies, so the two are transposes
 * up to FP32 rounding of the sums.  Geometries whose panel windows exceed
 * 64 KB of LDS even for 8 x 7 x 4 voxel bricks run a one-thread-per-voxel
 * kernel with the same weights (slower).
 * The bricked kernel first writes the projections times each ray's length
 * per plane (FP32, C x n_angles*nv*nu values) into a device buffer the
 * library owns, one per device, kept until the process ends and grown when
 * a call needs more: the first call on a device, and any larger one,
 * allocates (so it must not be the one captured into a graph).  Calls on
 * different streams are ordered on that buffer (each waits for the previous
 * call's work); allocation failure returns CBCT_E_HIP.
 */
cbct_status cbct_adjoint(const cbct_geom *g, const void *sino, cbct_dtype st,
                         void *vol, cbct_dtype vt, int n_channels, void *stream);

/*
 * Batched forward over n >= 1 independent single-channel cases, each with
 * its own geometry handle and buffers (host arrays of n handles and n device
 * pointers), in one launch over all cases' work items (batches of more than
 * 16 cases run as one launch per 16 cases; cases whose geometry takes the
 * one-thread-per-ray kernel are launched on their own).  Like cbct_forward
 * it first writes each case's volume with x and y swapped into the
 * library-owned device buffer.  Results are
 * bitwise identical to n separate cbct_forward calls.  With FP32 storage, cases that share one
 * handle (e.g. the channels of a stack, as in Alg. 1) are instead cut into
 * groups of four or two that share each sample's geometry (packed into a
 * library-owned device buffer first, as cbct_adjoint's, and launched
 * separately); cbct_forward does the same for n_channels > 1.  The bits do
 * not change.
 */
cbct_status cbct_batch_forward(int n, const cbct_geom *const *g, const void *const *vols,
                               void *const *sinos, cbct_dtype vt, cbct_dtype st, void *stream);

/* Batched adjoint, the counterpart of cbct_batch_forward: one launch per 16
 * cases whose geometry takes the bricked kernel (the others on their own).
 * It uses the same library-owned buffer as cbct_adjoint, sized for the
 * cases of one launch together. */
cbct_status cbct_batch_adjoint(int n, const cbct_geom *const *g, const void *const *sinos,
                               void *const *vols, cbct_dtype st, cbct_dtype vt, void *stream);

/* Host-only handle: the same validation, tables, plans and sample count as
 * cbct_geom_create, without touching any device.  Compute calls on it return
 * CBCT_E_ARG.  For inspection and for testing host logic on machines without
 * a GPU. */
cbct_status cbct_geom_create_host(const cbct_geom_desc *desc, cbct_geom **out);

/* Copy a host table of a handle into dst (cap bytes); *bytes receives its
 * size (dst may be NULL to query it).  which: 0 per-(angle, column) records
 * {pb, ps, t0, tau, dsf, n2, 0, 0} (float32 x 8, angle-major); 1 per-angle
 * records {cos, sin (float32), x_lo, x_hi (int32)}; 2 per-row {V/vz, V^2}
 * (float32 x 2); 3 forward tiles {angle, axis, u0, n_u, v0, n_v, p_lo, p_hi}
 * (int32 x 8); 4 the scalar block {n_angles, nu, nv, nx, ny, nz (int32), Kb,
 * vx, vy, vz, ox, oy, oz, sid, sdd, du, dv, off_u, off_v, cu, cv, rv0, rvs
 * (float32)}; 5 adjoint panel windows per angle and 8 x 7 brick column
 * ([n_angles][ceil(ny/7)][ceil(nx/8)], empty when the adjoint runs the
 * one-thread-per-voxel kernel) {lambda_min, lambda_max (float32), u0 | u1 << 16,
 * row taps (int32)}. */
cbct_status cbct_geom_table(const cbct_geom *g, int which, void *dst, size_t cap, size_t *bytes);

/* Diagnostics: the launch plan chosen for a geometry.  Fills up to n of
 * {forward tiled (1/0), rays per thread, box in-plane, box z, tile count,
 *  adjoint bricked (1/0), window columns, window rows, LDS row stride,
 *  max row taps, voxels per adjoint thread along z (bricks are 4 times that
 *  deep), forward tile columns (64 or 32), adjoint brick width along x,
 *  adjoint brick width along y}.  A 0 in either flag means that operator
 *  runs the one-thread-per-output kernels. */
cbct_status cbct_geom_plan_info(const cbct_geom *g, int *info, int n);

/* Static, human-readable description of a status code. */
const char *cbct_error_string(cbct_status e);

/* Text of the last HIP error seen by this thread ("" if none). */
const char *cbct_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CBCT_H */
