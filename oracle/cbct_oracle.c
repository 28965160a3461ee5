/*
 * cbct_oracle.c -- plain FP64 CPU oracle for the circular-orbit cone-beam
 * projector pair (TEST INFRASTRUCTURE ONLY).
 *
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark load
 * this file's shared library.  It shares no code, header, table or constant
 * with the HIP library: every quantity below is recomputed from the
 * definitions, in double precision, one ray or one voxel at a time.
 *
 * What is computed (paper, Sec. 2.2, definition of the cone-beam transform
 * P(mu)(t,u) = integral of mu over the line from the source to detector
 * element u at time t, and its adjoint, the backprojection P*):
 *
 *   World frame: isocenter at the origin, rotation axis z.  For angle theta
 *     source      S  = sid (cos th, sin th, 0)
 *     e_u         = (-sin th, cos th, 0)     (direction of source motion)
 *     e_v         = (0, 0, 1)
 *     detector    D  = -(sdd - sid)(cos th, sin th, 0) + off_u e_u + off_v e_v
 *     pixel       P(iu,iv) = D + (iu - (nu-1)/2) du e_u + (iv - (nv-1)/2) dv e_v
 *   (Sec. 2.2: source-isocenter 1000 mm, isocenter-detector 536 mm, detector
 *   offset to the side in the direction of rotation.)
 *   Voxel centres: c(i,j,k) = origin + ((i-(nx-1)/2) vx, (j-(ny-1)/2) vy,
 *   (k-(nz-1)/2) vz); memory index (k*ny + j)*nx + i.
 *
 *   Discrete line integral (the paper states only the continuous integral;
 *   this is the discretisation the whole repository defines): ray direction
 *   d = P - S.  Its major axis m is x when |d_x| >= |d_y|, else y.  The ray is
 *   sampled exactly where it crosses the voxel-centre planes of m, strictly
 *   between source and pixel (0 < t < 1); on such a plane the trilinear
 *   interpolant of the zero-padded volume reduces to bilinear interpolation
 *   in the two remaining axes.  The ray value is the sum of the samples times
 *   the length of ray per plane spacing, ds = vox_m |d| / |d_m|.
 *
 *   The adjoint is the Euclidean transpose: x_v = sum_r A[r,v] y_r.
 *
 * Everything is FP64.  Parallel loops (OpenMP) only split independent rays;
 * the scatter adjoint keeps one accumulator volume per thread and sums them
 * in thread order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double sid, sdd;          /* source-isocenter, source-detector distance (mm) */
    int n_angles;
    const double *angles;     /* n_angles source angles (rad) */
    int nu, nv;               /* detector columns (along e_u), rows (along e_v) */
    double du, dv;            /* detector pitch (mm) */
    double off_u, off_v;      /* detector centre offset along e_u, e_v (mm) */
    int nx, ny, nz;           /* voxel counts */
    double vx, vy, vz;        /* voxel pitch (mm) */
    double ox, oy, oz;        /* volume centre (mm, relative to isocenter) */
} orc_geom;

/* ---- ray geometry ------------------------------------------------------ */

/* Source position and direction d = P(iu,iv) - S for angle index a. */
void orc_ray(const orc_geom *g, int a, int iu, int iv, double S[3], double d[3])
{
    double th = g->angles[a];
    double c = cos(th), s = sin(th);
    double eu[3] = {-s, c, 0.0};
    double ev[3] = {0.0, 0.0, 1.0};
    double D[3], P[3];
    double pu = (iu - 0.5 * (g->nu - 1)) * g->du;
    double pv = (iv - 0.5 * (g->nv - 1)) * g->dv;
    S[0] = g->sid * c;
    S[1] = g->sid * s;
    S[2] = 0.0;
    for (int q = 0; q < 3; ++q) {
        double toward = (q == 0) ? c : (q == 1) ? s : 0.0;
        D[q] = -(g->sdd - g->sid) * toward + g->off_u * eu[q] + g->off_v * ev[q];
        P[q] = D[q] + pu * eu[q] + pv * ev[q];
        d[q] = P[q] - S[q];
    }
}

static double norm3(const double d[3])
{
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

static double centre(int idx, int n, double pitch, double org)
{
    return org + (idx - 0.5 * (n - 1)) * pitch;
}

/* Fractional voxel index of world coordinate w along an axis. */
static double findex(double w, int n, double pitch, double org)
{
    return (w - org) / pitch + 0.5 * (n - 1);
}

static double hat(double s)
{
    double a = 1.0 - fabs(s);
    return a > 0.0 ? a : 0.0;
}

/* Volume value with zero padding. */
static double vox(const orc_geom *g, const double *vol, long i, long j, long k)
{
    if (i < 0 || j < 0 || k < 0 || i >= g->nx || j >= g->ny || k >= g->nz)
        return 0.0;
    return vol[(k * g->ny + j) * (long)g->nx + i];
}

/*
 * Visit every sample of ray (a,iu,iv).  For each plane crossing that lies
 * strictly between source and pixel and inside the open support
 * (-1, n) of both in-plane fractional indices, call visit() with the plane
 * index, the two in-plane fractional indices and ds.  Returns the sample
 * count.  The visitor receives the in-plane pair as (x-or-y index, z index).
 */
typedef void (*sample_fn)(void *ctx, int major_is_x, int p, double f1, double fz);

static long walk_ray(const orc_geom *g, int a, int iu, int iv, double *ds_out,
                     sample_fn visit, void *ctx)
{
    double S[3], d[3];
    orc_ray(g, a, iu, iv, S, d);
    int major_is_x = fabs(d[0]) >= fabs(d[1]);
    int m = major_is_x ? 0 : 1;        /* sampled axis */
    int o = major_is_x ? 1 : 0;        /* other in-plane axis */
    int nm = major_is_x ? g->nx : g->ny;
    int no = major_is_x ? g->ny : g->nx;
    double pm = major_is_x ? g->vx : g->vy;
    double po = major_is_x ? g->vy : g->vx;
    double om = major_is_x ? g->ox : g->oy;
    double oo = major_is_x ? g->oy : g->ox;
    *ds_out = pm * norm3(d) / fabs(d[m]);
    long count = 0;
    for (int p = 0; p < nm; ++p) {
        double cm = centre(p, nm, pm, om);
        double t = (cm - S[m]) / d[m];
        if (!(t > 0.0 && t < 1.0))
            continue;
        double qo = S[o] + t * d[o];
        double qz = S[2] + t * d[2];
        double f1 = findex(qo, no, po, oo);
        double fz = findex(qz, g->nz, g->vz, g->oz);
        if (!(f1 > -1.0 && f1 < no && fz > -1.0 && fz < g->nz))
            continue;
        ++count;
        if (visit)
            visit(ctx, major_is_x, p, f1, fz);
    }
    return count;
}

/* ---- forward ----------------------------------------------------------- */

typedef struct {
    const orc_geom *g;
    const double *vol;
    double acc;
} fwd_ctx;

static void fwd_visit(void *vctx, int major_is_x, int p, double f1, double fz)
{
    fwd_ctx *c = (fwd_ctx *)vctx;
    long j0 = (long)floor(f1), k0 = (long)floor(fz);
    double s = 0.0;
    for (long dj = 0; dj <= 1; ++dj)
        for (long dk = 0; dk <= 1; ++dk) {
            long jj = j0 + dj, kk = k0 + dk;
            double w = hat(f1 - jj) * hat(fz - kk);
            double v = major_is_x ? vox(c->g, c->vol, p, jj, kk) : vox(c->g, c->vol, jj, p, kk);
            s += w * v;
        }
    c->acc += s;
}

static double forward_ray(const orc_geom *g, const double *vol, int a, int iu, int iv)
{
    fwd_ctx c = {g, vol, 0.0};
    double ds;
    walk_ray(g, a, iu, iv, &ds, fwd_visit, &c);
    return c.acc * ds;
}

/* sino[(a*nv + iv)*nu + iu] = (A vol) */
int orc_forward(const orc_geom *g, const double *vol, double *sino, int nthreads)
{
    long nrow = (long)g->n_angles * g->nv;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (long r = 0; r < nrow; ++r) {
        int a = (int)(r / g->nv), iv = (int)(r % g->nv);
        for (int iu = 0; iu < g->nu; ++iu)
            sino[r * g->nu + iu] = forward_ray(g, vol, a, iu, iv);
    }
    return 0;
}

/* Forward values for an explicit list of flat ray indices (a*nv+iv)*nu+iu. */
int orc_forward_rays(const orc_geom *g, const double *vol, const int64_t *rays, int64_t n,
                     double *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t q = 0; q < n; ++q) {
        int64_t r = rays[q];
        int iu = (int)(r % g->nu);
        int iv = (int)((r / g->nu) % g->nv);
        int a = (int)(r / ((int64_t)g->nu * g->nv));
        out[q] = forward_ray(g, vol, a, iu, iv);
    }
    return 0;
}

/* ---- adjoint, scatter form --------------------------------------------- */

typedef struct {
    const orc_geom *g;
    double *vol;
    double yds;   /* y_r * ds_r */
} adj_ctx;

static void adj_visit(void *vctx, int major_is_x, int p, double f1, double fz)
{
    adj_ctx *c = (adj_ctx *)vctx;
    const orc_geom *g = c->g;
    long j0 = (long)floor(f1), k0 = (long)floor(fz);
    for (long dj = 0; dj <= 1; ++dj)
        for (long dk = 0; dk <= 1; ++dk) {
            long jj = j0 + dj, kk = k0 + dk;
            long ii = major_is_x ? p : jj;
            long yy = major_is_x ? jj : p;
            if (ii < 0 || yy < 0 || kk < 0 || ii >= g->nx || yy >= g->ny || kk >= g->nz)
                continue;
            double w = hat(f1 - jj) * hat(fz - kk);
            c->vol[(kk * g->ny + yy) * (long)g->nx + ii] += w * c->yds;
        }
}

/* vol = A^T sino, by scattering every ray's samples (one accumulator volume
 * per thread, summed in thread order afterwards). */
int orc_adjoint(const orc_geom *g, const double *sino, double *vol, int nthreads)
{
    long nvox = (long)g->nx * g->ny * g->nz;
    long nrow = (long)g->n_angles * g->nv;
    int nt = 1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
    nt = omp_get_max_threads();
#endif
    double *part = (double *)calloc((size_t)nt * (size_t)nvox, sizeof(double));
    if (!part)
        return -1;
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = part + (size_t)tid * (size_t)nvox;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (long r = 0; r < nrow; ++r) {
            int a = (int)(r / g->nv), iv = (int)(r % g->nv);
            for (int iu = 0; iu < g->nu; ++iu) {
                double y = sino[r * g->nu + iu];
                if (y == 0.0)
                    continue;
                double S[3], d[3], ds;
                orc_ray(g, a, iu, iv, S, d);
                int major_is_x = fabs(d[0]) >= fabs(d[1]);
                double pm = major_is_x ? g->vx : g->vy;
                adj_ctx c = {g, mine, y * pm * norm3(d) / fabs(d[major_is_x ? 0 : 1])};
                walk_ray(g, a, iu, iv, &ds, adj_visit, &c);
            }
        }
    }
    for (long v = 0; v < nvox; ++v) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t)
            s += part[(size_t)t * (size_t)nvox + v];
        vol[v] = s;
    }
    free(part);
    return 0;
}

/* ---- adjoint, gather form for selected voxels --------------------------- */

/* Detector coordinates (fractional column, row) of world point w at angle a,
 * by intersecting the line S->w with the detector plane. */
static void project_point(const orc_geom *g, int a, const double w[3], double *fu, double *fv)
{
    double th = g->angles[a];
    double c = cos(th), s = sin(th);
    double S[3] = {g->sid * c, g->sid * s, 0.0};
    double r[3] = {w[0] - S[0], w[1] - S[1], w[2] - S[2]};
    double depth = r[0] * c + r[1] * s;        /* along (cos, sin): -sdd at the panel */
    double lam = -g->sdd / depth;
    double U = lam * (r[0] * (-s) + r[1] * c);
    double V = lam * r[2];
    *fu = (U - g->off_u) / g->du + 0.5 * (g->nu - 1);
    *fv = (V - g->off_v) / g->dv + 0.5 * (g->nv - 1);
}

/* Weight A[r, v] of voxel (i,j,k) in ray (a,iu,iv), from the definition. */
double orc_weight(const orc_geom *g, int a, int iu, int iv, int i, int j, int k)
{
    double S[3], d[3];
    orc_ray(g, a, iu, iv, S, d);
    int major_is_x = fabs(d[0]) >= fabs(d[1]);
    int m = major_is_x ? 0 : 1, o = major_is_x ? 1 : 0;
    int p = major_is_x ? i : j, q = major_is_x ? j : i;
    int nm = major_is_x ? g->nx : g->ny, no = major_is_x ? g->ny : g->nx;
    double pm = major_is_x ? g->vx : g->vy, po = major_is_x ? g->vy : g->vx;
    double om = major_is_x ? g->ox : g->oy, oo = major_is_x ? g->oy : g->ox;
    double t = (centre(p, nm, pm, om) - S[m]) / d[m];
    if (!(t > 0.0 && t < 1.0))
        return 0.0;
    double f1 = findex(S[o] + t * d[o], no, po, oo);
    double fz = findex(S[2] + t * d[2], g->nz, g->vz, g->oz);
    if (!(f1 > -1.0 && f1 < no && fz > -1.0 && fz < g->nz))
        return 0.0;
    double ds = pm * norm3(d) / fabs(d[m]);
    return ds * hat(f1 - q) * hat(fz - k);
}

/*
 * out[q] = (A^T sino)[vox[q]] for flat voxel indices (k*ny+j)*nx+i, by
 * gathering over every ray whose weight at the voxel can be non-zero.  Those
 * rays pass within one voxel pitch of the centre along each axis, so they
 * hit the detector inside the projection of the box centre +- pitch; the
 * window scanned is that projection's bounding box widened by two pixels,
 * and the function returns -2 if any weight on the window's border is
 * non-zero (the window would then have been too small).
 */
int orc_adjoint_voxels(const orc_geom *g, const double *sino, const int64_t *voxels, int64_t n,
                       double *out, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
#endif
    for (int64_t q = 0; q < n; ++q) {
        int64_t v = voxels[q];
        int i = (int)(v % g->nx);
        int j = (int)((v / g->nx) % g->ny);
        int k = (int)(v / ((int64_t)g->nx * g->ny));
        double c[3] = {centre(i, g->nx, g->vx, g->ox), centre(j, g->ny, g->vy, g->oy),
                       centre(k, g->nz, g->vz, g->oz)};
        double acc = 0.0;
        for (int a = 0; a < g->n_angles; ++a) {
            double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
            for (int corner = 0; corner < 8; ++corner) {
                double w[3] = {c[0] + ((corner & 1) ? g->vx : -g->vx),
                               c[1] + ((corner & 2) ? g->vy : -g->vy),
                               c[2] + ((corner & 4) ? g->vz : -g->vz)};
                double fu, fv;
                project_point(g, a, w, &fu, &fv);
                umin = fmin(umin, fu); umax = fmax(umax, fu);
                vmin = fmin(vmin, fv); vmax = fmax(vmax, fv);
            }
            int u0 = (int)floor(umin) - 2, u1 = (int)ceil(umax) + 2;
            int v0 = (int)floor(vmin) - 2, v1 = (int)ceil(vmax) + 2;
            for (int iv = v0; iv <= v1; ++iv) {
                if (iv < 0 || iv >= g->nv)
                    continue;
                for (int iu = u0; iu <= u1; ++iu) {
                    if (iu < 0 || iu >= g->nu)
                        continue;
                    double w = orc_weight(g, a, iu, iv, i, j, k);
                    if (w == 0.0)
                        continue;
                    if (iu == u0 || iu == u1 || iv == v0 || iv == v1)
                        bad = 1;
                    acc += w * sino[((int64_t)a * g->nv + iv) * g->nu + iu];
                }
            }
        }
        out[q] = acc;
    }
    return bad ? -2 : 0;
}

/* ---- sample count ------------------------------------------------------ */

/* Number of (ray, plane) pairs with non-empty support, the unit of work. */
int64_t orc_sample_count(const orc_geom *g, int nthreads)
{
    int64_t total = 0;
    long nrow = (long)g->n_angles * g->nv;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : total)
#endif
    for (long r = 0; r < nrow; ++r) {
        int a = (int)(r / g->nv), iv = (int)(r % g->nv);
        for (int iu = 0; iu < g->nu; ++iu) {
            double ds;
            total += walk_ray(g, a, iu, iv, &ds, NULL, NULL);
        }
    }
    return total;
}

/* ---- independent references for the pins -------------------------------- */

/* Segment parameter interval [t0,t1] of S + t d inside box [lo,hi] (slab
 * clipping), intersected with [tmin,tmax].  Returns 0 if empty. */
static int clip_box(const double S[3], const double d[3], const double lo[3], const double hi[3],
                    double tmin, double tmax, double *t0, double *t1)
{
    double a = tmin, b = tmax;
    for (int q = 0; q < 3; ++q) {
        if (d[q] == 0.0) {
            if (S[q] < lo[q] || S[q] > hi[q])
                return 0;
            continue;
        }
        double ta = (lo[q] - S[q]) / d[q], tb = (hi[q] - S[q]) / d[q];
        if (ta > tb) {
            double tmp = ta; ta = tb; tb = tmp;
        }
        if (ta > a) a = ta;
        if (tb < b) b = tb;
    }
    *t0 = a;
    *t1 = b;
    return b > a;
}

/* Exact length (mm) of ray (a,iu,iv) inside the axis-aligned box [lo,hi]. */
double orc_chord_box(const orc_geom *g, int a, int iu, int iv, const double lo[3], const double hi[3])
{
    double S[3], d[3], t0, t1;
    orc_ray(g, a, iu, iv, S, d);
    if (!clip_box(S, d, lo, hi, 0.0, 1.0, &t0, &t1))
        return 0.0;
    return (t1 - t0) * norm3(d);
}

/*
 * Brute-force Siddon matrix: L[r*nvox + v] = exact length of ray r inside the
 * cube of voxel v (every ray is clipped against every voxel box).  Tiny
 * volumes only.
 */
int orc_siddon_dense(const orc_geom *g, double *L)
{
    long nvox = (long)g->nx * g->ny * g->nz;
    long nray = (long)g->n_angles * g->nv * g->nu;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (long r = 0; r < nray; ++r) {
        int iu = (int)(r % g->nu), iv = (int)((r / g->nu) % g->nv), a = (int)(r / ((long)g->nu * g->nv));
        for (long v = 0; v < nvox; ++v) {
            int i = (int)(v % g->nx), j = (int)((v / g->nx) % g->ny), k = (int)(v / ((long)g->nx * g->ny));
            double c[3] = {centre(i, g->nx, g->vx, g->ox), centre(j, g->ny, g->vy, g->oy),
                           centre(k, g->nz, g->vz, g->oz)};
            double lo[3] = {c[0] - 0.5 * g->vx, c[1] - 0.5 * g->vy, c[2] - 0.5 * g->vz};
            double hi[3] = {c[0] + 0.5 * g->vx, c[1] + 0.5 * g->vy, c[2] + 0.5 * g->vz};
            L[r * nvox + v] = orc_chord_box(g, a, iu, iv, lo, hi);
        }
    }
    return 0;
}

/*
 * Exact line integral, over the whole source-to-pixel segment, of the
 * trilinear interpolant of the zero-padded volume.  The interpolant is a
 * trilinear polynomial inside each dual cell (the box spanned by eight
 * neighbouring voxel centres, pad layer included), so along a straight
 * segment it is a cubic in t; two-point Gauss-Legendre per cell segment
 * integrates it exactly.  Cells are visited by clipping the ray against
 * every dual cell of the padded grid (small volumes only).
 */
double orc_interp_integral(const orc_geom *g, const double *vol, int a, int iu, int iv)
{
    double S[3], d[3];
    orc_ray(g, a, iu, iv, S, d);
    double len = norm3(d);
    const double gl = 0.5 / sqrt(3.0);
    double total = 0.0;
    for (int k = -1; k < g->nz; ++k)
        for (int j = -1; j < g->ny; ++j)
            for (int i = -1; i < g->nx; ++i) {
                double lo[3] = {centre(i, g->nx, g->vx, g->ox), centre(j, g->ny, g->vy, g->oy),
                                centre(k, g->nz, g->vz, g->oz)};
                double hi[3] = {lo[0] + g->vx, lo[1] + g->vy, lo[2] + g->vz};
                double t0, t1;
                if (!clip_box(S, d, lo, hi, 0.0, 1.0, &t0, &t1))
                    continue;
                double seg = 0.0;
                for (int n = 0; n < 2; ++n) {
                    double t = 0.5 * (t0 + t1) + (n ? gl : -gl) * (t1 - t0);
                    double x = (S[0] + t * d[0] - lo[0]) / g->vx;
                    double y = (S[1] + t * d[1] - lo[1]) / g->vy;
                    double z = (S[2] + t * d[2] - lo[2]) / g->vz;
                    double f = 0.0;
                    for (int c = 0; c < 8; ++c) {
                        int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
                        double w = (bx ? x : 1 - x) * (by ? y : 1 - y) * (bz ? z : 1 - z);
                        f += w * vox(g, vol, i + bx, j + by, k + bz);
                    }
                    seg += 0.5 * f;
                }
                total += seg * (t1 - t0) * len;
            }
    return total;
}

/* ---- noise model of the projection simulator ----------------------------
 *
 * Poisson counts and the log transform follow the paper's primary model and
 * normalisation (Sec. 2.2, noisy primary projections; Sec. 2.4, negative
 * log of counts over the air scan clamped at 1), in its monochromatic form:
 * counts ~ Poisson(I0 exp(-p)), y = -log(min(max(counts, 1) / I0, 1)).
 * Random numbers come from the counter-based generator Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, SC'11), written here from its published
 * definition: ten rounds of two 32x32->64-bit multiplications with
 * multipliers 0xD2511F53 and 0xCD9E8D57, the high halves xored with the other
 * counter words and the key, and a Weyl key schedule with increments
 * 0x9E3779B9 and 0xBB67AE85.  Element i, trial j of generator stream s with
 * 64-bit seed uses counter (i mod 2^32, i div 2^32, j, s) and key
 * (seed mod 2^32, seed div 2^32).
 */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
        uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
        c0 = h1 ^ c1 ^ k0;
        c1 = l1;
        c2 = h0 ^ c3 ^ k1;
        c3 = l0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static void draw(uint64_t seed, uint32_t stream, uint64_t i, uint32_t j, uint32_t w[4])
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), j, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

/* 53-bit uniform in [0, 1) from two words. */
static double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/*
 * Poisson variate with mean lam >= 0.  Below 10: inversion of the CDF by
 * sequential search with one uniform.  From 10 up: the transformed rejection
 * method with squeeze of Hormann (1993, "The transformed rejection method for
 * generating Poisson random variables", algorithm PTRS), one (U, V) pair per
 * trial, trials numbered from 0; after 64 rejected trials the rounded mean
 * is returned (probability far below 1e-30).
 */
static int64_t poisson_ctr(double lam, uint64_t seed, uint32_t stream, uint64_t i,
                           uint32_t trial0);

int64_t orc_poisson(double lam, uint64_t seed, uint32_t stream, uint64_t i)
{
    return poisson_ctr(lam, seed, stream, i, 0);
}

/* The same variate with the trial counters starting at trial0 (trial j of the
 * variate uses counter word 2 = trial0 + j). */
static int64_t poisson_ctr(double lam, uint64_t seed, uint32_t stream, uint64_t i,
                           uint32_t trial0)
{
    uint32_t w[4];
    if (!(lam > 0.0))
        return 0;
    if (lam < 10.0) {
        draw(seed, stream, i, trial0, w);
        double u = u53(w[0], w[1]);
        double p = exp(-lam), F = p;
        int64_t k = 0;
        while (u > F && k < 1000) {
            k += 1;
            p *= lam / (double)k;
            F += p;
        }
        return k;
    }
    double sl = sqrt(lam), ll = log(lam);
    double b = 0.931 + 2.53 * sl;
    double a = -0.059 + 0.02483 * b;
    double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
    double v_r = 0.9277 - 3.6224 / (b - 2.0);
    for (uint32_t j = 0; j < 64; ++j) {
        draw(seed, stream, i, trial0 + j, w);
        double U = u53(w[0], w[1]) - 0.5;
        double V = u53(w[2], w[3]);
        double us = 0.5 - fabs(U);
        double kf = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= v_r)
            return (int64_t)kf;
        if (kf < 0.0 || (us < 0.013 && V > us))
            continue;
        double lhs = log(V) + log(inv_alpha) - log(a / (us * us) + b);
        double rhs = -lam + kf * ll - lgamma(kf + 1.0);
        if (lhs <= rhs)
            return (int64_t)kf;
    }
    return (int64_t)floor(lam + 0.5);
}

/* y[i] = -log(min(max(n_i, 1) / I0, 1)), n_i ~ Poisson(I0 exp(-p[i])). */
void orc_sim_poisson_log(int64_t n, const double *p, double I0, uint64_t seed, uint32_t stream,
                         int64_t *counts, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = orc_poisson(I0 * exp(-p[i]), seed, stream, (uint64_t)i);
        if (counts)
            counts[i] = c;
        double r = (double)(c < 1 ? 1 : c) / I0;
        y[i] = -log(r < 1.0 ? r : 1.0);
    }
}

/*
 * Noisy polychromatic primary signal (Sec. 2.2, eq. primarymodel) and its
 * normalised negative log (Sec. 2.4, eq. normprimary), given the two
 * material line integrals of each ray, pw = P(rho_w) and pb = P(rho_b)
 * (by linearity of P, the line integral of the energy-e attenuation
 * mu_w[e] rho_w + mu_b[e] rho_b is mu_w[e] pw + mu_b[e] pb):
 *   c_e   ~ Poisson(I0_e(pixel) exp(-(mu_w[e] pw + mu_b[e] pb)))   per bin e,
 *   s     = sum_e resp[e] c_e,                 (bins in index order)
 *   s_air = sum_e resp[e] I0_e(pixel)          (the noise-free air scan),
 *   y     = -log(min(max(s, r_min) / s_air, 1)),
 * r_min = the smallest positive resp[e] (a signal of zero photons counts as
 * one photon of the least-weighted bin); y = 0 where s_air <= 0.
 * Element i sits at pixel i mod npix (I0 is [nbins][npix], the same for
 * every projection).  Bin e's variate uses Philox trial counters from
 * 256 e (trials per variate < 64), so bin 0 draws exactly as the
 * monochromatic model does.  counts (optional) is [nbins][n].
 */
void orc_sim_poly(int64_t n, int64_t npix, const double *pw, const double *pb, int nbins,
                  const double *mu_w, const double *mu_b, const double *resp, const double *I0,
                  uint64_t seed, uint32_t stream, int64_t *counts, double *signal, double *y)
{
    double r_min = 0.0;
    for (int e = 0; e < nbins; ++e)
        if (resp[e] > 0.0 && (r_min == 0.0 || resp[e] < r_min))
            r_min = resp[e];
    for (int64_t i = 0; i < n; ++i) {
        const int64_t pix = i % npix;
        double sig = 0.0, air = 0.0;
        for (int e = 0; e < nbins; ++e) {
            const double i0 = I0[(int64_t)e * npix + pix];
            const double lam = i0 * exp(-(mu_w[e] * pw[i] + mu_b[e] * pb[i]));
            const int64_t c = poisson_ctr(lam, seed, stream, (uint64_t)i, 256u * (uint32_t)e);
            if (counts)
                counts[(int64_t)e * n + i] = c;
            sig += resp[e] * (double)c;
            air += resp[e] * i0;
        }
        if (signal)
            signal[i] = sig;
        if (!(air > 0.0)) {
            y[i] = 0.0;
            continue;
        }
        const double r = (sig < r_min ? r_min : sig) / air;
        y[i] = -log(r < 1.0 ? r : 1.0);
    }
}

/* out[i] = clean[i] + sigma z_i, z_i standard normal by the Box-Muller
 * transform of the first two 53-bit uniforms of element i (trial 0). */
void orc_sim_gaussian(int64_t n, const double *clean, double sigma, uint64_t seed, uint32_t stream,
                      double *out)
{
    uint32_t w[4];
    for (int64_t i = 0; i < n; ++i) {
        draw(seed, stream, (uint64_t)i, 0, w);
        double u1 = 1.0 - u53(w[0], w[1]);          /* (0, 1] */
        double u2 = u53(w[2], w[3]);
        double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
        out[i] = clean[i] + sigma * z;
    }
}

/* ---- scatter simulator (Sec. 2.3: the path-integral scatter model and its
 * quasi-Monte Carlo evaluation, Alg. 2 SamplePath and Alg. 3 Integrate;
 * appendix: Beer-Lambert escape probability eq. beer, the travel-distance
 * measure eq. lambdameas, inverse-transform sampling eq. distsample, the
 * material and interaction-type Bernoulli choices and the Compton energy).
 *
 * Readings (the paper states the model, not its discretisation):
 *   * The attenuation is piecewise constant on voxel cubes: voxel (i,j,k)
 *     holds relative densities rho_w, rho_b on the cube of its pitch centred
 *     at its centre; zero outside the volume.  mu_tot,e(x) =
 *     rho_w(x) mu_w(e) + rho_b(x) mu_b(e), mu_m(e) = p + c + r components.
 *   * Cross sections are tables on the energy grid e_k = e0 + k de, linear
 *     in e between grid points and constant beyond the ends; angular
 *     distributions per material and scatter type are tables too: the
 *     inverse CDF of cos(theta) on u = j / (J - 1) and the density of
 *     scatter directions per steradian on cos(theta) = -1 + 2 i / (I - 1),
 *     both bilinear in (energy, abscissa).
 *   * A scattered direction: cos(theta) from the inverse CDF at the first
 *     point, azimuth phi = 2 pi u at the second, around the incoming v in
 *     the frame a = normalise(v x z) (v x x when |v_z| >= 0.9), b = v x a:
 *     v' = cos(theta) v + sin(theta) (cos(phi) a + sin(phi) b).
 *   * The weight after a scatter is w (1 - mu_p / mu_tot) of the chosen
 *     material (the printed w (1 - mu_p) / mu_tot is read this way); W
 *     appends each weight (the printed W <- [w] restarts the list).
 *   * Sobol point i has 5 n + 1 coordinates: 0 for the first distance,
 *     then for scatter j = 1..n, k = 1 + 5 (j - 1): material, type, cos,
 *     azimuth, distance.
 *   * Integrate scores each interaction point x_o (o = 1..n+1) with the
 *     direction v, energy e and weight w the photon arrived with (the
 *     printed zip pairs the source point with the first direction); the
 *     scatter density at x is sum_m (mu_m / mu_tot)(x) (mu_T,m / mu_tot,m)
 *     dens_T,m(cos theta, e) for T = Compton, Rayleigh; the escape
 *     probability toward a pixel integrates up to the pixel centre (the
 *     panel lies beyond the volume); the accumulation index is the pixel.
 *   * A photon whose first ray misses the volume has weight 0 and stays at
 *     the source.  Where mu_tot(x) = 0 the material is water.
 * FP64 throughout; one photon (paths) or one pixel (integration) at a time.
 */

typedef struct {
    int K;
    double e0, de;          /* energy grid (keV) */
    const double *mu;       /* [2 materials][3 kinds: p, c, r][K], mm^-1 at unit density */
    int J;
    const double *icdf;     /* [2][2 types: c, r][K][J] cos(theta) at u = j / (J - 1) */
    int I;
    const double *dens;     /* [2][2][K][I] per steradian at cos = -1 + 2 i / (I - 1) */
} orc_xs;

static const double ORC_ME_C2 = 510.99895;   /* electron rest energy, keV */

static void e_index(const orc_xs *x, double e, int *k, double *f)
{
    double t = (e - x->e0) / x->de;
    if (t < 0.0)
        t = 0.0;
    if (t > x->K - 1)
        t = x->K - 1;
    int kk = (int)floor(t);
    if (kk > x->K - 2)
        kk = x->K - 2;
    *k = kk;
    *f = t - kk;
}

static double xs_mu(const orc_xs *x, int m, int kind, double e)
{
    int k;
    double f;
    e_index(x, e, &k, &f);
    const double *t = x->mu + ((size_t)m * 3 + kind) * x->K;
    return (1.0 - f) * t[k] + f * t[k + 1];
}

static double xs_tot(const orc_xs *x, int m, double e)
{
    return xs_mu(x, m, 0, e) + xs_mu(x, m, 1, e) + xs_mu(x, m, 2, e);
}

/* bilinear in (energy, abscissa) on a [K][n] table; s in [0, n - 1] */
static double table2(const orc_xs *x, const double *tab, int n, double e, double s)
{
    int k;
    double f;
    e_index(x, e, &k, &f);
    if (s < 0.0)
        s = 0.0;
    if (s > n - 1)
        s = n - 1;
    int j = (int)floor(s);
    if (j > n - 2)
        j = n - 2;
    double g = s - j;
    const double *r0 = tab + (size_t)k * n, *r1 = tab + (size_t)(k + 1) * n;
    double a = (1.0 - g) * r0[j] + g * r0[j + 1];
    double b = (1.0 - g) * r1[j] + g * r1[j + 1];
    return (1.0 - f) * a + f * b;
}

static double xs_icdf(const orc_xs *x, int m, int T, double e, double u)
{
    return table2(x, x->icdf + ((size_t)m * 2 + T) * x->K * x->J, x->J, e, u * (x->J - 1));
}

static double xs_dens(const orc_xs *x, int m, int T, double e, double cth)
{
    return table2(x, x->dens + ((size_t)m * 2 + T) * x->K * x->I, x->I, e,
                  (cth + 1.0) * 0.5 * (x->I - 1));
}

double orc_compton_energy(double e, double cth)
{
    return e / (1.0 + e * (1.0 - cth) / ORC_ME_C2);
}

/* resp(e): piecewise linear through (20, 5), (60, 20), (120, 10) keV, the end
 * values beyond (Sec. 2.2). */
double orc_resp(double e)
{
    if (e <= 20.0)
        return 5.0;
    if (e <= 60.0)
        return 5.0 + (e - 20.0) * 15.0 / 40.0;
    if (e < 120.0)
        return 20.0 - (e - 60.0) * 10.0 / 60.0;
    return 10.0;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Segments of the ray p + t d (|d| = 1), 0 <= t <= tmax, through the voxel
 * cubes: every parameter where it crosses a voxel face or the volume's
 * bounds, sorted; on each segment the voxel is the one holding its midpoint.
 * Returns the number of breakpoints written to ts (room for nx+ny+nz+5). */
static int ray_breaks(const orc_geom *g, const double p[3], const double d[3], double tmax,
                      double *ts)
{
    const int n[3] = {g->nx, g->ny, g->nz};
    const double v[3] = {g->vx, g->vy, g->vz}, o[3] = {g->ox, g->oy, g->oz};
    double t0 = 0.0, t1 = tmax;
    for (int q = 0; q < 3; ++q) {
        double lo = o[q] - 0.5 * n[q] * v[q], hi = o[q] + 0.5 * n[q] * v[q];
        if (d[q] == 0.0) {
            if (p[q] <= lo || p[q] >= hi)
                return 0;
            continue;
        }
        double ta = (lo - p[q]) / d[q], tb = (hi - p[q]) / d[q];
        if (ta > tb) {
            double s = ta;
            ta = tb;
            tb = s;
        }
        if (ta > t0)
            t0 = ta;
        if (tb < t1)
            t1 = tb;
    }
    if (!(t1 > t0))
        return 0;
    int cnt = 0;
    ts[cnt++] = t0;
    for (int q = 0; q < 3; ++q) {
        if (d[q] == 0.0)
            continue;
        double lo = o[q] - 0.5 * n[q] * v[q];
        for (int m = 1; m < n[q]; ++m) {
            double t = (lo + m * v[q] - p[q]) / d[q];
            if (t > t0 && t < t1)
                ts[cnt++] = t;
        }
    }
    ts[cnt++] = t1;
    qsort(ts, cnt, sizeof(double), cmp_double);
    return cnt;
}

static long voxel_at(const orc_geom *g, const double x[3])
{
    const int n[3] = {g->nx, g->ny, g->nz};
    const double v[3] = {g->vx, g->vy, g->vz}, o[3] = {g->ox, g->oy, g->oz};
    long idx[3];
    for (int q = 0; q < 3; ++q) {
        double f = (x[q] - (o[q] - 0.5 * n[q] * v[q])) / v[q];
        if (!(f >= 0.0 && f < n[q]))
            return -1;
        idx[q] = (long)floor(f);
    }
    return (idx[2] * g->ny + idx[1]) * g->nx + idx[0];
}

/* Material line integrals (int rho_w, int rho_b) along p + t d, t in [0, tmax]. */
void orc_march(const orc_geom *g, const double *rw, const double *rb, const double p[3],
               const double d[3], double tmax, double out[2])
{
    double *ts = malloc(sizeof(double) * (g->nx + g->ny + g->nz + 5));
    int cnt = ray_breaks(g, p, d, tmax, ts);
    out[0] = out[1] = 0.0;
    for (int s = 0; s + 1 < cnt; ++s) {
        double len = ts[s + 1] - ts[s];
        if (!(len > 0.0))
            continue;
        double tm = 0.5 * (ts[s] + ts[s + 1]);
        double xm[3] = {p[0] + tm * d[0], p[1] + tm * d[1], p[2] + tm * d[2]};
        long vi = voxel_at(g, xm);
        if (vi < 0)
            continue;
        out[0] += len * rw[vi];
        out[1] += len * rb[vi];
    }
    free(ts);
}

/* Interaction distance along p + t d at energy e (eq. distsample): the t at
 * which the optical depth reaches -log(1 - (1 - p0) ubar); p0 the escape
 * probability (eq. beer) of the whole ray.  Returns t (0 if the ray never
 * meets attenuating matter). */
static double sample_distance(const orc_geom *g, const double *rw, const double *rb,
                              const orc_xs *xs, const double p[3], const double d[3], double e,
                              double ubar, double *p0)
{
    const double big = 1e7;
    double *ts = malloc(sizeof(double) * (g->nx + g->ny + g->nz + 5));
    int cnt = ray_breaks(g, p, d, big, ts);
    double mw = xs_tot(xs, 0, e), mb = xs_tot(xs, 1, e);
    double tau = 0.0;
    for (int s = 0; s + 1 < cnt; ++s) {
        double len = ts[s + 1] - ts[s];
        if (!(len > 0.0))
            continue;
        double tm = 0.5 * (ts[s] + ts[s + 1]);
        double xm[3] = {p[0] + tm * d[0], p[1] + tm * d[1], p[2] + tm * d[2]};
        long vi = voxel_at(g, xm);
        if (vi >= 0)
            tau += len * (rw[vi] * mw + rb[vi] * mb);
    }
    *p0 = exp(-tau);
    double l = 0.0;
    if (tau > 0.0) {
        double target = -log(1.0 - (1.0 - *p0) * ubar);
        double acc = 0.0;
        for (int s = 0; s + 1 < cnt; ++s) {
            double len = ts[s + 1] - ts[s];
            if (!(len > 0.0))
                continue;
            double tm = 0.5 * (ts[s] + ts[s + 1]);
            double xm[3] = {p[0] + tm * d[0], p[1] + tm * d[1], p[2] + tm * d[2]};
            long vi = voxel_at(g, xm);
            double mu = vi >= 0 ? rw[vi] * mw + rb[vi] * mb : 0.0;
            if (mu > 0.0 && acc + len * mu >= target) {
                l = ts[s] + (target - acc) / mu;
                break;
            }
            acc += len * mu;
            l = ts[s + 1];
        }
    }
    free(ts);
    return l;
}

static void normalise3(double v[3])
{
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n;
    v[1] /= n;
    v[2] /= n;
}

/* v' at polar cos(theta) and azimuth phi around v (frame as stated above). */
void orc_scatter_direction(const double v[3], double cth, double phi, double out[3])
{
    double a[3];
    if (fabs(v[2]) < 0.9) {          /* v x z */
        a[0] = v[1];
        a[1] = -v[0];
        a[2] = 0.0;
    } else {                         /* v x x */
        a[0] = 0.0;
        a[1] = v[2];
        a[2] = -v[1];
    }
    normalise3(a);
    double b[3] = {v[1] * a[2] - v[2] * a[1], v[2] * a[0] - v[0] * a[2], v[0] * a[1] - v[1] * a[0]};
    double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
    for (int q = 0; q < 3; ++q)
        out[q] = cth * v[q] + sth * (cos(phi) * a[q] + sin(phi) * b[q]);
}

/*
 * SamplePath (Alg. 2) at projection angle index a: photon i leaves the source
 * S(theta_a) with direction R_a src[i][0..2] (src directions are given for
 * the source at angle 0; R_a rotates about z by theta_a) and energy
 * src[i][3].  sob: [N][5 n + 1] quasi-random points.  rec: [N][n + 1][8]
 * records (x, y, z of the interaction point, the direction and energy the
 * photon arrived with, its weight).
 */
void orc_scatter_paths(const orc_geom *g, const double *rw, const double *rb, const orc_xs *xs,
                       int a, int64_t N, const double *src, const double *sob, int n,
                       double *rec)
{
    const double th = g->angles[a], c = cos(th), s = sin(th);
    const int D = 5 * n + 1;
    for (int64_t i = 0; i < N; ++i) {
        const double *sp = src + 4 * i, *u = sob + (size_t)i * D;
        double x[3] = {g->sid * c, g->sid * s, 0.0};
        double v[3] = {c * sp[0] - s * sp[1], s * sp[0] + c * sp[1], sp[2]};
        normalise3(v);
        double e = sp[3], w = 1.0;
        for (int o = 0; o <= n; ++o) {
            double p0;
            const double l = sample_distance(g, rw, rb, xs, x, v, e, u[5 * o], &p0);
            w *= 1.0 - p0;
            for (int q = 0; q < 3; ++q)
                x[q] += l * v[q];
            double *r = rec + ((size_t)i * (n + 1) + o) * 8;
            r[0] = x[0];
            r[1] = x[1];
            r[2] = x[2];
            r[3] = v[0];
            r[4] = v[1];
            r[5] = v[2];
            r[6] = e;
            r[7] = w;
            if (o == n)
                break;
            const int k = 1 + 5 * o;
            const long vi = voxel_at(g, x);
            const double aw = vi >= 0 ? rw[vi] * xs_tot(xs, 0, e) : 0.0;
            const double ab = vi >= 0 ? rb[vi] * xs_tot(xs, 1, e) : 0.0;
            const double fw = (aw + ab) > 0.0 ? aw / (aw + ab) : 1.0;
            const int m = u[k] < fw ? 0 : 1;
            const double mc = xs_mu(xs, m, 1, e), mr = xs_mu(xs, m, 2, e);
            const int T = u[k + 1] < mc / (mc + mr) ? 0 : 1;
            w *= 1.0 - xs_mu(xs, m, 0, e) / xs_tot(xs, m, e);
            const double cth = xs_icdf(xs, m, T, e, u[k + 2]);
            double vn[3];
            orc_scatter_direction(v, cth, 2.0 * M_PI * u[k + 3], vn);
            normalise3(vn);
            v[0] = vn[0];
            v[1] = vn[1];
            v[2] = vn[2];
            if (T == 0)
                e = orc_compton_energy(e, cth);
        }
    }
}

/*
 * Integrate (Alg. 3) at projection angle index a over nrec records (as
 * written by orc_scatter_paths): out[iv][iu] (the panel of g at angle a,
 * pixel centres as in orc_ray) receives, per record in order,
 *   s w |<n, v_s>| du dv / |sigma - x|^2,
 *   s = s_c p0(x, v_s, e') resp(e') + s_r p0(x, v_s, e) resp(e),
 * n the panel normal, v_s the unit vector from x to the pixel centre, e' the
 * Compton energy for the angle between v and v_s.  The caller scales by
 * I_Sigma / |Src|.
 */
void orc_scatter_integrate(const orc_geom *g, const double *rw, const double *rb,
                           const orc_xs *xs, int a, int64_t nrec, const double *rec, double *out)
{
    const double th = g->angles[a];
    const double nrm[3] = {cos(th), sin(th), 0.0};
    for (int iv = 0; iv < g->nv; ++iv)
        for (int iu = 0; iu < g->nu; ++iu) {
            double S[3], d[3];
            orc_ray(g, a, iu, iv, S, d);
            const double pix[3] = {S[0] + d[0], S[1] + d[1], S[2] + d[2]};
            double acc = 0.0;
            for (int64_t r = 0; r < nrec; ++r) {
                const double *q = rec + 8 * r;
                const double w = q[7];
                if (!(w > 0.0))
                    continue;
                const double x[3] = {q[0], q[1], q[2]}, v[3] = {q[3], q[4], q[5]};
                const double e = q[6];
                double vs[3] = {pix[0] - x[0], pix[1] - x[1], pix[2] - x[2]};
                const double r2 = vs[0] * vs[0] + vs[1] * vs[1] + vs[2] * vs[2];
                const double dist = sqrt(r2);
                vs[0] /= dist;
                vs[1] /= dist;
                vs[2] /= dist;
                const double cth = v[0] * vs[0] + v[1] * vs[1] + v[2] * vs[2];
                const double ec = orc_compton_energy(e, cth);
                double P[2];
                orc_march(g, rw, rb, x, vs, dist, P);
                const long vi = voxel_at(g, x);
                const double aw = vi >= 0 ? rw[vi] * xs_tot(xs, 0, e) : 0.0;
                const double ab = vi >= 0 ? rb[vi] * xs_tot(xs, 1, e) : 0.0;
                const double tot = aw + ab;
                const double f[2] = {tot > 0.0 ? aw / tot : 1.0, tot > 0.0 ? ab / tot : 0.0};
                double sc = 0.0, sr = 0.0;
                for (int m = 0; m < 2; ++m) {
                    const double mt = xs_tot(xs, m, e);
                    sc += f[m] * xs_mu(xs, m, 1, e) / mt * xs_dens(xs, m, 0, e, cth);
                    sr += f[m] * xs_mu(xs, m, 2, e) / mt * xs_dens(xs, m, 1, e, cth);
                }
                const double p0c = exp(-(xs_tot(xs, 0, ec) * P[0] + xs_tot(xs, 1, ec) * P[1]));
                const double p0r = exp(-(xs_tot(xs, 0, e) * P[0] + xs_tot(xs, 1, e) * P[1]));
                const double sv = sc * p0c * orc_resp(ec) + sr * p0r * orc_resp(e);
                const double cn = fabs(nrm[0] * vs[0] + nrm[1] * vs[1] + nrm[2] * vs[2]);
                acc += sv * w * cn * g->du * g->dv / r2;
            }
            out[(size_t)iv * g->nu + iu] = acc;
        }
}
