// Host-side geometry set-up of libcbct.so: validation, FP64 per-angle and
// per-column tables, FP32 upload, and the FP64 sample count.
//
// The geometry follows the circular orbit of arXiv 2512.21180, Sec. 2.2
// (source-isocenter and source-detector distances, lateral panel offset,
// full 2 pi orbit); the tables are the closed-form ray parameters of the
// plane-sampled line integral documented in cbct.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "cbct_internal.h"

namespace cbct {

static thread_local char g_hip_msg[256];

void set_hip_error(hipError_t e)
{
    std::snprintf(g_hip_msg, sizeof g_hip_msg, "%s (%d)", hipGetErrorString(e), (int)e);
}

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Ray direction of column iu at angle (c, s), z component excluded.
inline void ray_xy(const cbct_geom_desc &d, double c, double s, int iu, double *dx, double *dy)
{
    double U = d.off_u_mm + (iu - 0.5 * (d.nu - 1)) * d.du_mm;
    *dx = -d.sdd_mm * c - U * s;
    *dy = -d.sdd_mm * s + U * c;
}

// Integer range [lo, hi] of p with L < b + p*s < H (p unrestricted).
inline void open_range(double b, double s, double L, double H, int64_t *lo, int64_t *hi)
{
    if (s == 0.0) {
        if (L < b && b < H) {
            *lo = INT64_MIN / 4;
            *hi = INT64_MAX / 4;
        } else {
            *lo = 1;
            *hi = 0;
        }
        return;
    }
    double a = (L - b) / s, z = (H - b) / s;
    if (s < 0.0)
        std::swap(a, z);
    *lo = (int64_t)std::floor(a) + 1;
    *hi = (int64_t)std::ceil(z) - 1;
}

}  // namespace

}  // namespace cbct

using namespace cbct;

extern "C" const char *cbct_error_string(cbct_status e)
{
    switch (e) {
    case CBCT_OK: return "ok";
    case CBCT_E_NULL: return "null pointer argument";
    case CBCT_E_GEOM: return "invalid geometry";
    case CBCT_E_DTYPE: return "unsupported storage type";
    case CBCT_E_SHAPE: return "size out of range";
    case CBCT_E_HIP: return "HIP runtime error";
    case CBCT_E_ALLOC: return "allocation failed";
    case CBCT_E_ARG: return "invalid argument";
    }
    return "unknown status";
}

extern "C" const char *cbct_last_hip_error(void) { return g_hip_msg; }

static cbct_status validate(const cbct_geom_desc &d, const std::vector<double> &ang,
                            std::vector<AngRec> &angs)
{
    if (!finite_pos(d.sid_mm) || !finite_pos(d.sdd_mm) || !(d.sdd_mm > d.sid_mm))
        return CBCT_E_GEOM;
    if (d.n_angles <= 0 || d.nu <= 0 || d.nv <= 0 || d.nx <= 0 || d.ny <= 0 || d.nz <= 0)
        return CBCT_E_GEOM;
    if (!finite_pos(d.du_mm) || !finite_pos(d.dv_mm) || !finite_pos(d.vx_mm) ||
        !finite_pos(d.vy_mm) || !finite_pos(d.vz_mm))
        return CBCT_E_GEOM;
    if (!std::isfinite(d.off_u_mm) || !std::isfinite(d.off_v_mm) ||
        !std::isfinite(d.origin_mm[0]) || !std::isfinite(d.origin_mm[1]) ||
        !std::isfinite(d.origin_mm[2]))
        return CBCT_E_GEOM;
    if ((int64_t)d.n_angles * d.nv * d.nu >= (int64_t(1) << 31) ||
        (int64_t)d.nx * d.ny * d.nz >= (int64_t(1) << 31))
        return CBCT_E_GEOM;
    for (double a : ang)
        if (!std::isfinite(a))
            return CBCT_E_GEOM;

    // Support of the in-plane interpolation reaches one voxel beyond the
    // outer centres; all of it must be strictly between source and panel.
    double hx = 0.5 * (d.nx + 1) * d.vx_mm, hy = 0.5 * (d.ny + 1) * d.vy_mm;
    double R = 0.0;
    for (int q = 0; q < 4; ++q) {
        double x = d.origin_mm[0] + ((q & 1) ? hx : -hx);
        double y = d.origin_mm[1] + ((q & 2) ? hy : -hy);
        R = std::max(R, std::sqrt(x * x + y * y));
    }
    if (!(R < std::min(d.sid_mm, d.sdd_mm - d.sid_mm)))
        return CBCT_E_GEOM;

    double vmax = std::max(std::fabs(d.off_v_mm - 0.5 * (d.nv - 1) * d.dv_mm),
                           std::fabs(d.off_v_mm + 0.5 * (d.nv - 1) * d.dv_mm));
    angs.resize(d.n_angles);
    for (int a = 0; a < d.n_angles; ++a) {
        double c = std::cos(ang[a]), s = std::sin(ang[a]);
        int switches = 0, prev = -1, x_lo = 0, x_hi = 0;
        bool any_x = false;
        for (int iu = 0; iu < d.nu; ++iu) {
            double dx, dy;
            ray_xy(d, c, s, iu, &dx, &dy);
            if (!(vmax < std::max(std::fabs(dx), std::fabs(dy))))
                return CBCT_E_GEOM;
            int is_x = std::fabs(dx) >= std::fabs(dy);
            if (prev >= 0 && is_x != prev)
                ++switches;
            prev = is_x;
            if (is_x) {
                if (!any_x)
                    x_lo = iu;
                any_x = true;
                x_hi = iu + 1;
            }
        }
        if (switches > 1)
            return CBCT_E_GEOM;
        angs[a].c = (float)c;
        angs[a].s = (float)s;
        angs[a].x_lo = any_x ? x_lo : 0;
        angs[a].x_hi = any_x ? x_hi : 0;
    }
    return CBCT_OK;
}

// FP64 ray-family constants for column iu at angle index a.
static void column_constants(const cbct_geom_desc &d, double th, int iu, ColRec *r, int *is_x)
{
    double c = std::cos(th), s = std::sin(th);
    double Sx = d.sid_mm * c, Sy = d.sid_mm * s;
    double dx, dy;
    ray_xy(d, c, s, iu, &dx, &dy);
    bool xm = std::fabs(dx) >= std::fabs(dy);
    double dm = xm ? dx : dy, dq = xm ? dy : dx;
    double Sm = xm ? Sx : Sy, Sq = xm ? Sy : Sx;
    double vm = xm ? d.vx_mm : d.vy_mm, vq = xm ? d.vy_mm : d.vx_mm;
    double om = xm ? d.origin_mm[0] : d.origin_mm[1], oq = xm ? d.origin_mm[1] : d.origin_mm[0];
    int nm = xm ? d.nx : d.ny, nq = xm ? d.ny : d.nx;
    double c0 = om - 0.5 * (nm - 1) * vm;          // centre of plane 0 along m
    double t0 = (c0 - Sm) / dm, tau = vm / dm;
    r->pb = (float)((Sq - oq + t0 * dq) / vq + 0.5 * (nq - 1));
    r->ps = (float)(tau * dq / vq);
    r->t0 = (float)t0;
    r->tau = (float)tau;
    r->dsf = (float)(vm / std::fabs(dm));
    r->n2 = (float)(dx * dx + dy * dy);
    r->pad0 = r->pad1 = 0.0f;
    *is_x = xm;
}

// Samples with non-empty support, in FP64 from the closed-form ray lines.
static uint64_t count_samples(const cbct_geom_desc &d, const std::vector<double> &ang)
{
    double Kb = 0.5 * (d.nz - 1) - d.origin_mm[2] / d.vz_mm;
    uint64_t total = 0;
    for (int a = 0; a < d.n_angles; ++a) {
        double th = ang[a];
        double c = std::cos(th), s = std::sin(th);
        double Sx = d.sid_mm * c, Sy = d.sid_mm * s;
        for (int iu = 0; iu < d.nu; ++iu) {
            double dx, dy;
            ray_xy(d, c, s, iu, &dx, &dy);
            bool xm = std::fabs(dx) >= std::fabs(dy);
            double dm = xm ? dx : dy, dq = xm ? dy : dx;
            double Sm = xm ? Sx : Sy, Sq = xm ? Sy : Sx;
            double vm = xm ? d.vx_mm : d.vy_mm, vq = xm ? d.vy_mm : d.vx_mm;
            double om = xm ? d.origin_mm[0] : d.origin_mm[1];
            double oq = xm ? d.origin_mm[1] : d.origin_mm[0];
            int nm = xm ? d.nx : d.ny, nq = xm ? d.ny : d.nx;
            double t0 = (om - 0.5 * (nm - 1) * vm - Sm) / dm, tau = vm / dm;
            double pb = (Sq - oq + t0 * dq) / vq + 0.5 * (nq - 1), ps = tau * dq / vq;
            int64_t lq, hq;
            open_range(pb, ps, -1.0, (double)nq, &lq, &hq);
            lq = std::max<int64_t>(lq, 0);
            hq = std::min<int64_t>(hq, nm - 1);
            if (hq < lq)
                continue;
            for (int iv = 0; iv < d.nv; ++iv) {
                double Vz = (d.off_v_mm + (iv - 0.5 * (d.nv - 1)) * d.dv_mm) / d.vz_mm;
                int64_t lk, hk;
                open_range(Kb + t0 * Vz, tau * Vz, -1.0, (double)d.nz, &lk, &hk);
                int64_t lo = std::max(lq, lk), hi = std::min(hq, hk);
                if (hi >= lo)
                    total += (uint64_t)(hi - lo + 1);
            }
        }
    }
    return total;
}

extern "C" cbct_status cbct_geom_create(const cbct_geom_desc *desc, cbct_geom **out)
{
    if (!desc || !out)
        return CBCT_E_NULL;
    *out = nullptr;
    const cbct_geom_desc &d = *desc;
    if (d.n_angles <= 0)
        return CBCT_E_GEOM;
    std::vector<double> ang((size_t)d.n_angles);
    for (int a = 0; a < d.n_angles; ++a)
        ang[a] = d.angles_rad ? d.angles_rad[a] : kTwoPi * a / d.n_angles;
    std::vector<AngRec> angs;
    cbct_status st = validate(d, ang, angs);
    if (st != CBCT_OK)
        return st;

    cbct_geom *g = new (std::nothrow) cbct_geom();
    if (!g)
        return CBCT_E_ALLOC;
    g->desc = d;
    g->angles = std::move(ang);
    g->desc.angles_rad = g->angles.data();
    g->angs = std::move(angs);

    g->cols.resize((size_t)d.n_angles * d.nu);
    for (int a = 0; a < d.n_angles; ++a)
        for (int iu = 0; iu < d.nu; ++iu) {
            int is_x;
            column_constants(d, g->angles[a], iu, &g->cols[(size_t)a * d.nu + iu], &is_x);
        }
    std::vector<float2> rows((size_t)d.nv);
    for (int iv = 0; iv < d.nv; ++iv) {
        double V = d.off_v_mm + (iv - 0.5 * (d.nv - 1)) * d.dv_mm;
        rows[iv] = make_float2((float)(V / d.vz_mm), (float)(V * V));
    }

    size_t ncol = g->cols.size() * sizeof(ColRec);
    size_t nang = g->angs.size() * sizeof(AngRec);
    size_t nrow = rows.size() * sizeof(float2);
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t total = up(ncol) + up(nang) + up(nrow);

    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess)
        e = hipMalloc(&g->dev_block, total);
    if (e == hipSuccess) {
        char *base = (char *)g->dev_block;
        e = hipMemcpy(base, g->cols.data(), ncol, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(base + up(ncol), g->angs.data(), nang, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(base + up(ncol) + up(nang), rows.data(), nrow, hipMemcpyHostToDevice);
        g->dev.cols = (const ColRec *)base;
        g->dev.angs = (const AngRec *)(base + up(ncol));
        g->dev.rows = (const float2 *)(base + up(ncol) + up(nang));
    }
    if (e != hipSuccess) {
        set_hip_error(e);
        if (g->dev_block)
            (void)hipFree(g->dev_block);
        delete g;
        return e == hipErrorOutOfMemory ? CBCT_E_ALLOC : CBCT_E_HIP;
    }

    DevGeom &v = g->dev;
    v.n_angles = d.n_angles;
    v.nu = d.nu;
    v.nv = d.nv;
    v.nx = d.nx;
    v.ny = d.ny;
    v.nz = d.nz;
    v.Kb = (float)(0.5 * (d.nz - 1) - d.origin_mm[2] / d.vz_mm);
    v.vx = (float)d.vx_mm;
    v.vy = (float)d.vy_mm;
    v.vz = (float)d.vz_mm;
    v.ox = (float)d.origin_mm[0];
    v.oy = (float)d.origin_mm[1];
    v.oz = (float)d.origin_mm[2];
    v.sid = (float)d.sid_mm;
    v.sdd = (float)d.sdd_mm;
    v.du = (float)d.du_mm;
    v.dv = (float)d.dv_mm;
    v.off_u = (float)d.off_u_mm;
    v.off_v = (float)d.off_v_mm;
    v.cu = (float)(0.5 * (d.nu - 1));
    v.cv = (float)(0.5 * (d.nv - 1));
    v.rv0 = (float)(d.off_v_mm / d.vz_mm);
    v.rvs = (float)(d.dv_mm / d.vz_mm);

    g->samples = count_samples(g->desc, g->angles);
    *out = g;
    return CBCT_OK;
}

extern "C" cbct_status cbct_geom_destroy(cbct_geom *g)
{
    if (!g)
        return CBCT_OK;
    cbct_status st = CBCT_OK;
    if (g->dev_block) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != g->device)
            (void)hipSetDevice(g->device);
        hipError_t e = hipFree(g->dev_block);
        if (cur != g->device && cur >= 0)
            (void)hipSetDevice(cur);
        if (e != hipSuccess) {
            set_hip_error(e);
            st = CBCT_E_HIP;
        }
    }
    delete g;
    return st;
}

extern "C" cbct_status cbct_sample_count(const cbct_geom *g, uint64_t *samples)
{
    if (!g || !samples)
        return CBCT_E_NULL;
    *samples = g->samples;
    return CBCT_OK;
}

extern "C" cbct_status cbct_geom_sizes(const cbct_geom *g, uint64_t *n_vox, uint64_t *n_sino)
{
    if (!g)
        return CBCT_E_NULL;
    if (n_vox)
        *n_vox = (uint64_t)g->desc.nx * g->desc.ny * g->desc.nz;
    if (n_sino)
        *n_sino = (uint64_t)g->desc.n_angles * g->desc.nv * g->desc.nu;
    return CBCT_OK;
}
