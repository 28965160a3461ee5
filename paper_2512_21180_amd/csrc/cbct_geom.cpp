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
#include <cstddef>
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
    // kernels index one projection with 24-bit multiplies
    if (d.nu > 65536 || d.nv > 65536 || d.nx > 65536 || d.ny > 65536 || d.nz > 65536)
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

// FP32 table record of column iu at angle th.
static void column_constants(const cbct_geom_desc &d, double th, int iu, ColRec *r, int *is_x)
{
    Col64 k = col_consts64(d, std::cos(th), std::sin(th), iu);
    double vm = k.xm ? d.vx_mm : d.vy_mm;
    r->pb = (float)k.pb;
    r->ps = (float)k.ps;
    r->t0 = (float)k.t0;
    r->tau = (float)k.tau;
    r->dsf = (float)(vm / std::fabs(k.xm ? k.dx : k.dy));
    r->n2 = (float)(k.dx * k.dx + k.dy * k.dy);
    r->pad0 = r->pad1 = 0.0f;
    *is_x = k.xm;
}

// Samples with non-empty support, in FP64 from the closed-form ray lines.
static uint64_t count_samples(const cbct_geom_desc &d, const std::vector<double> &ang)
{
    double Kb = 0.5 * (d.nz - 1) - d.origin_mm[2] / d.vz_mm;
    uint64_t total = 0;
    for (int a = 0; a < d.n_angles; ++a) {
        double c = std::cos(ang[a]), s = std::sin(ang[a]);
        for (int iu = 0; iu < d.nu; ++iu) {
            Col64 k = col_consts64(d, c, s, iu);
            int nm = k.xm ? d.nx : d.ny, nq = k.xm ? d.ny : d.nx;
            int64_t lq, hq;
            open_range(k.pb, k.ps, -1.0, (double)nq, &lq, &hq);
            lq = std::max<int64_t>(lq, 0);
            hq = std::min<int64_t>(hq, nm - 1);
            if (hq < lq)
                continue;
            for (int iv = 0; iv < d.nv; ++iv) {
                double Vz = (d.off_v_mm + (iv - 0.5 * (d.nv - 1)) * d.dv_mm) / d.vz_mm;
                int64_t lk, hk;
                open_range(Kb + k.t0 * Vz, k.tau * Vz, -1.0, (double)d.nz, &lk, &hk);
                int64_t lo = std::max(lq, lk), hi = std::min(hq, hk);
                if (hi >= lo)
                    total += (uint64_t)(hi - lo + 1);
            }
        }
    }
    return total;
}

// Everything that needs no device: validation, FP64 tables rounded to FP32,
// launch plans and the sample count.
static cbct_status host_setup(const cbct_geom_desc *desc, cbct_geom **out)
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
    g->rows.resize((size_t)d.nv);
    for (int iv = 0; iv < d.nv; ++iv) {
        double V = d.off_v_mm + (iv - 0.5 * (d.nv - 1)) * d.dv_mm;
        g->rows[iv] = make_float2((float)(V / d.vz_mm), (float)(V * V));
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

    plan_host(g);
    g->samples = count_samples(g->desc, g->angles);
    *out = g;
    return CBCT_OK;
}

// Upload the tables and the tile list to the current device.
static hipError_t device_upload(cbct_geom *g)
{
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t ncol = g->cols.size() * sizeof(ColRec);
    size_t nang = g->angs.size() * sizeof(AngRec);
    size_t nrow = g->rows.size() * sizeof(float2);
    size_t ntile = g->tiles.size() * sizeof(TileRec);
    size_t nwin = g->wins.size() * sizeof(BrickWin);
    size_t total = up(ncol) + up(nang) + up(nrow) + up(ntile) + up(nwin);
    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess)
        e = hipMalloc(&g->dev_block, total);
    if (e != hipSuccess)
        return e;
    char *base = (char *)g->dev_block;
    char *pc = base, *pa = pc + up(ncol), *pr = pa + up(nang), *pt = pr + up(nrow);
    char *pw = pt + up(ntile);
    e = hipMemcpy(pc, g->cols.data(), ncol, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(pa, g->angs.data(), nang, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(pr, g->rows.data(), nrow, hipMemcpyHostToDevice);
    if (e == hipSuccess && ntile)
        e = hipMemcpy(pt, g->tiles.data(), ntile, hipMemcpyHostToDevice);
    if (e == hipSuccess && nwin)
        e = hipMemcpy(pw, g->wins.data(), nwin, hipMemcpyHostToDevice);
    g->dev.cols = (const ColRec *)pc;
    g->dev.angs = (const AngRec *)pa;
    g->dev.rows = (const float2 *)pr;
    g->fwd.tiles = ntile ? (const TileRec *)pt : nullptr;
    g->adj.wins = nwin ? (const BrickWin *)pw : nullptr;
    return e;
}

extern "C" cbct_status cbct_geom_create(const cbct_geom_desc *desc, cbct_geom **out)
{
    cbct_geom *g = nullptr;
    cbct_status st = host_setup(desc, &g);
    if (st != CBCT_OK)
        return st;
    hipError_t e = device_upload(g);
    if (e != hipSuccess) {
        set_hip_error(e);
        cbct_geom_destroy(g);
        return e == hipErrorOutOfMemory ? CBCT_E_ALLOC : CBCT_E_HIP;
    }
    *out = g;
    return CBCT_OK;
}

extern "C" cbct_status cbct_geom_create_host(const cbct_geom_desc *desc, cbct_geom **out)
{
    return host_setup(desc, out);
}

extern "C" cbct_status cbct_geom_table(const cbct_geom *g, int which, void *dst, size_t cap,
                                       size_t *bytes)
{
    if (!g || !bytes)
        return CBCT_E_NULL;
    const void *src = nullptr;
    size_t n = 0;
    switch (which) {
    case 0: src = g->cols.data(); n = g->cols.size() * sizeof(ColRec); break;
    case 1: src = g->angs.data(); n = g->angs.size() * sizeof(AngRec); break;
    case 2: src = g->rows.data(); n = g->rows.size() * sizeof(float2); break;
    case 3: src = g->tiles.data(); n = g->tiles.size() * sizeof(TileRec); break;
    case 4: src = &g->dev; n = offsetof(DevGeom, cols); break;
    case 5: src = g->wins.data(); n = g->wins.size() * sizeof(BrickWin); break;
    default: return CBCT_E_ARG;
    }
    *bytes = n;
    if (dst) {
        if (cap < n)
            return CBCT_E_SHAPE;
        std::memcpy(dst, src, n);
    }
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
