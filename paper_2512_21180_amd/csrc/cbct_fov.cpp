// Field-of-view tensor V of the learned primal-dual (arXiv 2512.21180,
// Sec. 2.6: V(p) is the fraction of projections in which voxel p is
// visible).  Host FP64, once per geometry, like the rest of the set-up.
//
// A voxel is visible at source angle theta when the ray from the source
// through its centre meets the panel's sensitive area
//   |u - off_u| <= nu du / 2  and  |v - off_v| <= nv dv / 2,
// with u = sdd (c_y cos - c_x sin) / D, v = sdd c_z / D and depth
// D = sid - (c_x cos + c_y sin) > 0 along the central ray.  For one column
// (x, y) and angle the visible z form an interval, so each (column, angle)
// adds one to a run of z: a difference array per column.  The run's ends
// are found by division and then settled by the direct test of the voxels
// at and next to them, so every decision is the direct test in FP64.
#include <cmath>
#include <vector>

#include "cbct_internal.h"
#include "cbct_nn.h"

namespace {

struct VTest {
    double sdd, half_v, off_v;
    bool operator()(double cz, double D) const
    {
        const double v = sdd * cz / D;
        return v >= off_v - half_v && v <= off_v + half_v;
    }
};

}  // namespace

extern "C" cbct_status cbct_fov_fraction(const cbct_geom *g, float *out)
{
    if (!g || !out)
        return CBCT_E_NULL;
    const cbct_geom_desc &d = g->desc;
    const int nx = d.nx, ny = d.ny, nz = d.nz, na = d.n_angles;
    const double half_u = 0.5 * d.nu * d.du_mm;
    const VTest vt{d.sdd_mm, 0.5 * d.nv * d.dv_mm, d.off_v_mm};
    std::vector<double> cs(na), sn(na);
    for (int a = 0; a < na; ++a) {
        cs[a] = std::cos(g->angles[a]);
        sn[a] = std::sin(g->angles[a]);
    }
    auto cz_of = [&](int iz) { return d.origin_mm[2] + (iz - 0.5 * (nz - 1)) * d.vz_mm; };
    std::vector<int> diff(nz + 1);
    for (int iy = 0; iy < ny; ++iy) {
        const double cy = d.origin_mm[1] + (iy - 0.5 * (ny - 1)) * d.vy_mm;
        for (int ix = 0; ix < nx; ++ix) {
            const double cx = d.origin_mm[0] + (ix - 0.5 * (nx - 1)) * d.vx_mm;
            std::fill(diff.begin(), diff.end(), 0);
            for (int a = 0; a < na; ++a) {
                const double D = d.sid_mm - (cx * cs[a] + cy * sn[a]);
                if (!(D > 0))
                    continue;
                const double u = d.sdd_mm * (cy * cs[a] - cx * sn[a]) / D;
                if (!(u >= d.off_u_mm - half_u && u <= d.off_u_mm + half_u))
                    continue;
                // z range from the v bounds, as fractional voxel indices
                const double zl = (vt.off_v - vt.half_v) * D / vt.sdd;
                const double zh = (vt.off_v + vt.half_v) * D / vt.sdd;
                const double fl = (zl - d.origin_mm[2]) / d.vz_mm + 0.5 * (nz - 1);
                const double fh = (zh - d.origin_mm[2]) / d.vz_mm + 0.5 * (nz - 1);
                if (fh < -1.0 || fl > nz)
                    continue;
                int lo = (int)std::max(0.0, std::min((double)nz - 1, std::ceil(fl)));
                int hi = (int)std::max(0.0, std::min((double)nz - 1, std::floor(fh)));
                // settle both ends by the direct test
                while (lo > 0 && vt(cz_of(lo - 1), D))
                    --lo;
                while (lo < nz && !vt(cz_of(lo), D))
                    ++lo;
                while (hi < nz - 1 && vt(cz_of(hi + 1), D))
                    ++hi;
                while (hi >= 0 && !vt(cz_of(hi), D))
                    --hi;
                if (lo > hi)
                    continue;
                diff[lo] += 1;
                diff[hi + 1] -= 1;
            }
            int run = 0;
            for (int iz = 0; iz < nz; ++iz) {
                run += diff[iz];
                out[((size_t)iz * ny + iy) * nx + ix] = (float)((double)run / na);
            }
        }
    }
    return CBCT_OK;
}
