// Internal definitions shared by the host set-up and the HIP kernels of
// libcbct.so.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "cbct.h"

namespace cbct {

// Per (angle, column) ray-family constants, rounded from FP64.  For a column
// sampled along axis m (x or y) with in-plane axis o, plane index p:
//   in-plane fractional index   q(p) = pb + p * ps
//   ray parameter               t(p) = t0 + p * tau
//   z fractional index          k(p) = Kb + t(p) * Vz(iv)   (Vz = V(iv) / vz)
//   length per plane            ds   = dsf * sqrt(n2 + V(iv)^2)
struct ColRec {
    float pb, ps;      // in-plane fractional index base and slope
    float t0, tau;     // ray parameter at plane 0 and per plane
    float dsf, n2;     // vox_m / |d_m|, d_x^2 + d_y^2
    float pad0, pad1;
};
static_assert(sizeof(ColRec) == 32, "ColRec layout");

// Per-angle constants.
struct AngRec {
    float c, s;        // cos, sin of the source angle
    int x_lo, x_hi;    // columns [x_lo, x_hi) are sampled along x, the others along y
};
static_assert(sizeof(AngRec) == 16, "AngRec layout");

// Everything a kernel needs about one geometry, passed by value.
struct DevGeom {
    int n_angles, nu, nv, nx, ny, nz;
    float Kb;          // (nz-1)/2 - oz/vz
    float vx, vy, vz;  // voxel pitch
    float ox, oy, oz;  // volume centre
    float sid, sdd;
    float du, dv, off_u, off_v;
    float cu, cv;      // (nu-1)/2, (nv-1)/2
    float rv0, rvs;    // Vz(iv) = rv0 + (iv - cv) * rvs
    const ColRec *cols;  // [n_angles][nu]
    const float2 *rows;  // [nv]: (Vz, V^2)
    const AngRec *angs;  // [n_angles]
};

}  // namespace cbct

struct cbct_geom {
    cbct_geom_desc desc;             // copy; desc.angles_rad points at `angles`
    std::vector<double> angles;
    int device = -1;
    cbct::DevGeom dev{};             // device-table pointers live in `dev`
    void *dev_block = nullptr;       // one allocation for all tables
    uint64_t samples = 0;            // cbct_sample_count, computed at creation
    // Host copies, kept for the batch scheduler and for tests.
    std::vector<cbct::ColRec> cols;
    std::vector<cbct::AngRec> angs;
};

namespace cbct {

void set_hip_error(hipError_t e);

// Kernel launchers (cbct_kernels.hip).  They assume validated arguments.
hipError_t launch_forward(const DevGeom &g, const void *vol, cbct_dtype vt, void *sino,
                          cbct_dtype st, int channels, hipStream_t s);
hipError_t launch_adjoint(const DevGeom &g, const void *sino, cbct_dtype st, void *vol,
                          cbct_dtype vt, int channels, hipStream_t s);

}  // namespace cbct
