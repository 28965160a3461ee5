// Internal definitions shared by the host set-up and the HIP kernels of
// libcbct.so.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
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

// One forward work item: a tile of up to 64 columns x TV rows of one angle,
// all sampled along the same axis, swept over planes [p_lo, p_hi].
struct TileRec {
    int a, cls;        // angle index; 0 = x planes, 1 = y planes
    int u0, nu_t;      // first column, column count (<= 64)
    int v0, nv_t;      // first row, row count (<= TV)
    int p_lo, p_hi;    // planes whose staging box meets the padded volume
};
static_assert(sizeof(TileRec) == 32, "TileRec layout");

// Forward plan: LDS box per plane is BQ (in-plane) x BK (z) voxels.
struct FwdPlan {
    bool ok = false;   // false: fall back to the one-thread-per-ray kernel
    int R = 4;         // rays per thread along v
    int TU = 64;       // tile columns, 64 or 32 (a wave then holds two row groups);
                       // tiles are TU x (256 / TU) R rays
    int BQ = 0, BK = 0;
    int n_tiles = 0;   // padded to a multiple of 8 (padding tiles have nu_t = 0)
    const TileRec *tiles = nullptr;   // device
};

// Row taps the adjoint reads per voxel and column: the needed count rounded
// up to a count its kernel is instantiated for (4..16, 18, 20, 24, 28, 32).
__host__ __device__ inline int adj_taps_rounded(int nt)
{
    if (nt <= 4)
        return 4;
    if (nt <= 16)
        return nt;
    if (nt <= 18)
        return 18;
    if (nt <= 20)
        return 20;
    if (nt <= 24)
        return 24;
    if (nt <= 28)
        return 28;
    return 32;
}

// The adjoint's row runs start at floor(v_c + 1 - delta), v_c the row where a
// ray crosses a voxel's lower z support: delta exceeds the FP32 rounding of
// v_c (a few units of the last place of a row index up to nv) several
// times, and is at least 2^-12 row.
__host__ __device__ inline float adj_start_delta(int nv)
{
    const float d = (float)nv * (1.0f / 1048576.0f);
    return d > (1.0f / 4096.0f) ? d : (1.0f / 4096.0f);
}

// Adjoint bricks: kAdjBI x kAdjBJ output voxel columns (x, y) and 4 KV
// voxels along z.  One wave's 64 lanes serve the brick's in-plane segments
// on either sampling axis: 8 planes x 8 segments on x planes (seven output
// rows need eight segments), 7 planes x 9 segments on y planes.
constexpr int kAdjBI = 8, kAdjBJ = 7;

// Adjoint plan: per angle the brick's panel
// footprint (at most W x H pixels, clipped to the panel) is staged in LDS.
// Panel window of one adjoint brick column (kAdjBI x kAdjBJ voxels, all z)
// at one angle, from the FP64 projections of its support box (voxel centres +- one
// pitch): columns [u0, u1] (u0 > u1: the column is not seen), the extreme
// source-panel scales (a point at height z lands at V = lambda z) and the
// row taps per voxel and column its rays need.
struct BrickWin {
    float lmin, lmax;
    uint32_t u01;      // u0 | u1 << 16 (columns below 65536)
    int nt;
};
static_assert(sizeof(BrickWin) == 16, "BrickWin layout");

struct AdjPlan {
    bool ok = false;   // false: fall back to the one-thread-per-voxel kernel
    int W = 0, H = 0;  // footprint bounds (columns, rows)
    int WS = 0;        // LDS column stride of the window (floats, 2 mod 4, > H)
    int NTmax = 0;     // largest row-tap count
    int KV = 4;        // voxels per thread along z: bricks are kAdjBI x kAdjBJ x 4 KV
    const BrickWin *wins = nullptr;   // device: [n_angles][nby][nbx]
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
    std::vector<float2> rows;
    std::vector<cbct::TileRec> tiles;
    std::vector<cbct::BrickWin> wins;   // adjoint brick-column windows
    cbct::FwdPlan fwd;               // fwd.tiles points into dev_block
    cbct::AdjPlan adj;
};

namespace cbct {

void set_hip_error(hipError_t e);

// FP64 constants of the rays of column iu at source angle (c, s): sampling
// axis and the closed-form lines of the in-plane index q(p) = pb + p ps and
// ray parameter t(p) = t0 + p tau over plane index p.
struct Col64 {
    bool xm;             // sampled on x planes
    double dx, dy;       // ray direction (xy part)
    double pb, ps, t0, tau;
};

inline Col64 col_consts64(const cbct_geom_desc &d, double c, double s, int iu)
{
    Col64 r;
    double U = d.off_u_mm + (iu - 0.5 * (d.nu - 1)) * d.du_mm;
    r.dx = -d.sdd_mm * c - U * s;
    r.dy = -d.sdd_mm * s + U * c;
    r.xm = (r.dx < 0 ? -r.dx : r.dx) >= (r.dy < 0 ? -r.dy : r.dy);
    double Sx = d.sid_mm * c, Sy = d.sid_mm * s;
    double dm = r.xm ? r.dx : r.dy, dq = r.xm ? r.dy : r.dx;
    double Sm = r.xm ? Sx : Sy, Sq = r.xm ? Sy : Sx;
    double vm = r.xm ? d.vx_mm : d.vy_mm, vq = r.xm ? d.vy_mm : d.vx_mm;
    double om = r.xm ? d.origin_mm[0] : d.origin_mm[1];
    double oq = r.xm ? d.origin_mm[1] : d.origin_mm[0];
    int nm = r.xm ? d.nx : d.ny, nq = r.xm ? d.ny : d.nx;
    r.t0 = (om - 0.5 * (nm - 1) * vm - Sm) / dm;
    r.tau = vm / dm;
    r.pb = (Sq - oq + r.t0 * dq) / vq + 0.5 * (nq - 1);
    r.ps = r.tau * dq / vq;
    return r;
}

// Library-owned device scratch (cbct_scratch.cpp): one buffer per device,
// grown on demand.  scratch_acquire locks the device's buffer, makes stream s
// wait for the previous user's work and returns the buffer in lease.ptr;
// after enqueueing its work on s the caller must call scratch_release, which
// records the completion event and unlocks.  Calls on different streams are
// thereby ordered on the buffer; the first call (and any that needs a larger
// buffer) allocates, so it must not run under stream capture.
struct ScratchLease {
    void *ptr = nullptr;
    int device = -1;
    std::unique_lock<std::mutex> lock;
};
hipError_t scratch_acquire(size_t bytes, hipStream_t s, ScratchLease &lease);
hipError_t scratch_release(hipStream_t s, ScratchLease &lease);

// Plans (cbct_plan.cpp): host FP64 analysis of tile boxes and brick
// footprints; fills g->tiles, g->fwd and g->adj (no device work).
void plan_host(cbct_geom *g);

// Kernel launchers.  They assume validated arguments.
hipError_t launch_forward_simple(const DevGeom &g, const void *vol, cbct_dtype vt, void *sino,
                                 cbct_dtype st, int channels, hipStream_t s);
hipError_t launch_adjoint_simple(const DevGeom &g, const void *sino, cbct_dtype st, void *vol,
                                 cbct_dtype vt, int channels, hipStream_t s);
hipError_t launch_forward_tiled(const DevGeom &g, const FwdPlan &p, const void *vol,
                                cbct_dtype vt, void *sino, cbct_dtype st, int channels,
                                hipStream_t s);
hipError_t launch_adjoint_brick(const DevGeom &g, const AdjPlan &p, const void *sino,
                                cbct_dtype st, void *vol, cbct_dtype vt, int channels,
                                hipStream_t s);

// Batched launches: one kernel launch over all cases' work items (one item
// per workgroup, the hardware dispatcher balances them).  All
// cases must have tiled (forward) or bricked (adjoint) plans.
constexpr int kMaxBatch = 16;
hipError_t launch_forward_batch(int n, const cbct_geom *const *g, const void *const *vols,
                                void *const *sinos, cbct_dtype vt, cbct_dtype st, hipStream_t s);
hipError_t launch_adjoint_batch(int n, const cbct_geom *const *g, const void *const *sinos,
                                void *const *vols, cbct_dtype st, cbct_dtype vt, hipStream_t s);

// Multichannel forward (cbct_forward_mc.hip): n groups of C = 2 or 4
// channels, each group one geometry with a tiled plan; vols and sinos hold
// n * C FP32 pointers, group-major.  The channels are first packed (vectors
// of C channels per voxel) into the library's scratch buffer.  Every
// channel's output is bitwise equal to the single-channel tiled kernel's.
// The largest C a geometry allows: 4 where its boxes fit 39 x 19 voxels
// (staged in 41 x 20 LDS rows), else 2 (65 x 32), 0 where the plan is not
// tiled or 16 bytes per voxel reach 4 GiB with 64 more z planes.
constexpr int kMaxMcChannels = 4;
constexpr int kMaxMcGroups = 8;
int forward_mc_max_channels(const cbct_geom *g);
hipError_t launch_forward_mc(int n, const cbct_geom *const *g, const float *const *vols,
                             float *const *sinos, int C, hipStream_t s);

// Dispatch to the tiled kernels when the plan allows, else the simple ones.
hipError_t launch_forward(const cbct_geom *g, const void *vol, cbct_dtype vt, void *sino,
                          cbct_dtype st, int channels, hipStream_t s);
hipError_t launch_adjoint(const cbct_geom *g, const void *sino, cbct_dtype st, void *vol,
                          cbct_dtype vt, int channels, hipStream_t s);

}  // namespace cbct
