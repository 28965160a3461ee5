// Forward projector A for gfx950: plane sweep over LDS-staged boxes.
//
// Operator: the plane-sampled cone-beam line integral (arXiv 2512.21180,
// Sec. 2.2, projection operator P).  A workgroup owns one tile of up to 64
// columns x 4R rows of one angle, all sampled along the same axis; wave w
// holds rows [w R, w R + R) and lane l column u0 + l, so each thread carries
// R rays of one column and shares their in-plane interpolation index.
//
// The tile sweeps the voxel-centre planes of its axis.  On plane p every ray
// of the tile lands inside a BQ x BK box of (in-plane, z) voxels whose origin
// follows the corner rays; the box is staged in LDS (zero outside the
// volume) one plane ahead of its use, double-buffered, one barrier per plane.
// Each sample is the bilinear interpolant read from LDS; each ray keeps its
// own running sum in a register, so the summation order is the plane order
// whatever the launch shape, and the result is written once, coalesced along
// the detector row.  Tiles are assigned XCD-contiguously so that the
// workgroups sharing an L2 work on neighbouring tiles of the same angle.
#include <hip/hip_runtime.h>

#include "cbct_internal.h"
#include "cbct_storage.h"

namespace cbct {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxStage = 4;   // staged voxels per thread per plane (BQ*BK <= 1024)

struct SweepArgs {
    DevGeom g;
    const TileRec *tiles;
    int n_tiles;
    int BQ, BK;
};

template <int R, class VS, class SS>
__global__ void __launch_bounds__(kThreads)
forward_sweep(SweepArgs A, const typename VS::T *__restrict__ vol,
              typename SS::T *__restrict__ sino)
{
    extern __shared__ float lds[];
    const DevGeom &g = A.g;
    // XCD-contiguous tile order: workgroups are dealt to the 8 XCDs round
    // robin, so XCD x receives ids x, x+8, ...; give it tiles
    // [x * n/8, (x+1) * n/8).
    const int nb = gridDim.x;
    const int t = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    const TileRec T = A.tiles[t];
    if (T.nu_t == 0)
        return;
    const int ch = blockIdx.y;
    const size_t nvox = (size_t)g.nx * g.ny * g.nz;
    const size_t nsino = (size_t)g.n_angles * g.nv * g.nu;
    const typename VS::T *v = vol + ch * nvox;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int ul = min(lane, T.nu_t - 1);
    const ColRec c = g.cols[(size_t)T.a * g.nu + T.u0 + ul];

    float kb[R], ks[R], acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int vr = T.v0 + min(w * R + r, T.nv_t - 1);
        const float vz = g.rows[vr].x;
        kb[r] = fmaf(c.t0, vz, g.Kb);
        ks[r] = c.tau * vz;
        acc[r] = 0.0f;
    }

    // corner rays (uniform): columns u0 and u0 + nu_t - 1, rows v0 and v0 + nv_t - 1
    const ColRec cA = g.cols[(size_t)T.a * g.nu + T.u0];
    const ColRec cB = g.cols[(size_t)T.a * g.nu + T.u0 + T.nu_t - 1];
    const float zA = g.rows[T.v0].x, zB = g.rows[T.v0 + T.nv_t - 1].x;
    const float kbA0 = fmaf(cA.t0, zA, g.Kb), ksA0 = cA.tau * zA;
    const float kbA1 = fmaf(cA.t0, zB, g.Kb), ksA1 = cA.tau * zB;
    const float kbB0 = fmaf(cB.t0, zA, g.Kb), ksB0 = cB.tau * zA;
    const float kbB1 = fmaf(cB.t0, zB, g.Kb), ksB1 = cB.tau * zB;

    const int BQ = A.BQ, BK = A.BK, box = BQ * BK;
    const bool xp = T.cls == 0;
    const int nq = xp ? g.ny : g.nx;
    const size_t sp = xp ? 1 : (size_t)g.nx;     // plane stride
    const size_t sq = xp ? (size_t)g.nx : 1;     // in-plane stride
    const size_t sk = (size_t)g.nx * g.ny;       // z stride

    // this thread's staged voxels: box cells e = tid + 256 s
    int eq[kMaxStage], ek[kMaxStage];
#pragma unroll
    for (int s = 0; s < kMaxStage; ++s) {
        const int e = tid + kThreads * s;
        ek[s] = e / BQ;
        eq[s] = e - ek[s] * BQ;
    }

    auto origin = [&](int p, int &qlo, int &klo) {
        const float fp = (float)p;
        const float qa = fmaf(fp, cA.ps, cA.pb), qb = fmaf(fp, cB.ps, cB.pb);
        const float k0 = fmaf(fp, ksA0, kbA0), k1 = fmaf(fp, ksA1, kbA1);
        const float k2 = fmaf(fp, ksB0, kbB0), k3 = fmaf(fp, ksB1, kbB1);
        qlo = (int)floorf(fminf(qa, qb)) - 1;
        klo = (int)floorf(fminf(fminf(k0, k1), fminf(k2, k3))) - 1;
    };
    auto fetch = [&](int p, int qlo, int klo, float (&st)[kMaxStage]) {
#pragma unroll
        for (int s = 0; s < kMaxStage; ++s) {
            st[s] = 0.0f;
            const int q = qlo + eq[s], k = klo + ek[s];
            if (tid + kThreads * s < box && q >= 0 && q < nq && k >= 0 && k < g.nz)
                st[s] = VS::ld(v, (size_t)k * sk + (size_t)q * sq + (size_t)p * sp);
        }
    };

    int p = T.p_lo;
    int qlo = 0, klo = 0;
    float stage[kMaxStage];
    if (p <= T.p_hi) {
        origin(p, qlo, klo);
        fetch(p, qlo, klo, stage);
    }
    for (; p <= T.p_hi; ++p) {
        float *buf = lds + (p & 1) * box;
#pragma unroll
        for (int s = 0; s < kMaxStage; ++s)
            if (tid + kThreads * s < box)
                buf[tid + kThreads * s] = stage[s];
        const int qc = qlo, kc = klo;
        __syncthreads();
        if (p < T.p_hi) {
            origin(p + 1, qlo, klo);
            fetch(p + 1, qlo, klo, stage);
        }
        const float fp = (float)p;
        const float q = fmaf(fp, c.ps, c.pb);
        const float qf = floorf(q);
        const float wq = q - qf;
        const int qi = (int)qf - qc;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float k = fmaf(fp, ks[r], kb[r]);
            const float kf = floorf(k);
            const float wk = k - kf;
            const int idx = ((int)kf - kc) * BQ + qi;
            const float v00 = buf[idx], v10 = buf[idx + 1];
            const float v01 = buf[idx + BQ], v11 = buf[idx + BQ + 1];
            const float lo = fmaf(wq, v10 - v00, v00);
            const float hi = fmaf(wq, v11 - v01, v01);
            acc[r] += fmaf(wk, hi - lo, lo);
        }
    }

    if (lane < T.nu_t) {
        const float ds0 = c.dsf;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int vr = w * R + r;
            if (vr < T.nv_t) {
                const int iv = T.v0 + vr;
                const float ds = ds0 * sqrtf(c.n2 + g.rows[iv].y);
                SS::st(sino, ch * nsino + ((size_t)T.a * g.nv + iv) * g.nu + T.u0 + lane,
                       acc[r] * ds);
            }
        }
    }
}

}  // namespace

hipError_t launch_forward_tiled(const DevGeom &g, const FwdPlan &p, const void *vol,
                                cbct_dtype vt, void *sino, cbct_dtype st, int channels,
                                hipStream_t s)
{
    SweepArgs A{g, p.tiles, p.n_tiles, p.BQ, p.BK};
    const size_t lds = 2 * (size_t)p.BQ * p.BK * sizeof(float);
    dim3 grid(p.n_tiles, channels), block(kThreads);
    return dispatch_storage(vt, st, [&](auto vs, auto ss) -> hipError_t {
        using VS = decltype(vs);
        using SS = decltype(ss);
        const auto *x = (const typename VS::T *)vol;
        auto *y = (typename SS::T *)sino;
        switch (p.R) {
        case 4: hipLaunchKernelGGL((forward_sweep<4, VS, SS>), grid, block, lds, s, A, x, y); break;
        case 2: hipLaunchKernelGGL((forward_sweep<2, VS, SS>), grid, block, lds, s, A, x, y); break;
        default: hipLaunchKernelGGL((forward_sweep<1, VS, SS>), grid, block, lds, s, A, x, y); break;
        }
        return hipGetLastError();
    });
}

}  // namespace cbct
