// Forward projector A over C = 2 or 4 channels that share one geometry.
//
// Alg. 1 (arXiv 2512.21180) applies the projector to channel stacks (the
// dual block's input holds P applied to four primal channels and to the
// reconstruction).  Every channel's samples sit at the same points, so the
// geometry of a sample (the z index of the ray on the plane, its floor and
// fraction, the LDS address) is computed once here and used for all C
// channels; the plane boxes, their table and the staging offsets are shared
// too.  Per channel the interpolation is the single-channel kernel's
// (forward_sweep: same expressions, same plane order, same final ds
// product), so each channel's result is bitwise equal to a single-channel
// call.  FP32 storage only.
//
// The channels are first packed into a volume of C-float vectors per voxel
// (into the library's scratch buffer; 2 C x 4 bytes moved per voxel): each
// cache line a tile stages then serves every channel.  Staged from C
// separate volumes, the tiles' lines outgrew the L2 (the clinical 5-channel
// sweep took 2.6x the time of five single-channel calls); an extra volume
// for a fifth (or third) channel still doubled the lines and cost more than
// it saved, so stacks run as chunks of 4 and 2 channels (and one channel on
// the single-channel kernel).
//
// LDS holds the staged boxes in the same layout (one ds_read_b128 or _b64
// per bilinear corner).  Box rows have a compile-time stride QS and count
// ROWS: 41 x 20 where the plan's boxes fit 39 x 19 voxels (the clinical
// case and its coarser levels: four workgroups per CU at C = 4), else
// 65 x 32 (any tiled plan, two channels so that a workgroup stays within
// 64 KB of LDS).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cbct_internal.h"
#include "cbct_lds.h"
#include "cbct_transpose.h"
#include "cbct_storage.h"

namespace cbct {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxR = 8;        // rays per thread
constexpr int kBoxChunk = 256;  // planes whose boxes are tabulated at a time
static_assert(kBoxChunk == kThreads, "the box table is filled one plane per thread");


template <int N> struct VecOf;
template <> struct VecOf<2> { using T = float2; };
template <> struct VecOf<4> { using T = float4; };

// One packed voxel through a buffer resource (zero outside its range).
template <class V> __device__ __forceinline__ V buf_vec(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ float2 buf_vec<float2>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ float4 buf_vec<float4>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

__device__ __forceinline__ float comp(float2 v, int i) { return i == 0 ? v.x : v.y; }
__device__ __forceinline__ float comp(float4 v, int i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

template <int C, int QS, int ROWS>
struct McLayout {
    static_assert(C == 2 || C == 4, "2 or 4 channels");
    static_assert(ROWS % 4 == 0, "rows are staged four waves at a time");
    static constexpr int kSlots = ROWS / 4;
    static constexpr int kBuf = ROWS * QS * C;            // floats per staging buffer
    static constexpr size_t kLds = 2 * (size_t)kBuf * sizeof(float) + kBoxChunk * 16;
    static_assert(kLds <= 64 * 1024, "one workgroup within 64 KB of LDS");
};

// A group's volume as staged: the packed copy of its C channels.
struct McGroup {
    DevGeom g;
    const TileRec *tiles;
    int R, tub, n_tiles;
    const void *vg;      // [nz][ny][nx] vectors of C channels
    const void *vgt;     // the same with x and y swapped, [nz][nx][ny]
    float *sino[kMaxMcChannels];
};

constexpr int kMaxGroups = kMaxMcGroups;

struct McArgs {
    int n_groups, n_items;
    int first[kMaxGroups + 1];   // first item of each group
    McGroup grp[kMaxGroups];
};

template <int C, int QS, int ROWS, int RC>
__device__ __forceinline__ void sweep_tile_mc(const McGroup &M, const TileRec &T, float *lds)
{
    using L = McLayout<C, QS, ROWS>;
    using V0 = typename VecOf<C>::T;
    constexpr int kSlots = L::kSlots;
    const DevGeom &g = M.g;
    const int R = RC > 0 ? RC : M.R, tub = M.tub;   // RC: rays per thread fixed at compile time
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int uc = lane & ((1 << tub) - 1);
    const int row0 = ((w << (6 - tub)) + (lane >> tub)) * R;
    const int ul = min(uc, T.nu_t - 1);
    const ColRec c = g.cols[(size_t)T.a * g.nu + T.u0 + ul];

    float kb[kMaxR], ks[kMaxR], acc[C][kMaxR];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
        const int vr = T.v0 + min(row0 + min(r, R - 1), T.nv_t - 1);
        const float vz = g.rows[vr].x;
        kb[r] = fmaf(c.t0, vz, g.Kb);
        ks[r] = c.tau * vz;
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
            acc[ch][r] = 0.0f;
    }

    // corner rays and plane boxes: the single-channel kernel's arithmetic
    const ColRec cA = g.cols[(size_t)T.a * g.nu + T.u0];
    const ColRec cB = g.cols[(size_t)T.a * g.nu + T.u0 + T.nu_t - 1];
    const float zA = g.rows[T.v0].x, zB = g.rows[T.v0 + T.nv_t - 1].x;
    const float kbA0 = fmaf(cA.t0, zA, g.Kb), ksA0 = cA.tau * zA;
    const float kbA1 = fmaf(cA.t0, zB, g.Kb), ksA1 = cA.tau * zB;
    const float kbB0 = fmaf(cB.t0, zA, g.Kb), ksB0 = cB.tau * zA;
    const float kbB1 = fmaf(cB.t0, zB, g.Kb), ksB1 = cB.tau * zB;

    // tiles that sweep x planes stage from the transposed packed volume, so
    // a box row is contiguous there too (as in the single-channel sweep)
    const bool xp = T.cls == 0;
    const int nq = xp ? g.ny : g.nx;
    const void *src = xp ? M.vgt : M.vg;
    const int sp = xp ? g.ny : g.nx;
    const int sq = 1;
    const int sk = g.nx * g.ny;

    struct Box {
        int qlo, klo, qw, kw;
    };
    int4 *boxes = (int4 *)(lds + 2 * L::kBuf);
    auto fill_boxes = [&](int base) {
        const int p = base + tid;
        if (p <= T.p_hi) {
            const float fp = (float)p;
            const float qa = fmaf(fp, cA.ps, cA.pb), qb = fmaf(fp, cB.ps, cB.pb);
            const float k0 = fmaf(fp, ksA0, kbA0), k1 = fmaf(fp, ksA1, kbA1);
            const float k2 = fmaf(fp, ksB0, kbB0), k3 = fmaf(fp, ksB1, kbB1);
            const int qlo = (int)floorf(fminf(qa, qb)) - 1;
            const int klo = (int)floorf(fminf(fminf(k0, k1), fminf(k2, k3))) - 1;
            const int qw = min((int)floorf(fmaxf(qa, qb)) + 3 - qlo, QS - 1);
            const int kw = min((int)floorf(fmaxf(fmaxf(k0, k1), fmaxf(k2, k3))) + 3 - klo, ROWS);
            boxes[tid] = make_int4(qlo, klo, qw, kw);
        }
    };
    auto box_of = [&](int p, int base) {
        const int4 v = boxes[p - base];
        Box b;
        b.qlo = __builtin_amdgcn_readfirstlane(v.x);
        b.klo = __builtin_amdgcn_readfirstlane(v.y);
        b.qw = __builtin_amdgcn_readfirstlane(v.z);
        b.kw = __builtin_amdgcn_readfirstlane(v.w);
        return b;
    };
    // Slot s of wave w holds box row w + 4 s: one vector load per slot from
    // the packed volume through a buffer resource (zero outside it, as in
    // the single-channel sweep: slots below or above the volume, and lanes
    // outside it in plane, whose first offset is set to the end; 32-bit
    // offsets, the volume with 64 more planes stays under 4 GiB where this
    // kernel runs).
    const uint32_t vbytes = (uint32_t)sk * (uint32_t)g.nz * (uint32_t)sizeof(V0);
    const __amdgpu_buffer_rsrc_t vres =
        __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, (int)vbytes, kBufferWord3);
    const uint32_t step = 4u * (uint32_t)sk * (uint32_t)sizeof(V0);
    auto fetch = [&](int p, const Box &b, V0 (&st0)[kSlots]) {
        const int q = b.qlo + lane;
        const bool qin = lane < b.qw && (unsigned)q < (unsigned)nq;
        const int n_sl = (b.kw - w + 3) >> 2;
        const uint32_t off0 =
            qin ? (__umul24((uint32_t)q, (uint32_t)sq) + (uint32_t)p * (uint32_t)sp +
                   (uint32_t)(b.klo + w) * (uint32_t)sk) *
                      (uint32_t)sizeof(V0)
                : vbytes;
#pragma unroll
        for (int s = 0; s < kSlots; ++s)
            if (s < n_sl)
                st0[s] = buf_vec<V0>(vres, off0 + (uint32_t)s * step);
    };

    __syncthreads();   // the previous work item's readers of lds are done
    int p = T.p_lo, base = T.p_lo;
    fill_boxes(base);
    __syncthreads();
    Box nb{0, 0, 0, 0};
    V0 stage0[kSlots];
    if (p <= T.p_hi) {
        nb = box_of(p, base);
        fetch(p, nb, stage0);
    }
    for (; p <= T.p_hi; ++p) {
        float *buf = lds + (p & 1) * L::kBuf;
        V0 *P0 = (V0 *)buf;
        const Box cb = nb;
        // the slots inside the box rows, as a wave-uniform bit mask
        const uint32_t rows = (1u << ((cb.kw - w + 3) >> 2)) - 1u;
        if (lane < QS) {
#pragma unroll
            for (int s = 0; s < kSlots; ++s)
                if (rows & (1u << s))
                    P0[(w + 4 * s) * QS + lane] = stage0[s];
        }
        __syncthreads();
        if (p < T.p_hi) {
            if (p + 1 - base == kBoxChunk) {
                base += kBoxChunk;
                fill_boxes(base);
                __syncthreads();
            }
            nb = box_of(p + 1, base);
            fetch(p + 1, nb, stage0);
        }
        const float fp = (float)p;
        const float q = fmaf(fp, c.ps, c.pb);
        const float qf = floorf(q);
        const float wq = q - qf;
        // byte address this column would have in z row 0 (as in the
        // single-channel sweep)
        const int colz = (int)(lds_addr(buf) + (uint32_t)sizeof(V0) * (uint32_t)((int)qf - cb.qlo)) -
                         cb.klo * (int)(sizeof(V0) * QS);
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
            if (r < R) {
                // as in the single-channel sweep: the exact fraction of the
                // ray's z index and its row address from one floor conversion
                const float k = fmaf(fp, ks[r], kb[r]);
                const float wk = __builtin_amdgcn_fractf(k);
                // (a generic pointer made from the LDS address: the
                // compiler still reads it from LDS)
                const V0 *row = (const V0 *)(lds_ptr(
                    (uint32_t)mad_i24(floor_i32(k), (int)(sizeof(V0) * QS), colz)));
                const V0 a00 = row[0], a10 = row[1];
                const V0 a01 = row[QS], a11 = row[QS + 1];
#pragma unroll
                for (int ch = 0; ch < C; ++ch) {
                    const float v00 = comp(a00, ch), v10 = comp(a10, ch);
                    const float v01 = comp(a01, ch), v11 = comp(a11, ch);
                    const float lo = fmaf(wq, v10 - v00, v00);
                    const float hi = fmaf(wq, v11 - v01, v01);
                    acc[ch][r] += fmaf(wk, hi - lo, lo);
                }
            }
        }
    }

    if (uc < T.nu_t) {
        // length factors first, the row records loaded together (as in the
        // single-channel sweep)
        // (the row index passes through an empty asm here, so that the
        // loads are not hoisted above the sweep, where they would hold
        // eight registers throughout)
        int rb = row0;
        asm volatile("" : "+v"(rb));
        float ds[kMaxR];
#pragma unroll
        for (int r = 0; r < kMaxR; ++r)
            ds[r] = g.rows[T.v0 + min(rb + r, T.nv_t - 1)].y;
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
            ds[r] = ray_ds(c.dsf, c.n2, ds[r]);
            asm volatile("" : "+v"(ds[r]));
        }
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
            const int vr = row0 + r;
            if (r < R && vr < T.nv_t) {
                const size_t at = ((size_t)T.a * g.nv + T.v0 + vr) * g.nu + T.u0 + uc;
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    M.sino[ch][at] = acc[ch][r] * ds[r];
            }
        }
    }
}

// One launch over the (group, tile) items of up to kMaxGroups groups, one
// item per workgroup in XCD-contiguous order (as the single-channel batch).
// Up to four waves per SIMD (at most 128 VGPRs) for four channels or the
// 65 x 32 boxes, five for two channels in 41 x 20 boxes (as the
// single-channel sweep).
template <int C, int QS, int ROWS, int RC>
__global__ void __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(1, C == 2 && QS == 41 ? 5 : 4)))
forward_mc(McArgs B)
{
    extern __shared__ float lds[];
    const int per = gridDim.x >> 3;
    const int item = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (item >= B.n_items)
        return;
    int gi = 0;
    while (gi + 1 < B.n_groups && item >= B.first[gi + 1])
        ++gi;
    const McGroup &M = B.grp[gi];
    const TileRec T = M.tiles[item - B.first[gi]];
    if (T.nu_t == 0)
        return;
    sweep_tile_mc<C, QS, ROWS, RC>(M, T, lds);
}

// Pack one group's C channel-first volumes into a volume of C-float vectors.
struct PackArgs {
    size_t n;
    const float *in[kMaxMcChannels];
    void *out;
};

template <int C>
__global__ void __launch_bounds__(kThreads) pack_channels(PackArgs P)
{
    using V = typename VecOf<C>::T;
    const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= P.n)
        return;
    V o;
    if constexpr (C == 4)
        o = make_float4(P.in[0][i], P.in[1][i], P.in[2][i], P.in[3][i]);
    else
        o = make_float2(P.in[0][i], P.in[1][i]);
    ((V *)P.out)[i] = o;
}

template <int C, int QS, int ROWS>
hipError_t launch_mc(const McArgs &B, hipStream_t s)
{
    using L = McLayout<C, QS, ROWS>;
    const int grid = (B.n_items + 7) / 8 * 8;
    bool all8 = true;   // every group's plan takes 8 rays per thread
    for (int i = 0; i < B.n_groups; ++i)
        all8 = all8 && B.grp[i].R == kMaxR;
    if (all8)
        hipLaunchKernelGGL((forward_mc<C, QS, ROWS, kMaxR>), dim3(grid), dim3(kThreads), L::kLds, s, B);
    else
        hipLaunchKernelGGL((forward_mc<C, QS, ROWS, 0>), dim3(grid), dim3(kThreads), L::kLds, s, B);
    return hipGetLastError();
}

template <int C>
hipError_t launch_mc_layout(const McArgs &B, bool small, hipStream_t s)
{
    if constexpr (C == 2)
        return small ? launch_mc<2, 41, 20>(B, s) : launch_mc<2, 65, 32>(B, s);
    else
        return launch_mc<4, 41, 20>(B, s);
}

// The plan's box extents bound the kernel's FP32 boxes up to one voxel of
// rounding per axis; the 41 x 20 layout keeps that voxel in reserve (boxes
// of at most 39 x 19 voxels in the plan; a host test checks the FP32 boxes).
bool small_layout(const FwdPlan &p) { return p.BQ <= 39 && p.BK <= 19; }

// Fill the groups' tile records and output pointers (B.grp[i].vg is set)
// and launch the sweep over all groups' tiles.
hipError_t launch_mc_groups(McArgs &B, const cbct_geom *const *gs, float *const *sinos, int C,
                            int n, hipStream_t s)
{
    bool small = true;
    int items = 0;
    for (int i = 0; i < n; ++i) {
        const cbct_geom *g = gs[i];
        small = small && small_layout(g->fwd);
        B.first[i] = items;
        McGroup &M = B.grp[i];
        M.g = g->dev;
        M.tiles = g->fwd.tiles;
        M.R = g->fwd.R;
        M.tub = g->fwd.TU == 32 ? 5 : 6;
        M.n_tiles = g->fwd.n_tiles;
        for (int ch = 0; ch < C; ++ch)
            M.sino[ch] = sinos[(size_t)i * C + ch];
        items += g->fwd.n_tiles;
    }
    B.first[n] = items;
    B.n_items = items;
    return C == 4 ? launch_mc_layout<4>(B, small, s) : launch_mc_layout<2>(B, small, s);
}

}  // namespace

int forward_mc_max_channels(const cbct_geom *g)
{
    const FwdPlan &p = g->fwd;
    const uint64_t nvox64 = (uint64_t)g->desc.nx * g->desc.ny * (g->desc.nz + 64);
    if (!p.ok || p.BQ > 64 || p.BK > 32 || nvox64 * 16 >= (1ull << 32))
        return 0;
    return small_layout(p) ? 4 : 2;
}

// Packs every group's channels into the library's scratch buffer (held
// until the sweep is enqueued), then launches the sweep.
hipError_t launch_forward_mc(int n, const cbct_geom *const *gs, const float *const *vols,
                             float *const *sinos, int C, hipStream_t s)
{
    if (n < 1 || n > kMaxGroups || (C != 2 && C != 4))
        return hipErrorInvalidValue;
    size_t off[kMaxGroups + 1] = {0};
    for (int i = 0; i < n; ++i) {
        const cbct_geom *g = gs[i];
        if (forward_mc_max_channels(g) < C)
            return hipErrorInvalidValue;   // 65 x 32 boxes of 4 channels exceed 64 KB of LDS
        const size_t nvox = (size_t)g->desc.nx * g->desc.ny * g->desc.nz;
        off[i + 1] = off[i] + 2 * ((nvox * C * sizeof(float) + 255) / 256 * 256);   // + transposed
    }
    McArgs B{};
    B.n_groups = n;
    ScratchLease lease;
    hipError_t e = scratch_acquire(off[n], s, lease);
    if (e == hipSuccess) {
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            const cbct_geom *g = gs[i];
            PackArgs P{};
            P.n = (size_t)g->desc.nx * g->desc.ny * g->desc.nz;
            for (int ch = 0; ch < C; ++ch)
                P.in[ch] = vols[(size_t)i * C + ch];
            P.out = (char *)lease.ptr + off[i];
            void *outt = (char *)lease.ptr + (off[i] + off[i + 1]) / 2;
            const dim3 grid((unsigned)((P.n + kThreads - 1) / kThreads));
            const int nx = g->desc.nx, ny = g->desc.ny, nz = g->desc.nz;
            if (C == 4) {
                hipLaunchKernelGGL(pack_channels<4>, grid, dim3(kThreads), 0, s, P);
                launch_transpose_xy((const float4 *)P.out, (float4 *)outt, nx, ny, nz, s);
            } else {
                hipLaunchKernelGGL(pack_channels<2>, grid, dim3(kThreads), 0, s, P);
                launch_transpose_xy((const float2 *)P.out, (float2 *)outt, nx, ny, nz, s);
            }
            e = hipGetLastError();
            B.grp[i].vg = P.out;
            B.grp[i].vgt = outt;
        }
        if (e == hipSuccess)
            e = launch_mc_groups(B, gs, sinos, C, n, s);
    }
    const hipError_t r = scratch_release(s, lease);
    return e != hipSuccess ? e : r;
}

}  // namespace cbct
