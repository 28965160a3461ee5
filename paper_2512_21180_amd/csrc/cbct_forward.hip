// Forward projector A for gfx950: plane sweep over LDS-staged boxes.
//
// Operator: the plane-sampled cone-beam line integral (arXiv 2512.21180,
// Sec. 2.2, projection operator P).  A workgroup owns one tile of up to 64
// columns x 4R rows of one angle, all sampled along the same axis; wave w
// holds rows [w R, w R + R) and lane l column u0 + l, so each thread carries
// R rays of one column and shares their in-plane interpolation index.  Where
// 64 columns of rays spread over more than 64 voxels (pixels coarser than
// voxels), tiles are 32 columns x 8R rows: lane l then holds column l % 32
// and the rows of row group 2w + l / 32.
//
// The tile sweeps the voxel-centre planes of its axis.  On plane p every ray
// of the tile lands inside a box of at most 64 (in-plane) x 32 (z) voxels
// spanned by the corner rays (the boxes of all planes are tabulated in LDS
// at the tile's start); the box is staged in LDS (zero outside the volume)
// one plane ahead of its use, double-buffered, one barrier per plane.
// Each sample is the bilinear interpolant read from LDS; each ray keeps its
// own running sum in a register, so the summation order is the plane order
// whatever the launch shape, and the result is written once, coalesced along
// the detector row.  Tiles are assigned XCD-contiguously so that the
// workgroups sharing an L2 work on neighbouring tiles of the same angle.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cbct_internal.h"
#include "cbct_lds.h"
#include "cbct_transpose.h"
#include "cbct_storage.h"

namespace cbct {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxR = 8;       // rays per thread

constexpr int kQS = 65;        // LDS row stride (floats): box rows are <= 64 wide
constexpr int kMaxRows = 32;   // box rows (z) per plane
constexpr int kSlots = kMaxRows / 4;
constexpr int kBoxChunk = 256; // planes whose boxes are tabulated at a time
static_assert(kBoxChunk == kThreads, "the box table is filled one plane per thread");
// LDS: two staging boxes, then the box table (one int4 per plane of a chunk)
constexpr size_t kFwdLds = 2 * (size_t)kMaxRows * kQS * sizeof(float) + kBoxChunk * 16;

// Sweep one tile.  R (rays per thread, 1..8) is uniform per tile; the per
// ray arithmetic does not depend on it, so any launch shape gives the same
// bits.  `lds` holds two boxes of kMaxRows x kQS floats and the box table.
//
// On plane p the box spans in-plane indices [qlo, qlo + qw) and z indices
// [klo, klo + kw), from the corner rays' crossings widened by one voxel for
// rounding; wave w stages rows w, w + 4, ... with lane l holding column l,
// so each row is one load per lane.
// tub: log2 of the tile width (6 or 5).  RC > 0 fixes R at compile time (the
// plans' usual 8 rays per thread): the per-ray tests then vanish, which
// matters because the sweep issues nearly as many scalar as vector
// instructions and a SIMD takes one of each per four cycles.
// vt: the volume with x and y swapped ([nz][nx][ny]) or null.  Tiles that
// sweep x planes read their boxes from it, so a box row (fixed z, in-plane
// index y) is contiguous; in the volume itself its voxels lie nx apart, a
// cache line each (the clinical forward: 12.2 ms reading them strided,
// 8.8 ms from the transposed copy).
template <class VS, class SS, int RC = 0>
__device__ __forceinline__ void sweep_tile(const DevGeom &g, const TileRec &T, int R_rt, int tub,
                           const typename VS::T *__restrict__ v,
                           const typename VS::T *__restrict__ vt,
                           typename SS::T *__restrict__ sino, float *lds)
{
    const int R = RC > 0 ? RC : R_rt;
    const int tid = threadIdx.x;
    // the wave index is uniform: the staging's slot ranges below are
    // scalar, so their tests are scalar branches
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int uc = lane & ((1 << tub) - 1);                   // tile column
    const int row0 = ((w << (6 - tub)) + (lane >> tub)) * R;  // first tile row
    const int ul = min(uc, T.nu_t - 1);
    const ColRec c = g.cols[(size_t)T.a * g.nu + T.u0 + ul];

    float kb[kMaxR], ks[kMaxR], acc[kMaxR];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
        const int vr = T.v0 + min(row0 + min(r, R - 1), T.nv_t - 1);
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

    const bool xp = T.cls == 0;
    const int nq = xp ? g.ny : g.nx;
    const bool tr = xp && vt != nullptr;   // x planes from the transposed copy
    const typename VS::T *src = tr ? vt : v;
    const int sp = xp ? (tr ? g.ny : 1) : g.nx;   // plane stride
    const int sq = xp && !tr ? g.nx : 1;         // in-plane stride
    const int sk = g.nx * g.ny;        // z stride (volumes have < 2^31 voxels)

    struct Box {
        int qlo, klo, qw, kw;
    };
    // The box of every plane is computed once per tile, one plane per
    // thread, into an LDS table of kBoxChunk planes (refilled when the sweep
    // passes a chunk); the sweep reads it back as wave-uniform values.
    int4 *boxes = (int4 *)(lds + 2 * kMaxRows * kQS);
    auto fill_boxes = [&](int base) {
        const int p = base + tid;
        if (p <= T.p_hi) {
            const float fp = (float)p;
            const float qa = fmaf(fp, cA.ps, cA.pb), qb = fmaf(fp, cB.ps, cB.pb);
            const float k0 = fmaf(fp, ksA0, kbA0), k1 = fmaf(fp, ksA1, kbA1);
            const float k2 = fmaf(fp, ksB0, kbB0), k3 = fmaf(fp, ksB1, kbB1);
            const int qlo = (int)floorf(fminf(qa, qb)) - 1;
            const int klo = (int)floorf(fminf(fminf(k0, k1), fminf(k2, k3))) - 1;
            const int qw = min((int)floorf(fmaxf(qa, qb)) + 3 - qlo, 64);
            const int kw = min((int)floorf(fmaxf(fmaxf(k0, k1), fmaxf(k2, k3))) + 3 - klo, kMaxRows);
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
    // stored values stay raw until the LDS store, so the loads of the next
    // plane stay in flight while this plane is summed
    using Raw = typename VS::Raw;
    // Slot s of wave w holds box row w + 4 s, z index k0 + 4 s with
    // k0 = klo + w; the wave loads the slots inside the box rows (a uniform
    // count).  FP32 loads go through a buffer resource over the volume,
    // whose range check returns zero for everything outside it: slots below
    // z index 0 (their 32-bit offsets wrap past the end; the plan keeps the
    // volume with 64 more planes under 4 GiB), slots past the top, and lanes
    // outside the volume in plane (their first offset is set to the end).
    const uint32_t vbytes = (uint32_t)sk * (uint32_t)g.nz * (uint32_t)sizeof(typename VS::T);
    const __amdgpu_buffer_rsrc_t vres =
        __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, (int)vbytes, kBufferWord3);
    const uint32_t step = 4u * (uint32_t)sk * (uint32_t)sizeof(typename VS::T);
    auto fetch = [&](int p, const Box &b, Raw (&st)[kSlots]) {
        const int q = b.qlo + lane;
        const bool qin = lane < b.qw && (unsigned)q < (unsigned)nq;
        if constexpr (sizeof(typename VS::T) == 4) {
            const int n_sl = (b.kw - w + 3) >> 2;
            // modular: exact for slots inside the volume
            const uint32_t off0 =
                qin ? (__umul24((uint32_t)q, (uint32_t)sq) + (uint32_t)p * (uint32_t)sp +
                       (uint32_t)(b.klo + w) * (uint32_t)sk) *
                          (uint32_t)sizeof(typename VS::T)
                    : vbytes;
#pragma unroll
            for (int s = 0; s < kSlots; ++s)
                if (s < n_sl)
                    st[s] = VS::buf_at(vres, off0 + (uint32_t)s * step);
        } else {
            // 16-bit volumes: masked global loads (slots inside the box rows
            // and the volume as a wave-uniform bit mask, the lane test one
            // exec region): 16-bit buffer loads staged them more slowly
            const int k0 = b.klo + w;
            const int s_lo = k0 >= 0 ? 0 : (3 - k0) >> 2;
            const int s_hi = min((b.kw - w + 3) >> 2, (g.nz - k0 + 3) >> 2);
            const uint32_t live =
                s_hi > s_lo ? ((1u << s_hi) - 1u) & ~((1u << s_lo) - 1u) : 0u;
            const uint32_t off0 =
                (uint32_t)(q * sq + p * sp + k0 * sk) * (uint32_t)sizeof(typename VS::T);
#pragma unroll
            for (int s = 0; s < kSlots; ++s)
                st[s] = Raw(0);
            if (qin) {
#pragma unroll
                for (int s = 0; s < kSlots; ++s)
                    if (live & (1u << s))
                        st[s] = VS::raw_at(src, off0 + (uint32_t)s * step);
            }
        }
    };

    __syncthreads();   // the previous work item's readers of lds are done
    int p = T.p_lo, base = T.p_lo;
    fill_boxes(base);
    __syncthreads();
    Box nb{0, 0, 0, 0};
    Raw stage[kSlots];
    if (p <= T.p_hi) {
        nb = box_of(p, base);
        fetch(p, nb, stage);
    }
    for (; p <= T.p_hi; ++p) {
        float *buf = lds + (p & 1) * (kMaxRows * kQS);
        const Box cb = nb;
        // the slots inside the box rows, as a wave-uniform bit mask
        const uint32_t rows = (1u << ((cb.kw - w + 3) >> 2)) - 1u;
#pragma unroll
        for (int s = 0; s < kSlots; ++s)
            if (rows & (1u << s))
                buf[(w + 4 * s) * kQS + lane] = VS::wide(stage[s]);
        __syncthreads();
        if (p < T.p_hi) {
            if (p + 1 - base == kBoxChunk) {   // uniform: next chunk of boxes
                base += kBoxChunk;
                fill_boxes(base);   // every reader of the old chunk is past the barrier
                __syncthreads();
            }
            nb = box_of(p + 1, base);
            fetch(p + 1, nb, stage);
        }
        const float fp = (float)p;
        const float q = fmaf(fp, c.ps, c.pb);
        const float qf = floorf(q);
        const float wq = q - qf;
        // byte address this column would have in z row 0 (the box's first
        // row, klo, lies at its position in box row 0)
        const int colz =
            (int)(lds_addr(buf) + 4u * (uint32_t)((int)qf - cb.qlo)) - cb.klo * (4 * kQS);
        // all rays' reads first, then their arithmetic: the reads of the
        // rays overlap instead of each ray waiting for its own
        float wk[kMaxR], v00[kMaxR], v10[kMaxR], v01[kMaxR], v11[kMaxR];
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
            if (r < R) {
                // z index k of the ray on this plane: its weight is the
                // exact fraction of k, its row address one floor conversion
                // and one multiply-add (every ray's floor(k) lies in the box
                // rows [klo, klo + kw - 1), so the address is inside the box)
                const float k = fmaf(fp, ks[r], kb[r]);
                wk[r] = __builtin_amdgcn_fractf(k);
                const lds_float *row = lds_ptr((uint32_t)mad_i24(floor_i32(k), 4 * kQS, colz));
                v00[r] = row[0];
                v10[r] = row[1];
                v01[r] = row[kQS];
                v11[r] = row[kQS + 1];
            }
        }
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
            if (r < R) {
                const float lo = fmaf(wq, v10[r] - v00[r], v00[r]);
                const float hi = fmaf(wq, v11[r] - v01[r], v01[r]);
                acc[r] += fmaf(wk[r], hi - lo, lo);
            }
        }
    }

    if (uc < T.nu_t) {
        // every ray's length factor first, its row record loaded with the
        // others' (the empty asm keeps the compiler from moving each load
        // behind its ray's store test, where the loads would wait one by one)
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
            if (r < R && vr < T.nv_t)
                SS::st(sino, ((size_t)T.a * g.nv + T.v0 + vr) * g.nu + T.u0 + uc, acc[r] * ds[r]);
        }
    }
}

struct SweepArgs {
    DevGeom g;
    const TileRec *tiles;
    int R, tub;   // rays per thread, log2 of the tile width
};

// At most five waves per SIMD: with more resident tiles the planes' boxes of
// different tiles compete for the caches (clinical case, earlier build:
// 15.3 ms at six waves, 13.5 ms at five, 14.5 ms at four).  At the current
// register count the occupancy is four; five would need 96 VGPRs, which
// spills.
template <class VS, class SS, int RC>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 5)))
forward_sweep(SweepArgs A, const typename VS::T *__restrict__ vol,
              const typename VS::T *__restrict__ volt, typename SS::T *__restrict__ sino)
{
    extern __shared__ float lds[];
    // XCD-contiguous tile order: workgroups are dealt to the 8 XCDs round
    // robin, so XCD x receives ids x, x+8, ...; give it tiles
    // [x * n/8, (x+1) * n/8).
    const int nb = gridDim.x;
    const int t = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    const TileRec T = A.tiles[t];
    if (T.nu_t == 0)
        return;
    const int ch = blockIdx.y;
    const size_t nvox = (size_t)A.g.nx * A.g.ny * A.g.nz;
    const size_t nsino = (size_t)A.g.n_angles * A.g.nv * A.g.nu;
    sweep_tile<VS, SS, RC>(A.g, T, A.R, A.tub, vol + ch * nvox, volt + ch * nvox,
                           sino + ch * nsino, lds);
}

// ---- batched forward: one launch over all (case, tile) items ----------------

struct FwdCase {
    DevGeom g;
    const TileRec *tiles;
    int R, tub, n_tiles;
    const void *vol, *volt;   // the volume, and with x and y swapped
    void *sino;
};

struct BatchFwdArgs {
    int n_cases, n_items;
    int first[kMaxBatch + 1];   // first item of each case
    FwdCase c[kMaxBatch];
};

template <class VS, class SS>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 5)))
forward_batch(BatchFwdArgs B)
{
    extern __shared__ float lds[];
    // one item per workgroup, XCD-contiguous as in forward_sweep; the
    // hardware dispatcher balances the uneven items
    const int per = gridDim.x >> 3;
    const int item = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (item >= B.n_items)
        return;
    int cs = 0;
    while (cs + 1 < B.n_cases && item >= B.first[cs + 1])
        ++cs;
    const FwdCase &C = B.c[cs];
    const TileRec T = C.tiles[item - B.first[cs]];
    if (T.nu_t == 0)
        return;
    // cases with the usual rays per thread take the sweep specialised for it
    // (a uniform branch; the bits do not depend on the variant)
    if (C.R == kMaxR)
        sweep_tile<VS, SS, kMaxR>(C.g, T, C.R, C.tub, (const typename VS::T *)C.vol,
                                  (const typename VS::T *)C.volt, (typename SS::T *)C.sino, lds);
    else
        sweep_tile<VS, SS>(C.g, T, C.R, C.tub, (const typename VS::T *)C.vol,
                           (const typename VS::T *)C.volt, (typename SS::T *)C.sino, lds);
}

}  // namespace

hipError_t launch_forward_tiled(const DevGeom &g, const FwdPlan &p, const void *vol,
                                cbct_dtype vt, void *sino, cbct_dtype st, int channels,
                                hipStream_t s)
{
    SweepArgs A{g, p.tiles, p.R, p.TU == 32 ? 5 : 6};
    const size_t lds = kFwdLds;
    dim3 grid(p.n_tiles, channels), block(kThreads);
    // the volume with x and y swapped, in the library's device buffer, for
    // the tiles that sweep x planes
    const size_t nvox = (size_t)g.nx * g.ny * g.nz;
    ScratchLease lease;
    hipError_t e = scratch_acquire(nvox * channels * storage_bytes(vt), s, lease);
    if (e == hipSuccess)
        e = dispatch_storage(vt, st, [&](auto vs, auto ss) -> hipError_t {
            using VS = decltype(vs);
            using SS = decltype(ss);
            using T = typename VS::T;
            const T *x = (const T *)vol;
            T *xt = (T *)lease.ptr;
            launch_transpose_xy(x, xt, g.nx, g.ny, g.nz * channels, s);
            if (p.R == kMaxR)
                hipLaunchKernelGGL((forward_sweep<VS, SS, kMaxR>), grid, block, lds, s, A, x, xt,
                                   (typename SS::T *)sino);
            else
                hipLaunchKernelGGL((forward_sweep<VS, SS, 0>), grid, block, lds, s, A, x, xt,
                                   (typename SS::T *)sino);
            return hipGetLastError();
        });
    const hipError_t r = scratch_release(s, lease);
    return e != hipSuccess ? e : r;
}

hipError_t launch_forward_batch(int n, const cbct_geom *const *gs, const void *const *vols,
                                void *const *sinos, cbct_dtype vt, cbct_dtype st, hipStream_t s)
{
    BatchFwdArgs B{};
    B.n_cases = n;
    int items = 0;
    size_t off[kMaxBatch], total = 0;   // the cases' transposed volumes in the library's buffer
    for (int i = 0; i < n; ++i) {
        const cbct_geom *g = gs[i];
        B.first[i] = items;
        B.c[i] = FwdCase{g->dev, g->fwd.tiles, g->fwd.R, g->fwd.TU == 32 ? 5 : 6,
                         g->fwd.n_tiles, vols[i], nullptr, sinos[i]};
        items += g->fwd.n_tiles;
        off[i] = total;
        total += ((size_t)g->dev.nx * g->dev.ny * g->dev.nz * storage_bytes(vt) + 255) & ~(size_t)255;
    }
    B.first[n] = items;
    B.n_items = items;
    const int grid = (items + 7) / 8 * 8;
    ScratchLease lease;
    hipError_t e = scratch_acquire(total, s, lease);
    if (e == hipSuccess)
        e = dispatch_storage(vt, st, [&](auto vs, auto ss) -> hipError_t {
            using VS = decltype(vs);
            using SS = decltype(ss);
            using T = typename VS::T;
            for (int i = 0; i < n; ++i) {
                T *xt = (T *)((char *)lease.ptr + off[i]);
                launch_transpose_xy((const T *)vols[i], xt, gs[i]->dev.nx, gs[i]->dev.ny,
                                    gs[i]->dev.nz, s);
                B.c[i].volt = xt;
            }
            hipLaunchKernelGGL((forward_batch<VS, SS>), dim3(grid), dim3(kThreads), kFwdLds, s, B);
            return hipGetLastError();
        });
    const hipError_t r = scratch_release(s, lease);
    return e != hipSuccess ? e : r;
}

}  // namespace cbct
