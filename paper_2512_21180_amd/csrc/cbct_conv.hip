// 3x3x3 convolutions of the learned primal-dual blocks on the gfx950 matrix
// cores (see cbct_nn.h).  arXiv 2512.21180, Alg. 1: the dual and primal
// blocks are 3x3x3 convolution stacks with LeakyReLU, added to half of a
// latent.
//
// Forward / data gradient (conv3): implicit GEMM per wavefront: M = 16
// consecutive x positions of one (z, y) row, N = 16 output channels,
// K = 27 taps x 16 input channels, two taps per v_mfma_f32_16x16x32_bf16
// (14 MFMAs per tile).  Lane l supplies, for MFMA p, 8 input channels
// (8 (l/16) % 16 ..) of tap 2p + l/32 at position x0 + l%16: one 16-byte
// LDS read of the staged channel-last activations.  The weights stay in
// registers while a workgroup walks a column of z planes with a rolling
// halo.  The result tile (lane l holds rows 4 (l/16) .. +3 of column l%16)
// goes through the epilogue: bias, LeakyReLU derivative mask, LeakyReLU,
// then bf16 channel-last and/or FP32 channel-first stores.
//
// Weight gradient (conv3_wgrad): per wavefront, per 32-position chunk of a
// row, 27 v_mfma_f32_16x16x32_bf16 with M = 16 output channels, N = 16
// input channels, K = 32 positions, from rows staged transposed in the
// wave's LDS; each wave keeps its 27 tiles in registers and writes them to
// a workspace; one ordered reduction follows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "cbct_internal.h"
#include "cbct_nn.h"

namespace cbct {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr int kMaxCF = 16;

__device__ inline uint16_t f2bf(float v)
{
    uint32_t b = __float_as_uint(v);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu))
        return (uint16_t)((b >> 16) | 0x0040u);
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

__device__ inline float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

struct PtrList {
    float *p[kMaxCF];
};

struct CPtrList {
    const float *p[kMaxCF];
    float scale[kMaxCF];
};

// ---- pack: channel-first FP32 -> channel-last bf16 x 16 -------------------

__global__ void __launch_bounds__(kT) k_pack16(size_t S, int n_in, CPtrList in, uint16_t *out)
{
    const size_t s = (size_t)blockIdx.x * kT + threadIdx.x;
    if (s >= S)
        return;
    uint32_t w[8];
#pragma unroll
    for (int c = 0; c < 16; c += 2) {
        const float a = c < n_in ? in.scale[c] * in.p[c][s] : 0.0f;
        const float b = c + 1 < n_in ? in.scale[c + 1] * in.p[c + 1][s] : 0.0f;
        w[c / 2] = (uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16);
    }
    uint4 *o = reinterpret_cast<uint4 *>(out + s * 16);
    o[0] = make_uint4(w[0], w[1], w[2], w[3]);
    o[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

// ---- conv3 -------------------------------------------------------------------

struct ConvArgs {
    int nz, ny, nx;               // grid
    int zb;                       // z planes per workgroup
    const uint16_t *x, *w;
    const float *bias;
    const uint16_t *mask;
    int transpose_w, act;
    float slope;
    uint16_t *y_cl;
    int n_cf, accumulate;
    float alpha;
    PtrList y_cf;
};

// A workgroup computes an output column of kRows rows x 64 positions along
// x over zb consecutive z planes (zb from the host: long columns where the
// grid gives enough workgroups, short ones on small grids).  Wave w takes row
// y0 + w and its four 16-position tiles on every plane.  The input halo
// (kRows + 2 rows x 66 positions x 16 channels per plane) rolls through a
// ring of four planes in LDS: while plane z is computed from the planes
// z - 1, z, z + 1, the loads of plane z + 2 are in flight and land in the
// slot plane z - 2 held; one barrier per plane.  Each MFMA's A operand is
// one 16-byte LDS read per lane (channels 0-7 and 8-15 in separate halves,
// so the 16 lanes of a group read consecutive words).  The weights are read
// once per workgroup straight into registers (the transposed kernel of the
// data gradient gathered from the untransposed array).
constexpr int kRows = 4, kBX = 64;
constexpr int kHX = kBX + 2, kHY = kRows + 2, kHPlane = kHY * kHX;   // halo positions per plane
constexpr int kRing = 4;
constexpr int kStageIt = (2 * kHPlane + kT - 1) / kT;   // 16-byte loads per thread and plane

// Three workgroups per CU (the ring takes 50.7 KB of LDS): at most 168 VGPRs.
// MASK: the data gradient's variant, which also holds the LeakyReLU-
// derivative mask of the plane (its registers come from not holding the
// taps' LDS indices).
template <bool MASK>
__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_conv3(ConvArgs A)
{
    __shared__ uint4 halo[kRing][2][kHPlane];   // [slot][channel half][position]

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nbx = (A.nx + kBX - 1) / kBX, nby = (A.ny + kRows - 1) / kRows;
    const int bx = blockIdx.x % nbx;
    const int by = (blockIdx.x / nbx) % nby;
    const int bz = blockIdx.x / (nbx * nby);
    const int x0 = bx * kBX, y0 = by * kRows;
    const int z0 = bz * A.zb, z1 = min(z0 + A.zb, A.nz);
    const size_t plane = (size_t)A.ny * A.nx * 16;   // bf16 elements per input plane

    // this thread's staging items: element e = tid + kT j of a plane's halo
    // (position e / 2, channel half e % 2), offset within the plane
    int soff[kStageIt];
    bool sval[kStageIt];
#pragma unroll
    for (int j = 0; j < kStageIt; ++j) {
        const int e = tid + kT * j;
        const int hp = e >> 1, h = e & 1;
        const int hx = hp % kHX, hy = hp / kHX;
        const int xx = x0 - 1 + hx, yy = y0 - 1 + hy;
        sval[j] = e < 2 * kHPlane && (unsigned)xx < (unsigned)A.nx && (unsigned)yy < (unsigned)A.ny;
        soff[j] = (yy * A.nx + xx) * 16 + 8 * h;
    }
    auto load_plane = [&](int zz, uint4 (&r)[kStageIt]) {
        const bool zin = (unsigned)zz < (unsigned)A.nz;
#pragma unroll
        for (int j = 0; j < kStageIt; ++j) {
            r[j] = make_uint4(0u, 0u, 0u, 0u);
            if (zin && sval[j])
                r[j] = *reinterpret_cast<const uint4 *>(A.x + (size_t)zz * plane + soff[j]);
        }
    };
    auto store_plane = [&](int zz, const uint4 (&r)[kStageIt]) {
        uint4 *dst = &halo[(zz + kRing) & (kRing - 1)][0][0];
#pragma unroll
        for (int j = 0; j < kStageIt; ++j) {
            const int e = tid + kT * j;
            if (e < 2 * kHPlane)
                dst[(e & 1) * kHPlane + (e >> 1)] = r[j];
        }
    };

    const int m = lane & 15;          // position within the tile (A rows) / output channel (B cols)
    const int kb = lane >> 4;         // k block: tap 2p + (kb >> 1), channels 8 (kb & 1) ..
    const int hh = kb & 1;

    // weights: staged once in LDS (27 x 16 x 16 bf16, coalesced), then
    // B[k][n] for n = m (output channel), 8 input channels of half hh, into
    // registers (the data gradient's transposed kernel gathered from LDS)
    {
        uint4 *wl = &halo[0][0][0];
        const uint4 *wg = reinterpret_cast<const uint4 *>(A.w);
        constexpr int kW4 = 27 * 16 * 16 / 8;   // 16-byte words: 3 full rounds + 96
        static_assert(kW4 > 3 * kT && kW4 <= 4 * kT, "four rounds of loads");
        const bool last = tid < kW4 - 3 * kT;
        const uint4 w0 = wg[tid], w1 = wg[tid + kT], w2 = wg[tid + 2 * kT];
        const uint4 w3 = last ? wg[tid + 3 * kT] : make_uint4(0u, 0u, 0u, 0u);
        wl[tid] = w0;
        wl[tid + kT] = w1;
        wl[tid + 2 * kT] = w2;
        if (last)
            wl[tid + 3 * kT] = w3;
    }
    __syncthreads();
    bf16x8 wr[14];
    {
        const uint16_t *wl = reinterpret_cast<const uint16_t *>(&halo[0][0][0]);
#pragma unroll
        for (int p = 0; p < 14; ++p) {
            const int t = 2 * p + (kb >> 1);
            bf16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (t < 27) {
                if (!A.transpose_w) {
                    v = *reinterpret_cast<const bf16x8 *>(wl + (t * 16 + m) * 16 + 8 * hh);
                } else {
                    // w'[t][co][ci] = w[26 - t][ci][co]
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        v[j] = (short)wl[((26 - t) * 16 + 8 * hh + j) * 16 + m];
                }
            }
            wr[p] = v;
        }
    }
    __syncthreads();   // weights read before the halo overwrites them
    const int co = m;
    const float b = A.bias ? A.bias[co] : 0.0f;
    const int y = y0 + w;
    const bool row_live = y < A.ny;   // uniform per wave
    const int ntx = min(kBX / 16, (A.nx - x0 + 15) / 16);   // live tiles (uniform)

    uint4 pre[kStageIt];
    load_plane(z0 - 1, pre);
    store_plane(z0 - 1, pre);
    load_plane(z0, pre);
    store_plane(z0, pre);
    load_plane(z0 + 1, pre);
    store_plane(z0 + 1, pre);
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 1 < z1;   // uniform: the next plane needs z + 2
        // the epilogue's mask values, loaded ahead of the halo prefetch so
        // that waiting for them does not wait for it
        uint16_t mk[kBX / 16][4];
        if (MASK && row_live) {
#pragma unroll
            for (int tx = 0; tx < kBX / 16; ++tx)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int xo = x0 + 16 * tx + 4 * kb + i;
                    mk[tx][i] = xo < A.nx
                        ? A.mask[(((size_t)z * A.ny + y) * A.nx + xo) * 16 + co] : (uint16_t)0;
                }
        }
        if (more)
            load_plane(z + 2, pre);      // in flight during this plane's MFMAs
        if (row_live) {
            // per-lane LDS index of each MFMA's tap at tile 0: ring slot of
            // its plane, channel half, row w + dy, position m + dx
            auto base = [&](int p) {
                const int t = min(2 * p + (kb >> 1), 26);
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;   // offsets + 1
                const int slot = (z - 1 + dz + kRing) & (kRing - 1);
                return (slot * 2 + hh) * kHPlane + (w + dy) * kHX + m + dx;
            };
            int bases[MASK ? 1 : 14];
            if (!MASK) {
#pragma unroll
                for (int p = 0; p < 14; ++p)
                    bases[p] = base(p);
            }
            // all tiles' MFMAs first (four independent chains), then the
            // epilogues, whose loads would otherwise wait for the prefetch
            f32x4 acc[kBX / 16];
#pragma unroll
            for (int tx = 0; tx < kBX / 16; ++tx)
                acc[tx] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int p = 0; p < 14; ++p) {
                const int t = 2 * p + (kb >> 1);
#pragma unroll
                for (int tx = 0; tx < kBX / 16; ++tx) {
                    if (tx < ntx) {
                        bf16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
                        if (t < 27)
                            a = __builtin_bit_cast(
                                bf16x8, (&halo[0][0][0])[(MASK ? base(p) : bases[MASK ? 0 : p]) + 16 * tx]);
                        acc[tx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wr[p], acc[tx], 0, 0, 0);
                    }
                }
            }
            // epilogue: lane holds rows 4 kb + i (positions), column m (output channel)
#pragma unroll
            for (int tx = 0; tx < kBX / 16; ++tx) {
                if (tx >= ntx)
                    break;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int xo = x0 + 16 * tx + 4 * kb + i;
                    if (xo >= A.nx)
                        continue;
                    const size_t pos = ((size_t)z * A.ny + y) * A.nx + xo;
                    float v = acc[tx][i] + b;
                    if (MASK) {
                        const uint16_t hm = mk[tx][i];
                        const bool positive = !(hm & 0x8000u) && (hm & 0x7fffu);
                        v = positive ? v : A.slope * v;
                    }
                    if (A.act)
                        v = v > 0.0f ? v : A.slope * v;
                    if (A.y_cl)
                        A.y_cl[pos * 16 + co] = f2bf(v);
                    if (co < A.n_cf) {
                        float *dst = A.y_cf.p[co] + pos;
                        *dst = A.accumulate ? fmaf(A.alpha, v, *dst) : v;
                    }
                }
            }
        }
        if (more)
            store_plane(z + 2, pre);     // into the slot plane z - 2 held
        __syncthreads();
    }
}

// ---- conv3 weight gradient ---------------------------------------------------
//
// dw[t][co][ci] = sum_s dy[s][co] x[s + offset(t)][ci] is a product with the
// positions as the reduction dimension, but the activations are stored
// channel-last, so a matrix-core operand (8 consecutive positions of one
// channel per lane) is a strided gather.  Each wave therefore stages the
// rows it needs transposed (channel-major, positions contiguous) in its own
// LDS region and reads operands as aligned 16-byte words.  With the
// substitution p = s + dx (the x position) the in-row shift moves onto dy:
// dw[t][co][ci] = sum_p dy[p - dx][co] x[p][ci] (dx in {-1, 0, 1}; both zero
// outside the grid), so the 9 x rows of a 32-position chunk are read at the
// chunk's own aligned positions and only the one dy row is read shifted
// (two staged copies, offset by one position, keep every read aligned).
// Per chunk: 27 v_mfma_f32_16x16x32_bf16 (M = 16 output channels, N = 16
// input channels, K = 32 positions), 9 + 4 LDS reads per lane.  Work split:
// chunk c goes to wave c mod kWgWaves, in order; each wave writes its 27
// tiles and its bias sums to the workspace; one ordered reduction follows.
constexpr int kWgBlocks = 512;                // fixed (two per CU): the reduction order is fixed
constexpr int kWgWaves = kWgBlocks * 4;
constexpr int kWgCells = 27 * 256 + 16;       // dw tiles + db
constexpr int kXS = 40;                       // staged channel row: 32 positions + pad (bf16)
constexpr int kDS = 40;                       // staged dy channel row: 34 positions + pad

struct WgradArgs {
    int nz, ny, nx, nxc;                      // grid, 32-position chunks per row
    const uint16_t *x, *dy;
    float *ws;
};

// Order this wave's LDS writes before its later reads (and reads before
// later writes): wait for outstanding LDS operations and stop the compiler
// from moving memory accesses across.  The staging area is private to the
// wave, so no workgroup barrier is involved.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Two channel-last positions (8 channels each, one half) to four 32-bit
// words per channel pair: word for channel 2k = (a.ch2k, b.ch2k), for
// channel 2k + 1 = (a.ch2k+1, b.ch2k+1), a the lower position.
__device__ inline uint32_t lo_pair(uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_perm(b, a, 0x05040100u);
}
__device__ inline uint32_t hi_pair(uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_perm(b, a, 0x07060302u);
}

// Staging items of a chunk per lane: x rows (r9, position pair, channel
// half), 9 x 16 x 2 = 288 over 64 lanes; the dy row (copy, pair, half),
// 2 x 17 x 2 = 68.
constexpr int kXIt = (9 * 16 * 2 + 63) / 64, kDIt = (2 * 17 * 2 + 63) / 64;

struct WgStage {
    uint4 xa[kXIt], xb[kXIt], da[kDIt], db[kDIt];
};

// Issue the loads of chunk c (rows zero outside the grid).
__device__ inline void wg_fetch(const WgradArgs &A, long c, int lane, WgStage &S)
{
    const int xc = (int)(c % A.nxc);
    const long row = c / A.nxc;
    const int y = (int)(row % A.ny), z = (int)(row / A.ny);
    const int x0 = xc * 32;
#pragma unroll
    for (int it = 0; it < kXIt; ++it) {
        const int e = lane + 64 * it;
        const int h = e & 1, pp = (e >> 1) & 15, r9 = e >> 5;
        const int zz = z + r9 / 3 - 1, yy = y + r9 % 3 - 1, xx = x0 + 2 * pp;
        S.xa[it] = S.xb[it] = make_uint4(0, 0, 0, 0);
        if (e < 9 * 16 * 2 && (unsigned)zz < (unsigned)A.nz && (unsigned)yy < (unsigned)A.ny) {
            const uint16_t *src = A.x + (((size_t)zz * A.ny + yy) * A.nx + xx) * 16 + 8 * h;
            if (xx < A.nx)
                S.xa[it] = *reinterpret_cast<const uint4 *>(src);
            if (xx + 1 < A.nx)
                S.xb[it] = *reinterpret_cast<const uint4 *>(src + 16);
        }
    }
#pragma unroll
    for (int it = 0; it < kDIt; ++it) {
        const int e = lane + 64 * it;
        const int h = e & 1, pp = (e >> 1) % 17, cp = (e >> 1) / 17;
        const int xx = x0 - 1 + cp + 2 * pp;
        S.da[it] = S.db[it] = make_uint4(0, 0, 0, 0);
        if (e < 2 * 17 * 2) {
            const size_t rowb = ((size_t)z * A.ny + y) * A.nx;
            if ((unsigned)xx < (unsigned)A.nx)
                S.da[it] = *reinterpret_cast<const uint4 *>(A.dy + (rowb + xx) * 16 + 8 * h);
            if ((unsigned)(xx + 1) < (unsigned)A.nx)
                S.db[it] = *reinterpret_cast<const uint4 *>(A.dy + (rowb + xx + 1) * 16 + 8 * h);
        }
    }
}

// Write a fetched chunk into the wave's LDS, transposed: channel rows of
// positions, two positions per 32-bit word.
__device__ inline void wg_store(const WgStage &S, int lane, uint16_t *xT, uint16_t *dT)
{
#pragma unroll
    for (int it = 0; it < kXIt; ++it) {
        const int e = lane + 64 * it;
        if (e < 9 * 16 * 2) {
            const int h = e & 1, pp = (e >> 1) & 15, r9 = e >> 5;
            uint32_t *d = reinterpret_cast<uint32_t *>(xT + (r9 * 16 + 8 * h) * kXS + 2 * pp);
            const uint32_t av[4] = {S.xa[it].x, S.xa[it].y, S.xa[it].z, S.xa[it].w};
            const uint32_t bv[4] = {S.xb[it].x, S.xb[it].y, S.xb[it].z, S.xb[it].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                d[(2 * k) * (kXS / 2)] = lo_pair(av[k], bv[k]);
                d[(2 * k + 1) * (kXS / 2)] = hi_pair(av[k], bv[k]);
            }
        }
    }
#pragma unroll
    for (int it = 0; it < kDIt; ++it) {
        const int e = lane + 64 * it;
        if (e < 2 * 17 * 2) {
            const int h = e & 1, pp = (e >> 1) % 17, cp = (e >> 1) / 17;
            uint32_t *d = reinterpret_cast<uint32_t *>(dT + (cp * 16 + 8 * h) * kDS + 2 * pp);
            const uint32_t av[4] = {S.da[it].x, S.da[it].y, S.da[it].z, S.da[it].w};
            const uint32_t bv[4] = {S.db[it].x, S.db[it].y, S.db[it].z, S.db[it].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                d[(2 * k) * (kDS / 2)] = lo_pair(av[k], bv[k]);
                d[(2 * k + 1) * (kDS / 2)] = hi_pair(av[k], bv[k]);
            }
        }
    }
}

__global__ void __launch_bounds__(kT) k_wgrad(WgradArgs A)
{
    // per wave: x rows [9][16 ch][kXS], dy rows [2 copies][16 ch][kDS] (bf16)
    __shared__ __attribute__((aligned(16))) uint32_t stage[4][(9 * 16 * kXS + 2 * 16 * kDS) / 2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = blockIdx.x * 4 + wv;          // global wave index, fixed work split
    const int m = lane & 15, kb = lane >> 4;     // M = output channel m, K block kb
    uint16_t *xT = reinterpret_cast<uint16_t *>(stage[wv]);
    uint16_t *dT = xT + 9 * 16 * kXS;
    const long n_chunks = (long)A.nz * A.ny * A.nxc;

    f32x4 acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t)
        acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float dbp = 0.0f;

    WgStage S;
    if (gw < n_chunks)
        wg_fetch(A, gw, lane, S);
    for (long c = gw; c < n_chunks; c += kWgWaves) {
        wg_store(S, lane, xT, dT);
        wave_sync();   // staged rows visible to every lane of this wave
        if (c + kWgWaves < n_chunks)
            wg_fetch(A, c + kWgWaves, lane, S);   // in flight during the MFMAs
        // A operands (dy^T, row co = m, positions x0 + 8 kb + j - (dx - 1)):
        // dx = 0 reads copy 0 at 8 kb + 2 (4-byte aligned), dx = 1 copy 1 at
        // 8 kb, dx = 2 copy 0 at 8 kb (16-byte aligned)
        bf16x8 ad[3];
        {
            const uint16_t *c0 = dT + m * kDS, *c1 = dT + (16 + m) * kDS;
            const uint32_t *w0 = reinterpret_cast<const uint32_t *>(c0 + 8 * kb + 2);
            ad[0] = __builtin_bit_cast(bf16x8, make_uint4(w0[0], w0[1], w0[2], w0[3]));
            ad[1] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(c1 + 8 * kb));
            ad[2] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(c0 + 8 * kb));
        }
        // bias gradient: the unshifted copy covers the chunk's positions once
#pragma unroll
        for (int j = 0; j < 8; ++j)
            dbp += bf2f((uint16_t)ad[1][j]);
#pragma unroll
        for (int r9 = 0; r9 < 9; ++r9) {
            // B operand: x row r9, input channel m, positions x0 + 8 kb ..
            const bf16x8 bx = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4 *>(xT + (r9 * 16 + m) * kXS + 8 * kb));
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
                acc[r9 * 3 + dx] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(ad[dx], bx, acc[r9 * 3 + dx], 0, 0, 0);
        }
        wave_sync();   // every lane done reading before the next chunk's writes
    }
    // acc[t]: lane holds rows (co) 4 kb + i, column (ci) m
    float *o = A.ws + (size_t)gw * kWgCells;
#pragma unroll
    for (int t = 0; t < 27; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            o[t * 256 + (4 * kb + i) * 16 + m] = acc[t][i];
    // db: lanes m, m+16, m+32, m+48 hold partial sums of channel m
    dbp += __shfl_xor(dbp, 16);
    dbp += __shfl_xor(dbp, 32);
    if (kb == 0)
        o[27 * 256 + m] = dbp;
}

// Ordered reduction of the waves' partial tiles in two fixed levels: group
// g of kWgGroups sums waves [g G, g G + G) in order into a row after the
// waves' rows, then each cell sums the group rows in order.
constexpr int kWgGroups = 32, kWgPerGroup = kWgWaves / kWgGroups;
static_assert(kWgWaves % kWgGroups == 0, "groups of equal size");

__global__ void __launch_bounds__(kT) k_wgrad_reduce1(float *ws)
{
    const int e = blockIdx.x * kT + threadIdx.x, g = blockIdx.y;
    if (e >= kWgCells)
        return;
    const float *src = ws + (size_t)g * kWgPerGroup * kWgCells + e;
    float s = 0.0f;
    for (int w = 0; w < kWgPerGroup; ++w)
        s += src[(size_t)w * kWgCells];
    ws[((size_t)kWgWaves + g) * kWgCells + e] = s;
}

__global__ void __launch_bounds__(kT) k_wgrad_reduce2(const float *ws, float *dw, float *db)
{
    const int e = blockIdx.x * kT + threadIdx.x;
    if (e >= kWgCells)
        return;
    float s = 0.0f;
    for (int g = 0; g < kWgGroups; ++g)
        s += ws[((size_t)kWgWaves + g) * kWgCells + e];
    if (e < 27 * 256)
        dw[e] = s;
    else if (db)
        db[e - 27 * 256] = s;
}

// ---- conv1: 1x1x1 convolution of channel-first FP32 channels ---------------

__global__ void __launch_bounds__(kT) k_conv1(size_t S, int n_in, CPtrList in, const float *w,
                                              float *out, int accumulate, float alpha)
{
    const size_t s = (size_t)blockIdx.x * kT + threadIdx.x;
    if (s >= S)
        return;
    float v = w[n_in];
    for (int c = 0; c < n_in; ++c)
        v = fmaf(w[c], in.p[c][s], v);
    out[s] = accumulate ? fmaf(alpha, v, out[s]) : v;
}

cbct_status nn_done(hipError_t e)
{
    if (e == hipSuccess)
        return CBCT_OK;
    set_hip_error(e);
    return CBCT_E_HIP;
}

bool grid_ok(int nz, int ny, int nx)
{
    return nz > 0 && ny > 0 && nx > 0 && (int64_t)nz * ny * nx < (int64_t(1) << 31);
}

}  // namespace
}  // namespace cbct

using namespace cbct;

extern "C" cbct_status cbct_pack16(size_t S, int n_in, const float *const *in, const float *scale,
                                   uint16_t *out, void *stream)
{
    if (!out || (n_in > 0 && !in))
        return CBCT_E_NULL;
    if (n_in < 0 || n_in > 16)
        return CBCT_E_SHAPE;
    CPtrList L{};
    for (int c = 0; c < n_in; ++c) {
        if (!in[c])
            return CBCT_E_NULL;
        L.p[c] = in[c];
        L.scale[c] = scale ? scale[c] : 1.0f;
    }
    if (S == 0)
        return CBCT_OK;
    hipLaunchKernelGGL(k_pack16, dim3((unsigned)((S + kT - 1) / kT)), dim3(kT), 0,
                       (hipStream_t)stream, S, n_in, L, out);
    return nn_done(hipGetLastError());
}

extern "C" cbct_status cbct_conv3(int nz, int ny, int nx, const uint16_t *x, const uint16_t *w,
                                  int transpose_w, const float *bias, const uint16_t *act_mask,
                                  int act, float slope, uint16_t *y_cl, int n_cf,
                                  float *const *y_cf, int accumulate, float alpha, void *stream)
{
    if (!x || !w)
        return CBCT_E_NULL;
    if (!grid_ok(nz, ny, nx) || n_cf < 0 || n_cf > 16)
        return CBCT_E_SHAPE;
    if (!y_cl && n_cf == 0)
        return CBCT_E_ARG;
    ConvArgs A{};
    A.nz = nz;
    A.ny = ny;
    A.nx = nx;
    A.x = x;
    A.w = w;
    A.bias = bias;
    A.mask = act_mask;
    A.transpose_w = transpose_w ? 1 : 0;
    A.act = act ? 1 : 0;
    A.slope = slope;
    A.y_cl = y_cl;
    A.n_cf = n_cf;
    A.accumulate = accumulate ? 1 : 0;
    A.alpha = alpha;
    for (int c = 0; c < n_cf; ++c) {
        if (!y_cf || !y_cf[c])
            return CBCT_E_NULL;
        A.y_cf.p[c] = y_cf[c];
    }
    // z planes per workgroup: up to 16 (the halo of a plane is staged once
    // per 16 output planes plus two), fewer where the grid would otherwise
    // give under about 2048 workgroups
    const long bxy = (long)((ny + kRows - 1) / kRows) * ((nx + kBX - 1) / kBX);
    A.zb = (int)std::max(1L, std::min(16L, (long)nz * bxy / 2048));
    const long blocks = bxy * ((nz + A.zb - 1) / A.zb);
    if (blocks >= 0x7fffffffL)
        return CBCT_E_SHAPE;
    if (act_mask)
        hipLaunchKernelGGL(k_conv3<true>, dim3((unsigned)blocks), dim3(kT), 0, (hipStream_t)stream, A);
    else
        hipLaunchKernelGGL(k_conv3<false>, dim3((unsigned)blocks), dim3(kT), 0, (hipStream_t)stream, A);
    return nn_done(hipGetLastError());
}

extern "C" size_t cbct_conv3_wgrad_workspace(size_t)
{
    return (size_t)(kWgWaves + kWgGroups) * kWgCells;
}

extern "C" cbct_status cbct_conv3_wgrad(int nz, int ny, int nx, const uint16_t *x,
                                        const uint16_t *dy, float *dw, float *db, float *ws,
                                        void *stream)
{
    if (!x || !dy || !dw || !ws)
        return CBCT_E_NULL;
    if (!grid_ok(nz, ny, nx))
        return CBCT_E_SHAPE;
    WgradArgs A{nz, ny, nx, (nx + 31) / 32, x, dy, ws};
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_wgrad, dim3(kWgBlocks), dim3(kT), 0, s, A);
    hipLaunchKernelGGL(k_wgrad_reduce1, dim3((kWgCells + kT - 1) / kT, kWgGroups), dim3(kT), 0,
                       s, ws);
    hipLaunchKernelGGL(k_wgrad_reduce2, dim3((kWgCells + kT - 1) / kT), dim3(kT), 0, s,
                       (const float *)ws, dw, db);
    return nn_done(hipGetLastError());
}

extern "C" cbct_status cbct_conv1(size_t S, int n_in, const float *const *in, const float *w,
                                  float *out, int accumulate, float alpha, void *stream)
{
    if (!out || !w || (n_in > 0 && !in))
        return CBCT_E_NULL;
    if (n_in < 0 || n_in > kMaxCF)
        return CBCT_E_SHAPE;
    CPtrList L{};
    for (int c = 0; c < n_in; ++c) {
        if (!in[c])
            return CBCT_E_NULL;
        L.p[c] = in[c];
    }
    if (S == 0)
        return CBCT_OK;
    hipLaunchKernelGGL(k_conv1, dim3((unsigned)((S + kT - 1) / kT)), dim3(kT), 0,
                       (hipStream_t)stream, S, n_in, L, w, out, accumulate ? 1 : 0, alpha);
    return nn_done(hipGetLastError());
}
