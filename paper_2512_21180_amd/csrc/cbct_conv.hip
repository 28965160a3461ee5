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
// LDS read of the staged channel-last activations.  The weights are staged
// once per workgroup and stay in registers over the wave's four tiles.  The result tile (lane l holds rows 4 (l/16) .. +3 of
// column l%16) goes through the epilogue: bias, LeakyReLU derivative mask,
// LeakyReLU, then bf16 channel-last and/or FP32 channel-first stores.
//
// Weight gradient (conv3_wgrad): per wavefront, per 16-position chunk of a
// row, one v_mfma_f32_16x16x16_bf16 per tap with M = 16 output channels,
// N = 16 input channels, K = 16 positions; the 9 neighbouring input rows of
// the chunk are staged in LDS per wave.  Each wave keeps its 27 tiles in
// registers and writes them to a workspace; one ordered reduction follows.
#include <hip/hip_runtime.h>

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

// A workgroup computes an output block of one z plane, kRows rows and 64
// positions along x (4 x-tiles of 16): wave w takes row y0 + w and its four
// tiles.  The block's input halo (3 planes x (kRows + 2) rows x 66 positions
// x 16 channels) and the layer's weights are staged in LDS once; each MFMA's
// A operand is one 16-byte LDS read per lane (channels 0-7 and 8-15 in
// separate planes, so the 16 lanes of a group read consecutive words).
constexpr int kRows = 4, kBX = 64;
constexpr int kHX = kBX + 2, kHY = kRows + 2, kHP = 3 * kHY * kHX;   // halo positions

__global__ void __launch_bounds__(kT) k_conv3(ConvArgs A)
{
    __shared__ uint4 halo[2][kHP];            // [channel half][position] 8 bf16 each
    __shared__ uint4 wsh[27 * 16 * 2];        // [tap][cout][channel half]

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nbx = (A.nx + kBX - 1) / kBX, nby = (A.ny + kRows - 1) / kRows;
    const int bx = blockIdx.x % nbx;
    const int by = (blockIdx.x / nbx) % nby;
    const int z = blockIdx.x / (nbx * nby);
    const int x0 = bx * kBX, y0 = by * kRows;

    // ---- stage the weights: wsh[t][co][h] = 8 input channels 8h.. of w'[t][co]
    for (int e = tid; e < 27 * 16 * 2; e += kT) {
        const int t = e >> 5, co = (e >> 1) & 15, h = e & 1;
        uint4 q;
        if (!A.transpose_w) {
            q = *reinterpret_cast<const uint4 *>(A.w + ((size_t)t * 16 + co) * 16 + 8 * h);
        } else {
            // w'[t][co][ci] = w[26 - t][ci][co]
            uint16_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[j] = A.w[((size_t)(26 - t) * 16 + 8 * h + j) * 16 + co];
            q = make_uint4((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                           (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16));
        }
        wsh[e] = q;
    }
    // ---- stage the input halo (zero outside the grid)
    for (int e = tid; e < 2 * kHP; e += kT) {
        const int hp = e >> 1, h = e & 1;
        const int hx = hp % kHX, hy = (hp / kHX) % kHY, hz = hp / (kHX * kHY);
        const int xx = x0 - 1 + hx, yy = y0 - 1 + hy, zz = z - 1 + hz;
        uint4 q = make_uint4(0u, 0u, 0u, 0u);
        if ((unsigned)xx < (unsigned)A.nx && (unsigned)yy < (unsigned)A.ny &&
            (unsigned)zz < (unsigned)A.nz) {
            const size_t pos = ((size_t)zz * A.ny + yy) * A.nx + xx;
            q = *reinterpret_cast<const uint4 *>(A.x + pos * 16 + 8 * h);
        }
        halo[h][hp] = q;
    }
    __syncthreads();

    const int y = y0 + w;
    if (y >= A.ny)
        return;   // whole wave; no barrier follows

    const int m = lane & 15;          // position within the tile (A rows) / output channel (B cols)
    const int kb = lane >> 4;         // k block: tap 2p + (kb >> 1), channels 8 (kb & 1) ..
    const int hh = kb & 1;

    // weights: B[k][n] for n = m (output channel), 8 input channels of half hh
    bf16x8 wr[14];
#pragma unroll
    for (int p = 0; p < 14; ++p) {
        const int t = 2 * p + (kb >> 1);
        bf16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
        if (t < 27)
            v = __builtin_bit_cast(bf16x8, wsh[(t * 16 + m) * 2 + hh]);
        wr[p] = v;
    }
    const int co = m;
    const float b = A.bias ? A.bias[co] : 0.0f;

    for (int tx = 0; tx < kBX / 16; ++tx) {
        const int xt0 = x0 + 16 * tx;
        if (xt0 >= A.nx)
            break;   // uniform
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int p = 0; p < 14; ++p) {
            const int t = 2 * p + (kb >> 1);
            bf16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
            if (t < 27) {
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;   // offsets + 1
                const int hp = (dz * kHY + (w + dy)) * kHX + 16 * tx + m + dx;
                a = __builtin_bit_cast(bf16x8, halo[hh][hp]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wr[p], acc, 0, 0, 0);
        }
        // epilogue: lane holds rows 4 kb + i (positions), column m (output channel)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int xo = xt0 + 4 * kb + i;
            if (xo >= A.nx)
                continue;
            const size_t pos = ((size_t)z * A.ny + y) * A.nx + xo;
            float v = acc[i] + b;
            if (A.mask) {
                const uint16_t hm = A.mask[pos * 16 + co];
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

// ---- conv3 weight gradient ---------------------------------------------------

constexpr int kWgBlocks = 256;               // fixed: the reduction order is fixed
constexpr int kWgWaves = kWgBlocks * 4;
constexpr int kWgCells = 27 * 256 + 16;      // dw tiles + db

struct WgradArgs {
    int nz, ny, nx, nxt;
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

// Wave-private LDS: 9 neighbouring rows x 18 positions (x0-1 .. x0+16) x 16 ch.
constexpr int kRowPos = 18;

__global__ void __launch_bounds__(kT) k_wgrad(WgradArgs A)
{
    __shared__ uint16_t stage[4][9][kRowPos][16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = blockIdx.x * 4 + wv;          // global wave index, fixed work split
    const int n_rows = A.nz * A.ny;
    const int m = lane & 15, kb = lane >> 4;     // M = output channel m, K block kb
    uint16_t(*st)[kRowPos][16] = stage[wv];

    f32x4 acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t)
        acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float dbp = 0.0f;

    for (int row = gw; row < n_rows; row += kWgWaves) {
        const int y = row % A.ny, z = row / A.ny;
        for (int xt = 0; xt < A.nxt; ++xt) {
            const int x0 = xt * 16;
            // stage the 9 neighbouring rows: 9 * 18 positions * 2 halves of 8 channels
            for (int e = lane; e < 9 * kRowPos * 2; e += 64) {
                const int half = e & 1, pe = (e >> 1) % kRowPos, r9 = (e >> 1) / kRowPos;
                const int zz = z + r9 / 3 - 1, yy = y + r9 % 3 - 1, xx = x0 - 1 + pe;
                uint4 q = make_uint4(0, 0, 0, 0);
                if ((unsigned)zz < (unsigned)A.nz && (unsigned)yy < (unsigned)A.ny &&
                    (unsigned)xx < (unsigned)A.nx)
                    q = *reinterpret_cast<const uint4 *>(
                        A.x + (((size_t)zz * A.ny + yy) * A.nx + xx) * 16 + half * 8);
                *reinterpret_cast<uint4 *>(&st[r9][pe][half * 8]) = q;
            }
            wave_sync();   // staged rows visible to every lane of this wave
            // A[m = co][k = 4 positions of block kb] = dy
            bf16x4 a;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int xo = x0 + 4 * kb + j;
                uint16_t h = 0;
                if (xo < A.nx)
                    h = A.dy[(((size_t)z * A.ny + y) * A.nx + xo) * 16 + m];
                a[j] = (short)h;
                dbp += bf2f(h);
            }
#pragma unroll
            for (int t = 0; t < 27; ++t) {
                const int r9 = t / 3, dx = t % 3 - 1;
                // B[k = positions][n = ci = m]: x at position x0 + 4 kb + j + dx
                bf16x4 bv;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bv[j] = (short)st[r9][4 * kb + j + dx + 1][m];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[t], 0, 0, 0);
            }
            wave_sync();   // every lane done reading before the next chunk's writes
        }
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

__global__ void __launch_bounds__(kT) k_wgrad_reduce(const float *ws, float *dw, float *db)
{
    const int e = blockIdx.x * kT + threadIdx.x;
    if (e >= kWgCells)
        return;
    float s = 0.0f;
    for (int w = 0; w < kWgWaves; ++w)
        s += ws[(size_t)w * kWgCells + e];
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
    const long blocks = (long)nz * ((ny + kRows - 1) / kRows) * ((nx + kBX - 1) / kBX);
    if (blocks >= 0x7fffffffL)
        return CBCT_E_SHAPE;
    hipLaunchKernelGGL(k_conv3, dim3((unsigned)blocks), dim3(kT), 0, (hipStream_t)stream, A);
    return nn_done(hipGetLastError());
}

extern "C" size_t cbct_conv3_wgrad_workspace(size_t) { return (size_t)kWgWaves * kWgCells; }

extern "C" cbct_status cbct_conv3_wgrad(int nz, int ny, int nx, const uint16_t *x,
                                        const uint16_t *dy, float *dw, float *db, float *ws,
                                        void *stream)
{
    if (!x || !dy || !dw || !ws)
        return CBCT_E_NULL;
    if (!grid_ok(nz, ny, nx))
        return CBCT_E_SHAPE;
    WgradArgs A{nz, ny, nx, (nx + 15) / 16, x, dy, ws};
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_wgrad, dim3(kWgBlocks), dim3(kT), 0, s, A);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((kWgCells + kT - 1) / kT), dim3(kT), 0, s,
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
