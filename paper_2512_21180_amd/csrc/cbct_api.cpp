// C-ABI compute entry points of libcbct.so: argument validation and kernel
// launches for the projector pair (arXiv 2512.21180, Sec. 2.2; multi-channel
// and multi-resolution use as in Alg. 1).
#include <hip/hip_runtime.h>

#include <vector>

#include "cbct_internal.h"

namespace cbct {

// The next chunk of a stack with `left` channels still to project: 4
// channels where the geometry allows them (cmax = 4), else 2, and a last
// single channel on the single-channel kernel (5 channels: 4 + 1).
static int chunk_size(int left, int cmax)
{
    return left >= 4 && cmax >= 4 ? 4 : left >= 2 ? 2 : 1;
}

hipError_t launch_forward(const cbct_geom *g, const void *vol, cbct_dtype vt, void *sino,
                          cbct_dtype st, int channels, hipStream_t s)
{
    if (!g->fwd.ok)
        return launch_forward_simple(g->dev, vol, vt, sino, st, channels, s);
    const int cmax = forward_mc_max_channels(g);
    if (channels < 2 || vt != CBCT_F32 || st != CBCT_F32 || cmax < 2)
        return launch_forward_tiled(g->dev, g->fwd, vol, vt, sino, st, channels, s);
    // FP32 channel stacks: chunks of up to cmax channels share each sample's
    // geometry (bitwise the same results as one channel at a time)
    const size_t nvox = (size_t)g->desc.nx * g->desc.ny * g->desc.nz;
    const size_t nsino = (size_t)g->desc.n_angles * g->desc.nv * g->desc.nu;
    const float *x = (const float *)vol;
    float *y = (float *)sino;
    for (int c0 = 0; c0 < channels;) {
        const int c = chunk_size(channels - c0, cmax);
        hipError_t e;
        if (c == 1) {
            e = launch_forward_tiled(g->dev, g->fwd, x + c0 * nvox, vt, y + c0 * nsino, st, 1, s);
        } else {
            const float *xs[kMaxMcChannels];
            float *ys[kMaxMcChannels];
            for (int i = 0; i < c; ++i) {
                xs[i] = x + (c0 + i) * nvox;
                ys[i] = y + (c0 + i) * nsino;
            }
            e = launch_forward_mc(1, &g, xs, ys, c, s);
        }
        if (e != hipSuccess)
            return e;
        c0 += c;
    }
    return hipSuccess;
}

hipError_t launch_adjoint(const cbct_geom *g, const void *sino, cbct_dtype st, void *vol,
                          cbct_dtype vt, int channels, hipStream_t s)
{
    if (g->adj.ok)
        return launch_adjoint_brick(g->dev, g->adj, sino, st, vol, vt, channels, s);
    return launch_adjoint_simple(g->dev, sino, st, vol, vt, channels, s);
}

}  // namespace cbct

using namespace cbct;

static bool dtype_ok(cbct_dtype t) { return t == CBCT_F32 || t == CBCT_BF16 || t == CBCT_F16; }

static cbct_status check_device(const cbct_geom *g)
{
    if (!g->dev_block)
        return CBCT_E_ARG;   // host-only handle
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) {
        set_hip_error(e);
        return CBCT_E_HIP;
    }
    if (cur != g->device) {
        set_hip_error(hipErrorInvalidDevice);
        return CBCT_E_HIP;
    }
    return CBCT_OK;
}

static cbct_status finish(hipError_t e)
{
    if (e == hipSuccess)
        return CBCT_OK;
    set_hip_error(e);
    return e == hipErrorInvalidValue ? CBCT_E_DTYPE : CBCT_E_HIP;
}

extern "C" cbct_status cbct_forward(const cbct_geom *g, const void *vol, cbct_dtype vt,
                                    void *sino, cbct_dtype st, int n_channels, void *stream)
{
    if (!g || !vol || !sino)
        return CBCT_E_NULL;
    if (!dtype_ok(vt) || !dtype_ok(st))
        return CBCT_E_DTYPE;
    if (n_channels < 1 || n_channels > 65535 ||
        (!g->fwd.ok && (int64_t)n_channels * g->desc.n_angles > 65535))
        return CBCT_E_SHAPE;
    cbct_status s = check_device(g);
    if (s != CBCT_OK)
        return s;
    return finish(launch_forward(g, vol, vt, sino, st, n_channels, (hipStream_t)stream));
}

extern "C" cbct_status cbct_adjoint(const cbct_geom *g, const void *sino, cbct_dtype st,
                                    void *vol, cbct_dtype vt, int n_channels, void *stream)
{
    if (!g || !vol || !sino)
        return CBCT_E_NULL;
    if (!dtype_ok(vt) || !dtype_ok(st))
        return CBCT_E_DTYPE;
    if (n_channels < 1 || n_channels > 65535)
        return CBCT_E_SHAPE;
    cbct_status s = check_device(g);
    if (s != CBCT_OK)
        return s;
    return finish(launch_adjoint(g, sino, st, vol, vt, n_channels, (hipStream_t)stream));
}

// Channel groups of a batch: the cases of each geometry handle that occurs
// more than once (tiled plan) are cut into chunks of up to the plan's
// channel limit; chunks of two or more channels are launched through the
// multichannel kernel, up to kMaxMcGroups chunks of one size per launch, and
// marked done.  Single leftover cases stay for the single-channel batch.
static hipError_t batch_forward_groups(int n, const cbct_geom *const *g,
                                       const void *const *vols, void *const *sinos,
                                       std::vector<char> &done, hipStream_t s)
{
    // pending chunks per channel count
    const cbct_geom *gg[kMaxMcChannels + 1][kMaxMcGroups];
    const float *xx[kMaxMcChannels + 1][kMaxMcGroups * kMaxMcChannels];
    float *yy[kMaxMcChannels + 1][kMaxMcGroups * kMaxMcChannels];
    int m[kMaxMcChannels + 1] = {};
    auto flush = [&](int c) -> hipError_t {
        hipError_t e = m[c] ? launch_forward_mc(m[c], gg[c], xx[c], yy[c], c, s) : hipSuccess;
        m[c] = 0;
        return e;
    };
    std::vector<int> idx;
    for (int i = 0; i < n; ++i) {
        if (done[i] || !g[i]->fwd.ok)
            continue;
        const int cmax = forward_mc_max_channels(g[i]);
        idx.clear();
        for (int j = i; j < n; ++j)
            if (!done[j] && g[j] == g[i])
                idx.push_back(j);
        const int cnt = (int)idx.size();
        if (cnt < 2 || cmax < 2)
            continue;
        for (int c0 = 0; c0 < cnt;) {
            const int c = chunk_size(cnt - c0, cmax);
            if (c >= 2) {
                gg[c][m[c]] = g[i];
                for (int t = 0; t < c; ++t) {
                    const int j = idx[c0 + t];
                    xx[c][m[c] * c + t] = (const float *)vols[j];
                    yy[c][m[c] * c + t] = (float *)sinos[j];
                    done[j] = 1;
                }
                if (++m[c] == kMaxMcGroups) {
                    hipError_t e = flush(c);
                    if (e != hipSuccess)
                        return e;
                }
            }
            c0 += c;
        }
    }
    for (int c = 2; c <= kMaxMcChannels; ++c) {
        hipError_t e = flush(c);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

static cbct_status check_batch(int n, const cbct_geom *const *g, const void *const *a,
                               const void *const *b, cbct_dtype t1, cbct_dtype t2)
{
    if (n < 1)
        return CBCT_E_SHAPE;
    if (!g || !a || !b)
        return CBCT_E_NULL;
    if (!dtype_ok(t1) || !dtype_ok(t2))
        return CBCT_E_DTYPE;
    for (int i = 0; i < n; ++i) {
        if (!g[i] || !a[i] || !b[i])
            return CBCT_E_NULL;
        cbct_status s = check_device(g[i]);
        if (s != CBCT_OK)
            return s;
    }
    return CBCT_OK;
}

// Batches run as single launches over the work items of up to kMaxBatch cases; a case
// whose plan fell back to the one-thread-per-output kernels is launched on
// its own (same arithmetic, so the results are the same bits either way).
extern "C" cbct_status cbct_batch_forward(int n, const cbct_geom *const *g, const void *const *vols,
                                          void *const *sinos, cbct_dtype vt, cbct_dtype st,
                                          void *stream)
{
    cbct_status s = check_batch(n, g, vols, (const void *const *)sinos, vt, st);
    if (s != CBCT_OK)
        return s;
    hipStream_t hs = (hipStream_t)stream;
    // FP32 cases that share a geometry handle run as channel groups of the
    // multichannel kernel (same bits as one case at a time), the rest as below
    std::vector<char> done(n, 0);
    if (vt == CBCT_F32 && st == CBCT_F32) {
        hipError_t e = batch_forward_groups(n, g, vols, sinos, done, hs);
        if (e != hipSuccess)
            return finish(e);
    }
    const cbct_geom *gg[kMaxBatch];
    const void *xx[kMaxBatch];
    void *yy[kMaxBatch];
    int m = 0;
    auto flush = [&]() -> hipError_t {
        hipError_t e = m ? launch_forward_batch(m, gg, xx, yy, vt, st, hs) : hipSuccess;
        m = 0;
        return e;
    };
    for (int i = 0; i < n; ++i) {
        hipError_t e = hipSuccess;
        if (done[i])
            continue;
        if (!g[i]->fwd.ok) {
            e = launch_forward(g[i], vols[i], vt, sinos[i], st, 1, hs);
        } else {
            gg[m] = g[i];
            xx[m] = vols[i];
            yy[m] = sinos[i];
            if (++m == kMaxBatch)
                e = flush();
        }
        if (e != hipSuccess)
            return finish(e);
    }
    return finish(flush());
}

extern "C" cbct_status cbct_batch_adjoint(int n, const cbct_geom *const *g, const void *const *sinos,
                                          void *const *vols, cbct_dtype st, cbct_dtype vt,
                                          void *stream)
{
    cbct_status s = check_batch(n, g, sinos, (const void *const *)vols, st, vt);
    if (s != CBCT_OK)
        return s;
    hipStream_t hs = (hipStream_t)stream;
    const cbct_geom *gg[kMaxBatch];
    const void *yy[kMaxBatch];
    void *xx[kMaxBatch];
    int m = 0;
    auto flush = [&]() -> hipError_t {
        hipError_t e = m ? launch_adjoint_batch(m, gg, yy, xx, st, vt, hs) : hipSuccess;
        m = 0;
        return e;
    };
    for (int i = 0; i < n; ++i) {
        hipError_t e = hipSuccess;
        if (!g[i]->adj.ok) {
            e = launch_adjoint(g[i], sinos[i], st, vols[i], vt, 1, hs);
        } else {
            gg[m] = g[i];
            yy[m] = sinos[i];
            xx[m] = vols[i];
            if (++m == kMaxBatch)
                e = flush();
        }
        if (e != hipSuccess)
            return finish(e);
    }
    return finish(flush());
}

extern "C" cbct_status cbct_geom_plan_info(const cbct_geom *g, int *info, int n)
{
    if (!g || !info)
        return CBCT_E_NULL;
    int v[14] = {g->fwd.ok ? 1 : 0, g->fwd.R,  g->fwd.BQ, g->fwd.BK,    g->fwd.n_tiles,
                 g->adj.ok ? 1 : 0, g->adj.W,  g->adj.H,  g->adj.WS,    g->adj.NTmax,
                 g->adj.KV,         g->fwd.TU, kAdjBI,    kAdjBJ};
    for (int i = 0; i < n && i < 14; ++i)
        info[i] = v[i];
    return CBCT_OK;
}
