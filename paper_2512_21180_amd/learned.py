"""Learned primal-dual reconstruction (multiscale) on the library's kernels.

arXiv 2512.21180, Alg. 1, with n unrolled iterations: primal latent f (8
volumes), dual latent h (8 sinograms), reconstruction x, normalised
operators A / L (L = ||A||_2) and normalised data y.  Iteration i runs at
resolution 1/r_i (r_i in {1, 2, 4}, non-increasing; all 1 gives the
single-resolution net): the operator is the projector of the geometry with
r_i-times coarser voxels, pixels and angle step (P_alpha), the data and the
field of view are pooled to it (ProjDown, Downsample), and the latents and
x are carried to the next iteration's resolution by nearest upsampling.
At one resolution iteration i reads:

    d1, d2 = halves of h;   p1, p2 = halves of f
    d2 <- d2 + Gamma_i([A p2 / L, A x / L, d1, y])           10 -> 4 channels
    p2 <- p2 + Lambda_i([A^T d2 / L, p1, x, LW, V])         11 -> 4 channels
          LW = A^T (A x / L - y) / L   (the Landweber term)
    x  <- x + o_i . [p1, p2] + o_i,bias                     1x1x1 convolution
    h, f <- Perm(h, rho_i), Perm(f, rho_i)   new channel k = old channel rho_i[k]

Blocks Gamma and Lambda are conv3 -> LeakyReLU -> conv3 -> LeakyReLU -> conv3
with 16 hidden channels (the paper's dual block has the same three-layer
shape with 64 filters; its primal block is a P4-equivariant U-Net, here the
same plain three-layer block).  V is the field-of-view fraction of Sec. 2.6.
Start: x_0 = 0 or the FDK reconstruction (Alg. 1), f = [x_0, A^T y / L] x 4,
h = [y] x 8.  The couplings are
additive, so an iteration is inverted by recomputing the block and
subtracting (Sec. 2.6: gradients without stored activations): training keeps
only the latents of the last iteration and the reconstructions x_1..x_n
(the output list I of Alg. 1) and rebuilds every earlier latent in the
backward pass.

Arithmetic: projector pair FP32; 3x3x3 convolutions BF16 operands with FP32
accumulation on the matrix cores (cbct_nn.h); latents FP32; every step runs
in the library's kernels.  PyTorch holds device memory, the parameters and
the Adam optimiser.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import cbct

SLOPE = 0.01
NCH = 8


def mixing_permutation(rng: np.random.Generator) -> list:
    """A random permutation rho of 0..7 (new channel k = old channel rho[k])
    that mixes the two halves: some channel moves between them."""
    while True:
        p = [int(v) for v in rng.permutation(NCH)]
        if any(v >= NCH // 2 for v in p[:NCH // 2]):
            return p


def _dw_to_param(dw: torch.Tensor, co: int, ci: int) -> torch.Tensor:
    """[27][16][16] gradient -> [co][ci][3][3][3] (tap t = 9 kz + 3 ky + kx)."""
    return dw.view(3, 3, 3, 16, 16).permute(3, 4, 0, 1, 2)[:co, :ci].contiguous()


class PDNet(torch.nn.Module):
    """Parameters of the n-iteration net (FP32 masters), its fixed
    permutations and the resolution divisor r_i of every iteration
    (Alg. 1: iteration i runs at resolution 1/r_i; 1 = full)."""

    DUAL_IN = 10
    PRIMAL_IN = 11

    def __init__(self, n_iter: int = 8, seed: int = 0, width: int = 16, scales=None,
                 init: str = "zero"):
        super().__init__()
        if init not in ("zero", "fdk"):
            raise ValueError("init is 'zero' or 'fdk'")
        self.init = init
        if width != 16:
            raise ValueError("the convolution kernels are built for 16 channels")
        self.scales = [1] * n_iter if scales is None else [int(r) for r in scales]
        if len(self.scales) != n_iter or any(r not in (1, 2, 4) for r in self.scales) or \
                any(b > a for a, b in zip(self.scales, self.scales[1:])):
            raise ValueError("one non-increasing scale in {1, 2, 4} per iteration")
        gen = torch.Generator().manual_seed(seed)
        rng = np.random.default_rng(seed)
        self.n_iter = n_iter

        def conv(co, ci, gain):
            return torch.nn.Parameter(torch.randn(co, ci, 3, 3, 3, generator=gen)
                                      * (gain / math.sqrt(27 * ci)))

        def block(ci):
            return torch.nn.ParameterList([
                conv(16, ci, math.sqrt(2.0)), torch.nn.Parameter(torch.zeros(16)),
                conv(16, 16, math.sqrt(2.0)), torch.nn.Parameter(torch.zeros(16)),
                conv(4, 16, 0.1), torch.nn.Parameter(torch.zeros(4))])

        self.dual = torch.nn.ModuleList([block(self.DUAL_IN) for _ in range(n_iter)])
        self.primal = torch.nn.ModuleList([block(self.PRIMAL_IN) for _ in range(n_iter)])
        self.out = torch.nn.ParameterList([
            torch.nn.Parameter(torch.cat([0.05 * torch.randn(8, generator=gen), torch.zeros(1)]))
            for _ in range(n_iter)])
        self.perms = [mixing_permutation(rng) for _ in range(n_iter)]

    def oracle_params(self) -> list:
        """The parameters as FP64 numpy arrays in the oracle's layout."""
        out = []
        for i in range(self.n_iter):
            out.append({
                "dual": [p.detach().double().cpu().numpy() for p in self.dual[i]],
                "primal": [p.detach().double().cpu().numpy() for p in self.primal[i]],
                "out": self.out[i].detach().double().cpu().numpy(),
                "perm": list(self.perms[i])})
        return out


class _Prepared:
    """Device copies of the parameters in the kernels' formats."""

    def __init__(self, net: PDNet, zero_blocks: bool = False):
        dev = net.out[0].device
        self.zero_blocks = zero_blocks

        def blk(ps):
            ws = [cbct.conv3_weights(ps[k]) for k in (0, 2, 4)]
            bs = []
            for k in (1, 3, 5):
                b = torch.zeros(16, dtype=torch.float32, device=dev)
                b[:ps[k].numel()] = ps[k].detach()
                bs.append(b)
            return ws, bs

        self.dual = [blk(net.dual[i]) for i in range(net.n_iter)]
        self.primal = [blk(net.primal[i]) for i in range(net.n_iter)]
        # conv1 weights: [o_0..o_7, 1 (the previous x), bias] at full
        # resolution, where x is a ninth input; [o_0..o_7, bias] otherwise
        self.out = []
        for i in range(net.n_iter):
            o = net.out[i].detach().float()
            if net.scales[i] == 1:
                self.out.append(torch.cat([o[:8], torch.ones(1, device=dev), o[8:9]]).contiguous())
            else:
                self.out.append(o.contiguous())
        self.out_host = [net.out[i].detach().double().cpu().numpy() for i in range(net.n_iter)]
        self.perms = [list(p) for p in net.perms]


def scaled_geometry(g: dict, r: int) -> dict:
    """Geometry of the operator at resolution 1/r (Alg. 1, P_alpha with
    alpha = 1/r): every r-th projection, voxels and pixels r times larger,
    same volume, panel and orbit."""
    if r == 1:
        return dict(g)
    n = int(g["n_angles"])
    ang = g.get("angles")
    ang = (2.0 * np.pi * np.arange(n) / n) if ang is None else np.asarray(ang, np.float64)
    h = dict(g)
    h["angles"] = ang[::r].copy()
    h["n_angles"] = int(h["angles"].size)
    for nk, dk in (("nx", "vx"), ("ny", "vy"), ("nz", "vz"), ("nu", "du"), ("nv", "dv")):
        if int(g[nk]) % r:
            raise ValueError(f"{nk} = {g[nk]} is not divisible by {r}")
        h[nk] = int(g[nk]) // r
        h[dk] = float(g[dk]) * r
    return h


class _Buffers:
    """Work buffers for one geometry (allocated once, reused every call)."""

    def __init__(self, geo: cbct.Geometry, train: bool):
        dev = geo.device
        vs, ss = geo.vol_shape, geo.sino_shape
        self.Sv = int(np.prod(vs))
        self.Ss = int(np.prod(ss))
        S = max(self.Sv, self.Ss)
        f32 = dict(dtype=torch.float32, device=dev)
        self.sA = [torch.empty(ss, **f32) for _ in range(5)]     # A p2 (4), A x
        self.sR = torch.empty(ss, **f32)                         # A x / L - y
        self.vB = [torch.empty(vs, **f32) for _ in range(5)]     # A^T d2 (4), A^T r
        self.vX = torch.empty(vs, **f32)                         # Downsample(x)
        self.vC = torch.empty(vs, **f32)                         # output convolution
        nbf = 5 if train else 3
        self.act = [torch.empty((S, 16), dtype=torch.bfloat16, device=dev) for _ in range(nbf)]
        if train:
            self.sT = [torch.empty(ss, **f32) for _ in range(5)]
            self.vG = [torch.empty(vs, **f32) for _ in range(5)]
            self.vT = torch.empty(vs, **f32)
            self.vGX = torch.empty(vs, **f32)                    # gradient of Downsample(x)
            self.ones = torch.ones(vs, **f32)
            self.wg_ws = cbct.conv3_wgrad_workspace(S, dev)
            self.dot_ws = cbct.dot_workspace(max(self.Sv, self.Ss), dev)
            self.dW = [torch.empty((27, 16, 16), **f32) for _ in range(3)]
            self.dB = [torch.empty(16, **f32) for _ in range(3)]

    def acts(self, S):
        return [a[:S] for a in self.act]


class LearnedPD:
    """The net bound to one full-resolution geometry: inference and
    reversible training, at the resolutions the net's scales name."""

    def __init__(self, net: PDNet, geo: cbct.Geometry, V: torch.Tensor, L: float):
        self.net = net
        self.geo = geo
        self.V = V.contiguous()
        self.L = float(L)
        self.levels = {}
        for r in sorted(set(net.scales)):
            gr = geo if r == 1 else cbct.Geometry(scaled_geometry(geo.params, r), geo.device)
            Vr = self.V if r == 1 else cbct.pool(self.V, r)
            self.levels[r] = {"geo": gr, "V": Vr, "vgrid": tuple(gr.vol_shape),
                              "sgrid": tuple(gr.sino_shape), "bufs": {}}
        # full-resolution grids (the output resolution)
        self.vgrid = tuple(geo.vol_shape)
        self.sgrid = tuple(geo.sino_shape)

    def _buf(self, r, train):
        lv = self.levels[r]
        if train not in lv["bufs"]:
            lv["bufs"][train] = _Buffers(lv["geo"], train)
        return lv["bufs"][train]

    # ---- blocks -------------------------------------------------------------

    def _block_forward(self, grid, S, inputs, scales, wb, targets, alpha, B):
        """targets += alpha * block(inputs); leaves the packed input and both
        hidden activations in B.act[0..2]."""
        X0, H1, H2 = B.acts(S)[:3]
        (W1, W2, W3), (b1, b2, b3) = wb
        cbct.pack16(inputs, out=X0, scale=scales)
        cbct.conv3(grid, X0, W1, bias=b1, act=True, slope=SLOPE, y_cl=H1)
        cbct.conv3(grid, H1, W2, bias=b2, act=True, slope=SLOPE, y_cl=H2)
        cbct.conv3(grid, H2, W3, bias=b3, y_cf=targets, accumulate=True, alpha=alpha)

    def _block_backward(self, grid, S, g_out, wb, grad_dst, B, params):
        """Backward through a block whose activations are in B.act[0..2];
        grad_dst[c] += d loss / d (packed input channel c); parameter
        gradients into params[k].grad."""
        X0, H1, H2, Ga, Gb = B.acts(S)
        (W1, W2, W3), _ = wb
        cbct.pack16(g_out, out=Ga)
        cbct.conv3_wgrad(grid, H2, Ga, B.dW[2], B.dB[2], B.wg_ws)
        cbct.conv3(grid, Ga, W3, transpose_w=True, mask=H2, slope=SLOPE, y_cl=Gb)
        cbct.conv3_wgrad(grid, H1, Gb, B.dW[1], B.dB[1], B.wg_ws)
        cbct.conv3(grid, Gb, W2, transpose_w=True, mask=H1, slope=SLOPE, y_cl=Ga)
        cbct.conv3_wgrad(grid, X0, Ga, B.dW[0], B.dB[0], B.wg_ws)
        cbct.conv3(grid, Ga, W1, transpose_w=True, y_cf=grad_dst, accumulate=True, alpha=1.0)
        for k in range(3):
            w, b = params[2 * k], params[2 * k + 1]
            w.grad = _dw_to_param(B.dW[k], w.shape[0], w.shape[1])
            b.grad = B.dB[k][:b.numel()].clone()

    # ---- forward ------------------------------------------------------------

    def _data(self, y):
        """ProjDown(y) for every resolution the net uses."""
        return {r: (y if r == 1 else cbct.projdown(y, r)) for r in self.levels}

    def init_state(self, y: torch.Tensor, ys=None):
        """Latents at the first iteration's resolution and x_0 (zero, or the
        FDK reconstruction of Alg. 1 with the Hann-apodised ramp: since
        A x = L y for normalised data, x_0 = L FDK(y))."""
        geo, L = self.geo, self.L
        r0 = self.net.scales[0]
        ys = self._data(y) if ys is None else ys
        xbp = cbct.adjoint(geo, y)
        cbct.axpby(xbp, 1.0 / L, xbp, 0.0, xbp)
        if r0 != 1:
            xbp = cbct.pool(xbp, r0)
        if self.net.init == "fdk":
            x = cbct.fdk(geo, y, window="hann")
            cbct.axpby(x, L, x, 0.0, x)
            xb = x if r0 == 1 else cbct.pool(x, r0)
        else:
            x = torch.zeros(geo.vol_shape, dtype=torch.float32, device=y.device)
            xb = torch.zeros_like(xbp)
        f = []
        for k in range(NCH):
            f.append(xb.clone() if k % 2 == 0 else xbp.clone())
        h = [ys[r0].clone() for _ in range(NCH)]
        return f, h, x

    def _iteration(self, P, i, f, h, x, ys, x_out):
        """One iteration: couplings at resolution 1/r_i, x_out = x + Up(conv1),
        then the permutation.  Returns (f, h, x_out)."""
        L = self.L
        r = self.net.scales[i]
        lv = self.levels[r]
        geo, B, V, y = lv["geo"], self._buf(r, False), lv["V"], ys[r]
        xb = x if r == 1 else cbct.pool(x, r, out=B.vX)
        d1, d2 = h[:4], h[4:]
        p1, p2 = f[:4], f[4:]
        if not P.zero_blocks:
            cbct.batch_forward([geo] * 5, p2 + [xb], outs=B.sA)
            self._block_forward(lv["sgrid"], B.Ss, B.sA + d1 + [y], [1.0 / L] * 5 + [1.0] * 5,
                                P.dual[i], d2, 1.0, B)
            cbct.axpby(B.sR, 1.0 / L, B.sA[4], -1.0, y)
            cbct.batch_adjoint([geo] * 5, d2 + [B.sR], outs=B.vB)
            self._block_forward(lv["vgrid"], B.Sv, B.vB[:4] + p1 + [xb, B.vB[4], V],
                                [1.0 / L] * 4 + [1.0] * 5 + [1.0 / L, 1.0],
                                P.primal[i], p2, 1.0, B)
        if r == 1:
            cbct.conv1(p1 + p2 + [x], P.out[i], x_out)
        else:
            cbct.conv1(p1 + p2, P.out[i], B.vC)
            cbct.axpby(x_out, 1.0, x, 0.0, x)
            cbct.upsample(B.vC, r, out=x_out, accumulate=True)
        rho = P.perms[i]
        return [f[k] for k in rho], [h[k] for k in rho], x_out

    def _refine(self, i, f, h):
        """Nearest upsampling of the latents to the next iteration's resolution."""
        sc = self.net.scales
        if i + 1 < len(sc) and sc[i + 1] < sc[i]:
            q = sc[i] // sc[i + 1]
            f = [cbct.upsample(z, q) for z in f]
            h = [cbct.upsample(z, q) for z in h]
        return f, h

    @torch.no_grad()
    def reconstruct(self, y: torch.Tensor, zero_blocks: bool = False, callback=None):
        """x_n for normalised data y; callback(i, x_i) after each iteration."""
        P = _Prepared(self.net, zero_blocks)
        ys = self._data(y)
        f, h, x = self.init_state(y, ys)
        pair = [x, torch.empty_like(x)]       # x_i and x_{i+1} alternate
        for i in range(self.net.n_iter):
            f, h, x = self._iteration(P, i, f, h, pair[i % 2], ys, pair[1 - i % 2])
            f, h = self._refine(i, f, h)
            if callback is not None:
                callback(i + 1, x)
        return x

    # ---- training -----------------------------------------------------------

    def loss_and_grad(self, y: torch.Tensor, x_true: torch.Tensor, wmask: torch.Tensor) -> float:
        """loss = sum_i 0.5 sum_p wmask_p (x_i,p - x_true,p)^2 over the n
        iterates; fills .grad of every parameter.  Reversible: latents of
        earlier iterations are rebuilt by inverting the couplings (and the
        nearest upsampling between resolutions, by block averages)."""
        net, L = self.net, self.L
        sc = net.scales
        P = _Prepared(net)
        dev = y.device
        with torch.no_grad():
            ys = self._data(y)
            f, h, x = self.init_state(y, ys)
            xs = [x]
            for i in range(net.n_iter):
                f, h, xn = self._iteration(P, i, f, h, xs[-1], ys, torch.empty_like(x))
                f, h = self._refine(i, f, h)
                xs.append(xn)
            n = net.n_iter
            res = torch.empty_like(x)                 # weighted residual of an iterate
            res_ws = cbct.dot_workspace(x.numel(), dev)
            cells = torch.zeros(2 * n + 9 * n, dtype=torch.float64, device=dev)
            gf = gh = None
            gx = torch.zeros_like(x)
            for i in reversed(range(n)):
                r = sc[i]
                lv = self.levels[r]
                geo, B, V, yb = lv["geo"], self._buf(r, True), lv["V"], ys[r]
                if gf is None:
                    gf = [torch.zeros(geo.vol_shape, dtype=torch.float32, device=dev)
                          for _ in range(NCH)]
                    gh = [torch.zeros(geo.sino_shape, dtype=torch.float32, device=dev)
                          for _ in range(NCH)]
                elif sc[i + 1] < r:
                    # back to this resolution: block averages undo the nearest
                    # upsampling of the latents; block sums are its adjoint
                    q = r // sc[i + 1]
                    f = [cbct.pool(z, q) for z in f]
                    h = [cbct.pool(z, q) for z in h]
                    gf = [cbct.pool(z, q, scale=1.0) for z in gf]
                    gh = [cbct.pool(z, q, scale=1.0) for z in gh]
                # loss term of x_{i+1}
                cbct.wresid(res, wmask, xs[i + 1], x_true)
                cbct.dot(res, xs[i + 1], res_ws, cells[2 * i:2 * i + 1])
                cbct.dot(res, x_true, res_ws, cells[2 * i + 1:2 * i + 2])
                cbct.axpby(gx, 1.0, gx, 1.0, res)
                # undo the permutation (states and their gradients)
                rho = P.perms[i]
                fn, hn, gfn, ghn = [None] * NCH, [None] * NCH, [None] * NCH, [None] * NCH
                for k, rr in enumerate(rho):
                    fn[rr], hn[rr], gfn[rr], ghn[rr] = f[k], h[k], gf[k], gh[k]
                # output convolution: x_{i+1} = x_i + Up_r(o . fn + bias)
                gc = gx if r == 1 else cbct.pool(gx, r, out=B.vC, scale=1.0)
                oc = cells[2 * n + 9 * i:2 * n + 9 * i + 9]
                for c in range(NCH):
                    cbct.dot(fn[c], gc, B.dot_ws, oc[c:c + 1])
                cbct.dot(B.ones, gc, B.dot_ws, oc[8:9])
                oh = P.out_host[i]
                for c in range(NCH):
                    cbct.axpby(gfn[c], 1.0, gfn[c], float(oh[c]), gc)
                # Downsample(x_i) and the buffer for its gradient
                if r == 1:
                    xb, gxb = xs[i], gx
                else:
                    xb = cbct.pool(xs[i], r, out=B.vX)
                    gxb = B.vGX
                    gxb.zero_()
                p1, p2, d1, d2 = fn[:4], fn[4:], hn[:4], hn[4:]
                # primal coupling: rebuild its input, invert, backpropagate
                cbct.forward(geo, xb, out=B.sA[4])
                cbct.axpby(B.sR, 1.0 / L, B.sA[4], -1.0, yb)
                cbct.batch_adjoint([geo] * 5, d2 + [B.sR], outs=B.vB)
                self._block_forward(lv["vgrid"], B.Sv, B.vB[:4] + p1 + [xb, B.vB[4], V],
                                    [1.0 / L] * 4 + [1.0] * 5 + [1.0 / L, 1.0],
                                    P.primal[i], p2, -1.0, B)
                for t in B.vG:
                    t.zero_()
                self._block_backward(lv["vgrid"], B.Sv, gfn[4:], P.primal[i],
                                     B.vG[:4] + gfn[:4] + [gxb, B.vG[4]], B, net.primal[i])
                # d(A^T d2 / L): g_d2 += A g / L;  d(LW): g_xb += A^T A g / L^2
                cbct.batch_forward([geo] * 5, B.vG, outs=B.sT)
                for c in range(4):
                    cbct.axpby(ghn[4 + c], 1.0, ghn[4 + c], 1.0 / L, B.sT[c])
                cbct.adjoint(geo, B.sT[4], out=B.vT)
                cbct.axpby(gxb, 1.0, gxb, 1.0 / (L * L), B.vT)
                # dual coupling
                cbct.batch_forward([geo] * 4, p2, outs=B.sA[:4])
                self._block_forward(lv["sgrid"], B.Ss, B.sA + d1 + [yb], [1.0 / L] * 5 + [1.0] * 5,
                                    P.dual[i], d2, -1.0, B)
                for t in B.sT:
                    t.zero_()
                self._block_backward(lv["sgrid"], B.Ss, ghn[4:], P.dual[i], B.sT + ghn[:4], B,
                                     net.dual[i])
                cbct.batch_adjoint([geo] * 5, B.sT, outs=B.vG)
                for c in range(4):
                    cbct.axpby(gfn[4 + c], 1.0, gfn[4 + c], 1.0 / L, B.vG[c])
                cbct.axpby(gxb, 1.0, gxb, 1.0 / L, B.vG[4])
                if r != 1:       # adjoint of average pooling
                    cbct.upsample(gxb, r, out=gx, scale=1.0 / r ** 3, accumulate=True)
                f, h, gf, gh = fn, hn, gfn, ghn
            self.rebuilt = (f, h)      # latents before the first iteration, rebuilt
            vals = cells.cpu().numpy()
            loss = 0.5 * float(sum(vals[2 * i] - vals[2 * i + 1] for i in range(n)))
            for i in range(n):
                net.out[i].grad = torch.tensor(vals[2 * n + 9 * i:2 * n + 9 * i + 9],
                                               dtype=torch.float32, device=dev)
        return loss
