"""ctypes binding of libcbct.so: argument marshalling only.

Every computation runs in the library's HIP kernels; PyTorch tensors serve as
device buffers and PyTorch's current stream as the launch stream.  There is
no fallback: if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbct.so")

F32, BF16, F16 = 0, 1, 2
_TORCH2CODE = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}


class CbctError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.cbct_error_string(status).decode()
        if status == -5:
            msg += ": " + _lib.cbct_last_hip_error().decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [
        ("sid_mm", ctypes.c_double), ("sdd_mm", ctypes.c_double),
        ("n_angles", ctypes.c_int), ("angles_rad", ctypes.POINTER(ctypes.c_double)),
        ("nu", ctypes.c_int), ("nv", ctypes.c_int),
        ("du_mm", ctypes.c_double), ("dv_mm", ctypes.c_double),
        ("off_u_mm", ctypes.c_double), ("off_v_mm", ctypes.c_double),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("vx_mm", ctypes.c_double), ("vy_mm", ctypes.c_double), ("vz_mm", ctypes.c_double),
        ("origin_mm", ctypes.c_double * 3),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u64p = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)
    lib.cbct_geom_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp)]
    lib.cbct_geom_destroy.argtypes = [vp]
    lib.cbct_sample_count.argtypes = [vp, u64p]
    lib.cbct_geom_sizes.argtypes = [vp, u64p, u64p]
    lib.cbct_forward.argtypes = [vp, vp, i32, vp, i32, i32, vp]
    lib.cbct_adjoint.argtypes = [vp, vp, i32, vp, i32, i32, vp]
    lib.cbct_batch_forward.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(vp), i32, i32, vp]
    lib.cbct_batch_adjoint.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(vp), i32, i32, vp]
    lib.cbct_geom_plan_info.argtypes = [vp, ctypes.POINTER(i32), i32]
    lib.cbct_geom_create_host.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp)]
    lib.cbct_geom_table.argtypes = [vp, i32, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    sz, dp = ctypes.c_size_t, ctypes.c_double
    lib.cbct_dot_workspace.argtypes = [sz]
    lib.cbct_dot_workspace.restype = sz
    lib.cbct_dot.argtypes = [sz, vp, vp, vp, vp, vp]
    lib.cbct_dot_noalloc.argtypes = [sz, vp, vp, vp, vp]
    lib.cbct_dot_noalloc_max_cells.argtypes = []
    lib.cbct_dot_noalloc_max_cells.restype = sz
    lib.cbct_axpy_ratio.argtypes = [sz, vp, vp, vp, vp, dp, vp]
    lib.cbct_xpay_ratio.argtypes = [sz, vp, vp, vp, vp, vp]
    lib.cbct_axpby.argtypes = [sz, vp, ctypes.c_float, vp, ctypes.c_float, vp, vp]
    u32, u64 = ctypes.c_uint32, ctypes.c_uint64
    lib.cbct_philox_blocks.argtypes = [sz, u64, u32, vp, vp]
    lib.cbct_sim_poisson_log.argtypes = [sz, vp, vp, vp, dp, u64, u32, vp]
    lib.cbct_sim_gaussian.argtypes = [sz, vp, vp, dp, u64, u32, vp]
    lib.cbct_water_bone.argtypes = [sz, vp, vp, vp, vp]
    lib.cbct_poly_bins.argtypes = [i32, vp, vp, ctypes.POINTER(i32)]
    lib.cbct_sim_poly.argtypes = [sz, sz, vp, vp, i32, vp, vp, vp, vp, u64, u32, vp, vp, vp, vp]
    i64 = ctypes.c_int64
    lib.cbct_scatter_paths.argtypes = [vp, vp, vp, i32, i64, vp, vp, i32, vp, vp]
    lib.cbct_scatter_integrate.argtypes = [vp, vp, vp, i32, i64, vp, vp, vp]
    fl = ctypes.c_float
    lib.cbct_pack16.argtypes = [sz, i32, ctypes.POINTER(vp), ctypes.POINTER(fl), vp, vp]
    lib.cbct_conv3.argtypes = [i32, i32, i32, vp, vp, i32, vp, vp, i32, fl, vp, i32,
                               ctypes.POINTER(vp), i32, fl, vp]
    lib.cbct_conv3_wgrad_workspace.argtypes = [sz]
    lib.cbct_conv3_wgrad_workspace.restype = sz
    lib.cbct_conv3_wgrad.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.cbct_wresid.argtypes = [sz, vp, vp, vp, vp, vp]
    lib.cbct_pool.argtypes = [i32, i32, i32, i32, vp, vp, fl, vp]
    lib.cbct_projdown.argtypes = [i32, i32, i32, i32, vp, vp, fl, vp]
    lib.cbct_upsample.argtypes = [i32, i32, i32, i32, vp, vp, fl, i32, vp]
    lib.cbct_fdk.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.cbct_conv1.argtypes = [sz, i32, ctypes.POINTER(vp), vp, vp, i32, fl, vp]
    lib.cbct_fov_fraction.argtypes = [vp, vp]
    lib.cbct_probe_threads.argtypes = []
    lib.cbct_probe_threads.restype = i32
    lib.cbct_probe_valu.argtypes = [i32, i32, vp, vp]
    lib.cbct_probe_lds.argtypes = [i32, i32, vp, vp]
    lib.cbct_error_string.argtypes = [i32]
    lib.cbct_error_string.restype = ctypes.c_char_p
    lib.cbct_last_hip_error.argtypes = []
    lib.cbct_last_hip_error.restype = ctypes.c_char_p
    for name in ("cbct_geom_create", "cbct_geom_destroy", "cbct_sample_count", "cbct_geom_sizes",
                 "cbct_forward", "cbct_adjoint", "cbct_batch_forward", "cbct_batch_adjoint",
                 "cbct_geom_plan_info", "cbct_geom_create_host", "cbct_geom_table",
                 "cbct_dot", "cbct_axpy_ratio", "cbct_xpay_ratio", "cbct_axpby",
                 "cbct_philox_blocks", "cbct_sim_poisson_log", "cbct_sim_gaussian",
                 "cbct_pack16", "cbct_conv3", "cbct_conv3_wgrad", "cbct_conv1", "cbct_wresid",
                 "cbct_pool", "cbct_projdown", "cbct_upsample", "cbct_fdk",
                 "cbct_fov_fraction", "cbct_probe_valu", "cbct_probe_lds"):
        getattr(lib, name).restype = i32
    return lib


_lib = _load()


def lib():
    return _lib


def _check(status: int, where: str):
    if status != 0:
        raise CbctError(status, where)


def make_desc(g: dict):
    """C descriptor for a geometry dict; returns (desc, keep-alive angle array)."""
    import numpy as np
    ang = g.get("angles")
    arr = None
    ptr = None
    if ang is not None:
        arr = np.ascontiguousarray(np.asarray(ang, dtype=np.float64))
        ptr = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    o = g.get("origin", (0.0, 0.0, 0.0))
    d = Desc(float(g["sid"]), float(g["sdd"]), int(g["n_angles"]), ptr,
             int(g["nu"]), int(g["nv"]), float(g["du"]), float(g["dv"]),
             float(g.get("off_u", 0.0)), float(g.get("off_v", 0.0)),
             int(g["nx"]), int(g["ny"]), int(g["nz"]),
             float(g["vx"]), float(g["vy"]), float(g["vz"]),
             (ctypes.c_double * 3)(*[float(v) for v in o]))
    return d, arr


class Geometry:
    """A validated geometry with its device tables (on the current device)."""

    def __init__(self, g: dict, device=None):
        self.params = dict(g)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        desc, keep = make_desc(g)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.cbct_geom_create(ctypes.byref(desc), ctypes.byref(h)), "cbct_geom_create")
        del keep
        self._h = h
        self.vol_shape = (g["nz"], g["ny"], g["nx"])
        self.sino_shape = (g["n_angles"], g["nv"], g["nu"])

    @property
    def handle(self):
        return self._h

    def sample_count(self) -> int:
        s = ctypes.c_uint64()
        _check(_lib.cbct_sample_count(self._h, ctypes.byref(s)), "cbct_sample_count")
        return int(s.value)

    def plan_info(self) -> dict:
        v = (ctypes.c_int * 12)()
        _check(_lib.cbct_geom_plan_info(self._h, v, 12), "cbct_geom_plan_info")
        keys = ("fwd_tiled", "rays_per_thread", "box_q", "box_k", "tiles",
                "adj_bricked", "win_cols", "win_rows", "lds_stride", "nt_max", "adj_kv",
                "fwd_tile_cols")
        return dict(zip(keys, list(v)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.cbct_geom_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _code(t: torch.Tensor) -> int:
    try:
        return _TORCH2CODE[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}") from None


def _stream(dev) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _prep(t: torch.Tensor, geom: Geometry, shape, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a CUDA (HIP) tensor")
    if t.device != geom.device:
        raise ValueError(f"{what} is on {t.device}, geometry on {geom.device}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if tuple(t.shape[-3:]) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected [..., {shape}]")
    return t.numel() // (shape[0] * shape[1] * shape[2])


def forward(geom: Geometry, vol: torch.Tensor, out: torch.Tensor | None = None,
            out_dtype: torch.dtype | None = None) -> torch.Tensor:
    """Sinogram(s) A vol.  vol: [..., nz, ny, nx] (channels flattened)."""
    C = _prep(vol, geom, geom.vol_shape, "vol")
    if out is None:
        out = torch.empty(tuple(vol.shape[:-3]) + geom.sino_shape, device=vol.device,
                          dtype=out_dtype or vol.dtype)
    else:
        if _prep(out, geom, geom.sino_shape, "out") != C:
            raise ValueError("channel count of out does not match vol")
    with torch.cuda.device(geom.device):
        _check(_lib.cbct_forward(geom.handle, ctypes.c_void_p(vol.data_ptr()), _code(vol),
                                 ctypes.c_void_p(out.data_ptr()), _code(out), C,
                                 _stream(geom.device)), "cbct_forward")
    return out


def adjoint(geom: Geometry, sino: torch.Tensor, out: torch.Tensor | None = None,
            out_dtype: torch.dtype | None = None) -> torch.Tensor:
    """Volume(s) A^T sino.  sino: [..., n_angles, nv, nu]."""
    C = _prep(sino, geom, geom.sino_shape, "sino")
    if out is None:
        out = torch.empty(tuple(sino.shape[:-3]) + geom.vol_shape, device=sino.device,
                          dtype=out_dtype or sino.dtype)
    else:
        if _prep(out, geom, geom.vol_shape, "out") != C:
            raise ValueError("channel count of out does not match sino")
    with torch.cuda.device(geom.device):
        _check(_lib.cbct_adjoint(geom.handle, ctypes.c_void_p(sino.data_ptr()), _code(sino),
                                 ctypes.c_void_p(out.data_ptr()), _code(out), C,
                                 _stream(geom.device)), "cbct_adjoint")
    return out


def _ptrs(ts):
    return (ctypes.c_void_p * len(ts))(*[ctypes.c_void_p(t.data_ptr()) for t in ts])


def batch_forward(geoms, vols, outs=None, out_dtype=None):
    """sinos[i] = A_i vols[i] for single-channel cases: FP32 cases that share a
    geometry object run as channel groups of four or two (the multichannel
    kernel), the rest in one launch over all their work items (same bits
    either way)."""
    n = len(geoms)
    assert len(vols) == n and n > 0
    for g, v in zip(geoms, vols):
        if _prep(v, g, g.vol_shape, "vol") != 1:
            raise ValueError("batch entries are single-channel")
    if outs is None:
        outs = [torch.empty(g.sino_shape, device=v.device, dtype=out_dtype or v.dtype)
                for g, v in zip(geoms, vols)]
    vt, st = _code(vols[0]), _code(outs[0])
    if any(_code(v) != vt for v in vols) or any(_code(o) != st for o in outs):
        raise TypeError("batch entries must share storage types")
    for g, o in zip(geoms, outs):
        _prep(o, g, g.sino_shape, "out")
    hs = (ctypes.c_void_p * n)(*[g.handle for g in geoms])
    with torch.cuda.device(geoms[0].device):
        _check(_lib.cbct_batch_forward(n, hs, _ptrs(vols), _ptrs(outs), vt, st,
                                       _stream(geoms[0].device)), "cbct_batch_forward")
    return outs


def batch_adjoint(geoms, sinos, outs=None, out_dtype=None):
    """vols[i] = A_i^T sinos[i] for heterogeneous single-channel cases, in one
    launch per 16 cases."""
    n = len(geoms)
    assert len(sinos) == n and n > 0
    for g, s in zip(geoms, sinos):
        if _prep(s, g, g.sino_shape, "sino") != 1:
            raise ValueError("batch entries are single-channel")
    if outs is None:
        outs = [torch.empty(g.vol_shape, device=s.device, dtype=out_dtype or s.dtype)
                for g, s in zip(geoms, sinos)]
    st, vt = _code(sinos[0]), _code(outs[0])
    if any(_code(s) != st for s in sinos) or any(_code(o) != vt for o in outs):
        raise TypeError("batch entries must share storage types")
    for g, o in zip(geoms, outs):
        _prep(o, g, g.vol_shape, "out")
    hs = (ctypes.c_void_p * n)(*[g.handle for g in geoms])
    with torch.cuda.device(geoms[0].device):
        _check(_lib.cbct_batch_adjoint(n, hs, _ptrs(sinos), _ptrs(outs), st, vt,
                                       _stream(geoms[0].device)), "cbct_batch_adjoint")
    return outs


# ---- BLAS-1 (cbct_solve.h) -------------------------------------------------

def _f32(t: torch.Tensor, what: str):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous float32 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _f64cell(t: torch.Tensor, what: str):
    if not (t.is_cuda and t.dtype == torch.float64 and t.numel() >= 1):
        raise ValueError(f"{what} must be a float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def dot_workspace(n: int, device) -> torch.Tensor:
    return torch.empty(int(_lib.cbct_dot_workspace(n)), dtype=torch.float64, device=device)


def dot(a: torch.Tensor, b: torch.Tensor, ws: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """out[0] = sum(a*b) in FP64, deterministic; a, b float32; out float64 cell."""
    if a.numel() != b.numel():
        raise ValueError("size mismatch")
    _check(_lib.cbct_dot(a.numel(), _f32(a, "a"), _f32(b, "b"), _f64cell(ws, "ws"),
                         _f64cell(out, "out"), _stream(a.device)), "cbct_dot")
    return out


def dot_noalloc(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """As dot(), with the library's fixed per-device partial-sum array
    instead of a workspace (the call allocates nothing)."""
    if a.numel() != b.numel():
        raise ValueError("size mismatch")
    _check(_lib.cbct_dot_noalloc(a.numel(), _f32(a, "a"), _f32(b, "b"), _f64cell(out, "out"),
                                 _stream(a.device)), "cbct_dot_noalloc")
    return out


def axpy_ratio(y, x, num, den, sign=1.0):
    """y += sign * (num/den) * x with device FP64 scalars."""
    if y.numel() != x.numel():
        raise ValueError("size mismatch")
    _check(_lib.cbct_axpy_ratio(y.numel(), _f32(y, "y"), _f32(x, "x"), _f64cell(num, "num"),
                                _f64cell(den, "den"), float(sign), _stream(y.device)),
           "cbct_axpy_ratio")
    return y


def xpay_ratio(y, x, num, den):
    """y = x + (num/den) * y with device FP64 scalars."""
    if y.numel() != x.numel():
        raise ValueError("size mismatch")
    _check(_lib.cbct_xpay_ratio(y.numel(), _f32(y, "y"), _f32(x, "x"), _f64cell(num, "num"),
                                _f64cell(den, "den"), _stream(y.device)), "cbct_xpay_ratio")
    return y


def axpby(z, alpha, x, beta, y):
    """z = alpha*x + beta*y (z may alias x or y)."""
    if not (z.numel() == x.numel() == y.numel()):
        raise ValueError("size mismatch")
    _check(_lib.cbct_axpby(z.numel(), _f32(z, "z"), float(alpha), _f32(x, "x"), float(beta),
                           _f32(y, "y"), _stream(z.device)), "cbct_axpby")
    return z


def wresid(g, w, x, t):
    """g = w * (x - t) elementwise."""
    if not (g.numel() == w.numel() == x.numel() == t.numel()):
        raise ValueError("size mismatch")
    _check(_lib.cbct_wresid(g.numel(), _f32(g, "g"), _f32(w, "w"), _f32(x, "x"), _f32(t, "t"),
                            _stream(g.device)), "cbct_wresid")
    return g


# ---- simulator (cbct_sim.h) ------------------------------------------------

def philox_blocks(n_blocks: int, seed: int, stream_id: int, device="cuda") -> torch.Tensor:
    """[n_blocks, 4] raw Philox4x32-10 words (as int32 bit patterns)."""
    out = torch.empty((n_blocks, 4), dtype=torch.int32, device=device)
    _check(_lib.cbct_philox_blocks(n_blocks, seed, stream_id, ctypes.c_void_p(out.data_ptr()),
                                   _stream(out.device)), "cbct_philox_blocks")
    return out


def sim_poisson_log(p: torch.Tensor, I0: float, seed: int, stream_id: int = 0,
                    out: torch.Tensor | None = None, counts: bool = False):
    """y = -log(min(max(Poisson(I0 exp(-p)), 1) / I0, 1)); returns y (and counts)."""
    if out is None:
        out = torch.empty_like(p)
    c = torch.empty(p.shape, dtype=torch.int64, device=p.device) if counts else None
    _check(_lib.cbct_sim_poisson_log(p.numel(), _f32(p, "p"), _f32(out, "out"),
                                     ctypes.c_void_p(c.data_ptr()) if c is not None else None,
                                     float(I0), seed, stream_id, _stream(p.device)),
           "cbct_sim_poisson_log")
    return (out, c) if counts else out


def water_bone(hu: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """[2, *hu.shape]: water and bone relative densities of a CT volume in HU
    (channel 0 rho_w, channel 1 rho_b), ready for a two-channel forward."""
    if out is None:
        out = torch.empty((2,) + tuple(hu.shape), dtype=torch.float32, device=hu.device)
    if out.shape[0] != 2 or out[0].numel() != hu.numel():
        raise ValueError("out must be [2, *hu.shape]")
    _check(_lib.cbct_water_bone(hu.numel(), _f32(hu, "hu"), _f32(out[0], "rho_w"),
                                _f32(out[1], "rho_b"), _stream(hu.device)), "cbct_water_bone")
    return out


def poly_bins():
    """(centres_keV, resp): the paper's ten energy bins and detector response."""
    import numpy as np
    c = np.zeros(32)
    r = np.zeros(32)
    n = ctypes.c_int32()
    _check(_lib.cbct_poly_bins(32, c.ctypes.data_as(ctypes.c_void_p),
                               r.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)), "cbct_poly_bins")
    return c[:n.value].copy(), r[:n.value].copy()


def sim_poly(pw: torch.Tensor, pb: torch.Tensor, mu_w, mu_b, resp, I0: torch.Tensor, seed: int,
             stream_id: int = 0, signal: bool = False, counts: bool = False):
    """Noisy polychromatic primary signal and its normalised negative log
    (cbct_sim_poly).  pw, pb: material line integrals (same shape, last two
    dims the panel); I0: [n_bins, nv, nu] float32; mu_w, mu_b, resp: n_bins
    host floats.  Returns y, plus the signal and/or the counts [n_bins, ...]
    when asked."""
    import numpy as np
    if pw.shape != pb.shape:
        raise ValueError("pw and pb differ in shape")
    nb = I0.shape[0]
    npix = I0[0].numel()
    tabs = [np.ascontiguousarray(t, dtype=np.float64).ravel() for t in (mu_w, mu_b, resp)]
    if any(t.size != nb for t in tabs):
        raise ValueError("tables must have one entry per bin")
    y = torch.empty_like(pw)
    sg = torch.empty_like(pw) if signal else None
    c = torch.empty((nb,) + tuple(pw.shape), dtype=torch.int64, device=pw.device) if counts else None
    _check(_lib.cbct_sim_poly(pw.numel(), npix, _f32(pw, "pw"), _f32(pb, "pb"), nb,
                              *[t.ctypes.data_as(ctypes.c_void_p) for t in tabs],
                              _f32(I0, "I0"), seed, stream_id, _f32(y, "y"),
                              ctypes.c_void_p(sg.data_ptr()) if sg is not None else None,
                              ctypes.c_void_p(c.data_ptr()) if c is not None else None,
                              _stream(pw.device)), "cbct_sim_poly")
    out = (y,) + ((sg,) if signal else ()) + ((c,) if counts else ())
    return out if len(out) > 1 else y


def sim_gaussian(clean: torch.Tensor, sigma: float, seed: int, stream_id: int = 0,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    if out is None:
        out = torch.empty_like(clean)
    _check(_lib.cbct_sim_gaussian(clean.numel(), _f32(clean, "clean"), _f32(out, "out"),
                                  float(sigma), seed, stream_id, _stream(clean.device)),
           "cbct_sim_gaussian")
    return out


# ---- 3x3x3 convolutions (cbct_nn.h) ----------------------------------------

def _bf16(t, what):
    if not (t.is_cuda and t.dtype == torch.bfloat16 and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous bfloat16 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _cf_list(ts, what):
    arr = (ctypes.c_void_p * max(1, len(ts)))()
    for i, t in enumerate(ts):
        arr[i] = _f32(t, f"{what}[{i}]").value
    return arr


def pack16(channels, out=None, scale=None) -> torch.Tensor:
    """Channel-last bf16 [S, 16] from up to 16 channel-first FP32 tensors of S
    elements each (remaining channels zero; optional per-channel scale)."""
    S = channels[0].numel()
    if any(c.numel() != S for c in channels) or len(channels) > 16:
        raise ValueError("channel sizes differ or more than 16 channels")
    if out is None:
        out = torch.empty((S, 16), dtype=torch.bfloat16, device=channels[0].device)
    sc = None
    if scale is not None:
        sc = (ctypes.c_float * len(channels))(*[float(v) for v in scale])
    _check(_lib.cbct_pack16(S, len(channels), _cf_list(channels, "channels"), sc,
                            _bf16(out, "out"), _stream(out.device)), "cbct_pack16")
    return out


def conv3(grid, x, w, bias=None, act=False, slope=0.01, mask=None, transpose_w=False,
          y_cl=None, y_cf=(), accumulate=False, alpha=1.0):
    """3x3x3 convolution on a (nz, ny, nx) grid of channel-last bf16 [S,16]
    activations with bf16 weights [27,16,16]; stores into y_cl (bf16 [S,16])
    and/or the channel-first FP32 tensors y_cf (see cbct_nn.h)."""
    nz, ny, nx = grid
    S = nz * ny * nx
    if x.shape != (S, 16) or w.shape != (27, 16, 16):
        raise ValueError("bad activation or weight shape")
    if mask is not None and mask.shape != (S, 16):
        raise ValueError("bad mask shape")
    if y_cl is not None and y_cl.shape != (S, 16):
        raise ValueError("bad output shape")
    if bias is not None and not (bias.numel() >= 16):
        raise ValueError("bias needs 16 entries")
    for t in y_cf:
        if t.numel() != S:
            raise ValueError("channel-first output of the wrong size")
    _check(_lib.cbct_conv3(nz, ny, nx, _bf16(x, "x"), _bf16(w, "w"), int(bool(transpose_w)),
                           _f32(bias, "bias") if bias is not None else None,
                           _bf16(mask, "mask") if mask is not None else None,
                           int(bool(act)), float(slope),
                           _bf16(y_cl, "y_cl") if y_cl is not None else None,
                           len(y_cf), _cf_list(list(y_cf), "y_cf"), int(bool(accumulate)),
                           float(alpha), _stream(x.device)), "cbct_conv3")
    return y_cl


def conv3_wgrad_workspace(S: int, device) -> torch.Tensor:
    return torch.empty(int(_lib.cbct_conv3_wgrad_workspace(S)), dtype=torch.float32, device=device)


def conv3_wgrad(grid, x, dy, dw, db, ws):
    """dw [27,16,16] FP32 and db [16] FP32 (or None) of a 3x3x3 convolution."""
    nz, ny, nx = grid
    S = nz * ny * nx
    if x.shape != (S, 16) or dy.shape != (S, 16) or dw.shape != (27, 16, 16):
        raise ValueError("bad shapes")
    _check(_lib.cbct_conv3_wgrad(nz, ny, nx, _bf16(x, "x"), _bf16(dy, "dy"), _f32(dw, "dw"),
                                 _f32(db, "db") if db is not None else None, _f32(ws, "ws"),
                                 _stream(x.device)), "cbct_conv3_wgrad")
    return dw, db


def conv3_weights(w: torch.Tensor) -> torch.Tensor:
    """bf16 [27,16,16] device weights from a [cout, cin, 3, 3, 3] tensor
    (cout, cin <= 16; tap t = 9 kz + 3 ky + kx; missing channels zero)."""
    co, ci = w.shape[0], w.shape[1]
    out = torch.zeros((27, 16, 16), dtype=torch.float32, device=w.device)
    out[:, :co, :ci] = w.detach().float().permute(2, 3, 4, 0, 1).reshape(27, co, ci)
    return out.to(torch.bfloat16).contiguous()


def conv1(channels, w, out, accumulate=False, alpha=1.0):
    """out (+)= w[:n] . channels + w[n] (1x1x1 convolution; w a device FP32
    tensor of n + 1 entries)."""
    n = len(channels)
    S = out.numel()
    if any(c.numel() != S for c in channels) or w.numel() < n + 1:
        raise ValueError("channel sizes differ or too few weights")
    _check(_lib.cbct_conv1(S, n, _cf_list(channels, "channels"), _f32(w, "w"), _f32(out, "out"),
                           int(bool(accumulate)), float(alpha), _stream(out.device)), "cbct_conv1")
    return out


def fov_fraction(g: dict):
    """Field-of-view tensor V [nz][ny][nx] (numpy float32), computed on the
    host by the library for geometry dict g."""
    import numpy as np
    h = ctypes.c_void_p()
    d, _keep = make_desc(g)
    _check(_lib.cbct_geom_create_host(ctypes.byref(d), ctypes.byref(h)), "cbct_geom_create_host")
    try:
        out = np.empty((g["nz"], g["ny"], g["nx"]), dtype=np.float32)
        _check(_lib.cbct_fov_fraction(h, out.ctypes.data_as(ctypes.c_void_p)), "cbct_fov_fraction")
    finally:
        _lib.cbct_geom_destroy(h)
    return out


# ---- resolution changes (multiscale scheme) ---------------------------------

def _fine_dims(t, r):
    if t.dim() != 3 or any(d % r for d in t.shape):
        raise ValueError("need a 3-D tensor with sizes divisible by r")
    return tuple(int(d) for d in t.shape)


def pool(x, r, out=None, scale=None):
    """Block sums over r^3 blocks times scale (default 1/r^3: average pooling)."""
    n0, n1, n2 = _fine_dims(x, r)
    if out is None:
        out = torch.empty((n0 // r, n1 // r, n2 // r), dtype=torch.float32, device=x.device)
    sc = 1.0 / r ** 3 if scale is None else scale
    _check(_lib.cbct_pool(r, n0, n1, n2, _f32(x, "in"), _f32(out, "out"), float(sc),
                          _stream(x.device)), "cbct_pool")
    return out


def projdown(y, r, out=None, scale=None):
    """Every r-th projection, r x r pixel blocks summed times scale (default
    1/r^2: averaged)."""
    n0, n1, n2 = _fine_dims(y, r)
    if out is None:
        out = torch.empty((n0 // r, n1 // r, n2 // r), dtype=torch.float32, device=y.device)
    sc = 1.0 / r ** 2 if scale is None else scale
    _check(_lib.cbct_projdown(r, n0, n1, n2, _f32(y, "in"), _f32(out, "out"), float(sc),
                              _stream(y.device)), "cbct_projdown")
    return out


def upsample(c, r, out=None, scale=1.0, accumulate=False):
    """Nearest upsampling by r times scale into out (or added to it)."""
    if out is None:
        out = torch.empty(tuple(int(d) * r for d in c.shape), dtype=torch.float32,
                          device=c.device)
    n0, n1, n2 = _fine_dims(out, r)
    if tuple(c.shape) != (n0 // r, n1 // r, n2 // r):
        raise ValueError("coarse and fine shapes do not match")
    _check(_lib.cbct_upsample(r, n0, n1, n2, _f32(c, "in"), _f32(out, "out"), float(scale),
                              int(bool(accumulate)), _stream(c.device)), "cbct_upsample")
    return out


def fdk(geom: Geometry, sino: torch.Tensor, out: torch.Tensor | None = None,
        work: torch.Tensor | None = None, window: str = "ramlak") -> torch.Tensor:
    """FDK reconstruction with offset-detector redundancy weights (FP32);
    window "ramlak" or "hann"."""
    win = {"ramlak": 0, "hann": 1}[window]
    if tuple(sino.shape) != tuple(geom.sino_shape):
        raise ValueError("sinogram shape does not match the geometry")
    if out is None:
        out = torch.empty(geom.vol_shape, dtype=torch.float32, device=sino.device)
    if work is None:
        work = torch.empty(geom.sino_shape, dtype=torch.float32, device=sino.device)
    with torch.cuda.device(geom.device):
        _check(_lib.cbct_fdk(geom.handle, _f32(sino, "sino"), win, _f32(work, "work"),
                             _f32(out, "out"), _stream(geom.device)), "cbct_fdk")
    return out


# ---- peak probes (diagnostics) ----------------------------------------------

def probe_threads() -> int:
    return int(_lib.cbct_probe_threads())


def probe_valu(n_blocks: int, iters: int, out: torch.Tensor):
    """Launch the FMA-issue probe (8 FMA chains per thread, iters steps);
    out: float32 CUDA tensor of n_blocks * probe_threads() elements.
    Lane FMAs = n_blocks * probe_threads() * iters * 8."""
    if out.numel() < n_blocks * probe_threads():
        raise ValueError("out too small")
    _check(_lib.cbct_probe_valu(int(n_blocks), int(iters), _f32(out, "out"),
                                _stream(out.device)), "cbct_probe_valu")


def probe_lds(n_blocks: int, iters: int, out: torch.Tensor):
    """Launch the LDS-read probe (four conflict-free 16-byte reads per
    thread and step); LDS bytes = n_blocks * probe_threads() * iters * 64."""
    if out.numel() < n_blocks * probe_threads():
        raise ValueError("out too small")
    _check(_lib.cbct_probe_lds(int(n_blocks), int(iters), _f32(out, "out"),
                               _stream(out.device)), "cbct_probe_lds")


# ---- scatter simulator (cbct_scatter.h) --------------------------------------

class _Xs(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int), ("e0", ctypes.c_double), ("de", ctypes.c_double),
                ("mu", ctypes.c_void_p), ("J", ctypes.c_int), ("icdf", ctypes.c_void_p),
                ("I", ctypes.c_int), ("dens", ctypes.c_void_p)]


class ScatterTables:
    """Cross-section tables of the scatter model, uploaded once (cbct_xs):
    xs = dict(e0, de, mu [2, 3, K], icdf [2, 2, K, J], dens [2, 2, K, I])."""

    def __init__(self, xs: dict, device="cuda"):
        import numpy as np
        f = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device=device).contiguous()
        self.mu, self.icdf, self.dens = f(xs["mu"]), f(xs["icdf"]), f(xs["dens"])
        K = self.mu.shape[-1]
        if self.mu.shape != (2, 3, K) or self.icdf.shape[:3] != (2, 2, K) or \
                self.dens.shape[:3] != (2, 2, K):
            raise ValueError("scatter tables have the wrong shapes")
        self.s = _Xs(K, float(xs["e0"]), float(xs["de"]), self.mu.data_ptr(),
                     self.icdf.shape[3], self.icdf.data_ptr(), self.dens.shape[3],
                     self.dens.data_ptr())


def scatter_paths(geom: Geometry, rho: torch.Tensor, xs: ScatterTables, angle: int,
                  src: torch.Tensor, qmc: torch.Tensor, n_scatter: int,
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """SamplePath (Alg. 2): records [N, n_scatter + 1, 8] of the photons src
    [N, 4] with quasi-random points qmc [N, 5 n_scatter + 1] at projection
    `angle`; rho = [2, nz, ny, nx] water and bone densities."""
    if tuple(rho.shape) != (2,) + geom.vol_shape:
        raise ValueError("rho must be [2, nz, ny, nx]")
    N = src.shape[0]
    if tuple(src.shape) != (N, 4) or tuple(qmc.shape) != (N, 5 * n_scatter + 1):
        raise ValueError("src must be [N, 4] and qmc [N, 5 n + 1]")
    if out is None:
        out = torch.empty((N, n_scatter + 1, 8), dtype=torch.float32, device=src.device)
    with torch.cuda.device(geom.device):
        _check(_lib.cbct_scatter_paths(geom.handle, _f32(rho, "rho"), ctypes.byref(xs.s),
                                       int(angle), N, _f32(src, "src"), _f32(qmc, "qmc"),
                                       int(n_scatter), _f32(out, "rec"), _stream(geom.device)),
               "cbct_scatter_paths")
    return out


def scatter_integrate(geom: Geometry, rho: torch.Tensor, xs: ScatterTables, angle: int,
                      rec: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Integrate (Alg. 3): the scatter image [nv, nu] of the records rec
    [..., 8] on geom's panel at projection `angle` (before I_Sigma / |Src|)."""
    if tuple(rho.shape) != (2,) + geom.vol_shape:
        raise ValueError("rho must be [2, nz, ny, nx]")
    if rec.shape[-1] != 8:
        raise ValueError("records have 8 values")
    if out is None:
        out = torch.empty(geom.sino_shape[1:], dtype=torch.float32, device=rec.device)
    with torch.cuda.device(geom.device):
        _check(_lib.cbct_scatter_integrate(geom.handle, _f32(rho, "rho"), ctypes.byref(xs.s),
                                           int(angle), rec.numel() // 8, _f32(rec, "rec"),
                                           _f32(out, "out"), _stream(geom.device)),
               "cbct_scatter_integrate")
    return out
