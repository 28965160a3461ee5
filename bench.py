"""Benchmark of the cone-beam projector pair on one MI355X.

One step = one forward projection A and one adjoint A^T of the clinical-size
case (256^3 volume at 2 mm, 360 angles over 2 pi, 512^2 panel at 0.8 mm with a
115 mm lateral offset, source-isocenter 1000 mm, source-panel 1536 mm) in
FP32, on a seeded synthetic phantom already resident in HBM.  Throughput is
(S_A + S_AT) / time in Gsamples/s, where S is the library's sample count
(ray-plane pairs with non-empty support; A^T applies the same samples).

Also measured (key "recon"): the metric's second half, seconds to a fixed
PSNR for the learned primal-dual net against CGLS on one held-out phantom
(see recon_comparison).

Prints one JSON line.  `--gpus N` with N > 1 exits: the benchmark runs on
one GPU only.

`--workload` selects another case for the same measurement (the default is
the clinical-size FP32 case above; the others skip the reconstruction
comparison and the CPU baseline):
  c2-bf16  the clinical-size case with BF16 volume and sinogram storage;
  c1       64^3 at 4 mm, 64 angles, 128^2 panel at 3.2 mm, FP32;
  c3       twelve heterogeneous cases (96^3..256^3, 2-4 mm, 90-360 angles,
           256^2..512^2 panels) in one batched launch per operator, BF16
           storage, FP32 accumulation;
  c4       a batch of four 128^3 volumes at 2 mm, 180 angles, 256^2 panel at
           1.6 mm with the 115 mm offset, FP32, one batched launch per operator.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A+A^T Gsamples/s at 256³×360×512²; recon s to fixed PSNR, learned vs CGLS"

# Algorithmic VALU lane-operations per sample (one bilinear sample on a
# voxel-centre plane, the unit of both operators):
#   2  FMAs for the in-plane and z fractional indices,
#   2  floors,
#   2  fraction subtractions,
#   6  three linear interpolations (subtract + FMA each),
#   1  FMA accumulating the sample into the ray (or voxel) sum,
#   2  integer operations forming the voxel address,
#   -- 15 in all.
OPS_PER_SAMPLE = 15
# Non-packed FP32 VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


# HBM traffic per launch of the projector kernels, from rocprofv3 FETCH_SIZE
# and WRITE_SIZE runs (each scaled by what the counter reads for a 512 MiB
# device copy), valid for the kernel sources whose hash it records.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "projector_c2_f32_hbm_traffic.json")
KERNEL_SOURCES = ("cbct_adjoint.hip", "cbct_forward.hip", "cbct_internal.h", "cbct_storage.h", "cbct_lds.h",
                  "cbct_transpose.h", "cbct_plan.cpp", "cbct_geom.cpp", "cbct_api.cpp", "cbct_scratch.cpp")
# The adjoint operator is two launches: the ds_weight pre-pass (projection
# values times each ray's length per plane) and the gather adjoint_brick.


def algorithmic_bytes(g):
    """Compulsory HBM bytes of one FP32 launch: the input read once and the
    output written once (volume and sinogram, 4 bytes per element)."""
    return 4 * (g["nx"] * g["ny"] * g["nz"] + g["n_angles"] * g["nv"] * g["nu"])


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_21180_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """Bytes per launch of `kernel` from the recorded counter runs, or None
    when there is no record or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else int(k["traffic_bytes"])


def record_traffic(fetch_csv, write_csv, fetch_cmd, write_cmd):
    """Write TRAFFIC_FILE from the counter_collection CSVs of a FETCH_SIZE and
    a WRITE_SIZE run made with --copy-calibration."""
    import csv

    def per_kernel(path, counter):
        out, copies = {}, []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"]
                key = ("copy" if "copyBuffer" in name else
                       "adjoint" if "adjoint_brick" in name else
                       "adjoint_pre" if "ds_weight" in name else
                       "forward" if "forward_sweep" in name else None)
                if key == "copy":
                    if int(r["Grid_Size"]) >= 4096:   # not the small staging copies
                        copies.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
                elif key:
                    out.setdefault(key, []).append(float(r["Counter_Value"]))
        # the calibration copies are the run's last two large copies
        out["copy"] = [v for _, v in sorted(copies)[-2:]]
        return out

    fe, wr = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy_kib = 512 * 1024
    ff = copy_kib / (sum(fe["copy"]) / len(fe["copy"]))
    fw = copy_kib / (sum(wr["copy"]) / len(wr["copy"]))
    rec = {"source_sha256": kernel_source_hash(), "command_fetch": fetch_cmd,
           "command_write": write_cmd, "copy_bytes": copy_kib * 1024,
           "copy_fetch_kib": fe["copy"], "copy_write_kib": wr["copy"],
           "fetch_factor": round(ff, 5), "write_factor": round(fw, 5), "kernels": {}}
    for k in ("adjoint", "adjoint_pre", "forward"):
        f_kib = sum(fe[k]) / len(fe[k]) * ff
        w_kib = sum(wr[k]) / len(wr[k]) * fw
        rec["kernels"][k] = {"fetch_kib": fe[k], "write_kib": wr[k],
                             "traffic_bytes": int(round((f_kib + w_kib) * 1024))}
    # the operator's traffic: pre-pass and gather together
    rec["kernels"]["adjoint_operator"] = {"traffic_bytes": rec["kernels"]["adjoint"]["traffic_bytes"]
                                          + rec["kernels"]["adjoint_pre"]["traffic_bytes"]}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def recon_comparison(seed=50_000):
    """Second half of the metric: seconds to a fixed PSNR, learned net vs
    CGLS, on one held-out phantom of the same case (Poisson I0 = 1e5).  The
    fixed PSNR is the best CGLS reaches in 50 iterations; both methods run on
    the same FP32 projector pair with the data in HBM, timed per iteration
    with HIP events.  Weights: the committed multiscale net (8 iterations,
    resolutions 1/4, 1/4, 1/4, 1/2, 1/2, 1/2, 1, 1, FDK start)."""
    from paper_2512_21180_amd import compare

    S = compare.Setup(compare.DEFAULT_WEIGHTS)
    r = compare.compare_one(S, seed, log=lambda m: print(m, file=sys.stderr, flush=True))
    return {
        "fixed_psnr_db": r["target_psnr_db"],
        "cgls_s": r["cgls_time_to_target_s"],
        "learned_s": r["learned_time_to_target_s"],
        "cgls_iterations": r["cgls_best_iter"],
        "learned_final_psnr_db": r["learned_psnr_db"][-1],
        "learned_total_s": r["learned_time_s"][-1],
        "blocks_zeroed_psnr_db": r["zero_block_psnr_db"][-1],
        "fdk_psnr_db": r["fdk_psnr_db"],
        "phantom_seed": seed,
        "net": {"iterations": S.net.n_iter, "scales": list(S.net.scales), "init": S.net.init},
    }


def _oracle_pair(orc, g, x, n_angles, threads):
    """Time the FP64 oracle's forward then scatter adjoint on g restricted to
    n_angles of its angles (every n/n_angles-th); returns (samples, tA, tAT)."""
    all_ang = orc.angles_of(g)
    step = max(1, g["n_angles"] // n_angles)
    sub = dict(g, n_angles=len(all_ang[::step][:n_angles]), angles=all_ang[::step][:n_angles])
    S = orc.sample_count(sub)
    t0 = time.perf_counter()
    y = orc.forward(sub, x, nthreads=threads)
    t1 = time.perf_counter()
    orc.adjoint(sub, y, nthreads=threads)
    t2 = time.perf_counter()
    return S, sub["n_angles"], t1 - t0, t2 - t1


def cpu_baseline(g, n_angles=72, n_angles_1t=6):
    """The FP64 oracle on the same geometry restricted to a subset of its
    angles, forward then adjoint: on all host threads (n_angles angles) and
    on one thread (n_angles_1t angles)."""
    from oracle import oracle as orc
    from paper_2512_21180_amd import workloads as W

    x, _, _ = W.phantom_c2(g, 2025)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    S, na, tA, tAT = _oracle_pair(orc, g, x, n_angles, threads)
    S1, na1, tA1, tAT1 = _oracle_pair(orc, g, x, n_angles_1t, 1)
    return {
        "value": round(2 * S / (tA + tAT) / 1e9, 4),
        "unit": "Gsamples/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"FP64 oracle A then scatter A^T on the same case restricted to {na} "
                  f"of its {g['n_angles']} angles ({S} samples each); forward {tA:.1f} s, "
                  f"adjoint {tAT:.1f} s",
        "single_thread": {
            "value": round(2 * S1 / (tA1 + tAT1) / 1e9, 4),
            "unit": "Gsamples/s",
            "cores": 1,
            "sample": f"the same on {na1} of the {g['n_angles']} angles ({S1} samples each); "
                      f"forward {tA1:.1f} s, adjoint {tAT1:.1f} s",
        },
    }


def copy_bandwidth(reps=5):
    """Achievable HBM bandwidth: a 1 GiB device-to-device copy (read + write
    bytes over the HIP-event time, mean of reps), far larger than the caches."""
    import torch
    src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    bw = 2 * src.numel() * 4 / t
    del src, dst
    torch.cuda.empty_cache()
    return bw


def gather_bound(S, elem_bytes, tA, tAT, bw):
    """Fraction of the gather-bound HBM rate: every sample reads four voxels
    (A) or four panel values (A^T) of elem_bytes each; F_g = those bytes per
    second over the measured device-copy bandwidth (above 1 when staging and
    caches serve the gathers)."""
    b = S * 4 * elem_bytes
    return {
        "F_g": round(2 * b / (tA + tAT) / bw, 3),
        "F_g_forward": round(b / tA / bw, 3),
        "F_g_adjoint": round(b / tAT / bw, 3),
        "gather_bytes_per_operator": b,
        "copy_bw_TBps": round(bw / 1e12, 3),
    }


WORKLOADS = {
    "c2-bf16": "256^3 @2 mm volume, 360 angles over 2 pi, 512^2 panel @0.8 mm, 115 mm lateral "
               "offset; 50-ellipsoid phantom in a 300 mm body cylinder; BF16 volume and sinogram "
               "storage, FP32 accumulation; A + A^T",
    "c1": "64^3 @4 mm volume, 64 angles over 2 pi, 128^2 panel @3.2 mm, no offset; 1-10 "
          "ellipsoids; FP32 A + A^T",
    "c3": "12 heterogeneous cases (96^3..256^3 at 2-4 mm, 90-360 angles, 256^2..512^2 panels, "
          "half with the 115 mm offset) in one batched launch per operator; BF16 storage, FP32 "
          "accumulation; A + A^T",
    "c4": "batch of 4 volumes 128^3 @2 mm, 180 angles over 2 pi, 256^2 panel @1.6 mm, 115 mm "
          "lateral offset, one batched launch per operator; FP32 A + A^T",
}


def secondary_workload(name, steps, warmup):
    """Time A and A^T on one of the other cases.  Single cases go through
    cbct_forward/cbct_adjoint, batches through cbct_batch_forward/adjoint (one
    launch per operator).  Throughput is 2 x the summed sample counts over the
    wall time of the timed steps; the roofline is that of the slower operator,
    as for the default case."""
    import torch
    from paper_2512_21180_amd import cbct
    from paper_2512_21180_amd import workloads as W

    if name in ("c2-bf16", "c1"):
        g = W.C2 if name == "c2-bf16" else W.C1
        x_host = W.phantom_c2(g, 2025)[0] if name == "c2-bf16" else W.phantom_c1(g, 0)[0]
        dt = torch.bfloat16 if name == "c2-bf16" else torch.float32
        geos, vols = [cbct.Geometry(g)], [torch.tensor(x_host, device="cuda").to(dt)]
        dtype = "bf16" if name == "c2-bf16" else "f32"
    elif name == "c3":
        gs = W.c3_geometries()
        geos = [cbct.Geometry(g) for g in gs]
        vols = [torch.tensor(W.phantom_c3(g, 1000 + i)[0], device="cuda").to(torch.bfloat16)
                for i, g in enumerate(gs)]
        dt, dtype = torch.bfloat16, "bf16"
    else:
        geo = cbct.Geometry(W.C4)
        geos = [geo] * 4
        vols = [torch.tensor(W.phantom_c1(W.C4, 4000 + i)[0], device="cuda").to(torch.float32)
                for i in range(4)]
        dt, dtype = torch.float32, "f32"
    S = sum(g.sample_count() for g in geos)
    sinos = [torch.empty(g.sino_shape, dtype=dt, device="cuda") for g in geos]
    backs = [torch.empty(g.vol_shape, dtype=dt, device="cuda") for g in geos]

    def fwd():
        if len(geos) == 1:
            cbct.forward(geos[0], vols[0], out=sinos[0])
        else:
            cbct.batch_forward(geos, vols, outs=sinos)

    def adj():
        if len(geos) == 1:
            cbct.adjoint(geos[0], sinos[0], out=backs[0])
        else:
            cbct.batch_adjoint(geos, sinos, outs=backs)

    for _ in range(warmup):
        fwd()
        adj()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        fwd()
        ev[k][1].record()
        adj()
        ev[k][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tA = sum(e[0].elapsed_time(e[1]) for e in ev) / steps * 1e-3
    tAT = sum(e[1].elapsed_time(e[2]) for e in ev) / steps * 1e-3
    dom, tdom = ("adjoint", tAT) if tAT >= tA else ("forward", tA)
    if len(geos) > 1:
        dom += "_batch"
    achieved = OPS_PER_SAMPLE * S / tdom / 1e12
    elem = 2 if dtype == "bf16" else 4
    bw = copy_bandwidth()
    return {
        "metric": "A+A^T Gsamples/s",
        "value": round(2 * S * steps / wall / 1e9, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(wall / steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": WORKLOADS[name], "cases": len(geos),
                   "samples_per_operator": S},
        "kernels": {
            "forward_ms": round(tA * 1e3, 3),
            "adjoint_ms": round(tAT * 1e3, 3),
            "forward_gsamples_s": round(S / tA / 1e9, 2),
            "adjoint_gsamples_s": round(S / tAT / 1e9, 2),
        },
        "roofline": {
            "bound": "alu",
            "kernel": dom,
            "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 3),
            "unit": "TOP/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": None,
            "algorithmic_bytes": sum(elem * (math.prod(g.vol_shape) + math.prod(g.sino_shape))
                                     for g in geos),
        },
        "gather_bound": gather_bound(S, elem, tA, tAT, bw),
    }


def measure_peaks():
    """Measured ceilings of the three resources, next to the published ones:
    FP32 FMA issue (lane-operations/s, 8 independent chains per thread on
    8 workgroups per CU), conflict-free LDS reads (bytes/s) and a 1 GiB
    device-to-device copy (read + write bytes/s)."""
    import torch
    from paper_2512_21180_amd import cbct

    nb, th = 256 * 8, cbct.probe_threads()
    out = torch.empty(nb * th, dtype=torch.float32, device="cuda")

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    it_v, it_l = 20000, 5000
    t_v = timed(lambda: cbct.probe_valu(nb, it_v, out))
    t_l = timed(lambda: cbct.probe_lds(nb, it_l, out))
    src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    t_c = timed(lambda: dst.copy_(src))
    valu = nb * th * it_v * 8 / t_v / 1e12
    lds = nb * th * it_l * 64 / t_l / 1e12
    hbm = 2 * src.numel() * 4 / t_c / 1e12
    return {
        "valu_fma": {"measured": round(valu, 2), "published": round(VALU_PEAK_TOPS, 2),
                     "unit": "T lane-ops/s", "frac_of_published": round(valu / VALU_PEAK_TOPS, 3)},
        "lds_read": {"measured": round(lds, 2), "unit": "TB/s",
                     "per_cu_bytes_per_clock": round(lds * 1e12 / 256 / 2.4e9, 1)},
        "hbm_copy": {"measured": round(hbm, 2), "published": 8.0, "unit": "TB/s",
                     "frac_of_published": round(hbm / 8.0, 3)},
    }


CONV_GRIDS = {
    "volume 256^3": (256, 256, 256),
    "sinogram stack 360x512^2 (r=1)": (360, 512, 512),
    "sinogram stack 90x128^2 (r=4)": (90, 128, 128),
}


def measure_convs(reps=5):
    """HIP-event times of the learned blocks' 3x3x3 convolution kernels at the
    net's real grids (16 -> 16 channels, BF16 operands, FP32 accumulation):
    the forward (bias + LeakyReLU, BF16 channel-last store), the data
    gradient (transposed weights + LeakyReLU-derivative mask) and the weight
    gradient.  FLOP = 2 x 27 x 16 x 16 per position for each kernel; the
    HBM bytes are the compulsory ones (BF16 x 16 channels read once per
    operand, written once)."""
    import torch
    from paper_2512_21180_amd import cbct

    gen = torch.Generator("cuda").manual_seed(0)
    res = {}
    for name, grid in CONV_GRIDS.items():
        S = grid[0] * grid[1] * grid[2]
        x = torch.randn((S, 16), device="cuda", generator=gen).to(torch.bfloat16)
        m = torch.randn((S, 16), device="cuda", generator=gen).to(torch.bfloat16)
        w = (0.1 * torch.randn((27, 16, 16), device="cuda", generator=gen)).to(torch.bfloat16)
        b = torch.zeros(16, device="cuda")
        y = torch.empty((S, 16), dtype=torch.bfloat16, device="cuda")
        dw = torch.empty((27, 16, 16), device="cuda")
        db = torch.empty(16, device="cuda")
        ws = cbct.conv3_wgrad_workspace(S, "cuda")
        runs = {
            "conv3": (lambda: cbct.conv3(grid, x, w, bias=b, act=True, y_cl=y), 4 * 16 * S),
            "conv3_transposed_masked": (
                lambda: cbct.conv3(grid, x, w, mask=m, transpose_w=True, y_cl=y), 6 * 16 * S),
            "wgrad": (lambda: cbct.conv3_wgrad(grid, x, m, dw, db, ws), 4 * 16 * S),
        }
        out = {}
        for k, (fn, hbm) in runs.items():
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / reps * 1e-3
            flop = 2 * 27 * 256 * S
            out[k] = {"ms": round(t * 1e3, 3), "tflops": round(flop / t / 1e12, 1),
                      "frac_mfma_bf16": round(flop / t / 2.5e15, 4),
                      "compulsory_hbm_TBps": round(hbm / t / 1e12, 3)}
        res[name] = {"positions": S, **out}
        print(json.dumps({name: res[name]}), file=sys.stderr, flush=True)
        del x, m, y, ws
        torch.cuda.empty_cache()
    return res


def measure_simulators(reps=3):
    """HIP-event times of the two projection-data simulators beyond the
    monochromatic one, at the clinical geometry with synthetic tables:

    * polychromatic primary (NEXT-3): water/bone densities of a 256^3 HU
      phantom, their two line integrals in one two-channel forward projection
      (360 angles, 512^2 panel), and the ten-bin Poisson signal with its
      normalised log; the Poisson kernel reads two FP32 line integrals and
      writes y per element (12 B; the bin maps stay in the caches);
    * scatter (NEXT-4) for one projection: path sampling of 4096 source
      photons with two scatters each, and integration of the 3 x 4096 records
      toward a 128^2 panel at 3.2 mm (a quarter of the primary resolution),
      one march per record and pixel."""
    import numpy as np
    import torch
    from paper_2512_21180_amd import cbct, simulate
    from paper_2512_21180_amd import workloads as W

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    g = W.C2
    geo = cbct.Geometry(g)
    hu = torch.tensor(W.hu_phantom(g, 2025), device="cuda")
    c, resp = cbct.poly_bins()
    mw, mb = W.poly_tables(c)
    I0 = torch.tensor(W.intensity_maps(g, c), device="cuda")
    rho = cbct.water_bone(hu)
    p = cbct.forward(geo, rho)
    t_wb = timed(lambda: cbct.water_bone(hu, out=rho))
    t_fw = timed(lambda: cbct.forward(geo, rho, out=p))
    t_po = timed(lambda: cbct.sim_poly(p[0], p[1], mw, mb, resp, I0, 7, 0))
    n_el = p[0].numel()
    poly = {"water_bone_ms": round(t_wb * 1e3, 3), "forward_2ch_ms": round(t_fw * 1e3, 3),
            "poisson_10_bins_ms": round(t_po * 1e3, 3),
            "poisson_elements_per_s": round(n_el / t_po, 1),
            "poisson_hbm_TBps": round(12 * n_el / t_po / 1e12, 3),
            "total_ms": round((t_wb + t_fw + t_po) * 1e3, 3)}
    print(json.dumps({"poly": poly}), file=sys.stderr, flush=True)
    del p, I0
    torch.cuda.empty_cache()

    gs = W.geometry(360, 128, 128, 3.2, 3.2, 256, 256, 256, 2.0, off_u=115.0)
    geos = cbct.Geometry(gs)
    xs = cbct.ScatterTables(W.scatter_tables(), "cuda")
    N, n = 4096, 2
    src = torch.tensor(W.scatter_sources(N, gs, 11).astype(np.float32), device="cuda")
    qmc = torch.tensor(W.sobol_points(N, 5 * n + 1).astype(np.float32), device="cuda")
    rec = cbct.scatter_paths(geos, rho, xs, 0, src, qmc, n)
    img = cbct.scatter_integrate(geos, rho, xs, 0, rec)
    t_pa = timed(lambda: cbct.scatter_paths(geos, rho, xs, 0, src, qmc, n, out=rec))
    t_in = timed(lambda: cbct.scatter_integrate(geos, rho, xs, 0, rec, out=img))
    scat = {"photons": N, "scatters": n, "panel": [128, 128],
            "paths_ms": round(t_pa * 1e3, 3), "integrate_ms": round(t_in * 1e3, 3),
            "record_pixel_pairs_per_s": round(N * (n + 1) * 128 * 128 / t_in, 1)}
    print(json.dumps({"scatter": scat}), file=sys.stderr, flush=True)
    return {"poly_primary_c2": poly, "scatter_one_projection": scat}


def measure_channels(reps=5):
    """HIP-event times of channel stacks at the clinical geometry (FP32):
    five single-channel forward calls against one five-channel stack (the
    dual block's input of Alg. 1 at full resolution), through cbct_forward
    on a [5, ...] tensor and through cbct_batch_forward on five cases of one
    geometry (the learned net's call), and the same for 2, 3 and 4 channels;
    likewise at the half- and quarter-resolution geometries of the net."""
    import torch
    from paper_2512_21180_amd import cbct
    from paper_2512_21180_amd import workloads as W
    from paper_2512_21180_amd.learned import scaled_geometry

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    res = {}
    for r in (1, 2, 4):
        g = scaled_geometry(W.C2, r)
        geo = cbct.Geometry(g)
        x = torch.stack([torch.tensor(W.random_volume(g, 40 + c), device="cuda")
                         for c in range(5)]).float()
        y = torch.empty((5,) + geo.sino_shape, device="cuda")
        row = {}
        for C in (2, 3, 4, 5):
            t1 = timed(lambda: [cbct.forward(geo, x[c], out=y[c]) for c in range(C)])
            ts = timed(lambda: cbct.forward(geo, x[:C], out=y[:C]))
            tb = timed(lambda: cbct.batch_forward([geo] * C, [x[c] for c in range(C)],
                                                  outs=[y[c] for c in range(C)]))
            row[f"C{C}"] = {"single_ms": round(t1 * 1e3, 3), "stack_ms": round(ts * 1e3, 3),
                            "batch_ms": round(tb * 1e3, 3), "ratio": round(ts / t1, 3)}
        res[f"r{r}"] = row
        print(json.dumps({f"r{r}": row}), file=sys.stderr, flush=True)
        del x, y
        torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sims", action="store_true",
                    help="time the polychromatic primary and the scatter simulators instead")
    ap.add_argument("--channels", action="store_true",
                    help="time five-channel forward stacks against single channels instead")
    ap.add_argument("--convs", action="store_true",
                    help="time the learned blocks' convolution kernels at the net's grids instead")
    ap.add_argument("--peaks", action="store_true",
                    help="measure FMA issue, LDS read and device-copy rates instead")
    ap.add_argument("--workload", default="c2", choices=("c2", "c2-bf16", "c1", "c3", "c4"),
                    help="case to time (default: the clinical-size FP32 case)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recon", action="store_true",
                    help="skip the reconstruction comparison (learned net vs CGLS)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 512 MiB device-to-device copy (for counter calibration)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic record from two counter runs and exit (no GPU use)")
    args = ap.parse_args()
    if args.record_traffic:
        cmd = ("timeout -s KILL 120 rocprofv3 --pmc {c} -f csv -d {d} -o run -- python3 -u "
               "bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-recon --copy-calibration")
        f_csv, w_csv = args.record_traffic
        rec = record_traffic(f_csv, w_csv,
                             cmd.format(c="FETCH_SIZE", d=os.path.dirname(f_csv)),
                             cmd.format(c="WRITE_SIZE", d=os.path.dirname(w_csv)))
        print(json.dumps({k: v["traffic_bytes"] for k, v in rec["kernels"].items()}))
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on a single GPU; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_21180_amd import cbct
    from paper_2512_21180_amd import workloads as W

    torch.cuda.set_device(0)
    if args.peaks:
        print(json.dumps(measure_peaks()), flush=True)
        return
    if args.sims:
        print(json.dumps(measure_simulators()), flush=True)
        return
    if args.convs:
        print(json.dumps(measure_convs()), flush=True)
        return
    if args.channels:
        print(json.dumps(measure_channels()), flush=True)
        return
    if args.workload != "c2":
        print(json.dumps(secondary_workload(args.workload, args.steps, args.warmup)), flush=True)
        return
    g = W.C2
    geo = cbct.Geometry(g)
    S = geo.sample_count()
    x_host, _, _ = W.phantom_c2(g, 2025)
    x = torch.tensor(x_host, dtype=torch.float32, device="cuda")
    y = torch.empty(geo.sino_shape, dtype=torch.float32, device="cuda")
    xb = torch.empty(geo.vol_shape, dtype=torch.float32, device="cuda")

    for _ in range(args.warmup):
        cbct.forward(geo, x, out=y)
        cbct.adjoint(geo, y, out=xb)
    torch.cuda.synchronize()

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        ev[k][0].record()
        cbct.forward(geo, x, out=y)
        ev[k][1].record()
        cbct.adjoint(geo, y, out=xb)
        ev[k][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    tA = sum(e[0].elapsed_time(e[1]) for e in ev) / K * 1e-3
    tAT = sum(e[1].elapsed_time(e[2]) for e in ev) / K * 1e-3
    value = 2 * S * K / wall / 1e9
    dom, tdom = ("adjoint", tAT) if tAT >= tA else ("forward", tA)
    achieved = OPS_PER_SAMPLE * S / tdom / 1e12
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "256^3 @2 mm volume, 360 angles over 2 pi, 512^2 panel @0.8 mm, "
                        "115 mm lateral offset, sid 1000 / sdd 1536 mm; 50-ellipsoid phantom "
                        "in a 300 mm body cylinder; FP32 A + A^T",
            "samples_per_operator": S,
        },
        "kernels": {
            "forward_ms": round(tA * 1e3, 3),
            "adjoint_ms": round(tAT * 1e3, 3),
            "forward_gsamples_s": round(S / tA / 1e9, 2),
            "adjoint_gsamples_s": round(S / tAT / 1e9, 2),
        },
        "roofline": {
            "bound": "alu",
            # the adjoint is timed as its two launches, pre-pass and gather
            "kernel": "adjoint (ds_weight + adjoint_brick)" if dom == "adjoint" else dom,
            "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 3),
            "unit": "TOP/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": measured_traffic("adjoint_operator" if dom == "adjoint" else dom),
            "algorithmic_bytes": algorithmic_bytes(g),
        },
        # (counter runs with --copy-calibration leave out the bandwidth copies,
        # so that the calibration copies are the only large ones)
        "gather_bound": None if args.copy_calibration else
        gather_bound(S, 4, tA, tAT, copy_bandwidth()),
    }
    if args.copy_calibration:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_recon:
        out["recon"] = recon_comparison()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
