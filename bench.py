#!/usr/bin/env python3
"""Benchmark of the PXST reconstruction loop on one MI355X.

One step = one full main-loop solve of the realistic scan (256 x 1024 detector,
121 frames, +-10 px window with paraboloid refinement, 5 iterations and a final
reference update) starting from the same initial map, with the inputs resident in
HBM.  The headline value is pixel-map candidate evaluations (good pixels x window
candidates x frames, summed over the iterations) per second of whole-solve time.

Also reported: the dominant kernel's (interior-tile pixel-map search) roofline
fraction from HIP events around its launches inside the timed region, the FP64
oracle timed on host cores on a sampled subset of the same workload, the divergent
scan (512 x 512, 400 frames, translation update on) and per-solve latencies.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pixel-map candidate evals/s (pixels×shifts×frames); p50/p99 solve latency"
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz for non-packed float32
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12      # 78.6
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PEAK_INT8_MFMA_TOPS = 5000.0   # dense int8 matrix-core peak
PEAK_FP64_TFLOPS = 78.6        # float64 (vector and matrix)
FLOP_PER_EVAL = 4   # r = I - W g (1 FMA) and E += r^2 (1 FMA)


def pm_source_hash() -> str:
    """Hash of the pixel-map search's code (comments and blank space left out, so that
    an edited comment keeps the counters taken on the same code)."""
    import re
    h = hashlib.sha256()
    for f in ("pxst_pixel_map.hip", "pxst_device.hpp", "pxst_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2003_12726_amd", "csrc", f), encoding="utf-8") as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they were taken
    on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "pm_fast_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    ent = d.get(workload)
    if not ent or ent.get("source_hash") != pm_source_hash():
        return None
    return ent


def _counter_rows(d: str):
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, counter):
    """Counter value per dispatch (summed over the dimensions rocprofv3 reports)."""
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        ent = per.setdefault(key, [r["Kernel_Name"], int(r["Grid_Size"]), 0.0])
        ent[2] += float(r["Counter_Value"])
    return list(per.values())


def write_traffic(fetch_dir: str, write_dir: str, copy_mib: int):
    """HBM bytes per launch of the interior-tile pixel-map search from FETCH_SIZE /
    WRITE_SIZE (KiB per dispatch),
    each scaled by what the same counter reads for a device-to-device copy of known
    size in the same run (copy_mib MiB read and written)."""
    if copy_mib <= 0:
        raise SystemExit("--copy-calibration-mib must give the calibration copy's size")
    nb = copy_mib << 20
    res = {}
    for name, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        disp = _per_dispatch(_counter_rows(d), counter)
        pm = [v for k, g, v in disp if ("k_pm_mma_" in k and "edge" not in k) or "k_pm_fast" in k]
        cp = [v for k, g, v in disp if "copyBuffer" in k or "copy" in k.lower()]
        if not pm or not cp:
            raise SystemExit(f"{counter}: pixel-map dispatches {len(pm)}, copy dispatches {len(cp)}")
        copy_kib = max(cp)
        factor = (nb / 1024.0) / copy_kib
        kib = sum(pm) / len(pm)
        res[name] = {"kib_per_dispatch_raw": kib, "dispatches": len(pm),
                     "copy_kib_raw": copy_kib, "factor": factor, "bytes": kib * 1024.0 * factor}
    p = os.path.join(ROOT, "profiles", "pm_fast_traffic.json")
    d = {}
    if os.path.exists(p):
        with open(p) as fh:
            d = json.load(fh)
    d["realistic"] = {"source_hash": pm_source_hash(), "copy_mib": copy_mib,
                      "fetch": res["fetch"], "write": res["write"],
                      "bytes_per_launch": res["fetch"]["bytes"] + res["write"]["bytes"]}
    with open(p, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d["realistic"], indent=1))
    print(kernel_traffic_table(fetch_dir, write_dir, copy_mib))


def kernel_traffic_table(fetch_dir: str, write_dir: str, copy_mib: int) -> str:
    """Markdown table of every kernel's HBM bytes per dispatch in the two counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by the calibration copy's reading)."""
    import re
    nb = copy_mib << 20
    per = {}
    for d, counter in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        disp = _per_dispatch(_counter_rows(d), counter)
        cp = [v for k, g, v in disp if "copyBuffer" in k or "copy" in k.lower()]
        factor = (nb / 1024.0) / max(cp)
        for k, g, v in disp:
            name = re.sub(r"\(anonymous namespace\)::", "", k)
            name = re.sub(r"\(.*", "", name).replace("void ", "").replace("pxst::", "").strip()
            ent = per.setdefault(name, {"FETCH_SIZE": [], "WRITE_SIZE": []})
            ent[counter].append(v * 1024.0 * factor)
    rows = ["| kernel | dispatches | fetch MB / dispatch | write MB / dispatch |", "|---|---|---|---|"]
    for name, ent in sorted(per.items(), key=lambda kv: -sum(kv[1]["FETCH_SIZE"] + kv[1]["WRITE_SIZE"])):
        f, w = ent["FETCH_SIZE"], ent["WRITE_SIZE"]
        fm = sum(f) / len(f) / 1e6 if f else float("nan")
        wm = sum(w) / len(w) / 1e6 if w else float("nan")
        rows.append(f"| `{name}` | {max(len(f), len(w))} | {fm:.2f} | {wm:.2f} |")
    return "\n".join(rows)


def roofline(int8_ops_per_launch, avg_ms, launches, evals_per_launch, achieved_tflops, traffic):
    """Roofline of the dominant kernel, the interior-tile pixel-map search, on the basis of
    the method's own arithmetic: 4 flop per candidate evaluation (r = I - W g and E += r^2,
    two FMAs) times the evaluations one launch covers, over the launch's average duration,
    against the float32 vector peak (157.3 TFLOP/s).  The kernel reaches that work through
    an exact int8 contraction on the matrix cores; what it issues there (2 ops per int8
    multiply-add, six byte pairs per frame, padded regions and frames) is reported beside it
    against the dense int8 peak."""
    out = {"kernel": "pixel-map search, interior tiles (k_pm_mma_half_planes_lds on the realistic scan: "
                     "int8 matrix cores)",
           "bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_PACKED_TFLOPS, "unit": "TFLOP/s",
           "frac": achieved_tflops / PEAK_FP32_PACKED_TFLOPS if achieved_tflops else None,
           "traffic": traffic["bytes_per_launch"] if traffic else None,
           "basis": "4 flop per candidate evaluation (pixels x candidates x frames of the launch's tiles) "
                    "/ average launch time (HIP events on the launch stream) / float32 vector peak",
           "flop_per_eval": FLOP_PER_EVAL, "evals_per_launch": evals_per_launch,
           "avg_launch_ms": avg_ms, "launches": launches}
    if int8_ops_per_launch and avg_ms:
        ops = int8_ops_per_launch
        tops = ops / (avg_ms * 1e-3) / 1e12
        out["int8_mfma"] = {"achieved_tops": tops, "peak_tops": PEAK_INT8_MFMA_TOPS,
                            "frac": tops / PEAK_INT8_MFMA_TOPS, "int8_ops_per_launch": ops}
    return out


# --------------------------------------------------------------------- oracle leg
_ORC = {}


def _oracle_worker(args):
    rows, cols = args
    import numpy as np  # noqa: F401
    import oracle
    s = _ORC["scan"]
    t = time.perf_counter()
    oracle.update_pixel_map(s.frames, s.white, s.mask, _ORC["ref"], _ORC["w"], s.dx0, s.u0, s.origin,
                            s.window, s.refine, pixels=(rows, cols))
    return time.perf_counter() - t


def cpu_baseline(scan, n_workers: int, px_per_worker: int):
    """FP64 oracle pixel-map update on sampled pixels of the same scan, one process per
    host core; returns evals/s of the wall time."""
    import numpy as np
    _ORC["scan"] = scan
    _ORC["ref"] = scan.ref_true
    _ORC["w"] = np.ones_like(scan.ref_true)
    rng = np.random.default_rng(7)
    H, W = scan.det
    jobs = [(rng.integers(0, H, px_per_worker), rng.integers(0, W, px_per_worker))
            for _ in range(n_workers)]
    rx, ry = scan.window
    evals = n_workers * px_per_worker * (2 * rx + 1) * (2 * ry + 1) * scan.n_frames
    ctx = mp.get_context("fork")
    t = time.perf_counter()
    with ctx.Pool(n_workers) as pool:
        per = pool.map(_oracle_worker, jobs)
        pool.close()
        pool.join()    # every worker has exited before the GPU is touched
    wall = time.perf_counter() - t
    return {
        "value": evals / wall,
        "unit": "evals/s",
        "cores": n_workers,
        "kind": "oracle",
        "sample": (f"FP64 NumPy oracle pixel-map update of {n_workers * px_per_worker} sampled pixels "
                   f"of the realistic scan (all {(2 * rx + 1) * (2 * ry + 1)} candidates x "
                   f"{scan.n_frames} frames, refinement on), {n_workers} processes x "
                   f"{px_per_worker} pixels, wall {wall:.1f} s"),
        "single_core_evals_per_s": (px_per_worker * (2 * rx + 1) * (2 * ry + 1) * scan.n_frames
                                    / (sum(per) / len(per))),
    }


# ---------------------------------------------------------------- served stream
def _gen_job(args):
    k, spec, arrival = args
    from synth import make_scan
    s = make_scan(spec)
    return (k, arrival, s.frames, s.white, s.mask, s.u0, s.dx0, tuple(s.ref_shape), tuple(s.origin),
            s.iters, tuple(s.window))


def served_requests(n_jobs: int, workers: int, seed: int = 5000):
    """The served stream's jobs (Poisson arrivals, mean gap 0.5 s), generated in parallel."""
    from synth import served_job_specs
    specs, gaps = served_job_specs(n_jobs, seed=seed)
    arrivals = [float(x) for x in __import__("numpy").cumsum(gaps)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        rows = pool.map(_gen_job, [(k, specs[k], arrivals[k]) for k in range(n_jobs)], chunksize=1)
        pool.close()
        pool.join()
    return rows


def run_served(rows, time_scale: float):
    from paper_2003_12726_amd import serve
    reqs = [serve.Request(job_id=k, arrival=arr, frames=f, white=w, mask=m, u0=u, dx0=d, ref_shape=rs,
                          origin=o, n_iter=it, window=win, refine=True)
            for (k, arr, f, w, m, u, d, rs, o, it, win) in rows]
    evals = sum(r.pm_evals() for r in reqs)
    out = {}
    for mode in ("one_by_one", "batched", "batched_srpt", "batched_all"):
        print(f"[served] {len(reqs)} jobs replayed {time_scale:g}x, {mode}", file=sys.stderr, flush=True)
        if mode != "one_by_one":
            srv = serve.Server(budget_bytes=200 << 30, max_slots=64, keep_results=False,
                               policy={"batched": "aged", "batched_srpt": "srpt", "batched_all": "all"}[mode])
            res = srv.run(reqs, time_scale=time_scale)
        else:
            res = serve.run_one_by_one(reqs, time_scale=time_scale, keep_results=False)
        first = min(r.arrival for r in res.values())
        last = max(r.finished for r in res.values())
        st = serve.latency_stats(res)
        st["pm_evals_per_s"] = evals / (last - first)
        st["makespan_s"] = last - first
        if mode != "one_by_one":
            st["ticks"] = srv.ticks
            st["max_resident"] = srv.max_resident
        out[mode] = st
    out["workload"] = (f"{len(reqs)} jobs, Poisson arrivals (mean 2 jobs/s) replayed {time_scale:g}x "
                       f"faster, detectors from 128x128 to 512x512, 16-400 frames, windows +-4..15 px, "
                       f"5 iterations, HBM budget 200 GB")
    out["pm_evals_total"] = evals
    return out


# ------------------------------------------------------------------------ GPU leg
class Job:
    """A scan resident on the GPU with its state, workspace and initial map."""

    def __init__(self, scan, dev, n_iter=None):
        import numpy as np
        import torch
        import paper_2003_12726_amd as pxst
        self.s = scan
        self.pxst = pxst
        f16 = scan.frames.view(np.int16)
        self.scan = pxst.Scan(torch.from_numpy(f16).to(dev), torch.from_numpy(scan.white).to(dev),
                              torch.from_numpy(scan.mask).to(dev), scan.ref_shape, scan.origin)
        self.n_iter = scan.iters if n_iter is None else n_iter
        self.opts = pxst.make_opts(self.n_iter, scan.window, scan.refine, scan.update_dx,
                                   scan.tr_window, True)
        self.u0 = torch.from_numpy(scan.u0).to(dev)
        self.dx0 = torch.from_numpy(scan.dx0).to(dev)
        self.u = torch.empty_like(self.u0)
        self.dx = torch.empty_like(self.dx0)
        self.ref = torch.empty(scan.ref_shape, dtype=torch.float32, device=dev)
        self.wsum = torch.empty(scan.ref_shape, dtype=torch.float64, device=dev)
        self.hist = torch.zeros(max(self.n_iter, 1), dtype=torch.float64, device=dev)
        self.ws = pxst.alloc_workspace(self.scan.geom, self.opts, dev)

    def step(self):
        self.u.copy_(self.u0)
        self.dx.copy_(self.dx0)
        self.pxst.solve(self.scan, self.opts, self.u, self.dx, self.ref, self.wsum, self.hist, self.ws)

    def pm_evals(self):
        return self.s.pm_evals() * self.n_iter


def time_steps(job, steps, warmup):
    import torch
    for _ in range(warmup):
        job.step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        job.step()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = sorted(a.elapsed_time(b) for a, b in evs)
    return wall, lat


def regularisation_bench(scan, dev, reps: int = 10, sigma: float = 5.0):
    """Pixel-map regularisation of the realistic map: Gaussian filter (sigma 5) then the
    irrotational constraint, timed per family with HIP events."""
    import torch
    import paper_2003_12726_amd as pxst
    H, W = scan.det
    g = pxst.make_geom(scan.n_frames, scan.det, scan.ref_shape, scan.origin)
    ws = pxst.alloc_workspace(g, pxst.make_opts(1, scan.window, integrate=True), device=dev)
    u = torch.from_numpy(scan.u0).to(dev)
    v = torch.empty_like(u)
    for _ in range(2):
        pxst.regularise_pixel_map(g, u, v, sigma, True, ws)
    torch.cuda.synchronize()
    pxst.profile_enable(True)
    for fam in ("reg_filter", "reg_integrate"):
        pxst.profile_read(fam)
    t0 = time.perf_counter()
    for _ in range(reps):
        pxst.regularise_pixel_map(g, u, v, sigma, True, ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    f_ms, f_n, f_work = pxst.profile_read("reg_filter")
    i_ms, i_n, i_work = pxst.profile_read("reg_integrate")
    pxst.profile_enable(False)
    HW = H * W
    f_avg, i_avg = f_ms / max(f_n, 1), i_ms / max(i_n, 1)
    # algorithmic bytes of the two filter passes: float32 map in, float64 intermediate
    # out and back in, float32 map out
    f_bytes = 2 * HW * (4 + 8) * 2
    i_flops = i_work / max(i_n, 1)
    return {
        "workload": f"{H}x{W} map, Gaussian filter sigma {sigma:g} then least-squares integration",
        "ms_per_call": 1000.0 * wall / reps,
        "filter_ms": f_avg,
        "filter_GBps": f_bytes / (f_avg * 1e-3) / 1e9 if f_n else None,
        "integrate_ms": i_avg,
        "integrate_fp64_TFLOPs": i_flops / (i_avg * 1e-3) / 1e12 if i_n else None,
        "integrate_fp64_frac": (i_flops / (i_avg * 1e-3) / 1e12) / PEAK_FP64_TFLOPS if i_n else None,
    }


def fractional_bench(scan, dev, reps: int = 3, steps: int = 3):
    """Fractional-step pixel-map search of the realistic scan (window +-10 px, 1/3 px
    grid: 63 x 63 candidates per pixel) with the true reference, timed with HIP events."""
    import numpy as np
    import torch
    import paper_2003_12726_amd as pxst
    H, W = scan.det
    f16 = scan.frames.view(np.int16)
    sc = pxst.Scan(torch.from_numpy(f16).to(dev), torch.from_numpy(scan.white).to(dev),
                   torch.from_numpy(scan.mask).to(dev), scan.ref_shape, scan.origin)
    ws = pxst.alloc_workspace(sc.geom, pxst.make_opts(1, scan.window), device=dev)
    ref = torch.from_numpy(scan.ref_true.astype(np.float32)).to(dev)
    wsum = torch.ones(scan.ref_shape, dtype=torch.float64, device=dev)
    dx = torch.from_numpy(scan.dx0).to(dev)
    u = torch.from_numpy(scan.u0).to(dev)
    uo = torch.empty_like(u)
    win = pxst.make_window(scan.window[0], scan.window[1], False)
    pxst.update_pixel_map_fractional(sc, ref, wsum, dx, u, win, steps, uo, None, None, ws)
    torch.cuda.synchronize()
    pxst.profile_enable(True)
    pxst.profile_read("pm_frac")
    for _ in range(reps):
        pxst.update_pixel_map_fractional(sc, ref, wsum, dx, u, win, steps, uo, None, None, ws)
    torch.cuda.synchronize()
    ms, n, _ = pxst.profile_read("pm_frac")
    pxst.profile_enable(False)
    h = (steps - 1) // 2
    nc = (2 * (scan.window[0] * steps + h) + 1) * (2 * (scan.window[1] * steps + h) + 1)
    evals = int((scan.mask > 0).sum()) * nc * scan.n_frames
    avg = ms / max(n, 1)
    return {"workload": f"{H}x{W}, {scan.n_frames} frames, window +-{scan.window[0]} px on a 1/{steps} px "
                        f"grid ({nc} candidates per pixel), true reference",
            "ms_per_search": avg, "evals_per_s": evals / (avg * 1e-3) if n else None}


def split_half_bench(scan, dev, reps: int = 2):
    """Split-half analysis of the realistic scan (window +-10 px with refinement, random
    halves of the (frame, pixel) terms, 64-bin histograms), timed with HIP events."""
    import numpy as np
    import torch
    import paper_2003_12726_amd as pxst
    H, W = scan.det
    f16 = scan.frames.view(np.int16)
    sc = pxst.Scan(torch.from_numpy(f16).to(dev), torch.from_numpy(scan.white).to(dev),
                   torch.from_numpy(scan.mask).to(dev), scan.ref_shape, scan.origin)
    ws = pxst.alloc_workspace(sc.geom, pxst.make_opts(1, scan.window), device=dev)
    ref = torch.from_numpy(scan.ref_true.astype(np.float32)).to(dev)
    wsum = torch.ones(scan.ref_shape, dtype=torch.float64, device=dev)
    dx = torch.from_numpy(scan.dx0).to(dev)
    u = torch.from_numpy(scan.u0).to(dev)
    half = torch.from_numpy(np.random.default_rng(5).integers(0, 2, scan.frames.shape).astype(np.uint8)).to(dev)
    ua, ub = torch.empty_like(u), torch.empty_like(u)
    hist = torch.empty((2, 64), dtype=torch.int32, device=dev)
    win = pxst.make_window(scan.window[0], scan.window[1], True)
    pxst.split_half_pixel_map(sc, ref, wsum, dx, u, win, half, ua, ub, 1.0, 64, hist, ws)
    torch.cuda.synchronize()
    pxst.profile_enable(True)
    pxst.profile_read("pm_split")
    for _ in range(reps):
        pxst.split_half_pixel_map(sc, ref, wsum, dx, u, win, half, ua, ub, 1.0, 64, hist, ws)
    torch.cuda.synchronize()
    ms, n, _ = pxst.profile_read("pm_split")
    pxst.profile_enable(False)
    nc = (2 * scan.window[0] + 1) * (2 * scan.window[1] + 1)
    evals = int((scan.mask > 0).sum()) * nc * scan.n_frames   # both halves together
    avg = ms / max(n, 1)
    return {"workload": f"{H}x{W}, {scan.n_frames} frames split at random per (frame, pixel), "
                        f"window +-{scan.window[0]} px with refinement, 64-bin histograms",
            "ms_per_analysis": avg, "evals_per_s": evals / (avg * 1e-3) if n else None}


def defocus_bench(scan, dev):
    """Defocus-by-registration sweep of the realistic scan: 5 x 5 per-axis map scales
    around 1 (reference update and contrast per candidate), timed with HIP events."""
    import numpy as np
    import torch
    import paper_2003_12726_amd as pxst
    H, W = scan.det
    f16 = scan.frames.view(np.int16)
    sc = pxst.Scan(torch.from_numpy(f16).to(dev), torch.from_numpy(scan.white).to(dev),
                   torch.from_numpy(scan.mask).to(dev), scan.ref_shape, scan.origin)
    ws = pxst.alloc_workspace(sc.geom, None, device=dev)
    dx = torch.from_numpy(scan.dx0).to(dev)
    scales = np.array([(a, b) for a in (0.98, 0.99, 1.0, 1.01, 1.02) for b in (0.98, 0.99, 1.0, 1.01, 1.02)],
                      dtype=np.float32)
    c = torch.empty(len(scales), dtype=torch.float64, device=dev)
    best = torch.empty(1, dtype=torch.int32, device=dev)
    pxst.defocus_sweep(sc, dx, scales[:2], c, best, None, ws)
    torch.cuda.synchronize()
    pxst.profile_enable(True)
    pxst.profile_read("defocus_sweep")
    pxst.defocus_sweep(sc, dx, scales, c, best, None, ws)
    torch.cuda.synchronize()
    ms, n, _ = pxst.profile_read("defocus_sweep")
    pxst.profile_enable(False)
    return {"workload": f"{H}x{W}, {scan.n_frames} frames, 25 candidate map scales (5 x 5 around 1)",
            "ms_per_sweep": ms, "ms_per_candidate": ms / len(scales),
            "best_scale": [float(x) for x in scales[int(best.cpu().numpy()[0])]]}


def precision_study(scan, dev, reps: int = 4):
    """The precision study on the realistic scan: for each reference-update arithmetic of
    the library (exact -- terms on a power-of-two grid summed exactly in 64-bit integers,
    the default and the stand-in for an FP64 update; fp32 -- float32 numerator with
    compensated sums; bf16 -- the exact update stored in bfloat16), one reference update,
    one pixel-map update and one translation update (+-2 px) from the start state
    (u0, dx0), compared with the FP64 oracle's results of the same steps stored in
    tests/golden/precision_realistic.npz (written by the oracle alone), and the full
    solve's time with that arithmetic."""
    import numpy as np
    import torch
    import paper_2003_12726_amd as pxst
    g = np.load(os.path.join(ROOT, "tests", "golden", "precision_realistic.npz"))
    H, W = scan.det
    f16 = scan.frames.view(np.int16)
    sc = pxst.Scan(torch.from_numpy(f16).to(dev), torch.from_numpy(scan.white).to(dev),
                   torch.from_numpy(scan.mask).to(dev), scan.ref_shape, scan.origin)
    base = pxst.make_opts(scan.iters, scan.window, scan.refine, scan.update_dx, scan.tr_window)
    ws = pxst.alloc_workspace(sc.geom, base, device=dev)
    u0 = torch.from_numpy(scan.u0).to(dev)
    dx0 = torch.from_numpy(scan.dx0).to(dev)
    rows, cols = g["rows"], g["cols"]
    frames = [int(x) for x in g["frames"]]

    def stats(x):
        x = np.abs(np.asarray(x, dtype=np.float64).ravel())
        return {"max": float(x.max()), "p99": float(np.percentile(x, 99))} if x.size else None

    out = {"workload": "realistic scan, one step of each kind from (u0, dx0): the reference at 8192 "
                       "well-covered pixels, the map at 400 sampled pixels, translations of 6 frames; "
                       "the full solve per arithmetic", "modes": {}}
    for mode in ("exact", "fp32", "bf16"):
        ref = torch.empty(scan.ref_shape, dtype=torch.float32, device=dev)
        w = torch.empty(scan.ref_shape, dtype=torch.float64, device=dev)
        pxst.update_reference(sc, u0, dx0, ref, w, ws, mode=mode)
        u1 = torch.empty_like(u0)
        kg = torch.empty((H, W), dtype=torch.int32, device=dev)
        pxst.update_pixel_map(sc, ref, w, dx0, u0, pxst.make_window(scan.window[0], scan.window[1], scan.refine),
                              u1, None, kg, ws)
        dx1 = torch.empty_like(dx0)
        pxst.update_translations(sc, ref, w, u0, dx0, pxst.make_window(2, 2, True), dx1, None, None, ws)
        torch.cuda.synchronize()
        rg = ref.cpu().numpy().ravel()[g["ref_index"]].astype(np.float64)
        rel = np.abs(rg - g["ref_value"]) / np.maximum(np.abs(g["ref_value"]), 1e-30)
        ug = u1.cpu().numpy()[:, rows, cols]
        kgs = kg.cpu().numpy()[rows, cols]
        ko = g["argmin"]
        fin = (ko >= 0) & (kgs >= 0)
        same = fin & (kgs == ko)
        ties = 0
        for p in np.nonzero(fin & ~same)[0]:
            hit = np.nonzero(g["top_index"][p] == kgs[p])[0]
            eo = g["top_error"][p, 0]
            if hit.size and abs(g["top_error"][p, hit[0]] - eo) <= 1e-6 * abs(eo):
                ties += 1
        du = np.abs(ug[:, same] - g["u"][:, same]).max(axis=0)
        ddx = np.abs(dx1.cpu().numpy()[frames] - g["dx"]).max(axis=1)
        o = pxst.make_opts(scan.iters, scan.window, scan.refine, scan.update_dx, scan.tr_window, ref_mode=mode)
        hist = torch.zeros(max(scan.iters, 1), dtype=torch.float64, device=dev)
        times = []
        for rep in range(reps + 1):
            u = u0.clone()
            dx = dx0.clone()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            pxst.solve(sc, o, u, dx, ref, w, hist, ws)
            b.record()
            torch.cuda.synchronize()
            if rep:
                times.append(a.elapsed_time(b))
        ms = float(np.median(times))
        out["modes"][mode] = {
            "ref_rel": stats(rel), "ref_max_abs_over_scale": float(np.abs(rg - g["ref_value"]).max() / g["ref_scale"]),
            "u_px": stats(du), "argmin_equal": int(same.sum()), "argmin_ties": int(ties),
            "argmin_other": int((fin & ~same).sum() - ties), "pixels": int(fin.sum()),
            "dx_px": stats(ddx), "solve_ms": ms,
            "pm_evals_per_s": scan.pm_evals() * scan.iters / (ms * 1e-3)}
    return out


def pct(xs, q):
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[k]


def served_study(n_jobs: int, seeds, rates, workers: int):
    """The served stream over several arrival seeds, at each replay rate (1 = the real
    arrival rate): latency p50 / p99 / max and throughput, batched and one by one."""
    import torch
    import paper_2003_12726_amd as pxst
    streams = []
    # the generator forks worker processes: every stream is made before this process
    # loads the HIP library or touches the GPU
    for seed in seeds:
        print(f"[served] generating stream seed {seed}", file=sys.stderr, flush=True)
        streams.append((seed, served_requests(n_jobs, workers, seed)))
    pxst.load_library()
    runs = []
    for seed, rows in streams:
        for rate in rates:
            r = run_served(rows, rate)
            r["seed"] = seed
            r["replay_rate"] = rate
            runs.append(r)
            torch.cuda.empty_cache()
    table = []
    for r in runs:
        for mode in ("one_by_one", "batched", "batched_srpt", "batched_all"):
            st = r[mode]
            table.append({"seed": r["seed"], "replay_rate": r["replay_rate"], "mode": mode,
                          "p50_s": st["p50_s"], "p99_s": st["p99_s"], "max_s": st["max_s"],
                          "pm_evals_per_s": st["pm_evals_per_s"], "makespan_s": st["makespan_s"]})
    return {"workload": runs[0]["workload"].split(" replayed")[0] if runs else None, "runs": table}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-divergent", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the regularisation, fractional, split-half and defocus sections")
    ap.add_argument("--section", choices=["precision_study", "regularisation", "fractional_search", "split_half",
                                          "defocus_sweep"],
                    help="profiling aid: run only this extras section on the realistic scan and print its JSON")
    ap.add_argument("--divergent-only", action="store_true",
                    help="profiling aid: time only the divergent scan's solve and print its line")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--served-jobs", type=int, default=64)
    ap.add_argument("--served-speedup", type=float, default=50.0)
    ap.add_argument("--served-study", nargs="*", type=int, metavar="SEED",
                    help="only the served stream: these arrival seeds (default 5000 6000 7000), "
                         "each replayed at the rates of --served-rates; prints one JSON line")
    ap.add_argument("--served-rates", nargs="+", type=float, default=[1.0, 50.0])
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="end with one device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU: turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--copy-calibration-mib run into profiles/pm_fast_traffic.json")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(*args.traffic_from, copy_mib=args.copy_calibration_mib)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the reconstruction of one scan runs on one device "
              f"(--gpus {args.gpus} is not supported; multi-GPU sharding is not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2003_12726_amd as pxst
    from synth.scans import cached_scan

    if args.served_study is not None:
        seeds = args.served_study or [5000, 6000, 7000]
        print(json.dumps(served_study(args.served_jobs, seeds, args.served_rates,
                                      args.cpu_workers or min(16, os.cpu_count() or 1))), flush=True)
        return

    if args.section:
        pxst.load_library()
        fn = {"precision_study": precision_study, "regularisation": regularisation_bench,
              "fractional_search": fractional_bench, "split_half": split_half_bench,
              "defocus_sweep": defocus_bench}[args.section]
        print(json.dumps({args.section: fn(cached_scan("realistic"), torch.device("cuda:0"))}), flush=True)
        return

    if args.divergent_only:
        pxst.load_library()
        dev = torch.device("cuda:0")
        d = cached_scan("divergent")
        dj = Job(d, dev)
        dwall, _ = time_steps(dj, args.steps, args.warmup)
        print(json.dumps({"workload": "divergent: 512x512, 400 frames, window +-15 x +-3 px, 8 iterations, "
                                      "translation update +-2 px on",
                          "ms_per_solve": 1000.0 * dwall / args.steps,
                          "pm_evals_per_s": dj.pm_evals() / (dwall / args.steps)}), flush=True)
        return

    scan = cached_scan("realistic")
    # the oracle leg forks worker processes: run it before this process loads the HIP
    # library or touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        nw = args.cpu_workers or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(scan, nw, 3072)
    served_rows = None
    if args.served_jobs > 0:
        served_rows = served_requests(args.served_jobs, args.cpu_workers or min(16, os.cpu_count() or 1))
    pxst.load_library()
    dev = torch.device("cuda:0")
    job = Job(scan, dev)

    # Timed region: HIP events around the dominant kernel's launches only (each event
    # record holds the stream for a few microseconds, so the other families are timed in
    # a pass of their own below).
    pxst.profile_enable(True)
    pxst.profile_select(["pm_fast"])
    # warm-up outside the profiled window
    for _ in range(args.warmup):
        job.step()
    torch.cuda.synchronize()
    pxst.profile_read("pm_fast")
    wall, lat = time_steps(job, args.steps, 0)
    f_ms, f_n, _ = pxst.profile_read("pm_fast")
    # Breakdown pass (after the timed region, same steps): every family with its device
    # work counters.  Each step solves from the same initial state, so the work per
    # launch is that of the timed steps.
    fams = ("pm_fast", "pm_fast_int8_ops", "pm_edge", "pm_edge_mma", "pm_generic", "pm_planes",
            "ref_gather", "err_pixels")
    pxst.profile_select(None)
    for fam in fams:
        pxst.profile_read(fam)
    bsteps = max(1, min(args.steps, 3))
    for _ in range(bsteps):
        job.step()
    torch.cuda.synchronize()
    kern = {fam: pxst.profile_read(fam) for fam in fams}
    pxst.profile_enable(False)
    mm = kern.pop("pm_fast_int8_ops")

    ms_per_step = 1000.0 * wall / args.steps
    evals_per_step = job.pm_evals()
    value = evals_per_step / (wall / args.steps)

    avg_ms = f_ms / max(f_n, 1)
    evals_per_launch = kern["pm_fast"][2] / max(kern["pm_fast"][1], 1)
    achieved_tflops = FLOP_PER_EVAL * evals_per_launch / (avg_ms * 1e-3) / 1e12 if f_n else None
    int8_ops_per_launch = mm[2] / mm[1] if mm[1] else None
    pm_total_ms = sum(kern[k][0] for k in ("pm_fast", "pm_edge", "pm_edge_mma", "pm_generic"))
    pm_total_evals = sum(kern[k][2] for k in ("pm_fast", "pm_edge", "pm_edge_mma", "pm_generic"))
    traffic = load_traffic("realistic")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8 MFMA: uint16 counts x 22-bit fixed-point reference, FP64 combine; FP32 elsewhere",
        "data": "synthetic (seeded scan shaped like the realistic workload)",
        "config": {
            "workload": "realistic: 256x1024 uint16 detector, 121 frames (11x11 grid, 8 px step), "
                        "reference 512x1536, window +-10 px (441 candidates) with 3x3 refinement, "
                        "5 iterations + final reference update",
            "pm_evals_per_step": evals_per_step,
            "parallelism": "single GPU",
        },
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": lat[-1],
                       "kind": "one full solve per job, jobs run one by one"},
        "roofline": roofline(int8_ops_per_launch, avg_ms, f_n, evals_per_launch, achieved_tflops, traffic),
        "kernels_ms_per_step": {k: v[0] / bsteps for k, v in kern.items()},
        "kernels_ms_per_step_basis": f"HIP events around every family's launches in {bsteps} steps "
                                     "after the timed region",
        "pixel_map_only_evals_per_s": pm_total_evals / (pm_total_ms * 1e-3) if pm_total_ms else None,
    }

    if not args.no_divergent:
        del job
        torch.cuda.empty_cache()
        d = cached_scan("divergent")
        dj = Job(d, dev)
        dwall, dlat = time_steps(dj, max(2, args.steps // 3), 1)
        nst = max(2, args.steps // 3)
        out["divergent"] = {
            "workload": "divergent: 512x512, 400 frames, window +-15 x +-3 px, 8 iterations, "
                        "translation update +-2 px on",
            "ms_per_solve": 1000.0 * dwall / nst,
            "pm_evals_per_s": dj.pm_evals() / (dwall / nst),
            "pm_plus_tr_evals_per_s": (dj.pm_evals() + d.tr_evals() * dj.n_iter) / (dwall / nst),
        }
        del dj
        torch.cuda.empty_cache()

    if not args.no_extras:
        out["precision_study"] = precision_study(scan, dev)
        out["regularisation"] = regularisation_bench(scan, dev)
        out["fractional_search"] = fractional_bench(scan, dev)
        out["split_half"] = split_half_bench(scan, dev)
        out["defocus_sweep"] = defocus_bench(scan, dev)

    if served_rows is not None:
        torch.cuda.empty_cache()
        out["served"] = run_served(served_rows, args.served_speedup)
        latency = out["latency_ms"]
        latency["served_p50_s"] = out["served"]["batched"]["p50_s"]
        latency["served_p99_s"] = out["served"]["batched"]["p99_s"]

    if cpu is not None:
        out["cpu_baseline"] = cpu

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
