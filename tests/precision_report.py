"""Precision study and parity statistics of the GPU path against the FP64 oracle.

Run on a machine with the GPU (it is not collected by pytest):

    python -u tests/precision_report.py [--configs tiny realistic divergent]
                                        [--modes exact fp32 bf16] [--json OUT]

For every scan and reference-update arithmetic ("exact": quantised terms summed
exactly in FP64, stored as float32 -- the default; "fp32": float32 numerator with
compensated sums; "bf16": the exact update rounded to bfloat16), starting from the
scan's initial state (u0, dx0):

* I_ref: one reference update, the whole reference against the oracle's: per-pixel
  relative error |dI| / |I| over pixels with weight > 1e-3 median (max, p99), and the
  acceptance metric max |dI| / max |I|;
* u: one pixel-map update of the whole detector with that reference; the oracle
  updates sampled pixels with its own reference; |du| in px (max, p99) and the
  argmin agreement (a different index is a tie when the oracle's errors at both
  indices differ by < 1e-6 relative);
* dx: one translation update (+-2 px, refined) with that reference and u0; the
  oracle updates sampled frames: |d dx| in px (max, p99);
* throughput: the scan's full solve with that arithmetic (ms and pixel-map candidate
  evaluations per second).

Prints a markdown table.  The errors of the default arithmetic are the parity
statistics of the GPU path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import paper_2003_12726_amd as pxst  # noqa: E402
from gpu_util import ARGMIN_TIE_REL, dev_scan, empty, ref_rel_error, to_dev  # noqa: E402
from oracle import pxst_oracle as oracle  # noqa: E402
from synth.scans import cached_scan  # noqa: E402

SAMPLES = {"tiny": (None, None), "realistic": (400, [0, 30, 60, 61, 90, 120]),
           "divergent": (120, [0, 187, 399])}


def say(msg):
    print(msg, flush=True)


def stats(x):
    x = np.abs(np.asarray(x, dtype=np.float64).ravel())
    x = x[np.isfinite(x)]
    if x.size == 0:
        return {"max": None, "p99": None, "n": 0}
    return {"max": float(x.max()), "p99": float(np.percentile(x, 99)), "n": int(x.size)}


def sample_pixels(s, n, seed=7):
    H, W = s.det
    if n is None:
        r, c = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        return r.ravel(), c.ravel()
    rng = np.random.default_rng(seed)
    return rng.integers(0, H, n), rng.integers(0, W, n)


def run_config(name, modes, torch):
    s = cached_scan(name)
    npx, frames = SAMPLES[name]
    frames = list(range(s.n_frames)) if frames is None else frames
    rows, cols = sample_pixels(s, npx)
    say(f"[{name}] oracle reference ({s.n_frames} frames, {s.det[0]}x{s.det[1]})")
    ro, wo = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    say(f"[{name}] oracle pixel map ({rows.size} pixels)")
    uo, eo, ko, Eo = oracle.update_pixel_map(s.frames, s.white, s.mask, ro, wo, s.dx0, s.u0, s.origin,
                                             s.window, refine=s.refine, pixels=(rows, cols),
                                             return_errors=True)
    say(f"[{name}] oracle translations ({len(frames)} frames)")
    dxo, _, _ = oracle.update_translations(s.frames[frames], s.white, s.mask, ro, wo, s.u0,
                                           s.dx0[frames], s.origin, (2, 2), refine=True)
    sc = dev_scan(s)
    opts = pxst.make_opts(s.iters, s.window, s.refine, s.update_dx, s.tr_window)
    ws = pxst.alloc_workspace(sc.geom, opts)
    H, W = s.det
    out = {}
    for mode in modes:
        say(f"[{name}] GPU, reference arithmetic {mode}")
        ref = empty(s.ref_shape, torch.float32)
        w = empty(s.ref_shape, torch.float64)
        u0, dx0 = to_dev(s.u0), to_dev(s.dx0)
        pxst.update_reference(sc, u0, dx0, ref, w, ws, mode=mode)
        u1 = empty((2, H, W), torch.float32)
        kg = empty((H, W), torch.int32)
        pxst.update_pixel_map(sc, ref, w, dx0, u0, pxst.make_window(s.window[0], s.window[1], s.refine),
                              u1, None, kg, ws)
        dx1 = empty((s.n_frames, 2), torch.float32)
        pxst.update_translations(sc, ref, w, u0, dx0, pxst.make_window(2, 2, True), dx1, None, None, ws)
        torch.cuda.synchronize()
        rg, wg = ref.cpu().numpy(), w.cpu().numpy()
        ug, kgn, dxg = u1.cpu().numpy(), kg.cpu().numpy(), dx1.cpu().numpy()
        thr = 1e-3 * np.median(wo[wo > 0])
        sel = wo > thr
        rel = np.abs(rg[sel].astype(np.float64) - ro[sel]) / np.maximum(np.abs(ro[sel]), 1e-30)
        acc, _ = ref_rel_error(rg, ro, wo)
        # pixel map at the sampled pixels
        ugs = ug[:, rows, cols]
        kgs = kgn[rows, cols]
        fin = (ko >= 0) & (kgs >= 0)
        same = fin & (kgs == ko)
        ties = 0
        Ef = Eo.reshape(-1, Eo.shape[-1]) if Eo is not None else None
        good_col = np.cumsum(s.mask[rows, cols] > 0) - 1
        for p in np.nonzero(fin & (kgs != ko))[0]:
            eg, e_o = Ef[kgs[p], good_col[p]], Ef[ko[p], good_col[p]]
            if np.isfinite(eg) and np.isfinite(e_o) and abs(eg - e_o) <= ARGMIN_TIE_REL * abs(e_o):
                ties += 1
        du = np.abs(ugs[:, same] - uo[:, same]).max(axis=0) if same.any() else np.zeros(0)
        ddx = np.abs(dxg[frames] - dxo).max(axis=1)
        # throughput of the full solve
        u = to_dev(s.u0)
        dx = to_dev(s.dx0)
        hist = empty((max(s.iters, 1),), torch.float64)
        o = pxst.make_opts(s.iters, s.window, s.refine, s.update_dx, s.tr_window, ref_mode=mode)
        times = []
        for rep in range(4):
            u.copy_(to_dev(s.u0))
            dx.copy_(to_dev(s.dx0))
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            pxst.solve(sc, o, u, dx, ref, w, hist, ws)
            b.record()
            torch.cuda.synchronize()
            if rep:
                times.append(a.elapsed_time(b))
        ms = float(np.median(times))
        out[mode] = {
            "ref_rel": stats(rel), "ref_acceptance_metric": float(acc),
            "u_px": stats(du), "argmin_equal": int(same.sum()), "argmin_ties": int(ties),
            "argmin_other": int((fin & (kgs != ko)).sum() - ties), "pixels": int(fin.sum()),
            "dx_px": stats(ddx), "frames": len(frames),
            "solve_ms": ms, "pm_evals_per_s": s.pm_evals() * s.iters / (ms * 1e-3),
        }
        say(f"    {json.dumps(out[mode])}")
    return out


def fmt(x, f="{:.2e}"):
    return "—" if x is None else f.format(x)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", nargs="+", default=["tiny", "realistic", "divergent"])
    ap.add_argument("--modes", nargs="+", default=["exact", "fp32", "bf16"])
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    import torch
    pxst.load_library()
    res = {}
    for name in args.configs:
        res[name] = run_config(name, args.modes, torch)
    lines = ["| scan | reference arithmetic | I_ref rel. max / p99 | max\\|dI\\|/max\\|I\\| | u px max / p99 "
             "| argmin equal / ties / other | dx px max / p99 | solve ms | PM evals/s |",
             "|---|---|---|---|---|---|---|---|---|"]
    for name, per in res.items():
        for mode, r in per.items():
            lines.append(
                f"| {name} | {mode} | {fmt(r['ref_rel']['max'])} / {fmt(r['ref_rel']['p99'])} | "
                f"{fmt(r['ref_acceptance_metric'])} | {fmt(r['u_px']['max'])} / {fmt(r['u_px']['p99'])} | "
                f"{r['argmin_equal']} / {r['argmin_ties']} / {r['argmin_other']} of {r['pixels']} | "
                f"{fmt(r['dx_px']['max'])} / {fmt(r['dx_px']['p99'])} | {r['solve_ms']:.2f} | "
                f"{r['pm_evals_per_s']:.3g} |")
    print("\n".join(lines), flush=True)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
