"""Write the FP64 oracle's results that the benchmark's precision study compares with.

The study (the realistic scan's start state (u0, dx0), one step of each kind, for each
reference-update arithmetic of the library) needs the oracle's reference image,
pixel-map update and translation update of that state.  They are computed here, by the
oracle alone, once, and stored at sampled positions in ``precision_realistic.npz``:

* the reference at 8192 well-covered pixels (weight > 1e-3 of the median), with the
  scale max(max |I_ref|, mean |I_ref|) of all well-covered pixels;
* the pixel-map update (window +-10, refinement) of 400 sampled pixels with the
  oracle's own reference: the map, the argmin and each pixel's eight smallest
  candidate errors with their indices (to apply the tie rule to a different argmin);
* the translation update (+-2, refinement) of six frames with that reference and u0.

Run: python tests/golden/make_precision_refs.py   (a few tens of seconds)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth.scans import cached_scan  # noqa: E402

OUT = os.path.join(HERE, "precision_realistic.npz")
FRAMES = [0, 30, 60, 61, 90, 120]


def sample(s, seed=7, npx=400, nref=8192):
    rng = np.random.default_rng(seed)
    H, W = s.det
    return rng.integers(0, H, npx), rng.integers(0, W, npx), rng


def main():
    s = cached_scan("realistic")
    rows, cols, rng = sample(s)
    print("oracle reference", flush=True)
    ro, wo = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    sel = wo > 1e-3 * np.median(wo[wo > 0])
    flat = np.flatnonzero(sel)
    ridx = np.sort(rng.choice(flat, 8192, replace=False))
    scale = max(np.abs(ro[sel]).max(), np.abs(ro[sel]).mean())
    print("oracle pixel map", flush=True)
    uo, eo, ko, E = oracle.update_pixel_map(s.frames, s.white, s.mask, ro, wo, s.dx0, s.u0, s.origin,
                                            s.window, refine=s.refine, pixels=(rows, cols),
                                            return_errors=True)
    good = s.mask[rows, cols] > 0
    flatE = E.reshape(-1, E.shape[-1])
    top_i = np.full((rows.size, 8), -1, dtype=np.int32)
    top_e = np.full((rows.size, 8), np.inf)
    gi = np.nonzero(good)[0]
    for c, p in enumerate(gi):
        order = np.argsort(flatE[:, c], kind="stable")[:8]
        top_i[p] = order
        top_e[p] = flatE[order, c]
    print("oracle translations", flush=True)
    dxo, _, _ = oracle.update_translations(s.frames[FRAMES], s.white, s.mask, ro, wo, s.u0,
                                           s.dx0[FRAMES], s.origin, (2, 2), refine=True)
    np.savez_compressed(OUT, ref_index=ridx.astype(np.int64), ref_value=ro.ravel()[ridx],
                        ref_scale=np.float64(scale), n_valid=np.int64((wo > 0).sum()),
                        rows=rows.astype(np.int64), cols=cols.astype(np.int64), u=uo, argmin=ko,
                        top_index=top_i, top_error=top_e, frames=np.array(FRAMES), dx=dxo)
    print(f"wrote {OUT} ({os.path.getsize(OUT)} bytes)", flush=True)


if __name__ == "__main__":
    main()
