"""The stored oracle results of the benchmark's precision study are the oracle's: the
reference at the stored pixels, the pixel map of some of the sampled pixels and one
frame's translation update are recomputed from the same seeded scan and compared."""
import os

import numpy as np

import oracle
from synth.scans import cached_scan

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "precision_realistic.npz")


def test_precision_golden_is_the_oracle():
    g = np.load(GOLD)
    s = cached_scan("realistic")
    ro, wo = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    np.testing.assert_array_equal(ro.ravel()[g["ref_index"]], g["ref_value"])
    sel = wo > 1e-3 * np.median(wo[wo > 0])
    assert g["ref_scale"] == max(np.abs(ro[sel]).max(), np.abs(ro[sel]).mean())
    k = slice(0, 12)
    rows, cols = g["rows"][k], g["cols"][k]
    uo, eo, ko = oracle.update_pixel_map(s.frames, s.white, s.mask, ro, wo, s.dx0, s.u0, s.origin,
                                         s.window, refine=s.refine, pixels=(rows, cols))
    np.testing.assert_array_equal(uo, g["u"][:, k])
    np.testing.assert_array_equal(ko, g["argmin"][k])
    np.testing.assert_array_equal(eo[ko >= 0], g["top_error"][k][ko >= 0, 0])
    n = int(g["frames"][2])
    dxo, _, _ = oracle.update_translations(s.frames[n:n + 1], s.white, s.mask, ro, wo, s.u0,
                                           s.dx0[n:n + 1], s.origin, (2, 2), refine=True)
    np.testing.assert_array_equal(dxo[0], g["dx"][2])
