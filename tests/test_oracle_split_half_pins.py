"""Pins of the split-half analysis of the oracle (Sec. 2.3; CPU only)."""
import numpy as np

import oracle
from oracle import bruteforce
from synth import random_small_scan


def _scan_and_ref(seed=71):
    s = random_small_scan(det=(12, 15), n_frames=6, seed=seed, window=(2, 2))
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    return s, ref, w


def test_whole_frames_equal_the_search_on_a_frame_subset():
    """A split by whole frames is the ordinary search on each subset of frames."""
    s, ref, w = _scan_and_ref()
    half = np.zeros(s.frames.shape, dtype=np.uint8)
    half[[1, 3, 4]] = 1
    ua, ub, _ = oracle.split_half_pixel_maps(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin,
                                             (2, 2), half)
    for sel, got in (([0, 2, 5], ua), ([1, 3, 4], ub)):
        want, _, _ = oracle.update_pixel_map(s.frames[sel], s.white, s.mask, ref, w, s.dx0[sel], s.u0,
                                             s.origin, (2, 2))
        np.testing.assert_array_equal(got, want)


def test_empty_half_leaves_the_map_and_other_half_is_full_search():
    """All terms in half 0: half 0 is the full search, half 1 has no term, keeps u."""
    s, ref, w = _scan_and_ref(72)
    half = np.zeros(s.frames.shape, dtype=np.uint8)
    ua, ub, hist = oracle.split_half_pixel_maps(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin,
                                                (2, 2), half)
    want, _, _ = oracle.update_pixel_map(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin, (2, 2))
    np.testing.assert_array_equal(ua, want)
    np.testing.assert_array_equal(ub, s.u0)
    assert hist.sum() == 0


def test_per_pixel_split_matches_brute_force_loops():
    """Random (frame, pixel) halves: each pixel's map equals the explicit-loop search over
    that pixel's own frames of the half (no paraboloid)."""
    s, ref, w = _scan_and_ref(73)
    rng = np.random.default_rng(9)
    half = rng.integers(0, 2, s.frames.shape).astype(np.uint8)
    ua, ub, _ = oracle.split_half_pixel_maps(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin,
                                             (2, 2), half, refine=False)
    H, W = s.det
    for i, j in [(0, 0), (5, 7), (11, 14), (6, 2)]:
        for hv, got in ((0, ua), (1, ub)):
            sel = np.nonzero(half[:, i, j] == hv)[0]
            m = np.zeros((H, W), dtype=s.mask.dtype)
            m[i, j] = s.mask[i, j]
            res = bruteforce.pixel_map(s.frames[sel], s.white, m, ref, w, s.dx0[sel], s.u0, s.origin, 2, 2)
            u0, u1 = res[i][j][0], res[i][j][1]
            np.testing.assert_array_equal(got[:, i, j], [u0, u1])


def test_histogram_counts_the_pixels_in_range():
    """The histogram holds every pixel with a result in both halves whose difference
    lies in the range."""
    s, ref, w = _scan_and_ref(74)
    rng = np.random.default_rng(10)
    half = rng.integers(0, 2, s.frames.shape).astype(np.uint8)
    ua, ub, hist = oracle.split_half_pixel_maps(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin,
                                                (2, 2), half, hist_range=3.0, nbins=12)
    assert hist.shape == (2, 12)
    _, _, ka = oracle.update_pixel_map(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin, (2, 2),
                                       frame_mask=(half == 0))
    _, _, kb = oracle.update_pixel_map(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin, (2, 2),
                                       frame_mask=(half == 1))
    good = (s.mask > 0) & (ka >= 0) & (kb >= 0)
    for ax in range(2):
        d = (ua[ax] - ub[ax])[good]
        assert hist[ax].sum() == np.count_nonzero(np.abs(d) <= 3.0)
