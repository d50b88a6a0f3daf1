"""Parity of the split-half analysis with the FP64 oracle (GPU).

Bar: each half's map as the pixel-map search's (identical argmin except oracle ties
within 1e-6 relative, u within 1e-3 px where the argmin agrees); the histogram is
checked exactly against numpy's histogram of the GPU's own maps over the pixels with a
result in both halves, and against the oracle's histogram up to the pixels whose
difference lies within 1e-3 px of a bin edge (or, with a different argmin, anywhere).
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2003_12726_amd as pxst
from synth import random_small_scan
from synth.scans import cached_scan
from gpu_util import dev_scan, to_dev, empty, ARGMIN_TIE_REL, U_TOL_PX

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pxst.load_library()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(s, ref, w, window, refine, half, R, nb):
    sc = dev_scan(s)
    ws = pxst.alloc_workspace(sc.geom, pxst.make_opts(1, window))
    H, W = s.det
    ua = empty((2, H, W), torch.float32)
    ub = empty((2, H, W), torch.float32)
    hist = empty((2, nb), torch.int32)
    pxst.split_half_pixel_map(sc, to_dev(ref.astype(np.float32)), to_dev(w.astype(np.float64)), to_dev(s.dx0),
                              to_dev(s.u0), pxst.make_window(window[0], window[1], refine), to_dev(half), ua, ub,
                              R, nb, hist, ws)
    torch.cuda.synchronize()
    return ua.cpu().numpy(), ub.cpu().numpy(), hist.cpu().numpy()


def check_half(s, ref32, w, window, refine, mask_h, got, rows=None, cols=None):
    H, W = s.det
    if rows is None:
        rows, cols = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        rows, cols = rows.ravel(), cols.ravel()
    uo, eo, ko, E = oracle.update_pixel_map(s.frames, s.white, s.mask, ref32, w, s.dx0, s.u0, s.origin, window,
                                            refine, pixels=(rows, cols), return_errors=True, frame_mask=mask_h)
    g = got[:, rows, cols]
    found = ko >= 0
    same = found & np.all(np.abs(g - uo) <= U_TOL_PX, axis=0)
    # pixels that differ must be oracle ties: the GPU's position is another candidate whose
    # oracle error is within 1e-6 relative of the minimum
    good = s.mask[rows, cols] > 0
    col = np.cumsum(good) - 1
    flat = E.reshape(-1, E.shape[-1]) if E is not None else None
    c = oracle.round_half_up(s.u0[:, rows, cols])
    NY = 2 * window[1] + 1
    bad = []
    for p in np.nonzero(found & ~same)[0]:
        kx = int(round(g[0, p] - c[0, p])) + window[0]
        ky = int(round(g[1, p] - c[1, p])) + window[1]
        if not (0 <= kx < 2 * window[0] + 1 and 0 <= ky < NY):
            bad.append(p)
            continue
        a, b = flat[kx * NY + ky, col[p]], flat[ko[p], col[p]]
        if not (np.isfinite(a) and abs(a - b) <= ARGMIN_TIE_REL * abs(b)):
            bad.append(p)
    assert not bad, f"{len(bad)} pixels differ, e.g. {(rows[bad[0]], cols[bad[0]])}"
    np.testing.assert_array_equal(g[:, ~found], s.u0[:, rows[~found], cols[~found]])
    return ko


@pytest.mark.parametrize("window,refine", [((2, 2), True), ((3, 1), False)])
def test_split_half_small(window, refine):
    say(f"[split-half] small window={window} refine={refine}")
    s = random_small_scan(det=(27, 35), n_frames=8, seed=81, window=window)
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    ref32 = ref.astype(np.float32).astype(np.float64)
    half = np.random.default_rng(82).integers(0, 2, s.frames.shape).astype(np.uint8)
    R, nb = 2.0, 16
    ua, ub, hist = run(s, ref32, w, window, refine, half, R, nb)
    ka = check_half(s, ref32, w, window, refine, half == 0, ua)
    kb = check_half(s, ref32, w, window, refine, half == 1, ub)
    both = (s.mask.ravel() > 0) & (ka >= 0) & (kb >= 0)
    for ax in range(2):
        d = (ua[ax].astype(np.float64) - ub[ax].astype(np.float64)).ravel()[both]
        np.testing.assert_array_equal(hist[ax], np.histogram(d, bins=nb, range=(-R, R))[0])
    # against the oracle's histogram: differences only from pixels near bin edges
    _, _, ho = oracle.split_half_pixel_maps(s.frames, s.white, s.mask, ref32, w, s.dx0, s.u0, s.origin, window,
                                            half, refine, R, nb)
    assert np.abs(hist - ho).sum() <= 2 * 2 * max(1, int(0.02 * both.sum()))


def test_split_half_realistic_full_size():
    """Realistic scan at full size (256x1024, 121 frames, +-4 px window with refinement),
    random halves; 64 sampled pixels of each half against the oracle."""
    s = cached_scan("realistic")
    say("[split-half] realistic full size, window (4, 4)")
    ref = s.ref_true
    w = np.ones_like(ref)
    half = np.random.default_rng(83).integers(0, 2, s.frames.shape).astype(np.uint8)
    ua, ub, hist = run(s, ref, w, (4, 4), True, half, 1.0, 64)
    rng = np.random.default_rng(84)
    rows, cols = rng.integers(0, 256, 64), rng.integers(0, 1024, 64)
    ref32 = ref.astype(np.float32).astype(np.float64)
    check_half(s, ref32, w, (4, 4), True, half == 0, ua, rows, cols)
    check_half(s, ref32, w, (4, 4), True, half == 1, ub, rows, cols)
    assert hist.sum() > 0
