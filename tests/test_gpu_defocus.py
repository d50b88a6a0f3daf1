"""Parity of the defocus-by-registration sweep with the FP64 oracle (GPU).

Bar: contrasts within 1e-5 relative (the reference agrees to ~6e-8 per pixel; the
contrast is a small variance over a large squared mean, which amplifies that by about
1/sqrt(contrast)); the chosen candidate identical.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2003_12726_amd as pxst
from synth.scans import cached_scan
from gpu_util import dev_scan, to_dev, empty

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


class _S:
    pass


def gpu_sweep(frames, white, mask, dx, origin, ref_shape, scales, centre=None):
    s = _S()
    s.frames, s.white, s.mask, s.ref_shape, s.origin = frames, white.astype(np.float32), mask, ref_shape, origin
    sc = dev_scan(s)
    ws = pxst.alloc_workspace(sc.geom, None)
    n = len(scales)
    c = empty((n,), torch.float64)
    b = empty((1,), torch.int32)
    pxst.defocus_sweep(sc, to_dev(np.asarray(dx, np.float32)), scales, c, b, centre, ws)
    torch.cuda.synchronize()
    return c.cpu().numpy(), int(b.cpu().numpy()[0])


def magnified_scan(s_true, seed=3):
    from scipy import ndimage
    rng = np.random.default_rng(seed)
    H, W = 40, 44
    Rs, Rf = 110, 116
    ref = 100.0 + 400.0 * ndimage.gaussian_filter(rng.random((Rs, Rf)), 2.0, mode="wrap")
    origin = (-35, -35)
    g = np.array([[a, b] for a in (0, 10, 20, 30) for b in (0, 10, 20, 30)], dtype=np.float64)
    u = oracle.linear_map((H, W), s_true)
    valid = np.ones((Rs, Rf), dtype=bool)
    frames = np.empty((g.shape[0], H, W))
    for n in range(g.shape[0]):
        v, ok = oracle.bilinear_gather(ref, valid, u[0] - g[n, 0] - origin[0], u[1] - g[n, 1] - origin[1])
        frames[n] = v
    return np.round(frames).astype(np.uint16), np.ones((H, W)), np.ones((H, W), np.uint8), g, origin, (Rs, Rf)


def test_sweep_small_picks_true_scale():
    say("[defocus] 40x44, 16 frames, 25 candidates")
    frames, white, mask, dx, origin, shape = magnified_scan((1.1, 0.9))
    scales = np.array([(a, b) for a in (1.0, 1.05, 1.1, 1.15, 1.2) for b in (0.8, 0.85, 0.9, 0.95, 1.0)],
                      dtype=np.float32)
    cg, bg = gpu_sweep(frames, white, mask, dx, origin, shape, scales)
    co, bo = oracle.defocus_sweep(frames, white, mask, dx.astype(np.float32).astype(np.float64), origin, shape,
                                  scales.astype(np.float64))
    np.testing.assert_allclose(cg, co, rtol=1e-5, atol=0)
    assert bg == bo
    assert tuple(scales[bg]) == (np.float32(1.1), np.float32(0.9))


def test_sweep_realistic_full_size():
    s = cached_scan("realistic")
    say("[defocus] realistic 256x1024, 121 frames, 3 candidates, off-centre fixed point")
    scales = np.array([(0.99, 1.0), (1.0, 1.0), (1.0, 1.01)], dtype=np.float32)
    centre = (100.0, 400.0)
    cg, bg = gpu_sweep(s.frames, s.white, s.mask, s.dx0, s.origin, s.ref_shape, scales, centre)
    co, bo = oracle.defocus_sweep(s.frames, s.white, s.mask, s.dx0, s.origin, s.ref_shape,
                                  scales.astype(np.float64), centre)
    np.testing.assert_allclose(cg, co, rtol=1e-5, atol=0)
    assert bg == bo
