"""Parity of the pixel-map regularisation with the FP64 oracle (GPU).

Bar: the map is float32 and the GPU sums in float64, so every value must agree with
the oracle within the float32 rounding of the map's magnitude, 2^-22 max|u| (half a
unit of the last place, doubled for the filter's intermediate and the final
rounding).  Small cases against the conjugate-gradient oracle (the paper's method),
the full realistic detector against the oracle's direct solution.
"""
import sys

import numpy as np
import pytest

import paper_2003_12726_amd as pxst
from oracle import regularise as reg
from gpu_util import to_dev, empty

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


def field(shape, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    H, W = shape
    ii, jj = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    u = np.stack([ii + 3.0 * np.sin(jj / 5.0) + rng.normal(0, 0.5, (H, W)),
                  jj + 2.0 * np.cos(ii / 7.0) + rng.normal(0, 0.5, (H, W))]) * scale
    return u.astype(np.float32)


def gpu_regularise(u, sigma, integrate, inplace=False):
    H, W = u.shape[1:]
    g = pxst.make_geom(1, (H, W), (H + 8, W + 8), (-4, -4))
    ws = pxst.alloc_workspace(g, pxst.make_opts(1, (1, 1), integrate=integrate))
    ui = to_dev(u)
    uo = ui if inplace else empty((2, H, W), torch.float32)
    pxst.regularise_pixel_map(g, ui, uo, sigma, integrate, ws)
    torch.cuda.synchronize()
    return uo.cpu().numpy()


def check(got, want, u):
    tol = 2.0 ** -22 * float(np.abs(u).max()) + 1e-12
    d = np.abs(got.astype(np.float64) - want)
    assert d.max() <= tol, (d.max(), tol)
    return d.max()


@pytest.mark.parametrize("shape,sigma", [((37, 53), 0.8), ((37, 53), 2.0), ((20, 70), 5.0), ((1, 9), 1.5)])
def test_filter(shape, sigma):
    say(f"[regularise] filter shape={shape} sigma={sigma}")
    u = field(shape, 11)
    check(gpu_regularise(u, sigma, False), reg.gaussian_filter_map(u, sigma), u)


@pytest.mark.parametrize("shape", [(7, 9), (33, 45), (1, 17), (17, 1), (2, 6), (3, 3), (64, 40)])
def test_integrate_against_cg(shape):
    say(f"[regularise] integrate shape={shape}")
    u = field(shape, 12)
    check(gpu_regularise(u, 0.0, True), reg.integrate_map(u), u)


def test_filter_then_integrate_in_place():
    say("[regularise] filter + integrate in place (41, 66)")
    u = field((41, 66), 13)
    want = reg.regularise_pixel_map(u, 1.7, True)
    check(gpu_regularise(u, 1.7, True, inplace=True), want, u)


def test_realistic_detector_full_size():
    """256 x 1024 map at the realistic scan's scale (coordinates up to ~1300 px):
    sigma 5 then integration, against the oracle's direct solution, every pixel."""
    say("[regularise] realistic 256x1024, sigma 5, integrate")
    u = field((256, 1024), 14) + np.float32(141.0)
    want = reg.regularise_pixel_map(u, 5.0, True, direct=True)
    got = gpu_regularise(u, 5.0, True)
    d = check(got, want, u)
    say(f"    max |du| = {d:.2e} px")
    np.testing.assert_allclose(reg.curl(got.astype(np.float64)), 0.0, atol=4e-3)


def test_solve_applies_regularisation_after_the_search():
    """The main loop with sigma/integrate equals the entry points composed: one
    iteration = reference update, pixel-map search, regularisation, error."""
    from synth import random_small_scan
    from gpu_util import dev_scan
    say("[regularise] solve with sigma 1.2 + integrate vs composed entry points")
    s = random_small_scan(det=(31, 37), n_frames=6, seed=41, window=(2, 2))
    sc = dev_scan(s)
    opts = pxst.make_opts(1, (2, 2), True, sigma=1.2, integrate=True)
    ws = pxst.alloc_workspace(sc.geom, opts)
    H, W = s.det
    # composed
    ref = empty(s.ref_shape, torch.float32)
    w = empty(s.ref_shape, torch.float64)
    u0, dx0 = to_dev(s.u0), to_dev(s.dx0)
    pxst.update_reference(sc, u0, dx0, ref, w, ws)
    u1 = empty((2, H, W), torch.float32)
    pxst.update_pixel_map(sc, ref, w, dx0, u0, pxst.make_window(2, 2, True), u1, None, None, ws)
    pxst.regularise_pixel_map(sc.geom, u1, u1, 1.2, True, ws)
    torch.cuda.synchronize()
    want = u1.cpu().numpy()
    # loop
    u = to_dev(s.u0)
    dx = to_dev(s.dx0)
    hist = empty((1,), torch.float64)
    pxst.solve(sc, opts, u, dx, ref, w, hist, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u.cpu().numpy(), want)
