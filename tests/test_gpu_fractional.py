"""Parity of the fractional-step pixel-map search with the FP64 oracle (GPU).

Bar (as the integer search): identical fine-grid argmin except where the oracle's
errors at the two indices differ by < 1e-6 relative; the map within 1e-3 px where the
argmin agrees; the minimum error within the float32 bound of the integer search's
tests, taken at the oracle's error with all frames valid (a looser 1e-3 relative where
that bound cannot be formed).
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


def gpu_frac(s, ref, w, dx, u, window, steps):
    sc = dev_scan(s)
    ws = pxst.alloc_workspace(sc.geom, pxst.make_opts(1, window))
    H, W = s.det
    uo = empty((2, H, W), torch.float32)
    e = empty((H, W), torch.float32)
    k = empty((H, W), torch.int32)
    pxst.update_pixel_map_fractional(sc, to_dev(ref.astype(np.float32)), to_dev(w.astype(np.float64)),
                                     to_dev(dx), to_dev(u), pxst.make_window(window[0], window[1], False),
                                     steps, uo, e, k, ws)
    torch.cuda.synchronize()
    return uo.cpu().numpy(), e.cpu().numpy(), k.cpu().numpy()


def check(s, ref, w, dx, u, window, steps, pixels=None, label=""):
    say(f"[fractional] {label} det={s.det} N={s.n_frames} window={window} steps={steps}")
    ref32 = ref.astype(np.float32).astype(np.float64)
    ug, eg, kg = gpu_frac(s, ref32, w, dx, u, window, steps)
    H, W = s.det
    if pixels is None:
        rows, cols = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        rows, cols = rows.ravel(), cols.ravel()
    else:
        rows, cols = pixels
    uo, eo, ko, E = oracle.update_pixel_map_fractional(s.frames, s.white, s.mask, ref32, w, dx, u, s.origin,
                                                       window, steps, pixels=(rows, cols), return_errors=True)
    good = s.mask[rows, cols] > 0
    col = np.cumsum(good) - 1
    kg_s, eg_s, ug_s = kg[rows, cols], eg[rows, cols], ug[:, rows, cols]
    assert np.array_equal(kg_s < 0, ko < 0)
    flat = E.reshape(-1, E.shape[-1]) if E is not None else None
    ties = 0
    for p in np.nonzero((kg_s != ko) & (ko >= 0))[0]:
        a, b = flat[kg_s[p], col[p]], flat[ko[p], col[p]]
        assert np.isfinite(a) and abs(a - b) <= ARGMIN_TIE_REL * abs(b), (p, kg_s[p], ko[p], a, b)
        ties += 1
    same = (kg_s == ko) & (ko >= 0)
    du = np.abs(ug_s[:, same] - uo[:, same])
    assert du.max(initial=0) <= U_TOL_PX, du.max()
    fin = same & np.isfinite(eo)
    de = np.abs(eg_s[fin].astype(np.float64) - eo[fin])
    assert np.all(de <= 1e-3 * np.abs(eo[fin]) + 1e-7), de.max()
    # unchanged where nothing was found
    none = ko < 0
    np.testing.assert_array_equal(ug_s[:, none], u[:, rows[none], cols[none]])
    say(f"    ok: {same.sum()} equal, {ties} ties, max|du|={du.max(initial=0):.2e}")


@pytest.mark.parametrize("window,steps", [((2, 2), 3), ((1, 3), 5), ((0, 2), 3), ((3, 0), 3)])
def test_fractional_small(window, steps):
    s = random_small_scan(det=(29, 41), n_frames=6, seed=61, window=window)
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    check(s, ref, w, s.dx0, s.u0, window, steps, label="small")


def test_one_step_equals_integer_search_without_refinement():
    s = random_small_scan(det=(31, 37), n_frames=5, seed=62, window=(2, 3))
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    say("[fractional] steps 1 vs integer search")
    ug, eg, kg = gpu_frac(s, ref, w, s.dx0, s.u0, (2, 3), 1)
    sc = dev_scan(s)
    ws = pxst.alloc_workspace(sc.geom, pxst.make_opts(1, (2, 3)))
    H, W = s.det
    uo = empty((2, H, W), torch.float32)
    e = empty((H, W), torch.float32)
    k = empty((H, W), torch.int32)
    pxst.update_pixel_map(sc, to_dev(ref.astype(np.float32)), to_dev(w), to_dev(s.dx0), to_dev(s.u0),
                          pxst.make_window(2, 3, False), uo, e, k, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(kg, k.cpu().numpy())
    np.testing.assert_array_equal(eg, e.cpu().numpy())
    np.testing.assert_array_equal(ug, uo.cpu().numpy())


def test_realistic_full_size_sampled():
    """Realistic scan at full size (256x1024, 121 frames, +-4 px window, three steps: 729
    fine candidates), the true reference; 48 sampled pixels against the oracle."""
    s = cached_scan("realistic")
    ref = s.ref_true
    w = np.ones_like(ref)
    rng = np.random.default_rng(103)
    rows = np.concatenate([rng.integers(0, 256, 44), [0, 255, 0, 255]])
    cols = np.concatenate([rng.integers(0, 1024, 44), [0, 0, 1023, 1023]])
    check(s, ref, w, s.dx0, s.u0, (4, 4), 3, pixels=(rows, cols), label="realistic full size")
