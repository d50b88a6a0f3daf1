"""Parity of every C-ABI call with the FP64 oracle on the same seeded inputs (GPU).

Bar: identical argmin except where the oracle's errors at the two indices differ by
< 1e-6 relative; refined map / translations within 1e-3 px; reference within 1e-5
relative; error figures within 1e-5 relative.  Inputs of each single-step test come
from the generator or the oracle, never from the GPU path.
"""
import sys

import dataclasses

import numpy as np
import pytest

import oracle
import paper_2003_12726_amd as pxst
from synth import make_scan, spec_for, random_small_scan, exact_scan, CONFIGS
from synth.scans import ScanSpec, cached_scan
from gpu_util import (dev_scan, to_dev, empty, ref_rel_error, compare_argmin, emin_bound, U_TOL_PX,
                      REF_TOL_REL, ERR_TOL_REL, fixed_point_step)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pxst.load_library()


# ------------------------------------------------------------------------ helpers

def gpu_reference(s, u, dx, mode="exact"):
    sc = dev_scan(s)
    ref = empty(s.ref_shape, torch.float32)
    w = empty(s.ref_shape, torch.float64)
    ws = pxst.alloc_workspace(sc.geom, None)
    pxst.update_reference(sc, to_dev(u), to_dev(dx), ref, w, ws, mode=mode)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), w.cpu().numpy()


def gpu_pixel_map(s, ref, w, dx, u, window, refine, inplace=False):
    sc = dev_scan(s)
    opts = pxst.make_opts(1, window, refine)
    ws = pxst.alloc_workspace(sc.geom, opts)
    u_in = to_dev(u)
    u_out = u_in if inplace else torch.empty_like(u_in)
    H, W = s.det
    e = empty((H, W), torch.float32)
    k = empty((H, W), torch.int32)
    pxst.update_pixel_map(sc, to_dev(ref.astype(np.float32)), to_dev(w.astype(np.float64)),
                          to_dev(dx), u_in, pxst.make_window(window[0], window[1], refine), u_out, e,
                          k, ws)
    torch.cuda.synchronize()
    return u_out.cpu().numpy(), e.cpu().numpy(), k.cpu().numpy()


def check_pixel_map(s, ref, w, dx, u, window, refine, pixels=None, inplace=False, label="",
                    info=None, fixed_point=False):
    """Run both sides and apply the bar; returns the GPU outputs.  ``info`` (a dict), if
    given, receives the oracle's per-pixel outputs and which compared pixels had a
    candidate with an invalid lookup in some frame (pixels of edge tiles)."""
    say(f"[pixel-map] {label} det={s.det} N={s.n_frames} window={window} refine={refine}")
    ref32 = ref.astype(np.float32).astype(np.float64)
    ug, eg, kg = gpu_pixel_map(s, ref32, w, dx, u, window, refine, inplace)
    H, W = s.det
    if pixels is None:
        rows, cols = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        rows, cols = rows.ravel(), cols.ravel()
    else:
        rows, cols = pixels
    uo, eo, ko, (E, (esum, vsum, nsum)) = oracle.update_pixel_map(
        s.frames, s.white, s.mask, ref32, w, dx, u, s.origin, window, refine, pixels=(rows, cols),
        return_errors="sums")
    good = s.mask[rows, cols] > 0
    gidx = np.full(rows.shape[0], -1)
    gidx[good] = np.arange(good.sum())
    kg_s = kg[rows, cols]
    eg_s = eg[rows, cols]
    ug_s = ug[:, rows, cols]
    ok, nbad, bad = compare_argmin(kg_s, ko, E, gidx)
    assert nbad == 0, f"{nbad} argmin mismatches, e.g. pixel {(rows[bad[0]], cols[bad[0]])}: gpu {kg_s[bad[0]]} oracle {ko[bad[0]]}"
    same = kg_s == ko
    fin = same & np.isfinite(eo)
    assert np.all(np.isinf(eg_s[same & ~np.isfinite(eo)]))
    if fin.any():
        # bound from the float32 rounding of the residuals at the chosen candidate
        cols_g = gidx[fin]
        kk = ko[fin]
        nv = nsum.reshape(-1, nsum.shape[-1])[kk, cols_g]
        var = vsum.reshape(-1, vsum.shape[-1])[kk, cols_g]
        imax = s.frames[:, rows[fin], cols[fin]].max(axis=0).astype(np.float64)
        wq = s.white[rows[fin], cols[fin]] * fixed_point_step(ref32, w) if fixed_point else 0.0
        bound = emin_bound(eo[fin], nv, var, imax, wq=wq)
        dE = np.abs(eg_s[fin].astype(np.float64) - eo[fin])
        assert np.all(dE <= bound), (dE / bound).max()
    du = np.abs(ug_s[:, same] - uo[:, same])
    assert du.max(initial=0) <= U_TOL_PX, du.max()
    if info is not None:
        nfull = (nsum.reshape(-1, nsum.shape[-1]) < s.n_frames).any(axis=0)
        edge = np.zeros(rows.shape[0], dtype=bool)
        edge[good] = nfull
        info.update(u=uo, e=eo, k=ko, edge=edge, rows=rows, cols=cols, kg=kg_s)
    say(f"    ok: {same.sum()} equal, {ok} tie-swaps, max|du|={du.max(initial=0):.2e}")
    return ug, eg, kg


def oracle_state(s, u=None, dx=None):
    u = s.u0 if u is None else u
    dx = s.dx0 if dx is None else dx
    return oracle.update_reference(s.frames, s.white, s.mask, u, dx, s.origin, s.ref_shape)


# --------------------------------------------------------------- reference update

@pytest.mark.parametrize("case", ["tiny", "small_masked", "small_dx_int", "exact"])
def test_reference_parity(case):
    if case == "tiny":
        s = make_scan(CONFIGS["tiny"])
    elif case == "small_masked":
        s = random_small_scan(det=(37, 53), n_frames=7, seed=21)
    elif case == "small_dx_int":
        s = random_small_scan(det=(29, 31), n_frames=5, seed=22)
        s.dx0 = np.round(s.dx0)
    else:
        s = exact_scan()
    say(f"[reference] {case} det={s.det} N={s.n_frames} ref={s.ref_shape}")
    rg, wg = gpu_reference(s, s.u0, s.dx0)
    ro, wo = oracle_state(s)
    np.testing.assert_array_equal(wg > 0, wo > 0)
    err, sel = ref_rel_error(rg, ro, wo)
    assert err < REF_TOL_REL, err
    pos = wo > 0
    np.testing.assert_allclose(wg[pos], wo[pos], rtol=1e-6)
    assert np.all(rg[~pos] == 0)


@pytest.mark.parametrize("mode", ["fp32", "bf16"])
def test_reference_modes(mode):
    """The other reference-update arithmetics of the precision study: the float32
    gather meets the same bar as the default; bfloat16 storage is the exact update
    rounded to bfloat16 (ties to even), within 2^-8 relative of the oracle (bfloat16
    keeps 8 significand bits)."""
    s = random_small_scan(det=(37, 53), n_frames=7, seed=23)
    say(f"[reference] mode {mode} det={s.det} N={s.n_frames}")
    rg, wg = gpu_reference(s, s.u0, s.dx0, mode=mode)
    ro, wo = oracle_state(s)
    np.testing.assert_array_equal(wg > 0, wo > 0)
    pos = wo > 0
    np.testing.assert_allclose(wg[pos], wo[pos], rtol=1e-6)
    if mode == "fp32":
        err, _ = ref_rel_error(rg, ro, wo)
        assert err < REF_TOL_REL, err
    else:
        bits = rg.view(np.uint32)
        assert np.all(bits & 0xFFFF == 0)
        re_, _ = gpu_reference(s, s.u0, s.dx0, mode="exact")
        # the rounding of the exact result, ties to even
        b = re_.view(np.uint32).astype(np.uint64)
        rounded = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32).view(np.float32)
        np.testing.assert_array_equal(rg, rounded)
        rel = np.abs(rg[pos].astype(np.float64) - ro[pos]) / np.abs(ro[pos]).clip(1e-30)
        assert rel.max() <= 2.0 ** -8 + 1e-5, rel.max()


@pytest.mark.parametrize("name", ["realistic", "divergent"])
def test_reference_parity_full_size(name):
    """Full-size scans (256x1024 with 121 frames; 512x512 with 400 frames, whose splat
    runs in frame chunks combined afterwards): whole reference compared."""
    s = cached_scan(name)
    say(f"[reference] {name} full det={s.det} N={s.n_frames}")
    rg, wg = gpu_reference(s, s.u0, s.dx0)
    ro, wo = oracle_state(s)
    np.testing.assert_array_equal(wg > 0, wo > 0)
    err, _ = ref_rel_error(rg, ro, wo)
    assert err < REF_TOL_REL, err


def test_reference_deterministic():
    s = random_small_scan(det=(37, 53), n_frames=7, seed=23)
    a = gpu_reference(s, s.u0, s.dx0)
    b = gpu_reference(s, s.u0, s.dx0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------------------- pixel map

@pytest.mark.parametrize("refine", [False, True])
def test_pixel_map_tiny(refine):
    s = make_scan(CONFIGS["tiny"])
    ref, w = oracle_state(s)
    check_pixel_map(s, ref, w, s.dx0, s.u0, s.window, refine, label="tiny")


@pytest.mark.parametrize("window", [(3, 2), (0, 3), (2, 0), (0, 0), (5, 1), (1, 6)])
def test_pixel_map_small_windows(window):
    s = random_small_scan(det=(37, 53), n_frames=7, seed=24)
    ref, w = oracle_state(s)
    check_pixel_map(s, ref, w, s.dx0, s.u0, window, True, label=f"small {window}")


def test_pixel_map_large_window_ragged():
    s = random_small_scan(det=(33, 45), n_frames=5, seed=25, window=(15, 15))
    ref, w = oracle_state(s)
    check_pixel_map(s, ref, w, s.dx0, s.u0, (15, 15), True, label="ragged R=15")


@pytest.mark.parametrize("r,n_frames,mask", [(13, 49, "ones"), (15, 150, "parity")])
def test_pixel_map_large_window_tile_halves(r, n_frames, mask):
    """Windows whose error tables of a whole 8x8 tile do not fit the LDS (31x31 and
    27x27 candidates): the matrix-core search takes each tile as two halves of 32
    pixels, interior and edge tiles alike.  Served-stream job shape (128x128, speckle
    reference, Gaussian white field); sampled pixels plus the detector's corners."""
    gx = int(np.ceil(np.sqrt(n_frames)))
    spec = ScanSpec(name=f"halves{r}", det=(128, 128), n_grid=(gx, int(np.ceil(n_frames / gx))),
                    step=4.0, jitter=0.5, disp_ss=(float(r), r / 2.0), disp_fs=(float(r), r / 2.0),
                    window=(r, r), iters=1, ref=None, ref_sigma=1.5, ref_contrast=0.15, white="gauss",
                    white_sigma=64.0, white_mean=4000.0, refine=True, n_frames=n_frames, seed=77 + r)
    s = make_scan(spec, mask=mask)
    ref, w = oracle_state(s)
    rng = np.random.default_rng(103)
    rows = np.concatenate([rng.integers(0, 128, 160), [0, 0, 127, 127, 64]])
    cols = np.concatenate([rng.integers(0, 128, 160), [0, 127, 0, 127, 64]])
    pxst.profile_enable(True)
    try:
        for fam in ("pm_fast_int8_ops", "pm_edge_mma", "pm_edge"):
            pxst.profile_read(fam)
        check_pixel_map(s, ref, w, s.dx0, s.u0, (r, r), True, pixels=(rows, cols),
                        label=f"tile halves R={r}")
        _, n_fast, ops = pxst.profile_read("pm_fast_int8_ops")
        _, n_edge, _ = pxst.profile_read("pm_edge_mma")
    finally:
        pxst.profile_enable(False)
    # both matrix-core launches ran, and interior tiles were searched on them
    assert n_fast == 1 and ops > 0 and n_edge == 1


def test_pixel_map_reference_valid_to_its_edge():
    """A reference grid cropped inside its valid area (every pixel of its first and last
    rows and columns valid), so that lookups reach row -1 and the last row and column
    and beyond: an edge tile's slow frame takes each corner inside the grid from its own
    row and column, also where the 2x2 block read was moved into the grid, and counts
    the corners outside as invalid, as the oracle's masked interpolation does (Sec. 4)."""
    s = make_scan(CONFIGS["tiny"])
    ref, w = oracle_state(s)
    rows = np.nonzero((w > 0).any(axis=1))[0]
    cols = np.nonzero((w > 0).any(axis=0))[0]
    r0, r1, c0, c1 = rows[0] + 6, rows[-1] - 6, cols[0] + 6, cols[-1] - 6
    ref_c = np.ascontiguousarray(ref[r0:r1 + 1, c0:c1 + 1])
    w_c = np.ascontiguousarray(w[r0:r1 + 1, c0:c1 + 1])
    for edge in (w_c[0], w_c[-1], w_c[:, 0], w_c[:, -1]):
        assert np.all(edge > 0)
    s2 = dataclasses.replace(s, origin=(s.origin[0] + int(r0), s.origin[1] + int(c0)), ref_shape=ref_c.shape)
    # lookups at the first and last rows of the grid exist
    p0 = np.floor(s.u0[0][None] - s.dx0[:, 0, None, None] - s2.origin[0]).astype(int)
    assert (p0 + s.window[0] >= ref_c.shape[0] - 1).any() and (p0 - s.window[0] <= -1).any()
    for refine in (False, True):
        check_pixel_map(s2, ref_c, w_c, s.dx0, s.u0, s.window, refine, label=f"reference cropped, refine={refine}")


def test_pixel_map_in_place_and_all_masked():
    s = random_small_scan(det=(21, 19), n_frames=4, seed=26)
    ref, w = oracle_state(s)
    check_pixel_map(s, ref, w, s.dx0, s.u0, (2, 2), True, inplace=True, label="in place")
    s.mask[:] = 0
    ug, eg, kg = gpu_pixel_map(s, ref, w, s.dx0, s.u0, (2, 2), True)
    np.testing.assert_array_equal(ug, s.u0)
    assert np.all(np.isinf(eg)) and np.all(kg == -1)


def test_pixel_map_single_frame():
    s = random_small_scan(det=(17, 23), n_frames=1, seed=27)
    ref, w = oracle_state(s)
    check_pixel_map(s, ref, w, s.dx0, s.u0, (2, 3), True, label="N=1")


def test_pixel_map_scattered_map_uses_generic_path():
    """A map with outliers far from their tile: staged regions exceed the LDS budget."""
    s = random_small_scan(det=(24, 24), n_frames=4, seed=28)
    ref, w = oracle_state(s)
    u = s.u0.copy()
    u[0, 3, 4] += 140.0
    u[1, 17, 9] -= 150.0
    check_pixel_map(s, ref, w, s.dx0, u, (2, 2), True, label="scattered")


def test_pixel_map_exact_recovery():
    s = exact_scan(window=(3, 3))
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u_true, s.dx_true, s.origin,
                                     s.ref_shape)
    rng = np.random.default_rng(5)
    u_start = s.u_true + rng.integers(-2, 3, s.u_true.shape).astype(np.float32)
    ug, eg, kg = check_pixel_map(s, ref, w, s.dx_true, u_start, (3, 3), False, label="exact")
    b = 4
    np.testing.assert_array_equal(ug[:, b:-b, b:-b], s.u_true[:, b:-b, b:-b])


def test_pixel_map_realistic_full_size_sampled():
    """Realistic scan at full size (256x1024, 121 frames, +-10 px, refinement): the GPU
    runs the whole detector in the benchmark's launch configuration; the oracle checks
    400 sampled pixels one by one.  Reference input: the generator's true reference."""
    s = cached_scan("realistic")
    ref = s.ref_true
    w = np.ones_like(ref)
    rng = np.random.default_rng(101)
    H, W = s.det
    rows = np.concatenate([rng.integers(0, H, 360), [0, H - 1, 0, H - 1, 5, 250, 128, 64]])
    cols = np.concatenate([rng.integers(0, W, 360), [0, 0, W - 1, W - 1, 1000, 3, 512, 700]])
    rows = np.concatenate([rows, np.full(32, 100)])
    cols = np.concatenate([cols, np.arange(300, 332)])
    check_pixel_map(s, ref, w, s.dx0, s.u0, s.window, True, pixels=(rows, cols),
                    label="realistic full size")


def test_pixel_map_divergent_full_size_sampled():
    """Divergent scan at full size (512x512, 400 frames, +-15 x +-3 px)."""
    s = cached_scan("divergent")
    ref = s.ref_true
    w = np.ones_like(ref)
    rng = np.random.default_rng(102)
    rows = rng.integers(0, 512, 120)
    cols = rng.integers(0, 512, 120)
    check_pixel_map(s, ref, w, s.dx_true, s.u0, s.window, True, pixels=(rows, cols),
                    label="divergent full size")


def test_pixel_map_zero_white_exact_ties():
    """Pixels whose white-field is 0 (Sec. 2.2.2): every residual is the count itself, so
    each candidate's error equals its variance and E is exactly 1 for every candidate with
    a valid frame; the first such candidate wins.  The GPU must pick exactly the oracle's
    candidate there (not merely one within the tie tolerance), in interior and edge tiles
    alike: the reference is cropped inside its valid area so that border tiles have
    candidates with invalid lookups in some frames but not all, and in all frames."""
    s = loop_scan()
    rng = np.random.default_rng(8)
    s.white[rng.random(s.white.shape) < 0.06] = 0.0
    ref, w = oracle_state(s)
    rows = np.nonzero((w > 0).any(axis=1))[0]
    cols = np.nonzero((w > 0).any(axis=0))[0]
    r0, r1, c0, c1 = rows[0] + 10, rows[-1] - 10, cols[0] + 10, cols[-1] - 10
    ref_c = np.ascontiguousarray(ref[r0:r1 + 1, c0:c1 + 1])
    w_c = np.ascontiguousarray(w[r0:r1 + 1, c0:c1 + 1])
    s2 = dataclasses.replace(s, origin=(s.origin[0] + int(r0), s.origin[1] + int(c0)), ref_shape=ref_c.shape)
    fams = ("pm_fast", "pm_edge_mma", "pm_edge")
    pxst.profile_enable(True)
    try:
        for f in fams:
            pxst.profile_read(f)
        info = {}
        check_pixel_map(s2, ref_c, w_c, s.dx0, s.u0, (3, 3), True, label="zero white", info=info)
        work = {f: pxst.profile_read(f)[2] for f in fams}
    finally:
        pxst.profile_enable(False)
    zw = ((s.white == 0) & (s.mask > 0)).ravel()
    kg, ko = info["kg"], info["k"]
    assert zw.sum() > 50 and (zw & info["edge"]).sum() > 5, (zw.sum(), (zw & info["edge"]).sum())
    np.testing.assert_array_equal(kg[zw], ko[zw])
    say(f"    zero-white pixels {zw.sum()} (edge {(zw & info['edge']).sum()}), work per family {work}")
    assert work["pm_fast"] > 0 and work["pm_edge_mma"] > 0 and work["pm_edge"] > 0, work


def _edge_band_pixels(H, W, band, n, seed):
    """Sampled pixels within ``band`` pixels of the detector's edges, plus its corners."""
    rng = np.random.default_rng(seed)
    side = rng.integers(0, 4, n)
    a = rng.integers(0, band, n)
    rows = np.where(side == 0, a, np.where(side == 1, H - 1 - a, rng.integers(0, H, n)))
    cols = np.where(side == 2, a, np.where(side == 3, W - 1 - a, rng.integers(0, W, n)))
    rows = np.concatenate([rows, [0, 0, H - 1, H - 1]])
    cols = np.concatenate([cols, [0, W - 1, 0, W - 1]])
    return rows, cols


@pytest.mark.parametrize("name", ["realistic", "divergent"])
def test_pixel_map_edge_tiles_full_size(name):
    """Full-size scans with the oracle's own reference made from the start state (u0, dx0),
    the first search of the benchmark's solve: the reference is valid only where frames
    fell, so the tiles at the detector's border have slow frames (realistic: up to 64 per
    tile over 2 frame blocks; divergent: up to 96 over 7 blocks) and are searched by the
    edge-tile matrix-core kernel.  Sampled pixels in the border bands are checked one by
    one against the oracle; the edge launch must have searched pixels, and the sampled
    set must hold pixels with invalid lookups."""
    s = cached_scan(name)
    say(f"[pixel-map] {name} edge tiles: oracle reference from the start state")
    ref, w = oracle_state(s)
    H, W = s.det
    rows, cols = _edge_band_pixels(H, W, 2 * max(s.window) + 4, 260 if name == "realistic" else 150, 105)
    pxst.profile_enable(True)
    try:
        for f in ("pm_fast", "pm_edge_mma", "pm_edge", "pm_generic"):
            pxst.profile_read(f)
        info = {}
        check_pixel_map(s, ref, w, s.dx0, s.u0, s.window, True, pixels=(rows, cols),
                        label=f"{name} edge tiles", info=info)
        work = {f: pxst.profile_read(f)[2] for f in ("pm_fast", "pm_edge_mma", "pm_edge", "pm_generic")}
    finally:
        pxst.profile_enable(False)
    n_edge = int(info["edge"].sum())
    say(f"    sampled pixels with invalid lookups: {n_edge} of {len(rows)}; work per family {work}")
    assert n_edge >= 20, n_edge
    assert work["pm_edge_mma"] > 0 and work["pm_fast"] > 0, work


def test_pixel_map_high_dynamic_range_reference():
    """A reference with isolated bright pixels, 1 % of them 100x the speckle (the splat
    reference's largest value is about 77x its median): the matrix-core search scales the
    whole reference by one power of two (lookups are multiples of 2^-14 here, against a
    float32 rounding of 6e-8 for a pixel near 1), so ordinary pixels keep the fewest bits
    here.  Sampled pixels, pixels next to the bright ones included: argmin identical up
    to ties, map within 1e-3 px, E_min within the bound that adds W 2^-F to each
    residual's error."""
    spec = ScanSpec(name="hdr", det=(128, 256), n_grid=(7, 7), step=6.0, jitter=0.5,
                    disp_ss=(6.0, 3.0), disp_fs=(6.0, 3.0), window=(6, 6), iters=1, ref=None,
                    ref_sigma=1.5, ref_contrast=0.15, white="gauss", white_sigma=128.0,
                    white_mean=250.0, refine=True, seed=91, bright_frac=0.01, bright_gain=100.0)
    s = make_scan(spec)
    ref, w = oracle_state(s)
    v = w > 0
    assert ref[v].max() > 50 * np.median(ref[v])
    rng = np.random.default_rng(106)
    H, W = s.det
    rows = rng.integers(0, H, 400)
    cols = rng.integers(0, W, 400)
    # detector pixels whose start-state lookup in the middle frame is near a bright pixel
    n = s.n_frames // 2
    pa = np.rint(s.u0[0] - s.dx0[n, 0] - s.origin[0]).astype(int).clip(0, ref.shape[0] - 1)
    pb = np.rint(s.u0[1] - s.dx0[n, 1] - s.origin[1]).astype(int).clip(0, ref.shape[1] - 1)
    near = np.argwhere(ref[pa, pb] > 10 * np.median(ref[v]))[:100]
    rows = np.concatenate([rows, near[:, 0]])
    cols = np.concatenate([cols, near[:, 1]])
    assert fixed_point_step(ref.astype(np.float32), w) == 2.0 ** -14
    check_pixel_map(s, ref, w, s.dx0, s.u0, s.window, True, pixels=(rows, cols), label="high dynamic range",
                    fixed_point=True)


def test_profile_selection_times_only_the_named_family():
    """With a restricted selection only the named family records its launches (without
    device work counters) and the others none; selecting every family again restores
    the counts; the search's results do not depend on the timing."""
    s = random_small_scan(det=(37, 53), n_frames=7, seed=29)
    ref, w = oracle_state(s)
    fams = ("pm_fast", "pm_edge", "pm_generic")
    pxst.profile_enable(True)
    try:
        pxst.profile_select(["pm_fast"])
        for f in fams:
            pxst.profile_read(f)
        a = gpu_pixel_map(s, ref, w, s.dx0, s.u0, (3, 3), True)
        sel = {f: pxst.profile_read(f) for f in fams}
        pxst.profile_select(None)
        b = gpu_pixel_map(s, ref, w, s.dx0, s.u0, (3, 3), True)
        full = {f: pxst.profile_read(f) for f in fams}
    finally:
        pxst.profile_select(None)
        pxst.profile_enable(False)
    assert sel["pm_fast"][1] == 1 and sel["pm_fast"][2] == 0, sel
    assert sel["pm_edge"][1] == 0 and sel["pm_generic"][1] == 0, sel
    assert all(full[f][1] == 1 for f in fams), full
    assert sum(full[f][2] for f in fams) > 0, full
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_pixel_map_deterministic():
    s = random_small_scan(det=(37, 53), n_frames=7, seed=29)
    ref, w = oracle_state(s)
    a = gpu_pixel_map(s, ref, w, s.dx0, s.u0, (3, 3), True)
    b = gpu_pixel_map(s, ref, w, s.dx0, s.u0, (3, 3), True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ----------------------------------------------------------------- translations

def gpu_translations(s, ref, w, u, dx, window, refine):
    sc = dev_scan(s)
    opts = pxst.make_opts(1, (1, 1), True, True, window, refine)
    ws = pxst.alloc_workspace(sc.geom, opts)
    dxo = empty((s.n_frames, 2), torch.float32)
    e = empty((s.n_frames,), torch.float32)
    k = empty((s.n_frames,), torch.int32)
    pxst.update_translations(sc, to_dev(ref.astype(np.float32)), to_dev(w), to_dev(u), to_dev(dx),
                             pxst.make_window(window[0], window[1], refine), dxo, e, k, ws)
    torch.cuda.synchronize()
    return dxo.cpu().numpy(), e.cpu().numpy(), k.cpu().numpy()


def check_translations(s, ref, w, u, dx, window, refine, frames=None, label=""):
    say(f"[translations] {label} det={s.det} N={s.n_frames} window={window} refine={refine}")
    ref32 = ref.astype(np.float32).astype(np.float64)
    dg, eg, kg = gpu_translations(s, ref32, w, u, dx, window, refine)
    frames = range(s.n_frames) if frames is None else frames
    for n in frames:
        do, eo, ko, E = oracle.update_translations(s.frames[n:n + 1], s.white, s.mask, ref32, w, u,
                                                   dx[n:n + 1], s.origin, window, refine,
                                                   return_errors=True)
        if kg[n] != ko[0]:
            flat = E[0].ravel()
            assert kg[n] >= 0 and ko[0] >= 0
            assert abs(flat[kg[n]] - flat[ko[0]]) <= 1e-6 * abs(flat[ko[0]]), (n, kg[n], ko[0])
            continue
        assert np.abs(dg[n] - do[0]).max() <= U_TOL_PX, (n, dg[n], do[0])
        if np.isfinite(eo[0]):
            assert abs(eg[n] - eo[0]) <= ERR_TOL_REL * abs(eo[0]) + 1e-12
    return dg


@pytest.mark.parametrize("refine", [False, True])
def test_translations_tiny(refine):
    s = make_scan(CONFIGS["tiny"])
    ref, w = oracle_state(s)
    u, _, _ = oracle.update_pixel_map(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin,
                                      s.window, False)
    u = u.astype(np.float32)
    rng = np.random.default_rng(3)
    dx = (s.dx0 + rng.uniform(-1.5, 1.5, s.dx0.shape)).astype(np.float32)
    check_translations(s, ref, w, u, dx, (2, 2), refine, label="tiny")


@pytest.mark.parametrize("window", [(1, 1), (0, 2), (2, 1)])
def test_translations_small(window):
    s = random_small_scan(det=(37, 53), n_frames=7, seed=31)
    ref, w = oracle_state(s)
    check_translations(s, ref, w, s.u0, s.dx0, window, True, label=f"small {window}")


def test_translations_exact_recovery():
    s = exact_scan(window=(3, 3))
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u_true, s.dx_true, s.origin,
                                     s.ref_shape)
    rng = np.random.default_rng(6)
    dx_start = (s.dx_true + rng.integers(-2, 3, s.dx_true.shape)).astype(np.float32)
    dg = check_translations(s, ref, w, s.u_true, dx_start, (2, 2), False, label="exact")
    np.testing.assert_array_equal(dg, s.dx_true)


def test_translations_divergent_full_size_sampled():
    """Divergent scan at full size (512x512, 400 frames, +-2 px); 3 frames checked by the oracle."""
    s = cached_scan("divergent")
    ref = s.ref_true
    w = np.ones_like(ref)
    check_translations(s, ref, w, s.u_true, s.dx0, (2, 2), True, frames=[0, 187, 399],
                       label="divergent full size")


# ------------------------------------------------------------------------ errors

def gpu_error(s, ref, w, u, dx, ref_err=True):
    sc = dev_scan(s)
    ws = pxst.alloc_workspace(sc.geom, None)
    H, W = s.det
    pe = empty((H, W), torch.float32)
    fe = empty((s.n_frames,), torch.float64)
    tot = empty((1,), torch.float64)
    re = empty(s.ref_shape, torch.float32) if ref_err else None
    pxst.error(sc, to_dev(ref.astype(np.float32)), to_dev(w), to_dev(u), to_dev(dx), tot, pe, fe, re, ws)
    torch.cuda.synchronize()
    return (pe.cpu().numpy(), fe.cpu().numpy(), float(tot.cpu()[0]),
            re.cpu().numpy() if ref_err else None)


@pytest.mark.parametrize("case", ["tiny", "small_masked"])
def test_error_parity(case):
    s = make_scan(CONFIGS["tiny"]) if case == "tiny" else random_small_scan(det=(37, 53), n_frames=7,
                                                                              seed=41)
    say(f"[error] {case}")
    ref, w = oracle_state(s)
    ref32 = ref.astype(np.float32).astype(np.float64)
    u = (s.u0 + 0.3).astype(np.float32)
    pe, fe, tot, re = gpu_error(s, ref32, w, u, s.dx0)
    o = oracle.calc_error(s.frames, s.white, s.mask, ref32, w, u, s.dx0, s.origin, ref_error=True)
    assert abs(tot - o["total"]) <= ERR_TOL_REL * o["total"]
    np.testing.assert_allclose(fe, o["frame"], rtol=ERR_TOL_REL)
    np.testing.assert_allclose(pe, o["pixel"], rtol=ERR_TOL_REL, atol=1e-6 * o["pixel"].max())
    np.testing.assert_allclose(re, o["ref"], rtol=ERR_TOL_REL, atol=1e-6 * o["ref"].max())


@pytest.mark.parametrize("name", ["realistic", "divergent"])
def test_error_full_size(name):
    """The error pass at the benchmark scans' full size (256x1024 with 121 frames;
    512x512 with 400 frames) and initial state, with the true reference minus two bands
    of invalid pixels (the reference grid is the union of the frames' footprints, so the
    bands are looked up: lookups with all, some and no valid corners all occur): frame
    errors, total and pixel errors against the oracle."""
    s = cached_scan(name)
    ref32 = s.ref_true.astype(np.float32).astype(np.float64)
    w = np.ones_like(ref32)
    w[: ref32.shape[0] // 6, :] = 0.0
    w[:, ref32.shape[1] - ref32.shape[1] // 8:] = 0.0
    say(f"[error] {name} full size")
    pe, fe, tot, _ = gpu_error(s, ref32, w, s.u0, s.dx0, ref_err=False)
    o = oracle.calc_error(s.frames, s.white, s.mask, ref32, w, s.u0, s.dx0, s.origin)
    assert o["total"] > 0
    assert abs(tot - o["total"]) <= ERR_TOL_REL * o["total"]
    np.testing.assert_allclose(fe, o["frame"], rtol=ERR_TOL_REL, atol=1e-9 * o["frame"].max())
    np.testing.assert_allclose(pe, o["pixel"], rtol=ERR_TOL_REL, atol=1e-6 * o["pixel"].max())


def test_maximum_frame_count():
    """The largest frame count the library takes (1920): the reference update, the
    pixel-map search on the matrix cores with 30 frame blocks (the contraction's byte
    classes then combine in float64) and the error evaluation at its largest LDS use,
    each against the oracle on a small detector."""
    s = random_small_scan(det=(16, 24), n_frames=1920, window=(2, 2), seed=61, n_grid=(40, 48), step=1.0)
    say(f"[max frames] det={s.det} N={s.n_frames} ref={s.ref_shape}")
    rg, wg = gpu_reference(s, s.u0, s.dx0)
    ro, wo = oracle_state(s)
    np.testing.assert_array_equal(wg > 0, wo > 0)
    err, _ = ref_rel_error(rg, ro, wo)
    assert err < REF_TOL_REL, err
    check_pixel_map(s, ro, wo, s.dx0, s.u0, (2, 2), True, label="1920 frames")
    ref32 = ro.astype(np.float32).astype(np.float64)
    pe, fe, tot, re = gpu_error(s, ref32, wo, s.u0, s.dx0)
    o = oracle.calc_error(s.frames, s.white, s.mask, ref32, wo, s.u0, s.dx0, s.origin, ref_error=True)
    assert abs(tot - o["total"]) <= ERR_TOL_REL * o["total"]
    np.testing.assert_allclose(fe, o["frame"], rtol=ERR_TOL_REL, atol=1e-9 * o["frame"].max())
    np.testing.assert_allclose(pe, o["pixel"], rtol=ERR_TOL_REL, atol=1e-6 * o["pixel"].max())


# ------------------------------------------------------------------------ solve

def gpu_solve(s, n_iter, window, refine, update_dx=False, tr=(2, 2)):
    sc = dev_scan(s)
    opts = pxst.make_opts(n_iter, window, refine, update_dx, tr)
    ws = pxst.alloc_workspace(sc.geom, opts)
    u = to_dev(s.u0).clone()
    dx = to_dev(s.dx0).clone()
    ref = empty(s.ref_shape, torch.float32)
    w = empty(s.ref_shape, torch.float64)
    h = torch.zeros(max(n_iter, 1), dtype=torch.float64, device="cuda")
    pxst.solve(sc, opts, u, dx, ref, w, h, ws)
    torch.cuda.synchronize()
    return u.cpu().numpy(), dx.cpu().numpy(), ref.cpu().numpy(), w.cpu().numpy(), h.cpu().numpy()


def test_solve_tiny():
    """Main loop (Sec. 2.2), tiny scan, 3 iterations without refinement: the error history,
    the integer map (identical), the final reference, every iteration's state."""
    s = make_scan(CONFIGS["tiny"])
    say("[solve] tiny 3 iterations")
    ug, dg, rg, wg, hg = gpu_solve(s, 3, s.window, False)
    o = oracle.solve(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape, 3, s.window,
                     refine=False)
    np.testing.assert_allclose(hg, o["err_hist"], rtol=ERR_TOL_REL)
    np.testing.assert_array_equal(ug, o["u"].astype(np.float32))
    np.testing.assert_array_equal(wg > 0, o["w"] > 0)
    err, _ = ref_rel_error(rg, o["ref"], o["w"])
    assert err < REF_TOL_REL, err


def loop_scan():
    """Small scan for the loop with the translation update: odd-sized, 1 % masked pixels
    plus a masked border, 1 % zero white-field pixels, translations started up to 0.8 px
    off the truth."""
    s = random_small_scan(det=(48, 40), n_frames=9, seed=51, window=(3, 3))
    s.dx0 = (s.dx0 + np.random.default_rng(2).uniform(-0.8, 0.8, s.dx0.shape)).astype(np.float32)
    return s


@pytest.mark.parametrize("n_iter", [1, 2, 3])
def test_solve_with_translations(n_iter):
    """Main loop with the translation update (Sec. 2.2; Sec. 2.2.3), every iteration held
    to the single-step bar: error history 1e-5 relative, map and translations 1e-3 px at
    every pixel and frame, final reference 1e-5.  (The oracle itself moves by under 1e-4 px
    when its start translations are moved by 1e-5 px, so float32 state differences do not
    grow over these iterations; an argmin taken differently at an exact tie would.)"""
    s = loop_scan()
    say(f"[solve] small with translation update, {n_iter} iterations")
    ug, dg, rg, wg, hg = gpu_solve(s, n_iter, (3, 3), True, True, (1, 1))
    o = oracle.solve(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape, n_iter, (3, 3),
                     refine=True, update_dx=True, tr_window=(1, 1))
    np.testing.assert_allclose(hg, o["err_hist"], rtol=ERR_TOL_REL)
    assert np.abs(dg - o["dx"]).max() < U_TOL_PX, np.abs(dg - o["dx"]).max()
    assert np.abs(ug - o["u"]).max() < U_TOL_PX, np.abs(ug - o["u"]).max()
    # the final reference against the oracle's update from the same (GPU) state: the map
    # agrees to ~1e-4 px, which moves a reference pixel by about its gradient times that
    ro, wo = oracle.update_reference(s.frames, s.white, s.mask, ug, dg, s.origin, s.ref_shape)
    np.testing.assert_array_equal(wg > 0, wo > 0)
    err, _ = ref_rel_error(rg, ro, wo)
    assert err < REF_TOL_REL, err


def test_solve_step_by_step_from_oracle_state():
    """Each of three loop iterations with the translation update, started from the
    oracle's own state (u_k, dx_k): the GPU's reference update, pixel-map search,
    translation search and error evaluation, each fed the oracle's inputs of that step,
    and one whole GPU iteration (solve of one iteration) from the same state, all at the
    single-step bar."""
    s = loop_scan()
    u, dx = s.u0.copy(), s.dx0.copy()
    for k in range(3):
        say(f"[solve] step {k + 1} from the oracle state")
        ro, wo = oracle.update_reference(s.frames, s.white, s.mask, u, dx, s.origin, s.ref_shape)
        rg, wg = gpu_reference(s, u, dx)
        np.testing.assert_array_equal(wg > 0, wo > 0)
        err, _ = ref_rel_error(rg, ro, wo)
        assert err < REF_TOL_REL, (k, err)
        ref32 = ro.astype(np.float32).astype(np.float64)
        check_pixel_map(s, ref32, wo, dx, u, (3, 3), True, label=f"step {k + 1}")
        u1, _, _ = oracle.update_pixel_map(s.frames, s.white, s.mask, ref32, wo, dx, u, s.origin,
                                           (3, 3), True)
        u1 = u1.astype(np.float32)
        check_translations(s, ref32, wo, u1, dx, (1, 1), True, label=f"step {k + 1}")
        dx1, _, _ = oracle.update_translations(s.frames, s.white, s.mask, ref32, wo, u1, dx, s.origin,
                                               (1, 1), True)
        dx1 = dx1.astype(np.float32)
        pe, fe, tot, _ = gpu_error(s, ref32, wo, u1, dx1, ref_err=False)
        oe = oracle.calc_error(s.frames, s.white, s.mask, ref32, wo, u1, dx1, s.origin)
        assert abs(tot - oe["total"]) <= ERR_TOL_REL * oe["total"], (k, tot, oe["total"])
        # one whole iteration of the library's loop from the same state
        s_k = dataclasses.replace(s, u0=u, dx0=dx)
        ug, dg, rg1, wg1, hg = gpu_solve(s_k, 1, (3, 3), True, True, (1, 1))
        assert abs(hg[0] - oe["total"]) <= ERR_TOL_REL * oe["total"], (k, hg[0], oe["total"])
        assert np.abs(ug - u1).max() < U_TOL_PX, (k, np.abs(ug - u1).max())
        assert np.abs(dg - dx1).max() < U_TOL_PX, (k, np.abs(dg - dx1).max())
        u, dx = u1, dx1


def test_solve_resume_with_translations():
    """solve(2) then solve(1) from the returned state equals solve(3) bitwise, with the
    translation update on: no step keeps state between calls or iterations beyond
    (u, dx)."""
    s = loop_scan()
    full = gpu_solve(s, 3, (3, 3), True, True, (1, 1))
    part = gpu_solve(s, 2, (3, 3), True, True, (1, 1))
    s2 = dataclasses.replace(s, u0=part[0], dx0=part[1])
    rest = gpu_solve(s2, 1, (3, 3), True, True, (1, 1))
    for a, b in zip(full[:4], rest[:4]):
        assert np.array_equal(a, b)
    assert full[4][2] == rest[4][0]


def test_solve_resume_equals_full_run():
    """solve(2) then solve(1) from the returned state equals solve(3) bitwise."""
    s = random_small_scan(det=(37, 53), n_frames=7, seed=52)
    full = gpu_solve(s, 3, (3, 2), True)
    part = gpu_solve(s, 2, (3, 2), True)
    s2 = random_small_scan(det=(37, 53), n_frames=7, seed=52)
    s2.u0, s2.dx0 = part[0], part[1]
    rest = gpu_solve(s2, 1, (3, 2), True)
    assert np.array_equal(full[0], rest[0]) and np.array_equal(full[2], rest[2])
    assert full[4][2] == rest[4][0]


def test_solves_from_two_host_threads_on_two_streams():
    """Two solves enqueued at once from two host threads, each on its own stream (the
    loop's second stream and events are shared per device; their enqueueing is
    serialised), give bitwise the results of the same solves run one after the other."""
    import threading
    scans = [random_small_scan(det=(37, 53), n_frames=7, seed=61),
             random_small_scan(det=(40, 48), n_frames=9, seed=62, window=(2, 2))]
    runs = [(s, 3, s.window, True, k == 1) for k, s in enumerate(scans)]
    say("[solve] sequential reference runs")
    want = [gpu_solve(s, n, w, r, update_dx=dxu) for s, n, w, r, dxu in runs]
    say("[solve] two host threads, two streams")
    got = [None, None]
    errors = []

    def work(k):
        try:
            s, n, w, r, dxu = runs[k]
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                sc = dev_scan(s)
                opts = pxst.make_opts(n, w, r, dxu, (2, 2))
                ws = pxst.alloc_workspace(sc.geom, opts)
                u = to_dev(s.u0).clone()
                dx = to_dev(s.dx0).clone()
                ref = empty(s.ref_shape, torch.float32)
                wsum = empty(s.ref_shape, torch.float64)
                h = torch.zeros(n, dtype=torch.float64, device="cuda")
                for _ in range(3):   # several solves in flight per thread
                    u.copy_(to_dev(s.u0))
                    dx.copy_(to_dev(s.dx0))
                    pxst.solve(sc, opts, u, dx, ref, wsum, h, ws, stream=st)
            st.synchronize()
            got[k] = (u.cpu().numpy(), dx.cpu().numpy(), ref.cpu().numpy(), wsum.cpu().numpy(), h.cpu().numpy())
        except Exception as e:   # reported below, in the test's thread
            errors.append(e)

    th = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for k in range(2):
        for a, b in zip(want[k], got[k]):
            assert np.array_equal(a, b), k
