"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage it pins.  None of them re-types the oracle's own
formula: they use worked values, closed forms, library routines (scipy), brute
force on tiny inputs, exact special cases and invariants.
"""
import os

import numpy as np
import pytest
from scipy import ndimage, signal

import oracle
from oracle import bruteforce
from synth import exact_scan, make_scan, spec_for, random_small_scan

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Sec. 4, Eq. 4

def test_bilinear_weights_sum_to_one():
    """Sec. 4: the four rectangle areas fill the unit square, so the weights sum to 1."""
    rng = np.random.default_rng(0)
    fa, fb = rng.random(1000), rng.random(1000)
    w = oracle.bilinear_weights(fa, fb)
    np.testing.assert_allclose(sum(w.values()), 1.0, atol=1e-15)
    assert all((v >= 0).all() for v in w.values())


def test_bilinear_worked_values():
    """Sec. 4 Eq. 4 and the masked form: hand-worked values on a 2x2 array."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "bilinear_eq4.txt"))
            if l.strip() and not l.startswith("#")]
    F = np.array([[1.0, 2.0], [3.0, 5.0]])        # F[x, y]
    for r in rows:
        x, y = float(r[0]), float(r[1])
        m00, m10, m01, m11 = (int(v) for v in r[2:6])
        V = np.array([[m00, m01], [m10, m11]], dtype=bool)
        g, ok = oracle.bilinear_gather(F, V, np.array([x]), np.array([y]))
        if r[6] == "nan":
            assert not ok[0]
        else:
            assert ok[0]
            assert abs(g[0] - float(r[6])) < 1e-14, r


def test_gather_matches_map_coordinates():
    """Unmasked interior lookups equal scipy's order-1 spline (plain bilinear)."""
    rng = np.random.default_rng(1)
    F = rng.random((17, 23))
    a = rng.uniform(0, 16, 500)
    b = rng.uniform(0, 22, 500)
    g, ok = oracle.bilinear_gather(F, np.ones_like(F, bool), a, b)
    ref = ndimage.map_coordinates(F, [a, b], order=1)
    assert ok.all()
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-13)


def test_gather_out_of_grid_corners_are_unknown():
    """Corners outside the array are dropped and the rest renormalised (reading of Sec. 4)."""
    F = np.array([[2.0, 4.0], [6.0, 8.0]])
    V = np.ones_like(F, bool)
    g, ok = oracle.bilinear_gather(F, V, np.array([1.5]), np.array([0.25]))
    # only corners (1,0) and (1,1) are in the grid: (0.75*6 + 0.25*8) / 1
    assert ok[0] and abs(g[0] - 6.5) < 1e-14
    g, ok = oracle.bilinear_gather(F, V, np.array([-1.5]), np.array([0.0]))
    assert not ok[0]


def test_splat_single_contribution_gives_ratio():
    """Sec. 2.2.1: one value at a fractional point -> I/W at each touched corner."""
    frames = np.array([[[700]]], dtype=np.uint16)
    white = np.array([[350.0]], np.float32)
    mask = np.ones((1, 1), np.uint8)
    u = np.array([[[3.3]], [[4.8]]], np.float32)
    dx = np.zeros((1, 2), np.float32)
    ref, w = oracle.update_reference(frames, white, mask, u, dx, (0, 0), (8, 8))
    touched = w > 0
    assert touched.sum() == 4
    assert touched[3, 4] and touched[4, 4] and touched[3, 5] and touched[4, 5]
    np.testing.assert_allclose(ref[touched], 2.0, rtol=1e-14)
    assert (ref[~touched] == 0).all()
    np.testing.assert_allclose(w.sum(), 350.0 ** 2, rtol=1e-14)


def test_splat_drops_out_of_grid_corners():
    """Sec. 2.2.1 with the reading for corners outside the reference grid: a point half
    a pixel above the first row adds only to its two in-grid corners (each then holds
    I/W, with weight W^2 times its bilinear share); nothing lands anywhere else, also
    not on a pixel that a second point at an integer position fills on its own."""
    frames = np.array([[[900, 500]]], dtype=np.uint16)
    white = np.array([[300.0, 200.0]], np.float32)
    mask = np.ones((1, 2), np.uint8)
    u = np.array([[[-0.5, 0.0]], [[2.25, 0.0]]], np.float32)
    ref, w = oracle.update_reference(frames, white, mask, u, np.zeros((1, 2), np.float32), (0, 0), (4, 5))
    assert np.argwhere(w > 0).tolist() == [[0, 0], [0, 2], [0, 3]]
    np.testing.assert_allclose(ref[0, 2:4], 3.0, rtol=1e-14)
    np.testing.assert_allclose(w[0, 2:4], 300.0 ** 2 * 0.5 * np.array([0.75, 0.25]), rtol=1e-14)
    assert ref[0, 0] == 2.5 and w[0, 0] == 200.0 ** 2
    assert np.count_nonzero(ref) == 3


def test_identity_map_gives_weighted_mean():
    """Integer identity map and integer translations: I_ref[p] = sum W I / sum W^2 (Sec. 2.2.1).

    With all translations zero this is mean_n(I_n) / W -- the white-field weighted
    merge of the frames (Sec. 1).
    """
    rng = np.random.default_rng(2)
    N, H, W = 5, 6, 7
    frames = rng.integers(0, 3000, (N, H, W)).astype(np.uint16)
    white = rng.uniform(100, 900, (H, W)).astype(np.float32)
    mask = np.ones((H, W), np.uint8)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u = np.stack([ii, jj]).astype(np.float32)
    ref, w = oracle.update_reference(frames, white, mask, u, np.zeros((N, 2), np.float32), (0, 0), (H, W))
    np.testing.assert_allclose(ref, frames.astype(np.float64).mean(0) / white, rtol=1e-12)
    # integer shifts: reference pixel p collects frame n at detector pixel p + dx_n
    dx = np.array([[0, 0], [1, 0], [0, 2], [-1, 1], [2, -1]], np.float32)
    org = (-2, -2)
    ref, w = oracle.update_reference(frames, white, mask, u, dx, org, (H + 4, W + 5))
    num = np.zeros(ref.shape)
    den = np.zeros(ref.shape)
    W64 = white.astype(np.float64)
    for n in range(N):
        p0 = ii - int(dx[n, 0]) - org[0]
        p1 = jj - int(dx[n, 1]) - org[1]
        num[p0, p1] += W64 * frames[n]
        den[p0, p1] += W64 ** 2
    cov = den > 0
    np.testing.assert_array_equal(w > 0, cov)
    np.testing.assert_allclose(ref[cov], num[cov] / den[cov], rtol=1e-12)


def test_splat_then_gather_is_not_invertible():
    """Sec. 4: interpolating onto a grid shifted by a fraction and back loses information."""
    rng = np.random.default_rng(3)
    F = rng.random((12, 12))
    ii, jj = np.meshgrid(np.arange(12.0), np.arange(12.0), indexing="ij")
    a, b = ii + 0.3, jj + 0.6
    num, den = oracle.bilinear_splat((14, 14), a.ravel(), b.ravel(), F.ravel(), np.ones(144))
    moved = np.where(den > 0, num / np.where(den > 0, den, 1), 0)
    back, ok = oracle.bilinear_gather(moved, den > 0, a.ravel(), b.ravel())
    inner = ok.reshape(12, 12)[2:-2, 2:-2]
    diff = np.abs(back.reshape(12, 12) - F)[2:-2, 2:-2][inner]
    assert diff.max() > 1e-3


# --------------------------------------------------------------- Sec. 2.2.2 / 2.2.3

def test_round_half_up_and_float32_edges():
    x = np.array([0.5, -0.5, 1.5, -1.5, 2.4999, -2.5001, 7.0], np.float64)
    np.testing.assert_array_equal(oracle.round_half_up(x), [1, 0, 2, -1, 2, -3, 7])
    # the float32 just below 1/2 stays at 0 (floor(x + 0.5) in float32 would give 1)
    x32 = np.nextafter(np.float32(0.5), np.float32(0))
    assert np.float32(np.floor(x32 + np.float32(0.5))) == 1.0
    assert oracle.round_half_up(np.float64(x32)) == 0.0
    # the same in float64: the double just below 1/2 plus 1/2 rounds to 1 in float64
    x64 = np.nextafter(0.5, 0.0)
    assert np.floor(x64 + 0.5) == 1.0
    assert oracle.round_half_up(x64) == 0.0 and oracle.round_half_up(-x64) == 0.0


def test_quadratic_refine_exact_on_quadrics():
    """The 3x3 paraboloid fit (Sec. 2.2.2) returns the exact vertex of any convex quadric."""
    rng = np.random.default_rng(4)
    x = np.array([-1.0, 0.0, 1.0])
    X, Y = np.meshgrid(x, x, indexing="ij")
    for _ in range(200):
        A = rng.uniform(0.5, 3.0)
        C = rng.uniform(0.5, 3.0)
        B = rng.uniform(-1, 1) * np.sqrt(A * C) * 0.9 * 2
        x0, y0 = rng.uniform(-0.5, 0.5, 2)
        E = 7.0 + A * (X - x0) ** 2 + B * (X - x0) * (Y - y0) + C * (Y - y0) ** 2
        ox, oy = oracle.quadratic_refine(E)
        assert abs(ox - x0) < 1e-12 and abs(oy - y0) < 1e-12
    # a maximum and a saddle are rejected
    assert oracle.quadratic_refine(-(X ** 2 + Y ** 2)) == (0.0, 0.0)
    assert oracle.quadratic_refine(X ** 2 - Y ** 2) == (0.0, 0.0)
    # also when the maximum's stationary point lies off the centre
    assert oracle.quadratic_refine(-((X - 0.2) ** 2 + 2.0 * (Y + 0.1) ** 2)) == (0.0, 0.0)
    # vertex outside the cell is clamped
    ox, oy = oracle.quadratic_refine((X - 0.9) ** 2 + (Y + 2.0) ** 2)
    assert ox == 0.5 and oy == -0.5
    from oracle.pxst_oracle import parabola_refine
    for x0 in (-0.4, 0.0, 0.3):
        e = [(k - x0) ** 2 * 2.0 + 1.0 for k in (-1, 0, 1)]
        assert abs(parabola_refine(*e) - x0) < 1e-14


def _exact_state(s):
    """Reference made from the true (integer) map and translations of an exact scan."""
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u_true, s.dx_true, s.origin,
                                     s.ref_shape)
    return ref, w


def test_exact_truth_reproduces_reference_and_zero_error():
    """Integer u and dx with noiseless integer frames: Eq. 3 holds exactly, so the
    reference equals the truth where it is covered and the total error is 0."""
    s = exact_scan()
    ref, w = _exact_state(s)
    cov = w > 0
    np.testing.assert_allclose(ref[cov], s.ref_true[cov], rtol=1e-13)
    e0 = oracle.calc_error(s.frames, s.white, s.mask, ref, w, s.u_true, s.dx_true, s.origin)
    u_off = s.u_true.copy()
    u_off[1] += 1.0
    e1 = oracle.calc_error(s.frames, s.white, s.mask, ref, w, u_off, s.dx_true, s.origin)
    assert e1["total"] > 0
    assert e0["total"] <= 1e-12 * e1["total"]


def test_pixel_map_recovers_integer_truth():
    """Sec. 2.2.2 with refinement off: the true integer map is the unique minimiser."""
    s = exact_scan(window=(3, 3))
    ref, w = _exact_state(s)
    rng = np.random.default_rng(5)
    u_start = s.u_true + rng.integers(-2, 3, s.u_true.shape).astype(np.float32)
    u, e, k = oracle.update_pixel_map(s.frames, s.white, s.mask, ref, w, s.dx_true, u_start,
                                      s.origin, (3, 3), refine=False)
    # the minimum is the exact fit everywhere; at the detector border a candidate whose
    # lookups are valid in only a few frames can tie with it, so equality is required
    # away from the border
    assert np.all(e <= 1e-20)
    b = 4
    np.testing.assert_array_equal(u[:, b:-b, b:-b], s.u_true[:, b:-b, b:-b])


def test_translations_recover_integer_truth():
    """Sec. 2.2.3: integer translations are recovered exactly from a +-2 px start error."""
    s = exact_scan(window=(3, 3))
    ref, w = _exact_state(s)
    rng = np.random.default_rng(6)
    dx_start = s.dx_true + rng.integers(-2, 3, s.dx_true.shape).astype(np.float32)
    dx, e, k = oracle.update_translations(s.frames, s.white, s.mask, ref, w, s.u_true, dx_start,
                                          s.origin, (2, 2), refine=False)
    np.testing.assert_array_equal(dx, s.dx_true)


def test_translation_errors_equal_fft_block_matching():
    """Identity integer map, all lookups valid: the translation error numerator is the
    sum of squared differences, which FFT correlation (scipy) computes independently."""
    rng = np.random.default_rng(7)
    H, W, T = 9, 11, 2
    ref = rng.uniform(0.5, 1.5, (H + 2 * T + 4, W + 2 * T + 4))
    white = rng.uniform(50, 150, (H, W)).astype(np.float32)
    frames = rng.integers(10, 300, (3, H, W)).astype(np.uint16)
    mask = np.ones((H, W), np.uint8)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u = np.stack([ii, jj]).astype(np.float32)
    dx = np.array([[0, 0], [1, -1], [-1, 2]], np.float32)
    org = (-(T + 3), -(T + 3))
    _, _, _, E = oracle.update_translations(frames, white, mask, ref, np.ones_like(ref), u, dx, org,
                                            (T, T), refine=False, return_errors=True)
    W64 = white.astype(np.float64)
    for n in range(3):
        I = frames[n].astype(np.float64)
        var = ((I - W64) ** 2).sum()
        # lookup of pixel (i, j) under shift s: ref[i - dx - s - org]
        p0 = -int(dx[n, 0]) - org[0]
        p1 = -int(dx[n, 1]) - org[1]
        sub = ref[p0 - T:p0 + H + T, p1 - T:p1 + W + T]        # rows i - s for s in [-T, T]
        c1 = signal.fftconvolve(sub, (W64 * I)[::-1, ::-1], mode="valid")
        c2 = signal.fftconvolve(sub ** 2, (W64 ** 2)[::-1, ::-1], mode="valid")
        ssd = (I ** 2).sum() - 2 * c1 + c2                      # indexed by T - s
        ssd = ssd[::-1, ::-1]                                   # now indexed by s + T
        np.testing.assert_allclose(E[n] * var, ssd, rtol=1e-9)


def test_vectorised_matches_bruteforce_8x8():
    """Explicit loops of Sec. 2.2.1 / 2.2.2 equal the vectorised oracle on an 8x8 scan."""
    s = random_small_scan(det=(8, 8), n_frames=4, window=(2, 1), mask="parity", zero_white=False,
                          seed=31)
    m = s.mask.copy()
    m[3, 4] = 0
    m[1:7, 1:7] = 1
    m[2, 5] = 0
    ref, w = oracle.update_reference(s.frames, s.white, m, s.u0, s.dx0, s.origin, s.ref_shape)
    R, wb = bruteforce.make_reference(s.frames.tolist(), s.white.tolist(), m.tolist(),
                                      s.u0.tolist(), s.dx0.tolist(), s.origin, s.ref_shape)
    np.testing.assert_allclose(ref, np.array(R), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(w, np.array(wb), rtol=1e-12)
    ref32 = ref.astype(np.float32).astype(np.float64)
    # a partly empty reference exercises the masked lookups
    w2 = w.copy()
    w2[:, : s.ref_shape[1] // 2 - 2] = 0
    u, e, k = oracle.update_pixel_map(s.frames, s.white, m, ref32, w2, s.dx0, s.u0, s.origin, (2, 1),
                                      refine=False)
    bf = bruteforce.pixel_map(s.frames.tolist(), s.white.tolist(), m.tolist(), ref32.tolist(),
                              w2.tolist(), s.dx0.tolist(), s.u0.tolist(), s.origin, 2, 1)
    for i in range(8):
        for j in range(8):
            b0, b1, be, bk = bf[i][j]
            assert k[i, j] == bk
            assert u[0, i, j] == b0 and u[1, i, j] == b1
            if np.isfinite(be):
                assert abs(e[i, j] - be) <= 1e-12 * abs(be)
            else:
                assert not np.isfinite(e[i, j])


def test_masked_pixels_keep_their_map():
    s = random_small_scan(det=(12, 10), n_frames=3, window=(2, 2), seed=41)
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    u, e, k = oracle.update_pixel_map(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin,
                                      (2, 2))
    bad = s.mask == 0
    assert bad.any()
    np.testing.assert_array_equal(u[:, bad], s.u0[:, bad])
    assert np.all(np.isinf(e[bad])) and np.all(k[bad] == -1)


def _rendered_scan(offsets_u=None, offsets_dx=None, seed=11):
    """Noiseless float frames of a smooth speckle reference, rendered with scipy's
    order-1 spline at fractional true positions (a routine neither side uses)."""
    rng = np.random.default_rng(seed)
    H, W, N = 14, 16, 16
    F = ndimage.gaussian_filter(rng.standard_normal((H + 24, W + 24)), 2.0, mode="wrap")
    F = 1.0 + 0.2 * F / F.std()
    white = np.full((H, W), 1000.0)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u_id = np.stack([ii, jj]).astype(np.float64)
    a, b = np.meshgrid(np.arange(4) - 1.5, np.arange(4) - 1.5, indexing="ij")
    dx_grid = np.round(np.stack([3 * a.ravel(), 3 * b.ravel()], 1))
    u_true = u_id if offsets_u is None else u_id + offsets_u
    dx_true = dx_grid if offsets_dx is None else dx_grid + offsets_dx
    org = (-12, -12)
    frames = np.stack([white * ndimage.map_coordinates(
        F, [u_true[0] - dx_true[n, 0] - org[0], u_true[1] - dx_true[n, 1] - org[1]], order=1)
        for n in range(N)])
    return F, white, np.ones((H, W), np.uint8), u_id, dx_grid, u_true, dx_true, org


def test_pixel_map_refinement_moves_towards_truth():
    """Sec. 2.2.2, paraboloid refinement: with the truth 0.3 px (slow axis) and 0.2 px
    (fast axis) off the integer grid, in signs alternating between pixels, the integer
    search lands on the nearest grid point and the refinement must move each axis
    towards the truth (a wrong sign or swapped axes moves it away)."""
    H, W = 14, 16
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    sgn = np.where((ii + jj) % 2 == 0, 1.0, -1.0)
    F, white, mask, u_id, dx, u_true, _, org = _rendered_scan(np.stack([0.3 * sgn, -0.2 * sgn]))
    frames = np.stack([white * ndimage.map_coordinates(
        F, [u_true[0] - dx[n, 0] - org[0], u_true[1] - dx[n, 1] - org[1]], order=1) for n in range(dx.shape[0])])
    u_int, _, _ = oracle.update_pixel_map(frames, white, mask, F, np.ones_like(F), dx, u_id, org, (2, 2),
                                          refine=False)
    np.testing.assert_array_equal(u_int, u_id)            # nearest grid point
    u_ref, _, _ = oracle.update_pixel_map(frames, white, mask, F, np.ones_like(F), dx, u_id, org, (2, 2),
                                          refine=True)
    d = np.abs(u_ref - u_true)
    for ax, t in ((0, 0.3), (1, 0.2)):
        assert d[ax].mean() < 0.4 * t, (ax, d[ax].mean())
        assert np.mean(d[ax] < t) > 0.9, (ax, np.mean(d[ax] < t))


def test_translation_refinement_moves_towards_truth():
    """Sec. 2.2.3: frames rendered with translations 0.3 px / 0.2 px off the integer
    start, in signs that differ between frames and axes; the integer search keeps the
    start and the refined translation of every frame is closer to the truth on each
    axis separately."""
    N = 16
    off = np.stack([np.where(np.arange(N) % 2 == 0, 0.3, -0.3), np.where(np.arange(N) % 3 == 0, -0.2, 0.2)], 1)
    F, white, mask, u_id, dx, _, dx_true, org = _rendered_scan(offsets_dx=off)
    frames = np.stack([white * ndimage.map_coordinates(
        F, [u_id[0] - dx_true[n, 0] - org[0], u_id[1] - dx_true[n, 1] - org[1]], order=1) for n in range(N)])
    d_int, _, _ = oracle.update_translations(frames, white, mask, F, np.ones_like(F), u_id, dx, org, (1, 1),
                                             refine=False)
    np.testing.assert_array_equal(d_int, dx)
    d_ref, _, _ = oracle.update_translations(frames, white, mask, F, np.ones_like(F), u_id, dx, org, (1, 1),
                                             refine=True)
    assert np.all(np.abs(d_ref - dx_true) < 0.5 * np.abs(off)), np.abs(d_ref - dx_true)


def _constant_band_case():
    """Reference of constant value c with an invalid band; frames kappa c W everywhere.
    Every valid lookup gives g = c, so each term is r = c W (kappa - 1) against
    v = W (kappa c - 1) and any ratio of sums over one set of terms is
    c^2 (kappa - 1)^2 / (kappa c - 1)^2, whichever terms the band removes."""
    c, kappa = 1.3, 1.1
    H, W, N = 9, 11, 3
    rng = np.random.default_rng(19)
    white = rng.uniform(200, 900, (H, W))
    frames = np.broadcast_to(kappa * c * white, (N, H, W)).copy()
    ref = np.full((H + 10, W + 10), c)
    w = np.ones_like(ref)
    w[:, 8:11] = 0
    ref[:, 8:11] = 0
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u = np.stack([ii, jj]).astype(np.float64) + 0.25
    dx = np.array([[0.0, 0.0], [1.0, -1.0], [-1.0, 2.0]])
    return frames, white, np.ones((H, W), np.uint8), ref, w, u, dx, (-5, -5), c * c * (kappa - 1) ** 2 / (kappa * c - 1) ** 2


def test_translation_error_is_ratio_over_valid_pixels():
    """Sec. 2.2.3 (the ratio of Sec. 2.2.2 with the sums over pixels): both sums run
    over the same set of pixels with a valid lookup, so the closed-form ratio holds for
    every shift although the band removes a different set of pixels for each."""
    frames, white, mask, ref, w, u, dx, org, E0 = _constant_band_case()
    _, _, _, E = oracle.update_translations(frames, white, mask, ref, w, u, dx, org, (2, 2), refine=False,
                                            return_errors=True)
    np.testing.assert_allclose(E, E0, rtol=1e-12)
    # the band does remove lookups: a lookup column inside it exists for some shift
    cols = np.floor(u[1] - dx[0, 1] - org[1]).astype(int)
    assert any(((cols - s >= 7) & (cols - s <= 10)).any() for s in range(-2, 3))


def test_pixel_map_error_is_ratio_over_valid_frames():
    """Sec. 2.2.2: err and var are summed over the frames whose lookup is valid (the
    reading of var's candidate index), so the closed-form ratio holds for every
    candidate with at least one valid frame."""
    frames, white, mask, ref, w, u, dx, org, E0 = _constant_band_case()
    _, e, k, E = oracle.update_pixel_map(frames, white, mask, ref, w, dx, u, org, (2, 2), refine=False,
                                         return_errors=True)
    fin = np.isfinite(E)
    assert fin.mean() > 0.5
    np.testing.assert_allclose(E[fin], E0, rtol=1e-12)


def test_zero_variance_perfect_fit_is_zero_error():
    """Reading of Sec. 2.2.2 for var = 0: frames equal to the white-field against a
    reference of ones fit perfectly with no variance; the error is 0 (a perfect fit),
    not undefined, so every candidate ties at 0 and the first is taken; the same in
    the translation search."""
    H, W, N = 5, 6, 3
    white = np.full((H, W), 250.0, np.float32)
    frames = np.full((N, H, W), 250, np.uint16)
    mask = np.ones((H, W), np.uint8)
    ref = np.ones((H + 12, W + 12))
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u = np.stack([ii, jj]).astype(np.float32)
    dx = np.zeros((N, 2), np.float32)
    u1, e, k = oracle.update_pixel_map(frames, white, mask, ref, np.ones_like(ref), dx, u, (-6, -6), (2, 1),
                                       refine=False)
    assert np.all(e == 0) and np.all(k == 0)
    np.testing.assert_array_equal(u1[0], ii - 2.0)
    np.testing.assert_array_equal(u1[1], jj - 1.0)
    d1, e, k = oracle.update_translations(frames, white, mask, ref, np.ones_like(ref), u, dx, (-6, -6), (1, 1),
                                          refine=False)
    assert np.all(e == 0) and np.all(k == 0)
    np.testing.assert_array_equal(d1, np.full((N, 2), -1.0))


# ----------------------------------------------------------------------- Sec. 2.2.4

def test_error_equals_frames_times_search_minimum():
    """Sec. 2.2.4 vs Sec. 2.2.2: at an interior pixel the pixel error of the map the
    search returns is N times the search's minimum (both normalise by sum (I-W)^2)."""
    s = make_scan(spec_for("tiny", det=(20, 24), ref=None, n_grid=(2, 3), seed=9,
                           disp_ss=(2.0, 1.0), disp_fs=(2.0, 1.0)))
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    u, e, k = oracle.update_pixel_map(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin,
                                      s.window, refine=False)
    r = oracle.calc_error(s.frames, s.white, s.mask, ref, w, u, s.dx0, s.origin)
    N = s.n_frames
    inner = np.zeros_like(e, bool)
    inner[5:-5, 5:-5] = True
    inner &= np.isfinite(e)
    np.testing.assert_allclose(r["pixel"][inner], N * e[inner], rtol=1e-10)
    assert abs(r["total"] - r["frame"].sum()) <= 1e-9 * r["total"]
    assert abs(r["total"] - r["pixel"].sum()) <= 1e-9 * r["total"]


def test_sigma2_is_state_independent_and_zero_at_whitefield():
    s = random_small_scan(det=(9, 11), n_frames=4, seed=51, zero_white=False)
    a = oracle.pixel_variance(s.frames, s.white, s.mask)
    frames = np.broadcast_to(np.round(s.white).astype(np.uint16), s.frames.shape)
    b = oracle.pixel_variance(frames, np.round(s.white), s.mask)
    assert np.all(b == 0) and np.all(a[s.mask > 0] > 0)


def test_reference_plane_error_single_and_two_contributions():
    """Sec. 2.2.4, error mapped to the reference plane "the same way the reference is
    formed": a reference pixel reached by a single (frame, pixel) term holds that term's
    error whatever its bilinear weight; one reached by two terms at integer positions
    holds their plain mean (the reading: weights omega M, not omega M W).

    1x2 detector, pixels A and B with different white-field values, two frames shifted
    by one pixel along the fast axis: node 1 receives (A, frame 0) and (B, frame 1),
    node 2 only (B, frame 0), node 0 only (A, frame 1)."""
    rng = np.random.default_rng(17)
    frames = rng.integers(200, 900, (2, 1, 2)).astype(np.uint16)
    white = np.array([[300.0, 700.0]], np.float32)
    mask = np.ones((1, 2), np.uint8)
    u = np.array([[[0.0, 0.0]], [[0.0, 1.0]]], np.float32)
    dx = np.array([[0.0, 0.0], [0.0, 1.0]], np.float32)
    ref = rng.uniform(0.5, 1.5, (2, 4))
    r = oracle.calc_error(frames, white, mask, ref, np.ones_like(ref), u, dx, (0, -1), ref_error=True)
    e_B0, e_A1 = r["ref"][0, 2], r["ref"][0, 0]
    e_A0 = r["pixel"][0, 0] - e_A1
    e_B1 = r["pixel"][0, 1] - e_B0
    assert e_A0 > 0 and e_B1 > 0 and abs(e_A0 - e_B1) > 0.1 * max(e_A0, e_B1)
    np.testing.assert_allclose(r["frame"], [e_A0 + e_B0, e_A1 + e_B1], rtol=1e-12)
    np.testing.assert_allclose(r["ref"][0, 1], 0.5 * (e_A0 + e_B1), rtol=1e-12)
    assert np.all(r["ref"][1] == 0) and r["ref"][0, 3] == 0
    # a single term at a fractional position: every touched pixel holds its error
    f1 = np.array([[[640]]], np.uint16)
    w1 = np.array([[400.0]], np.float32)
    u1 = np.array([[[0.3]], [[1.6]]], np.float32)
    r1 = oracle.calc_error(f1, w1, np.ones((1, 1), np.uint8), ref, np.ones_like(ref), u1,
                           np.zeros((1, 2), np.float32), (0, 0), ref_error=True)
    touched = r1["ref"] != 0
    assert touched.sum() == 4
    np.testing.assert_allclose(r1["ref"][touched], r1["total"], rtol=1e-12)


def test_error_excludes_invalid_lookups():
    """Sec. 2.2.4 with the masked interpolation of Sec. 4: a lookup with no valid corner
    contributes nothing.  On an exact scan at its integer truth every valid lookup fits
    exactly, so with a band of the reference made invalid the total stays 0; counting
    the band's lookups (as if their value were 0) would add I^2 / sigma^2 > 0."""
    s = exact_scan()
    ref, w = _exact_state(s)
    w = w.copy()
    band = slice(ref.shape[1] // 2 - 2, ref.shape[1] // 2 + 2)
    w[:, band] = 0
    ref = np.where(w > 0, ref, 0.0)
    hits = 0
    for n in range(s.n_frames):
        cols = np.rint(s.u_true[1] - s.dx_true[n, 1] - s.origin[1]).astype(int)
        hits += int(((cols >= band.start) & (cols < band.stop)).sum())
    assert hits > 0
    e0 = oracle.calc_error(s.frames, s.white, s.mask, ref, w, s.u_true, s.dx_true, s.origin)
    u_off = s.u_true.copy()
    u_off[1] += 1.0
    e1 = oracle.calc_error(s.frames, s.white, s.mask, ref, w, u_off, s.dx_true, s.origin)
    assert e1["total"] > 0 and e0["total"] <= 1e-12 * e1["total"]


# ------------------------------------------------------------------------- Sec. 2.2

def test_main_loop_error_decreases_on_noiseless_scan():
    """Sec. 2.2: on a noiseless scan the total error falls over the first iterations
    (the paper reports the same trend on measured data; convergence is not guaranteed)."""
    s = make_scan(spec_for("tiny", ref=None, seed=12), variant="noiseless")
    out = oracle.solve(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape, 3, (4, 4),
                       refine=True)
    h = out["err_hist"]
    assert h[-1] < h[0]
    def dist(u):  # map error with the common offset removed (u + c, dx + c is the same model)
        d = (u - s.u_true)[:, 4:-4, 4:-4]
        return np.abs(d - d.mean(axis=(1, 2), keepdims=True)).mean()
    assert dist(out["u"]) < dist(s.u0)


def test_ties_take_the_first_candidate():
    """Reading of Sec. 2.2.2 (order of the window loops): on a constant reference every
    candidate has the same error, and the first one (slow-scan offset outer) is taken."""
    rng = np.random.default_rng(8)
    N, H, W = 3, 5, 6
    frames = rng.integers(50, 150, (N, H, W)).astype(np.uint16)
    white = np.full((H, W), 100.0, np.float32)
    mask = np.ones((H, W), np.uint8)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u = np.stack([ii, jj]).astype(np.float32) + 0.25
    ref = np.ones((H + 12, W + 12))
    u1, e, k = oracle.update_pixel_map(frames, white, mask, ref, np.ones_like(ref), np.zeros((N, 2)),
                                       u, (-6, -6), (2, 3), refine=False)
    assert np.all(k == 0)
    np.testing.assert_array_equal(u1[0], ii - 2.0)
    np.testing.assert_array_equal(u1[1], jj - 3.0)
    dx, e, k = oracle.update_translations(frames, white, mask, ref, np.ones_like(ref), u,
                                          np.zeros((N, 2), np.float32), (-6, -6), (1, 2), refine=False)
    assert np.all(k == 0)
    np.testing.assert_array_equal(dx, np.tile([[-1.0, -2.0]], (N, 1)))
