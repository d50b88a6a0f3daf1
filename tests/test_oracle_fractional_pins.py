"""Pins of the fractional-step pixel-map search of the oracle (Sec. 2.2.2, evaluation
at non-integer positions; CPU only)."""
import numpy as np
import pytest

import oracle
from synth import random_small_scan


def test_one_step_is_the_integer_search():
    """steps = 1: the fine grid is the integer grid, so the result is the integer
    search without refinement, value for value."""
    s = random_small_scan(det=(13, 17), n_frames=5, seed=51, window=(2, 3))
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    a = oracle.update_pixel_map(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin, (2, 3), refine=False)
    b = oracle.update_pixel_map_fractional(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin, (2, 3), 1)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_exact_fractional_truth_is_recovered():
    """Noiseless frames rendered by the bilinear model of Sec. 4 at positions on the
    one-third grid (integer reference values that are multiples of 9, W = 1, integer
    translations, so every count is an integer): the fractional search with three steps
    finds the true positions with zero error (up to the rounding of the thirds)."""
    rng = np.random.default_rng(5)
    H, W, N = 9, 11, 6
    Rs, Rf = 24, 26
    ref = 9.0 * rng.integers(1, 40, (Rs, Rf)).astype(np.float64)
    dx = np.array([[0, 0], [2, 1], [-1, 3], [3, -2], [1, 1], [-2, -1]], dtype=np.float64)[:N]
    origin = (-7, -7)
    ii, jj = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    frac = rng.integers(-1, 2, (2, H, W)) / 3.0
    u_true = np.stack([ii, jj]) + frac
    valid = np.ones((Rs, Rf), dtype=bool)
    frames = np.empty((N, H, W))
    for n in range(N):
        g, ok = oracle.bilinear_gather(ref, valid, u_true[0] - dx[n, 0] - origin[0],
                                       u_true[1] - dx[n, 1] - origin[1])
        assert ok.all()
        frames[n] = g
    assert np.allclose(frames, np.round(frames))
    frames = np.round(frames).astype(np.uint16)
    white = np.ones((H, W))
    mask = np.ones((H, W), dtype=np.uint8)
    u_start = np.stack([ii, jj]) + rng.integers(-1, 2, (2, H, W))
    w = np.ones((Rs, Rf))
    uo, eo, ko = oracle.update_pixel_map_fractional(frames, white, mask, ref, w, dx, u_start, origin,
                                                    (1, 1), 3)
    np.testing.assert_allclose(uo, u_true, atol=1e-12)
    assert np.all(eo <= 1e-20)   # zero up to the rounding of m / s


def test_fine_classes_are_shifted_integer_searches():
    """The candidates c + k + q/s of one class q are the integer search with every
    translation moved by -q/s: their errors coincide."""
    s = random_small_scan(det=(11, 14), n_frames=4, seed=52, window=(1, 2))
    ref, w = oracle.update_reference(s.frames, s.white, s.mask, s.u0, s.dx0, s.origin, s.ref_shape)
    st = 3
    _, _, _, E = oracle.update_pixel_map_fractional(s.frames, s.white, s.mask, ref, w, s.dx0, s.u0, s.origin,
                                                    (1, 2), st, return_errors=True)
    for q0 in (-1, 0, 1):
        for q1 in (-1, 0, 1):
            dxq = s.dx0.astype(np.float64) - np.array([q0, q1]) / st
            _, _, _, Eq = oracle.update_pixel_map(s.frames, s.white, s.mask, ref, w, dxq, s.u0, s.origin,
                                                  (1, 2), refine=False, return_errors=True)
            sub = E[(q0 + 1)::st, (q1 + 1)::st]
            np.testing.assert_allclose(sub, Eq, rtol=1e-12, atol=0)


def test_even_steps_rejected():
    with pytest.raises(ValueError):
        oracle.update_pixel_map_fractional(np.zeros((1, 2, 2), np.uint16), np.ones((2, 2)), np.ones((2, 2)),
                                           np.ones((4, 4)), np.ones((4, 4)), np.zeros((1, 2)),
                                           np.zeros((2, 2, 2)), (0, 0), (1, 1), 2)
