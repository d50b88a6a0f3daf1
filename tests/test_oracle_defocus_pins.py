"""Pins of the defocus-by-registration sweep of the oracle (Sec. 2.1; CPU only)."""
import numpy as np

import oracle


def test_contrast_closed_forms():
    """Contrast = variance / mean^2 over the weighted pixels: 0 for a constant image; for
    a two-level image with levels a and b in equal numbers, ((a-b)/(a+b))^2."""
    w = np.ones((6, 8))
    assert oracle.reference_contrast(np.full((6, 8), 3.5), w) == 0.0
    img = np.where(np.arange(48).reshape(6, 8) % 2 == 0, 2.0, 6.0)
    np.testing.assert_allclose(oracle.reference_contrast(img, w), ((6.0 - 2.0) / 8.0) ** 2, rtol=1e-14)
    # unweighted pixels do not count
    w2 = w.copy()
    w2[:, :4] = 0
    img2 = img.copy()
    img2[:, :4] = 1000.0
    np.testing.assert_allclose(oracle.reference_contrast(img2, w2), ((6.0 - 2.0) / 8.0) ** 2, rtol=1e-14)


def test_unit_scale_is_the_identity_map():
    u = oracle.linear_map((5, 7), (1.0, 1.0))
    ii, jj = np.meshgrid(np.arange(5.0), np.arange(7.0), indexing="ij")
    np.testing.assert_array_equal(u, np.stack([ii, jj]))
    v = oracle.linear_map((5, 7), (0.5, 2.0), centre=(0.0, 3.0))
    np.testing.assert_array_equal(v, np.stack([0.5 * ii, 3.0 + 2.0 * (jj - 3.0)]))


def _magnified_scan(s_true, seed=3):
    """Noiseless frames of a smooth random reference (speckle of about 2 px) seen through
    the linear map of s_true, translated by integer steps (the forward model of Eq. 3)."""
    from scipy import ndimage
    rng = np.random.default_rng(seed)
    H, W = 40, 44
    Rs, Rf = 110, 116
    ref = 100.0 + 400.0 * ndimage.gaussian_filter(rng.random((Rs, Rf)), 2.0, mode="wrap")
    origin = (-35, -35)
    g = np.array([[a, b] for a in (0, 10, 20, 30) for b in (0, 10, 20, 30)], dtype=np.float64)
    N = g.shape[0]
    u = oracle.linear_map((H, W), s_true)
    valid = np.ones((Rs, Rf), dtype=bool)
    frames = np.empty((N, H, W))
    for n in range(N):
        v, ok = oracle.bilinear_gather(ref, valid, u[0] - g[n, 0] - origin[0], u[1] - g[n, 1] - origin[1])
        assert ok.all()
        frames[n] = v
    return np.round(frames).astype(np.uint16), np.ones((H, W)), np.ones((H, W), np.uint8), g, origin, (Rs, Rf)


def test_true_magnification_has_the_greatest_contrast():
    """Sec. 2.1: a wrong magnification misregisters the frames and blurs the reference; the
    sweep picks the scale the frames were rendered with."""
    frames, white, mask, dx, origin, shape = _magnified_scan((1.1, 0.9))
    scales = [(a, b) for a in (1.0, 1.05, 1.1, 1.15, 1.2) for b in (0.8, 0.85, 0.9, 0.95, 1.0)]
    c, best = oracle.defocus_sweep(frames, white, mask, dx, origin, shape, scales)
    assert scales[best] == (1.1, 0.9), (scales[best], c)
    # contrast falls off with the misregistration along each axis
    c2 = c.reshape(5, 5)
    assert np.all(np.diff(c2[:3, 2]) > 0) and np.all(np.diff(c2[2:, 2]) < 0)
    assert np.all(np.diff(c2[2, :3]) > 0) and np.all(np.diff(c2[2, 2:]) < 0)
