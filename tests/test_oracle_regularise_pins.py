"""Pins of the regularisation oracle (Sec. 2.2.2, "sigma" and "integrate"; CPU only).

The filter is checked against scipy's Gaussian filter (an independent library); the
least-squares integration against scipy's sparse least-squares solver on the explicit
difference matrix, against closed forms (gradient fields of quadratic potentials are
reproduced exactly) and against an invariant (the result is curl-free).
"""
import numpy as np
import pytest
from scipy import ndimage, sparse
from scipy.sparse.linalg import lsqr

from oracle import regularise as reg


def _field(shape, seed):
    rng = np.random.default_rng(seed)
    H, W = shape
    ii, jj = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    u = np.stack([ii + 3.0 * np.sin(jj / 5.0) + rng.normal(0, 0.3, (H, W)),
                  jj + 2.0 * np.cos(ii / 7.0) + rng.normal(0, 0.3, (H, W))])
    return u


@pytest.mark.parametrize("sigma", [0.7, 1.0, 2.5, 5.0])
def test_filter_matches_scipy_gaussian(sigma):
    """Sec. 2.2.2 "sigma": the filter reading equals scipy.ndimage.gaussian_filter with
    nearest-pixel boundaries and a 4-sigma truncation."""
    u = _field((23, 31), 1)
    got = reg.gaussian_filter_map(u, sigma)
    for c in range(2):
        want = ndimage.gaussian_filter(u[c], sigma, mode="nearest", truncate=4.0)
        np.testing.assert_allclose(got[c], want, rtol=0, atol=1e-12)


def test_filter_zero_sigma_and_constant_field():
    """No filtering at sigma 0; a constant map is a fixed point at any sigma."""
    u = _field((9, 12), 2)
    np.testing.assert_array_equal(reg.gaussian_filter_map(u, 0.0), u)
    c = np.full((2, 9, 12), 3.25)
    np.testing.assert_allclose(reg.gaussian_filter_map(c, 3.0), c, atol=1e-13)


def _difference_matrix(H, W):
    """Explicit forward-difference operator (rows: axis-0 differences, then axis-1)."""
    n = H * W
    idx = np.arange(n).reshape(H, W)
    rows, cols, vals = [], [], []
    r = 0
    for i in range(H - 1):
        for j in range(W):
            rows += [r, r]; cols += [idx[i + 1, j], idx[i, j]]; vals += [1.0, -1.0]; r += 1
    for i in range(H):
        for j in range(W - 1):
            rows += [r, r]; cols += [idx[i, j + 1], idx[i, j]]; vals += [1.0, -1.0]; r += 1
    return sparse.csr_matrix((vals, (rows, cols)), shape=(r, n))


@pytest.mark.parametrize("shape", [(7, 9), (12, 5), (3, 3), (2, 6)])
def test_potential_is_the_least_squares_solution(shape):
    """Sec. 2.2.2 "integrate": the CG potential equals scipy's sparse least-squares
    solution of the difference equations (both taken with zero mean)."""
    H, W = shape
    u = _field(shape, 3)
    t0 = 0.5 * (u[0, 1:, :] + u[0, :-1, :])
    t1 = 0.5 * (u[1, :, 1:] + u[1, :, :-1])
    D = _difference_matrix(H, W)
    sol = lsqr(D, np.concatenate([t0.ravel(), t1.ravel()]), atol=1e-15, btol=1e-15,
               iter_lim=100000)[0].reshape(H, W)
    sol -= sol.mean()
    phi = reg.integrate_potential(u)
    np.testing.assert_allclose(phi, sol, atol=1e-8)


def test_direct_solution_equals_cg():
    """The DCT solution of the normal equations equals the CG one."""
    u = _field((21, 34), 4)
    np.testing.assert_allclose(reg.integrate_map_direct(u), reg.integrate_map(u), atol=1e-9)


@pytest.mark.parametrize("shape", [(16, 24), (5, 3), (3, 40)])
def test_gradient_fields_of_quadratics_are_reproduced(shape):
    """A sampled gradient of a quadratic potential is already irrotational: the
    trapezoid targets are exact differences of the potential and the second-order
    differences return the gradient, so the map comes back unchanged."""
    H, W = shape
    ii, jj = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    a, b, c, d, e = 0.013, -0.007, 0.021, 1.5, -0.75
    u = np.stack([2 * a * ii + b * jj + d + ii, b * ii + 2 * c * jj + e + jj])
    np.testing.assert_allclose(reg.integrate_map(u), u, atol=1e-8)
    np.testing.assert_allclose(reg.integrate_map_direct(u), u, atol=1e-9)


def test_result_is_curl_free():
    """The integrated map is the gradient of one function: zero discrete curl inside."""
    u = _field((25, 30), 5)
    v = reg.integrate_map_direct(u)
    assert np.abs(reg.curl(u)).max() > 0.05
    np.testing.assert_allclose(reg.curl(v), 0.0, atol=1e-9)


def test_single_row_keeps_the_other_component():
    """An axis of one pixel has no differences: that component is kept; the other is
    the 1-D integration."""
    u = _field((1, 17), 6)
    v = reg.integrate_map(u)
    np.testing.assert_array_equal(v[0], u[0])
    ref = reg.integrate_map_direct(u)
    np.testing.assert_allclose(v, ref, atol=1e-9)


def test_filter_then_integrate_order():
    """regularise_pixel_map filters first, then integrates."""
    u = _field((15, 18), 7)
    want = reg.integrate_map_direct(reg.gaussian_filter_map(u, 1.5))
    np.testing.assert_allclose(reg.regularise_pixel_map(u, 1.5, True, direct=True), want, atol=0)
