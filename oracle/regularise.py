"""FP64 CPU oracle of the pixel-map regularisation -- test infrastructure only.

Only the tests, the entry module's smoke check and the benchmark's CPU-baseline leg
may import this file.  Sec. 2.2.2 ends with two optional steps applied to the pixel
map after the search: a Gaussian filter of the map ("sigma", to regularise early
iterations) and an irrotational constraint ("integrate": a scalar function whose
gradient fits the map in the least-squares sense is found iteratively with conjugate
gradients, and the map is replaced by that function's numerical gradient, so its curl
vanishes).  The paper does not give the
discretisation; the readings taken here:

* filter: each component of ``u`` is convolved along both axes with the sampled
  Gaussian ``exp(-k^2 / (2 sigma^2))``, ``|k| <= int(4 sigma + 0.5)``, normalised to
  unit sum; outside the detector the nearest pixel is repeated; ``sigma <= 0`` leaves
  the map unchanged;
* integration: ``Phi`` minimises
  ``sum (Phi[i+1,j] - Phi[i,j] - (u0[i,j] + u0[i+1,j]) / 2)^2
   + sum (Phi[i,j+1] - Phi[i,j] - (u1[i,j] + u1[i,j+1]) / 2)^2``
  (forward differences against the trapezoid mean of the two end points, all pixels,
  good or not); the new map is the gradient of ``Phi`` by central differences inside
  and second-order one-sided differences at the edges (first order along an axis of
  two pixels; an axis of one pixel keeps its component);
* order: filter first, then integrate (the processing chain of Sec. 2.2 lists
  "regularise" before "apply irrotational constraint").

``integrate_map`` solves the normal equations by conjugate gradients, as the paper
does; ``integrate_map_direct`` solves the same least-squares problem exactly (the
normal-equation matrix is the Neumann Laplacian, diagonal in the type-II DCT basis)
and serves the large cases.
"""
from __future__ import annotations

import numpy as np


def _f64(x):
    return np.asarray(x, dtype=np.float64)


# ----------------------------------------------------------------------------- filter

def gaussian_kernel(sigma):
    """Sampled Gaussian of the filter reading, normalised to unit sum."""
    r = int(4.0 * sigma + 0.5)
    k = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def _convolve_axis(a, g, axis):
    """Correlation of a with the symmetric kernel g along one axis, nearest padding."""
    r = (g.size - 1) // 2
    a = np.moveaxis(a, axis, 0)
    n = a.shape[0]
    out = np.zeros_like(a)
    for k in range(-r, r + 1):
        idx = np.clip(np.arange(n) + k, 0, n - 1)
        out += g[k + r] * a[idx]
    return np.moveaxis(out, 0, axis)


def gaussian_filter_map(u, sigma):
    """Each component of the map filtered along both axes (Sec. 2.2.2, "sigma")."""
    u = _f64(u)
    if not sigma > 0.0:
        return u.copy()
    g = gaussian_kernel(float(sigma))
    out = np.empty_like(u)
    for c in range(u.shape[0]):
        out[c] = _convolve_axis(_convolve_axis(u[c], g, 0), g, 1)
    return out


# ------------------------------------------------------------------------ integration

def _targets(u):
    """Trapezoid means: targets of the forward differences along each axis."""
    t0 = 0.5 * (u[0, 1:, :] + u[0, :-1, :])
    t1 = 0.5 * (u[1, :, 1:] + u[1, :, :-1])
    return t0, t1


def _D(phi):
    """Forward differences along both axes."""
    return phi[1:, :] - phi[:-1, :], phi[:, 1:] - phi[:, :-1]


def _DT(d0, d1, shape):
    """Adjoint of _D."""
    out = np.zeros(shape)
    out[1:, :] += d0
    out[:-1, :] -= d0
    out[:, 1:] += d1
    out[:, :-1] -= d1
    return out


def _gradient(phi, u):
    """Numerical gradient of phi (the reading's differences); an axis of one pixel keeps
    that component of u."""
    out = np.empty((2,) + phi.shape)
    for ax in range(2):
        n = phi.shape[ax]
        if n == 1:
            out[ax] = u[ax]
        else:
            out[ax] = np.gradient(phi, axis=ax, edge_order=2 if n >= 3 else 1)
    return out


def integrate_potential(u, tol=1e-13, max_iter=None):
    """Least-squares potential of the map by conjugate gradients on the normal
    equations D^T D phi = D^T t (Sec. 2.2.2, "integrate").  The mean of phi is zero."""
    u = _f64(u)
    shape = u.shape[1:]
    t0, t1 = _targets(u)
    b = _DT(t0, t1, shape)

    def A(p):
        d0, d1 = _D(p)
        return _DT(d0, d1, shape)

    x = np.zeros(shape)
    r = b.copy()
    p = r.copy()
    rr = float((r * r).sum())
    bb = rr
    n_iter = max_iter if max_iter is not None else 20 * (shape[0] + shape[1]) + 100
    for _ in range(n_iter):
        if rr <= tol * tol * max(bb, 1e-300):
            break
        q = A(p)
        alpha = rr / float((p * q).sum())
        x += alpha * p
        r -= alpha * q
        rr_new = float((r * r).sum())
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x - x.mean()


def integrate_map(u, tol=1e-13, max_iter=None):
    """The map replaced by the gradient of its least-squares potential (CG)."""
    u = _f64(u)
    return _gradient(integrate_potential(u, tol, max_iter), u)


def integrate_map_direct(u):
    """Same least-squares problem solved exactly: the normal-equation matrix is the
    Neumann Laplacian, whose eigenvectors along an axis of n pixels are the type-II
    DCT vectors with eigenvalues 2 - 2 cos(pi k / n)."""
    from scipy.fft import dctn, idctn
    u = _f64(u)
    H, W = u.shape[1:]
    t0, t1 = _targets(u)
    b = _DT(t0, t1, (H, W))
    bh = dctn(b, type=2, norm="ortho")
    lam = (2.0 - 2.0 * np.cos(np.pi * np.arange(H) / H))[:, None] + \
          (2.0 - 2.0 * np.cos(np.pi * np.arange(W) / W))[None, :]
    lam[0, 0] = 1.0
    ph = bh / lam
    ph[0, 0] = 0.0
    phi = idctn(ph, type=2, norm="ortho")
    return _gradient(phi, u)


def regularise_pixel_map(u, sigma=0.0, integrate=False, direct=False):
    """Filter (sigma > 0), then integrate (if asked): the reading's order."""
    out = gaussian_filter_map(u, sigma)
    if integrate:
        out = integrate_map_direct(out) if direct else integrate_map(out)
    return out


def curl(u):
    """Discrete curl d u1 / d i - d u0 / d j by central differences (interior)."""
    u = _f64(u)
    d1di = 0.5 * (u[1, 2:, 1:-1] - u[1, :-2, 1:-1])
    d0dj = 0.5 * (u[0, 1:-1, 2:] - u[0, 1:-1, :-2])
    return d1di - d0dj
