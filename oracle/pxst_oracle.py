"""FP64 CPU oracle of the PXST reconstruction loop -- test infrastructure only.

Only the tests, the entry module's smoke check and the benchmark's CPU-baseline leg
may import this file.  It restates, in plain NumPy float64, what the paper computes:

* Sec. 4, Eq. 4: bilinear interpolation at a fractional point; the masked form that
  drops unknown corners and renormalises by the remaining weights; and the same
  weights used to *add* a value at a fractional point, with the weight sums kept for
  a later division.
* Sec. 2.2.1 (make reference image): every good pixel of every frame is added at
  ``u - dx_n`` with weight ``M W I`` into the reference and ``M W^2`` into ``w``; then
  the reference is divided by ``w``.
* Sec. 2.2.2 (update pixel mapping): brute-force search of integer coordinates in a
  window around the current estimate, ``error += M (I - W I_ref)^2``,
  ``var += M (I - W)^2``, normalised ``error / var``, argmin; optional quadratic
  (paraboloid) refinement on the 3x3 errors around the minimum.
* Sec. 2.2.3 (update translations): the same search over integer shifts of one
  frame, integrating over pixels instead of frames, refined by the paraboloid.
* Sec. 2.2.4 (figures of merit) with Eq. 2: the normalised error per pixel and
  frame, its sums over frames, pixels and both, and its map on the reference plane.
* Sec. 2.2 (main loop): reference, pixel map, translations, figures of merit.

Conventions (readings where the paper is silent): axis 0 = slow scan = ``x`` = ``i``;
the pixel map holds absolute reference coordinates and the reference index of
detector pixel ``(i, j)`` in frame ``n`` is ``u[:, i, j] - dx[n] - origin`` with an
integer ``origin``; reference pixels are valid where ``w > 0``; out-of-grid corners
count as unknown.  Inputs are the float32 / uint16 arrays the GPU path receives,
promoted exactly to float64.
"""
from __future__ import annotations

import numpy as np

INF = np.inf


def _f64(x):
    return np.asarray(x, dtype=np.float64)


# --------------------------------------------------------------------------- Sec. 4

def bilinear_weights(fa, fb):
    """Weights of the corners (0,0), (1,0), (0,1), (1,1) of the unit square at (fa, fb).

    Eq. 4: f(x, y) ~ [1-x, x] . F . [1-y, y]^T, so corner (p, q) gets the area of the
    rectangle opposite to it.  Returned as a dict keyed by the corner offset.
    """
    fa, fb = _f64(fa), _f64(fb)
    return {(0, 0): (1.0 - fa) * (1.0 - fb), (1, 0): fa * (1.0 - fb),
            (0, 1): (1.0 - fa) * fb, (1, 1): fa * fb}


def _corners(shape, a, b):
    """Integer corner grid, in-grid flags and weights for fractional points (a, b)."""
    a, b = _f64(a), _f64(b)
    a0, b0 = np.floor(a), np.floor(b)
    w = bilinear_weights(a - a0, b - b0)
    a0, b0 = a0.astype(np.int64), b0.astype(np.int64)
    out = []
    for (da, db), wt in w.items():
        ia, ib = a0 + da, b0 + db
        inb = (ia >= 0) & (ia < shape[0]) & (ib >= 0) & (ib < shape[1])
        out.append((np.where(inb, ia, 0), np.where(inb, ib, 0), inb, wt))
    return out


def bilinear_gather(F, valid, a, b):
    """Masked bilinear value of array F at fractional (a, b) (Sec. 4, masked form).

    ``(sum_c w_c M_c F_c) / (sum_c w_c M_c)`` over the four corners, where M_c is the
    validity of the corner and corners outside the grid count as invalid.  Returns
    ``(g, ok)``; ``ok`` is False where the denominator is zero (no usable corner).
    """
    F = _f64(F)
    valid = np.asarray(valid, dtype=bool)
    num = np.zeros(np.broadcast(_f64(a), _f64(b)).shape)
    den = np.zeros_like(num)
    for ia, ib, inb, wt in _corners(F.shape, a, b):
        m = wt * (inb & valid[ia, ib])
        num += m * F[ia, ib]
        den += m
    ok = den > 0
    g = np.where(ok, num / np.where(ok, den, 1.0), 0.0)
    return g, ok


def bilinear_splat(shape, a, b, values, weights):
    """Add ``values`` and ``weights`` at fractional points (a, b) with bilinear weights.

    Sec. 4 (assignment to fractional coordinates): the same corner weights are used;
    both sums are returned so that the caller can renormalise afterwards.  Corners
    outside the grid are dropped.
    """
    num = np.zeros(shape)
    den = np.zeros(shape)
    values, weights = _f64(values), _f64(weights)
    for ia, ib, inb, wt in _corners(shape, a, b):
        np.add.at(num, (ia[inb], ib[inb]), (wt * values)[inb])
        np.add.at(den, (ia[inb], ib[inb]), (wt * weights)[inb])
    return num, den


# ----------------------------------------------------------------------- Sec. 2.2.1

def update_reference(frames, white, mask, u, dx, origin, ref_shape):
    """Make the reference image (Sec. 2.2.1 with the splat of Sec. 4).

    I_ref[u - dx_n] += M W I_n ;  w[u - dx_n] += M W^2 ;  I_ref = I_ref / w.
    Pixels with w == 0 are set to 0 and are invalid for later lookups.
    Returns (I_ref, w), both float64 of ``ref_shape``.
    """
    frames = np.asarray(frames)
    W, M, u, dx = _f64(white), _f64(mask), _f64(u), _f64(dx)
    num = np.zeros(ref_shape)
    den = np.zeros(ref_shape)
    sel = M > 0
    for n in range(frames.shape[0]):
        a = u[0][sel] - dx[n, 0] - origin[0]
        b = u[1][sel] - dx[n, 1] - origin[1]
        I = _f64(frames[n])[sel]
        p, q = bilinear_splat(ref_shape, a, b, (M * W)[sel] * I, (M * W * W)[sel])
        num += p
        den += q
    ref = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    return ref, den


# ----------------------------------------------------------------------- Sec. 2.2.2

def round_half_up(x):
    """Nearest integer, halves rounded up, computed as floor plus a fraction test."""
    x = _f64(x)
    f = np.floor(x)
    return f + ((x - f) >= 0.5)


def _normalised(err, var, nv):
    """error / var with the empty and zero-variance cases of the search made explicit."""
    E = np.full(err.shape, INF)
    pos = (nv > 0) & (var > 0)
    E[pos] = err[pos] / var[pos]
    E[(nv > 0) & (var == 0) & (err == 0)] = 0.0
    return E


def quadratic_refine(E):
    """Sub-pixel offset from the errors on the 3x3 stencil around an integer minimum.

    Least-squares fit of q0 + q1 x + q2 y + q3 x^2 + q4 x y + q5 y^2 to E[x+1, y+1],
    x, y in {-1, 0, 1} (the 2-D paraboloid of Sec. 2.2.2 / 2.2.3).  The offset is the
    stationary point, accepted only if it is a minimum (q3 > 0 and 4 q3 q5 - q4^2 > 0),
    and clamped to [-0.5, 0.5] per axis.  Returns (dx, dy), zero when rejected.
    """
    E = _f64(E)
    x = np.array([-1.0, 0.0, 1.0])[:, None] * np.ones((1, 3))
    y = x.T
    s0 = E.sum()
    q1 = (x * E).sum() / 6.0
    q2 = (y * E).sum() / 6.0
    q4 = (x * y * E).sum() / 4.0
    q3 = (E[0, :].sum() + E[2, :].sum()) / 2.0 - s0 / 3.0
    q5 = (E[:, 0].sum() + E[:, 2].sum()) / 2.0 - s0 / 3.0
    D = 4.0 * q3 * q5 - q4 * q4
    if not (q3 > 0 and D > 0):
        return 0.0, 0.0
    ox = (q4 * q2 - 2.0 * q5 * q1) / D
    oy = (q4 * q1 - 2.0 * q3 * q2) / D
    return float(np.clip(ox, -0.5, 0.5)), float(np.clip(oy, -0.5, 0.5))


def parabola_refine(em, e0, ep):
    """1-D version on three points: vertex of the parabola through (-1, em), (0, e0), (1, ep)."""
    c = em - 2.0 * e0 + ep
    if not c > 0:
        return 0.0
    return float(np.clip((em - ep) / (2.0 * c), -0.5, 0.5))


def _refine_at(Egrid, kx, ky, rx, ry):
    """Offset at integer argmin (kx, ky) of a (2rx+1, 2ry+1) error grid, or (0, 0)."""
    cx, cy = kx + rx, ky + ry
    if rx > 0 and ry > 0:
        if abs(kx) < rx and abs(ky) < ry:
            sub = Egrid[cx - 1:cx + 2, cy - 1:cy + 2]
            if np.all(np.isfinite(sub)):
                return quadratic_refine(sub)
        return 0.0, 0.0
    if rx > 0:  # ry == 0: only the slow-scan axis is searched
        if abs(kx) < rx and np.all(np.isfinite(Egrid[cx - 1:cx + 2, cy])):
            return parabola_refine(*Egrid[cx - 1:cx + 2, cy]), 0.0
        return 0.0, 0.0
    if ry > 0:
        if abs(ky) < ry and np.all(np.isfinite(Egrid[cx, cy - 1:cy + 2])):
            return 0.0, parabola_refine(*Egrid[cx, cy - 1:cy + 2])
    return 0.0, 0.0


def _pixel_errors(frames, W, ref, V, dx, origin, rows, cols, c0, c1, rx, ry, use=None):
    """Normalised error for every candidate of the selected pixels: E[kx, ky, p].

    Follows the loop of Sec. 2.2.2: for each candidate (slow-scan index outer,
    fast-scan inner) the error and variance are summed over frames in frame order,
    counting only frames whose reference lookup is valid.  ``use`` (N, P) booleans, if
    given, keep only the (frame, pixel) terms it marks.
    """
    P = rows.shape[0]
    N = frames.shape[0]
    I = np.stack([_f64(frames[n])[rows, cols] for n in range(N)])  # (N, P)
    Wp = W[rows, cols]
    kx = np.arange(-rx, rx + 1)[:, None, None]
    ky = np.arange(-ry, ry + 1)[None, :, None]
    err = np.zeros((2 * rx + 1, 2 * ry + 1, P))
    var = np.zeros_like(err)
    nv = np.zeros_like(err)
    for n in range(N):
        a = c0[None, None, :] + kx - dx[n, 0] - origin[0]
        b = c1[None, None, :] + ky - dx[n, 1] - origin[1]
        g, ok = bilinear_gather(ref, V, a, b)
        if use is not None:
            ok = ok & use[n][None, None, :]
        r = I[n][None, None, :] - Wp[None, None, :] * g
        err += np.where(ok, r * r, 0.0)
        v = I[n] - Wp
        var += np.where(ok, (v * v)[None, None, :], 0.0)
        nv += ok
    return _normalised(err, var, nv), (err, var, nv)


def update_pixel_map(frames, white, mask, ref, w, dx, u, origin, window, refine=True,
                     pixels=None, return_errors=False, frame_mask=None):
    """Pixel-map update of Sec. 2.2.2.

    For each good pixel the candidates are the integer points ``c + k`` with
    ``c = round_half_up(u)`` and ``k`` in the window (r_ss, r_fs).  The first minimum
    of the normalised error (slow-scan offset outer, fast-scan inner) is taken; with
    ``refine`` the paraboloid offset is added.  Bad pixels, and pixels whose every
    candidate is empty, keep their map value with error +inf and index -1.

    ``pixels``: optional (rows, cols) subset; outputs then cover only those pixels.
    ``frame_mask``: optional (N, H, W) booleans; only the marked (frame, pixel) terms
    enter the sums (the data-set halves of the split-half analysis).
    Returns (u_out, err_min, argmin) -- full arrays, or per-subset arrays; with
    ``return_errors`` also the candidate errors E[kx, ky, p] of the good pixels (and,
    when it is "sums", the unnormalised (err, var, count) grids as well).
    """
    frames = np.asarray(frames)
    W, M, ref, dx, u = _f64(white), _f64(mask), _f64(ref), _f64(dx), _f64(u)
    V = _f64(w) > 0
    H, Wd = W.shape
    rx, ry = int(window[0]), int(window[1])
    if pixels is None:
        rows, cols = np.meshgrid(np.arange(H), np.arange(Wd), indexing="ij")
        rows, cols = rows.ravel(), cols.ravel()
    else:
        rows, cols = np.asarray(pixels[0]).ravel(), np.asarray(pixels[1]).ravel()
    u_sel = u[:, rows, cols].copy()
    out_u = u_sel.copy()
    out_e = np.full(rows.shape[0], INF)
    out_k = np.full(rows.shape[0], -1, dtype=np.int64)
    good = M[rows, cols] > 0
    E_all = None
    if good.any():
        gr, gc = rows[good], cols[good]
        c = round_half_up(u_sel[:, good])
        use = None if frame_mask is None else np.asarray(frame_mask, dtype=bool)[:, gr, gc]
        E, sums = _pixel_errors(frames, W, ref, V, dx, origin, gr, gc, c[0], c[1], rx, ry, use)
        E_all = (E, sums) if return_errors == "sums" else E
        flat = E.reshape(-1, E.shape[-1])
        k = np.argmin(flat, axis=0)                       # first minimum
        emin = flat[k, np.arange(flat.shape[1])]
        found = np.isfinite(emin)
        kx = k // (2 * ry + 1) - rx
        ky = k % (2 * ry + 1) - ry
        nu = c.copy()
        nu[0] += kx
        nu[1] += ky
        if refine:
            for p in np.nonzero(found)[0]:
                ox, oy = _refine_at(E[:, :, p], int(kx[p]), int(ky[p]), rx, ry)
                nu[0, p] += ox
                nu[1, p] += oy
        gi = np.nonzero(good)[0]
        out_u[:, gi[found]] = nu[:, found]
        out_e[gi[found]] = emin[found]
        out_k[gi[found]] = k[found]
    if pixels is None:
        res = (out_u.reshape(2, H, Wd), out_e.reshape(H, Wd), out_k.reshape(H, Wd))
    else:
        res = (out_u, out_e, out_k)
    if return_errors:
        return res + (E_all,)
    return res


def update_pixel_map_fractional(frames, white, mask, ref, w, dx, u, origin, window, steps,
                                pixels=None, return_errors=False):
    """Pixel-map search on a grid finer than the pixel (Sec. 2.2.2: the error evaluated
    at non-integer positions through the interpolation of Sec. 4, instead of the
    paraboloid refinement).

    Readings: ``steps`` s is odd; the candidates of a good pixel are ``c + m / s`` per
    axis with ``c = round_half_up(u)`` and ``m`` in [-(r s + (s-1)/2), r s + (s-1)/2]
    (the integer window, each integer point with its (s-1)/2 fine neighbours on both
    sides); each candidate's error is the normalised error of Sec. 2.2.2 with every
    lookup at ``c + m / s - dx_n - origin``; first minimum in fine-grid order (slow axis
    outer); no paraboloid.  argmin is the fine-grid index ``m0' * n1 + m1'`` with
    ``m' = m + r s + (s-1)/2`` and ``n1`` the fine candidates along the fast axis.
    Bad pixels and pixels without a finite candidate keep their map value with error
    +inf and index -1.  Returns (u_out, err_min, argmin) like update_pixel_map.
    """
    s = int(steps)
    if s < 1 or s % 2 == 0:
        raise ValueError("steps must be odd and >= 1")
    h = (s - 1) // 2
    frames = np.asarray(frames)
    W, M, ref, dx, u = _f64(white), _f64(mask), _f64(ref), _f64(dx), _f64(u)
    V = _f64(w) > 0
    H, Wd = W.shape
    rx, ry = int(window[0]), int(window[1])
    Mx, My = rx * s + h, ry * s + h
    if pixels is None:
        rows, cols = np.meshgrid(np.arange(H), np.arange(Wd), indexing="ij")
        rows, cols = rows.ravel(), cols.ravel()
    else:
        rows, cols = np.asarray(pixels[0]).ravel(), np.asarray(pixels[1]).ravel()
    u_sel = u[:, rows, cols].copy()
    out_u = u_sel.copy()
    out_e = np.full(rows.shape[0], INF)
    out_k = np.full(rows.shape[0], -1, dtype=np.int64)
    good = M[rows, cols] > 0
    E_all = None
    if good.any():
        gr, gc = rows[good], cols[good]
        c = round_half_up(u_sel[:, good])
        P = gr.shape[0]
        N = frames.shape[0]
        I = np.stack([_f64(frames[n])[gr, gc] for n in range(N)])
        Wp = W[gr, gc]
        fx = (np.arange(-Mx, Mx + 1) / s)[:, None, None]
        fy = (np.arange(-My, My + 1) / s)[None, :, None]
        err = np.zeros((2 * Mx + 1, 2 * My + 1, P))
        var = np.zeros_like(err)
        nv = np.zeros_like(err)
        for n in range(N):
            a = c[0][None, None, :] + fx - dx[n, 0] - origin[0]
            b = c[1][None, None, :] + fy - dx[n, 1] - origin[1]
            g, ok = bilinear_gather(ref, V, a, b)
            r = I[n][None, None, :] - Wp[None, None, :] * g
            err += np.where(ok, r * r, 0.0)
            v = I[n] - Wp
            var += np.where(ok, (v * v)[None, None, :], 0.0)
            nv += ok
        E = _normalised(err, var, nv)
        E_all = E
        flat = E.reshape(-1, P)
        k = np.argmin(flat, axis=0)
        emin = flat[k, np.arange(P)]
        found = np.isfinite(emin)
        m0 = k // (2 * My + 1) - Mx
        m1 = k % (2 * My + 1) - My
        nu = c.copy()
        nu[0] += m0 / s
        nu[1] += m1 / s
        gi = np.nonzero(good)[0]
        out_u[:, gi[found]] = nu[:, found]
        out_e[gi[found]] = emin[found]
        out_k[gi[found]] = k[found]
    if pixels is None:
        res = (out_u.reshape(2, H, Wd), out_e.reshape(H, Wd), out_k.reshape(H, Wd))
    else:
        res = (out_u, out_e, out_k)
    if return_errors:
        return res + (E_all,)
    return res


def split_half_pixel_maps(frames, white, mask, ref, w, dx, u, origin, window, half, refine=True,
                          hist_range=1.0, nbins=64):
    """Split-half analysis (Sec. 2.3, additional analysis): every pixel of every frame
    belongs to one of two halves (``half`` (N, H, W) in {0, 1}, drawn by the caller);
    a pixel map is searched from each half against the same reference, and the
    differences of the two maps are histogrammed per axis as an uncertainty estimate.

    Readings: the searches are the update of Sec. 2.2.2 restricted to the half's
    (frame, pixel) terms; the histogram takes the good pixels with a result in both
    halves, per axis, ``nbins`` equal bins over [-hist_range, hist_range] (values
    outside are not counted, the last bin includes its upper edge: numpy's rule).
    Returns (u_a, u_b, hist (2, nbins) int64).
    """
    half = np.asarray(half)
    ua, ea, ka = update_pixel_map(frames, white, mask, ref, w, dx, u, origin, window, refine,
                                  frame_mask=(half == 0))
    ub, eb, kb = update_pixel_map(frames, white, mask, ref, w, dx, u, origin, window, refine,
                                  frame_mask=(half == 1))
    both = (_f64(mask) > 0) & (ka >= 0) & (kb >= 0)
    hist = np.zeros((2, int(nbins)), dtype=np.int64)
    for ax in range(2):
        d = (ua[ax] - ub[ax])[both]
        hist[ax] = np.histogram(d, bins=int(nbins), range=(-hist_range, hist_range))[0]
    return ua, ub, hist


def linear_map(shape, scale, centre=None):
    """Pixel map of a pure magnification change on a fixed reference grid (Sec. 2.1:
    u = x for an ideal lens at the nominal magnification; a different magnification
    scales the detector coordinates about a fixed point).  Reading: u[0] = c0 + s0 (i -
    c0), u[1] = c1 + s1 (j - c1), c the detector centre ((H-1)/2, (W-1)/2) unless given."""
    H, W = shape
    c0, c1 = ((H - 1) / 2.0, (W - 1) / 2.0) if centre is None else (float(centre[0]), float(centre[1]))
    ii, jj = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    return np.stack([c0 + float(scale[0]) * (ii - c0), c1 + float(scale[1]) * (jj - c1)])


def reference_contrast(ref, w):
    """Contrast of a reference image: variance over mean squared of the pixels with a
    positive weight sum (the reading taken of the paper's remark that a wrong defocus
    leaves a reference image with little contrast); 0 without any."""
    ref, sel = _f64(ref), _f64(w) > 0
    if not sel.any():
        return 0.0
    v = ref[sel]
    m = v.mean()
    return float(((v - m) ** 2).mean() / (m * m)) if m != 0 else 0.0


def defocus_sweep(frames, white, mask, dx, origin, ref_shape, scales, centre=None):
    """Defocus by registration (Sec. 2.1, fit_defocus_registration): a reference image is
    built (Sec. 2.2.1) from the linear map of every candidate magnification (given as
    per-axis scale factors of the map), and the candidate with the greatest contrast
    (first maximum) is chosen.  The maps are rounded to float32, as the GPU holds them.
    Returns (contrast per candidate, index of the best)."""
    H, W = _f64(white).shape
    out = []
    for sc in np.asarray(scales, dtype=np.float64).reshape(-1, 2):
        u = linear_map((H, W), sc, centre).astype(np.float32)
        ref, w = update_reference(frames, white, mask, u, dx, origin, ref_shape)
        out.append(reference_contrast(ref.astype(np.float32), w))
    c = np.array(out)
    return c, int(np.argmax(c))


# ----------------------------------------------------------------------- Sec. 2.2.3

def update_translations(frames, white, mask, ref, w, u, dx, origin, window, refine=True,
                        return_errors=False):
    """Translation update of Sec. 2.2.3.

    For frame n and every integer shift s in the window, the candidate translation is
    ``dx_n + s``; its error integrates over good pixels with a valid lookup,
    ``sum (I - W g(u - dx_n - s - origin))^2 / sum (I - W)^2``.  First minimum, then
    the paraboloid offset (when ``refine``).  Frames with no finite candidate keep their
    translation with error +inf and index -1.  Returns (dx_out, err_min, argmin).
    """
    frames = np.asarray(frames)
    W, M, ref, u, dx = _f64(white), _f64(mask), _f64(ref), _f64(u), _f64(dx)
    V = _f64(w) > 0
    tx, ty = int(window[0]), int(window[1])
    sel = M > 0
    Wp = W[sel]
    ua, ub = u[0][sel], u[1][sel]
    N = frames.shape[0]
    out = dx.copy()
    emin = np.full(N, INF)
    kmin = np.full(N, -1, dtype=np.int64)
    Es = []
    for n in range(N):
        I = _f64(frames[n])[sel]
        v = I - Wp
        E = np.full((2 * tx + 1, 2 * ty + 1), INF)
        for sx in range(-tx, tx + 1):
            for sy in range(-ty, ty + 1):
                g, ok = bilinear_gather(ref, V, ua - (dx[n, 0] + sx) - origin[0],
                                        ub - (dx[n, 1] + sy) - origin[1])
                r = I - Wp * g
                err = np.where(ok, r * r, 0.0).sum()
                var = np.where(ok, v * v, 0.0).sum()
                E[sx + tx, sy + ty] = _normalised(np.array([err]), np.array([var]),
                                                  np.array([ok.sum()]))[0]
        Es.append(E)
        k = int(np.argmin(E.ravel()))
        e = E.ravel()[k]
        if not np.isfinite(e):
            continue
        sx, sy = k // (2 * ty + 1) - tx, k % (2 * ty + 1) - ty
        ox, oy = _refine_at(E, sx, sy, tx, ty) if refine else (0.0, 0.0)
        out[n, 0] = dx[n, 0] + sx + ox
        out[n, 1] = dx[n, 1] + sy + oy
        emin[n] = e
        kmin[n] = k
    if return_errors:
        return out, emin, kmin, np.stack(Es)
    return out, emin, kmin


# ----------------------------------------------------------------------- Sec. 2.2.4

def pixel_variance(frames, white, mask):
    """sigma^2[i, j]: variance of the signal about the white-field over the frames (Eq. 2)."""
    frames = np.asarray(frames)
    W, M = _f64(white), _f64(mask)
    acc = np.zeros(W.shape)
    for n in range(frames.shape[0]):
        v = _f64(frames[n]) - W
        acc += M * v * v
    return acc / frames.shape[0]


def calc_error(frames, white, mask, ref, w, u, dx, origin, ref_error=False):
    """Figures of merit (Sec. 2.2.4, integrand of Eq. 2).

    eps[n, i, j] = M (I - W g)^2 / sigma^2 for a valid lookup ``g`` at
    ``u - dx_n - origin`` and sigma^2 > 0, else 0.  Returns a dict with the pixel error
    (sum over frames), the frame error (sum over pixels), the total, sigma^2 and,
    if asked, the reference-plane error ``sum w M eps / sum w M`` formed with the
    splat of the reference update.
    """
    frames = np.asarray(frames)
    W, M, ref, u, dx = _f64(white), _f64(mask), _f64(ref), _f64(u), _f64(dx)
    V = _f64(w) > 0
    N = frames.shape[0]
    s2 = pixel_variance(frames, white, mask)
    pix = np.zeros(W.shape)
    frame = np.zeros(N)
    num = np.zeros(ref.shape)
    den = np.zeros(ref.shape)
    sel = M > 0
    for n in range(N):
        a = u[0] - dx[n, 0] - origin[0]
        b = u[1] - dx[n, 1] - origin[1]
        g, ok = bilinear_gather(ref, V, a, b)
        r = _f64(frames[n]) - W * g
        use = ok & (s2 > 0) & sel
        eps = np.where(use, r * r / np.where(s2 > 0, s2, 1.0), 0.0)
        pix += eps
        frame[n] = eps.sum()
        if ref_error:
            p, q = bilinear_splat(ref.shape, a[sel], b[sel], (M * eps)[sel], M[sel])
            num += p
            den += q
    out = {"pixel": pix, "frame": frame, "total": float(frame.sum()), "sigma2": s2}
    if ref_error:
        out["ref"] = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    return out


# ------------------------------------------------------------------------- Sec. 2.2

def solve(frames, white, mask, u, dx, origin, ref_shape, n_iter, window, refine=True,
          update_dx=False, tr_window=(2, 2), tr_refine=True, f32_state=True):
    """Main loop of Sec. 2.2: (i) reference, (ii) pixel map, (iii) translations (optional),
    (iv) total error; a final reference is made from the last map and translations.

    ``f32_state``: store the map, the translations and the reference in float32 between
    steps (w stays float64), the storage the library's interface uses, so that every
    step sees the same inputs as a call of the library would.
    Returns dict(u, dx, ref, w, err_hist).
    """
    cast = (lambda x: _f64(np.float32(x))) if f32_state else _f64
    u = cast(u).copy()
    dx = cast(dx).copy()
    hist = []
    for _ in range(n_iter):
        ref, w = update_reference(frames, white, mask, u, dx, origin, ref_shape)
        ref = cast(ref)
        u, _, _ = update_pixel_map(frames, white, mask, ref, w, dx, u, origin, window, refine)
        u = cast(u)
        if update_dx:
            dx, _, _ = update_translations(frames, white, mask, ref, w, u, dx, origin, tr_window,
                                           tr_refine)
            dx = cast(dx)
        hist.append(calc_error(frames, white, mask, ref, w, u, dx, origin)["total"])
    ref, w = update_reference(frames, white, mask, u, dx, origin, ref_shape)
    return {"u": u, "dx": dx, "ref": cast(ref), "w": w, "err_hist": np.array(hist)}
