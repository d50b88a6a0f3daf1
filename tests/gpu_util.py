"""Helpers shared by the GPU tests: device copies of synthetic scans and comparison
rules (the acceptance bar of the GPU path against the FP64 oracle)."""
import numpy as np

import paper_2003_12726_amd as pxst

# acceptance bar
ARGMIN_TIE_REL = 1e-6     # a different argmin is accepted only for oracle errors this close
U_TOL_PX = 1e-3           # refined map and translations
REF_TOL_REL = 1e-5        # reference image
ERR_TOL_REL = 1e-5        # error figures
U32 = 2.0 ** -24          # float32 unit roundoff


def emin_bound(E, nv, var, imax, kappa=8.0, wq=0.0):
    """Admissible |E_gpu - E_oracle| of a normalised error E = sum r^2 / var.

    Each float32 residual r = I - W g carries an error |e| <= kappa u (|I| + |W g|)
    <= 3 kappa u I_max (a few roundings in the lookup and the product), so
    |dE| <= 2 sqrt(E S) + S with S = nv (3 kappa u I_max)^2 / var, plus 1e-5 E for the
    summation.  For a near-perfect fit (tiny E) this is far above 1e-5 E.

    ``wq``: W times the fixed-point step q = 2^-F of the reference lookups on the matrix
    cores (F = 21 - e, max |I_ref| < 2^e), added to each residual's error: a lookup
    there is rounded to a multiple of q, after a float32 interpolation whose error is a
    fraction of q.  It matters only for references of a high dynamic range.
    """
    S = nv * (3.0 * kappa * U32 * imax + wq) ** 2 / np.maximum(var, 1e-300)
    return 1e-5 * E + 2.0 * np.sqrt(E * S) + S


def to_dev(x, dev="cuda"):
    import torch
    if x.dtype == np.uint16:
        x = x.view(np.int16)
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def dev_scan(s, dev="cuda"):
    return pxst.Scan(to_dev(s.frames, dev), to_dev(s.white, dev), to_dev(s.mask, dev), s.ref_shape,
                     s.origin)


def empty(shape, dtype, dev="cuda"):
    import torch
    return torch.empty(tuple(shape), dtype=dtype, device=dev)


def ref_rel_error(ref_gpu, ref_orc, w_orc):
    """max |dI| / max(|I|, mean |I|) over well-covered pixels (w > 1e-3 median w)."""
    pos = w_orc > 0
    thr = 1e-3 * np.median(w_orc[pos])
    sel = w_orc > thr
    scale = max(np.abs(ref_orc[sel]).max(), np.abs(ref_orc[sel]).mean())
    return np.abs(ref_gpu[sel] - ref_orc[sel]).max() / scale, sel


def compare_argmin(k_gpu, k_orc, E_orc_grid, good_index):
    """Indices must agree except where the oracle's errors at both differ < 1e-6 relative.

    E_orc_grid: (NX, NY, P) oracle errors of the P good pixels; good_index maps a pixel
    (flattened over the compared set) to its column in E_orc_grid or -1.
    Returns (n_mismatch_allowed, n_mismatch_bad, bad_positions).
    """
    k_gpu = np.asarray(k_gpu).ravel()
    k_orc = np.asarray(k_orc).ravel()
    diff = np.nonzero(k_gpu != k_orc)[0]
    ok, bad = 0, []
    flat = E_orc_grid.reshape(-1, E_orc_grid.shape[-1]) if E_orc_grid is not None else None
    for p in diff:
        col = good_index[p]
        if col < 0 or k_gpu[p] < 0 or k_orc[p] < 0:
            bad.append(p)
            continue
        eg, eo = flat[k_gpu[p], col], flat[k_orc[p], col]
        if np.isfinite(eg) and np.isfinite(eo) and abs(eg - eo) <= ARGMIN_TIE_REL * abs(eo):
            ok += 1
        else:
            bad.append(p)
    return ok, len(bad), bad


def fixed_point_step(ref, w):
    """Step 2^-F of the matrix-core search's fixed-point reference: F = 21 - e with e the
    exponent for which the largest |I_ref| of a valid pixel is below 2^e."""
    v = np.abs(np.asarray(ref, dtype=np.float64)[np.asarray(w) > 0])
    if v.size == 0 or v.max() <= 0:
        return 0.0
    e = int(np.frexp(v.max())[1])
    return 2.0 ** -(21 - e)
