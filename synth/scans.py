"""Seeded synthetic scans shaped like the PXST workloads.

Geometry follows the discrete forward model of the paper (Sec. 2.1, Eq. 3): frame
``n`` pixel ``(i, j)`` sees the reference at ``u[:, i, j] - dx[n] - origin`` (axis 0 =
slow scan, axis 1 = fast scan), scaled by the white-field.  The pixel map ``u`` is
stored as *absolute* reference coordinates; the generator draws a displacement
``d`` and sets ``u = (i, j) - d``.

Rendering uses ``scipy.ndimage.map_coordinates(order=1)``, a library routine that is
not used by either reconstruction implementation.  Random numbers come from
``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import Optional, Tuple

import numpy as np
from scipy import ndimage


@dataclasses.dataclass(frozen=True)
class ScanSpec:
    name: str
    det: Tuple[int, int]                 # (H, W): slow scan, fast scan
    n_grid: Tuple[int, int]              # translation grid (ss, fs)
    step: float                          # grid step, reference pixels
    jitter: float                        # uniform jitter half-width, px
    disp_ss: Tuple[float, float]         # (A2, A3) of d_ss = A2 s^2 + A3 s^3
    disp_fs: Tuple[float, float]
    window: Tuple[int, int]              # pixel-map search half-widths (r_ss, r_fs)
    iters: int
    ref: Optional[Tuple[int, int]] = None  # reference shape; None = computed
    ref_sigma: float = 1.5
    ref_contrast: float = 0.15
    white: str = "gauss"                 # "gauss" | "stripe"
    white_sigma: float = 24.0
    white_mean: Optional[float] = None   # scale so that mean(W) equals this
    white_peak: Optional[float] = None   # or so that max(W) equals this
    refine: bool = True
    update_dx: bool = False
    tr_window: Tuple[int, int] = (2, 2)
    dx_start: str = "true"               # "true" | "nominal"
    n_frames: Optional[int] = None       # first n frames of the grid
    seed: int = 0
    bright_frac: float = 0.0             # fraction of reference pixels made bright
    bright_gain: float = 1.0             # their brightness relative to the speckle


@dataclasses.dataclass
class Scan:
    spec: ScanSpec
    frames: np.ndarray      # (N, H, W) uint16 photon counts
    white: np.ndarray       # (H, W) float32
    mask: np.ndarray        # (H, W) uint8, 1 = good
    u0: np.ndarray          # (2, H, W) float32 initial pixel map
    dx0: np.ndarray         # (N, 2) float32 initial translations
    origin: Tuple[int, int]
    ref_shape: Tuple[int, int]
    window: Tuple[int, int]
    tr_window: Tuple[int, int]
    refine: bool
    iters: int
    update_dx: bool
    u_true: np.ndarray      # (2, H, W) float32
    dx_true: np.ndarray     # (N, 2) float32
    ref_true: np.ndarray    # (Rs, Rf) float64

    @property
    def n_frames(self) -> int:
        return int(self.frames.shape[0])

    @property
    def det(self) -> Tuple[int, int]:
        return int(self.frames.shape[1]), int(self.frames.shape[2])

    def pm_evals(self) -> int:
        """Candidate evaluations of one pixel-map update: good pixels x window x frames."""
        rx, ry = self.window
        return int(self.mask.astype(bool).sum()) * (2 * rx + 1) * (2 * ry + 1) * self.n_frames

    def tr_evals(self) -> int:
        tx, ty = self.tr_window
        return int(self.mask.astype(bool).sum()) * (2 * tx + 1) * (2 * ty + 1) * self.n_frames


CONFIGS = {
    # tiny: 64x64 detector, 32 frames, +-4 px window
    "tiny": ScanSpec(name="tiny", det=(64, 64), ref=(128, 128), ref_sigma=2.0, ref_contrast=0.2,
                     white="gauss", white_sigma=24.0, white_peak=1000.0,
                     disp_ss=(6.0, 2.0), disp_fs=(6.0, 2.0), n_grid=(4, 8), step=6.0, jitter=0.5,
                     window=(4, 4), refine=False, iters=3, seed=1),
    # realistic: 256x1024 detector, 121 frames, +-10 px window, quadratic refinement
    "realistic": ScanSpec(name="realistic", det=(256, 1024), ref=(512, 1536), ref_sigma=1.5,
                          ref_contrast=0.15, white="stripe", white_mean=4000.0,
                          disp_ss=(14.0, 6.0), disp_fs=(14.0, 6.0), n_grid=(11, 11), step=8.0,
                          jitter=0.5, window=(10, 10), refine=True, iters=5, seed=2),
    # highly divergent: 512x512, 400 frames, anisotropic window, translation update on
    "divergent": ScanSpec(name="divergent", det=(512, 512), ref=(640, 640), ref_sigma=1.5,
                          ref_contrast=0.15, white="gauss", white_sigma=256.0, white_mean=5000.0,
                          disp_ss=(30.0, 10.0), disp_fs=(8.0, 2.0), n_grid=(20, 20), step=4.0,
                          jitter=0.5, window=(15, 3), refine=True, iters=8, update_dx=True,
                          tr_window=(2, 2), dx_start="nominal", seed=3),
}


def spec_for(name: str, **overrides) -> ScanSpec:
    return dataclasses.replace(CONFIGS[name], **overrides)


def _coord(n: int) -> np.ndarray:
    """Normalised coordinate s in [-1, 1] along an axis of n pixels."""
    if n == 1:
        return np.zeros(1)
    h = (n - 1) / 2.0
    return (np.arange(n) - h) / h


def _white(spec: ScanSpec, H: int, W: int) -> np.ndarray:
    i = np.arange(H)[:, None].astype(np.float64)
    j = np.arange(W)[None, :].astype(np.float64)
    ci, cj = (H - 1) / 2.0, (W - 1) / 2.0
    if spec.white == "stripe":
        w = np.exp(-(i - ci) ** 2 / (2 * (H / 4.0) ** 2)) * np.exp(-(((j - cj) / (0.547 * W)) ** 8))
    else:
        w = np.exp(-((i - ci) ** 2 + (j - cj) ** 2) / (2 * spec.white_sigma ** 2))
    if spec.white_mean is not None:
        w = w * (spec.white_mean / w.mean())
    elif spec.white_peak is not None:
        w = w * (spec.white_peak / w.max())
    return w


def _speckle(rng: np.random.Generator, shape, sigma: float, contrast: float) -> np.ndarray:
    z = ndimage.gaussian_filter(rng.standard_normal(shape), sigma, mode="wrap")
    z = (z - z.mean()) / z.std()
    return np.clip(1.0 + contrast * z, 0.05, None)


def _grid_dx(spec: ScanSpec, rng: np.random.Generator, jitter: bool) -> np.ndarray:
    gx, gy = spec.n_grid
    a, b = np.meshgrid(np.arange(gx) - (gx - 1) / 2.0, np.arange(gy) - (gy - 1) / 2.0, indexing="ij")
    dx = spec.step * np.stack([a.ravel(), b.ravel()], axis=1)
    if jitter and spec.jitter > 0:
        dx = dx + rng.uniform(-spec.jitter, spec.jitter, size=dx.shape)
    if spec.n_frames is not None:
        dx = dx[: spec.n_frames]
    return dx


def _displacement(spec: ScanSpec, H: int, W: int):
    si, sj = _coord(H), _coord(W)
    d_ss = spec.disp_ss[0] * si ** 2 + spec.disp_ss[1] * si ** 3
    d_fs = spec.disp_fs[0] * sj ** 2 + spec.disp_fs[1] * sj ** 3
    d0_ss = spec.disp_ss[0] * si ** 2          # known "defocus" part = initial estimate
    d0_fs = spec.disp_fs[0] * sj ** 2
    for d, n in ((d_ss, H), (d_fs, W)):
        if n > 1:
            assert np.abs(np.diff(d)).max() < 1.0, "displacement folds over"
    return d_ss, d_fs, d0_ss, d0_fs


def _place_reference(spec: ScanSpec, coords, margin: int):
    """Integer origin and reference shape holding every coordinate plus a margin."""
    lo = np.array([min(float(c[k].min()) for c in coords) for k in (0, 1)])
    hi = np.array([max(float(c[k].max()) for c in coords) for k in (0, 1)])
    span = [int(math.ceil(hi[k])) - int(math.floor(lo[k])) for k in (0, 1)]
    need = [span[k] + 2 + 2 * margin for k in (0, 1)]
    if spec.ref is None:
        shape = tuple(need)
    else:
        shape = tuple(int(s) for s in spec.ref)
        assert shape[0] >= need[0] and shape[1] >= need[1], (shape, need)
    pad = [(shape[k] - span[k] - 2) // 2 for k in (0, 1)]
    origin = tuple(int(math.floor(lo[k])) - pad[k] for k in (0, 1))
    for c in coords:
        for k in (0, 1):
            assert c[k].min() - origin[k] >= margin and c[k].max() - origin[k] <= shape[k] - 2 - margin
    return origin, shape


def make_scan(spec: ScanSpec, variant: str = "poisson", mask: str = "ones") -> Scan:
    """Render a scan.

    variant: "poisson" (Poisson counts), "noiseless" (rounded expected counts) or
    "exact" (integer map, integer translations, integer-valued W * I_ref, no noise:
    the forward model then holds exactly at the truth).
    mask: "ones" or "parity" (1 % random bad pixels plus a one-pixel bad border).
    """
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    H, W = spec.det
    d_ss, d_fs, d0_ss, d0_fs = _displacement(spec, H, W)
    exact = variant == "exact"
    if exact:
        d_ss, d_fs = np.round(d_ss), np.round(d_fs)
        d0_ss, d0_fs = np.round(d0_ss), np.round(d0_fs)
    ii, jj = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    u_true = np.stack([ii - d_ss[:, None], jj - d_fs[None, :]]).astype(np.float32)
    u0 = np.stack([ii - d0_ss[:, None], jj - d0_fs[None, :]]).astype(np.float32)

    dx_true = _grid_dx(spec, rng, jitter=not exact)
    if exact:
        dx_true = np.round(dx_true)
    dx_true = dx_true.astype(np.float32)
    dx_start = dx_true if spec.dx_start == "true" else _grid_dx(spec, rng, jitter=False).astype(np.float32)
    if exact:
        dx_start = np.round(dx_start).astype(np.float32)

    r_ss, r_fs = spec.window
    t_ss, t_fs = spec.tr_window
    margin = max(r_ss, r_fs) + max(t_ss, t_fs) + 3
    # coordinate ranges of u - dx over every frame, for both the true and the start state
    coords = []
    for uu in (u_true, u0):
        for dd in (dx_true, dx_start):
            coords.append(tuple(np.array([float(uu[k].min()) - float(dd[:, k].max()),
                                          float(uu[k].max()) - float(dd[:, k].min())])
                                for k in (0, 1)))
    origin, ref_shape = _place_reference(spec, coords, margin)

    ref_true = _speckle(rng, ref_shape, spec.ref_sigma, spec.ref_contrast)
    if spec.bright_frac > 0:
        # isolated bright pixels (a high dynamic range), from a generator of their own so
        # that the other draws of the scan stay those of the plain speckle
        hot = np.random.Generator(np.random.PCG64(spec.seed + 7919)).random(ref_shape) < spec.bright_frac
        ref_true = np.where(hot, ref_true * spec.bright_gain, ref_true)
    white = _white(spec, H, W)
    if exact:
        white = np.maximum(np.round(white), 1.0)
        ref_true = np.clip(np.round(10.0 + 4.0 * (ref_true - 1.0) / max(spec.ref_contrast, 1e-6)),
                           1.0, 20.0)

    N = dx_true.shape[0]
    frames = np.empty((N, H, W), dtype=np.uint16)
    u64 = u_true.astype(np.float64)
    for n in range(N):
        a = u64[0] - float(dx_true[n, 0]) - origin[0]
        b = u64[1] - float(dx_true[n, 1]) - origin[1]
        lam = white * ndimage.map_coordinates(ref_true, [a, b], order=1, mode="nearest")
        if variant == "poisson":
            cnt = rng.poisson(lam)
        else:
            cnt = np.round(lam)
        frames[n] = np.clip(cnt, 0, 65535).astype(np.uint16)

    m = np.ones((H, W), dtype=np.uint8)
    if mask == "parity":
        m[rng.random((H, W)) < 0.01] = 0
        m[0, :] = m[-1, :] = 0
        m[:, 0] = m[:, -1] = 0

    return Scan(spec=spec, frames=frames, white=white.astype(np.float32), mask=m, u0=u0,
                dx0=dx_start.astype(np.float32), origin=origin, ref_shape=ref_shape,
                window=tuple(spec.window), tr_window=tuple(spec.tr_window), refine=spec.refine,
                iters=spec.iters, update_dx=spec.update_dx, u_true=u_true, dx_true=dx_true,
                ref_true=ref_true)


@functools.lru_cache(maxsize=4)
def cached_scan(name: str, variant: str = "poisson", mask: str = "ones") -> Scan:
    return make_scan(CONFIGS[name], variant, mask)


def exact_scan(det=(24, 20), n_grid=(2, 3), step=3.0, window=(3, 3), disp=(2.0, 1.0), seed=11,
               mask="ones") -> Scan:
    """Small scan on which the forward model holds exactly at the truth."""
    spec = ScanSpec(name="exact", det=det, n_grid=n_grid, step=step, jitter=0.0,
                    disp_ss=disp, disp_fs=disp, window=window, iters=3, ref=None,
                    ref_sigma=0.8, ref_contrast=0.3, white="gauss", white_sigma=0.8 * max(det),
                    white_peak=900.0, refine=False, seed=seed)
    return make_scan(spec, variant="exact", mask=mask)


def random_small_scan(det=(37, 53), n_frames=7, window=(3, 2), seed=21, mask="parity",
                      zero_white=True, refine=True, variant="poisson", n_grid=(3, 3),
                      step=5.0, tr_window=(2, 2)) -> Scan:
    """Odd-sized scan with masked pixels and (optionally) zero white-field pixels."""
    amp = min(3.0, 0.12 * min(det))
    spec = ScanSpec(name="small", det=det, n_grid=n_grid, step=step, jitter=0.5,
                    disp_ss=(amp, amp / 3.0), disp_fs=(0.7 * amp, amp / 3.0), window=window,
                    iters=3, ref=None,
                    ref_sigma=1.5, ref_contrast=0.2, white="gauss", white_sigma=0.6 * max(det),
                    white_mean=2000.0, refine=refine, tr_window=tr_window,
                    n_frames=n_frames, seed=seed)
    s = make_scan(spec, variant=variant, mask=mask)
    if zero_white:
        rng = np.random.Generator(np.random.PCG64(seed + 1000))
        z = rng.random(s.white.shape) < 0.01
        s.white[z] = 0.0
    return s


def served_job_specs(n_jobs: int = 64, seed: int = 5000, iters: int = 5):
    """Job mix of the served stream: sizes, frame counts and windows per job, plus arrival gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [(128, 128), (256, 256), (256, 1024), (512, 512)]
    specs, gaps = [], []
    for k in range(n_jobs):
        det = sizes[int(rng.integers(0, len(sizes)))]
        n = int(rng.integers(16, 401))
        r = int(rng.integers(4, 16))
        gx = int(math.ceil(math.sqrt(n)))
        gy = int(math.ceil(n / gx))
        specs.append(ScanSpec(name=f"job{k}", det=det, n_grid=(gx, gy), step=4.0, jitter=0.5,
                              disp_ss=(float(r), r / 2.0), disp_fs=(float(r), r / 2.0),
                              window=(r, r), iters=iters, ref=None, ref_sigma=1.5,
                              ref_contrast=0.15, white="gauss", white_sigma=max(det) / 2.0,
                              white_mean=4000.0, refine=True, n_frames=n, seed=seed + k))
        gaps.append(float(rng.exponential(0.5)))
    return specs, gaps
