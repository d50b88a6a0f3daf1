"""Python binding of libpxst (PXST reconstruction loop on MI355X / gfx950).

Argument marshalling only: every call passes device pointers of torch tensors and
the current HIP stream to the C entry points declared in include/pxst.h and raises
on a negative status.  Nothing here computes; when the built library is missing the
import fails loudly (build it with ``python -m paper_2003_12726_amd.build`` or
``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpxst.so")

PXST_OK = 0
PXST_EINVAL = -1
PXST_EWORKSPACE = -2
PXST_EUNSUPPORTED = -3
PXST_EHIP = -4


class PxstError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pxst error {code}: {msg}")
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("det_ss", ctypes.c_int32), ("det_fs", ctypes.c_int32),
                ("ref_ss", ctypes.c_int32), ("ref_fs", ctypes.c_int32),
                ("org_ss", ctypes.c_int32), ("org_fs", ctypes.c_int32)]


class Window(ctypes.Structure):
    _fields_ = [("r_ss", ctypes.c_int32), ("r_fs", ctypes.c_int32), ("refine", ctypes.c_int32)]


class CScan(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_void_p), ("white", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("geom", Geom)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int32), ("pm", Window), ("update_dx", ctypes.c_int32),
                ("tr", Window), ("ref_mode", ctypes.c_int32), ("pm_sigma", ctypes.c_float),
                ("pm_integrate", ctypes.c_int32)]


class CJob(ctypes.Structure):
    _fields_ = [("scan", CScan), ("opts", SolveOpts), ("u", ctypes.c_void_p), ("dx", ctypes.c_void_p),
                ("ref", ctypes.c_void_p), ("wsum", ctypes.c_void_p), ("err_hist", ctypes.c_void_p),
                ("iter", ctypes.c_int32), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


SYMBOLS = ("pxst_workspace_bytes", "pxst_update_reference", "pxst_update_reference_ex",
           "pxst_update_pixel_map", "pxst_update_pixel_map_fractional", "pxst_split_half_pixel_map",
           "pxst_defocus_sweep", "pxst_update_translations", "pxst_error", "pxst_error_noalloc", "pxst_solve",
           "pxst_batch_workspace_bytes",
           "pxst_batch_iterate", "pxst_regularise_pixel_map", "pxst_profile_enable",
           "pxst_profile_read", "pxst_profile_select", "pxst_last_error", "pxst_abi_version")

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpxst and declare its signatures (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libpxst is not built ({path} missing); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    P = ctypes.POINTER
    lib.pxst_workspace_bytes.argtypes = [P(Geom), P(SolveOpts)]
    lib.pxst_workspace_bytes.restype = sz
    lib.pxst_update_reference.argtypes = [P(CScan), vp, vp, vp, vp, vp, sz, vp]
    lib.pxst_update_reference_ex.argtypes = [P(CScan), vp, vp, i32, vp, vp, vp, sz, vp]
    lib.pxst_update_pixel_map.argtypes = [P(CScan), vp, vp, vp, vp, Window, vp, vp, vp, vp, sz, vp]
    lib.pxst_update_pixel_map_fractional.argtypes = [P(CScan), vp, vp, vp, vp, Window, i32, vp, vp, vp, vp,
                                                     sz, vp]
    lib.pxst_split_half_pixel_map.argtypes = [P(CScan), vp, vp, vp, vp, Window, vp, vp, vp, ctypes.c_float,
                                              i32, vp, vp, sz, vp]
    lib.pxst_defocus_sweep.argtypes = [P(CScan), vp, P(ctypes.c_float), i32, ctypes.c_float, ctypes.c_float, vp,
                                       vp, vp, sz, vp]
    lib.pxst_update_translations.argtypes = [P(CScan), vp, vp, vp, vp, Window, vp, vp, vp, vp, sz, vp]
    lib.pxst_error.argtypes = [P(CScan), vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pxst_error_noalloc.argtypes = [P(CScan), vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pxst_solve.argtypes = [P(CScan), P(SolveOpts), vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pxst_batch_workspace_bytes.argtypes = [i32]
    lib.pxst_batch_workspace_bytes.restype = sz
    lib.pxst_batch_iterate.argtypes = [P(CJob), i32, vp, sz, vp]
    lib.pxst_regularise_pixel_map.argtypes = [P(Geom), vp, vp, ctypes.c_float, i32, vp, sz, vp]
    lib.pxst_profile_enable.argtypes = [i32]
    lib.pxst_profile_read.argtypes = [ctypes.c_char_p, P(ctypes.c_double), P(ctypes.c_int64),
                                      P(ctypes.c_int64)]
    lib.pxst_profile_select.argtypes = [ctypes.c_char_p]
    lib.pxst_last_error.restype = ctypes.c_char_p
    lib.pxst_abi_version.restype = i32
    for name in ("pxst_update_reference", "pxst_update_reference_ex", "pxst_update_pixel_map",
                 "pxst_update_pixel_map_fractional", "pxst_split_half_pixel_map", "pxst_defocus_sweep",
                 "pxst_update_translations",
                 "pxst_error", "pxst_solve", "pxst_batch_iterate", "pxst_regularise_pixel_map",
                 "pxst_profile_enable",
                 "pxst_profile_read", "pxst_profile_select"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().pxst_last_error().decode()


def _check(rc: int):
    if rc != PXST_OK:
        raise PxstError(rc, last_error())


def _ptr(t) -> Optional[int]:
    """Device pointer of a tensor (None -> NULL); raw integers pass through."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def make_geom(n_frames: int, det: Sequence[int], ref_shape: Sequence[int], origin: Sequence[int]) -> Geom:
    return Geom(int(n_frames), int(det[0]), int(det[1]), int(ref_shape[0]), int(ref_shape[1]),
                int(origin[0]), int(origin[1]))


def make_window(r_ss: int, r_fs: int, refine: bool = True) -> Window:
    return Window(int(r_ss), int(r_fs), int(bool(refine)))


REF_MODES = {"exact": 0, "fp32": 1, "bf16": 2}   # PXST_REF_EXACT, _FP32, _BF16


def make_opts(n_iter: int, pm: Sequence[int], refine: bool = True, update_dx: bool = False,
              tr: Sequence[int] = (2, 2), tr_refine: bool = True, ref_mode: str = "exact",
              sigma: float = 0.0, integrate: bool = False) -> SolveOpts:
    return SolveOpts(int(n_iter), make_window(pm[0], pm[1], refine), int(bool(update_dx)),
                     make_window(tr[0], tr[1], tr_refine), REF_MODES[ref_mode], float(sigma),
                     int(bool(integrate)))


@dataclasses.dataclass
class Scan:
    """Device-resident scan: frames [N, H, W] uint16, white [H, W] float32, mask [H, W] uint8."""
    frames: object
    white: object
    mask: object
    ref_shape: Sequence[int]
    origin: Sequence[int]

    @property
    def geom(self) -> Geom:
        N, H, W = (int(x) for x in self.frames.shape)
        return make_geom(N, (H, W), self.ref_shape, self.origin)

    def c(self) -> CScan:
        return CScan(_ptr(self.frames), _ptr(self.white), _ptr(self.mask), self.geom)


def workspace_bytes(geom: Geom, opts: Optional[SolveOpts] = None) -> int:
    lib = load_library()
    n = lib.pxst_workspace_bytes(ctypes.byref(geom), ctypes.byref(opts) if opts is not None else None)
    if n == 0:
        raise PxstError(PXST_EINVAL, last_error())
    return int(n)


def alloc_workspace(geom: Geom, opts: Optional[SolveOpts] = None, device="cuda"):
    import torch
    return torch.empty(workspace_bytes(geom, opts), dtype=torch.uint8, device=device)


def _ws(ws):
    return (_ptr(ws), int(ws.numel()) if ws is not None and not isinstance(ws, int) else 0)


def update_reference(scan: Scan, u, dx, ref, wsum, ws, stream=None, mode: str = "exact"):
    """Reference update (Sec. 2.2.1): writes ref [Rs, Rf] float32 and wsum float64; mode
    selects the arithmetic ("exact", "fp32", "bf16")."""
    lib = load_library()
    p, n = _ws(ws)
    if mode == "exact":
        _check(lib.pxst_update_reference(ctypes.byref(scan.c()), _ptr(u), _ptr(dx), _ptr(ref),
                                         _ptr(wsum), p, n, _stream(stream)))
    else:
        _check(lib.pxst_update_reference_ex(ctypes.byref(scan.c()), _ptr(u), _ptr(dx), REF_MODES[mode],
                                            _ptr(ref), _ptr(wsum), p, n, _stream(stream)))


def update_pixel_map(scan: Scan, ref, wsum, dx, u_in, window: Window, u_out, err_min=None,
                     argmin=None, ws=None, stream=None):
    """Pixel-map search (Sec. 2.2.2)."""
    lib = load_library()
    p, n = _ws(ws)
    _check(lib.pxst_update_pixel_map(ctypes.byref(scan.c()), _ptr(ref), _ptr(wsum), _ptr(dx),
                                     _ptr(u_in), window, _ptr(u_out), _ptr(err_min), _ptr(argmin),
                                     p, n, _stream(stream)))


def update_pixel_map_fractional(scan: Scan, ref, wsum, dx, u_in, window: Window, steps: int, u_out,
                                err_min=None, argmin=None, ws=None, stream=None):
    """Pixel-map search on a grid of 1/steps pixel (Sec. 2.2.2, no paraboloid)."""
    lib = load_library()
    p, n = _ws(ws)
    _check(lib.pxst_update_pixel_map_fractional(ctypes.byref(scan.c()), _ptr(ref), _ptr(wsum), _ptr(dx),
                                                _ptr(u_in), window, int(steps), _ptr(u_out), _ptr(err_min),
                                                _ptr(argmin), p, n, _stream(stream)))


def split_half_pixel_map(scan: Scan, ref, wsum, dx, u_in, window: Window, half, u_a, u_b,
                         hist_range: float = 1.0, nbins: int = 64, hist=None, ws=None, stream=None):
    """Split-half analysis (Sec. 2.3): pixel maps from the two halves of the (frame,
    pixel) terms marked by half (uint8 0/1) and the histogram of their differences."""
    lib = load_library()
    p, n = _ws(ws)
    _check(lib.pxst_split_half_pixel_map(ctypes.byref(scan.c()), _ptr(ref), _ptr(wsum), _ptr(dx), _ptr(u_in),
                                         window, _ptr(half), _ptr(u_a), _ptr(u_b), float(hist_range),
                                         int(nbins), _ptr(hist), p, n, _stream(stream)))


def defocus_sweep(scan: Scan, dx, scales, contrast, best=None, centre=None, ws=None, stream=None):
    """Defocus by registration (Sec. 2.1): reference contrast for every candidate pair of
    per-axis map scales (host array [n, 2]); best receives the first maximum."""
    import numpy as np
    lib = load_library()
    p, n = _ws(ws)
    sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float32).reshape(-1, 2))
    c = (float("nan"), float("nan")) if centre is None else (float(centre[0]), float(centre[1]))
    _check(lib.pxst_defocus_sweep(ctypes.byref(scan.c()), _ptr(dx),
                                  sc.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(sc.shape[0]), c[0], c[1],
                                  _ptr(contrast), _ptr(best), p, n, _stream(stream)))


def update_translations(scan: Scan, ref, wsum, u, dx_in, window: Window, dx_out, err_min=None,
                        argmin=None, ws=None, stream=None):
    """Translation search (Sec. 2.2.3)."""
    lib = load_library()
    p, n = _ws(ws)
    _check(lib.pxst_update_translations(ctypes.byref(scan.c()), _ptr(ref), _ptr(wsum), _ptr(u),
                                        _ptr(dx_in), window, _ptr(dx_out), _ptr(err_min),
                                        _ptr(argmin), p, n, _stream(stream)))


def error(scan: Scan, ref, wsum, u, dx, total, pixel_err=None, frame_err=None, ref_err=None, ws=None,
          stream=None):
    """Figures of merit (Sec. 2.2.4)."""
    lib = load_library()
    p, n = _ws(ws)
    _check(lib.pxst_error(ctypes.byref(scan.c()), _ptr(ref), _ptr(wsum), _ptr(u), _ptr(dx),
                          _ptr(pixel_err), _ptr(frame_err), _ptr(total), _ptr(ref_err), p, n,
                          _stream(stream)))


def error_noalloc(scan: Scan, ref, wsum, u, dx, total, pixel_err=None, frame_err=None, stream=None):
    """Figures of merit (Sec. 2.2.4) with the library's fixed scratch array instead of a
    workspace: no device memory is allocated."""
    lib = load_library()
    _check(lib.pxst_error_noalloc(ctypes.byref(scan.c()), _ptr(ref), _ptr(wsum), _ptr(u), _ptr(dx),
                                  _ptr(pixel_err), _ptr(frame_err), _ptr(total), _stream(stream)))


def solve(scan: Scan, opts: SolveOpts, u, dx, ref, wsum, err_hist=None, ws=None, stream=None):
    """Main loop (Sec. 2.2); u and dx are updated in place."""
    lib = load_library()
    p, n = _ws(ws)
    _check(lib.pxst_solve(ctypes.byref(scan.c()), ctypes.byref(opts), _ptr(u), _ptr(dx), _ptr(ref),
                          _ptr(wsum), _ptr(err_hist), p, n, _stream(stream)))


def regularise_pixel_map(geom: Geom, u_in, u_out, sigma: float = 0.0, integrate: bool = False, ws=None,
                         stream=None):
    """Pixel-map regularisation (Sec. 2.2.2): Gaussian filter, then the irrotational
    constraint; the workspace must be laid out with integrate when it is asked for."""
    lib = load_library()
    p, n = _ws(ws)
    _check(lib.pxst_regularise_pixel_map(ctypes.byref(geom), _ptr(u_in), _ptr(u_out), float(sigma),
                                         int(bool(integrate)), p, n, _stream(stream)))


def batch_iterate(jobs: Sequence[CJob], batch_ws=None, stream=None):
    lib = load_library()
    arr = (CJob * len(jobs))(*jobs)
    p, n = _ws(batch_ws)
    _check(lib.pxst_batch_iterate(arr, len(jobs), p, n, _stream(stream)))


def batch_workspace_bytes(n_jobs: int) -> int:
    return int(load_library().pxst_batch_workspace_bytes(int(n_jobs)))


def profile_enable(on: bool = True):
    _check(load_library().pxst_profile_enable(int(bool(on))))


def profile_select(families=None):
    """Time only the named kernel families (an iterable of names), without device work
    counters; None times every family again."""
    sel = None if families is None else ",".join(families).encode()
    _check(load_library().pxst_profile_select(sel))


def profile_read(family: str):
    """(total milliseconds, launches, work units) of a kernel family since the last read."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    work = ctypes.c_int64()
    _check(load_library().pxst_profile_read(family.encode(), ctypes.byref(ms), ctypes.byref(cnt),
                                            ctypes.byref(work)))
    return ms.value, cnt.value, work.value


def abi_version() -> int:
    return int(load_library().pxst_abi_version())
