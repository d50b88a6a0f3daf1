"""C-ABI checks that need no GPU: the library loads, exports every symbol of
include/pxst.h, sizes workspaces, and rejects bad arguments before any GPU work."""
import ctypes
import os
import re

import pytest

import paper_2003_12726_amd as pxst

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "..", "include", "pxst.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pxst.LIB_PATH):
        from paper_2003_12726_amd import build
        build.build(verbose=False)
    return pxst.load_library()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pxst_\w+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pxst.SYMBOLS)
    assert pxst.abi_version() == 3


def test_workspace_bytes_grows_with_problem(lib):
    g1 = pxst.make_geom(32, (64, 64), (128, 128), (-37, -37))
    g2 = pxst.make_geom(121, (256, 1024), (512, 1536), (-141, -269))
    o = pxst.make_opts(3, (4, 4))
    a, b = pxst.workspace_bytes(g1, o), pxst.workspace_bytes(g2, o)
    assert 0 < a < b
    assert pxst.workspace_bytes(g1, None) > 0


def test_invalid_geometry_rejected(lib):
    g = pxst.make_geom(0, (64, 64), (128, 128), (0, 0))
    assert lib.pxst_workspace_bytes(ctypes.byref(g), None) == 0
    assert "positive" in pxst.last_error()
    o = pxst.make_opts(3, (16, 4))
    g = pxst.make_geom(4, (64, 64), (128, 128), (0, 0))
    assert lib.pxst_workspace_bytes(ctypes.byref(g), ctypes.byref(o)) == 0


def _scan(frames=0x1000, white=0x2000, mask=0x3000, geom=None):
    geom = geom or pxst.make_geom(4, (16, 16), (40, 40), (-10, -10))
    return pxst.CScan(frames, white, mask, geom)


def test_error_paths_return_before_gpu_work(lib):
    """Fake (never dereferenced) addresses: validation must fail before any launch."""
    sc = _scan()
    win = pxst.make_window(3, 3)
    P = 0x4000
    # null frames
    bad = _scan(frames=None)
    assert lib.pxst_update_reference(ctypes.byref(bad), P, P, P, P, P, 1 << 30, None) == pxst.PXST_EINVAL
    # null output
    assert lib.pxst_update_reference(ctypes.byref(sc), P, P, None, P, P, 1 << 30, None) == pxst.PXST_EINVAL
    # misaligned double pointer
    assert lib.pxst_update_reference(ctypes.byref(sc), P, P, P, P + 4, P, 1 << 30, None) == pxst.PXST_EINVAL
    # unknown reference-update mode
    assert lib.pxst_update_reference_ex(ctypes.byref(sc), P, P, 7, P, P, P, 1 << 30, None) == pxst.PXST_EINVAL
    assert "mode" in pxst.last_error()
    # workspace too small
    assert lib.pxst_update_reference(ctypes.byref(sc), P, P, P, P, 0x100000, 16, None) == pxst.PXST_EWORKSPACE
    assert "workspace" in pxst.last_error()
    # misaligned workspace
    assert lib.pxst_update_reference(ctypes.byref(sc), P, P, P, P, 0x100010, 1 << 30, None) == pxst.PXST_EINVAL
    # window too large
    big = pxst.make_window(16, 2)
    assert lib.pxst_update_pixel_map(ctypes.byref(sc), P, P, P, P, big, P, None, None, P, 1 << 30,
                                     None) == pxst.PXST_EUNSUPPORTED
    neg = pxst.make_window(-1, 2)
    assert lib.pxst_update_pixel_map(ctypes.byref(sc), P, P, P, P, neg, P, None, None, P, 1 << 30,
                                     None) == pxst.PXST_EINVAL
    # translation window too large
    assert lib.pxst_update_translations(ctypes.byref(sc), P, P, P, P, pxst.make_window(3, 1), P, None,
                                        None, P, 1 << 30, None) == pxst.PXST_EUNSUPPORTED
    # error: total is required
    assert lib.pxst_error(ctypes.byref(sc), P, P, P, P, None, None, None, None, P, 1 << 30,
                          None) == pxst.PXST_EINVAL
    # solve: null options, negative iterations
    assert lib.pxst_solve(ctypes.byref(sc), None, P, P, P, P, None, P, 1 << 30, None) == pxst.PXST_EINVAL
    o = pxst.make_opts(-1, (3, 3))
    assert lib.pxst_solve(ctypes.byref(sc), ctypes.byref(o), P, P, P, P, None, P, 1 << 30,
                          None) == pxst.PXST_EINVAL
    # solve: unknown reference-update mode
    o = pxst.make_opts(2, (3, 3))
    o.ref_mode = 5
    assert lib.pxst_solve(ctypes.byref(sc), ctypes.byref(o), P, P, P, P, None, P, 1 << 30,
                          None) == pxst.PXST_EINVAL
    assert "mode" in pxst.last_error()
    # oversized detector
    huge = _scan(geom=pxst.make_geom(4, (8192, 4096), (40, 40), (0, 0)))
    assert lib.pxst_update_reference(ctypes.byref(huge), P, P, P, P, P, 1 << 40, None) == pxst.PXST_EUNSUPPORTED


def test_batch_rejects_bad_jobs(lib):
    job = pxst.CJob()
    job.scan = _scan()
    job.opts = pxst.make_opts(2, (2, 2))
    job.iter = 5            # > n_iter
    job.ws = 0x100000
    job.ws_bytes = 1 << 30
    arr = (pxst.CJob * 1)(job)
    assert lib.pxst_batch_iterate(arr, 1, None, 0, None) == pxst.PXST_EINVAL
    assert lib.pxst_batch_iterate(None, 2, None, 0, None) == pxst.PXST_EINVAL


def test_batch_workspace_checked_before_any_launch(lib):
    """Valid jobs with a batch workspace one byte short of pxst_batch_workspace_bytes are
    refused with PXST_EWORKSPACE before anything is enqueued (no GPU here: a launch would
    fail differently); the size grows with the number of jobs."""
    sizes = [pxst.batch_workspace_bytes(n) for n in (1, 2, 8, 64)]
    assert all(b > a for a, b in zip(sizes, sizes[1:])), sizes
    jobs = []
    for k in range(3):
        job = pxst.CJob()
        job.scan = _scan()
        job.opts = pxst.make_opts(2, (2, 2))
        job.u, job.dx, job.ref, job.wsum = 0x10000, 0x20000, 0x30000, 0x40000
        job.err_hist = 0x50000
        job.iter = k % 3
        job.ws = 0x100000
        job.ws_bytes = pxst.workspace_bytes(job.scan.geom, job.opts)
        jobs.append(job)
    arr = (pxst.CJob * 3)(*jobs)
    need = pxst.batch_workspace_bytes(3)
    assert lib.pxst_batch_iterate(arr, 3, 0x1000000, need - 1, None) == pxst.PXST_EWORKSPACE
    assert "workspace" in pxst.last_error()
    # a job's own workspace one byte short is refused the same way
    jobs[1].ws_bytes -= 1
    arr = (pxst.CJob * 3)(*jobs)
    assert lib.pxst_batch_iterate(arr, 3, 0x1000000, need, None) == pxst.PXST_EWORKSPACE


def test_profile_selection_host_only(lib):
    """Timing selection is host state only: a restricted list, an empty one and NULL are
    accepted, and reading a family that recorded nothing gives zeros."""
    assert lib.pxst_profile_select(b"pm_fast, ref_gather") == 0
    assert lib.pxst_profile_select(b"") == 0
    assert lib.pxst_profile_select(None) == 0
    pxst.profile_select(["pm_fast"])
    pxst.profile_select(None)


def test_product_path_does_not_import_oracle():
    """The package and its sources never reference the oracle."""
    root = os.path.dirname(pxst.__file__)
    for dirpath, _, files in os.walk(root):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_regularise_argument_checks(lib):
    """Pixel-map regularisation: sigma and integrate are validated, and integration needs
    a workspace laid out with its buffers -- all before any GPU work."""
    g = pxst.make_geom(4, (16, 24), (40, 40), (-10, -10))
    P = 0x4000
    big = 1 << 30
    f = ctypes.c_float
    assert lib.pxst_regularise_pixel_map(ctypes.byref(g), P, P, f(-1.0), 0, P, big, None) == pxst.PXST_EINVAL
    assert lib.pxst_regularise_pixel_map(ctypes.byref(g), P, P, f(float("nan")), 0, P, big, None) == pxst.PXST_EINVAL
    assert lib.pxst_regularise_pixel_map(ctypes.byref(g), P, P, f(100.0), 0, P, big, None) == pxst.PXST_EUNSUPPORTED
    assert "sigma" in pxst.last_error()
    assert lib.pxst_regularise_pixel_map(ctypes.byref(g), P, P, f(1.0), 2, P, big, None) == pxst.PXST_EINVAL
    assert lib.pxst_regularise_pixel_map(ctypes.byref(g), None, P, f(1.0), 0, P, big, None) == pxst.PXST_EINVAL
    # the integration buffers (two float64 maps; the transform matrices are generated in
    # the kernels, not stored) are part of the workspace only when asked for
    plain = pxst.workspace_bytes(g, pxst.make_opts(1, (2, 2)))
    integ = pxst.workspace_bytes(g, pxst.make_opts(1, (2, 2), integrate=True))
    assert plain + 2 * 16 * 24 * 8 <= integ < plain + 2 * 16 * 24 * 8 + (16 * 16 + 24 * 24) * 8
    assert lib.pxst_regularise_pixel_map(ctypes.byref(g), P, P, f(1.0), 1, 0x100000, plain, None) == \
        pxst.PXST_EWORKSPACE
    # solve options carry the same checks
    o = pxst.make_opts(1, (2, 2), sigma=-2.0)
    assert lib.pxst_workspace_bytes(ctypes.byref(g), ctypes.byref(o)) == 0


def test_noalloc_error_rejects_geometry_beyond_its_scratch(lib):
    """The allocation-free error pass refuses, before any GPU work, a geometry whose
    scratch (reference, sigma^2, partial sums) exceeds the library's fixed array."""
    P = 0x4000
    big = _scan(geom=pxst.make_geom(400, (2048, 2048), (2200, 2200), (-50, -50)))
    assert lib.pxst_error_noalloc(ctypes.byref(big), P, P, P, P, None, None, P, None) == pxst.PXST_EUNSUPPORTED
    assert "scratch" in pxst.last_error()
    sc = _scan()
    assert lib.pxst_error_noalloc(ctypes.byref(sc), P, P, P, P, None, None, None, None) == pxst.PXST_EINVAL
