"""The allocation-free error entry point against the workspace one (GPU): two calls in a
row on the library's fixed scratch array, the second with a smaller scan, each equal to
pxst_error bit for bit (the same kernels) and so within the error bar of 1e-5."""
import sys

import numpy as np
import pytest

import paper_2003_12726_amd as pxst
from synth import random_small_scan
from synth.scans import cached_scan
from gpu_util import dev_scan, to_dev, empty

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pxst.load_library()


def _inputs(s):
    """Device inputs of one error call: a reference of the generator's true image with
    unit weights, and the start state shifted by 0.3 px."""
    ref = to_dev(np.asarray(s.ref_true, dtype=np.float32))
    w = to_dev(np.ones(s.ref_shape))
    u = to_dev((s.u0 + 0.3).astype(np.float32))
    dx = to_dev(s.dx0)
    return ref, w, u, dx


def _both(s):
    sc = dev_scan(s)
    ref, w, u, dx = _inputs(s)
    H, W = s.det
    out = []
    for noalloc in (False, True):
        pe = empty((H, W), torch.float32)
        fe = empty((s.n_frames,), torch.float64)
        tot = empty((1,), torch.float64)
        if noalloc:
            pxst.error_noalloc(sc, ref, w, u, dx, tot, pe, fe)
        else:
            ws = pxst.alloc_workspace(sc.geom, None)
            pxst.error(sc, ref, w, u, dx, tot, pe, fe, None, ws)
        torch.cuda.synchronize()
        out.append((pe.cpu().numpy(), fe.cpu().numpy(), float(tot.cpu()[0])))
    return out


def test_noalloc_error_equals_workspace_error():
    for s in (cached_scan("realistic"), random_small_scan(det=(37, 53), n_frames=7, seed=41)):
        say(f"[error noalloc] det={s.det} N={s.n_frames} ref={s.ref_shape}")
        (pa, fa, ta), (pb, fb, tb) = _both(s)
        np.testing.assert_array_equal(pb, pa)
        np.testing.assert_array_equal(fb, fa)
        assert tb == ta
        assert abs(tb - ta) <= 1e-5 * abs(ta) and ta > 0
