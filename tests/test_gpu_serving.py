"""Served stream on the GPU: continuous batching gives every job the same result as
solving it alone, jobs join mid-stream, and admission respects the HBM budget."""
import sys

import numpy as np
import pytest

import paper_2003_12726_amd as pxst
from paper_2003_12726_amd import serve
from synth import random_small_scan

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


def requests():
    shapes = [((37, 53), 7, (3, 2), 0.0, False), ((48, 40), 9, (2, 2), 0.0, True),
              ((33, 45), 5, (5, 5), 0.0, False), ((21, 19), 4, (1, 3), 0.02, False),
              ((40, 64), 6, (3, 3), 0.05, True),
              # 441 candidates: alone, the interior tiles are searched in halves against
              # the operand planes; batched, whole with the operand generated in the kernel
              ((48, 64), 9, (10, 10), 0.03, False),
              # 729 candidates: halves in both, against the planes alone, generated batched
              ((40, 48), 8, (13, 13), 0.04, False)]
    out = []
    for k, (det, n, win, arr, upd) in enumerate(shapes):
        s = random_small_scan(det=det, n_frames=n, window=win, seed=300 + k)
        out.append(serve.Request(job_id=k, arrival=arr, frames=s.frames, white=s.white, mask=s.mask,
                                 u0=s.u0, dx0=s.dx0, ref_shape=s.ref_shape, origin=s.origin,
                                 n_iter=3, window=win, refine=True, update_dx=upd,
                                 tr_window=(1, 1)))
    return out


def assert_same(a, b):
    for name in ("u", "dx", "ref", "wsum", "err_hist"):
        x, y = getattr(a, name), getattr(b, name)
        assert np.array_equal(x, y), (a.job_id, name, np.abs(x - y).max())


def test_batched_equals_alone_bitwise():
    reqs = requests()
    say("[serve] one by one")
    alone = serve.run_one_by_one(reqs)
    say("[serve] continuous batching")
    srv = serve.Server(budget_bytes=8 << 30, max_slots=16)
    mixed = srv.run(reqs)
    assert srv.max_resident >= 3, srv.max_resident
    for k in alone:
        assert_same(alone[k], mixed[k])
    assert all(r.finished >= r.arrival for r in mixed.values())


def test_admission_respects_budget():
    reqs = requests()
    sizes = [serve.job_bytes(r) for r in reqs]
    budget = max(sizes) + min(sizes)      # at most two jobs resident at once
    say(f"[serve] budget {budget} bytes")
    srv = serve.Server(budget_bytes=budget, max_slots=16)
    res = srv.run(reqs)
    assert srv.max_resident <= 2
    alone = serve.run_one_by_one(reqs)
    for k in alone:
        assert_same(alone[k], res[k])


def test_over_budget_job_rejected():
    reqs = requests()[:1]
    srv = serve.Server(budget_bytes=1024, max_slots=4)
    with pytest.raises(ValueError):
        srv.run(reqs)
