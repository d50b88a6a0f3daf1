"""Served stream on the GPU: continuous batching gives every job the same result as
solving it alone, jobs join mid-stream, and admission respects the HBM budget."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import paper_2003_12726_amd as pxst
from paper_2003_12726_amd import serve
from synth import random_small_scan
from gpu_util import ref_rel_error, U_TOL_PX, REF_TOL_REL, ERR_TOL_REL

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


@pytest.mark.parametrize("policy,tick_evals", [("aged", 2e10), ("srpt", 2e10), ("srpt", 1.0), ("all", 0.0)])
def test_batched_equals_alone_bitwise(policy, tick_evals):
    """tick_evals = 1 makes every srpt tick take one job (plus the jobs whose final
    reference update is due), so jobs overtake each other as often as possible."""
    reqs = requests()
    say("[serve] one by one")
    alone = serve.run_one_by_one(reqs)
    say(f"[serve] continuous batching, policy {policy}, tick work {tick_evals:g}")
    srv = serve.Server(budget_bytes=8 << 30, max_slots=16, policy=policy, tick_evals=tick_evals)
    mixed = srv.run(reqs)
    assert srv.max_resident >= 3, srv.max_resident
    for k in alone:
        assert_same(alone[k], mixed[k])
    assert all(r.finished >= r.arrival for r in mixed.values())


def _tied_pixel_ok(r, ref, w, i, j, u_gpu):
    """A pixel whose served map differs from the oracle's: accepted only where the
    oracle's two best candidate errors differ by < 1e-6 relative (the tie rule of the
    search) and the served value is one of the tied candidates (with its refinement)."""
    rows, cols = np.array([i]), np.array([j])
    _, _, _, E = oracle.update_pixel_map(r.frames, r.white, r.mask, ref, w, r.dx0, r.u0, r.origin,
                                         r.window, r.refine, pixels=(rows, cols), return_errors=True)
    Eg = E[:, :, 0]
    emin = Eg.min()
    tied = np.argwhere(np.isfinite(Eg) & (Eg - emin <= 1e-6 * abs(emin)))
    if len(tied) < 2:
        return False
    c = oracle.round_half_up(r.u0[:, i, j])
    rx, ry = r.window
    for kx, ky in tied:
        ox, oy = oracle._refine_at(Eg, kx - rx, ky - ry, rx, ry) if r.refine else (0.0, 0.0)
        cand = np.array([c[0] + kx - rx + ox, c[1] + ky - ry + oy])
        if np.abs(cand - u_gpu).max() <= 1e-3:
            return True
    return False


def test_served_results_match_oracle():
    """Every job served in the mix, one main-loop iteration each (Sec. 2.2: reference,
    pixel map, translations of Sec. 2.2.3 for two of the jobs, error; then the final
    reference), against the FP64 oracle from the same start state, at the single-step
    bar: error 1e-5 relative; map within 1e-3 px except at oracle ties, where the served
    value must be one of the tied candidates; translations within 1e-3 px; the final
    reference within 1e-5 of the oracle's update from the served state."""
    reqs = [dataclasses.replace(r, n_iter=1) for r in requests()]
    say("[serve] continuous batching vs the oracle, one iteration per job")
    srv = serve.Server(budget_bytes=8 << 30, max_slots=16)
    mixed = srv.run(reqs)
    assert srv.max_resident >= 3, srv.max_resident
    for r in reqs:
        o = oracle.solve(r.frames, r.white, r.mask, r.u0, r.dx0, r.origin, r.ref_shape, 1,
                         r.window, refine=r.refine, update_dx=r.update_dx, tr_window=r.tr_window)
        m = mixed[r.job_id]
        du = np.abs(m.u - o["u"]).max(axis=0)
        say(f"    job {r.job_id}: det {r.frames.shape[1:]} N={r.frames.shape[0]} window {r.window} "
            f"max|du| {du.max():.2e}")
        np.testing.assert_allclose(m.err_hist, o["err_hist"], rtol=ERR_TOL_REL)
        off = np.argwhere(du > U_TOL_PX)
        if len(off):
            ref, w = oracle.update_reference(r.frames, r.white, r.mask, r.u0, r.dx0, r.origin, r.ref_shape)
            ref = ref.astype(np.float32).astype(np.float64)
            for i, j in off:
                assert _tied_pixel_ok(r, ref, w, i, j, m.u[:, i, j]), (r.job_id, i, j)
        assert np.abs(m.dx - o["dx"]).max() < U_TOL_PX, (r.job_id, np.abs(m.dx - o["dx"]).max())
        ro, wo = oracle.update_reference(r.frames, r.white, r.mask, m.u, m.dx, r.origin, r.ref_shape)
        np.testing.assert_array_equal(m.wsum > 0, wo > 0)
        err, _ = ref_rel_error(m.ref, ro, wo)
        assert err < REF_TOL_REL, (r.job_id, err)


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


def test_batch_iterate_mixed_groups_bitwise():
    """pxst_batch_iterate over jobs that fall into different groups of every shared stage
    -- reference arithmetic (exact, bfloat16, float32 gather), frame counts, translation
    windows, regularisation -- with the jobs at different iterations, equals each job
    solved alone, bitwise."""
    from paper_2003_12726_amd import CJob
    from gpu_util import dev_scan, to_dev, empty
    specs = [
        dict(det=(37, 53), n=7, win=(3, 2), opts=dict(update_dx=True, tr=(1, 1))),
        dict(det=(48, 40), n=9, win=(2, 2), opts=dict(update_dx=True, tr=(2, 1), ref_mode="bf16")),
        dict(det=(33, 45), n=5, win=(2, 3), opts=dict(ref_mode="fp32")),
        dict(det=(40, 64), n=6, win=(3, 3), opts=dict(update_dx=True, tr=(2, 2), sigma=1.3)),
        dict(det=(64, 64), n=40, win=(2, 2), opts=dict(), grid=(7, 6)),   # many frames
        dict(det=(21, 80), n=6, win=(0, 3), opts=dict(update_dx=True, tr=(0, 2))),
    ]
    jobs = []
    for k, sp in enumerate(specs):
        s = random_small_scan(det=sp["det"], n_frames=sp["n"], window=sp["win"], seed=400 + k,
                              n_grid=sp.get("grid", (3, 3)))
        assert s.frames.shape[0] == sp["n"]
        opts = pxst.make_opts(3, sp["win"], True, **sp["opts"])
        jobs.append((s, opts))
    say("[batch] alone")
    alone = []
    for s, opts in jobs:
        sc = dev_scan(s)
        ws = pxst.alloc_workspace(sc.geom, opts)
        u, dx = to_dev(s.u0).clone(), to_dev(s.dx0).clone()
        ref, w = empty(s.ref_shape, torch.float32), empty(s.ref_shape, torch.float64)
        h = torch.zeros(3, dtype=torch.float64, device="cuda")
        pxst.solve(sc, opts, u, dx, ref, w, h, ws)
        torch.cuda.synchronize()
        alone.append([t.cpu().numpy() for t in (u, dx, ref, w, h)])
    say("[batch] batched, jobs starting at different ticks")
    state = []
    for s, opts in jobs:
        sc = dev_scan(s)
        ws = pxst.alloc_workspace(sc.geom, opts)
        st = dict(sc=sc, opts=opts, ws=ws, u=to_dev(s.u0).clone(), dx=to_dev(s.dx0).clone(),
                  ref=empty(s.ref_shape, torch.float32), w=empty(s.ref_shape, torch.float64),
                  h=torch.zeros(3, dtype=torch.float64, device="cuda"), it=0)
        state.append(st)
    start = [0, 1, 0, 2, 1, 0]          # tick at which each job joins
    bws = torch.empty(pxst.batch_workspace_bytes(len(jobs)), dtype=torch.uint8, device="cuda")
    tick = 0
    while any(st["it"] <= 3 for st in state):
        active = [k for k, st in enumerate(state) if start[k] <= tick and st["it"] <= 3]
        cj = []
        for k in active:
            st = state[k]
            j = CJob()
            j.scan = st["sc"].c()
            j.opts = st["opts"]
            j.u, j.dx, j.ref, j.wsum = (st[x].data_ptr() for x in ("u", "dx", "ref", "w"))
            j.err_hist = st["h"].data_ptr()
            j.iter = st["it"]
            j.ws, j.ws_bytes = st["ws"].data_ptr(), st["ws"].numel()
            cj.append(j)
        if cj:
            pxst.batch_iterate(cj, bws)
        for k in active:
            state[k]["it"] += 1
        tick += 1
    torch.cuda.synchronize()
    for k, st in enumerate(state):
        got = [st[x].cpu().numpy() for x in ("u", "dx", "ref", "w", "h")]
        for name, a, b in zip(("u", "dx", "ref", "wsum", "err_hist"), alone[k], got):
            assert np.array_equal(a, b), (k, name, np.nanmax(np.abs(a - b)))
