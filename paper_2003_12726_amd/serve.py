"""Served reconstruction stream: continuous batching of PXST solves on one GPU.

Requests (scans with their solve options) arrive over time.  The server keeps every
admitted job's frames, state and workspace resident in HBM, admits waiting jobs in
arrival order while the job-slot count and the HBM budget allow, and advances resident
jobs together: one tick is one call of ``pxst_batch_iterate``, which runs one
main-loop iteration (or the final reference update) of each job of the tick, every
stage of all of them in shared launches.  Which resident jobs a tick takes is the
policy: "srpt" takes them in order of least remaining work until the tick's
pixel-map work reaches ``tick_evals`` (enough to fill the device), so short jobs
overtake long ones as in shortest-remaining-processing-time scheduling and a tick
still fills the device; "aged" (default) orders them by remaining work expressed as
time at a nominal device rate minus the time waited since arrival, so that a long job
that has waited is no longer overtaken without bound; "all" advances every resident
job each tick.  Jobs join
and leave at tick boundaries; a finished job's memory is released before the next
tick's admission.  Latency is measured from a request's arrival to the end of the
tick that finishes it.

``run_one_by_one`` serves the same arrivals with one ``pxst_solve`` per job in arrival
order, for comparison.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import (CJob, Scan, alloc_workspace, batch_iterate, batch_workspace_bytes, make_opts,
               solve, workspace_bytes)


@dataclasses.dataclass
class Request:
    job_id: int
    arrival: float                 # seconds after the start of the stream
    frames: np.ndarray             # (N, H, W) uint16
    white: np.ndarray              # (H, W) float32
    mask: np.ndarray               # (H, W) uint8
    u0: np.ndarray                 # (2, H, W) float32
    dx0: np.ndarray                # (N, 2) float32
    ref_shape: Sequence[int]
    origin: Sequence[int]
    n_iter: int
    window: Sequence[int]
    refine: bool = True
    update_dx: bool = False
    tr_window: Sequence[int] = (2, 2)

    def pm_evals(self) -> int:
        return self.evals_per_iter() * int(self.n_iter)

    def evals_per_iter(self) -> int:
        rx, ry = self.window
        return int(self.mask.astype(bool).sum()) * (2 * rx + 1) * (2 * ry + 1) * int(self.frames.shape[0])


@dataclasses.dataclass
class Result:
    job_id: int
    arrival: float
    admitted: float
    finished: float
    u: np.ndarray
    dx: np.ndarray
    ref: np.ndarray
    wsum: np.ndarray
    err_hist: np.ndarray

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def job_bytes(req: Request) -> int:
    """HBM held by a resident job: inputs, state and workspace."""
    N, H, W = req.frames.shape
    Rs, Rf = req.ref_shape
    opts = make_opts(req.n_iter, req.window, req.refine, req.update_dx, req.tr_window)
    scan_geom = Scan(req.frames, req.white, req.mask, req.ref_shape, req.origin).geom
    state = N * H * W * 2 + H * W * 5 + 2 * H * W * 4 + N * 8 + Rs * Rf * 12 + 8 * (req.n_iter + 1)
    return int(state + workspace_bytes(scan_geom, opts))


class _Resident:
    """Device copies and state of an admitted job."""

    def __init__(self, req: Request, dev, stream):
        import torch
        self.req = req
        with torch.cuda.stream(stream):
            f = torch.from_numpy(np.ascontiguousarray(req.frames).view(np.int16)).pin_memory()
            self.frames = torch.empty(f.shape, dtype=torch.int16, device=dev)
            self.frames.copy_(f, non_blocking=True)
            self.white = torch.from_numpy(req.white).to(dev, non_blocking=True)
            self.mask = torch.from_numpy(req.mask).to(dev, non_blocking=True)
            self.u = torch.from_numpy(req.u0).to(dev, non_blocking=True)
            self.dx = torch.from_numpy(req.dx0).to(dev, non_blocking=True)
            self.ref = torch.empty(tuple(req.ref_shape), dtype=torch.float32, device=dev)
            self.wsum = torch.empty(tuple(req.ref_shape), dtype=torch.float64, device=dev)
            self.hist = torch.zeros(max(req.n_iter, 1), dtype=torch.float64, device=dev)
        self._pinned = f
        self.scan = Scan(self.frames, self.white, self.mask, req.ref_shape, req.origin)
        self.opts = make_opts(req.n_iter, req.window, req.refine, req.update_dx, req.tr_window)
        self.ws = alloc_workspace(self.scan.geom, self.opts, dev)
        self.iter = 0
        self.per_iter = req.evals_per_iter()

    def remaining(self) -> int:
        """Pixel-map work left (the final reference update counts as none)."""
        return self.per_iter * max(0, self.req.n_iter - self.iter)

    def cjob(self) -> CJob:
        j = CJob()
        j.scan = self.scan.c()
        j.opts = self.opts
        j.u = self.u.data_ptr()
        j.dx = self.dx.data_ptr()
        j.ref = self.ref.data_ptr()
        j.wsum = self.wsum.data_ptr()
        j.err_hist = self.hist.data_ptr()
        j.iter = self.iter
        j.ws = self.ws.data_ptr()
        j.ws_bytes = self.ws.numel()
        return j

    def result(self, arrival, admitted, finished) -> Result:
        return Result(self.req.job_id, arrival, admitted, finished, self.u.cpu().numpy(),
                      self.dx.cpu().numpy(), self.ref.cpu().numpy(), self.wsum.cpu().numpy(),
                      self.hist.cpu().numpy())


class Server:
    """Continuous-batching server for PXST solves on one GPU.

    budget_bytes: HBM budget for resident jobs; max_slots: resident job limit;
    policy: "aged", "srpt" or "all" (which resident jobs a tick advances); tick_evals:
    the pixel-map work at which an "aged" or "srpt" tick stops taking jobs; rate: the
    nominal device rate (pixel-map evaluations per second) that turns the remaining
    work of "aged" into time.
    """

    def __init__(self, budget_bytes: int, max_slots: int = 64, device="cuda", keep_results=True,
                 policy: str = "aged", tick_evals: float = 2e10, rate: float = 6e12):
        import torch
        if policy not in ("aged", "srpt", "all"):
            raise ValueError(f"unknown policy {policy!r}")
        self.policy = policy
        self.tick_evals = float(tick_evals)
        self.rate = float(rate)
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.dev = torch.device(device)
        self.stream = torch.cuda.current_stream(self.dev)
        self.keep_results = keep_results
        self.batch_ws = None
        self.ticks = 0
        self.max_resident = 0

    def _batch_ws(self, n):
        import torch
        need = batch_workspace_bytes(n)
        if self.batch_ws is None or self.batch_ws.numel() < need:
            self.batch_ws = torch.empty(need, dtype=torch.uint8, device=self.dev)
        return self.batch_ws

    def _pick(self, resident: List[tuple], now: float) -> List[tuple]:
        """The resident jobs this tick advances (resident entries: job, arrival, ...)."""
        if self.policy == "all":
            return resident
        if self.policy == "srpt":
            order = sorted(resident, key=lambda r: (r[0].remaining(), r[1]))
        else:
            order = sorted(resident, key=lambda r: (r[0].remaining() / self.rate - (now - r[1]), r[1]))
        tick, work = [], 0
        for r in order:
            if tick and work >= self.tick_evals:
                break
            tick.append(r)
            work += r[0].per_iter if r[0].iter < r[0].req.n_iter else 0
        return tick

    def run(self, requests: List[Request], time_scale: float = 1.0) -> Dict[int, Result]:
        """Serve requests whose arrivals are given in seconds (divided by time_scale)."""
        import torch
        pend = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        resident: List[tuple] = []          # (_Resident, arrival, admitted, bytes)
        used = 0
        out: Dict[int, Result] = {}
        for r in requests:
            if job_bytes(r) > self.budget:
                raise ValueError(f"job {r.job_id} needs {job_bytes(r)} bytes, over the budget")
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        def admit(held: int) -> List[tuple]:
            """Arrived jobs admitted in arrival order while slots and memory allow (held:
            jobs already resident); their uploads are queued on the stream."""
            nonlocal used
            t = now()
            while pend and pend[0].arrival / time_scale <= t:
                r = pend.popleft()
                waiting.append((r, r.arrival / time_scale))
            new = []
            while waiting and held + len(new) < self.max_slots:
                r, arr = waiting[0]
                nb = job_bytes(r)
                if used + nb > self.budget:
                    break
                waiting.popleft()
                res = _Resident(r, self.dev, self.stream)
                new.append((res, arr, now(), nb))
                used += nb
            return new

        while pend or waiting or resident:
            if not resident:
                resident = admit(0)
                if not resident:
                    if pend:
                        time.sleep(max(0.0, pend[0].arrival / time_scale - now()))
                    continue
            self.max_resident = max(self.max_resident, len(resident))
            tick = self._pick(resident, now())
            jobs = [r[0].cjob() for r in tick]
            batch_iterate(jobs, self._batch_ws(len(jobs)))
            # while the tick runs, admit what has arrived: the host-side staging of their
            # frames overlaps the device's work, their uploads follow the tick on the
            # stream, and they join from the next tick
            joining = admit(len(resident))
            torch.cuda.synchronize(self.dev)
            self.ticks += 1
            fin = now()
            keep = []
            advanced = set(id(r[0]) for r in tick)
            for res, arr, adm, nb in resident:
                if id(res) not in advanced:
                    keep.append((res, arr, adm, nb))
                    continue
                res.iter += 1
                if res.iter > res.req.n_iter:
                    if self.keep_results:
                        out[res.req.job_id] = res.result(arr, adm, fin)
                    else:
                        out[res.req.job_id] = Result(res.req.job_id, arr, adm, fin, None, None, None,
                                                     None, res.hist.cpu().numpy())
                    used -= nb
                else:
                    keep.append((res, arr, adm, nb))
            resident = keep + joining
        return out


def run_one_by_one(requests: List[Request], time_scale: float = 1.0, device="cuda",
                   keep_results=True) -> Dict[int, Result]:
    """Same arrivals, one full solve per job in arrival order (no batching)."""
    import torch
    dev = torch.device(device)
    stream = torch.cuda.current_stream(dev)
    out: Dict[int, Result] = {}
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda q: q.arrival):
        arr = r.arrival / time_scale
        wait = arr - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        adm = time.perf_counter() - t0
        res = _Resident(r, dev, stream)
        solve(res.scan, res.opts, res.u, res.dx, res.ref, res.wsum, res.hist, res.ws)
        torch.cuda.synchronize(dev)
        fin = time.perf_counter() - t0
        if keep_results:
            out[r.job_id] = res.result(arr, adm, fin)
        else:
            out[r.job_id] = Result(r.job_id, arr, adm, fin, None, None, None, None, res.hist.cpu().numpy())
        del res
    return out


def latency_stats(results: Dict[int, Result]) -> dict:
    lat = sorted(r.latency for r in results.values())
    if not lat:
        return {}

    def pct(q):
        k = min(len(lat) - 1, max(0, int(np.ceil(q / 100.0 * len(lat))) - 1))
        return lat[k]
    return {"p50_s": pct(50), "p99_s": pct(99), "max_s": lat[-1], "n": len(lat)}
