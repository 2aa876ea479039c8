"""Serving form: continuous batching of many real-time TDDFT propagation
requests on one GPU.

Requests (a system, its initial states, a number of ETRS steps) arrive over
time.  A request is admitted, first come first served, when a job slot is
free and its HBM footprint (states, the grid's workspace, v_ion, its dipole
and norm traces) fits the budget next to the jobs already resident; its
states and potentials then stay in HBM until its last step.  All resident
jobs advance together through one libks batch (ks_batch_*: one H.psi
launch per Taylor pass over the work items of every job, one step captured
as a HIP graph).  When a job joins or leaves, the batch is rebuilt and every job
resumes where it stopped; the trajectory of each request is bitwise the
one it has when propagated alone.

Latency of a (request, step) pair is the wall time from the moment the
request was ready for that step (the completion of its previous step, or
its admission) to the completion of the batch step that advanced it: the
rebuild of the batch and the admissions that delay a step are charged to
it.  Newly arrived requests join at the next departure (when the batch is
rebuilt anyway) unless that is more than `join_lag` steps away, which
halves the rebuilds of a mix whose requests leave every few steps.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import ks


def set_serving_launch(grid, spec):
    """Launch shape of a served job: the default tile rows with z-chunks of
    the whole axis.  With many jobs resident the batch has work items to
    spare, and every z-chunk re-reads the 8 planes around it (saturated
    serving mix, FP64: 10 % shorter steps than the single-grid default of up
    to two chunks).  States and dipoles do not depend on the shape; the norm
    diagnostics (sums of per-tile partials) do in their last bits, so a
    request is compared with its lone run in this same shape.  A grid whose
    LDS cannot hold the whole-axis chunk keeps its default."""
    try:
        grid.set_launch(0, spec.n[2])
    except ks.KSError:
        pass


@dataclass
class Request:
    rid: int
    arrival: float            # seconds (wall clock) or steps (step clock)
    spec: object
    vion: object              # host or device float64 tensor [N]
    psi: object               # host or device complex128 tensor
    nsteps: int
    dt: float
    kick: float = 0.0
    # filled in by the server
    t_admit: float = None
    t_done: float = None
    dipole: np.ndarray = None
    norms: np.ndarray = None
    final_psi: np.ndarray = None
    step_latency: list = field(default_factory=list)

    @property
    def pts_states(self):
        return self.spec.npoints * self.spec.nk * self.spec.nstates


class _Active:
    def __init__(self, req, grid, job):
        self.req, self.grid, self.job = req, grid, job
        self.fp = 0
        self.t_ready = 0.0     # wall time the request became ready to step


class Server:
    """Continuous-batching propagation server on one GPU.

    hbm_budget: bytes of HBM the resident jobs may hold together.
    max_slots: most jobs in one batch.
    clock: "wall" (arrivals in seconds since run() starts) or "steps"
        (arrivals in batch steps taken: a deterministic schedule).
    keep_states: copy each request's final states to the host.
    tune: run the launch-shape autotuner on each admitted grid.
    join_lag: a request that could be admitted while a batch runs waits
        for the next departure (which rebuilds the batch anyway) when that
        is at most this many steps away.
    """

    def __init__(self, hbm_budget, max_slots=64, precision=ks.KS_FP64,
                 clock="wall", keep_states=False, tune=False,
                 device="cuda", join_lag=4):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.clock = clock
        self.keep_states = keep_states
        self.tune = tune
        self.device = torch.device(device)
        self.join_lag = int(join_lag)
        self.stats = {}

    # ---- footprint ----
    def _footprint(self, req, grid):
        """HBM a resident request holds: its states, the grid's workspace
        and own tables, v_ion, the dipole and norm traces."""
        N, S = req.spec.npoints, req.spec.nk * req.spec.nstates
        return (16 * N * S + grid.workspace_bytes + grid.device_bytes +
                8 * N + 8 * (req.nsteps + 1) * (3 + S) + 4096)

    def _head_grid(self, waiting):
        """Give the request at the head of the queue its grid and
        footprint (the grid's tables are allocated here)."""
        if not waiting or waiting[0][1] is not None:
            return
        r = waiting[0][0]
        g = ks.Grid(r.spec, precision=self.precision, device=self.device,
                    workspace=False)
        set_serving_launch(g, r.spec)
        fp = self._footprint(r, g)
        if fp > self.budget:
            g.close()
            raise ValueError(f"request {r.rid} needs {fp} bytes, more than "
                             f"the budget {self.budget}")
        waiting[0][1:] = [g, fp]

    def _admit(self, req, grid, now):
        grid.ensure_workspace()
        psi = req.psi.to(self.device, non_blocking=True).contiguous()
        vion = req.vion.to(self.device, non_blocking=True).contiguous()
        if req.kick:
            grid.kick(psi, req.kick)
        if self.tune:
            grid.autotune(psi)
        job = ks.Job(grid, psi, vion, req.dt, req.nsteps, t0=0.0,
                     dipole=not any(req.spec.periodic), norms=True)
        req.t_admit = now
        a = _Active(req, grid, job)
        a.fp = self._footprint(req, grid)
        a.t_ready = time.perf_counter()
        return a

    def _retire(self, a, now):
        r = a.req
        j = a.job
        r.t_done = now
        r.dipole = j.dipole.cpu().numpy() if j.dipole is not None else None
        r.norms = j.norms.cpu().numpy()
        if self.keep_states:
            r.final_psi = j.psi.cpu().numpy()
        a.grid.close()
        a.job = None

    # ---- main loop ----
    def run(self, requests):
        """Serve `requests` (sorted by arrival) to completion; returns the
        statistics dict (also in self.stats).

        One batch step stays in flight: the next step is enqueued before
        the host waits for the previous one, unless a job leaves or joins
        after it (membership changes need the batch drained), so the GPU
        does not idle while the host does its per-step bookkeeping."""
        torch = self.torch
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        # [request, grid, footprint] arrived, not admitted; only the head
        # holds a grid (created when it is next to be admitted), so device
        # memory outside the budget is at most one grid's tables
        waiting = deque()
        active = []
        used = 0
        batch = None
        steps_taken = 0
        rebuilds = 0
        rebuild_s = 0.0
        max_active = 0
        lat = []
        work = 0.0
        busy = 0.0
        inflight = None          # (start event, end event, members)
        t_start = time.perf_counter()

        def now():
            if self.clock == "steps":
                return float(steps_taken)
            return time.perf_counter() - t_start

        def finish(rec):
            """Wait for an enqueued step and charge it to its members."""
            nonlocal busy, work
            ev0, ev1, members = rec
            ev1.synchronize()
            t1 = time.perf_counter()
            busy += ev0.elapsed_time(ev1) / 1e3
            for a in members:
                dt_step = t1 - a.t_ready
                a.t_ready = t1
                a.req.step_latency.append(dt_step)
                lat.append(dt_step)
                work += 8.0 * a.req.pts_states

        t_first = None
        while pending or waiting or active:
            tnow = now()
            while pending and pending[0].arrival <= tnow:
                waiting.append([pending.popleft(), None, 0])
            self._head_grid(waiting)
            # jobs whose last step has been enqueued leave: drain the batch
            done = [a for i, a in enumerate(active)
                    if batch is not None and
                    batch.steps_done(i) >= a.req.nsteps]
            if done:
                if inflight is not None:
                    finish(inflight)
                    inflight = None
                batch.close()
                batch = None
                tn = now()
                for a in done:
                    self._retire(a, tn)
                    used -= a.fp
                    active.remove(a)
            # while a batch runs, newly arrived requests join at the next
            # departure unless it is more than join_lag steps away
            join_now = batch is None or not active or min(
                a.req.nsteps - batch.steps_done(i)
                for i, a in enumerate(active)) > self.join_lag
            admit = (join_now and waiting and len(active) < self.max_slots
                     and used + waiting[0][2] <= self.budget)
            if admit and inflight is not None:
                finish(inflight)
                inflight = None
            changed = False
            while (join_now and waiting and len(active) < self.max_slots and
                   used + waiting[0][2] <= self.budget):
                r, g, fp = waiting.popleft()
                active.append(self._admit(r, g, tnow))
                used += active[-1].fp
                changed = True
                self._head_grid(waiting)
            if not active:
                if self.clock == "steps":
                    steps_taken += 1      # idle tick
                elif pending:
                    time.sleep(max(0.0, min(pending[0].arrival - now(),
                                            0.001)))
                continue
            if t_first is None:
                t_first = time.perf_counter()
            if changed or batch is None:
                t_rb = time.perf_counter()
                if batch is not None:
                    batch.close()
                batch = ks.Batch([a.job for a in active])
                rebuilds += 1
                rebuild_s += time.perf_counter() - t_rb
            max_active = max(max_active, len(active))
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record()
            batch.step(1)
            ev1.record()
            steps_taken += 1
            rec = (ev0, ev1, list(active))
            if inflight is not None:
                finish(inflight)
            inflight = rec
        if inflight is not None:
            finish(inflight)
        if batch is not None:
            batch.close()
        t_end = time.perf_counter()
        wall = t_end - (t_first if t_first is not None else t_end)
        lat_ms = 1e3 * np.asarray(lat) if lat else np.zeros(1)
        reqs = list(requests)
        waits = [r.t_admit - r.arrival for r in reqs if r.t_admit is not None]
        self.stats = dict(
            requests=len(reqs),
            request_steps=len(lat),
            batch_steps=int(steps_taken),
            rebuilds=rebuilds,
            rebuild_ms_mean=1e3 * rebuild_s / max(rebuilds, 1),
            max_concurrent=max_active,
            p50_step_ms=float(np.percentile(lat_ms, 50)),
            p99_step_ms=float(np.percentile(lat_ms, 99)),
            mean_step_ms=float(lat_ms.mean()),
            wall_s=wall,
            gpu_busy_frac=busy / wall if wall > 0 else 0.0,
            value=work / wall if wall > 0 else 0.0,
            unit="grid-point·states/s",
            mean_queue_wait=float(np.mean(waits)) if waits else 0.0,
        )
        return self.stats
