"""The serving loop's host logic without a GPU: admission by slots and HBM
footprint, the join-at-next-departure rule, departures, and the step kept
in flight, run against stand-ins for the library's Grid / Job / Batch and
for torch's CUDA events.  The stand-ins check that no job steps past its
last step, that the batch is only closed or rebuilt when no step is in
flight, and that at most two steps (the one being waited for and the next)
are ever enqueued."""
from types import SimpleNamespace

import numpy as np
import pytest
import torch

from paper_1912_07921_amd import serving


class _Log:
    def __init__(self):
        self.enqueued = 0          # steps enqueued
        self.completed = 0         # steps waited for
        self.max_in_flight = 0
        self.batches = []          # membership (request ids) of each batch


class FakeEvent:
    def __init__(self, log):
        self.log = log
        self.step = None

    def record(self):
        self.step = self.log.enqueued

    def synchronize(self):
        self.log.completed = max(self.log.completed, self.step)

    def elapsed_time(self, other):
        return 1.0


_LIVE = []          # grids created (each closes when its request leaves)


class FakeGrid:
    def __init__(self, spec, precision=0, device=None, workspace=False):
        self.spec = spec
        self.workspace_bytes = 1000 * spec.npoints
        self.device_bytes = 100 * spec.npoints
        self.h = object()
        _LIVE.append(self)

    def set_launch(self, *a):
        pass

    def ensure_workspace(self):
        pass

    def kick(self, psi, k):
        pass

    def autotune(self, psi):
        pass

    def close(self):
        self.h = None


class FakeJob:
    def __init__(self, grid, psi, vion, dt, max_steps, t0=0.0, dipole=True,
                 norms=True):
        self.grid, self.max_steps = grid, max_steps
        self.first_step = 0
        self.dipole = torch.zeros(max_steps + 1, 3, dtype=torch.float64)
        self.norms = torch.zeros(max_steps + 1, 2, dtype=torch.float64)
        self.psi = psi


def make_fakes(log):
    class FakeBatch:
        def __init__(self, jobs):
            # membership changes only with nothing in flight
            assert log.completed == log.enqueued
            self.jobs = list(jobs)
            self.taken = 0
            log.batches.append(sorted(j.rid for j in self.jobs))

        def step(self, n=1):
            for j in self.jobs:
                assert j.first_step + self.taken + n <= j.max_steps
            self.taken += n
            log.enqueued += n
            log.max_in_flight = max(log.max_in_flight,
                                    log.enqueued - log.completed)

        def steps_done(self, i):
            return self.jobs[i].first_step + self.taken

        def close(self):
            assert log.completed == log.enqueued
            for j in self.jobs:
                j.first_step += self.taken
            self.taken = 0

    def job(grid, psi, vion, dt, max_steps, **kw):
        j = FakeJob(grid, psi, vion, dt, max_steps, **kw)
        j.rid = grid.rid
        return j

    def grid(spec, **kw):
        g = FakeGrid(spec, **kw)
        g.rid = spec.rid
        return g

    ks = SimpleNamespace(Grid=grid, Job=job, Batch=FakeBatch,
                         KSError=RuntimeError, KS_FP64=0)
    tch = SimpleNamespace(cuda=SimpleNamespace(
        Event=lambda enable_timing=True: FakeEvent(log)))
    return ks, tch


def requests(arrivals, nsteps, npts):
    out = []
    for i, (t, ns, n) in enumerate(zip(arrivals, nsteps, npts)):
        spec = SimpleNamespace(rid=i, npoints=n, nk=1, nstates=4,
                               n=(8, 8, 8), periodic=(0, 0, 0))
        out.append(serving.Request(
            rid=i, arrival=float(t), spec=spec,
            vion=torch.zeros(n, dtype=torch.float64),
            psi=torch.zeros(1, 4, n, dtype=torch.complex128),
            nsteps=ns, dt=0.01))
    return out


def run(monkeypatch, reqs, budget, slots, join_lag=4):
    log = _Log()
    ks, tch = make_fakes(log)
    monkeypatch.setattr(serving, "ks", ks)
    srv = serving.Server(budget, max_slots=slots, clock="steps",
                         device="cpu", join_lag=join_lag)
    srv.torch = tch
    st = srv.run(reqs)
    return st, log


@pytest.mark.parametrize("slots,budget", [(2, 10 ** 12), (8, 10 ** 12),
                                          (8, 2_200_000)])
def test_every_request_gets_exactly_its_steps(monkeypatch, slots, budget):
    arrivals = [0, 0, 1, 3, 3, 3, 9, 30]
    nsteps = [5, 9, 4, 7, 2, 6, 3, 2]
    npts = [512, 1000, 512, 700, 512, 900, 512, 512]
    reqs = requests(arrivals, nsteps, npts)
    st, log = run(monkeypatch, reqs, budget, slots)
    assert st["requests"] == len(reqs)
    assert st["request_steps"] == sum(nsteps)
    for r in reqs:
        assert len(r.step_latency) == r.nsteps
        assert r.t_done is not None and r.t_admit >= r.arrival
    # the slot limit holds in every batch, and one step at most waits
    # behind the one in flight
    assert max(len(b) for b in log.batches) <= slots
    assert log.max_in_flight == 2
    assert log.completed == log.enqueued


def test_only_the_queue_head_holds_a_grid(monkeypatch):
    """Requests waiting for admission hold no device memory, except the
    next in line; every grid is closed when its request leaves."""
    _LIVE.clear()
    reqs = requests([0] * 6, [3, 4, 5, 6, 7, 8], [1000] * 6)
    log = _Log()
    ks, tch = make_fakes(log)
    monkeypatch.setattr(serving, "ks", ks)
    srv = serving.Server(10 ** 12, max_slots=2, clock="steps",
                         device="cpu")
    srv.torch = tch
    seen = []
    orig = srv._admit

    def admit(req, grid, now):
        # at each admission: the admitted grids, plus at most the head's
        seen.append(sum(g.h is not None for g in _LIVE))
        return orig(req, grid, now)

    srv._admit = admit
    srv.run(reqs)
    assert max(seen) <= 2 + 1
    assert all(g.h is None for g in _LIVE) and len(_LIVE) == len(reqs)


def test_budget_limits_the_resident_footprint(monkeypatch):
    """With a budget for about two of these requests, no batch holds
    three."""
    reqs = requests([0] * 5, [3, 4, 5, 6, 7], [1000] * 5)
    srv_probe = serving.Server(1, device="cpu")
    fp = srv_probe._footprint(reqs[0], FakeGrid(reqs[0].spec))
    st, log = run(monkeypatch, reqs, int(2.5 * fp), 8)
    assert max(len(b) for b in log.batches) == 2
    assert st["request_steps"] == sum(r.nsteps for r in reqs)


def test_join_waits_for_a_near_departure(monkeypatch):
    """A request arriving while the batch runs joins at the next departure
    when that is at most join_lag steps away (one rebuild instead of two),
    and at once when it is further."""
    # request 0 runs 6 steps; request 1 arrives at step 3, when request 0
    # has 3 steps left: with join_lag 4 it waits for the departure
    reqs = requests([0, 3], [6, 4], [512, 512])
    st, log = run(monkeypatch, reqs, 10 ** 12, 8, join_lag=4)
    assert log.batches == [[0], [1]]
    reqs = requests([0, 3], [6, 4], [512, 512])
    st, log = run(monkeypatch, reqs, 10 ** 12, 8, join_lag=1)
    assert log.batches == [[0], [0, 1], [1]]
    assert st["request_steps"] == 10


def test_latency_starts_when_a_request_is_ready(monkeypatch):
    """Latencies are positive and a request's first step is timed from its
    admission."""
    reqs = requests([0, 0, 2], [3, 5, 2], [512, 512, 512])
    st, log = run(monkeypatch, reqs, 10 ** 12, 8)
    lat = np.concatenate([np.asarray(r.step_latency) for r in reqs])
    assert (lat >= 0).all()
    assert st["p99_step_ms"] >= st["p50_step_ms"] >= 0
