#!/usr/bin/env python
"""Benchmark of the real-time TDDFT hot path on one MI355X.

One step = one ETRS step of every state of the workload (8 H.psi passes with
the projector gathers, the Taylor combines, the predictor density and LDA
update, the final density, potential, dipole and norms), inputs resident in
HBM.  Throughput is H.psi grid-point-states per second:
8 * N * (nk * nstates) * steps / time.

Prints one JSON line with the FP64 rate, the roofline of the dominant kernel
(the H.psi stencil, timed live with HIP events on its stream, beside a plain
device copy timed in the same run), the CPU oracle timed on the host on a
bounded sample, the FP32-mixed form, the CFM4 propagator and the step with
the Hartree term, the macroscopic current and the strength function on the
same workload, and the serving mix (continuous batching of propagation
requests) in both precisions.
"""
from __future__ import annotations

import argparse
import copy
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per grid point and state for one ETRS step (8 H.psi
# passes: 3 x (read t_{j-1}, write t_j) + (read t3, psi, t1, t2; write the
# sum), twice): FP64 16-byte terms / mixed 8-byte terms with 16-byte psi
STEP_BYTES = {0: 352.0, 1: 224.0}
# the timed steps carry events around one H.psi launch in this many (prime
# to the 8 passes of a step)
HPSI_SAMPLE = 7
METRIC = ("H·ψ grid-point·states/s + HBM GB/s frac; serving p50/p99 step, "
          "FP32-mix vs FP64")


PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1912_07921_amd", "csrc")
KERNEL_SOURCES = ["ks_device.h", "ks_internal.h", "ks_hpsi.hip",
                  "ks_batch.hip", "ks_kernels.hip"]


def kernel_source_hash():
    """Hash of the sources that determine the device code, with comments
    and whitespace left out (an edited comment does not make recorded
    counters stale; any change of code does)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def recorded_traffic(workload, key="traffic_bytes_per_launch"):
    """HBM bytes per H.psi launch recorded from rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs (scaled by the copy-kernel calibration), if the kernel
    source has not changed since; else None.  key: the FP64 kernel's line,
    or "mixed_traffic_bytes_per_launch" for the FP32 one."""
    path = os.path.join(PROFILES, f"hpsi_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^" + key + r":\s*([0-9.eE+]+)\s+"
                  r"kernel_source_sha256_16:\s*([0-9a-f]+)", text, re.M)
    if not m or m.group(2) != kernel_source_hash():
        return None
    return float(m.group(1))


def copy_bandwidth(torch, gib=2, reps=10):
    """GB/s (read + write) of a plain device-to-device copy of `gib` GiB,
    the practical streaming ceiling the H.psi kernel is also compared to."""
    n = gib * (1 << 30) // 16
    a = torch.empty(n, dtype=torch.complex128, device="cuda")
    a.real.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * gib * (1 << 30) / (ms / 1e3) / 1e9


def calibrate_copy(torch, gib=2):
    """A plain device copy of known size, for scaling the rocprofv3 HBM
    counters: `gib` GiB read and `gib` GiB written by one copy kernel."""
    n = gib * (1 << 30) // 8
    src = torch.empty(n, dtype=torch.float64, device="cuda")
    src.fill_(1.0)
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    flush.fill_(2.0)          # 1 GiB: evicts src from the 256 MB MALL
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copied {gib} GiB ({n * 8} bytes)")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    """The workload's inputs; the molecule workloads (c2, c5) are built on
    the GPU (same random draws as the CPU build, values equal to rounding)
    so that 256 states of 128^3 points take seconds."""
    from paper_1912_07921_amd import workloads as W
    if name in ("c2", "c5"):
        return {"c2": W.c2, "c5": W.c5}[name](device="cuda")
    return {"c1": W.c1, "c3": W.c3}[name]()


def sample_workload(name, nstates):
    """The same system with only its first `nstates` states, built on the
    CPU (the oracle's input); None when the workload has no fewer states."""
    from paper_1912_07921_amd import workloads as W
    if name == "c5":
        return W.c5(nstates=nstates)
    if name == "c2":
        return W.c2(nstates=nstates)
    if name == "c3":
        return W.c3(nstates=max(1, nstates // 4))
    return W.c1()


def to_dev(torch, x):
    """A fresh device copy of an input (numpy array or tensor)."""
    if isinstance(x, np.ndarray):
        return torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return x.detach().clone().cuda()


def run_gpu(w, precision, steps, warmup, torch, tune=True, shape=None,
            method="etrs"):
    """(seconds for `steps` steps, dipole trace, profile, grid, launch
    shape).  The launch shape is `shape` (tile rows, z-chunk) if given, else
    the autotuner's choice (tune) or the default."""
    from paper_1912_07921_amd import ks
    g = ks.Grid(w.spec, precision=precision)
    psi = to_dev(torch, w.psi0)
    vion = to_dev(torch, w.vion)
    if w.kick:
        g.kick(psi, w.kick)
    if shape:
        g.set_launch(*shape)
    elif tune:
        g.autotune(psi, reps=3)
    periodic = any(w.spec.periodic)
    prop = getattr(g, "propagate_" + method)
    if warmup:
        prop(psi, vion, warmup, w.dt, dipole=not periodic, norms=True)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # events around one H.psi launch in seven (seven is prime to the eight
    # passes of a step, so every pass type is sampled alike): events around
    # every launch cost ~6 % of the step, around every launch of every
    # class ~20 %
    # (short runs time every launch: a sample of few launches would not
    # hold the pass types in their proportions)
    every = HPSI_SAMPLE if steps >= 7 * HPSI_SAMPLE else 1
    g.profile_begin(64 * steps + 64, classes=("hpsi",), every=every)
    e0.record(st)
    d, n = prop(psi, vion, steps, w.dt, t0=warmup * w.dt,
                dipole=not periodic, norms=True)
    e1.record(st)
    prof = g.profile_end()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    dip = d.cpu().numpy() if d is not None else None
    # per-class kernel times over a few more steps (all classes timed)
    g.profile_begin(4096, every=1)
    prop(psi, vion, 10, w.dt, t0=(warmup + steps) * w.dt,
         dipole=not periodic, norms=True)
    prof_all = g.profile_end()
    prof = dict(prof_all, hpsi=prof["hpsi"])
    return sec, dip, n.cpu().numpy(), prof, g, g.get_launch()


def run_apply_h(g, w, torch, reps=5):
    """Standalone H.psi (ks_apply_h: projector gather and apply, then one
    stencil pass) over every state of the workload, one call per k-point;
    HIP events around `reps` rounds on the grid's stream.  Algorithmic
    bytes: 32 per point-state (read psi, write H psi)."""
    nk, ns, N = w.spec.nk, w.spec.nstates, w.spec.npoints
    psi = to_dev(torch, w.psi0).reshape(nk, ns * N)
    out = torch.empty_like(psi[0])
    for k in range(nk):
        g.apply_h(psi[k], out, k=k)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        for k in range(nk):
            g.apply_h(psi[k], out, k=k)
    e1.record(st)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    gbs = 32.0 * N * nk * ns / sec / 1e9
    return dict(value=N * nk * ns / sec, unit="grid-point·states/s",
                ms_per_call=round(1e3 * sec, 3), achieved_GBs=round(gbs, 1),
                frac=round(gbs / HBM_PEAK_GBS, 4))


def fft_length(n, periodic):
    """Transform length of the Hartree solver along an axis of n points:
    n (periodic) or the smallest product of 2, 3, 5 >= 2 n - 1."""
    if periodic:
        return n
    m = max(1, 2 * n - 1)
    while True:
        r = m
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1:
            return m
        m += 1


def hartree_pipeline_bytes(spec):
    """HBM bytes one Hartree solve moves through its five passes (x forward
    from the density, y forward, z forward * K * inverse, y inverse, x
    inverse into the potential): the work array holds nz planes of
    My x (Mx/2 + 1) complex values (the half spectrum of the real density
    along x), K an octant of real values."""
    nx, ny, nz = spec.n
    per = all(spec.periodic)
    Mx, My, Mz = (fft_length(n, per) for n in spec.n)
    Mh = Mx // 2 + 1
    c = 16
    xf = nx * ny * nz * 8 + ny * nz * Mh * c
    yf = Mh * nz * ny * c + Mh * nz * My * c
    zc = 2 * Mh * My * nz * c + (Mx // 2 + 1) * (My // 2 + 1) * \
        (Mz // 2 + 1) * 8
    yi = Mh * nz * My * c + Mh * nz * ny * c
    xi = ny * nz * Mh * c + nx * ny * nz * 8
    return xf + yf + zc + yi + xi, (Mx, My, Mz)


def run_hartree(w, torch, steps, warmup, tune, reps=50):
    """The same workload with the Hartree term in the potential: ETRS step
    rate (FP64 and mixed) and the solve alone (HIP events around `reps`
    back-to-back solves of the workload's density on the grid's stream)."""
    from paper_1912_07921_amd import ks
    wh = copy.copy(w)
    wh.spec = copy.copy(w.spec)
    wh.spec.hartree = 1
    N, S = w.spec.npoints, w.spec.nk * w.spec.nstates
    res = {}
    for prec, key in ((0, "fp64"), (1, "mixed")):
        log(f"Hartree {key}: {warmup} warmup + {steps} timed steps")
        sec, _, _, prof, _, shape = run_gpu(wh, prec, steps, warmup, torch,
                                            tune)
        res[key] = dict(value=8.0 * N * S * steps / sec,
                        ms_per_step=1e3 * sec / steps, launch_shape=shape)
    g = ks.Grid(wh.spec)
    rho = g.density(to_dev(torch, w.psi0))
    vh = torch.empty_like(rho)
    for _ in range(5):
        g.hartree(rho, vh)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        g.hartree(rho, vh)
    e1.record(st)
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    nbytes, M = hartree_pipeline_bytes(wh.spec)
    res["solve"] = dict(us=round(us, 2), transform_lengths=list(M),
                        pipeline_bytes=nbytes,
                        achieved_GBs=round(nbytes / (us * 1e-6) / 1e9, 1),
                        frac_of_hbm_peak=round(nbytes / (us * 1e-6) / 1e9 /
                                               HBM_PEAK_GBS, 4),
                        solves_per_step=2)
    return res


def run_observables(w, torch, dip, reps=20):
    """The macroscopic current of the workload's states (kernel time from
    the grid's events, and per call with the host sums) and the strength
    function of the benchmark's own dipole trace on 2000 frequencies."""
    from paper_1912_07921_amd import ks
    g = ks.Grid(w.spec)
    psi = to_dev(torch, w.psi0)
    g.current(psi, 0.0)
    torch.cuda.synchronize()
    g.profile_begin(4 * reps + 16, classes=("reduce",))
    t0 = time.perf_counter()
    for _ in range(reps):
        J = g.current(psi, 0.0)
    wall = (time.perf_counter() - t0) / reps
    prof = g.profile_end()
    ms, n = prof["reduce"]
    N, S = w.spec.npoints, w.spec.nk * w.spec.nstates
    kern_us = 1e3 * ms / max(n, 1)
    res = dict(current_kernel_us=round(kern_us, 2),
               current_call_us=round(1e6 * wall, 2),
               current_states_GBs=round(16.0 * N * S / (kern_us * 1e-6) /
                                        1e9, 1),
               current_sample=[float(x) for x in J])
    if dip is not None:
        d = torch.from_numpy(np.ascontiguousarray(dip)).cuda()
        om = torch.linspace(0.0, 2.0, 2000, dtype=torch.float64,
                            device="cuda")
        ks.strength_function(d, w.dt, w.kick or 1.0, 0.1, om)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            ks.strength_function(d, w.dt, w.kick or 1.0, 0.1, om)
        e1.record(st)
        torch.cuda.synchronize()
        res["spectrum_us"] = round(1e3 * e0.elapsed_time(e1) / reps, 2)
        res["spectrum_samples_x_freqs"] = [int(d.shape[0]), 2000]
    return res


def serving_requests(torch, nreq, steps, rate):
    """The serving mix: request inputs built on the GPU, then held in pinned
    host memory as the payload each request brings (copied to HBM on
    admission)."""
    from paper_1912_07921_amd import workloads as W
    from paper_1912_07921_amd.serving import Request
    arrivals, make = W.c4_stream(nreq, rate=rate, nsteps=steps)
    reqs = []
    for i in range(nreq):
        w = make(i, device="cuda")
        reqs.append(Request(rid=i, arrival=float(arrivals[i]), spec=w.spec,
                            vion=w.vion.cpu().pin_memory(),
                            psi=w.psi0.cpu().pin_memory(), nsteps=steps,
                            dt=w.dt, kick=w.kick))
        del w
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return reqs


def run_serving(torch, nreq, steps, budget_gib, slots, loads=(0.8,)):
    """FP64 and FP32-mixed serving of the same requests.  A saturated run
    (every request waiting at t = 0) gives the FP64 capacity C in
    requests/s; both precisions are then run with Poisson arrivals at 0.5,
    0.8 and 1.2 C.  Each run reports p50/p99 per-(request, step) latency and
    aggregate point-states/s (for the saturated runs also as algorithmic
    bandwidth against the HBM peak); the mixed runs also report their
    largest dipole deviation from the FP64 run of the same request."""
    from paper_1912_07921_amd.serving import Request, Server
    from paper_1912_07921_amd import workloads as W
    base = serving_requests(torch, nreq, steps, 1.0)
    mean_ns = float(np.mean([r.pts_states for r in base]))

    def fresh(arrivals):
        return [Request(rid=r.rid, arrival=float(a), spec=r.spec,
                        vion=r.vion, psi=r.psi, nsteps=r.nsteps, dt=r.dt,
                        kick=r.kick) for r, a in zip(base, arrivals)]

    def serve(precision, arrivals):
        srv = Server(budget_gib * (1 << 30), max_slots=slots,
                     precision=precision)
        reqs = fresh(arrivals)
        st = srv.run(reqs)
        return st, {r.rid: r.dipole for r in reqs}

    out = dict(workload="c4 serving mix: grids {24,32,48,64,80}^3, states "
                        "{4,...,64}, 2-12 atoms s+p, LDA exchange, kick "
                        "0.01 z", requests=nreq, steps_per_request=steps,
               mean_points_x_states=mean_ns, hbm_budget_gib=budget_gib,
               slots=slots, offered_loads_of_capacity=list(loads))
    log(f"serving FP64: saturated run, {nreq} requests x {steps} steps")
    sat, d64 = serve(0, np.zeros(nreq))
    cap = nreq / sat["wall_s"]
    out["fp64"] = {"saturated": sat, "capacity_req_per_s": cap}
    log("serving mixed: saturated run")
    msat, dmx = serve(1, np.zeros(nreq))
    out["mixed"] = {"saturated": msat,
                    "capacity_req_per_s": nreq / msat["wall_s"],
                    "speedup_vs_fp64_saturated": msat["value"] / sat["value"]}
    errs = [max(float(np.abs(dmx[k] - d64[k]).max()) for k in d64)]
    # offered loads relative to the FP64 capacity C; both precisions see the
    # same arrival times
    for f in loads:
        lam = f * cap
        arrivals, _ = W.c4_stream(nreq, rate=lam, nsteps=steps)
        for prec, key in ((0, "fp64"), (1, "mixed")):
            log(f"serving {key}: Poisson arrivals at {lam:.2f} req/s "
                f"({f} C)")
            st, dd = serve(prec, arrivals)
            out[key][f"poisson_{f}C"] = dict(rate_req_per_s=lam, **st)
            if prec == 1:
                errs.append(max(float(np.abs(dd[k] - d64[k]).max())
                                for k in d64))
    out["mixed"]["dipole_err_vs_fp64_max"] = max(errs)
    # aggregate roofline of the saturated runs: the H.psi passes' algorithmic
    # bytes (STEP_BYTES / 8 per point-state and pass) at the aggregate rate
    for prec, key in ((0, "fp64"), (1, "mixed")):
        gbs = out[key]["saturated"]["value"] * STEP_BYTES[prec] / 8.0 / 1e9
        out[key]["aggregate_roofline"] = dict(
            achieved_GBs=round(gbs, 1), peak=HBM_PEAK_GBS,
            frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


def cpu_baseline(ws, sample_steps, full_states):
    """The oracle, as it stands, on the host cores: `sample_steps` ETRS steps
    of the sample workload `ws` (the benchmark's system with a subset of its
    states).  Returns the baseline record and the oracle's results (final
    states, dipole trace, norms, density, energy) for the error report."""
    from oracle import oracle
    o = oracle.Oracle(ws.spec)
    psi = o.kick(ws.psi0, ws.kick) if ws.kick else ws.psi0
    t = time.perf_counter()
    psi, dip, nrm = o.propagate_etrs(psi, ws.vion, sample_steps, ws.dt)
    sec = time.perf_counter() - t
    N, S = ws.spec.npoints, ws.spec.nk * ws.spec.nstates
    finite = not any(ws.spec.periodic)
    ref = dict(psi=psi, dipole=dip if finite else None, norms=nrm,
               rho=o.density(psi),
               energy=o.energy(psi, ws.vion, sample_steps * ws.dt))
    rec = dict(value=8.0 * N * S * sample_steps / sec,
               unit="grid-point·states/s", cores=oracle.num_threads(),
               kind="oracle",
               sample=f"{sample_steps} ETRS steps of the same system "
                      f"({ws.name}) with {S} of its {full_states} states "
                      f"(exchange from their density), {sec:.2f} s wall")
    return rec, ref


def errors_vs_oracle(ws, ref, sample_steps, precision, shape, torch):
    """The library's run of the oracle's sample (same states, steps and
    launch shape as the timed run) and its errors against the oracle:
    states (largest relative 2-norm), density and energy at the end
    (relative), dipole trace (absolute a.u. and relative to its largest
    component), norms (absolute)."""
    from paper_1912_07921_amd import ks
    finite = not any(ws.spec.periodic)
    g = ks.Grid(ws.spec, precision=precision)
    g.set_launch(*shape)
    psi = to_dev(torch, ws.psi0)
    vion = to_dev(torch, ws.vion)
    if ws.kick:
        g.kick(psi, ws.kick)
    d, n = g.propagate_etrs(psi, vion, sample_steps, ws.dt, dipole=finite,
                            norms=True)
    g64 = ks.Grid(ws.spec)
    rho = g64.density(psi).cpu().numpy()
    E = g64.energy(psi, vion, sample_steps * ws.dt)
    got = psi.cpu().numpy()
    g64.close()
    g.close()
    want = ref["psi"]
    err = dict(
        states_rel=max(float(np.linalg.norm(got[k, s] - want[k, s]) /
                             np.linalg.norm(want[k, s]))
                       for k in range(ws.spec.nk)
                       for s in range(ws.spec.nstates)),
        density_rel=float(np.abs(rho - ref["rho"]).max() /
                          np.abs(ref["rho"]).max()),
        energy_rel=abs(E - ref["energy"]) / abs(ref["energy"]),
        energy_Ha=E,
        norms_abs=float(np.abs(n.cpu().numpy() - ref["norms"]).max()))
    if finite:
        dd = float(np.abs(d.cpu().numpy() - ref["dipole"]).max())
        err["dipole_abs_au"] = dd
        err["dipole_rel"] = dd / float(np.abs(ref["dipole"]).max())
    return err


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo where there is one)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def shape_tuple(shape):
    """(tile rows, z-chunk, rows per thread) of a get_launch() record."""
    return (shape["tile_rows"], shape["zchunk"], shape["rows_per_thread"])


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c3",
                                                         "c5"])
    ap.add_argument("--cpu-steps", type=int, default=3,
                    help="oracle ETRS steps timed for the CPU baseline")
    ap.add_argument("--cpu-states", type=int, default=16,
                    help="states of the workload the oracle runs (its "
                         "first ones; all of them if fewer)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 2 GiB device copy (counter calibration)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cfm4", action="store_true")
    ap.add_argument("--no-hartree", action="store_true")
    ap.add_argument("--no-observables", action="store_true")
    ap.add_argument("--hartree-only", action="store_true",
                    help="only the step with the Hartree term and the solve "
                         "alone (profiling runs)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shape (no autotuner)")
    ap.add_argument("--shape", default="",
                    help="FP64 launch shape 'tile_rows,zchunk,rows_per_thread'"
                         " instead of the autotuner's (profiling runs)")
    ap.add_argument("--mixed-shape", default="",
                    help="the same for the mixed-precision leg")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-steps", type=int, default=200,
                    help="ETRS steps per request")
    ap.add_argument("--serving-loads", default="0.8",
                    help="offered loads (fractions of the saturated FP64 "
                         "capacity) of the Poisson-arrival runs, e.g. "
                         "0.5,0.8,1.2")
    ap.add_argument("--serving-budget-gib", type=float, default=96.0)
    ap.add_argument("--serving-slots", type=int, default=64)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the "
              "path would shard over states with one density all-reduce per "
              "half step, which this benchmark does not run.",
              file=sys.stderr)
        sys.exit(2)

    loads = tuple(float(v) for v in args.serving_loads.split(",") if v)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    if args.serving_only:
        print(json.dumps(run_serving(torch, args.serving_requests,
                                     args.serving_steps,
                                     args.serving_budget_gib,
                                     args.serving_slots, loads)), flush=True)
        return
    log(f"workload {args.workload}: generating inputs")
    w = make_workload(args.workload)
    N, S = w.spec.npoints, w.spec.nk * w.spec.nstates
    units = 8.0 * N * S
    if args.hartree_only:
        print(json.dumps(dict(workload=w.name, hartree=run_hartree(
            w, torch, args.steps, args.warmup, not args.no_tune))),
            flush=True)
        return

    log(f"FP64: {args.warmup} warmup + {args.steps} timed steps")
    fixed = tuple(int(v) for v in args.shape.split(",")) if args.shape \
        else None
    dipc64 = None
    sec, dip64, nrm64, prof, g64, shape = run_gpu(w, 0, args.steps,
                                                  args.warmup, torch,
                                                  not args.no_tune, fixed)
    log("standalone H.psi (ks_apply_h) over every state")
    apply_h = {"fp64": run_apply_h(g64, w, torch)}
    g64.close()
    del g64
    value = units * args.steps / sec
    hp_ms, hp_n = prof["hpsi"]
    avg_ms = hp_ms / max(hp_n, 1)
    bytes_per_launch = STEP_BYTES[0] / 8.0 * N * S
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    traffic = recorded_traffic(args.workload)
    roofline = dict(bound="hbm", achieved=round(achieved, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=traffic,
                    algorithmic_bytes_per_launch=bytes_per_launch,
                    kernel="k_hpsi (H.psi stencil pass)",
                    kernel_avg_us=round(1e3 * avg_ms, 2),
                    launch_shape=shape)
    copy_gbs = copy_bandwidth(torch)
    roofline["copy_GBs"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)
    # the whole step against the same peak: the algorithmic bytes of the
    # eight passes over the measured step time
    step_gbs = STEP_BYTES[0] * N * S / (sec / args.steps) / 1e9
    step_roofline = dict(achieved=round(step_gbs, 1), peak=HBM_PEAK_GBS,
                         unit="GB/s", frac=round(step_gbs / HBM_PEAK_GBS, 4),
                         algorithmic_bytes_per_step=STEP_BYTES[0] * N * S)
    kernel_times = {k: dict(total_ms=round(v[0], 3), launches=v[1],
                            avg_us=round(1e3 * v[0] / max(v[1], 1), 2))
                    for k, v in prof.items()}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point·states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "grid": list(w.spec.n), "h": w.spec.h[0],
            "periodic": any(w.spec.periodic),
            "kpoints": w.spec.nk, "states": S, "atoms": w.spec.natoms,
            "projectors_per_atom": int((max(w.spec.lmax) + 1) ** 2)
            if w.spec.natoms else 0,
            "xc": "LDA exchange" if w.spec.xc else "none",
            "dt": w.dt, "kick": w.kick,
        },
        "roofline": roofline,
        "step_roofline": step_roofline,
        "kernels": kernel_times,
        "apply_h": apply_h,
        # the paper reports no H.psi rate or bandwidth, only relative
        # whole-run GPU speed-ups on other hardware (context, not a target)
        "paper_context": ("Octopus GPU port on NVIDIA V100: a full GPU node "
                          "(2x V100 PCIe) 4.8x faster per TD step than a "
                          "full CPU node (2x Xeon 6148); 1.95/3.70/5.97x on "
                          "2/4/8 NVLink V100s with states distributed"),
    }

    if not args.no_mixed:
        log(f"mixed: {args.warmup} warmup + {args.steps} timed steps")
        mfixed = (tuple(int(v) for v in args.mixed_shape.split(","))
                  if args.mixed_shape else None)
        msec, dipm, nrmm, mprof, gm, mshape = run_gpu(w, 1, args.steps,
                                                      args.warmup, torch,
                                                      not args.no_tune, mfixed)
        apply_h["mixed"] = run_apply_h(gm, w, torch)
        gm.close()
        del gm
        mh_ms, mh_n = mprof["hpsi"]
        mavg = mh_ms / max(mh_n, 1)
        mach = STEP_BYTES[1] / 8.0 * N * S / (mavg / 1e3) / 1e9
        mixed = dict(value=units * args.steps / msec,
                     ms_per_step=1e3 * msec / args.steps,
                     speedup_vs_fp64=sec / msec,
                     roofline_achieved_GBs=round(mach, 1),
                     roofline_frac=round(mach / HBM_PEAK_GBS, 4),
                     step_frac=round(STEP_BYTES[1] * N * S /
                                     (msec / args.steps) / 1e9 /
                                     HBM_PEAK_GBS, 4),
                     norm_drift_max=float(abs(nrmm - nrm64).max()),
                     launch_shape=mshape,
                     traffic=recorded_traffic(
                         args.workload, "mixed_traffic_bytes_per_launch"))
        if dip64 is not None:
            mixed["dipole_err_vs_fp64"] = float(abs(dipm - dip64).max())
        out["mixed"] = mixed

    if not args.no_cfm4:
        # the order-four propagator of the paper: 8 H.psi per step as ETRS
        cf = {}
        for prec, key in ((0, "fp64"), (1, "mixed")):
            log(f"CFM4 {key}: {args.warmup} warmup + {args.steps} steps")
            csec, cdip, _, cprof, _, cshape = run_gpu(
                w, prec, args.steps, args.warmup, torch, not args.no_tune,
                fixed if prec == 0 else None, method="cfm4")
            ch_ms, ch_n = cprof["hpsi"]
            cf[key] = dict(value=units * args.steps / csec,
                           ms_per_step=1e3 * csec / args.steps,
                           hpsi_avg_us=round(1e3 * ch_ms / max(ch_n, 1), 2),
                           launch_shape=cshape)
            if prec == 1 and cdip is not None and dipc64 is not None:
                cf[key]["dipole_err_vs_fp64"] = float(
                    abs(cdip - dipc64).max())
            if prec == 0:
                dipc64 = cdip
        out["cfm4"] = cf

    per = w.spec.periodic
    if not args.no_hartree and (all(per) or not any(per)):
        hr = run_hartree(w, torch, args.steps, args.warmup, not args.no_tune)
        hr["fp64"]["step_cost_vs_no_hartree"] = round(
            hr["fp64"]["ms_per_step"] / out["ms_per_step"], 4)
        out["hartree"] = hr

    if not args.no_observables:
        log("observables: current and strength function")
        out["observables"] = run_observables(w, torch, dip64)

    if not args.no_serving:
        out["serving"] = run_serving(torch, args.serving_requests,
                                     args.serving_steps,
                                     args.serving_budget_gib,
                                     args.serving_slots, loads)

    if not args.no_cpu:
        ws = sample_workload(args.workload, min(args.cpu_states, S))
        log(f"CPU oracle: {args.cpu_steps} steps of {ws.name} with "
            f"{ws.spec.nk * ws.spec.nstates} states")
        rec, ref = cpu_baseline(ws, args.cpu_steps, S)
        rec["cpu_model"] = cpu_model()
        out["cpu_baseline"] = rec
        # the error of every result against the FP64 oracle, on the
        # oracle's sample, in the launch shapes of the timed runs
        log("errors against the oracle on its sample")
        ev = dict(sample=rec["sample"].rsplit(",", 1)[0])
        ev["fp64"] = errors_vs_oracle(ws, ref, args.cpu_steps, 0,
                                      shape_tuple(shape), torch)
        if "mixed" in out:
            ev["mixed"] = errors_vs_oracle(ws, ref, args.cpu_steps, 1,
                                           shape_tuple(mshape), torch)
        out["error_vs_oracle"] = ev
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
