"""Batched form (ks_batch_*) on the GPU: several jobs of different grids,
state counts, boundary conditions and terms propagated together must give
bitwise the results of propagating each job alone with ks_propagate_etrs
(the same kernels' arithmetic per point, only the work split differs), in
FP64 and in the mixed form; a replayed HIP graph must match eager launches
step by step, with unrelated eager work between the replays; and the FP64
batch must match the CPU oracle to the propagation tolerance (1e-10).
"""
import numpy as np
import pytest

from paper_1912_07921_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def normalised(spec, psi):
    h3 = np.prod(spec.h)
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2, axis=-1, keepdims=True) * h3)


def job_specs():
    """(spec, vion, psi, dt, t0) of four unlike jobs: every term with a laser
    in the pulse window, periodic Bloch k-points with a laser, the harmonic
    oscillator, and a projector-free, exchange-free grid."""
    out = []
    spec, v, psi = W.tiny(n=(17, 15, 14), nk=1, nstates=3, natoms=2, lmax=2,
                          rc=1.2, sigma=0.4, xc=1,
                          laser=(0.3, 0.8, 3.0, 0.2, 0.1, 0.9))
    out.append((spec, 0.3 * v, normalised(spec, psi), 0.01, 0.2))
    spec, v, psi = W.tiny(n=(16, 14, 15), h=(0.35, 0.35, 0.35),
                          periodic=(1, 1, 1), nk=2, nstates=2, natoms=2,
                          lmax=1, rc=1.1, sigma=0.4, xc=1,
                          laser=(0.3, 0.8, 3.0, 0.0, 0.0, 1.0))
    out.append((spec, 0.3 * v, normalised(spec, psi), 0.01, 0.0))
    w = W.c1()
    out.append((w.spec, w.vion, w.psi0, w.dt, 0.0))
    spec, v, psi = W.tiny(n=(21, 9, 12), nk=1, nstates=4, natoms=0, xc=0,
                          seed=11)
    out.append((spec, 0.5 * v, normalised(spec, psi), 0.02, 0.0))
    return out


def run_alone(torch, specs, nsteps, prec=0):
    from paper_1912_07921_amd import ks
    res = []
    for spec, v, psi, dt, t0 in specs:
        g = ks.Grid(spec, precision=prec)
        p = dev(torch, psi)
        d, n = g.propagate_etrs(p, dev(torch, v), nsteps, dt, t0,
                                dipole=not any(spec.periodic), norms=True)
        res.append((p.cpu().numpy(), None if d is None else d.cpu().numpy(),
                    n.cpu().numpy()))
    return res


def make_batch(torch, specs, max_steps, prec=0, use_graph=True):
    from paper_1912_07921_amd import ks
    jobs = []
    for spec, v, psi, dt, t0 in specs:
        g = ks.Grid(spec, precision=prec)
        jobs.append(ks.Job(g, dev(torch, psi), dev(torch, v), dt, max_steps,
                           t0=t0, dipole=not any(spec.periodic)))
    return ks.Batch(jobs, use_graph=use_graph), jobs


def results(jobs):
    return [(j.psi.cpu().numpy(),
             None if j.dipole is None else j.dipole.cpu().numpy(),
             j.norms.cpu().numpy()) for j in jobs]


def assert_same(a, b, what):
    for i, (x, y) in enumerate(zip(a, b)):
        for name, u, w in zip(("psi", "dipole", "norms"), x, y):
            if u is None:
                assert w is None
                continue
            assert np.array_equal(u, w), (what, i, name,
                                          np.abs(u - w).max())


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_each_job_alone(torch_cuda, prec):
    torch = torch_cuda
    specs = job_specs()
    alone = run_alone(torch, specs, 5, prec)
    b, jobs = make_batch(torch, specs, 5, prec)
    b.step(2)
    b.step(3)
    torch.cuda.synchronize()
    assert [b.steps_done(i) for i in range(len(jobs))] == [5] * len(jobs)
    assert_same(results(jobs), alone, f"precision {prec}")
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_reductions_with_every_table_membership(torch_cuda, prec):
    """The batched reductions (predictor and end-of-step densities, dipoles,
    norms: one launch each over tables of the jobs that need them) with jobs
    in every combination of those tables: a periodic job without exchange
    (no density at all) and without norms, a finite job with exchange but
    no dipole and no norms, a finite job with only a dipole, and one with
    everything.  Each must end bitwise as it does alone."""
    torch = torch_cuda
    from paper_1912_07921_amd import ks
    cases = []
    spec, v, psi = W.tiny(n=(14, 13, 12), h=(0.35, 0.35, 0.35),
                          periodic=(1, 1, 1), nk=2, nstates=2, natoms=1,
                          lmax=1, rc=1.1, sigma=0.4, xc=0, seed=21)
    cases.append((spec, 0.3 * v, normalised(spec, psi), False, False))
    spec, v, psi = W.tiny(n=(15, 14, 13), nstates=3, natoms=2, lmax=1,
                          rc=1.2, sigma=0.4, xc=1, seed=22)
    cases.append((spec, 0.3 * v, normalised(spec, psi), False, False))
    spec, v, psi = W.tiny(n=(13, 16, 14), nstates=2, natoms=0, xc=0,
                          seed=23)
    cases.append((spec, 0.5 * v, normalised(spec, psi), True, False))
    spec, v, psi = W.tiny(n=(16, 15, 17), nstates=4, natoms=2, lmax=2,
                          rc=1.2, sigma=0.4, xc=1, seed=24)
    cases.append((spec, 0.3 * v, normalised(spec, psi), True, True))
    dt, nsteps = 0.01, 4
    alone = []
    for spec, v, psi, dip, nrm in cases:
        g = ks.Grid(spec, precision=prec)
        p = dev(torch, psi)
        d, n = g.propagate_etrs(p, dev(torch, v), nsteps, dt, dipole=dip,
                                norms=nrm)
        alone.append((p.cpu().numpy(),
                      None if d is None else d.cpu().numpy(),
                      None if n is None else n.cpu().numpy()))
    jobs = []
    for spec, v, psi, dip, nrm in cases:
        g = ks.Grid(spec, precision=prec)
        jobs.append(ks.Job(g, dev(torch, psi), dev(torch, v), dt, nsteps,
                           dipole=dip, norms=nrm))
    b = ks.Batch(jobs)
    b.step(nsteps)
    torch.cuda.synchronize()
    got = [(j.psi.cpu().numpy(),
            None if j.dipole is None else j.dipole.cpu().numpy(),
            None if j.norms is None else j.norms.cpu().numpy())
           for j in jobs]
    assert_same(got, alone, f"precision {prec}")
    b.close()


def test_batch_matches_oracle(torch_cuda, oracle_mod):
    torch = torch_cuda
    specs = job_specs()
    b, jobs = make_batch(torch, specs, 4)
    b.step(4)
    got = results(jobs)
    for (spec, v, psi, dt, t0), (gp, gd, gn) in zip(specs, got):
        o = oracle_mod.Oracle(spec)
        want, wd, wn = o.propagate_etrs(psi, v, 4, dt, t0)
        N = spec.npoints
        e = np.linalg.norm(gp.reshape(-1, N) - want.reshape(-1, N), axis=1) / \
            np.linalg.norm(want.reshape(-1, N), axis=1)
        assert e.max() < 1e-10, e.max()
        assert np.abs(gn - wn).max() < 1e-10
        if gd is not None:
            assert np.abs(gd - wd).max() < 1e-10 * max(np.abs(wd).max(), 1e-3)
    b.close()


def test_graph_replays_match_eager_steps(torch_cuda):
    """Each replay of the captured step against the same step launched
    eagerly, with the program's own eager work and synchronisations in
    between."""
    torch = torch_cuda
    specs = job_specs()
    bg, jg = make_batch(torch, specs, 6, use_graph=True)
    be, je = make_batch(torch, specs, 6, use_graph=False)
    scratch = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
    for step in range(6):
        bg.step(1)
        scratch.normal_()
        s = float(scratch.sum())            # eager work, synchronising
        assert np.isfinite(s)
        be.step(1)
        torch.cuda.synchronize()
        assert_same(results(jg), results(je), f"step {step + 1}")
    bg.close()
    be.close()


def test_batch_full_size_with_small_job(torch_cuda):
    """A 64^3 grid with 32 states next to a 1-state harmonic oscillator."""
    torch = torch_cuda
    w = W.c2(nsteps=3)
    from paper_1912_07921_amd import ks
    g0 = ks.Grid(w.spec)
    p0 = dev(torch, w.psi0)
    g0.kick(p0, w.kick)
    kicked = p0.cpu().numpy()
    c1 = W.c1()
    specs = [(w.spec, w.vion, kicked, w.dt, 0.0),
             (c1.spec, c1.vion, c1.psi0, c1.dt, 0.0)]
    alone = run_alone(torch, specs, 3)
    b, jobs = make_batch(torch, specs, 3)
    b.step(3)
    assert_same(results(jobs), alone, "c2 + c1")
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_with_a_wide_row_job(torch_cuda, prec):
    """A job of 512-point rows (a tile row fills the 512-thread workgroup)
    beside a small periodic one: the batch launches every job's items with
    the widest workgroup, and each job still ends bitwise as alone (or the
    batch refuses the mix cleanly)."""
    torch = torch_cuda
    from paper_1912_07921_amd import ks
    s1, v1, p1 = W.tiny(n=(512, 6, 7), h=(0.12, 0.4, 0.4), nstates=2,
                        natoms=2, lmax=2, rc=1.1, sigma=0.35, xc=1)
    s2, v2, p2 = W.tiny(n=(12, 11, 10), periodic=(1, 1, 1), nk=2,
                        nstates=3, natoms=2, lmax=1, rc=1.0, sigma=0.35,
                        xc=1, seed=5)
    specs = [(s1, 0.3 * v1, normalised(s1, p1), 0.01, 0.0),
             (s2, 0.3 * v2, normalised(s2, p2), 0.01, 0.0)]
    alone = run_alone(torch, specs, 3, prec)
    try:
        b, jobs = make_batch(torch, specs, 3, prec)
    except ks.KSError as e:
        assert e.code == -4, e      # KS_E_UNSUPPORTED, nothing launched
        return
    b.step(3)
    torch.cuda.synchronize()
    assert_same(results(jobs), alone, f"wide rows, precision {prec}")
    b.close()


def test_batch_error_paths(torch_cuda):
    torch = torch_cuda
    from paper_1912_07921_amd import ks
    specs = job_specs()[2:]
    b, jobs = make_batch(torch, specs, 2)
    with pytest.raises(ks.KSError) as e:
        b.step(3)                  # past max_steps
    assert e.value.code == -1
    b.step(2)
    with pytest.raises(ks.KSError) as e:
        b.step(1)
    assert e.value.code == -1
    b.close()
    spec, v, psi, dt, t0 = specs[0]
    g = ks.Grid(spec)
    j = ks.Job(g, dev(torch, psi), dev(torch, v), dt, 1)
    with pytest.raises(ks.KSError) as e:
        ks.Batch([j, j])           # one grid twice
    assert e.value.code == -1
    gm = ks.Grid(spec, precision=1)
    jm = ks.Job(gm, dev(torch, psi), dev(torch, v), dt, 1)
    with pytest.raises(ks.KSError) as e:
        ks.Batch([j, jm])          # precisions differ
    assert e.value.code == -1
    with pytest.raises(ks.KSError) as e:
        ks.ks_batch_create([], torch.cuda.current_stream())
    assert e.value.code == -1


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_changes_speed_only(torch_cuda, prec):
    """The autotuner picks a valid launch shape; H.psi, the propagated
    states and the dipoles are bitwise those of the default shape.  The norm
    diagnostics sum per-tile partials, so their last bits follow the tiling
    (1e-14)."""
    torch = torch_cuda
    from paper_1912_07921_amd import ks
    spec, v, psi = W.tiny(n=(40, 27, 33), h=(0.25, 0.25, 0.25), nstates=3,
                          natoms=3, lmax=2, rc=1.3, sigma=0.4)
    psi = normalised(spec, psi)
    ref = ks.Grid(spec, precision=prec)
    ref.update_vlocal(dev(torch, v))
    p_ref = dev(torch, psi)
    h_ref = ref.apply_h(p_ref[0]).cpu().numpy()
    d_ref, n_ref = ref.propagate_etrs(p_ref, dev(torch, v), 3, 0.01)
    g = ks.Grid(spec, precision=prec)
    p = dev(torch, psi)
    ty, zc, rpt, us = g.autotune(p, reps=2)
    sh = g.get_launch()
    assert (sh["tile_rows"], sh["zchunk"], sh["rows_per_thread"]) == \
        (ty, zc, rpt)
    assert 1 <= ty <= 27 and 1 <= zc <= 33 and rpt in (1, 2) and us > 0
    g.update_vlocal(dev(torch, v))
    assert np.array_equal(g.apply_h(p[0]).cpu().numpy(), h_ref)
    d, n = g.propagate_etrs(p, dev(torch, v), 3, 0.01)
    assert np.array_equal(p.cpu().numpy(), p_ref.cpu().numpy())
    assert np.array_equal(d.cpu().numpy(), d_ref.cpu().numpy())
    assert np.abs(n.cpu().numpy() - n_ref.cpu().numpy()).max() < 1e-14
