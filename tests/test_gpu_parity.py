"""GPU (libks through its C ABI) against the FP64 CPU oracle, element by
element on the same seeded inputs.

Tolerances: H.psi in FP64 to 1e-12 relative (max over states of the 2-norm
of the difference over the 2-norm of the oracle's H.psi); FP64 propagation to
1e-10 relative on states, dipoles and norms; the mixed form to 1e-5 on H.psi
and to 1e-6 (absolute, atomic units) on dipole traces.
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


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def rel_err(got, want):
    """max over states of ||got - want|| / ||want||"""
    want = np.atleast_2d(want)
    got = np.asarray(got).reshape(want.shape)
    d = np.linalg.norm(got - want, axis=-1)
    w = np.linalg.norm(want, axis=-1)
    return float(np.max(d / np.maximum(w, 1e-300)))


def grid(spec, prec=0):
    from paper_1912_07921_amd import ks
    return ks.Grid(spec, precision=prec)


def apply_parity(torch, oracle_mod, spec, v, psi, A_t=0.0, prec=0, tol=1e-12):
    o = oracle_mod.Oracle(spec)
    g = grid(spec, prec)
    g.update_vlocal(dev(torch, v))
    A = o.laser_A(A_t)
    worst = 0.0
    for k in range(spec.nk):
        want = o.apply_h(v, psi[k], k=k, A=A)
        got = g.apply_h(dev(torch, psi[k]), k=k, t=A_t).cpu().numpy()
        worst = max(worst, rel_err(got.reshape(want.shape), want))
    assert worst < tol, worst
    return worst


# ---------------------------------------------------------------------------
# H.psi
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 1), (0, 1, 1)])
def test_apply_h_tiny_all_terms(torch_cuda, oracle_mod, periodic):
    laser = (0.4, 0.7, 5.0, 0.3, -0.5, 0.8)
    spec, v, psi = W.tiny(periodic=periodic, nk=2, nstates=3, natoms=2,
                          lmax=2, laser=laser)
    apply_parity(torch_cuda, oracle_mod, spec, v, psi, A_t=1.3)


def test_apply_h_ragged_tiles_and_chunks(torch_cuda, oracle_mod):
    """Grid sizes that leave ragged y-tiles, several z-chunks and x rows that
    are not a multiple of the wavefront."""
    spec, v, psi = W.tiny(n=(37, 29, 23), h=(0.21, 0.23, 0.25), nstates=5,
                          natoms=3, lmax=2, rc=1.4, sigma=0.45)
    apply_parity(torch_cuda, oracle_mod, spec, v, psi)


def test_apply_h_ragged_periodic_bloch(torch_cuda, oracle_mod):
    spec, v, psi = W.tiny(n=(19, 13, 21), h=(0.3, 0.35, 0.28),
                          periodic=(1, 1, 1), nk=3, nstates=2, natoms=3,
                          lmax=1, rc=1.1, sigma=0.4,
                          laser=(0.2, 0.9, 4.0, 0.0, 0.0, 1.0))
    apply_parity(torch_cuda, oracle_mod, spec, v, psi, A_t=0.8)


@pytest.mark.parametrize("n", [(1, 1, 1), (1, 2, 3), (3, 1, 2), (2, 5, 1)])
@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 1)])
def test_apply_h_degenerate_grids(torch_cuda, oracle_mod, n, periodic):
    """Axes shorter than the stencil: zero padding, or Bloch wraps that go
    round the cell several times."""
    spec, v, psi = W.tiny(n=n, h=(0.3, 0.4, 0.5), periodic=periodic, nk=1,
                          nstates=2, natoms=0)
    if any(periodic):
        spec.kpts = np.array([[0.7, -1.1, 0.4]])
    apply_parity(torch_cuda, oracle_mod, spec, v, psi)


@pytest.mark.parametrize("nx,periodic", [(192, (0, 0, 0)), (192, (1, 1, 0)),
                                         (256, (0, 0, 0)), (256, (1, 1, 1)),
                                         (320, (0, 0, 0)), (300, (1, 0, 0)),
                                         (512, (0, 0, 0)), (512, (1, 1, 0))])
@pytest.mark.parametrize("prec", [0, 1])
def test_apply_h_wide_rows(torch_cuda, oracle_mod, nx, periodic, prec):
    """Wide x-rows up to the widest the kernel takes (nx = 512: one row is
    a tile of 512 threads, and in FP64 the LDS planes alone exceed the
    default share, so the z-chunk is bounded by the CU's LDS only), rows
    that are not a multiple of the wavefront (300, 320), with projectors,
    Bloch wraps and the gauge term."""
    spec, v, psi = W.tiny(n=(nx, 7, 9), h=(0.15, 0.4, 0.4),
                          periodic=periodic, nk=1, nstates=2, natoms=2,
                          lmax=2, rc=1.1, sigma=0.35,
                          laser=(0.3, 0.8, 4.0, 0.6, 0.0, 0.8))
    apply_parity(torch_cuda, oracle_mod, spec, v, psi, A_t=1.1, prec=prec,
                 tol=1e-12 if prec == 0 else 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
def test_propagate_widest_rows(torch_cuda, oracle_mod, prec):
    """ETRS (every pass type, the density, exchange and dipole) on a grid
    of 512-point rows."""
    spec, v, psi = W.tiny(n=(512, 6, 7), h=(0.12, 0.4, 0.4), nk=1,
                          nstates=2, natoms=2, lmax=2, rc=1.1, sigma=0.35,
                          xc=1, laser=(0.3, 0.8, 3.0, 0.2, 0.1, 0.9))
    h3 = np.prod(spec.h)
    psi = psi / np.sqrt(np.sum(np.abs(psi) ** 2, axis=2, keepdims=True) * h3)
    res = propagate_parity(torch_cuda, oracle_mod, spec, 0.3 * v, psi, 3,
                           0.01, t0=0.2, kick=0.05, prec=prec, dip_tol=1e-6)
    if prec:
        assert res["psi"] < 1e-5, res


def test_apply_h_largest_grid(torch_cuda, oracle_mod):
    """The largest grid the library takes: 512 x 512 x 511 points (just
    under 2^27, so a state's last bytes sit just under the 2^31 byte
    offsets of the buffer accesses), 512-point rows, an atom with s+p+d
    projectors; every point against the oracle."""
    spec, v, psi = W.tiny(n=(512, 512, 511), h=(0.1, 0.1, 0.1), nstates=1,
                          natoms=1, lmax=2, rc=0.45, sigma=0.15, seed=13)
    assert spec.npoints < 2 ** 27 and spec.npoints * 16 > 2 ** 31 - 2 ** 23
    apply_parity(torch_cuda, oracle_mod, spec, v, psi)


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_h_many_states(torch_cuda, oracle_mod, prec):
    """A launch of 136 states (at least 128: the projector apply takes 8
    states per wavefront instead of 4; 136 leaves a ragged state group),
    periodic with k-points so the Bloch phases of the apply run too."""
    spec, v, psi = W.tiny(n=(14, 13, 12), h=(0.35, 0.35, 0.35),
                          periodic=(1, 1, 1), nk=2, nstates=136, natoms=3,
                          lmax=2, rc=1.3, sigma=0.4,
                          laser=(0.2, 0.9, 4.0, 0.0, 0.0, 1.0))
    apply_parity(torch_cuda, oracle_mod, spec, v, psi, A_t=0.8, prec=prec,
                 tol=1e-12 if prec == 0 else 1e-5)


def test_apply_h_no_states_and_sub_ranges(torch_cuda, oracle_mod):
    """ns = 0 is a no-op; a state sub-range [s0, s0+ns) of a k-point gives
    the rows of the full application."""
    torch = torch_cuda
    from paper_1912_07921_amd import ks
    spec, v, psi = W.tiny(n=(12, 11, 10), nk=2, nstates=4, natoms=2,
                          periodic=(1, 1, 1))
    g = grid(spec)
    g.update_vlocal(dev(torch, v))
    full = g.apply_h(dev(torch, psi[1]), k=1).cpu().numpy().reshape(4, -1)
    a = torch.zeros(1, dtype=torch.complex128, device="cuda")
    b = torch.zeros(1, dtype=torch.complex128, device="cuda")
    ks.ks_apply_h(g.h, a, b, 1, 2, 0, 0.0)            # nothing to do
    assert float(b.abs().sum()) == 0.0
    sub = dev(torch, psi[1][1:3])
    got = torch.empty_like(sub)
    ks.ks_apply_h(g.h, sub, got, 1, 1, 2, 0.0)
    assert np.array_equal(got.cpu().numpy().reshape(2, -1), full[1:3])


def test_apply_h_c1(torch_cuda, oracle_mod):
    w = W.c1()
    apply_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0)


def test_apply_h_c2_full(torch_cuda, oracle_mod):
    w = W.c2(nsteps=1)
    apply_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0)


def test_apply_h_c3_full_with_laser(torch_cuda, oracle_mod):
    w = W.c3(nsteps=1)
    # at the envelope maximum, so the gauge term is large
    apply_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0,
                 A_t=0.5 * w.spec.laser[2])


def test_apply_h_mixed_c2(torch_cuda, oracle_mod):
    w = W.c2(nsteps=1)
    err = apply_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0,
                       prec=1, tol=1e-5)
    assert err > 1e-10   # the FP32 path really is FP32


# ---------------------------------------------------------------------------
# density, LDA potential, dipole, kick, norms, Gram, energy
# ---------------------------------------------------------------------------
def test_observables_match_oracle(torch_cuda, oracle_mod):
    torch = torch_cuda
    spec, v, psi = W.tiny(n=(21, 18, 17), nk=1, nstates=4, natoms=2, lmax=2,
                          rc=1.3, sigma=0.4)
    o = oracle_mod.Oracle(spec)
    g = grid(spec)
    dpsi = dev(torch, psi)
    rho = g.density(dpsi).cpu().numpy()
    want = o.density(psi)
    assert np.abs(rho - want).max() < 1e-13 * np.abs(want).max()
    d = g.dipole(dev(torch, want))
    assert np.abs(d - o.dipole(want)).max() < 1e-12 * np.abs(d).max()
    g.update_vlocal(dev(torch, v), dev(torch, want))
    # the potential is observable through H.psi
    hp = g.apply_h(dev(torch, psi[0])).cpu().numpy().reshape(psi[0].shape)
    assert rel_err(hp, o.apply_h(o.vlocal(v, want), psi[0])) < 1e-12
    nr = g.norms(dpsi).cpu().numpy()
    assert np.abs(nr - o.norms(psi)).max() < 1e-12 * nr.max()
    G = g.gram(dpsi).cpu().numpy()
    Go = o.gram(psi)
    assert np.abs(G - Go).max() < 1e-12 * np.abs(Go).max()
    e = g.energy(dpsi, dev(torch, v))
    eo = o.energy(psi, v)
    assert abs(e - eo) < 1e-11 * abs(eo)
    g.kick(dpsi, 0.37)
    assert np.abs(dpsi.cpu().numpy() - o.kick(psi, 0.37)).max() < 1e-14 * \
        np.abs(psi).max()


@pytest.mark.parametrize("nstates", [5, 32, 40, 64, 70, 130])
def test_gram_tiles(torch_cuda, oracle_mod, nstates):
    """The Gram matrix on the matrix cores: one small tile (5, 32 states),
    one large tile partly or wholly filled (40, 64), and several tiles with
    a ragged last one (70, 130), 4 k-points, against the oracle."""
    torch = torch_cuda
    w = W.c3(nsteps=1, nstates=nstates, n=16, h=0.45)
    o = oracle_mod.Oracle(w.spec)
    G = grid(w.spec).gram(dev(torch, w.psi0)).cpu().numpy()
    assert np.abs(G - o.gram(w.psi0)).max() < 1e-12
    if nstates <= 40:     # below the 16^3 grid's resolution: orthonormal
        assert np.abs(G - np.eye(nstates)[None]).max() < 1e-11


def test_gram_ragged_grid(torch_cuda, oracle_mod):
    """70 states (two 64-state tiles, the second ragged) on a 17^3 grid
    (4913 points: the last 32-point stage of a slice is partly empty)."""
    torch = torch_cuda
    w = W.c3(nsteps=1, nstates=70, n=17, h=0.45)
    o = oracle_mod.Oracle(w.spec)
    G = grid(w.spec).gram(dev(torch, w.psi0)).cpu().numpy()
    Go = o.gram(w.psi0)
    assert np.abs(G - Go).max() < 1e-12 * np.abs(Go).max()


# ---------------------------------------------------------------------------
# ETRS propagation
# ---------------------------------------------------------------------------
def propagate_parity(torch, oracle_mod, spec, v, psi, nsteps, dt, t0=0.0,
                     prec=0, kick=0.0, tol=1e-10, dip_tol=None,
                     method="etrs"):
    o = oracle_mod.Oracle(spec)
    if kick:
        psi = o.kick(psi, kick)
    want, wd, wn = getattr(o, "propagate_" + method)(psi, v, nsteps, dt, t0)
    g = grid(spec, prec)
    dpsi = dev(torch, psi)
    periodic = any(spec.periodic)
    d, n = getattr(g, "propagate_" + method)(dpsi, dev(torch, v), nsteps, dt,
                                             t0, dipole=not periodic,
                                             norms=True)
    got = dpsi.cpu().numpy()
    e_psi = rel_err(got.reshape(-1, o.N), want.reshape(-1, o.N))
    e_norm = np.abs(n.cpu().numpy() - wn).max()
    res = dict(psi=e_psi, norm=e_norm)
    if not periodic:
        dd = d.cpu().numpy()
        res["dip"] = np.abs(dd - wd).max()
        res["dip_scale"] = np.abs(wd).max()
    if prec == 0:
        assert e_psi < tol, res
        assert e_norm < tol, res
        if not periodic:
            assert res["dip"] < tol * max(res["dip_scale"], 1e-3), res
    else:
        if not periodic:
            assert res["dip"] < dip_tol, res
    return res


def test_propagate_c1_full_length(torch_cuda, oracle_mod):
    w = W.c1()
    propagate_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0,
                     w.nsteps, w.dt)


def test_propagate_tiny_every_term(torch_cuda, oracle_mod):
    spec, v, psi = W.tiny(n=(17, 15, 14), nk=1, nstates=3, natoms=2, lmax=2,
                          rc=1.2, sigma=0.4, xc=1,
                          laser=(0.3, 0.8, 3.0, 0.2, 0.1, 0.9))
    h3 = np.prod(spec.h)
    psi = psi / np.sqrt(np.sum(np.abs(psi) ** 2, axis=2, keepdims=True) * h3)
    propagate_parity(torch_cuda, oracle_mod, spec, 0.3 * v, psi, 6, 0.01,
                     t0=0.2, kick=0.05)


def test_propagate_periodic_kpoints(torch_cuda, oracle_mod):
    spec, v, psi = W.tiny(n=(16, 14, 15), h=(0.35, 0.35, 0.35),
                          periodic=(1, 1, 1), nk=2, nstates=2, natoms=2,
                          lmax=1, rc=1.1, sigma=0.4, xc=1,
                          laser=(0.3, 0.8, 3.0, 0.0, 0.0, 1.0))
    h3 = np.prod(spec.h)
    psi = psi / np.sqrt(np.sum(np.abs(psi) ** 2, axis=2, keepdims=True) * h3)
    propagate_parity(torch_cuda, oracle_mod, spec, 0.3 * v, psi, 4, 0.01)


def test_propagate_c2_full_size_few_steps(torch_cuda, oracle_mod):
    w = W.c2(nsteps=4)
    propagate_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0,
                     w.nsteps, w.dt, kick=w.kick)


def test_propagate_mixed_c2_dipole(torch_cuda, oracle_mod):
    w = W.c2(nsteps=8)
    res = propagate_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0,
                           w.nsteps, w.dt, kick=w.kick, prec=1,
                           dip_tol=1e-6)
    assert res["psi"] < 1e-4, res


def test_propagate_zero_steps_reports_initial_observables(torch_cuda,
                                                          oracle_mod):
    w = W.c1()
    propagate_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0, 0, w.dt)


# ---------------------------------------------------------------------------
# error paths (host-side checks; every kernel exits normally)
# ---------------------------------------------------------------------------
def test_error_paths(torch_cuda):
    torch = torch_cuda
    from paper_1912_07921_amd import ks
    spec, v, psi = W.tiny(nstates=2, natoms=1)
    g = grid(spec)
    dpsi = dev(torch, psi[0])
    with pytest.raises(ks.KSError) as e:
        g.apply_h(dpsi)            # no potential yet
    assert e.value.code == -5
    g.update_vlocal(dev(torch, v))
    with pytest.raises(ks.KSError) as e:
        g.apply_h(dpsi, k=3)
    assert e.value.code == -1
    with pytest.raises(ks.KSError) as e:
        ks.ks_apply_h(g.h, dpsi, dpsi, 0, 0, 2, 0.0)
    assert e.value.code == -1
    bad = W.tiny(periodic=(1, 1, 1), rc=5.0)[0]
    with pytest.raises(ks.KSError) as e:
        grid(bad)
    assert e.value.code == -4
    with pytest.raises(ValueError):
        g.dipole(dev(torch, np.zeros(spec.npoints + 1)))
    per, pv, _ = W.tiny(periodic=(1, 1, 1), natoms=0)
    gp = grid(per)
    with pytest.raises(ks.KSError) as e:
        gp.dipole(dev(torch, np.zeros(per.npoints)))
    assert e.value.code == -4


def test_apply_h_independent_of_launch_shape(torch_cuda, oracle_mod):
    """Tile height and z-chunking change only the work split: H.psi is
    bitwise the same for every shape."""
    torch = torch_cuda
    spec, v, psi = W.tiny(n=(40, 27, 33), h=(0.25, 0.25, 0.25), nstates=3,
                          natoms=3, lmax=2, rc=1.3, sigma=0.4)
    g = grid(spec)
    g.update_vlocal(dev(torch, v))
    dpsi = dev(torch, psi[0])
    ref = g.apply_h(dpsi).cpu().numpy()
    want = oracle_mod.Oracle(spec).apply_h(v, psi[0])
    assert rel_err(ref, want) < 1e-12
    # (tile rows, z-chunk, rows per thread)
    for ty, zc, rpt in [(1, 0, 1), (2, 5, 1), (3, 33, 1), (7, 1, 1),
                        (12, 16, 1), (12, 0, 1), (20, 0, 2), (24, 7, 2),
                        (8, 3, 2), (5, 0, 2), (2, 9, 2)]:
        g.set_launch(ty, zc, rpt)
        sh = g.get_launch()
        assert (sh["tile_rows"], sh["rows_per_thread"]) == (ty, rpt)
        got = g.apply_h(dpsi).cpu().numpy()
        assert np.array_equal(got, ref), (ty, zc, rpt)


def test_propagate_independent_of_launch_shape(torch_cuda, oracle_mod):
    torch = torch_cuda
    w = W.c1(nsteps=3)
    outs = []
    for ty, zc in [(0, 0), (3, 7), (16, 24)]:
        g = grid(w.spec)
        g.set_launch(ty, zc)
        dpsi = dev(torch, w.psi0)
        g.propagate_etrs(dpsi, dev(torch, w.vion), 3, w.dt)
        outs.append(dpsi.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


# ---------------------------------------------------------------------------
# CFM4 propagation
# ---------------------------------------------------------------------------
def test_cfm4_c1_full_length(torch_cuda, oracle_mod):
    w = W.c1()
    propagate_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0,
                     w.nsteps, w.dt, method="cfm4")


def test_cfm4_tiny_every_term(torch_cuda, oracle_mod):
    """Exchange, projectors and a laser: 7 steps cover the start-up
    extrapolation orders (1, 2, 3 points) and the steady cubic one."""
    spec, v, psi = W.tiny(n=(17, 15, 14), nk=1, nstates=3, natoms=2, lmax=2,
                          rc=1.2, sigma=0.4, xc=1,
                          laser=(0.3, 0.8, 3.0, 0.2, 0.1, 0.9))
    h3 = np.prod(spec.h)
    psi = psi / np.sqrt(np.sum(np.abs(psi) ** 2, axis=2, keepdims=True) * h3)
    propagate_parity(torch_cuda, oracle_mod, spec, 0.3 * v, psi, 7, 0.01,
                     t0=0.2, kick=0.05, method="cfm4")


def test_cfm4_periodic_kpoints(torch_cuda, oracle_mod):
    spec, v, psi = W.tiny(n=(16, 14, 15), h=(0.35, 0.35, 0.35),
                          periodic=(1, 1, 1), nk=2, nstates=2, natoms=2,
                          lmax=1, rc=1.1, sigma=0.4, xc=1,
                          laser=(0.3, 0.8, 3.0, 0.0, 0.0, 1.0))
    h3 = np.prod(spec.h)
    psi = psi / np.sqrt(np.sum(np.abs(psi) ** 2, axis=2, keepdims=True) * h3)
    propagate_parity(torch_cuda, oracle_mod, spec, 0.3 * v, psi, 5, 0.01,
                     method="cfm4")


def test_cfm4_c2_full_size_few_steps(torch_cuda, oracle_mod):
    w = W.c2(nsteps=5)
    propagate_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0,
                     w.nsteps, w.dt, kick=w.kick, method="cfm4")


def test_cfm4_mixed_c2_dipole(torch_cuda, oracle_mod):
    w = W.c2(nsteps=8)
    res = propagate_parity(torch_cuda, oracle_mod, w.spec, w.vion, w.psi0,
                           w.nsteps, w.dt, kick=w.kick, prec=1,
                           dip_tol=1e-6, method="cfm4")
    assert res["psi"] < 1e-4, res


def test_overlapped_halves_give_the_same_propagation(torch_cuda):
    """States propagated in two halves on two streams (projector kernels of
    one half beside the stencil of the other) end bitwise where one chain
    ends, dipole and norms included."""
    torch = torch_cuda
    w = W.c2(nsteps=3)
    outs = []
    for halves in (1, 2):
        g = grid(w.spec)
        g.set_overlap(halves)
        p = dev(torch, w.psi0)
        d, n = g.propagate_etrs(p, dev(torch, w.vion), 3, w.dt)
        d4, n4 = g.propagate_cfm4(p, dev(torch, w.vion), 2, w.dt)
        outs.append([x.cpu().numpy() for x in (p, d, n, d4, n4)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
