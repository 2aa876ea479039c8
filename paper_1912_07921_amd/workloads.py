"""Seeded synthetic inputs shaped like the paper's workloads.

This module produces *inputs* only: grid/atom descriptions, the ionic local
potential v_ion, and initial Kohn-Sham states.  It holds none of the method's
arithmetic (no stencil, no projector, no propagator, no density): the CPU
oracle and the GPU library both take what it returns and compute on it with
code of their own.

Workloads (all in Hartree atomic units):
  c1  24^3, h 0.3, zero boundary, harmonic v = w^2 r^2 / 2 (w = 0.5), no
      atoms, 4 HO states (000), (100), (010), (001) times seeded global
      phases; dt 0.01, 50 steps, linear (no exchange).
  c2  64^3, h 0.2, zero boundary, 8 atoms uniform in a 4-bohr ball, Z in
      {1,4,6}, v_ion = -Z erf(r/0.5)/r, s+p KB projectors (rc 2, sigma 0.5,
      E ~ U[-2,2] per (atom, l)), 32 smooth random orthonormal states, LDA
      exchange, kick 0.01 along z, dt 0.005, 500 steps.
  c3  48^3, h 0.3, periodic, 4 k-points (2 pi / L)(+-1/4, +-1/4, 0), 16 atoms
      on a perturbed 2x2x2 cubic lattice with a 2-atom basis, periodic
      Gaussian-charge v_ion (G = 0 removed), 64 states per k, velocity-gauge
      laser A(t) = A0 sin^2(pi t/T) cos(w t) z (A0 0.05, w 0.057, T 20 fs),
      dt 0.02, 1000 steps.
  c4  serving mix: requests with grids {24,32,48,64,80}^3, states
      {4,8,16,32,64}, 2-12 atoms, c2 pseudopotential form, kick 0.01 z,
      200 steps each, Poisson arrivals.
  c5  128^3, h 0.18, 64 atoms in a 10-bohr ball, s+p+d projectors (rc 2.5,
      sigma 0.625), 256 states, LDA exchange, kick 0.01 z, dt 0.005, 100 steps.

Seeds are PCG64(1912_07921 + config number).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.special import erf

SEED_BASE = 1912_07921
FS_AU = 1.0 / 0.02418884326585747  # atomic units of time per femtosecond


@dataclass
class SystemSpec:
    """What a user of the method supplies: grid, k-points, states, atoms."""
    n: tuple
    h: tuple
    periodic: tuple = (0, 0, 0)
    kpts: np.ndarray = field(default_factory=lambda: np.zeros((1, 3)))
    kw: np.ndarray = field(default_factory=lambda: np.ones(1))
    nstates: int = 1
    occ: np.ndarray = None
    pos: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    Z: np.ndarray = field(default_factory=lambda: np.zeros(0))
    lmax: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    rc: np.ndarray = field(default_factory=lambda: np.zeros(0))
    sigma: np.ndarray = field(default_factory=lambda: np.zeros(0))
    E: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    xc: int = 0
    laser: tuple = (0.0, 0.0, 0.0, 0.0, 0.0, 1.0)
    hartree: int = 0

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        self.h = tuple(float(v) for v in self.h)
        self.periodic = tuple(int(v) for v in self.periodic)
        self.kpts = np.asarray(self.kpts, dtype=np.float64).reshape(-1, 3)
        self.kw = np.asarray(self.kw, dtype=np.float64).reshape(-1)
        if self.occ is None:
            self.occ = np.full(self.nstates, 2.0)
        self.occ = np.asarray(self.occ, dtype=np.float64).reshape(-1)
        self.pos = np.asarray(self.pos, dtype=np.float64).reshape(-1, 3)
        self.Z = np.asarray(self.Z, dtype=np.float64).reshape(-1)
        self.lmax = np.asarray(self.lmax, dtype=np.int32).reshape(-1)
        self.rc = np.asarray(self.rc, dtype=np.float64).reshape(-1)
        self.sigma = np.asarray(self.sigma, dtype=np.float64).reshape(-1)
        self.E = np.asarray(self.E, dtype=np.float64).reshape(-1, 3)
        self.laser = tuple(float(v) for v in self.laser)

    @property
    def npoints(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def nk(self):
        return len(self.kw)

    @property
    def natoms(self):
        return self.pos.shape[0]


@dataclass
class Workload:
    name: str
    spec: SystemSpec
    vion: np.ndarray          # [nz, ny, nx] float64, flattened x-fastest
    psi0: np.ndarray          # [nk, ns, nz, ny, nx] complex128
    dt: float
    nsteps: int
    kick: float = 0.0


# --------------------------------------------------------------------------
# grid coordinates of the inputs (same convention the method uses: symmetric
# about 0 on a zero-boundary axis, i*h on a periodic axis)
# --------------------------------------------------------------------------
def axis_coords(n, h, periodic):
    i = np.arange(n, dtype=np.float64)
    return i * h if periodic else (i - 0.5 * (n - 1)) * h


def grid_xyz(spec):
    x = axis_coords(spec.n[0], spec.h[0], spec.periodic[0])
    y = axis_coords(spec.n[1], spec.h[1], spec.periodic[1])
    z = axis_coords(spec.n[2], spec.h[2], spec.periodic[2])
    return x, y, z


# --------------------------------------------------------------------------
# local potentials
# --------------------------------------------------------------------------
def vion_harmonic(spec, omega):
    x, y, z = grid_xyz(spec)
    r2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
    return (0.5 * omega * omega * r2).reshape(-1)


def vion_erf(spec, rloc=0.5):
    """sum_a -Z_a erf(|r - R_a| / rloc) / |r - R_a|, limit at r = 0."""
    x, y, z = grid_xyz(spec)
    v = np.zeros((spec.n[2], spec.n[1], spec.n[0]))
    lim = 2.0 / (rloc * np.sqrt(np.pi))
    for a in range(spec.natoms):
        X, Y, Zc = spec.pos[a]
        r = np.sqrt((z[:, None, None] - Zc) ** 2 + (y[None, :, None] - Y) ** 2
                    + (x[None, None, :] - X) ** 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            f = np.where(r > 1e-12, erf(r / rloc) / np.where(r > 0, r, 1.0),
                         lim)
        v -= spec.Z[a] * f
    return v.reshape(-1)


def vion_periodic(spec, rloc=0.5):
    """Periodic sum of -Z erf(r/rloc)/r with a neutralising background.

    Each term is the potential of a Gaussian charge of width rloc, whose
    Fourier transform is -Z 4 pi exp(-G^2 rloc^2 / 4) / G^2; G = 0 removed.
    """
    nx, ny, nz = spec.n
    L = [spec.n[i] * spec.h[i] for i in range(3)]
    gx = 2 * np.pi * np.fft.fftfreq(nx, d=1.0 / nx) / L[0]
    gy = 2 * np.pi * np.fft.fftfreq(ny, d=1.0 / ny) / L[1]
    gz = 2 * np.pi * np.fft.fftfreq(nz, d=1.0 / nz) / L[2]
    GZ, GY, GX = np.meshgrid(gz, gy, gx, indexing="ij")
    G2 = GX ** 2 + GY ** 2 + GZ ** 2
    vol = L[0] * L[1] * L[2]
    sf = np.zeros_like(G2, dtype=np.complex128)
    for a in range(spec.natoms):
        X, Y, Zc = spec.pos[a]
        sf += spec.Z[a] * np.exp(-1j * (GX * X + GY * Y + GZ * Zc))
    with np.errstate(divide="ignore", invalid="ignore"):
        vg = -4 * np.pi * np.exp(-G2 * rloc * rloc / 4) / np.where(
            G2 > 0, G2, 1.0) / vol * sf
    vg[0, 0, 0] = 0.0
    v = np.fft.ifftn(vg) * (nx * ny * nz)
    return np.ascontiguousarray(v.real).reshape(-1)


# --------------------------------------------------------------------------
# initial states
# --------------------------------------------------------------------------
def _grid_dvol(spec):
    return spec.h[0] * spec.h[1] * spec.h[2]


def orthonormalise(psi, dvol):
    """Orthonormalise rows of psi (ns x N) in the grid inner product,
    in index order (the result equals modified Gram-Schmidt up to
    rounding), via the Cholesky factor of the Gram matrix."""
    G = (psi @ psi.conj().T) * dvol          # G_ij = <psi_j|psi_i>
    L = np.linalg.cholesky(G)                 # G = L L^H
    return np.linalg.solve(L, psi)            # rows of L^-1 psi


def smooth_random_states(spec, rng, nstates, k=None, mmax=3):
    """Random smooth fields: complex normal coefficients on Fourier modes
    |m_a| <= mmax; zero-boundary grids add a Gaussian envelope of width
    (half box)/2; Bloch grids multiply by exp(i k.r).  Orthonormalised."""
    x, y, z = grid_xyz(spec)
    L = [spec.n[i] * spec.h[i] for i in range(3)]
    ms = np.arange(-mmax, mmax + 1)
    ex = np.exp(2j * np.pi * np.outer(ms, x) / L[0])   # [m, x]
    ey = np.exp(2j * np.pi * np.outer(ms, y) / L[1])
    ez = np.exp(2j * np.pi * np.outer(ms, z) / L[2])
    nm = len(ms)
    c = (rng.standard_normal((nstates, nm, nm, nm))
         + 1j * rng.standard_normal((nstates, nm, nm, nm))) / np.sqrt(2)
    t = np.tensordot(c, ez, axes=([3], [0]))         # s, a, b, z
    t = np.tensordot(t, ey, axes=([2], [0]))         # s, a, z, y
    f = np.tensordot(t, ex, axes=([1], [0]))         # s, z, y, x
    if not any(spec.periodic):
        R = 0.5 * min(L)
        w = R / 2
        env = np.exp(-(z[:, None, None] ** 2 + y[None, :, None] ** 2
                       + x[None, None, :] ** 2) / (2 * w * w))
        f = f * env
    if k is not None:
        ph = np.exp(1j * (k[2] * z[:, None, None] + k[1] * y[None, :, None]
                          + k[0] * x[None, None, :]))
        f = f * ph
    psi = f.reshape(nstates, -1)
    return orthonormalise(psi, _grid_dvol(spec))


def ho_states(spec, omega, rng):
    """HO states (000), (100), (010), (001), sampled on the grid, normalised
    in the grid inner product, each times a seeded global phase."""
    x, y, z = grid_xyz(spec)
    Zg, Yg, Xg = np.meshgrid(z, y, x, indexing="ij")
    g = np.exp(-0.5 * omega * (Xg ** 2 + Yg ** 2 + Zg ** 2))
    fs = [g, Xg * g, Yg * g, Zg * g]
    out = []
    for f in fs[: spec.nstates]:
        f = f.reshape(-1).astype(np.complex128)
        f /= np.sqrt(np.sum(np.abs(f) ** 2) * _grid_dvol(spec))
        out.append(f * np.exp(1j * rng.uniform(0, 2 * np.pi)))
    return np.array(out)


def _atoms_in_ball(rng, natoms, radius, zchoices=(1.0, 4.0, 6.0)):
    u = rng.standard_normal((natoms, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = radius * rng.uniform(0, 1, natoms) ** (1.0 / 3.0)
    pos = u * r[:, None]
    Z = rng.choice(np.array(zchoices), natoms)
    return pos, Z


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def c1(nsteps=50):
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 1))
    spec = SystemSpec(n=(24, 24, 24), h=(0.3,) * 3, nstates=4, xc=0)
    v = vion_harmonic(spec, 0.5)
    psi = ho_states(spec, 0.5, rng).reshape(1, 4, -1)
    return Workload("c1_ho_24", spec, v, psi, dt=0.01, nsteps=nsteps)


def molecule(n, h, natoms, nstates, radius, lmax, rc, sigma, seed,
             xc=1, name="molecule", device=None):
    """A finite molecule-like system.  With `device` (a torch device) the
    potential and states are built there by torch from the same random
    draws (values equal to the CPU build up to rounding) and returned as
    device tensors."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, Z = _atoms_in_ball(rng, natoms, radius)
    E = rng.uniform(-2.0, 2.0, (natoms, 3))
    spec = SystemSpec(n=(n, n, n), h=(h,) * 3, nstates=nstates, pos=pos, Z=Z,
                      lmax=np.full(natoms, lmax), rc=np.full(natoms, rc),
                      sigma=np.full(natoms, sigma), E=E, xc=xc)
    if device is not None:
        v = vion_erf_device(spec, device)
        psi = smooth_random_states_device(spec, rng, nstates, device)
        return spec, v, psi.reshape(1, nstates, -1)
    v = vion_erf(spec)
    psi = smooth_random_states(spec, rng, nstates).reshape(1, nstates, -1)
    return spec, v, psi


def c2(nsteps=500, nstates=32, device=None):
    spec, v, psi = molecule(64, 0.2, 8, nstates, 4.0, 1, 2.0, 0.5,
                            SEED_BASE + 2, device=device)
    return Workload("c2_molecule_64", spec, v, psi, dt=0.005, nsteps=nsteps,
                    kick=0.01)


def c3(nsteps=1000, nstates=64, n=48, h=0.3):
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 3))
    L = n * h
    a = L / 2
    base = np.array([[i, j, k] for i in range(2) for j in range(2)
                     for k in range(2)], dtype=np.float64) * a
    pos = np.concatenate([base, base + 0.5 * a])
    pos += rng.uniform(-0.2, 0.2, pos.shape)
    pos %= L
    natoms = pos.shape[0]
    Z = rng.choice(np.array([1.0, 4.0, 6.0]), natoms)
    E = rng.uniform(-2.0, 2.0, (natoms, 3))
    q = 2 * np.pi / L
    kpts = q * np.array([[0.25, 0.25, 0], [0.25, -0.25, 0],
                         [-0.25, 0.25, 0], [-0.25, -0.25, 0]])
    spec = SystemSpec(n=(n, n, n), h=(h,) * 3, periodic=(1, 1, 1), kpts=kpts,
                      kw=np.full(4, 0.25), nstates=nstates, pos=pos, Z=Z,
                      lmax=np.full(natoms, 1), rc=np.full(natoms, 2.0),
                      sigma=np.full(natoms, 0.5), E=E, xc=1,
                      laser=(0.05, 0.057, 20.0 * FS_AU, 0.0, 0.0, 1.0))
    v = vion_periodic(spec)
    psi = np.stack([smooth_random_states(spec, rng, nstates, k=kpts[i])
                    for i in range(4)])
    return Workload("c3_crystal_48", spec, v, psi, dt=0.02, nsteps=nsteps)


def c5(nsteps=100, nstates=256, device=None):
    spec, v, psi = molecule(128, 0.18, 64, nstates, 10.0, 2, 2.5, 0.625,
                            SEED_BASE + 5, device=device)
    return Workload("c5_large_128", spec, v, psi, dt=0.005, nsteps=nsteps,
                    kick=0.01)


def serving_request(rng, grids=(24, 32, 48, 64, 80),
                    states=(4, 8, 16, 32, 64), nsteps=200):
    """One request of the c4 mix (atoms uniform within 0.3 of the half box)."""
    n = int(rng.choice(np.array(grids)))
    ns = int(rng.choice(np.array(states)))
    natoms = int(rng.integers(2, 13))
    h = 0.2
    seed = int(rng.integers(0, 2 ** 31))
    spec, v, psi = molecule(n, h, natoms, ns, 0.3 * 0.5 * n * h, 1, 2.0, 0.5,
                            seed, name="request")
    return Workload(f"req_{n}_{ns}_{natoms}", spec, v, psi, dt=0.005,
                    nsteps=nsteps, kick=0.01)


# --------------------------------------------------------------------------
# the same request inputs built on a GPU (torch), for serving runs that need
# hundreds of them: identical random draws, the contractions, envelope,
# erf potential and orthonormalisation done by torch on `device`.  Values
# equal the CPU path's up to rounding.
# --------------------------------------------------------------------------
def _torch_axes(spec, torch, device):
    x, y, z = grid_xyz(spec)
    t = lambda a: torch.from_numpy(a).to(device)
    return t(x), t(y), t(z)


def vion_erf_device(spec, device, rloc=0.5):
    import torch
    x, y, z = _torch_axes(spec, torch, device)
    v = torch.zeros((spec.n[2], spec.n[1], spec.n[0]), dtype=torch.float64,
                    device=device)
    lim = 2.0 / (rloc * np.sqrt(np.pi))
    for a in range(spec.natoms):
        X, Y, Zc = (float(c) for c in spec.pos[a])
        r = torch.sqrt((z[:, None, None] - Zc) ** 2 + (y[None, :, None] - Y) ** 2
                       + (x[None, None, :] - X) ** 2)
        safe = torch.where(r > 1e-12, r, torch.ones_like(r))
        f = torch.where(r > 1e-12, torch.special.erf(r / rloc) / safe,
                        torch.full_like(r, lim))
        v -= float(spec.Z[a]) * f
    return v.reshape(-1)


def smooth_random_states_device(spec, rng, nstates, device, mmax=3):
    """smooth_random_states for a zero-boundary grid, built on `device`."""
    import torch
    x, y, z = _torch_axes(spec, torch, device)
    L = [spec.n[i] * spec.h[i] for i in range(3)]
    ms = torch.arange(-mmax, mmax + 1, dtype=torch.float64, device=device)
    ex = torch.exp(2j * np.pi * torch.outer(ms, x) / L[0])
    ey = torch.exp(2j * np.pi * torch.outer(ms, y) / L[1])
    ez = torch.exp(2j * np.pi * torch.outer(ms, z) / L[2])
    nm = len(ms)
    c = (rng.standard_normal((nstates, nm, nm, nm))
         + 1j * rng.standard_normal((nstates, nm, nm, nm))) / np.sqrt(2)
    c = torch.from_numpy(c).to(device)
    t = torch.tensordot(c, ez, dims=([3], [0]))
    t = torch.tensordot(t, ey, dims=([2], [0]))
    f = torch.tensordot(t, ex, dims=([1], [0]))
    R = 0.5 * min(L)
    w = R / 2
    env = torch.exp(-(z[:, None, None] ** 2 + y[None, :, None] ** 2
                      + x[None, None, :] ** 2) / (2 * w * w))
    psi = (f * env).reshape(nstates, -1)
    G = ((psi @ psi.conj().T) * _grid_dvol(spec)).cpu().numpy()
    Linv = np.linalg.inv(np.linalg.cholesky(G))       # nstates x nstates
    return torch.from_numpy(Linv).to(device) @ psi


def serving_request_device(rng, device, grids=(24, 32, 48, 64, 80),
                           states=(4, 8, 16, 32, 64), nsteps=200):
    """serving_request with v_ion and the states built on `device`:
    (Workload with vion / psi0 as device tensors)."""
    n = int(rng.choice(np.array(grids)))
    ns = int(rng.choice(np.array(states)))
    natoms = int(rng.integers(2, 13))
    h = 0.2
    seed = int(rng.integers(0, 2 ** 31))
    r = np.random.Generator(np.random.PCG64(seed))
    pos, Z = _atoms_in_ball(r, natoms, 0.3 * 0.5 * n * h)
    E = r.uniform(-2.0, 2.0, (natoms, 3))
    spec = SystemSpec(n=(n, n, n), h=(h,) * 3, nstates=ns, pos=pos, Z=Z,
                      lmax=np.full(natoms, 1), rc=np.full(natoms, 2.0),
                      sigma=np.full(natoms, 0.5), E=E, xc=1)
    v = vion_erf_device(spec, device)
    psi = smooth_random_states_device(spec, r, ns, device).reshape(1, ns, -1)
    return Workload(f"req_{n}_{ns}_{natoms}", spec, v, psi, dt=0.005,
                    nsteps=nsteps, kick=0.01)


def c4_stream(nreq=256, rate=1.0, **kw):
    """(arrival times, request generator) for the serving mix."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 4))
    gaps = rng.exponential(1.0 / rate, nreq)
    arrivals = np.cumsum(gaps) - gaps[0]
    seeds = rng.integers(0, 2 ** 31, nreq)

    def make(i, device=None):
        r = np.random.Generator(np.random.PCG64(int(seeds[i])))
        if device is not None:
            return serving_request_device(r, device, **kw)
        return serving_request(r, **kw)

    return arrivals, make


def tiny(n=(8, 7, 8), h=(0.4, 0.35, 0.3), periodic=(0, 0, 0), nk=1,
         nstates=3, natoms=2, lmax=2, rc=1.1, sigma=0.35, xc=1, seed=7,
         laser=(0.0, 0.0, 0.0, 0.0, 0.0, 1.0)):
    """Small random system exercising every term (for brute-force checks)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 100 + seed))
    L = np.array([n[i] * h[i] for i in range(3)])
    if any(periodic):
        kpts = rng.uniform(-1, 1, (nk, 3)) * np.pi / L * np.array(periodic)
    else:
        kpts = np.zeros((nk, 3))
    pos = rng.uniform(-0.25, 0.25, (natoms, 3)) * L
    for ax in range(3):
        if periodic[ax]:
            pos[:, ax] = rng.uniform(0, L[ax], natoms)
    spec = SystemSpec(n=n, h=h, periodic=periodic, kpts=kpts,
                      kw=np.full(nk, 1.0 / nk), nstates=nstates,
                      occ=rng.uniform(0.5, 2.0, nstates), pos=pos,
                      Z=rng.choice(np.array([1.0, 4.0]), natoms),
                      lmax=np.full(natoms, lmax), rc=np.full(natoms, rc),
                      sigma=np.full(natoms, sigma),
                      E=rng.uniform(-2, 2, (natoms, 3)), xc=xc, laser=laser)
    v = rng.uniform(-1.0, 1.0, spec.npoints)
    N = spec.npoints
    psi = (rng.standard_normal((nk, nstates, N))
           + 1j * rng.standard_normal((nk, nstates, N)))
    return spec, v, psi
