"""ctypes wrapper of the plain-C FP64 oracle (ks_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It imports
nothing from the product package; the system description it takes is any
object with the attributes listed in ``_Desc`` below (duck-typed), so the same
seeded inputs can be handed to both sides.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ks_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile ks_oracle.c into liboracle.so with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Desc(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3),
        ("h", C.c_double * 3),
        ("periodic", C.c_int * 3),
        ("nk", C.c_int),
        ("kpts", C.POINTER(C.c_double)),
        ("kw", C.POINTER(C.c_double)),
        ("nstates", C.c_int),
        ("occ", C.POINTER(C.c_double)),
        ("natoms", C.c_int),
        ("pos", C.POINTER(C.c_double)),
        ("lmax", C.POINTER(C.c_int)),
        ("rc", C.POINTER(C.c_double)),
        ("sigma", C.POINTER(C.c_double)),
        ("E", C.POINTER(C.c_double)),
        ("xc", C.c_int),
        ("laser", C.c_double * 6),
        ("hartree", C.c_int),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        vp = C.c_void_p
        lib.orc_create.restype = vp
        lib.orc_create.argtypes = [C.POINTER(_Desc)]
        lib.orc_destroy.argtypes = [vp]
        lib.orc_npoints.restype = C.c_long
        lib.orc_npoints.argtypes = [vp]
        lib.orc_atom_npts.restype = C.c_int
        lib.orc_atom_npts.argtypes = [vp, C.c_int]
        lib.orc_atom_table.argtypes = [vp, C.c_int, vp, vp]
        lib.orc_apply_h.argtypes = [vp, vp, C.c_int, vp, C.c_int, vp, vp]
        lib.orc_laser_A.argtypes = [vp, C.c_double, vp]
        lib.orc_density.argtypes = [vp, vp, vp]
        lib.orc_vlocal.argtypes = [vp, vp, vp, vp]
        lib.orc_exchange_energy.restype = C.c_double
        lib.orc_exchange_energy.argtypes = [vp, vp]
        lib.orc_dipole.argtypes = [vp, vp, vp]
        lib.orc_kick.argtypes = [vp, vp, C.c_double]
        lib.orc_norms.argtypes = [vp, vp, vp]
        lib.orc_gram.argtypes = [vp, vp, vp]
        lib.orc_energy.restype = C.c_double
        lib.orc_energy.argtypes = [vp, vp, vp, C.c_double]
        lib.orc_taylor4.argtypes = [vp, vp, C.c_int, vp, C.c_double, C.c_int,
                                    vp, vp]
        lib.orc_propagate_etrs.restype = C.c_int
        lib.orc_propagate_etrs.argtypes = [vp, vp, vp, C.c_int, C.c_double,
                                           C.c_double, vp, vp]
        lib.orc_propagate_cfm4.restype = C.c_int
        lib.orc_propagate_cfm4.argtypes = [vp, vp, vp, C.c_int, C.c_double,
                                           C.c_double, vp, vp]
        lib.orc_hartree.restype = C.c_int
        lib.orc_hartree.argtypes = [vp, vp, vp]
        lib.orc_hartree_at.restype = C.c_int
        lib.orc_hartree_at.argtypes = [vp, vp, vp, C.c_int, vp]
        lib.orc_hartree_energy.restype = C.c_double
        lib.orc_hartree_energy.argtypes = [vp, vp]
        lib.orc_coulomb_cell_mean.restype = C.c_double
        lib.orc_coulomb_cell_mean.argtypes = [vp]
        lib.orc_comm_r.argtypes = [vp, C.c_int, C.c_double, C.c_int, C.c_int,
                                   vp, vp]
        lib.orc_current.argtypes = [vp, vp, C.c_double, vp]
        lib.orc_strength_function.argtypes = [vp, C.c_int, C.c_double,
                                              C.c_double, C.c_double, vp,
                                              C.c_int, vp]
        lib.orc_conductivity.argtypes = [vp, C.c_int, C.c_double, C.c_double,
                                         C.c_double, vp, C.c_int, vp]
        lib.orc_num_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """One system (grid, k-points, occupations, atoms) on the CPU oracle.

    ``spec`` needs: n, h, periodic (3 each), kpts (nk x 3), kw (nk),
    nstates, occ (nstates), pos (natoms x 3), lmax, rc, sigma (natoms),
    E (natoms x 3), xc (0/1), laser (6); optionally hartree (0/1).
    """

    def __init__(self, spec):
        lib = _load()
        self.spec = spec
        self.n = tuple(int(v) for v in spec.n)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.nk = int(len(spec.kw))
        self.ns = int(spec.nstates)
        self._keep = [
            _f64(spec.kpts, (self.nk, 3)), _f64(spec.kw), _f64(spec.occ),
            _f64(spec.pos).reshape(-1, 3),
            np.ascontiguousarray(spec.lmax, dtype=np.int32),
            _f64(spec.rc), _f64(spec.sigma), _f64(spec.E).reshape(-1, 3),
        ]
        kp, kw, occ, pos, lmax, rc, sg, E = self._keep
        d = _Desc()
        d.n[:] = list(self.n)
        d.h[:] = [float(v) for v in spec.h]
        d.periodic[:] = [int(v) for v in spec.periodic]
        d.nk = self.nk
        d.kpts = kp.ctypes.data_as(C.POINTER(C.c_double))
        d.kw = kw.ctypes.data_as(C.POINTER(C.c_double))
        d.nstates = self.ns
        d.occ = occ.ctypes.data_as(C.POINTER(C.c_double))
        d.natoms = int(pos.shape[0])
        d.pos = pos.ctypes.data_as(C.POINTER(C.c_double))
        d.lmax = lmax.ctypes.data_as(C.POINTER(C.c_int))
        d.rc = rc.ctypes.data_as(C.POINTER(C.c_double))
        d.sigma = sg.ctypes.data_as(C.POINTER(C.c_double))
        d.E = E.ctypes.data_as(C.POINTER(C.c_double))
        d.xc = int(spec.xc)
        d.laser[:] = [float(v) for v in spec.laser]
        d.hartree = int(getattr(spec, "hartree", 0))
        self.natoms = d.natoms
        self._d = d
        h = lib.orc_create(C.byref(d))
        if not h:
            raise ValueError("oracle rejected the system description")
        self._h = C.c_void_p(h)
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and self._lib is not None:
            self._lib.orc_destroy(h)
            self._h = None

    # -- helpers -----------------------------------------------------------
    def _c128(self, psi, count):
        a = np.ascontiguousarray(psi, dtype=np.complex128)
        if a.size != count * self.N:
            raise ValueError(f"expected {count} states of {self.N} points")
        return a

    def atom_table(self, a):
        """(grid indices, nproj x npts projector table) of atom a."""
        npts = self._lib.orc_atom_npts(self._h, a)
        lmax = int(np.asarray(self.spec.lmax)[a])
        nproj = (lmax + 1) ** 2
        idx = np.zeros(max(npts, 1), dtype=np.int32)
        p = np.zeros((nproj, max(npts, 1)), dtype=np.float64)
        self._lib.orc_atom_table(self._h, a, _ptr(idx), _ptr(p))
        return idx[:npts], p[:, :npts]

    def laser_A(self, t):
        A = np.zeros(3)
        self._lib.orc_laser_A(self._h, float(t), _ptr(A))
        return A

    # -- operations ----------------------------------------------------------
    def apply_h(self, v, psi, k=0, A=(0.0, 0.0, 0.0)):
        """H psi for the states in psi (ns' x N complex) at k-point k;
        returns an (ns', N) array."""
        psi = np.ascontiguousarray(psi, dtype=np.complex128).reshape(
            -1, self.N)
        ns = psi.shape[0]
        psi = self._c128(psi, ns)
        v = _f64(v)
        A = _f64(A)
        out = np.empty_like(psi)
        self._lib.orc_apply_h(self._h, _ptr(v), int(k), _ptr(A), ns,
                              _ptr(psi), _ptr(out))
        return out

    def taylor4(self, v, psi, tau, k=0, A=(0.0, 0.0, 0.0)):
        psi = np.ascontiguousarray(psi, dtype=np.complex128).reshape(
            -1, self.N)
        ns = psi.shape[0]
        v = _f64(v)
        A = _f64(A)
        out = np.empty_like(psi)
        self._lib.orc_taylor4(self._h, _ptr(v), int(k), _ptr(A), float(tau),
                              ns, _ptr(psi), _ptr(out))
        return out

    def density(self, psi):
        psi = self._c128(psi, self.nk * self.ns)
        rho = np.empty(self.N)
        self._lib.orc_density(self._h, _ptr(psi), _ptr(rho))
        return rho

    def vlocal(self, vion, rho=None):
        vion = _f64(vion)
        v = np.empty(self.N)
        if rho is None:
            self._lib.orc_vlocal(self._h, _ptr(vion), None, _ptr(v))
        else:
            rho = _f64(rho)
            self._lib.orc_vlocal(self._h, _ptr(vion), _ptr(rho), _ptr(v))
        return v

    def exchange_energy(self, rho):
        rho = _f64(rho)
        return self._lib.orc_exchange_energy(self._h, _ptr(rho))

    def hartree(self, rho):
        """v_H[rho] (reading R11 of ks_oracle.c)."""
        rho = _f64(rho)
        if rho.size != self.N:
            raise ValueError(f"expected {self.N} density values")
        vh = np.empty(self.N)
        if self._lib.orc_hartree(self._h, _ptr(rho), _ptr(vh)) != 0:
            raise ValueError("Hartree potential of a mixed-periodicity grid")
        return vh

    def hartree_at(self, rho, idx):
        """v_H[rho] at the listed grid points of a finite grid."""
        rho = _f64(rho)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.empty(len(idx))
        if self._lib.orc_hartree_at(self._h, _ptr(rho), _ptr(idx), len(idx),
                                    _ptr(out)) != 0:
            raise ValueError("sampled Hartree potential of a periodic grid")
        return out

    def hartree_energy(self, rho):
        rho = _f64(rho)
        return self._lib.orc_hartree_energy(self._h, _ptr(rho))

    def comm_r(self, psi, axis, k=0, t=0.0):
        """[H(t), r_axis] psi for the states in psi at k-point k (R12)."""
        psi = np.ascontiguousarray(psi, dtype=np.complex128).reshape(
            -1, self.N)
        out = np.empty_like(psi)
        self._lib.orc_comm_r(self._h, int(k), float(t), int(axis),
                             psi.shape[0], _ptr(psi), _ptr(out))
        return out

    def current(self, psi, t=0.0, complex_values=False):
        """Macroscopic current J(t) (3 values; R12)."""
        psi = self._c128(psi, self.nk * self.ns)
        Jc = np.zeros(3, dtype=np.complex128)
        self._lib.orc_current(self._h, _ptr(psi), float(t), _ptr(Jc))
        return Jc if complex_values else Jc.real

    def dipole(self, rho):
        rho = _f64(rho)
        d = np.zeros(3)
        self._lib.orc_dipole(self._h, _ptr(rho), _ptr(d))
        return d

    def kick(self, psi, kappa):
        psi = self._c128(psi, self.nk * self.ns).reshape(
            self.nk, self.ns, self.N).copy()
        self._lib.orc_kick(self._h, _ptr(psi), float(kappa))
        return psi

    def norms(self, psi):
        psi = self._c128(psi, self.nk * self.ns)
        out = np.empty(self.nk * self.ns)
        self._lib.orc_norms(self._h, _ptr(psi), _ptr(out))
        return out

    def gram(self, psi):
        psi = self._c128(psi, self.nk * self.ns)
        out = np.empty((self.nk, self.ns, self.ns), dtype=np.complex128)
        self._lib.orc_gram(self._h, _ptr(psi), _ptr(out))
        return out

    def energy(self, psi, vion, t=0.0):
        psi = self._c128(psi, self.nk * self.ns)
        vion = _f64(vion)
        return self._lib.orc_energy(self._h, _ptr(psi), _ptr(vion), float(t))

    def propagate_etrs(self, psi, vion, nsteps, dt, t0=0.0):
        """Returns (psi(t0 + nsteps dt), dipole[(nsteps+1),3], norms)."""
        psi = self._c128(psi, self.nk * self.ns).reshape(
            self.nk, self.ns, self.N).copy()
        vion = _f64(vion)
        dip = np.zeros((nsteps + 1, 3))
        nrm = np.zeros((nsteps + 1, self.nk * self.ns))
        rc = self._lib.orc_propagate_etrs(self._h, _ptr(psi), _ptr(vion),
                                          int(nsteps), float(dt), float(t0),
                                          _ptr(dip), _ptr(nrm))
        if rc != 0:
            raise RuntimeError("oracle propagation failed")
        return psi, dip, nrm

    def propagate_cfm4(self, psi, vion, nsteps, dt, t0=0.0):
        """CFM4 (two Taylor-4 exponentials of Magnus-combined
        Hamiltonians per step).  Returns (psi, dipole, norms) as
        propagate_etrs."""
        psi = self._c128(psi, self.nk * self.ns).reshape(
            self.nk, self.ns, self.N).copy()
        vion = _f64(vion)
        dip = np.zeros((nsteps + 1, 3))
        nrm = np.zeros((nsteps + 1, self.nk * self.ns))
        rc = self._lib.orc_propagate_cfm4(self._h, _ptr(psi), _ptr(vion),
                                          int(nsteps), float(dt), float(t0),
                                          _ptr(dip), _ptr(nrm))
        if rc != 0:
            raise RuntimeError("oracle propagation failed")
        return psi, dip, nrm


def coulomb_cell_mean(h) -> float:
    """Mean of 1/|r| over the grid cell of sides h centred at the origin
    (the G(0) of reading R11)."""
    hh = _f64(h)
    return float(_load().orc_coulomb_cell_mean(_ptr(hh)))


def strength_function(d, dt, kappa, gamma, omega):
    """S(w) of a kicked run from the dipole component along the kick (R13)."""
    lib = _load()
    d = _f64(d)
    omega = _f64(omega)
    out = np.empty(len(omega))
    lib.orc_strength_function(_ptr(d), len(d), float(dt), float(kappa),
                              float(gamma), _ptr(omega), len(omega),
                              _ptr(out))
    return out


def conductivity(J, dt, E0, gamma, omega):
    """sigma(w) from a current component after an impulsive field (R13)."""
    lib = _load()
    J = _f64(J)
    omega = _f64(omega)
    out = np.empty(len(omega), dtype=np.complex128)
    lib.orc_conductivity(_ptr(J), len(J), float(dt), float(E0),
                         float(gamma), _ptr(omega), len(omega), _ptr(out))
    return out


def num_threads() -> int:
    return int(_load().orc_num_threads())
