"""Python binding of libks (the C ABI declared in include/ks.h).

Argument marshalling only: every step of the path runs in libks's HIP kernels.
PyTorch supplies device memory (tensors) and the stream.  The functions carry
the C names (ks_grid_create, ks_apply_h, ...); ``Grid`` bundles them with a
workspace tensor.  Importing this module does not load the library; the
first call does, and raises if libks.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libks.so")

KS_FP64, KS_MIXED = 0, 1
_STATUS = {0: "KS_OK", -1: "KS_E_ARG", -2: "KS_E_OOM", -3: "KS_E_HIP",
           -4: "KS_E_UNSUPPORTED", -5: "KS_E_STATE", -6: "KS_E_NONFINITE"}


class KSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class ks_grid_desc(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3),
        ("h", C.c_double * 3),
        ("periodic", C.c_int * 3),
        ("fd_half_width", C.c_int),
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
        ("precision", C.c_int),
        ("stream", C.c_void_p),
        ("hartree", C.c_int),
    ]


class ks_job(C.Structure):
    _fields_ = [
        ("grid", C.c_void_p),
        ("d_psi", C.c_void_p),
        ("d_vion", C.c_void_p),
        ("dt", C.c_double),
        ("t0", C.c_double),
        ("d_dipole", C.c_void_p),
        ("d_norms", C.c_void_p),
        ("max_steps", C.c_int),
        ("first_step", C.c_int),
    ]


EXPORTS = {
    # name: (restype, argtypes)
    "ks_grid_create": (C.c_int, [C.POINTER(ks_grid_desc),
                                 C.POINTER(C.c_void_p)]),
    "ks_grid_destroy": (C.c_int, [C.c_void_p]),
    "ks_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ks_workspace_bytes": (C.c_size_t, [C.c_void_p]),
    "ks_set_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ks_update_vlocal": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ks_hartree": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ks_apply_h": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                             C.c_int, C.c_int, C.c_double]),
    "ks_apply_h_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_int, C.c_int, C.c_int, C.c_double]),
    "ks_propagate_etrs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_int, C.c_double, C.c_double,
                                    C.c_void_p, C.c_void_p]),
    "ks_propagate_cfm4": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_int, C.c_double, C.c_double,
                                    C.c_void_p, C.c_void_p]),
    "ks_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ks_current": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double,
                             C.POINTER(C.c_double)]),
    "ks_strength_function": (C.c_int, [C.c_void_p, C.c_int, C.c_int,
                                       C.c_double, C.c_double, C.c_double,
                                       C.c_void_p, C.c_int, C.c_void_p,
                                       C.c_void_p]),
    "ks_conductivity": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double,
                                  C.c_double, C.c_double, C.c_void_p,
                                  C.c_int, C.c_void_p, C.c_void_p]),
    "ks_dipole": (C.c_int, [C.c_void_p, C.c_void_p,
                            C.POINTER(C.c_double)]),
    "ks_kick": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double]),
    "ks_norms": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ks_gram": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ks_energy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                            C.POINTER(C.c_double)]),
    "ks_set_launch": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "ks_get_launch": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "ks_set_overlap": (C.c_int, [C.c_void_p, C.c_int]),
    "ks_profile_begin": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "ks_profile_end": (C.c_int, [C.c_void_p, C.POINTER(C.c_double),
                                 C.POINTER(C.c_long)]),
    "ks_profile_every": (C.c_int, [C.c_void_p, C.c_int]),
    "ks_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int,
                              C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "ks_batch_create": (C.c_int, [C.POINTER(ks_job), C.c_int, C.c_void_p,
                                  C.POINTER(C.c_void_p)]),
    "ks_batch_step": (C.c_int, [C.c_void_p, C.c_int]),
    "ks_batch_set_graph": (C.c_int, [C.c_void_p, C.c_int]),
    "ks_batch_steps_done": (C.c_int, [C.c_void_p, C.c_int,
                                      C.POINTER(C.c_int)]),
    "ks_batch_destroy": (C.c_int, [C.c_void_p]),
    "ks_check_finite": (C.c_int, [C.c_void_p, C.c_long]),
    "ks_grid_device_bytes": (C.c_int, [C.c_void_p,
                                       C.POINTER(C.c_size_t)]),
    "ks_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libks (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise KSError(rc, lib().ks_last_error().decode())
    return rc


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, numel=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# C-named functions
# ---------------------------------------------------------------------------
def ks_grid_create(spec, precision=KS_FP64, stream=None):
    """Returns (handle, keep-alive host arrays)."""
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    keep = dict(kpts=f64(spec.kpts).reshape(-1), kw=f64(spec.kw),
                occ=f64(spec.occ), pos=f64(spec.pos).reshape(-1),
                lmax=np.ascontiguousarray(spec.lmax, dtype=np.int32),
                rc=f64(spec.rc), sigma=f64(spec.sigma),
                E=f64(spec.E).reshape(-1))
    P = lambda a, t=C.c_double: a.ctypes.data_as(C.POINTER(t))
    d = ks_grid_desc()
    d.n[:] = list(spec.n)
    d.h[:] = list(spec.h)
    d.periodic[:] = list(spec.periodic)
    d.fd_half_width = 4
    d.nk = len(keep["kw"])
    d.kpts = P(keep["kpts"])
    d.kw = P(keep["kw"])
    d.nstates = int(spec.nstates)
    d.occ = P(keep["occ"])
    d.natoms = int(len(keep["rc"]))
    d.pos = P(keep["pos"])
    d.lmax = P(keep["lmax"], C.c_int)
    d.rc = P(keep["rc"])
    d.sigma = P(keep["sigma"])
    d.E = P(keep["E"])
    d.xc = int(spec.xc)
    d.laser[:] = list(spec.laser)
    d.precision = int(precision)
    d.stream = _stream_handle(stream)
    d.hartree = int(getattr(spec, "hartree", 0))
    h = C.c_void_p()
    _check(lib().ks_grid_create(C.byref(d), C.byref(h)))
    return h, keep


def ks_grid_destroy(h):
    return _check(lib().ks_grid_destroy(h))


def ks_set_stream(h, stream):
    return _check(lib().ks_set_stream(h, _stream_handle(stream)))


def ks_workspace_bytes(h):
    return int(lib().ks_workspace_bytes(h))


def ks_grid_device_bytes(h):
    out = C.c_size_t(0)
    _check(lib().ks_grid_device_bytes(h, C.byref(out)))
    return int(out.value)


def ks_set_workspace(h, ws):
    return _check(lib().ks_set_workspace(h, _ptr(ws), ws.numel()))


def ks_update_vlocal(h, vion, rho=None):
    return _check(lib().ks_update_vlocal(h, _ptr(vion), _ptr(rho)))


def ks_hartree(h, rho, vh):
    return _check(lib().ks_hartree(h, _ptr(rho), _ptr(vh)))


def ks_apply_h(h, psi, hpsi, k, s0, ns, t):
    return _check(lib().ks_apply_h(h, _ptr(psi), _ptr(hpsi), k, s0, ns, t))


def ks_apply_h_noalloc(h, psi, hpsi, k, s0, ns, t):
    return _check(lib().ks_apply_h_noalloc(h, _ptr(psi), _ptr(hpsi), k, s0,
                                           ns, t))


def ks_propagate_etrs(h, psi, vion, nsteps, dt, t0, dipole, norms):
    return _check(lib().ks_propagate_etrs(h, _ptr(psi), _ptr(vion), nsteps,
                                          dt, t0, _ptr(dipole), _ptr(norms)))


def ks_propagate_cfm4(h, psi, vion, nsteps, dt, t0, dipole, norms):
    return _check(lib().ks_propagate_cfm4(h, _ptr(psi), _ptr(vion), nsteps,
                                          dt, t0, _ptr(dipole), _ptr(norms)))


def ks_current(h, psi, t):
    out = (C.c_double * 3)()
    _check(lib().ks_current(h, _ptr(psi), float(t), out))
    return np.array(out[:])


def ks_strength_function(trace, nt, stride, dt, kappa, gamma, omega, out,
                         stream=None):
    return _check(lib().ks_strength_function(
        _ptr(trace), int(nt), int(stride), float(dt), float(kappa),
        float(gamma), _ptr(omega), int(omega.numel()), _ptr(out),
        _stream_handle(stream)))


def ks_conductivity(trace, nt, stride, dt, E0, gamma, omega, out,
                    stream=None):
    return _check(lib().ks_conductivity(
        _ptr(trace), int(nt), int(stride), float(dt), float(E0),
        float(gamma), _ptr(omega), int(omega.numel()), _ptr(out),
        _stream_handle(stream)))


def _trace_view(trace, component):
    """(tensor, samples, stride) for a 1-D trace or one column of an
    (nt, k) trace (the column view's data pointer is offset to it)."""
    import torch
    if not (isinstance(trace, torch.Tensor) and trace.is_cuda and
            trace.dtype == torch.float64):
        raise TypeError("trace must be a float64 tensor on the GPU")
    if trace.dim() == 1:
        return trace, trace.numel(), 1
    if trace.dim() == 2 and trace.is_contiguous():
        return trace[:, component], trace.shape[0], trace.shape[1]
    raise ValueError("trace must be 1-D or a contiguous (nt, k) array")


def strength_function(trace, dt, kappa, gamma, omega, component=2):
    """S(w) of a kicked run from a device dipole trace ((nt, 3) as
    propagate_etrs returns it, or 1-D); omega: device float64 tensor."""
    import torch
    _dev(omega, torch.float64, None, "omega")
    col, nt, stride = _trace_view(trace, component)
    out = torch.empty_like(omega)
    ks_strength_function(col, nt, stride, dt, kappa, gamma, omega, out)
    return out


def conductivity(trace, dt, E0, gamma, omega, component=0):
    """sigma(w) (complex128 device tensor) from a device current trace."""
    import torch
    _dev(omega, torch.float64, None, "omega")
    col, nt, stride = _trace_view(trace, component)
    out = torch.empty(omega.numel(), dtype=torch.complex128,
                      device=omega.device)
    ks_conductivity(col, nt, stride, dt, E0, gamma, omega, out)
    return out


def ks_density(h, psi, rho):
    return _check(lib().ks_density(h, _ptr(psi), _ptr(rho)))


def ks_dipole(h, rho):
    out = (C.c_double * 3)()
    _check(lib().ks_dipole(h, _ptr(rho), out))
    return np.array(out[:])


def ks_kick(h, psi, kappa):
    return _check(lib().ks_kick(h, _ptr(psi), kappa))


def ks_norms(h, psi, norms):
    return _check(lib().ks_norms(h, _ptr(psi), _ptr(norms)))


def ks_gram(h, psi, gram):
    return _check(lib().ks_gram(h, _ptr(psi), _ptr(gram)))


def ks_energy(h, psi, vion, t):
    out = C.c_double()
    _check(lib().ks_energy(h, _ptr(psi), _ptr(vion), t, C.byref(out)))
    return out.value


def ks_set_launch(h, tile_rows, zchunk, rows_per_thread=0):
    return _check(lib().ks_set_launch(h, int(tile_rows), int(zchunk),
                                      int(rows_per_thread)))


def ks_set_overlap(h, halves):
    return _check(lib().ks_set_overlap(h, int(halves)))


def ks_get_launch(h):
    out = (C.c_int * 5)()
    _check(lib().ks_get_launch(h, out))
    return dict(tile_rows=out[0], zchunk=out[1], workgroups=out[2],
                threads=out[3], rows_per_thread=out[4])


PROFILE_CLASSES = ("hpsi", "gather", "reduce", "kbapply")


def ks_profile_begin(h, capacity, classes=PROFILE_CLASSES):
    mask = 0
    for c in classes:
        mask |= 1 << PROFILE_CLASSES.index(c)
    return _check(lib().ks_profile_begin(h, int(capacity), mask))


def ks_profile_every(h, every):
    return _check(lib().ks_profile_every(h, int(every)))


def ks_profile_end(h):
    """{class: (total_ms, launches)} for classes hpsi, gather, reduce,
    kbapply."""
    ms = (C.c_double * 4)()
    cnt = (C.c_long * 4)()
    _check(lib().ks_profile_end(h, ms, cnt))
    return {name: (ms[i], cnt[i]) for i, name in
            enumerate(("hpsi", "gather", "reduce", "kbapply"))}


def ks_autotune(h, psi, reps=3):
    """Returns (tile_rows, zchunk, rows_per_thread, microseconds per H.psi
    pass)."""
    shape = (C.c_int * 3)()
    us = C.c_double()
    _check(lib().ks_autotune(h, _ptr(psi), int(reps), shape, C.byref(us)))
    return shape[0], shape[1], shape[2], us.value


def ks_batch_create(jobs, stream):
    """jobs: sequence of ks_job.  Returns the batch handle."""
    arr = (ks_job * len(jobs))(*jobs)
    h = C.c_void_p()
    _check(lib().ks_batch_create(arr, len(jobs), _stream_handle(stream),
                                 C.byref(h)))
    return h


def ks_batch_step(b, nsteps):
    return _check(lib().ks_batch_step(b, int(nsteps)))


def ks_batch_set_graph(b, use_graph):
    return _check(lib().ks_batch_set_graph(b, int(bool(use_graph))))


def ks_batch_steps_done(b, job):
    out = C.c_int()
    _check(lib().ks_batch_steps_done(b, int(job), C.byref(out)))
    return out.value


def ks_batch_destroy(b):
    return _check(lib().ks_batch_destroy(b))


def ks_check_finite(values):
    """Raise KSError (KS_E_NONFINITE) if a value of the host float64 array
    is NaN or Inf."""
    a = np.ascontiguousarray(values, dtype=np.float64)
    return _check(lib().ks_check_finite(a.ctypes.data_as(C.c_void_p),
                                        a.size))


# ---------------------------------------------------------------------------
# convenience objects
# ---------------------------------------------------------------------------
class Grid:
    """A libks grid object plus its workspace tensor."""

    def __init__(self, spec, precision=KS_FP64, stream=None, device=None,
                 workspace=True):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        self.spec = spec
        self.N = spec.n[0] * spec.n[1] * spec.n[2]
        self.nk = len(spec.kw)
        self.ns = int(spec.nstates)
        self.precision = precision
        self.ws = None
        self.h, self._keep = ks_grid_create(spec, precision, stream)
        if workspace:
            self._alloc_ws()

    def ensure_workspace(self):
        """Lend the workspace now (a Grid made with workspace=False)."""
        if self.ws is None:
            self._alloc_ws()

    def _alloc_ws(self):
        torch = self.torch
        nbytes = ks_workspace_bytes(self.h)
        self.ws = None
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8,
                              device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self._ws_view = self.ws[off:off + nbytes]
        ks_set_workspace(self.h, self._ws_view)

    def close(self):
        if getattr(self, "h", None) is not None:
            ks_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self):
        return ks_workspace_bytes(self.h)

    @property
    def device_bytes(self):
        """Device memory the grid holds itself (tables, potential, Hartree
        plan; not the workspace)."""
        return ks_grid_device_bytes(self.h)

    def set_stream(self, stream):
        ks_set_stream(self.h, stream)

    def _psi(self, psi, nstates=None):
        nst = self.nk * self.ns if nstates is None else nstates
        return _dev(psi, self.torch.complex128, nst * self.N, "psi")

    def update_vlocal(self, vion, rho=None):
        _dev(vion, self.torch.float64, self.N, "vion")
        if rho is not None:
            _dev(rho, self.torch.float64, self.N, "rho")
        ks_update_vlocal(self.h, vion, rho)

    def current(self, psi, t=0.0):
        """Macroscopic current J(t) of the states (3 values, host)."""
        self._psi(psi)
        return ks_current(self.h, psi, float(t))

    def current_trace(self, psi, vion, nsteps, dt, t0=0.0,
                      method="etrs"):
        """Propagate psi in place by nsteps steps, recording J(t_n) before
        the first and after every step: an (nsteps+1, 3) host array."""
        prop = getattr(self, "propagate_" + method)
        out = np.zeros((nsteps + 1, 3))
        out[0] = self.current(psi, t0)
        for n in range(nsteps):
            prop(psi, vion, 1, dt, t0 + n * dt, dipole=False, norms=False)
            out[n + 1] = self.current(psi, t0 + (n + 1) * dt)
        return out

    def hartree(self, rho, out=None):
        """Hartree potential v_H[rho] (FP64, N values on the device)."""
        _dev(rho, self.torch.float64, self.N, "rho")
        if out is None:
            out = self.torch.empty_like(rho)
        _dev(out, self.torch.float64, self.N, "vh")
        ks_hartree(self.h, rho, out)
        return out

    def apply_h(self, psi, out=None, k=0, s0=0, t=0.0):
        _dev(psi, self.torch.complex128, None, "psi")
        ns = psi.numel() // self.N
        if ns * self.N != psi.numel():
            raise ValueError("psi is not a whole number of states")
        if out is None:
            out = self.torch.empty_like(psi)
        _dev(out, self.torch.complex128, psi.numel(), "hpsi")
        ks_apply_h(self.h, psi, out, int(k), int(s0), ns, float(t))
        return out

    def propagate_etrs(self, psi, vion, nsteps, dt, t0=0.0, dipole=True,
                       norms=True):
        self._psi(psi)
        _dev(vion, self.torch.float64, self.N, "vion")
        d = (self.torch.zeros((nsteps + 1, 3), dtype=self.torch.float64,
                              device=self.device) if dipole else None)
        n = (self.torch.zeros((nsteps + 1, self.nk * self.ns),
                              dtype=self.torch.float64, device=self.device)
             if norms else None)
        ks_propagate_etrs(self.h, psi, vion, int(nsteps), float(dt),
                          float(t0), d, n)
        return d, n

    def propagate_cfm4(self, psi, vion, nsteps, dt, t0=0.0, dipole=True,
                       norms=True):
        self._psi(psi)
        _dev(vion, self.torch.float64, self.N, "vion")
        d = (self.torch.zeros((nsteps + 1, 3), dtype=self.torch.float64,
                              device=self.device) if dipole else None)
        n = (self.torch.zeros((nsteps + 1, self.nk * self.ns),
                              dtype=self.torch.float64, device=self.device)
             if norms else None)
        ks_propagate_cfm4(self.h, psi, vion, int(nsteps), float(dt),
                          float(t0), d, n)
        return d, n

    def density(self, psi, rho=None):
        self._psi(psi)
        if rho is None:
            rho = self.torch.empty(self.N, dtype=self.torch.float64,
                                   device=self.device)
        ks_density(self.h, psi, rho)
        return rho

    def dipole(self, rho):
        _dev(rho, self.torch.float64, self.N, "rho")
        return ks_dipole(self.h, rho)

    def kick(self, psi, kappa):
        self._psi(psi)
        ks_kick(self.h, psi, float(kappa))
        return psi

    def norms(self, psi):
        self._psi(psi)
        out = self.torch.empty(self.nk * self.ns, dtype=self.torch.float64,
                               device=self.device)
        ks_norms(self.h, psi, out)
        return out

    def gram(self, psi):
        self._psi(psi)
        out = self.torch.empty((self.nk, self.ns, self.ns),
                               dtype=self.torch.complex128,
                               device=self.device)
        ks_gram(self.h, psi, out)
        return out

    def set_launch(self, tile_rows=0, zchunk=0, rows_per_thread=0):
        try:
            ks_set_launch(self.h, tile_rows, zchunk, rows_per_thread)
        except KSError as e:
            if e.code == -2:       # workspace too small: lend a larger one
                self._alloc_ws()
            else:
                raise

    def get_launch(self):
        return ks_get_launch(self.h)

    def set_overlap(self, halves=2):
        """Propagate the states in two overlapped halves (2) or one chain
        (1)."""
        ks_set_overlap(self.h, halves)

    def autotune(self, psi, reps=3):
        """Pick the fastest launch shape on these states; returns
        (tile_rows, zchunk, rows_per_thread, us per pass)."""
        self._psi(psi)
        return ks_autotune(self.h, psi, reps)

    def profile_begin(self, capacity=100000, classes=PROFILE_CLASSES,
                      every=1):
        """Start event timing of the given kernel classes, one launch in
        `every` of each."""
        ks_profile_every(self.h, every)
        ks_profile_begin(self.h, capacity, classes)

    def profile_end(self):
        return ks_profile_end(self.h)

    def energy(self, psi, vion, t=0.0):
        self._psi(psi)
        _dev(vion, self.torch.float64, self.N, "vion")
        return ks_energy(self.h, psi, vion, float(t))


class Job:
    """One member of a Batch: a Grid, its states (propagated in place), the
    ionic potential and the time axis; dipole / norms traces are allocated
    here with room for max_steps steps."""

    def __init__(self, grid, psi, vion, dt, max_steps, t0=0.0, dipole=True,
                 norms=True):
        torch = grid.torch
        grid._psi(psi)
        _dev(vion, torch.float64, grid.N, "vion")
        self.grid, self.psi, self.vion = grid, psi, vion
        self.dt, self.t0, self.max_steps = float(dt), float(t0), int(max_steps)
        self.first_step = 0        # steps taken in earlier batches
        self.dipole = (torch.zeros((max_steps + 1, 3), dtype=torch.float64,
                                   device=grid.device) if dipole else None)
        self.norms = (torch.zeros((max_steps + 1, grid.nk * grid.ns),
                                  dtype=torch.float64, device=grid.device)
                      if norms else None)

    def c_struct(self):
        j = ks_job()
        j.grid = self.grid.h
        j.d_psi = self.psi.data_ptr()
        j.d_vion = self.vion.data_ptr()
        j.dt = self.dt
        j.t0 = self.t0
        j.d_dipole = self.dipole.data_ptr() if self.dipole is not None else None
        j.d_norms = self.norms.data_ptr() if self.norms is not None else None
        j.max_steps = self.max_steps
        j.first_step = self.first_step
        return j


class Batch:
    """Jobs propagated together by ks_batch_* on a stream of its own (a
    captured HIP graph needs a non-default stream).  Work is ordered after
    the caller's current stream on entry and before it on return."""

    def __init__(self, jobs, use_graph=True):
        import torch
        self.torch = torch
        self.jobs = list(jobs)
        self.stream = torch.cuda.Stream()
        self._cur = torch.cuda.current_stream()
        self.stream.wait_stream(self._cur)
        self.h = ks_batch_create([j.c_struct() for j in self.jobs],
                                 self.stream)
        if not use_graph:
            ks_batch_set_graph(self.h, 0)
        self._cur.wait_stream(self.stream)

    def step(self, nsteps=1):
        cur = self.torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        ks_batch_step(self.h, nsteps)
        cur.wait_stream(self.stream)

    def steps_done(self, job):
        return ks_batch_steps_done(self.h, job)

    def close(self):
        """Free the batch; each job's first_step becomes the steps it has
        taken, so it can join a later batch and continue."""
        if getattr(self, "h", None) is not None:
            for i, j in enumerate(self.jobs):
                j.first_step = ks_batch_steps_done(self.h, i)
            h, self.h = self.h, None
            for j in self.jobs:
                if j.grid.h is not None:
                    j.grid.set_stream(self._cur)
            ks_batch_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
