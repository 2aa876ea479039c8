"""CPU-side checks of the boundary: the library loads and exports every entry
point the public header declares; the binding knows them all; the oracle's
shared object builds and loads.  No compute call (no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_1912_07921_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ks.h")


def declared_entry_points():
    text = open(HEADER).read()
    return sorted(set(re.findall(
        r"^(?:int|size_t|const char \*)\s*(ks_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for must in ["ks_grid_create", "ks_apply_h", "ks_propagate_etrs",
                 "ks_density", "ks_update_vlocal", "ks_dipole"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1912_07921_amd import ks
    if not os.path.exists(ks.LIB_PATH):
        pytest.fail("libks.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(ks.LIB_PATH)
    for name in declared_entry_points():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1912_07921_amd import ks
    for name in declared_entry_points():
        assert name in ks.EXPORTS, name
        assert callable(getattr(ks, name, None)) or name == "ks_last_error"


def test_library_refuses_nothing_at_load_and_reports_errors_without_gpu():
    from paper_1912_07921_amd import ks
    L = ks.lib()
    assert L.ks_last_error() is not None
    # a NULL grid is an argument error, reported without touching the GPU
    assert L.ks_set_stream(None, None) == -1
    assert b"NULL" in L.ks_last_error()
    assert L.ks_workspace_bytes(None) == 0
    assert L.ks_grid_destroy(None) == 0


def test_grid_description_errors_need_no_gpu():
    """Invalid descriptions are refused before any device call: an unknown
    Hartree flag (argument error) and the Hartree term on a grid with mixed
    periodicity (unsupported)."""
    from types import SimpleNamespace
    from paper_1912_07921_amd import ks
    null_stream = SimpleNamespace(cuda_stream=0)
    spec = W.SystemSpec(n=(8, 8, 8), h=(0.4,) * 3, nstates=1, hartree=2)
    with pytest.raises(ks.KSError) as e:
        ks.ks_grid_create(spec, 0, null_stream)
    assert e.value.code == -1
    spec = W.SystemSpec(n=(8, 8, 8), h=(0.4,) * 3, periodic=(1, 0, 1),
                        nstates=1, hartree=1)
    with pytest.raises(ks.KSError) as e:
        ks.ks_grid_create(spec, 0, null_stream)
    assert e.value.code == -4
    assert b"Hartree" in ks.lib().ks_last_error()


def test_grid_size_limits_need_no_gpu():
    """Axis lengths the kernels cannot index are refused before any device
    call: nx above 512 (tile rows of at most 512 threads), 2^27 points or
    more (32-bit byte offsets of a state), and with atoms ny above 1024 or
    nz above 2048 (packed point coordinates)."""
    from types import SimpleNamespace
    from paper_1912_07921_amd import ks
    null_stream = SimpleNamespace(cuda_stream=0)
    atom = dict(pos=[[0.0, 0.0, 0.0]], Z=[1.0], lmax=[1], rc=[1.0],
                sigma=[0.5], E=[[1.0, -1.0, 0.0]])
    for n, kw, word in [((513, 4, 4), {}, b"nx"),
                        ((512, 512, 512), {}, b"2^27"),
                        ((8, 1025, 4), atom, b"ny"),
                        ((8, 4, 2049), atom, b"nz")]:
        spec = W.SystemSpec(n=n, h=(0.4,) * 3, nstates=1, **kw)
        with pytest.raises(ks.KSError) as e:
            ks.ks_grid_create(spec, 0, null_stream)
        assert e.value.code == -4, n
        assert word in ks.lib().ks_last_error(), n


def test_oracle_builds_and_loads(oracle_mod):
    lib = oracle_mod._load()
    for name in ["orc_create", "orc_apply_h", "orc_propagate_etrs",
                 "orc_density", "orc_dipole", "orc_vlocal", "orc_kick",
                 "orc_gram", "orc_energy", "orc_hartree", "orc_hartree_at",
                 "orc_hartree_energy"]:
        assert hasattr(lib, name)


def test_product_does_not_import_the_oracle():
    """The product package neither imports nor loads anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_1912_07921_amd")
    pat = re.compile(r"(^\s*(from|import)\s+oracle)|liboracle|ks_oracle",
                     re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not pat.search(text), f


def test_check_finite_reports_injected_nan_and_inf():
    """The host check the propagators apply to the norms they copy back:
    a NaN or an Inf among finite norms is KS_E_NONFINITE naming its index;
    finite values (zeros, huge and tiny norms included) pass."""
    import numpy as np
    from paper_1912_07921_amd import ks
    L = ks.lib()
    ok = np.array([1.0, 0.0, 1e300, 5e-324, -2.0])
    assert ks.ks_check_finite(ok) == 0
    assert ks.ks_check_finite(np.zeros(0)) == 0
    for bad, what in ((np.nan, b"NaN"), (np.inf, b"infinite"),
                      (-np.inf, b"infinite")):
        v = np.ones(7)
        v[4] = bad
        with pytest.raises(ks.KSError) as e:
            ks.ks_check_finite(v)
        assert e.value.code == -6
        msg = L.ks_last_error()
        assert b"value 4" in msg and what in msg
    # the first bad index is named
    v = np.array([1.0, np.inf, np.nan])
    with pytest.raises(ks.KSError):
        ks.ks_check_finite(v)
    assert b"value 1" in L.ks_last_error()
    assert L.ks_check_finite(None, 3) == -1
