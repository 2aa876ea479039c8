"""The allocation-free H.psi entry point (ks_apply_h_noalloc, projector
scratch in a static device array) against ks_apply_h (scratch in the
caller's workspace), through the C ABI: two calls in a row, the second on a
smaller grid with fewer states, must give the same H.psi (the kernels are
shared, so the results agree bitwise; the bar asked of H.psi is 1e-12
relative).  A call whose states need more scratch than the static array
holds is refused before any launch."""
import numpy as np
import pytest

from paper_1912_07921_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def both(torch, spec, v, psi, t, precision=0):
    """(ks_apply_h, ks_apply_h_noalloc) of every k-point's states."""
    from paper_1912_07921_amd import ks
    g = ks.Grid(spec, precision=precision)
    g.update_vlocal(torch.from_numpy(v).cuda())
    outs = []
    for k in range(spec.nk):
        dpsi = torch.from_numpy(np.ascontiguousarray(psi[k])).cuda()
        want = torch.empty_like(dpsi)
        ks.ks_apply_h(g.h, dpsi, want, k, 0, spec.nstates, t)
        got = torch.full_like(dpsi, float("nan"))
        ks.ks_apply_h_noalloc(g.h, dpsi, got, k, 0, spec.nstates, t)
        torch.cuda.synchronize()
        outs.append((want.cpu().numpy(), got.cpu().numpy()))
    g.close()
    return outs


def check(outs):
    for want, got in outs:
        rel = np.linalg.norm(got - want, axis=1) / \
            np.linalg.norm(want, axis=1)
        assert rel.max() < 1e-12, rel.max()
        assert np.array_equal(got, want)


def test_noalloc_matches_apply_h_twice_second_smaller(torch_cuda):
    torch = torch_cuda
    # first call: periodic, two k-points, s+p+d projectors, a laser
    spec, v, psi = W.tiny(n=(20, 18, 16), h=(0.3, 0.3, 0.3),
                          periodic=(1, 1, 1), nk=2, nstates=4, natoms=3,
                          lmax=2, rc=1.2, sigma=0.4,
                          laser=(0.2, 0.7, 4.0, 0.0, 0.0, 1.0))
    check(both(torch, spec, v, psi, 1.0))
    # second call, smaller: a finite grid, one k-point, two states, s+p
    spec, v, psi = W.tiny(n=(12, 10, 9), h=(0.35, 0.3, 0.3), nstates=2,
                          natoms=2, lmax=1, rc=1.0, sigma=0.3, seed=9)
    check(both(torch, spec, v, psi, 0.0))


def test_noalloc_matches_apply_h_mixed_many_states(torch_cuda):
    """A grid in the mixed form (FP32 kernels, the potential's FP32 copy
    in the scratch too) with 136 states (the projector apply's wide state
    groups), then a smaller one: the same bitwise agreement."""
    torch = torch_cuda
    spec, v, psi = W.tiny(n=(14, 13, 12), h=(0.35, 0.35, 0.35),
                          periodic=(1, 1, 1), nk=1, nstates=136, natoms=3,
                          lmax=2, rc=1.3, sigma=0.4)
    check(both(torch, spec, v, psi, 0.0, precision=1))
    spec, v, psi = W.tiny(n=(10, 9, 8), nstates=3, natoms=2, lmax=1,
                          rc=1.0, sigma=0.3, seed=11)
    check(both(torch, spec, v, psi, 0.0, precision=1))


def test_noalloc_refuses_states_beyond_its_scratch(torch_cuda):
    from paper_1912_07921_amd import ks
    torch = torch_cuda
    # 48^3 with six large spheres: 29,824 projector-row points, so 256
    # states need about 120 MiB of scratch, more than the 64 MiB array
    spec, v, _ = W.tiny(n=(48, 48, 48), h=(0.2, 0.2, 0.2), nstates=256,
                        natoms=6, lmax=2, rc=2.4, sigma=0.6, seed=3)
    g = ks.Grid(spec, workspace=False)
    g.update_vlocal(torch.from_numpy(v).cuda())
    psi = torch.zeros((256, spec.npoints), dtype=torch.complex128,
                      device="cuda")
    out = torch.empty_like(psi)
    with pytest.raises(ks.KSError) as e:
        ks.ks_apply_h_noalloc(g.h, psi, out, 0, 0, 256, 0.0)
    assert e.value.code == -1 and "scratch" in str(e.value)
    # a few states fit, and need no workspace
    ks.ks_apply_h_noalloc(g.h, psi[:4], out[:4], 0, 0, 4, 0.0)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out[:4]).item() == 0
    g.close()
