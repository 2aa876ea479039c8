"""Failure detection on the GPU: a NaN in the states makes the
propagators return KS_E_NONFINITE (the end-of-call norm check), with and
without a norm trace, and makes a batch report the job whose norm is not
finite.  NaN values only flow through the arithmetic (no address depends on
a state value), so every kernel runs and exits as usual."""
import numpy as np
import pytest

from paper_1912_07921_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def system():
    spec, v, psi = W.tiny(n=(12, 11, 10), h=(0.3, 0.3, 0.3), nstates=3,
                          natoms=2, lmax=1, rc=1.0, sigma=0.3, xc=1)
    return spec, v, psi


@pytest.mark.parametrize("method", ["etrs", "cfm4"])
@pytest.mark.parametrize("norms", [True, False])
def test_propagator_reports_nan_state(torch_cuda, method, norms):
    from paper_1912_07921_amd import ks
    torch = torch_cuda
    spec, v, psi = system()
    g = ks.Grid(spec)
    vion = torch.from_numpy(v).cuda()
    good = torch.from_numpy(psi.copy()).cuda()
    prop = getattr(g, "propagate_" + method)
    prop(good, vion, 2, 0.01, dipole=True, norms=norms)   # finite: no error
    bad = psi.copy()
    bad[0, 1, 57] = np.nan
    dbad = torch.from_numpy(bad).cuda()
    with pytest.raises(ks.KSError) as e:
        prop(dbad, vion, 2, 0.01, dipole=True, norms=norms)
    assert e.value.code == -6
    assert "NaN" in str(e.value) or "infinite" in str(e.value)
    g.close()


def test_batch_reports_the_job_with_a_nan_norm(torch_cuda):
    from paper_1912_07921_amd import ks
    torch = torch_cuda
    spec, v, psi = system()
    bad = psi.copy()
    bad[0, 2, 11] = np.inf
    jobs = []
    for p in (psi, bad):
        g = ks.Grid(spec)
        jobs.append(ks.Job(g, torch.from_numpy(p.copy()).cuda(),
                           torch.from_numpy(v).cuda(), 0.01, 4))
    b = ks.Batch(jobs)
    b.step(1)
    torch.cuda.synchronize()
    with pytest.raises(ks.KSError) as e:
        b.step(1)
    assert e.value.code == -6 and "job 1" in str(e.value)
    b.close()
    # a batch of finite jobs reports nothing, through destroy as well
    jobs = [ks.Job(ks.Grid(spec), torch.from_numpy(psi.copy()).cuda(),
                   torch.from_numpy(v).cuda(), 0.01, 4)]
    b = ks.Batch(jobs)
    b.step(3)
    b.close()
    # the error of a step that was never followed by another is reported
    # when the batch is freed
    jobs = [ks.Job(ks.Grid(spec), torch.from_numpy(bad.copy()).cuda(),
                   torch.from_numpy(v).cuda(), 0.01, 4)]
    b = ks.Batch(jobs)
    b.step(2)
    with pytest.raises(ks.KSError) as e:
        b.close()
    assert e.value.code == -6
