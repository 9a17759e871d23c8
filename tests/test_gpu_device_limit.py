"""Device-memory cap (fd_set_device_limit): setups past it fail with FD_E_NOMEM and hold nothing.

The cap stands in for an exhausted device, so the FD_E_NOMEM paths of
fd_setup and fd_batch_create run without filling the GPU.
"""
import gc

import numpy as np
import pytest
import torch

from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
from oracle.fd import FDFactors, block_apply, velocity_weights
from paper_1712_00403_amd import fd, workloads
from paper_1712_00403_amd.precond import BlockPreconditioner

pytestmark = pytest.mark.gpu

NOMEM = 3


@pytest.fixture
def capped():
    # plans that earlier tests left to the garbage collector are freed now, so
    # that none is released (and the held bytes change) in the middle of a test
    gc.collect()
    yield
    fd.set_device_limit(0)


def _oracle_block_apply(prob, r):
    vel = [taylor_hood_velocity_1d(n, prob.p) for n in prob.n_el]
    facs = [FDFactors([v[0] for v in vel], [v[1] for v in vel], velocity_weights(3, k)) for k in range(3)]
    Mp = [pressure_1d(n, prob.p) for n in prob.n_el]
    return np.stack([block_apply(facs, Mp, r[j]) for j in range(r.shape[0])])


def test_setup_past_the_cap_is_nomem_and_holds_nothing(capped):
    torch.cuda.set_device(0)
    prob = workloads.taylor_hood_problem((6, 5, 7), 2)
    held0 = fd.device_bytes_held()
    pc = BlockPreconditioner(prob, precision="f64")
    need = [p.device_bytes for p in pc.plans]
    assert fd.device_bytes_held() == held0 + sum(need)
    pc.close()
    assert fd.device_bytes_held() == held0
    # room for the first block's plan only: the second block fails, the first is released
    for cap in (held0 + 1024, held0 + need[0]):
        fd.set_device_limit(cap)
        with pytest.raises(fd.FDError) as ei:
            BlockPreconditioner(prob, precision="f64")
        assert ei.value.status == NOMEM and "device allocation" in str(ei.value)
        assert fd.device_bytes_held() == held0
    # exactly enough: the preconditioner is built under the cap and applies correctly
    fd.set_device_limit(held0 + sum(need))
    pc = BlockPreconditioner(prob, precision="f64")
    assert fd.device_bytes_held() == held0 + sum(need)
    r = workloads.residuals(0, 2, pc.N)
    z = pc.apply(torch.from_numpy(r).cuda()).cpu().numpy()
    zo = _oracle_block_apply(prob, r)
    assert np.abs(z - zo).max() <= 1e-12 * np.abs(zo).max()
    pc.close()
    fd.set_device_limit(0)
    assert fd.device_bytes_held() == held0


def test_batch_create_past_the_cap_is_nomem(capped):
    torch.cuda.set_device(0)
    prob = workloads.taylor_hood_problem((6, 5, 7), 2)
    pc = BlockPreconditioner(prob, precision="f32")
    r = torch.zeros(1, pc.N, dtype=torch.float32, device="cuda")
    z = torch.zeros_like(r)
    works = pc.works(r.data_ptr(), z.data_ptr(), 1)
    held = fd.device_bytes_held()
    fd.set_device_limit(held + 64)  # below the batch's tables
    with pytest.raises(fd.FDError) as ei:
        fd.Batch(works)
    assert ei.value.status == NOMEM
    assert fd.device_bytes_held() == held
    fd.set_device_limit(0)
    b = fd.Batch(works)
    assert fd.device_bytes_held() > held
    b.close()
    assert fd.device_bytes_held() == held
    pc.close()
