"""The allocation-free persistent apply (fd_apply_persistent_static) against fd_batch_apply.

Both run the same works with the same configuration word as one persistent
launch; the results must agree bit for bit, on two calls in a row (the
second with a smaller list), and match the oracle. The static tables are
shared per GPU, so the second call also checks that nothing of the first
call's tables or counters leaks into it.
"""
import numpy as np
import pytest

from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
from oracle.fd import FDFactors, block_apply, velocity_weights
from paper_1712_00403_amd import workloads
from parity_util import check_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"[gpu case] {msg}", flush=True)


BIG = [((5, 7, 4), 2), ((9, 4, 6), 3), ((12, 10), 2), ((30, 6, 5), 4), ((7, 6, 5), 5), ((48, 3, 4), 4)]
SMALL = [((4, 4, 4), 1), ((10, 7), 3)]


def _oracle(n_el, p, r):
    d = len(n_el)
    vel = [taylor_hood_velocity_1d(n, p) for n in n_el]
    facs = [FDFactors([v[0] for v in vel], [v[1] for v in vel], velocity_weights(d, k)) for k in range(d)]
    return block_apply(facs, [pressure_1d(n, p) for n in n_el], r)


def _setup(patches, prec, seed):
    from paper_1712_00403_amd.precond import BlockPreconditioner
    dt = torch.float64 if prec == "f64" else torch.float32
    pcs, rs, bufs, works = [], [], [], []
    for i, (n_el, p) in enumerate(patches):
        pc = BlockPreconditioner(workloads.taylor_hood_problem(n_el, p), precision=prec)
        r = workloads.residuals(seed + i, 2, pc.N)
        rt = torch.from_numpy(r).to(dt).cuda()
        za = torch.full_like(rt, float("nan"))
        zb = torch.full_like(rt, float("nan"))
        pcs.append(pc)
        rs.append(r)
        bufs.append((rt, za, zb))
        works.append(pc.works(rt.data_ptr(), za.data_ptr(), 2))
    return pcs, rs, bufs, works


@pytest.mark.parametrize("prec,config", [("f64", 0), ("f32", 0b1010101010), ("bf16", 0b0110011000)])
def test_static_apply_matches_batch_twice(prec, config):
    _case(f"allocation-free persistent apply vs fd_batch, prec={prec}, config={config}")
    from paper_1712_00403_amd import fd
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    for call, (patches, seed) in enumerate(((BIG, 100), (SMALL, 200))):
        pcs, rs, bufs, works = _setup(patches, prec, seed)
        ref_works = [w for ws in works for w in ws]
        b = fd.Batch(ref_works)
        b.set_config(config)
        b.apply()
        b.check()
        # the same works writing the second output buffers
        st_works = [(w[0], w[1], bufs[i][2].data_ptr() + (w[2] - bufs[i][1].data_ptr()), w[3], w[4])
                    for i, ws in enumerate(works) for w in ws]
        fd.apply_persistent_static(st_works, config, status.data_ptr())
        torch.cuda.synchronize()
        assert int(status.item()) == 0, "a grid barrier gave up"
        for (n_el, p), pc, r, (rt, za, zb) in zip(patches, pcs, rs, bufs):
            a = za.cpu().numpy()
            s = zb.cpu().numpy()
            assert np.array_equal(a, s), f"call {call} patch {n_el} p={p}: results differ from fd_batch_apply"
            for j in range(2):
                zo = _oracle(n_el, p, r[j])
                for k, (lo, hi) in enumerate(zip(pc.offsets[:-1], pc.offsets[1:])):
                    check_close(s[j, lo:hi].astype(np.float64), zo[lo:hi], prec, f"call {call} {n_el} block {k}")
        b.close()
        for pc in pcs:
            pc.close()


def test_static_apply_limits():
    _case("allocation-free persistent apply: argument checks and table limit")
    from paper_1712_00403_amd import fd
    from paper_1712_00403_amd.precond import BlockPreconditioner
    pc = BlockPreconditioner(workloads.taylor_hood_problem((3, 3, 3), 1), precision="f32")
    r = torch.zeros((1, pc.N), dtype=torch.float32, device="cuda")
    z = torch.zeros_like(r)
    works = pc.works(r.data_ptr(), z.data_ptr(), 1)
    for bad in (-1, 3, 1 << 10):
        with pytest.raises(fd.FDError, match="FD_E_ARG"):
            fd.apply_persistent_static(works, bad)
    # 2500 copies of the block vector's 4 works: 12,500 passes, beyond the static table
    with pytest.raises(fd.FDError, match="static table"):
        fd.apply_persistent_static(works * 2500, 0)
    # an empty list only clears the status word
    status = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    fd.apply_persistent_static([], 0, status.data_ptr())
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    # and a valid call still works after the refusals
    fd.apply_persistent_static(works, 0, status.data_ptr())
    torch.cuda.synchronize()
    assert int(status.item()) == 0 and torch.isfinite(z).all()
    pc.close()
