"""GPU parity of the persistent batched apply (one launch for many heterogeneous patches)."""
import numpy as np
import pytest

from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
from oracle.fd import FDFactors, block_apply, velocity_weights
from paper_1712_00403_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2, "bf16_split": 1e-4, "f16": 5e-3, "f16_split": 1e-4}

# (n_el, p, geometry or None): 3D and 2D, every pressure degree 1..5, simple and
# coefficient-aware blocks, factor orders from 3 to 100
PATCHES = [((5, 7, 4), 2, None), ((9, 4, 6), 3, "sine"), ((3, 5, 8), 4, None), ((12, 10), 2, "warped"),
           ((7, 6, 5), 5, "sine"), ((4, 4, 4), 1, None), ((48, 3, 4), 4, None), ((30, 20), 3, "sine")]


def _case(msg):
    print(f"[gpu case] {msg}", flush=True)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _geometry(name, ndim):
    if name == "sine":
        return workloads.sine_geometry(ndim)
    return workloads.warped_geometry(ndim, nu=workloads.wavy_viscosity)


_REFS = []
_SETUP = {}


def _oracle_refs():
    """Oracle factors of every patch (computed once for all tests of this module)."""
    if not _REFS:
        from oracle.geometry import GeometryBlocks
        for n_el, p, geo in PATCHES:
            d = len(n_el)
            if geo is None:
                vel = [taylor_hood_velocity_1d(n, p) for n in n_el]
                facs = [FDFactors([v[0] for v in vel], [v[1] for v in vel], velocity_weights(d, k))
                        for k in range(d)]
                _REFS.append((facs, [pressure_1d(n, p) for n in n_el], None, None))
            else:
                gb = GeometryBlocks(n_el, p, _geometry(geo, d))
                _REFS.append(([FDFactors(gb.vel_K[k], gb.vel_M[k]) for k in range(d)], gb.pres_M, gb.pres_scale,
                              gb.vel_scales))
    return _REFS


def _build(prec):
    from paper_1712_00403_amd.geometry import GeometryPreconditioner, geometry_blocks
    from paper_1712_00403_amd.precond import BlockPreconditioner
    pcs = []
    for i, (n_el, p, geo) in enumerate(PATCHES):
        if geo is None:
            pcs.append(BlockPreconditioner(workloads.taylor_hood_problem(n_el, p), precision=prec))
        else:
            prob = workloads.taylor_hood_problem(n_el, p, unit_weights=True)
            g = _geometry(geo, len(n_el))
            if i not in _SETUP:  # the library's host setup of the coefficient-aware blocks
                _SETUP[i] = geometry_blocks(prob, g)
            pcs.append(GeometryPreconditioner(prob, g, precision=prec, blocks=_SETUP[i]))
    return pcs, _oracle_refs()


ALL_NARROW = 0b0101010101
ALL_PIPELINED = 0b1010101010
MIXED = 0b0110011000  # stages 0..4: wide, pipelined, narrow, pipelined, narrow


@pytest.mark.parametrize("prec,config", [("f64", 0), ("f32", 0), ("bf16", 0), ("f16", 0), ("bf16_split", 0),
                                         ("f32", ALL_NARROW), ("bf16", ALL_NARROW), ("f64", MIXED),
                                         ("f64", ALL_PIPELINED), ("f32", ALL_PIPELINED), ("bf16", ALL_PIPELINED),
                                         ("f16", ALL_PIPELINED), ("bf16_split", ALL_PIPELINED), ("f32", MIXED)])
def test_persistent_batch_matches_oracle(prec, config):
    _case(f"persistent batch of {len(PATCHES)} heterogeneous patches, prec={prec}, config={config}")
    from paper_1712_00403_amd import fd
    pcs, refs = _build(prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    nrhs = 2
    rs, zs, works = [], [], []
    for i, pc in enumerate(pcs):
        r = workloads.residuals(60 + i, nrhs, pc.N)
        rt = torch.from_numpy(r).to(dt).cuda()
        zt = torch.full_like(rt, float("nan"))
        rs.append(r)
        zs.append((rt, zt))
        works += pc.works(rt.data_ptr(), zt.data_ptr(), nrhs)
    batch = fd.Batch(works)
    if config:
        batch.set_config(config)  # stage s: bits 2s, 2s + 1 (0 wide, 1 narrow, 2 pipelined)
    info = batch.info()
    print(f"  tiles {info['tiles']}, grid {info['grid']}, config {info['config']}", flush=True)
    outs = []
    for rep in range(2):  # the barrier counter carries over between applies
        for _, zt in zs:
            zt.fill_(float("nan"))
        batch.apply()
        batch.check()
        torch.cuda.synchronize()
        outs.append([zt.cpu().numpy().astype(np.float64) for _, zt in zs])
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b), "two applies of one batch differ"
    for (facs, Mp, ps, vs), pc, r, z in zip(refs, pcs, rs, outs[0]):
        for j in range(nrhs):
            zo = block_apply(facs, Mp, r[j], pres_scale=ps, vel_scales=vs)
            for a, b in zip(pc.offsets[:-1], pc.offsets[1:]):
                err = _rel(z[j, a:b], zo[a:b])
                assert err < TOL[prec], f"block [{a},{b}) residual {j}: rel err {err:.3e}"
    batch.close()
    for pc in pcs:
        pc.close()


def test_persistent_batch_tuning_keeps_results():
    _case("persistent batch autotuning, prec=f32")
    from paper_1712_00403_amd import fd
    pcs, refs = _build("f32")
    rs, zs, works = [], [], []
    for i, pc in enumerate(pcs):
        r = workloads.residuals(80 + i, 1, pc.N)
        rt = torch.from_numpy(r).float().cuda()
        zt = torch.empty_like(rt)
        rs.append(r)
        zs.append((rt, zt))
        works += pc.works(rt.data_ptr(), zt.data_ptr(), 1)
    batch = fd.Batch(works)
    choice = batch.tune(reps=2)
    assert batch.info()["config"] == choice
    assert 0 <= choice < 1024 and all(c < 3 for c in fd.Batch.choices_of(choice))
    batch.apply()
    batch.check()
    torch.cuda.synchronize()
    for (facs, Mp, ps, vs), pc, r, (rt, zt) in zip(refs, pcs, rs, zs):
        z = zt.cpu().numpy().astype(np.float64)
        zo = block_apply(facs, Mp, r[0], pres_scale=ps, vel_scales=vs)
        for a, b in zip(pc.offsets[:-1], pc.offsets[1:]):
            assert _rel(z[0, a:b], zo[a:b]) < TOL["f32"]
    batch.close()
    for pc in pcs:
        pc.close()


def test_persistent_batch_rejects_large_factors():
    _case("persistent batch argument checks")
    from paper_1712_00403_amd import fd
    from paper_1712_00403_amd.precond import BlockPreconditioner
    pc = BlockPreconditioner(workloads.taylor_hood_problem((70, 3, 3), 2), precision="f32")  # n = 140
    r = torch.zeros((1, pc.N), dtype=torch.float32, device="cuda")
    with pytest.raises(fd.FDError):
        fd.Batch(pc.works(r.data_ptr(), r.data_ptr(), 1))
    pc.close()
    pc = BlockPreconditioner(workloads.taylor_hood_problem((4, 4, 4), 2), precision="f32")
    r = torch.zeros((1, pc.N), dtype=torch.float32, device="cuda")
    z = torch.zeros_like(r)
    batch = fd.Batch(pc.works(r.data_ptr(), z.data_ptr(), 1))
    for bad in (-1, 3, 1 << 10):  # a choice of 3, words out of range
        with pytest.raises(fd.FDError):
            batch.set_config(bad)
    batch.close()
    pc.close()
