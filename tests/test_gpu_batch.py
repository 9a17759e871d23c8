"""GPU parity of the persistent batched apply (one launch for many heterogeneous patches)."""
import os
import sys
import time

import numpy as np
import pytest

from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
from oracle.fd import FDFactors, block_apply, velocity_weights
from paper_1712_00403_amd import workloads
from parity_util import TOL, TOL_MAX, check_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (n_el, p, geometry or None): 3D and 2D, every pressure degree 1..5, simple and
# coefficient-aware blocks, factor orders from 3 to 100
PATCHES = [((5, 7, 4), 2, None), ((9, 4, 6), 3, "sine"), ((3, 5, 8), 4, None), ((12, 10), 2, "warped"),
           ((7, 6, 5), 5, "sine"), ((4, 4, 4), 1, None), ((48, 3, 4), 4, None), ((30, 20), 3, "sine")]


def _case(msg):
    print(f"[gpu case] {msg}", flush=True)


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


SEGMENTS = 1 << 11  # the segment route


@pytest.mark.parametrize("prec,config", [("f64", 0), ("f32", 0), ("bf16", 0), ("f16", 0), ("bf16_split", 0),
                                         ("f32", ALL_NARROW), ("bf16", ALL_NARROW), ("f64", MIXED),
                                         ("f64", ALL_PIPELINED), ("f32", ALL_PIPELINED), ("bf16", ALL_PIPELINED),
                                         ("f16", ALL_PIPELINED), ("bf16_split", ALL_PIPELINED), ("f32", MIXED),
                                         ("f64", MIXED | SEGMENTS), ("f32", ALL_PIPELINED | SEGMENTS),
                                         ("bf16", SEGMENTS), ("f16_split", ALL_NARROW | SEGMENTS)])
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
                check_close(z[j, a:b], zo[a:b], prec, f"block [{a},{b}) residual {j}")
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
    assert 0 <= (choice & ~fd.Batch.SEGMENTS) < 1024 and all(c < 3 for c in fd.Batch.choices_of(choice))
    batch.apply()
    batch.check()
    torch.cuda.synchronize()
    for (facs, Mp, ps, vs), pc, r, (rt, zt) in zip(refs, pcs, rs, zs):
        z = zt.cpu().numpy().astype(np.float64)
        zo = block_apply(facs, Mp, r[0], pres_scale=ps, vel_scales=vs)
        for a, b in zip(pc.offsets[:-1], pc.offsets[1:]):
            check_close(z[0, a:b], zo[a:b], "f32", f"block [{a},{b})")
    batch.close()
    for pc in pcs:
        pc.close()


# 3D patches only (every work a slab-route plan in BF16/FP16): the staged route
STAGED_PATCHES = [i for i, (n_el, _, _) in enumerate(PATCHES) if len(n_el) == 3]


def _batch_io(pcs, idx, nrhs, seed0, dt):
    rs, zs, works = [], [], []
    for i in idx:
        pc = pcs[i]
        r = workloads.residuals(seed0 + i, nrhs, pc.N)
        rt = torch.from_numpy(r).to(dt).cuda()
        zt = torch.full_like(rt, float("nan"))
        rs.append(r)
        zs.append((rt, zt))
        works += pc.works(rt.data_ptr(), zt.data_ptr(), nrhs)
    return rs, zs, works


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_staged_route_matches_oracle(prec):
    """The staged route of a batch of 3D patches (simple and coefficient-aware blocks):
    slab passes and the 16-bit fused pass over device tables, one launch per stage and
    row-tile group. Compared with the oracle element-wise, repeated bitwise, in place
    (z == r), and against the persistent route of the same batch within the tolerance."""
    _case(f"staged batch route of {len(STAGED_PATCHES)} 3D patches, prec={prec}")
    from paper_1712_00403_amd import fd
    pcs, refs = _build(prec)
    nrhs = 2
    rs, zs, works = _batch_io(pcs, STAGED_PATCHES, nrhs, 90, torch.float32)
    batch = fd.Batch(works)
    batch.set_config(fd.Batch.STAGED)
    assert batch.info()["config"] == fd.Batch.STAGED
    fd.timing_enable(True)
    try:
        batch.apply()
        torch.cuda.synchronize()
        fd.timing_read()
        fams = {(rec["stage"], rec["family"]) for rec in fd.timing_launches()}
    finally:
        fd.timing_enable(False)
    assert fams == {("mode1_fwd", 5), ("last_mode_fused", 3), ("mode1_bwd", 5)}, fams
    outs = []
    for rep in range(2):
        for _, zt in zs:
            zt.fill_(float("nan"))
        batch.apply()
        batch.check()
        torch.cuda.synchronize()
        outs.append([zt.cpu().numpy().astype(np.float64) for _, zt in zs])
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b), "two applies of one batch differ"
    for k, i in enumerate(STAGED_PATCHES):
        facs, Mp, ps, vs = refs[i]
        for j in range(nrhs):
            zo = block_apply(facs, Mp, rs[k][j], pres_scale=ps, vel_scales=vs)
            for a, b in zip(pcs[i].offsets[:-1], pcs[i].offsets[1:]):
                check_close(outs[0][k][j, a:b], zo[a:b], prec, f"patch {i} block [{a},{b}) residual {j}")
    # the persistent route of the same works
    batch.set_config(0)
    for _, zt in zs:
        zt.fill_(float("nan"))
    batch.apply()
    batch.check()
    torch.cuda.synchronize()
    for k, (_, zt) in enumerate(zs):
        zp = zt.cpu().numpy().astype(np.float64)
        for j in range(nrhs):
            e = np.linalg.norm(zp[j] - outs[0][k][j]) / np.linalg.norm(zp[j])
            assert e < TOL[prec], f"patch {STAGED_PATCHES[k]}: routes differ by {e:.3e}"
    batch.close()
    # in place: z == r
    rs2, zs2, works2 = [], [], []
    for k, i in enumerate(STAGED_PATCHES):
        rt = torch.from_numpy(rs[k]).float().cuda()
        zs2.append(rt)
        works2 += pcs[i].works(rt.data_ptr(), rt.data_ptr(), nrhs)
    batch = fd.Batch(works2)
    batch.set_config(fd.Batch.STAGED)
    batch.apply()
    batch.check()
    torch.cuda.synchronize()
    for k, rt in enumerate(zs2):
        assert np.array_equal(rt.cpu().numpy().astype(np.float64), outs[0][k]), "in-place staged apply differs"
    batch.close()
    for pc in pcs:
        pc.close()


def test_staged_route_availability():
    """Only batches whose works are all 3D BF16/FP16 slab-route plans have the staged route."""
    _case("staged route availability")
    from paper_1712_00403_amd import fd
    for prec, idx in (("f32", STAGED_PATCHES), ("bf16", list(range(len(PATCHES))))):
        pcs, _ = _build(prec)
        _, _, works = _batch_io(pcs, idx, 1, 95, torch.float32)
        batch = fd.Batch(works)
        with pytest.raises(fd.FDError):
            batch.set_config(fd.Batch.STAGED)
        cfg = batch.tune(reps=1)
        assert cfg != fd.Batch.STAGED
        batch.close()
        for pc in pcs:
            pc.close()


def test_batch_signature_and_tuning_cache(tmp_path):
    """Equal layouts give equal signatures whatever the buffers; a different nrhs or
    precision changes it; tune(cache=...) stores the word and a second batch with the
    same signature takes it from the file."""
    _case("batch signature and tuning cache")
    from paper_1712_00403_amd import fd
    pcs, _ = _build("f32")
    _, zs_a, works_a = _batch_io(pcs, STAGED_PATCHES, 1, 100, torch.float32)
    _, zs_b, works_b = _batch_io(pcs, STAGED_PATCHES, 1, 110, torch.float32)
    _, zs_c, works_c = _batch_io(pcs, STAGED_PATCHES, 2, 120, torch.float32)
    a, b, c = fd.Batch(works_a), fd.Batch(works_b), fd.Batch(works_c)
    assert a.signature() == b.signature() != c.signature()
    cache = str(tmp_path / "tune.json")
    cfg = a.tune(reps=1, cache=cache)
    import json
    with open(cache) as fh:
        assert json.load(fh) == {format(a.signature(), "016x"): cfg}
    b.set_config(0)
    assert b.tune(reps=1, cache=cache) == cfg and b.info()["config"] == cfg
    b.apply()
    b.check()
    torch.cuda.synchronize()
    for x in (a, b, c):
        x.close()
    for pc in pcs:
        pc.close()


@pytest.mark.parametrize("prec,config", [("f64", MIXED), ("f32", ALL_PIPELINED), ("bf16", 0)])
def test_segment_route_equals_persistent_route(prec, config):
    """The segment route runs the same bodies on the same tiles as the persistent
    launch, one launch per segment: the results agree bit for bit."""
    _case(f"segment route vs persistent launch, prec={prec}, config={config}")
    from paper_1712_00403_amd import fd
    pcs, _ = _build(prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    _, zs, works = _batch_io(pcs, range(len(PATCHES)), 2, 130, dt)
    batch = fd.Batch(works)
    outs = []
    for cfg in (config, config | fd.Batch.SEGMENTS):
        batch.set_config(cfg)
        assert batch.info()["config"] == cfg
        for _, zt in zs:
            zt.fill_(float("nan"))
        batch.apply()
        batch.check()
        torch.cuda.synchronize()
        outs.append([zt.cpu().numpy() for _, zt in zs])
    for a, b in zip(*outs):
        assert np.array_equal(a, b), "segment route differs from the persistent launch"
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


GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_C4 = {}


def _c4_setup():
    """The 256-patch coefficient-aware batch: descriptors, residuals, the library's host setup (once)."""
    if not _C4:
        from concurrent.futures import ThreadPoolExecutor
        from paper_1712_00403_amd.geometry import geometry_blocks
        sys.path.insert(0, GOLDEN_DIR)
        import make_batch_golden as mk
        patches, sizes, res = mk.batch_inputs()
        geo = workloads.sine_geometry(3)
        probs = [workloads.taylor_hood_problem(n_el, p, unit_weights=True) for n_el, p in patches]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=16) as ex:
            blocks = list(ex.map(lambda pr: geometry_blocks(pr, geo), probs))
        print(f"  host setup of {len(probs)} patches: {time.perf_counter() - t0:.1f} s", flush=True)
        golden = dict(np.load(os.path.join(GOLDEN_DIR, "batch_256_sampled.npz")))
        _C4.update(mk=mk, patches=patches, sizes=sizes, res=res, geo=geo, probs=probs, blocks=blocks,
                   golden=golden)
    return _C4


def check_c4_samples(Z, offs, pcs, c4, prec, what):
    """Compare the sampled pencils of the checked patches with the oracle's values; returns worst errors."""
    mk, golden = c4["mk"], c4["golden"]
    worst = (0.0, 0.0)
    for i in golden["patches"]:
        n_el, p = c4["patches"][i]
        zi = Z[offs[i]:offs[i + 1]]
        po = pcs[i].offsets
        assert len(po) - 1 == len(mk.patch_blocks(n_el, p))
        for b in range(len(po) - 1):
            zb = zi[po[b]:po[b + 1]]
            idx = golden[f"p{i}_b{b}_idx"]
            zo = golden[f"p{i}_b{b}_val"]
            d = zb[idx] - zo
            assert np.all(np.isfinite(zb[idx])), f"{what} patch {i} block {b}: non-finite entries"
            e2 = float(np.sqrt(np.mean(d * d)) / golden[f"p{i}_b{b}_rms"])
            emax = float(np.max(np.abs(d)) / golden[f"p{i}_b{b}_max"])
            assert e2 < TOL[prec] and emax < TOL_MAX[prec], (
                f"{what} patch {i} n_el={n_el} p={p} block {b}: sampled rel err {e2:.3e}, rel max err {emax:.3e}")
            worst = (max(worst[0], e2), max(worst[1], emax))
    return worst


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN_DIR, "batch_256_sampled.npz")),
                    reason="stored oracle values not generated (tests/golden/make_batch_golden.py)")
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_c4_batch_256_patches_largest_and_drawn(prec):
    """The 256-patch batch in one persistent launch (default and tuned configurations, as timed by the bench).

    The 8 largest patches (n up to 96 per direction) and 8 drawn ones are
    compared with the oracle at whole sampled pencils of every block (corner
    pencils in the first and last tiles of every pass, two drawn ones), in
    the RMS and element-wise, each relative to the block's oracle RMS / max.
    """
    _case(f"256-patch coefficient-aware batch, prec={prec}")
    from paper_1712_00403_amd import fd
    from paper_1712_00403_amd.geometry import GeometryPreconditioner
    c4 = _c4_setup()
    pcs = [GeometryPreconditioner(pr, c4["geo"], precision=prec, blocks=b) for pr, b in zip(c4["probs"], c4["blocks"])]
    assert [pc.N for pc in pcs] == c4["sizes"]
    dt = torch.float64 if prec == "f64" else torch.float32
    offs = np.concatenate([[0], np.cumsum(c4["sizes"])]).astype(np.int64)
    R = torch.from_numpy(np.concatenate(c4["res"])).to(dt).cuda()
    Z = torch.full_like(R, float("nan"))
    eb = R.element_size()
    works = []
    for i, pc in enumerate(pcs):
        works += pc.works(R.data_ptr() + int(offs[i]) * eb, Z.data_ptr() + int(offs[i]) * eb, 1)
    batch = fd.Batch(works)
    batch.apply()
    batch.check()
    torch.cuda.synchronize()
    e = check_c4_samples(Z.double().cpu().numpy(), offs, pcs, c4, prec, "default config")
    print(f"  default config {batch.info()['config']}: sampled rel err {e[0]:.3e}, rel max err {e[1]:.3e}")
    cfg = batch.tune(reps=2)
    Z.fill_(float("nan"))
    batch.apply()
    batch.check()
    torch.cuda.synchronize()
    e = check_c4_samples(Z.double().cpu().numpy(), offs, pcs, c4, prec, f"tuned config {cfg}")
    print(f"  tuned config {cfg}: sampled rel err {e[0]:.3e}, rel max err {e[1]:.3e}")
    if prec in ("bf16", "f16"):  # the staged route (every patch is a slab-route plan)
        batch.set_config(fd.Batch.STAGED)
        Z.fill_(float("nan"))
        batch.apply()
        batch.check()
        torch.cuda.synchronize()
        e = check_c4_samples(Z.double().cpu().numpy(), offs, pcs, c4, prec, "staged route")
        print(f"  staged route: sampled rel err {e[0]:.3e}, rel max err {e[1]:.3e}")
    batch.close()
    for pc in pcs:
        pc.close()
