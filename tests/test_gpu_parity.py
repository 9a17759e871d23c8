"""GPU parity: the HIP FD apply against the FP64 oracle, element by element.

Each case prints its name before touching the GPU. Errors are per residual
and per block (the pressure block's entries are orders of magnitude larger
than the velocity ones, so one norm over the whole block vector would hide
velocity errors), in the relative 2-norm and element-wise (relative
max-norm), each against the precision's tolerance.
"""
import numpy as np
import pytest

from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
from oracle.fd import FDFactors, block_apply, fd_apply, mass_solve_banded, velocity_weights
from paper_1712_00403_amd import workloads
from parity_util import TOL, check_blocks, check_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _fd():
    from paper_1712_00403_amd import fd
    return fd


def _case(msg):
    print(f"[gpu case] {msg}", flush=True)


def _vel_factors(n_el, p):
    vel = [taylor_hood_velocity_1d(n, p) for n in n_el]
    return [v[0] for v in vel], [v[1] for v in vel]


def _run_plan(plan, r, inplace=False, ld=None):
    """Apply plan to host residuals r (nrhs, N) through device tensors; returns host z."""
    dt = torch.float64 if plan.io_dtype == "float64" else torch.float32
    nrhs, N = r.shape
    ld = N if ld is None else ld
    buf = torch.zeros((nrhs, ld), dtype=dt, device="cuda")
    buf[:, :N] = torch.from_numpy(r).to(dt).cuda()
    out = buf if inplace else torch.full_like(buf, float("nan"))
    plan.apply_ptr(buf.data_ptr(), out.data_ptr(), nrhs, ld, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    if not inplace and ld > N:
        assert np.all(np.isnan(res[:, N:])), "apply wrote outside the vectors"
    return res[:, :N].astype(np.float64)


# orders 16 (MT - 1) + 1 (17, 33, 65: one row in the last row tile) in every
# direction, i.e. in each of the three pass kinds
CASES_3D = [((3, 4, 5), 2, (2.0, 1.0, 1.0)), ((18, 10, 22), 3, (1.0, 2.0, 1.0)),
            ((8, 33, 5), 1, (1.0, 1.0, 2.0)), ((6, 7, 9), 5, (1.0, 1.0, 1.0)),
            ((8, 16, 32), 3, (1.0, 1.0, 1.0)), ((32, 8, 16), 3, (1.0, 3.0, 1.0))]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "bf16_split", "f16", "f16_split", "fp8_split"])
@pytest.mark.parametrize("n_el,p,w", CASES_3D)
def test_fd3d_velocity_block(prec, n_el, p, w):
    _case(f"fd3d velocity n_el={n_el} p={p} w={w} prec={prec}")
    Ks, Ms = _vel_factors(n_el, p)
    f = FDFactors(Ks, Ms, np.array(w))
    plan = _fd().Plan(Ks, Ms, weights=np.array(w), precision=prec)
    r = workloads.residuals(11, 3, plan.N)
    z = _run_plan(plan, r)
    for j in range(r.shape[0]):
        check_close(z[j], fd_apply(f, r[j]), prec, f"residual {j}")
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "bf16_split", "f16", "f16_split", "fp8_split"])
# ((10, 80), 3): n_2 = 161, the FP64 last mode beyond the fused pipelined kernel
@pytest.mark.parametrize("n_el,p", [((16, 16), 2), ((13, 29), 3), ((2, 3), 1), ((60, 40), 4), ((16, 32), 3),
                                    ((10, 80), 3)])
def test_fd2d_velocity_block(prec, n_el, p):
    _case(f"fd2d velocity n_el={n_el} p={p} prec={prec}")
    Ks, Ms = _vel_factors(n_el, p)
    f = FDFactors(Ks, Ms)
    plan = _fd().Plan(Ks, Ms, precision=prec)
    r = workloads.residuals(12, 4, plan.N)
    z = _run_plan(plan, r)
    for j in range(r.shape[0]):
        check_close(z[j], fd_apply(f, r[j]), prec, f"residual {j}")
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16", "fp8_split"])
@pytest.mark.parametrize("n_el,p", [((5, 9, 4), 2), ((20, 11, 17), 3), ((7, 12), 2)])
def test_pressure_mass_block(prec, n_el, p):
    _case(f"pressure mass n_el={n_el} p={p} prec={prec}")
    Ms = [pressure_1d(n, p) for n in n_el]
    plan = _fd().Plan(None, Ms, precision=prec)
    r = workloads.residuals(13, 2, plan.N)
    z = _run_plan(plan, r)
    for j in range(r.shape[0]):
        check_close(z[j], mass_solve_banded(Ms, r[j]), prec, f"residual {j}")
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_inplace_and_strided(prec):
    _case(f"in-place and ld > N, prec={prec}")
    Ks, Ms = _vel_factors((9, 6, 11), 2)
    f = FDFactors(Ks, Ms)
    plan = _fd().Plan(Ks, Ms, precision=prec)
    r = workloads.residuals(14, 3, plan.N)
    for inplace in (True, False):
        z = _run_plan(plan, r, inplace=inplace, ld=plan.N + 37)
        for j in range(3):
            check_close(z[j], fd_apply(f, r[j]), prec)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16"])
def test_scaled_variant(prec):
    _case(f"diagonal scaling, prec={prec}")
    Ks, Ms = _vel_factors((5, 7, 6), 3)
    f = FDFactors(Ks, Ms, np.array([1.0, 1.0, 2.0]))
    rng = np.random.default_rng(21)
    N = int(np.prod(f.n))
    # diag(P) computed from the 1D diagonals, target = diag(P) * D
    dK = [np.diag(K) for K in Ks]
    dM = [np.diag(M) for M in Ms]
    diagP = (2.0 * np.einsum("k,j,i->kji", dK[2], dM[1], dM[0]) + np.einsum("k,j,i->kji", dM[2], dK[1], dM[0])
             + np.einsum("k,j,i->kji", dM[2], dM[1], dK[0])).reshape(-1)
    D = 0.5 + rng.random(N)
    plan = _fd().Plan(Ks, Ms, weights=np.array([1.0, 1.0, 2.0]), diag_target=diagP * D, precision=prec)
    r = workloads.residuals(15, 2, plan.N)
    z = _run_plan(plan, r)
    s = 1.0 / np.sqrt(D)
    for j in range(2):
        zo = s * fd_apply(f, s * r[j])
        check_close(z[j], zo, prec)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_block_preconditioner_mixed_batch(prec):
    """2D and 3D problems, velocity and pressure blocks, in one fd_apply_batched call."""
    _case(f"batched heterogeneous block preconditioners, prec={prec}")
    from paper_1712_00403_amd.precond import BlockPreconditioner
    fd = _fd()
    probs = [workloads.taylor_hood_problem((4, 6, 5), 2), workloads.taylor_hood_problem((10, 7), 3),
             workloads.taylor_hood_problem((3, 3, 8), 4)]
    pcs = [BlockPreconditioner(pr, precision=prec) for pr in probs]
    dt = torch.float64 if prec == "f64" else torch.float32
    rs, zs, works = [], [], []
    for i, pc in enumerate(pcs):
        r = workloads.residuals(30 + i, 2, pc.N)
        rt = torch.from_numpy(r).to(dt).cuda()
        zt = torch.empty_like(rt)
        rs.append(r)
        zs.append((rt, zt))
        works += pc.works(rt.data_ptr(), zt.data_ptr(), 2)
    fd.apply_batched(works)
    torch.cuda.synchronize()
    for pr, pc, r, (rt, zt) in zip(probs, pcs, rs, zs):
        z = zt.cpu().numpy().astype(np.float64)
        d, p = pr.ndim, pr.p
        Ks, Ms = _vel_factors(pr.n_el, p)
        wts = [np.array(b.weights) for b in pr.blocks[:d]]
        facs = [FDFactors(Ks, Ms, wts[k]) for k in range(d)]
        Mp = [pressure_1d(n, p) for n in pr.n_el]
        for j in range(2):
            zo = block_apply(facs, Mp, r[j])
            for a, b in zip(pc.offsets[:-1], pc.offsets[1:]):
                check_close(z[j, a:b], zo[a:b], prec)
        pc.close()


_FULL = {}


def _full_size_oracle(name, n_el, p, nrhs, seed):
    """Residuals and oracle block vectors of a full-size TH patch (computed once per module)."""
    if name not in _FULL:
        Ks, Ms = _vel_factors(n_el, p)
        facs = [FDFactors(Ks, Ms, velocity_weights(3, k)) for k in range(3)]
        Mp = [pressure_1d(n, p) for n in n_el]
        N = 3 * int(np.prod([K.shape[0] for K in Ks])) + int(np.prod([M.shape[0] for M in Mp]))
        r = workloads.residuals(seed, nrhs, N)
        _FULL[name] = (r, [block_apply(facs, Mp, r[j]) for j in range(nrhs)])
    return _FULL[name]


def _full_size_case(name, n_el, p, nrhs, seed, prec, sizes):
    from paper_1712_00403_amd.precond import BlockPreconditioner
    prob = workloads.taylor_hood_problem(n_el, p)
    pc = BlockPreconditioner(prob, precision=prec)
    assert pc.sizes == sizes
    r, zo = _full_size_oracle(name, n_el, p, nrhs, seed)
    dt = torch.float64 if prec == "f64" else torch.float32
    z = pc.apply(torch.from_numpy(r).to(dt).cuda())
    torch.cuda.synchronize()
    z = z.cpu().numpy().astype(np.float64)
    for j in range(nrhs):
        for k, (a, b) in enumerate(zip(pc.offsets[:-1], pc.offsets[1:])):
            e2, emax = check_close(z[j, a:b], zo[j][a:b], prec, f"residual {j} block {k}")
            print(f"  residual {j} block {k}: rel err {e2:.3e}, rel max err {emax:.3e}")
    pc.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16", "bf16_split", "f16_split", "fp8_split"])
def test_full_size_64cube_p3(prec):
    """The 64^3, p = 3 patch (n_V = 129, n_Q = 67) in the launch configuration of the bench, every residual."""
    _case(f"full-size 64^3 p=3 block vector, 2 residuals, prec={prec}")
    _full_size_case("64_p3", (64, 64, 64), 3, 2, 1, prec, [129 ** 3] * 3 + [67 ** 3])


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_full_size_96cube_p4(prec):
    """The 96^3, p = 4 patch of the serving mix: n_V = 194 in all three directions (FP64: split last mode)."""
    _case(f"full-size 96^3 p=4 block vector, prec={prec}")
    _full_size_case("96_p4", (96, 96, 96), 4, 1, 4, prec, [194 ** 3] * 3 + [100 ** 3])


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "bf16_split"])
def test_global_fragment_kernels(prec, monkeypatch):
    """The kernels that read packed factor fragments from global memory (FD_KERNEL=v1)."""
    _case(f"global-fragment kernels, prec={prec}")
    monkeypatch.setenv("FD_KERNEL", "v1")
    Ks, Ms = _vel_factors((7, 12, 5), 3)
    f = FDFactors(Ks, Ms, np.array([1.0, 2.0, 1.0]))
    plan = _fd().Plan(Ks, Ms, weights=np.array([1.0, 2.0, 1.0]), precision=prec)
    r = workloads.residuals(16, 2, plan.N)
    z = _run_plan(plan, r)
    for j in range(2):
        check_close(z[j], fd_apply(f, r[j]), prec)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "bf16_split"])
@pytest.mark.parametrize("n_el", [(96, 5, 4), (4, 96, 3), (3, 4, 96)])
def test_large_factor_96_elements_p4(prec, n_el):
    """n = 194 in one direction (96 elements, p = 4): factor beyond the FP64 LDS image."""
    _case(f"n=194 direction, n_el={n_el}, prec={prec}")
    Ks, Ms = _vel_factors(n_el, 4)
    f = FDFactors(Ks, Ms, np.array([2.0, 1.0, 1.0]))
    plan = _fd().Plan(Ks, Ms, weights=np.array([2.0, 1.0, 1.0]), precision=prec)
    r = workloads.residuals(17, 2, plan.N)
    z = _run_plan(plan, r)
    for j in range(2):
        check_close(z[j], fd_apply(f, r[j]), prec)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("ndim,n_el,p,geo", [(3, (6, 9, 5), 2, "sine"), (3, (5, 4, 7), 3, "warped"),
                                              (2, (12, 9), 2, "warped")])
def test_geometry_variant_block_apply(prec, ndim, n_el, p, geo):
    """Coefficient-aware P_D: per-component factors, D_V / D_Q scalings (Sec. 6, Appendix)."""
    _case(f"geometry variant ndim={ndim} n_el={n_el} p={p} geometry={geo} prec={prec}")
    from oracle.geometry import GeometryBlocks
    from paper_1712_00403_amd.geometry import GeometryPreconditioner
    g = (workloads.sine_geometry(ndim) if geo == "sine"
         else workloads.warped_geometry(ndim, nu=workloads.wavy_viscosity))
    prob = workloads.taylor_hood_problem(n_el, p, unit_weights=True)
    pc = GeometryPreconditioner(prob, g, precision=prec)
    gb = GeometryBlocks(n_el, p, g)
    facs = [FDFactors(gb.vel_K[k], gb.vel_M[k]) for k in range(ndim)]
    r = workloads.residuals(50, 2, pc.N)
    dt = torch.float64 if prec == "f64" else torch.float32
    z = pc.apply(torch.from_numpy(r).to(dt).cuda())
    torch.cuda.synchronize()
    z = z.cpu().numpy().astype(np.float64)
    for j in range(2):
        zo = block_apply(facs, gb.pres_M, r[j], pres_scale=gb.pres_scale, vel_scales=gb.vel_scales)
        for a, b in zip(pc.offsets[:-1], pc.offsets[1:]):
            check_close(z[j, a:b], zo[a:b], prec, f"residual {j} block [{a},{b})")
    pc.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_largest_factor_order_256(prec):
    """n = 256 (the largest factor order a plan accepts) in direction 1, tiny elsewhere."""
    _case(f"n=256 direction, prec={prec}")
    Ks, Ms = _vel_factors((128, 2, 3), 2)
    assert Ks[0].shape[0] == 256
    f = FDFactors(Ks, Ms, np.array([1.0, 2.0, 1.0]))
    plan = _fd().Plan(Ks, Ms, weights=np.array([1.0, 2.0, 1.0]), precision=prec)
    r = workloads.residuals(18, 2, plan.N)
    z = _run_plan(plan, r)
    for j in range(2):
        check_close(z[j], fd_apply(f, r[j]), prec)
    plan.close()


def test_smallest_factor_order_2_and_empty_work():
    """n = 2 (pressure space of one linear element) and nrhs = 0 (a no-op)."""
    _case("n=2 directions and an empty work")
    Ms = [pressure_1d(1, 1), pressure_1d(3, 1), pressure_1d(1, 1)]
    assert [M.shape[0] for M in Ms] == [2, 4, 2]
    plan = _fd().Plan(None, Ms, precision="f64")
    r = workloads.residuals(19, 3, plan.N)
    z = _run_plan(plan, r)
    for j in range(3):
        check_close(z[j], mass_solve_banded(Ms, r[j]), "f64")
    buf = torch.full((1, plan.N), 7.0, dtype=torch.float64, device="cuda")
    plan.apply_ptr(buf.data_ptr(), buf.data_ptr(), 0, plan.N, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.all(buf == 7.0)
    plan.close()


def test_plan_rejects_order_above_256():
    _case("fd_setup argument checks")
    fd = _fd()
    Ks, Ms = _vel_factors((129, 2, 2), 2)  # n = 258
    with pytest.raises(fd.FDError) as e:
        fd.Plan(Ks, Ms)
    assert e.value.status == fd.FD_E_ARG


def test_fp8_split_limits():
    _case("FP8 split plan limits: no diag_target, n <= 224, no persistent batch")
    fd = _fd()
    Ks, Ms = _vel_factors((4, 5, 6), 2)
    with pytest.raises(fd.FDError, match="FD_E_UNSUPPORTED"):
        fd.Plan(Ks, Ms, precision="fp8_split", diag_target=np.ones(int(np.prod([k.shape[0] for k in Ks]))))
    Kb, Mb = _vel_factors((120, 3, 3), 2)  # n = 240 in direction 1
    with pytest.raises(fd.FDError, match="FD_E_UNSUPPORTED"):
        fd.Plan(Kb, Mb, precision="fp8_split")
    plan = fd.Plan(Ks, Ms, precision="fp8_split")
    r = torch.zeros((1, plan.N), dtype=torch.float32, device="cuda")
    z = torch.zeros_like(r)
    with pytest.raises(fd.FDError, match="FD_E_UNSUPPORTED"):
        fd.Batch([(plan, r.data_ptr(), z.data_ptr(), 1, plan.N)])
    plan.close()


def test_fp64_orders_up_to_224_run_pipelined():
    _case("FP64 n = 194: every pass, the split last mode included, on the pipelined kernels")
    fd = _fd()
    Ks, Ms = _vel_factors((3, 4, 96), 4)  # n = (10, 12, 194)
    f = FDFactors(Ks, Ms, velocity_weights(3, 2))
    plan = fd.Plan(Ks, Ms, weights=velocity_weights(3, 2), precision="f64")
    r = workloads.residuals(31, 2, plan.N)
    fd.timing_enable(True)
    try:
        z = _run_plan(plan, r)
        fd.timing_read()
        launches = fd.timing_launches()
    finally:
        fd.timing_enable(False)
    assert launches and all(l["family"] == 3 for l in launches), launches
    # the last mode (n = 194) runs as two launches in stage 2
    assert sum(l["count"] for l in launches if l["stage"] == "last_mode_fused") == 2
    for j in range(r.shape[0]):
        check_close(z[j], fd_apply(f, r[j]), "f64")
    plan.close()


def _random_cases(seed, count):
    """Seeded 3D/2D blocks with per-direction orders spread over 2..224 (small products)."""
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(count):
        d = int(rng.integers(2, 4))
        big = int(rng.integers(0, d))
        n = []
        for i in range(d):
            if i == big:
                n.append(int(rng.integers(2, 225)))
            else:
                n.append(int(rng.integers(2, 24 if d == 3 else 60)))
        cases.append(tuple(n))
    return cases


def _spd_pair(n, rng):
    """A random SPD pencil (K, M) of order n: M diagonally dominant, K = A A^T + n I."""
    A = rng.standard_normal((n, n))
    M = np.eye(n) * n + 0.1 * (A + A.T)
    B = rng.standard_normal((n, n))
    K = B @ B.T + n * np.eye(n)
    return K, M


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16", "bf16_split", "f16_split", "fp8_split"])
@pytest.mark.parametrize("shape", _random_cases(2024, 8))
def test_random_orders(prec, shape):
    _case(f"random-order block n={shape} prec={prec}")
    rng = np.random.default_rng(sum(shape) * 7 + len(shape))
    pairs = [_spd_pair(n, rng) for n in shape]
    Ks, Ms = [p[0] for p in pairs], [p[1] for p in pairs]
    w = rng.uniform(0.5, 2.0, len(shape))
    f = FDFactors(Ks, Ms, w)
    plan = _fd().Plan(Ks, Ms, weights=w, precision=prec)
    r = workloads.residuals(int(rng.integers(0, 1000)), 2, plan.N)
    z = _run_plan(plan, r)
    for j in range(r.shape[0]):
        check_close(z[j], fd_apply(f, r[j]), prec, f"residual {j}")
    plan.close()
