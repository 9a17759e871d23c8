"""GPU parity of the slab route of 3D BF16/FP16 plans against the FP64 oracle.

The slab route runs the products along directions 1 and 2 of Algorithm 1
(Sec. 5.2, steps 2 and 4) as one pass per i3-slab and keeps the tensor in
16 bits inside z between its three passes. These tests check it element by
element against the oracle on shapes that stress the slab kernel's edges
(n1 != n2, factor images narrower than the tile rows, the largest slab order
144, odd plane sizes), that it is the route that ran (launch family 5), that
it agrees with the five-stage route within the precision's tolerance, that
z == r and ld > N work, and that a non-finite residual does not reach its
neighbours through the shared LDS image.
"""
import numpy as np
import pytest

from oracle.assemble import taylor_hood_velocity_1d
from oracle.fd import FDFactors, fd_apply
from paper_1712_00403_amd import workloads
from parity_util import TOL, check_close, errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SLAB_FAMILY = 5


def _fd():
    from paper_1712_00403_amd import fd
    return fd


def _case(msg):
    print(f"[gpu case] {msg}", flush=True)


def _vel(n_el, p):
    vel = [taylor_hood_velocity_1d(n, p) for n in n_el]
    return [v[0] for v in vel], [v[1] for v in vel]


def _apply(plan, r, inplace=False, ld=None, timing=False):
    """Apply plan to host residuals r (nrhs, N); returns (host z, launch families by stage or None)."""
    fd = _fd()
    nrhs, N = r.shape
    ld = N if ld is None else ld
    buf = torch.zeros((nrhs, ld), dtype=torch.float32, device="cuda")
    buf[:, :N] = torch.from_numpy(r).float().cuda()
    out = buf if inplace else torch.full_like(buf, float("nan"))
    fams = None
    if timing:
        fd.timing_enable(True)
    try:
        plan.apply_ptr(buf.data_ptr(), out.data_ptr(), nrhs, ld, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        if timing:
            fd.timing_read()
            fams = {}
            for rec in fd.timing_launches():
                fams.setdefault(rec["stage"], set()).add(rec["family"])
    finally:
        if timing:
            fd.timing_enable(False)
    res = out.cpu().numpy().astype(np.float64)
    if not inplace and ld > N:
        assert np.all(np.isnan(res[:, N:])), "apply wrote outside the vectors"
    return res[:, :N], fams


# (n_el, p, weights): n_V = 2 n_el + p - 2 per direction
SLAB_CASES = [
    ((3, 4, 5), 2, (2.0, 1.0, 1.0)),     # n = (6, 8, 10): one tile
    ((18, 10, 22), 3, (1.0, 2.0, 1.0)),  # (37, 21, 45): odd plane size
    ((8, 33, 5), 1, (1.0, 1.0, 2.0)),    # (15, 65, 9): n2 = 16 (MT - 1) + 1
    ((3, 60, 5), 2, (1.0, 1.0, 1.0)),    # (6, 120, 10): F1 image narrower than the tile rows
    ((60, 3, 5), 2, (1.0, 1.0, 1.0)),    # (120, 6, 10)
    ((72, 72, 3), 2, (1.0, 1.0, 1.0)),   # (144, 144, 6): the largest slab
    ((64, 64, 8), 3, (1.0, 1.0, 2.0)),   # (129, 129, 17): the 64^3 p = 3 plane
]


@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("n_el,p,w", SLAB_CASES)
def test_slab_route_matches_oracle(prec, n_el, p, w):
    _case(f"slab route n_el={n_el} p={p} w={w} prec={prec}")
    Ks, Ms = _vel(n_el, p)
    f = FDFactors(Ks, Ms, np.array(w))
    plan = _fd().Plan(Ks, Ms, weights=np.array(w), precision=prec)
    r = workloads.residuals(31, 3, plan.N)
    z, fams = _apply(plan, r, timing=True)
    assert fams.get("mode1_fwd") == {SLAB_FAMILY} and fams.get("mode1_bwd") == {SLAB_FAMILY}, fams
    assert "mode2_fwd" not in fams and "mode2_bwd" not in fams, fams
    for j in range(r.shape[0]):
        check_close(z[j], fd_apply(f, r[j]), prec, f"residual {j}")
    plan.close()


@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("n_el,p", [((18, 10, 22), 3), ((64, 64, 8), 3)])
def test_slab_and_five_stage_routes_agree(prec, n_el, p, monkeypatch):
    _case(f"slab vs five-stage route n_el={n_el} p={p} prec={prec}")
    Ks, Ms = _vel(n_el, p)
    f = FDFactors(Ks, Ms)
    r = workloads.residuals(32, 2, int(np.prod([K.shape[0] for K in Ks])))
    plan_s = _fd().Plan(Ks, Ms, precision=prec)
    monkeypatch.setenv("FD_SLAB", "0")
    plan_5 = _fd().Plan(Ks, Ms, precision=prec)
    monkeypatch.delenv("FD_SLAB")
    zs, fs = _apply(plan_s, r, timing=True)
    z5, f5 = _apply(plan_5, r, timing=True)
    assert SLAB_FAMILY in fs["mode1_fwd"] and SLAB_FAMILY not in f5["mode1_fwd"], (fs, f5)
    for j in range(r.shape[0]):
        zo = fd_apply(f, r[j])
        check_close(zs[j], zo, prec, f"slab residual {j}")
        check_close(z5[j], zo, prec, f"five-stage residual {j}")
        # both round every operand to the 16-bit type once per product; the
        # routes differ in the order of the backward products only
        e2, _ = errors(zs[j], z5[j])
        assert e2 < TOL[prec], f"routes differ by {e2:.3e}"
    plan_s.close()
    plan_5.close()


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_slab_inplace_strided_and_repeatable(prec):
    """z == r and ld > N: the 16-bit layout stays inside each residual's FP32 footprint."""
    _case(f"slab in-place, ld > N, repeat, prec={prec}")
    Ks, Ms = _vel((9, 6, 11), 2)
    f = FDFactors(Ks, Ms)
    plan = _fd().Plan(Ks, Ms, precision=prec)
    r = workloads.residuals(33, 3, plan.N)
    ld = plan.N + 37
    z_out, _ = _apply(plan, r, inplace=False, ld=ld)
    z_in, _ = _apply(plan, r, inplace=True, ld=ld)
    z_again, _ = _apply(plan, r, inplace=False, ld=ld)
    assert np.array_equal(z_out, z_in), "in-place result differs from out-of-place"
    assert np.array_equal(z_out, z_again), "repeated apply differs"
    for j in range(3):
        check_close(z_out[j], fd_apply(f, r[j]), prec)
    plan.close()


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_slab_nonfinite_residual_stays_isolated(prec):
    """A NaN residual gives NaN only in its own result: the slab kernel clears
    its LDS image for every slab, so no padding entry carries a value of the
    previous slab (possibly of another residual) into a product."""
    _case(f"slab non-finite isolation, prec={prec}")
    Ks, Ms = _vel((18, 10, 22), 3)
    plan = _fd().Plan(Ks, Ms, precision=prec)
    r = workloads.residuals(34, 4, plan.N)
    z_clean, _ = _apply(plan, r)
    r_bad = r.copy()
    r_bad[1, :] = np.nan
    z_bad, _ = _apply(plan, r_bad)
    assert np.all(np.isnan(z_bad[1]))
    for j in (0, 2, 3):
        assert np.array_equal(z_bad[j], z_clean[j]), f"residual {j} changed next to a NaN residual"
    plan.close()


# scaled blocks (Sec. 6: z = D^{-1/2} P^{-1} D^{-1/2} r): the backward pass
# stages D^{-1/2} in LDS for orders up to 112 and loads it a slab ahead into
# registers above; the forward pass reads the columns past 128 separately
SCALED_CASES = [
    ((50, 7, 3), 3),   # n = (101, 15, 7): D^{-1/2} through LDS
    ((60, 4, 3), 3),   # (121, 9, 7): registers one slab ahead
    ((64, 10, 3), 3),  # (129, 21, 7): registers, columns past 128, odd rows
    ((4, 64, 3), 3),   # (9, 129, 7)
]


@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("n_el,p", SCALED_CASES)
def test_slab_scaled_matches_oracle(prec, n_el, p):
    _case(f"slab route with D^-1/2, n_el={n_el} p={p} prec={prec}")
    Ks, Ms = _vel(n_el, p)
    w = np.array([1.0, 2.0, 1.0])
    f = FDFactors(Ks, Ms, w)
    N = int(np.prod(f.n))
    dK = [np.diag(K) for K in Ks]
    dM = [np.diag(M) for M in Ms]
    diagP = (w[2] * np.einsum("k,j,i->kji", dK[2], dM[1], dM[0]) + w[1] * np.einsum("k,j,i->kji", dM[2], dK[1], dM[0])
             + w[0] * np.einsum("k,j,i->kji", dM[2], dM[1], dK[0])).reshape(-1)
    D = 0.5 + np.random.default_rng(36).random(N)
    plan = _fd().Plan(Ks, Ms, weights=w, diag_target=diagP * D, precision=prec)
    r = workloads.residuals(37, 2, plan.N)
    z, fams = _apply(plan, r, timing=True)
    assert fams.get("mode1_fwd") == {SLAB_FAMILY} and fams.get("mode1_bwd") == {SLAB_FAMILY}, fams
    s = 1.0 / np.sqrt(D)
    for j in range(2):
        check_close(z[j], s * fd_apply(f, s * r[j]), prec, f"residual {j}")
    plan.close()


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_slab_order_limit(prec):
    """n1 = 145 is past the slab kernel (144): the plan takes the five-stage route, still correct."""
    _case(f"slab order limit n1=145, prec={prec}")
    Ks, Ms = _vel((72, 4, 3), 3)  # n = (145, 9, 7)
    f = FDFactors(Ks, Ms)
    plan = _fd().Plan(Ks, Ms, precision=prec)
    r = workloads.residuals(35, 2, plan.N)
    z, fams = _apply(plan, r, timing=True)
    assert all(SLAB_FAMILY not in v for v in fams.values()), fams
    for j in range(2):
        check_close(z[j], fd_apply(f, r[j]), prec)
    plan.close()
