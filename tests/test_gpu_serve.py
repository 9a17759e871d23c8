"""Serving loop on the GPU: results do not depend on the batch a request lands in."""
import time

import numpy as np
import pytest

from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
from oracle.fd import FDFactors, block_apply, velocity_weights
from paper_1712_00403_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"[gpu case] {msg}", flush=True)


def _classes(prec):
    from paper_1712_00403_amd import serve
    return {"2d": serve.RequestClass("2d", lambda: workloads.taylor_hood_problem((16, 16), 2, unit_weights=True), prec),
            "3d_a": serve.RequestClass("3d_a", lambda: workloads.taylor_hood_problem((10, 12, 8), 3), prec),
            "3d_b": serve.RequestClass("3d_b", lambda: workloads.taylor_hood_problem((6, 5, 7), 2), prec)}


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_request_alone_equals_request_in_mix(prec):
    _case(f"serving: alone vs in a mixed step, prec={prec}")
    from paper_1712_00403_amd import serve
    classes = _classes(prec)
    ex = serve.GpuExecutor(classes, slots=3, seed=4)
    srv = serve.Server(classes, ex, hbm_budget=1 << 30)
    target = serve.Request(0, "3d_a", 0.0, slot=1)
    srv.submit(target)
    assert srv.step() == 1
    h_alone = srv.inflight[0][0]
    srv.collect(wait=True)
    alone = h_alone[1][0].cpu().numpy()
    mix = [serve.Request(1, "2d", 0.0, slot=0), serve.Request(2, "3d_b", 0.0, slot=2),
           serve.Request(3, "3d_a", 0.0, slot=1), serve.Request(4, "3d_a", 0.0, slot=0)]
    for r in mix:
        srv.submit(r)
    assert srv.step() == 4
    h_mix = srv.inflight[0][0]
    srv.collect(wait=True)
    in_mix = h_mix[1][2].cpu().numpy()
    assert np.array_equal(alone, in_mix)
    # and against the oracle
    r = ex.pools["3d_a"][1].double().cpu().numpy()
    n_el, p = (10, 12, 8), 3
    vel = [taylor_hood_velocity_1d(n, p) for n in n_el]
    facs = [FDFactors([v[0] for v in vel], [v[1] for v in vel], velocity_weights(3, k)) for k in range(3)]
    zo = block_apply(facs, [pressure_1d(n, p) for n in n_el], r)
    pc = srv.cache.entries["3d_a"][0]
    tol = 1e-12 if prec == "f64" else 2e-2
    for a, b in zip(pc.offsets[:-1], pc.offsets[1:]):
        assert np.linalg.norm(alone[a:b] - zo[a:b]) / np.linalg.norm(zo[a:b]) < tol


def test_poisson_stream_completes():
    _case("serving: short Poisson stream, prec=f32")
    from paper_1712_00403_amd import serve
    classes = _classes("f32")
    t0 = time.perf_counter()
    ex = serve.GpuExecutor(classes, slots=2, seed=4, t0=t0)
    srv = serve.Server(classes, ex, hbm_budget=1 << 30)
    arrivals = serve.poisson_arrivals(400.0, 0.5, {"2d": 0.6, "3d_a": 0.3, "3d_b": 0.1}, seed=4)
    reqs = serve.run_stream(srv, arrivals, lambda: time.perf_counter() - t0, {k: 2 for k in classes})
    assert len(reqs) == len(arrivals) and all(r.done is not None for r in reqs)
    s = serve.latency_summary(reqs, 0.5)
    print(f"  {s['requests']} requests, p50 {s['p50_ms']:.3f} ms, p99 {s['p99_ms']:.3f} ms, steps {srv.steps}")
    assert s["p50_ms"] > 0 and s["p99_ms"] >= s["p50_ms"]
    assert srv.steps <= len(arrivals)
