"""Benchmark: block FD preconditioner applies on the 3D 64^3, p = 3 Taylor-Hood patch.

One step = z = P_D^{-1} r for 16 synthetic Gaussian residual block vectors
(3 velocity blocks of 129^3 and the 67^3 pressure block each, 6,740,830 DOFs
per residual), every pass of Algorithm 1 on the GPU, inputs resident in HBM.

The headline `value` is the FP64 path (the paper's precision). The same
workload is also timed in every other precision class (the precision ladder),
each with its per-block relative errors (2-norm and element-wise) against the
FP64 oracle on every residual. The oracle itself is timed on the host cores
(all threads: `cpu_baseline`; one thread beside it).

Further legs: the 2D 16x16 p = 2 patch (microseconds per apply in FP64, 4
residuals; 64-residual batches in the reduced precisions with the
per-residual error distribution), the 256-patch coefficient-aware batch in
one persistent launch, and the Poisson serving stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--precisions f64,f32,...]
"""
import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FD applies/s & DOF/s, 3D p=3 64^3 elem; mixed vs FP64 at rel-err; p50/p99 latency"
# HBM traffic counters recorded in profiles/ count only while the library's
# sources (kernels, launch shapes, factor images) are unchanged
KERNEL_SOURCES = sorted(f for f in os.listdir(os.path.join(ROOT, "paper_1712_00403_amd", "csrc"))
                        if f.endswith((".hip", ".inc", ".h", ".cpp")))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fd_pass3_fused_64cube_p3_traffic.json")
PEAKS = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15, "bf16_split": 2.5e15, "f16": 2.5e15,
         "f16_split": 2.5e15, "fp8_split": 5.0e15}
HBM_PEAK = 8.0e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1712_00403_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(prec):
    """HBM bytes per launch of the dominant kernel from the committed counter runs, or None."""
    import json as _json
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = _json.load(fh)
    ent = rec.get(prec)
    if not ent or rec.get("source_hash") != kernel_source_hash():
        return None
    return ent["bytes_per_launch"]


def algorithmic_flops(sizes_per_block, ndim=3):
    """FLOPs of one block apply: 4 N sum_i n_i per block (Algorithm 1: 2 N n_i per mode product)."""
    return sum(4 * int(np.prod(n)) * sum(n) for n in sizes_per_block)


def stage_flops(n, stage):
    """FLOPs of one stage of the pass schedule for a 3D block of sizes n."""
    N = int(np.prod(n))
    if stage in (0, 4):
        return 2 * N * n[0]
    if stage in (1, 3):
        return 2 * N * n[1]
    return 4 * N * n[2]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precisions", default="f64,f32,bf16,f16,bf16_split,f16_split,fp8_split")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only", default=None, help="time only this precision (profiling runs)")
    ap.add_argument("--batch", default="bf16,f32",
                    help="precisions of the 256-patch persistent batch leg ('' to skip)")
    ap.add_argument("--batch-patches", type=int, default=256)
    ap.add_argument("--batch-only", action="store_true", help="run only the persistent batch leg")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of each serving run (0 to skip)")
    ap.add_argument("--serve", default="f64,bf16", help="precisions of the serving runs")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--small", default="f64,f32,bf16,f16,bf16_split,f16_split,fp8_split",
                    help="precisions of the 2D 16x16 legs ('' to skip)")
    ap.add_argument("--hbm-copy-gib", type=float, default=0.0,
                    help="first fill and copy a device buffer of this size (counter runs: the copy's FETCH_SIZE and "
                         "WRITE_SIZE readings give the bytes-per-KiB factors of the HBM traffic figures)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the residuals and blocks are independent: a multi-GPU run would shard them "
              "with no communication)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1712_00403_amd import fd, workloads
    from paper_1712_00403_amd.precond import BlockPreconditioner

    torch.cuda.set_device(0)
    if args.hbm_copy_gib > 0:
        n = int(args.hbm_copy_gib * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    if args.batch_only:
        print(json.dumps({"batch_256_patches": bench_batch(args, [p for p in args.batch.split(",") if p])}))
        return
    if args.serve_only:
        torch.cuda.set_device(0)
        print(json.dumps({"serving": bench_serve(args, [p for p in args.serve.split(",") if p])}))
        return
    cfg = workloads.CONFIGS["3d_64_p3_16rhs"]
    prob = cfg["problem"]()
    nrhs, seed = cfg["nrhs"], cfg["seed"]
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    precisions = [args.only] if args.only else args.precisions.split(",")

    log("building plans")
    t0 = time.perf_counter()
    pcs = {p: BlockPreconditioner(prob, precision=p) for p in precisions}
    setup_s = (time.perf_counter() - t0) / len(precisions)
    ref = pcs[precisions[0]]
    sizes = [(129, 129, 129)] * 3 + [(67, 67, 67)]
    assert ref.sizes == [int(np.prod(s)) for s in sizes]
    N = ref.N
    offs = ref.offsets
    log(f"block size {N}, {nrhs} residuals, seed {seed}")
    r_host = workloads.residuals(seed, nrhs, N)
    flops_apply = algorithmic_flops(sizes)

    # the oracle's block vectors of every residual (checked against every
    # precision), timed on all host threads as the CPU baseline
    zo_all, cpu = None, None
    if not args.only:
        zo_all, cpu = oracle_c2(args, r_host)

    results = {}
    for p in precisions:
        pc = pcs[p]
        dt = torch.float64 if pc.io_dtype == "float64" else torch.float32
        r = torch.from_numpy(r_host).to(dt).to(dev)
        z = torch.empty_like(r)
        for _ in range(args.warmup):
            pc.apply(r, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pc.apply(r, z)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        ms = dt_s * 1e3 / args.steps
        errs = None
        if zo_all is not None:
            zh = z.double().cpu().numpy()
            errs = block_errors(zh, zo_all, offs)
            del zh
        # per-stage kernel time, measured with HIP events on the launch stream
        fd.timing_enable(True)
        for _ in range(args.steps):
            pc.apply(r, z)
        stages = fd.timing_read()
        launches = fd.timing_launches()
        fd.timing_enable(False)
        # the dominant kernel: the launch of the fused last-mode pass that
        # covers the 129^3 velocity blocks (factor order 129)
        dom = [c for c in launches if c["stage"] == "last_mode_fused" and c["n"] == 129]
        dom_ms = dom[0]["ms"] / dom[0]["count"]
        applies = nrhs / (ms * 1e-3)
        results[p] = {"dominant_ms": dom_ms, "launches": launches, "ms_per_step": ms, "applies_per_s": applies,
                      "dof_per_s": applies * N, "tflops": flops_apply * applies / 1e12, "errors": errs,
                      "stage_ms": {k: v[0] / max(v[1], 1) for k, v in stages.items()}}
        msg = f"{p}: {ms:.3f} ms/step, {applies:.1f} applies/s, {results[p]['tflops']:.2f} TFLOP/s"
        if errs:
            msg += f", max rel err {errs['rel_err_max']:.2e}, max rel elementwise err {errs['rel_maxnorm_err_max']:.2e}"
        log(msg)
        del r, z
        torch.cuda.empty_cache()

    head = results["f64"] if "f64" in results else results[precisions[0]]
    head_prec = "f64" if "f64" in results else precisions[0]
    # dominant kernel: the fused last-mode pass over the three 129^3 velocity
    # blocks of the 16 residuals (one launch); algorithmic work 4 N n per block
    dom_flops = nrhs * 3 * 4 * 129 ** 3 * 129
    dom_ms = head["dominant_ms"]
    achieved = dom_flops / (dom_ms * 1e-3)
    peak = PEAKS[head_prec]
    traffic = recorded_traffic(head_prec)
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic,
                "kernel": ("fd_pass3_kernel<0,9,2,true>" if head_prec == "f64" else
                           "fd_pass3_kernel<1,9,2,true>" if head_prec == "f32" else
                           f"the {head_prec} class's fused pass kernel") +
                          " (fused last-mode pass, velocity blocks 129^3 x 3 x 16 residuals)",
                "algorithmic_gflop_per_launch": dom_flops / 1e9, "avg_launch_ms": dom_ms,
                "algorithmic_bytes_per_launch": nrhs * 3 * 129 ** 3 * (16 if head_prec == "f64" else 8),
                "kernel_source_hash": kernel_source_hash()}

    ladder = {}
    for p, v in results.items():
        e = v["errors"] or {}
        ladder[p] = {"applies_per_s": round(v["applies_per_s"], 2), "dof_per_s": v["dof_per_s"],
                     "ms_per_step": round(v["ms_per_step"], 4), "tflops": round(v["tflops"], 2),
                     "frac_of_peak": v["tflops"] * 1e12 / PEAKS[p],
                     "hbm_frac_of_peak": v["applies_per_s"] * N * (16 if p == "f64" else 8) / HBM_PEAK,
                     "rel_err_max": e.get("rel_err_max"), "rel_maxnorm_err_max": e.get("rel_maxnorm_err_max"),
                     "rel_err_blocks": e.get("rel_err_blocks"), "rel_maxnorm_err_blocks": e.get("rel_maxnorm_err_blocks"),
                     "speedup_vs_f64": (v["applies_per_s"] / results["f64"]["applies_per_s"]
                                        if "f64" in results else None),
                     "stage_ms": {k: round(x, 4) for k, x in v["stage_ms"].items()},
                     "dominant_kernel_ms": round(v["dominant_ms"], 4),
                     "dominant_kernel_hbm_bytes_counted": recorded_traffic(p)}
    for pc in pcs.values():
        pc.close()
    del zo_all
    pressure = None
    if not args.only:
        pressure = bench_pressure_route(args, [p for p in ("f64", "f32") if p in precisions])
    small = None
    if args.small and not args.only:
        small = bench_small(args, [p for p in args.small.split(",") if p])
    batch = None
    if args.batch and not args.only:
        batch = bench_batch(args, [p for p in args.batch.split(",") if p])
    serving = None
    if args.serve_seconds > 0 and args.serve and not args.only:
        serving = bench_serve(args, [p for p in args.serve.split(",") if p])

    out = {"metric": METRIC, "value": round(head["applies_per_s"], 3), "unit": "applies/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(head["ms_per_step"], 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": head_prec, "data": "synthetic",
           "config": {"workload": "3D unit cube 64^3 elements, Taylor-Hood p=3 (velocity degree 4, "
                                  "n_V=129, pressure n_Q=67), full block P_D^-1, 16 Gaussian residuals seed 1",
                      "global_batch": nrhs, "dofs_per_residual": N, "parallelism": "single GPU"},
           "dof_per_s": head["dof_per_s"],
           "rel_err_vs_oracle": (head["errors"] or {}).get("rel_err_max"),
           "rel_maxnorm_err_vs_oracle": (head["errors"] or {}).get("rel_maxnorm_err_max"),
           "plan_setup_s": round(setup_s, 3), "roofline": roofline, "cpu_baseline": cpu,
           "ladder": ladder, "pressure_route_67cube": pressure, "small_2d_16_p2": small, "batch_256_patches": batch, "serving": serving}
    print(json.dumps(out))


def block_errors(zh, zo_all, offs):
    """Per residual and block: relative 2-norm and relative max-norm errors against the oracle."""
    e2 = np.zeros((zh.shape[0], len(offs) - 1))
    em = np.zeros_like(e2)
    for j in range(zh.shape[0]):
        for k, (a, b) in enumerate(zip(offs[:-1], offs[1:])):
            d = zh[j, a:b] - zo_all[j][a:b]
            e2[j, k] = np.linalg.norm(d) / np.linalg.norm(zo_all[j][a:b])
            em[j, k] = np.max(np.abs(d)) / np.max(np.abs(zo_all[j][a:b]))
    return {"rel_err_max": float(e2.max()), "rel_maxnorm_err_max": float(em.max()),
            "rel_err_blocks": [float(x) for x in e2.max(axis=0)],
            "rel_maxnorm_err_blocks": [float(x) for x in em.max(axis=0)],
            "rel_err_per_residual": [float(x) for x in e2.max(axis=1)]}


def oracle_c2(args, r_host):
    """Oracle block vectors of every residual of the 64^3 p = 3 workload, and the CPU baseline timings.

    All host threads: the whole batch (also the reference values of the
    ladder). One thread: a bounded sample of residuals, beside it.
    """
    import threadpoolctl

    from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
    from oracle.fd import FDFactors, block_apply, velocity_weights
    log("oracle: setup and every residual on all host threads")
    t0 = time.perf_counter()
    Kv, Mv = taylor_hood_velocity_1d(64, 3)
    facs = [FDFactors([Kv] * 3, [Mv] * 3, velocity_weights(3, k)) for k in range(3)]
    Mp = [pressure_1d(64, 3)] * 3
    oracle_setup = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    t0 = time.perf_counter()
    zo_all = [block_apply(facs, Mp, r_host[j]) for j in range(r_host.shape[0])]
    t_all = time.perf_counter() - t0
    cpu = None
    if not args.no_cpu:
        cpu = {"value": r_host.shape[0] / t_all, "unit": "applies/s", "cores": int(threads), "kind": "oracle",
               "sample": f"all {r_host.shape[0]} residuals of one step (full 64^3 p=3 block apply each, numpy FP64, "
                         f"steps 2-4 of Algorithm 1 plus banded pressure solves; oracle setup "
                         f"{oracle_setup:.1f} s excluded)", "cpu": cpu_model()}
        done, t1 = 0, 0.0
        with threadpoolctl.threadpool_limits(1):
            while done < r_host.shape[0] and t1 < args.cpu_seconds:
                t0 = time.perf_counter()
                block_apply(facs, Mp, r_host[done])
                t1 += time.perf_counter() - t0
                done += 1
        cpu["one_thread"] = {"value": done / t1, "unit": "applies/s", "cores": 1,
                             "sample": f"{done} residuals, BLAS limited to one thread"}
        log(f"oracle: {cpu['value']:.2f} applies/s on {threads} threads, {cpu['one_thread']['value']:.3f} on one")
    return zo_all, cpu


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_pressure_route(args, precisions):
    """The 67^3 pressure block of the 64^3 p = 3 patch, 16 residuals: FD form (Lambda = I) vs banded solves.

    The FD form runs five mode products per apply on the MFMA kernels; the
    banded route (Sec. 5.2) one banded Cholesky solve per mode. Milliseconds
    per 16-residual apply (HIP events on the launch stream), and the relative
    difference of the two results.
    """
    import torch

    from oracle.assemble import pressure_1d
    from paper_1712_00403_amd import fd, workloads
    Ms = [pressure_1d(64, 3)] * 3
    out = {}
    for prec in precisions:
        plans = {"fd_form": fd.Plan(None, Ms, precision=prec), "banded": fd.Plan(None, Ms, precision=prec, banded=True)}
        dt = torch.float64 if prec == "f64" else torch.float32
        N = plans["banded"].N
        r = torch.from_numpy(workloads.residuals(5, 16, N)).to(dt).cuda()
        res, zs = {}, {}
        for name, plan in plans.items():
            z = torch.empty_like(r)
            for _ in range(args.warmup):
                plan.apply(r, z)
            torch.cuda.synchronize()
            fd.timing_enable(True)
            for _ in range(args.steps):
                plan.apply(r, z)
            stages = fd.timing_read()
            fd.timing_enable(False)
            ms = sum(v[0] for v in stages.values()) / args.steps
            res[name] = {"ms_per_apply": round(ms, 4),
                         "all_passes_gb_per_s": 16 * N * 2 * r.element_size() * (5 if name == "fd_form" else 3)
                         / (ms * 1e-3) / 1e9}
            zs[name] = z
        d = (zs["banded"] - zs["fd_form"]).double()
        res["rel_diff"] = float(d.norm() / zs["fd_form"].double().norm())
        res["speedup_banded"] = res["fd_form"]["ms_per_apply"] / res["banded"]["ms_per_apply"]
        out[prec] = res
        log(f"pressure 67^3 x 16 {prec}: FD form {res['fd_form']['ms_per_apply']:.3f} ms, banded "
            f"{res['banded']['ms_per_apply']:.3f} ms, rel diff {res['rel_diff']:.1e}")
        for plan in plans.values():
            plan.close()
    return out


def bench_small(args, precisions):
    """The 2D 16x16, p = 2 Taylor-Hood patch (n_V = 32, n_Q = 18): launch-latency bound.

    FP64 with 4 residuals (seed 0): microseconds per step and per residual
    apply. Every precision with 64 residuals (seed 2): microseconds per
    64-residual batch, and the distribution over residuals of the largest
    per-block relative error against the oracle.
    """
    import torch

    from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
    from oracle.fd import FDFactors, block_apply
    from paper_1712_00403_amd import workloads
    from paper_1712_00403_amd.precond import BlockPreconditioner
    Kv, Mv = taylor_hood_velocity_1d(16, 2)
    facs = [FDFactors([Kv] * 2, [Mv] * 2) for _ in range(2)]
    Mp = [pressure_1d(16, 2)] * 2
    out = {"workload": "2D unit square 16x16 elements, Taylor-Hood p=2 (n_V=32, n_Q=18), unit-weight velocity "
                       "blocks, 2372 DOFs per block vector", "legs": {}}
    reps = max(args.steps, 10) * 20
    for name, key, precs in (("fp64_4rhs", "2d_16_p2_4rhs", ["f64"]), ("ladder_64rhs", "2d_16_p2_64rhs", precisions)):
        cfg = workloads.CONFIGS[key]
        prob = cfg["problem"]()
        leg = {"nrhs": cfg["nrhs"], "seed": cfg["seed"], "precisions": {}}
        for p in precs:
            pc = BlockPreconditioner(prob, precision=p)
            r_host = workloads.residuals(cfg["seed"], cfg["nrhs"], pc.N)
            zo = [block_apply(facs, Mp, r_host[j]) for j in range(cfg["nrhs"])]
            dt = torch.float64 if pc.io_dtype == "float64" else torch.float32
            r = torch.from_numpy(r_host).to(dt).cuda()
            z = torch.empty_like(r)
            for _ in range(args.warmup * 10):
                pc.apply(r, z)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                pc.apply(r, z)
            torch.cuda.synchronize()
            us = (time.perf_counter() - t0) * 1e6 / reps
            # the same apply recorded once as a HIP graph and replayed
            g = pc.graph(r, z)
            for _ in range(args.warmup * 10):
                g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                g.replay()
            torch.cuda.synchronize()
            us_graph = (time.perf_counter() - t0) * 1e6 / reps
            del g
            # the same works as one fixed batch (one persistent launch, or the
            # staged route), where the class has one (FP8 split has none)
            from paper_1712_00403_amd import fd as _fd
            us_batch, bt_cfg = None, None
            try:
                bt = _fd.Batch(pc.works(r.data_ptr(), z.data_ptr(), cfg["nrhs"]))
            except _fd.FDError:
                bt = None
            if bt is not None:
                bt_cfg = bt.tune(reps=20)
                for _ in range(args.warmup * 10):
                    bt.apply()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    bt.apply()
                torch.cuda.synchronize()
                us_batch = (time.perf_counter() - t0) * 1e6 / reps
                bt.check()
                bt.close()
            e = block_errors(z.double().cpu().numpy(), zo, pc.offsets)
            per = np.array(e["rel_err_per_residual"])
            leg["precisions"][p] = {"us_per_step": round(us, 2), "us_per_residual_apply": round(us / cfg["nrhs"], 3),
                                    "us_per_step_graph_replay": round(us_graph, 2),
                                    "us_per_step_fixed_batch": None if us_batch is None else round(us_batch, 2),
                                    "fixed_batch_config": bt_cfg,
                                    "rel_err_max": e["rel_err_max"], "rel_maxnorm_err_max": e["rel_maxnorm_err_max"],
                                    "rel_err_per_residual_quantiles": {
                                        "min": float(per.min()), "p50": float(np.median(per)),
                                        "p90": float(np.percentile(per, 90)), "max": float(per.max())}}
            fb = "no fixed batch" if us_batch is None else f"{us_batch:.1f} us as a fixed batch"
            log(f"2D 16^2 {name} {p}: {us:.1f} us per {cfg['nrhs']}-residual step ({us_graph:.1f} us as a graph "
                f"replay, {fb}), rel err max {e['rel_err_max']:.2e}")
            pc.close()
        out["legs"][name] = leg
    return out


def bench_batch(args, precisions):
    """256 heterogeneous 3D patches (coefficient-aware blocks) as one fixed batch (fd_batch).

    The batch is tuned (persistent body choices per stage, and for BF16/FP16
    the staged route) and the chosen route is timed.

    Patches: n_el per direction uniform in [8, 48], p uniform in {2..5}
    (workloads.batch_patches, seed 3); geometry G(eta)_j = eta_j + 0.1 sin(pi
    eta_j) with nu(x) = 1 + 0.5 sin(2 pi x_1) cos(2 pi x_2); one Gaussian
    residual per patch. The host setup (coefficients, separable fits,
    factors, diagonals) is untimed.
    """
    import ctypes
    from concurrent.futures import ThreadPoolExecutor

    import torch

    from paper_1712_00403_amd import fd, workloads
    from paper_1712_00403_amd.geometry import GeometryPreconditioner, geometry_blocks

    # keep freed host buffers in the heap: the setup allocates and frees large
    # arrays per patch, and returning them to the kernel costs page faults
    try:
        libc = ctypes.CDLL("libc.so.6")
        libc.mallopt(-3, 1 << 30)   # M_MMAP_THRESHOLD
        libc.mallopt(-1, 2 ** 31 - 1)  # M_TRIM_THRESHOLD
    except OSError:
        pass
    patches, rng = workloads.batch_patches(args.batch_patches, seed=3)
    geo = workloads.sine_geometry(3)
    probs = [workloads.taylor_hood_problem(n_el, p, unit_weights=True) for n_el, p in patches]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=16) as ex:
        blocks = list(ex.map(lambda pr: geometry_blocks(pr, geo), probs))
    setup_s = time.perf_counter() - t0
    log(f"batch: host setup of {len(probs)} patches {setup_s:.1f} s")
    out = {"patches": len(probs), "host_setup_s": round(setup_s, 1), "geometry": "sine map 0.1, wavy viscosity",
           "precisions": {}}
    sizes = None
    for prec in precisions:
        pcs = [GeometryPreconditioner(pr, geo, precision=prec, blocks=b) for pr, b in zip(probs, blocks)]
        if sizes is None:
            sizes = [pc.N for pc in pcs]
            res = workloads.batch_residuals(rng, sizes)
        dt = torch.float64 if prec == "f64" else torch.float32
        offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        R = torch.empty(int(offs[-1]), dtype=dt, device="cuda")
        for i, r in enumerate(res):
            R[offs[i]:offs[i + 1]] = torch.from_numpy(r).to(dt)
        Z = torch.empty_like(R)
        eb = R.element_size()
        works = []
        for i, pc in enumerate(pcs):
            works += pc.works(R.data_ptr() + int(offs[i]) * eb, Z.data_ptr() + int(offs[i]) * eb, 1)
        b = fd.Batch(works)
        config = b.tune(reps=2)
        info = b.info()
        for _ in range(args.warmup):
            b.apply()
        b.check()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.apply()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        b.check()
        Zp = Z.double().cpu().numpy()   # the persistent launch's result, checked below
        # the same works through per-stage grouped launches, for comparison
        for _ in range(args.warmup):
            fd.apply_batched(works)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fd.apply_batched(works)
        torch.cuda.synchronize()
        ms_grouped = (time.perf_counter() - t0) * 1e3 / args.steps
        dofs = int(offs[-1])
        passes = sum(len(pc.problem.blocks) for pc in pcs)
        # algorithmic bytes of one apply: every block read once and written
        # once, and its D^{-1/2} read twice (before the first and after the
        # last product); what the five passes move is reported beside it
        alg_bytes = dofs * (2 * eb + 2 * eb)
        pass_bytes = 5 * 2 * dofs * eb + 2 * dofs * eb
        out["precisions"][prec] = {"ms_per_apply": round(ms, 4), "dof_per_s": dofs / (ms * 1e-3),
                                   "patch_applies_per_s": len(pcs) / (ms * 1e-3),
                                   "algorithmic_gb_per_apply": alg_bytes / 1e9,
                                   "algorithmic_gb_per_s": alg_bytes / (ms * 1e-3) / 1e9,
                                   "hbm_frac_of_peak": alg_bytes / (ms * 1e-3) / HBM_PEAK,
                                   "five_pass_gb_per_s": pass_bytes / (ms * 1e-3) / 1e9,
                                   "hbm_bytes_per_apply_counted": recorded_traffic(f"batch_{prec}"),
                                   "ms_per_apply_grouped_launches": round(ms_grouped, 4),
                                   "route": ("staged: one launch per stage and row-tile group (slab passes, "
                                             "16-bit fused pass)" if config == fd.Batch.STAGED else
                                             "persistent: one launch, grid barriers between stages"),
                                   "tiles": info["tiles"], "grid": info["grid"],
                                   "tuned_config": config, "dofs": dofs, "blocks": passes}
        log(f"batch {prec}: {ms:.3f} ms/apply (config {config}; grouped launches {ms_grouped:.3f} ms), "
            f"{dofs / (ms * 1e-3) / 1e9:.2f} GDOF/s, {alg_bytes / (ms * 1e-3) / 1e9:.0f} GB/s algorithmic")
        # oracle values at sampled pencils of the 8 largest and 8 drawn patches
        # (computed by tests/golden/make_batch_golden.py from the oracle alone)
        out["precisions"][prec].update(batch_sample_errors(Zp, offs, pcs, patches, prec))
        del Zp
        b.close()
        for pc in pcs:
            pc.close()
        del R, Z
        torch.cuda.empty_cache()
    return out


def batch_sample_errors(Zh, offs, pcs, patches, prec):
    """Sampled relative errors (RMS and element-wise) of the checked patches against the stored oracle values."""
    gdir = os.path.join(ROOT, "tests", "golden")
    path = os.path.join(gdir, "batch_256_sampled.npz")
    if not os.path.exists(path) or len(pcs) != 256:
        return {"rel_err_max_sampled": None}
    golden = dict(np.load(path))
    e2m, emm, checked = 0.0, 0.0, []
    for i in golden["patches"]:
        zi = Zh[offs[i]:offs[i + 1]]
        po = pcs[i].offsets
        for b in range(len(po) - 1):
            zb = zi[po[b]:po[b + 1]]
            d = zb[golden[f"p{i}_b{b}_idx"]] - golden[f"p{i}_b{b}_val"]
            e2m = max(e2m, float(np.sqrt(np.mean(d * d)) / golden[f"p{i}_b{b}_rms"]))
            emm = max(emm, float(np.max(np.abs(d)) / golden[f"p{i}_b{b}_max"]))
        checked.append(list(patches[int(i)][0]) + [patches[int(i)][1]])
    log(f"batch {prec}: sampled rel err {e2m:.2e}, rel max err {emm:.2e} over {len(checked)} patches")
    return {"rel_err_max_sampled": e2m, "rel_maxnorm_err_max_sampled": emm,
            "sampled_patches": checked,
            "sample": "8 largest and 8 drawn patches, whole pencils per direction of every block"}


def bench_serve(args, precisions):
    """Poisson stream of FD-apply requests of mixed sizes through the continuous-batching server.

    2000 requests/s (seed 4): 70% 2D 16x16 p = 2 block vectors, 25% 3D 64^3
    p = 3, 5% 3D 96^3 p = 4, each class in a lane (HIP stream) of its own;
    residuals from a seeded device pool per class; factors cached on the
    device under an HBM budget; latency = completion (HIP event on the lane's
    stream) minus arrival. The garbage collector stays on; the objects alive
    before the stream are frozen out of its generations. The first request of
    every class is compared with the oracle.
    """
    import torch

    from paper_1712_00403_amd import serve, workloads
    mix = {"2d_16_p2": 0.70, "3d_64_p3": 0.25, "3d_96_p4": 0.05}
    shapes = {"2d_16_p2": ((16, 16), 2, True), "3d_64_p3": ((64, 64, 64), 3, False),
              "3d_96_p4": ((96, 96, 96), 4, False)}
    problems = {k: (lambda v=v: workloads.taylor_hood_problem(v[0], v[1], unit_weights=v[2]))
                for k, v in shapes.items()}
    out = {"rate_per_s": 2000.0, "seconds": args.serve_seconds, "mix": mix, "lanes": "one HIP stream per class",
           "gc": "enabled; objects alive before the stream frozen (gc.freeze)", "precisions": {}}
    oracle_cache = {}
    for prec in precisions:
        classes = {k: serve.RequestClass(k, f, prec, lane) for lane, (k, f) in enumerate(problems.items())}
        arrivals = serve.poisson_arrivals(2000.0, args.serve_seconds, mix, seed=4)
        ex = serve.GpuExecutor(classes, slots=4, seed=4)
        srv = serve.Server(classes, ex, hbm_budget=16 << 30)
        # warm the plan cache and the kernels (untimed)
        warm = [serve.Request(-1 - i, k, 0.0) for i, k in enumerate(problems)]
        for r in warm:
            srv.submit(r)
        while srv.pending or srv.inflight:
            srv.step()
            srv.collect(wait=True)
        torch.cuda.synchronize()
        keep = {}
        for i, (_, c) in enumerate(arrivals):
            if c not in keep.values():
                keep[i] = c
        gc.collect()
        gc.freeze()
        t0 = time.perf_counter()
        ex.t0, ex.ev_ref = t0, None
        try:
            reqs = serve.run_stream(srv, arrivals, lambda: time.perf_counter() - t0, {k: 4 for k in problems},
                                    keep=keep)
        finally:
            gc.unfreeze()
        summ = serve.latency_summary(reqs, args.serve_seconds)
        summ.update({"steps": srv.steps, "plan_cache_bytes": srv.cache.bytes, "evictions": srv.cache.evictions,
                     "offered_dof_per_s": sum(r.dofs for r in reqs) / args.serve_seconds})
        log(f"serving {prec}: {summ['requests']} requests, p50 {summ['p50_ms']:.3f} ms, "
            f"p99 {summ['p99_ms']:.3f} ms, {summ['dof_per_s'] / 1e9:.2f} GDOF/s, {srv.steps} steps")
        summ["checked_requests"] = served_errors(ex, srv, classes, reqs, keep, shapes, oracle_cache)
        out["precisions"][prec] = summ
        for entry, _ in srv.cache.entries.values():
            entry.close()
        del ex, srv
        torch.cuda.empty_cache()
    return out


def served_errors(ex, srv, classes, reqs, keep, shapes, cache):
    """Per kept request: largest per-block relative errors (2-norm, element-wise) against the oracle."""
    from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
    from oracle.fd import FDFactors, block_apply, velocity_weights
    out = {}
    for rid, c in keep.items():
        n_el, p, unit = shapes[c]
        slot = reqs[rid].slot
        entry = srv.cache.entries[c][0]
        if (c, slot) not in cache:
            d = len(n_el)
            Kv, Mv = taylor_hood_velocity_1d(n_el[0], p)
            facs = [FDFactors([Kv] * d, [Mv] * d, np.ones(d) if unit else velocity_weights(d, k)) for k in range(d)]
            r = ex.pool_residuals(classes[c], entry.N)[slot]
            cache[(c, slot)] = block_apply(facs, [pressure_1d(n_el[0], p)] * d, r)
        zo = cache[(c, slot)]
        z = ex.kept[rid].double().cpu().numpy()
        e = block_errors(z[None, :], [zo], entry.pc.offsets)
        out[c] = {"request": rid, "rel_err_max": e["rel_err_max"], "rel_maxnorm_err_max": e["rel_maxnorm_err_max"]}
        log(f"  served {c} request {rid}: rel err {e['rel_err_max']:.2e}, rel max err {e['rel_maxnorm_err_max']:.2e}")
    return out


if __name__ == "__main__":
    main()
