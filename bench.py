"""Benchmark: block FD preconditioner applies on the 3D 64^3, p = 3 Taylor-Hood patch.

One step = z = P_D^{-1} r for 16 synthetic Gaussian residual block vectors
(3 velocity blocks of 129^3 and the 67^3 pressure block each, 6,740,830 DOFs
per residual), every pass of Algorithm 1 on the GPU, inputs resident in HBM.

The headline `value` is the FP64 path (the paper's precision). The same
workload is also timed in FP32, BF16 and BF16-split (the precision ladder),
each with its relative error against the FP64 oracle on residual 0. The
oracle itself is timed on the host cores as `cpu_baseline`.

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
# sources the dominant kernel is built from: HBM traffic counters recorded in
# profiles/ count only while these files are unchanged
KERNEL_SOURCES = ["fd_pass3.inc", "fd_pass2.inc", "fd_pass.inc", "fd_internal.h", "fd_pass_f64.hip", "fd_pass_f32.hip"]
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
    ap.add_argument("--serve-seconds", type=float, default=8.0, help="length of each serving run (0 to skip)")
    ap.add_argument("--serve", default="f64,bf16", help="precisions of the serving runs")
    ap.add_argument("--serve-only", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the residuals and blocks are independent: a multi-GPU run would shard them "
              "with no communication)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1712_00403_amd import fd, workloads
    from paper_1712_00403_amd.precond import BlockPreconditioner

    if args.batch_only:
        torch.cuda.set_device(0)
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
    log(f"block size {N}, {nrhs} residuals, seed {seed}")
    r_host = workloads.residuals(seed, nrhs, N)
    flops_apply = algorithmic_flops(sizes)

    results = {}
    z0 = {}
    stream = torch.cuda.current_stream()
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
        z0[p] = z[0].double().cpu().numpy()
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
        results[p] = {"dominant_ms": dom_ms, "launches": launches,"ms_per_step": ms, "applies_per_s": applies, "dof_per_s": applies * N,
                      "tflops": flops_apply * applies / 1e12,
                      "stage_ms": {k: v[0] / max(v[1], 1) for k, v in stages.items()}}
        log(f"{p}: {ms:.3f} ms/step, {applies:.1f} applies/s, {results[p]['tflops']:.2f} TFLOP/s")
        del r, z
        torch.cuda.empty_cache()

    # relative error of residual 0 against the FP64 oracle, per block
    log("oracle check of residual 0")
    from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
    from oracle.fd import FDFactors, block_apply, velocity_weights
    t0 = time.perf_counter()
    Kv, Mv = taylor_hood_velocity_1d(64, 3)
    facs = [FDFactors([Kv] * 3, [Mv] * 3, velocity_weights(3, k)) for k in range(3)]
    Mp = [pressure_1d(64, 3)] * 3
    oracle_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    zo = block_apply(facs, Mp, r_host[0])
    t_first = time.perf_counter() - t0
    offs = ref.offsets
    for p in precisions:
        errs = [float(np.linalg.norm(z0[p][a:b] - zo[a:b]) / np.linalg.norm(zo[a:b]))
                for a, b in zip(offs[:-1], offs[1:])]
        results[p]["rel_err_blocks"] = errs
        results[p]["rel_err_max"] = max(errs)

    cpu = None
    if not args.no_cpu:
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
        done, t_cpu = 1, t_first
        while done < nrhs and t_cpu < args.cpu_seconds:
            t0 = time.perf_counter()
            block_apply(facs, Mp, r_host[done])
            t_cpu += time.perf_counter() - t0
            done += 1
        cpu = {"value": done / t_cpu, "unit": "applies/s", "cores": int(threads), "kind": "oracle",
               "sample": f"{done} of the {nrhs} residuals of one step (full 64^3 p=3 block apply each, "
                         f"numpy FP64, steps 2-4 of Algorithm 1 plus banded pressure solves; "
                         f"oracle setup {oracle_setup:.1f} s excluded)"}

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
                "kernel": f"fd_pass3_kernel<{'0,9,2,true' if head_prec == 'f64' else '1,9,2,true'}> (fused last-mode pass, "
                          "velocity blocks 129^3 x 3 x 16 residuals)",
                "algorithmic_gflop_per_launch": dom_flops / 1e9, "avg_launch_ms": dom_ms,
                "algorithmic_bytes_per_launch": nrhs * 3 * 129 ** 3 * (16 if head_prec == "f64" else 8),
                "kernel_source_hash": kernel_source_hash()}

    ladder = {p: {"applies_per_s": round(v["applies_per_s"], 2), "dof_per_s": v["dof_per_s"],
                  "ms_per_step": round(v["ms_per_step"], 4), "tflops": round(v["tflops"], 2),
                  "frac_of_peak": v["tflops"] * 1e12 / PEAKS[p],
                  "rel_err_max": v["rel_err_max"], "rel_err_blocks": v["rel_err_blocks"],
                  "speedup_vs_f64": (v["applies_per_s"] / results["f64"]["applies_per_s"]
                                     if "f64" in results else None),
                  "stage_ms": {k: round(x, 4) for k, x in v["stage_ms"].items()},
                  "dominant_kernel_ms": round(v["dominant_ms"], 4)}
              for p, v in results.items()}
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
           "dof_per_s": head["dof_per_s"], "rel_err_vs_oracle": head["rel_err_max"],
           "plan_setup_s": round(setup_s, 3), "roofline": roofline, "cpu_baseline": cpu,
           "ladder": ladder, "batch_256_patches": batch, "serving": serving}
    print(json.dumps(out))
    for pc in pcs.values():
        pc.close()


def bench_batch(args, precisions):
    """256 heterogeneous 3D patches (coefficient-aware blocks) in one persistent launch per apply.

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
    with ThreadPoolExecutor(max_workers=4) as ex:
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
        # algorithmic bytes: every pass reads and writes the block once; the
        # scaled blocks read D^{-1/2} twice
        byts = sum(5 * 2 * N * eb + 2 * N * eb for N in [p.N for pc in pcs for p in pc.plans])
        out["precisions"][prec] = {"ms_per_apply": round(ms, 4), "dof_per_s": dofs / (ms * 1e-3),
                                   "patch_applies_per_s": len(pcs) / (ms * 1e-3),
                                   "algorithmic_gb_per_s": byts / (ms * 1e-3) / 1e9,
                                   "ms_per_apply_grouped_launches": round(ms_grouped, 4),
                                   "launches_per_apply": 1, "tiles": info["tiles"], "grid": info["grid"],
                                   "tuned_config": config, "dofs": dofs, "blocks": passes}
        log(f"batch {prec}: {ms:.3f} ms/apply (one launch; grouped launches {ms_grouped:.3f} ms), "
            f"{dofs / (ms * 1e-3) / 1e9:.2f} GDOF/s")
        # oracle check of the three smallest patches
        from oracle.fd import FDFactors, block_apply
        from oracle.geometry import GeometryBlocks
        small = sorted(range(len(pcs)), key=lambda i: sizes[i])[:3]
        errs = []
        zh = Z.double().cpu().numpy()
        for i in small:
            n_el, p = patches[i]
            gb = GeometryBlocks(n_el, p, geo)
            facs = [FDFactors(gb.vel_K[k], gb.vel_M[k]) for k in range(3)]
            zo = block_apply(facs, gb.pres_M, res[i], pres_scale=gb.pres_scale, vel_scales=gb.vel_scales)
            zi = zh[offs[i]:offs[i + 1]]
            po = pcs[i].offsets
            errs.append(max(float(np.linalg.norm(zi[a:c] - zo[a:c]) / np.linalg.norm(zo[a:c]))
                            for a, c in zip(po[:-1], po[1:])))
        out["precisions"][prec]["rel_err_max_sampled"] = max(errs)
        out["precisions"][prec]["sampled_patches"] = [list(patches[i][0]) + [patches[i][1]] for i in small]
        b.close()
        for pc in pcs:
            pc.close()
        del R, Z
        torch.cuda.empty_cache()
    return out


def bench_serve(args, precisions):
    """Poisson stream of FD-apply requests of mixed sizes through the continuous-batching server.

    2000 requests/s (seed 4): 70% 2D 16x16 p = 2 block vectors, 25% 3D 64^3
    p = 3, 5% 3D 96^3 p = 4; residuals from a seeded device pool per class;
    factors cached on the device under an HBM budget; latency = completion
    (HIP event on the launch stream) minus arrival.
    """
    import torch

    from paper_1712_00403_amd import serve, workloads
    mix = {"2d_16_p2": 0.70, "3d_64_p3": 0.25, "3d_96_p4": 0.05}
    problems = {"2d_16_p2": lambda: workloads.taylor_hood_problem((16, 16), 2, unit_weights=True),
                "3d_64_p3": lambda: workloads.taylor_hood_problem((64, 64, 64), 3),
                "3d_96_p4": lambda: workloads.taylor_hood_problem((96, 96, 96), 4)}
    out = {"rate_per_s": 2000.0, "seconds": args.serve_seconds, "mix": mix, "precisions": {}}
    for prec in precisions:
        classes = {k: serve.RequestClass(k, f, prec) for k, f in problems.items()}
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
        # no garbage-collector pauses inside the timed stream (a serving
        # process collects between bursts)
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        ex.t0, ex.ev_ref = t0, None
        try:
            reqs = serve.run_stream(srv, arrivals, lambda: time.perf_counter() - t0, {k: 4 for k in problems})
        finally:
            gc.enable()
        summ = serve.latency_summary(reqs, args.serve_seconds)
        summ.update({"steps": srv.steps, "plan_cache_bytes": srv.cache.bytes, "evictions": srv.cache.evictions,
                     "offered_dof_per_s": sum(r.dofs for r in reqs) / args.serve_seconds})
        out["precisions"][prec] = summ
        log(f"serving {prec}: {summ['requests']} requests, p50 {summ['p50_ms']:.3f} ms, "
            f"p99 {summ['p99_ms']:.3f} ms, {summ['dof_per_s'] / 1e9:.2f} GDOF/s, {srv.steps} steps")
        for pc, _ in srv.cache.entries.values():
            pc.close()
        del ex, srv
        torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
