"""Benchmark: Laplace-solve throughput of the spectral element free-surface
solver on one MI355X.

Workload (default): the 64x4-quad, P=6, periodic stream-function wave tank
(kh = 1, H/L = 90% of the limiting steepness, exact stream-function wave of
20 Fourier modes with a seeded crest position, over-integration at Pf = 9,
0.5% filter on the last two modes), advanced by RK4 steps; every step runs the whole hot path (gradient recovery,
coefficient update, Laplace GMRES solves, vertical-velocity projection,
over-integrated right-hand side, RK4 update, filter) with inputs resident in
HBM.  A step is one RK4 step.

value = Laplace-solve GDOF/s = sum over solves of n_free / sum of solve times.

Prints one JSON line.  --gpus above 1 exits: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_stiff_mfma_stream_series_64x4_P6.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1512_02548_amd", "csrc", "kernels_mfma.hip")


def measured_traffic():
    """HBM bytes per launch of the stiffness kernel from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's reading),
    or None when the kernel source has changed since it was taken."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if kv.get("source_sha256") != sha:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def stiffness_bytes_per_elem(P, word=8, gword=None):
    """Algorithmic HBM bytes of one matrix-free stiffness application per
    element: the geometric-factor stream (3 values per node, gword bytes
    each) plus reading and writing each degree of freedom once (P^2/2 owned
    nodes per element, word bytes each)."""
    Np = (P + 1) * (P + 2) // 2
    gword = word if gword is None else gword
    return 3 * Np * gword + 2 * (P * P / 2.0) * word


def stiffness_flops_per_elem(P):
    Np = (P + 1) * (P + 2) // 2
    return 8 * Np * Np + 6 * Np


def cpu_baseline(spec, budget_s=15.0, threads=1):
    """The oracle (element matrices -> CSR -> sparse LU) timed on the host for
    a bounded sample of the same workload's Laplace solves."""
    from threadpoolctl import threadpool_limits

    from oracle import laplace as olap
    from oracle import surface as osrf
    from oracle.mesh import Mesh as OMesh
    from paper_1512_02548_amd import workloads as wl

    with threadpool_limits(limits=threads):
        om = OMesh(spec.nx, spec.nz, spec.P, spec.length, spec.periodic)
        eta, phi, h, hx = wl.stream_series_state(om.xs_surf, spec)
        s1 = osrf.Surface1D(om)
        etax = s1.recover_dx(eta)
        t0 = time.perf_counter()
        count = 0
        while True:
            olap.laplace_solve(om, eta, etax, phi, h, hx)
            count += 1
            el = time.perf_counter() - t0
            if el > budget_s or count >= 200:
                break
    nfree = om.n - om.ns
    return dict(value=nfree * count / el / 1e9, unit="GDOF/s", cores=threads, kind="oracle",
                sample=f"{count} Laplace solves (assembly + sparse LU) of the initial state, "
                       f"{nfree} free DOF each, {el:.1f} s, BLAS limited to {threads} thread(s); "
                       "SciPy's sparse LU itself runs on one thread")


def large_tank(lib, wl, torch, reps=3, inner_rtol=None):
    """The 2048x8, P=6 walled tank over a trapezoidal bar with irregular
    waves: one Laplace solve of its initial state to rtol 1e-10 in FP64 and
    with FP32 / bfloat16-factor inner solves inside FP64 refinement, plus the
    stiffness apply at this size (HBM-sized factors)."""
    spec = wl.bar_irregular_spec()
    ns = spec.ns
    probe = lib.mesh_from_spec(spec, np.ones(ns), np.zeros(ns), bind=False)
    eta0, phi0, h, hx = wl.bar_irregular_state(probe.surface_x(), spec)
    m = lib.mesh_from_spec(spec, h, hx)
    dev = torch.device("cuda:0")
    eta = torch.tensor(eta0, device=dev)
    phis = torch.tensor(phi0, device=dev)
    etax = torch.zeros_like(eta)
    m.gradient_recover(lib.SEM_RECOVER_DX, eta, None, etax)
    out = {"workload": spec.name, "n_free": int(m.info.n_free), "elements": int(m.info.n_elem), "rtol": 1e-10}
    ref = None
    # inner tolerances: FP32 inner solves reach 1e-5 (two refinements to
    # 1e-10); inner solves with bfloat16 factors cannot go much below the
    # factors' rounding, so they stop at 1e-2 (measured best of 1e-2..1e-5)
    inner = {lib.SEM_PREC_FP32_IR: 1e-5, lib.SEM_PREC_BF16_IR: 1e-2}
    for name, prec in (("fp64", lib.SEM_PREC_FP64), ("fp32_ir", lib.SEM_PREC_FP32_IR),
                       ("bf16_ir", lib.SEM_PREC_BF16_IR)):
        o = lib.default_opts(rtol=1e-10, max_iter=20000, prec=prec,
                             inner_rtol=inner_rtol if inner_rtol else inner.get(prec, 1e-4))
        phi = torch.zeros(m.n, dtype=torch.float64, device=dev)
        best, st = None, None
        for _ in range(reps):
            phi.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = m.laplace_solve(eta, etax, phis, phi, o)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        if ref is None:
            ref = phi.clone()
        dev_rel = float((phi - ref).abs().max() / ref.abs().max())
        out[name] = {"gdof_s": m.info.n_free / best / 1e9, "solve_ms": best * 1e3, "iters": st["iters"],
                     "refinements": st["refinements"], "rel_residual": st["rel_residual"],
                     "max_rel_diff_vs_fp64": dev_rel}
    u = torch.randn(m.n, dtype=torch.float64, device=dev)
    y = torch.empty_like(u)
    E = m.info.n_elem
    for name, prec, word, dt in (("fp64", 0, 8, torch.float64), ("fp32", 1, 4, torch.float32),
                                 ("bf16_factors", 2, None, torch.float32)):
        uu = u.to(dt)
        yy = torch.empty_like(uu)
        ms = m.apply_timed(lib.SEM_OP_STIFFNESS, uu, yy, 200, prec)
        if word is None:
            b = stiffness_bytes_per_elem(spec.P, 4, gword=2) * E
        else:
            b = stiffness_bytes_per_elem(spec.P, word) * E
        out.setdefault("stiffness", {})[name] = {"mean_launch_ms": ms, "bytes_per_launch": b,
                                                 "achieved_gbs": b / (ms * 1e-3) / 1e9,
                                                 "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    # time stepping from the snapshot (FP64, rtol 1e-10): the stage solves of
    # a few RK4 steps, the later ones started by the stage predictor
    eta_s, phi_s = eta.clone(), phis.clone()
    ws = torch.zeros(m.n, dtype=torch.float64, device=dev)
    o = lib.default_opts(rtol=1e-10, max_iter=20000, warm_start=1)
    steps, t_step, t_solve, its = 8, [], 0.0, []
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = m.rk4_step(eta_s, phi_s, ws, spec.dt, o)
        torch.cuda.synchronize()
        t_step.append(time.perf_counter() - t0)
        if k >= steps // 2:
            t_solve += sum(x["seconds"] for x in st)
            its += [x["iters"] for x in st]
    tail = t_step[steps // 2:]
    out["rk4"] = {"steps": steps, "dt": spec.dt, "ms_per_step_last_half": 1e3 * sum(tail) / len(tail),
                  "mean_iters_per_solve_last_half": float(np.mean(its)),
                  "solve_gdof_s_last_half": m.info.n_free * len(its) / t_solve / 1e9,
                  "ms_first_step": 1e3 * t_step[0]}
    return out


def build_meshes(lib, specs, state_fn, threads=8, tiles=None):
    """Host-side mesh construction in parallel (the C calls release the GIL),
    then device binding; returns meshes and device states.  tiles: an
    autotuner table ((P, nz) -> stiffness tiles per workgroup) or None."""
    import torch
    from concurrent.futures import ThreadPoolExecutor

    from paper_1512_02548_amd import tune

    def probe(spec):
        return lib.mesh_from_spec(spec, np.ones(spec.ns), np.zeros(spec.ns), bind=False,
                                  tiles_per_block=tune.tiles_for(tiles, spec))

    with ThreadPoolExecutor(threads) as ex:
        probes = list(ex.map(probe, specs))
    states = [state_fn(p.surface_x(), sp) for p, sp in zip(probes, specs)]
    need = [i for i, (e, ph, h, hx) in enumerate(states) if not (np.all(h == 1.0) and np.all(hx == 0.0))]

    def rebuild(i):
        e, ph, h, hx = states[i]
        return lib.mesh_from_spec(specs[i], h, hx, bind=False, tiles_per_block=tune.tiles_for(tiles, specs[i]))

    with ThreadPoolExecutor(threads) as ex:
        for i, m in zip(need, ex.map(rebuild, need)):
            probes[i] = m
    dev = torch.device("cuda:0")
    out = []
    for m, (e, ph, h, hx) in zip(probes, states):
        m.bind("cuda:0")
        out.append(dict(mesh=m, eta=torch.tensor(e, device=dev), phi=torch.tensor(ph, device=dev),
                        ws=torch.zeros(m.n, dtype=torch.float64, device=dev)))
    return out


def batch_workload(args, modes=("lockstep_fp64", "lockstep_mixed", "concurrent_mixed", "sequential_fp64")):
    """256 periodic tanks of random size and order (seeded): RK4 steps of all
    tanks through the batch call with FP32 inner solves inside FP64
    refinement, against a per-tank sequential FP64 loop on the same GPU."""
    import torch

    from paper_1512_02548_amd import lib
    from paper_1512_02548_amd import workloads as wl
    from paper_1512_02548_amd import tune
    specs = wl.batch_tank_specs(count=args.tanks, rtol=1e-10)
    # element tiles of the stiffness kernel from the autotuner, per (P, nz) class
    if getattr(args, "tiles", 0):
        table = {k: args.tiles for k in tune.classes(specs)}
        trep = {"fixed": args.tiles}
    else:
        table, trep = tune.tune_batch(specs, wl.batch_tank_state)
    print(f"# autotune: {trep}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tanks = build_meshes(lib, specs, wl.batch_tank_state, tiles=table)
    t_build = time.perf_counter() - t0
    nfree = sum(int(t["mesh"].info.n_free) for t in tanks)
    dts = [sp.dt for sp in specs]
    res = {"workload": f"batch_tanks_{args.tanks}", "tanks": args.tanks, "sum_n_free": nfree,
           "host_build_s": t_build, "steps": args.batch_steps, "autotune": trep}
    save = [(t["eta"].clone(), t["phi"].clone()) for t in tanks]

    def restore():
        for t, (e, p) in zip(tanks, save):
            t["eta"].copy_(e)
            t["phi"].copy_(p)
            t["ws"].zero_()
            t["mesh"].reset_history()

    # the batched stiffness launch over every tank of an order (all live),
    # against the HBM roof: the C4 roofline
    bt = lib.Batch([t["mesh"] for t in tanks], 0)
    res["roofline_batch"] = {}
    for P in sorted({sp.P for sp in specs}):
        E = sum(2 * sp.nx * sp.nz for sp in specs if sp.P == P)
        for name, prec, word, gword in (("fp64", 0, 8, 8), ("fp32", 1, 4, 4), ("bf16_factors", 2, 4, 2)):
            ms = bt.apply_timed(P, prec, 20)
            byts = stiffness_bytes_per_elem(P, word, gword=gword) * E
            res["roofline_batch"][f"P{P}_{name}"] = {
                "bound": "hbm", "achieved": byts / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": byts, "mean_launch_ms": ms,
                "elements": E}
    del bt

    def batched(name, nstreams, opts):
        b = lib.Batch([t["mesh"] for t in tanks], nstreams)
        restore()
        b.rk4_step([t["eta"] for t in tanks], [t["phi"] for t in tanks], [t["ws"] for t in tanks], dts, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = 0
        for _ in range(args.batch_steps):
            code, st, it = b.rk4_step([t["eta"] for t in tanks], [t["phi"] for t in tanks],
                                      [t["ws"] for t in tanks], dts, opts=opts)
            if code != 0:
                raise RuntimeError(f"batch step failed: {[lib.STATUS_NAMES.get(x, x) for x in st if x]}")
            iters += sum(it)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        res[name] = {"tank_steps_per_s": args.tanks * args.batch_steps / tb,
                     "gdof_s": 4 * nfree * args.batch_steps / tb / 1e9, "seconds": tb,
                     "streams": nstreams, "mean_iters_per_solve": iters / (4 * args.tanks * args.batch_steps)}
        print(f"# {name}: {res[name]}", file=sys.stderr, flush=True)
        del b
        return tb

    fp64 = lib.default_opts(rtol=1e-10, warm_start=1, max_iter=20000)
    mixed = lib.default_opts(rtol=1e-10, warm_start=1, prec=lib.SEM_PREC_FP32_IR,
                             inner_rtol=getattr(args, "inner_rtol", 1e-5), max_iter=20000)
    tl = batched("lockstep_fp64", 0, fp64) if "lockstep_fp64" in modes else None
    if "lockstep_mixed" in modes:
        batched("lockstep_mixed", 0, mixed)
    tc = batched("concurrent_mixed", args.streams, mixed) if "concurrent_mixed" in modes else None
    if "sequential_fp64" not in modes:
        return res
    fp64 = lib.default_opts(rtol=1e-10, warm_start=1, max_iter=20000)
    restore()
    for t, dt in zip(tanks, dts):
        t["mesh"].rk4_step(t["eta"], t["phi"], t["ws"], dt, fp64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        for t, dt in zip(tanks, dts):
            t["mesh"].rk4_step(t["eta"], t["phi"], t["ws"], dt, fp64)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    res["sequential_fp64"] = {"tank_steps_per_s": args.tanks * args.batch_steps / ts,
                              "gdof_s": 4 * nfree * args.batch_steps / ts / 1e9, "seconds": ts}
    if tl:
        res["speedup_lockstep"] = ts / tl
    if tc:
        res["speedup_concurrent"] = ts / tc
    return res


def serving(args):
    """Served tank-steps/s and p50/p99 request latency: a Poisson stream of
    requests (tanks drawn like the 256-tank batch, half over a bar, exact
    stream-function waves, 200 RK4 steps each) served by continuous batching
    (lockstep batch, FP32 inner solves refined in FP64 to 1e-8) at a rate of
    `rho` times the batch's measured capacity, against a sequential server
    that runs one tank at a time in plain FP64 to the same tolerance."""
    import torch

    from paper_1512_02548_amd import lib, serve, tune
    from paper_1512_02548_amd import workloads as wl
    n, steps = args.serve_requests, args.serve_steps
    reqs = serve.make_requests(n, 1.0, steps)
    table, _ = tune.tune_batch([r.spec for r in reqs], wl.batch_tank_state)
    # capacity: tank-steps/s of the lockstep batch over the first 32 requests
    be = serve.GpuBackend(nstreams=0, tiles=table)
    tanks = [be.create(r.spec, wl.batch_tank_state) for r in reqs[:32]]
    be.step(tanks)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        be.step(tanks)
    torch.cuda.synchronize()
    cap = 3 * len(tanks) / (time.perf_counter() - t0)
    del tanks, be
    torch.cuda.empty_cache()
    rate = args.serve_rho * cap / steps
    arr = wl.poisson_arrivals(rate, n)
    out = {"requests": n, "steps_per_request": steps, "rho": args.serve_rho, "capacity_tank_steps_s": cap,
           "arrival_rate_per_s": rate, "filter": {"top_modes": 3, "sigma": 0.8}, "tolerance": 1e-8,
           "bar_fraction": 0.5}
    for mode in ("batched_mixed", "sequential_fp64"):
        rs = [serve.Request(r.rid, r.spec, float(a), steps) for r, a in zip(reqs, arr)]
        if mode == "batched_mixed":
            backend = serve.GpuBackend(nstreams=0, tiles=table)
            srv = serve.Server(backend, wl.batch_tank_state, max_slots=64)
        else:
            backend = serve.GpuBackend(nstreams=1, opts=lib.default_opts(rtol=1e-8, warm_start=1, lookahead=3))
            srv = serve.Server(backend, wl.batch_tank_state, max_slots=1)
        rep = srv.run(rs)
        rep["batch_rebuilds"] = getattr(backend, "rebuilds", None)
        out[mode] = rep
        print(f"# serving {mode}: {rep}", file=sys.stderr, flush=True)
        del srv, backend
        torch.cuda.empty_cache()
    b, s = out["batched_mixed"], out["sequential_fp64"]
    out["speedup_tank_steps"] = b["tank_steps_per_s"] / s["tank_steps_per_s"] if s["tank_steps_per_s"] else None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rtol", type=float, default=1e-12)
    ap.add_argument("--lookahead", type=int, default=1, help="Krylov steps the host queues ahead of the device")
    ap.add_argument("--predict", type=int, default=5,
                    help="past steps extrapolated into each stage solve's start vector (0..6)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-large", action="store_true", help="skip the 2048x8 bar-tank section")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-tank lockstep batch section")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--workload", choices=["stream_series", "batch"], default="stream_series",
                    help="batch: the 256-tank batching comparison (one JSON object, not the bench line)")
    ap.add_argument("--tanks", type=int, default=256)
    ap.add_argument("--batch-modes", default="lockstep_fp64,lockstep_mixed,concurrent_mixed,sequential_fp64",
                    help="comma-separated subset of the batch workload's modes")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--streams", type=int, default=8)
    ap.add_argument("--tiles", type=int, default=0, help="batch: stiffness tiles per workgroup (0: autotuner)")
    ap.add_argument("--inner-rtol", type=float, default=1e-5,
                    help="batch: relative tolerance of the FP32 inner solves of iterative refinement")
    ap.add_argument("--large-inner-rtol", type=float, default=None,
                    help="large tank: inner tolerance for both reduced precisions (default: per precision)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=200)
    ap.add_argument("--serve-rho", type=float, default=0.8, help="arrival rate as a fraction of batched capacity")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "the library runs on one GPU; runs on several GPUs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "batch":
        print(json.dumps(batch_workload(args, modes=tuple(args.batch_modes.split(",")))))
        return

    import torch

    from paper_1512_02548_amd import lib
    from paper_1512_02548_amd import workloads as wl

    dev = torch.device("cuda:0")
    spec = wl.stream_series_spec()
    ns = spec.ns
    m = lib.mesh_from_spec(spec, np.ones(ns), np.zeros(ns))
    xs = m.surface_x()
    eta0, phi0, h, hx = wl.stream_series_state(xs, spec)
    eta = torch.tensor(eta0, dtype=torch.float64, device=dev)
    phi = torch.tensor(phi0, dtype=torch.float64, device=dev)
    ws = torch.zeros(m.n, dtype=torch.float64, device=dev)
    opts = lib.default_opts(rtol=args.rtol, warm_start=1, lookahead=args.lookahead, predict=args.predict)
    n_free = m.info.n_free

    eta_init, phi_init = eta.clone(), phi.clone()
    state = {"step": 0, "onsets": []}

    def run(steps):
        # a step that fails (non-finite values or a non-positive water
        # column) leaves the state unchanged; its step number is recorded and
        # the wave restarts from the initial state
        tsolve, iters, nsolve = 0.0, 0, 0
        for _ in range(steps):
            state["step"] += 1
            code, st = m.rk4_step(eta, phi, ws, spec.dt, opts, raise_on_error=False)
            if code != lib.SEM_OK:
                state["onsets"].append((state["step"], lib.STATUS_NAMES.get(code, str(code))))
                eta.copy_(eta_init)
                phi.copy_(phi_init)
                ws.zero_()
                m.reset_history()
                continue
            for s in st:
                tsolve += s["seconds"]
                iters += s["iters"]
                nsolve += 1
        return tsolve, iters, nsolve

    run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tsolve, iters, nsolve = run(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the stiffness kernel timed live with HIP events around each of its
    # launches on the solve's stream, over further steps of the same run (the
    # event records themselves slow the steps, so they stay out of `value`)
    m.kernel_timing(True)
    run(min(args.steps, 50))
    torch.cuda.synchronize()
    nlaunch, kms = m.kernel_timing_read()
    m.kernel_timing(False)
    ms = kms / max(nlaunch, 1)

    # dominant kernel: the matrix-free stiffness apply on this tank's factors
    E = m.info.n_elem
    bytes_launch = stiffness_bytes_per_elem(spec.P) * E
    achieved = bytes_launch / (ms * 1e-3) / 1e9

    out = {
        "metric": "Laplace-solve GDOF/s",
        "value": n_free * nsolve / tsolve / 1e9,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": spec.name, "nx": spec.nx, "nz": spec.nz, "P": spec.P, "Pf": spec.Pf,
                   "n_free": int(n_free), "elements": int(E), "rtol": args.rtol, "precision": "fp64",
                   "solves": nsolve, "mean_iters": iters / max(nsolve, 1), "predict": args.predict,
                   "solve_time_fraction": tsolve / wall,
                   "initial_data": "exact stream-function wave, 20 Fourier modes",
                   "failed_steps": [list(o) for o in state["onsets"]]},
        "roofline": {"bound": "hbm", "kernel": "stiffness apply (k_stiff_mfma)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(), "mean_launch_ms": ms, "launches": nlaunch,
                     "bytes_per_launch": bytes_launch,
                     "flops_per_launch": stiffness_flops_per_elem(spec.P) * E},
    }
    if args.copy_probe:
        a = torch.empty(32 << 20, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": a.numel() * 8, "write": a.numel() * 8}
    if not args.no_large:
        out["large_tank"] = lt = large_tank(lib, wl, torch, inner_rtol=args.large_inner_rtol)
        # the same kernel at a size that streams its factors from HBM (31 MB
        # of FP64 factors and vectors per launch; 17 MB with FP32, 10 MB with
        # bfloat16 factors), timed by events around 200 launches
        out["roofline_large_tank"] = {
            k: {"bound": "hbm", "achieved": v["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": v["frac"], "bytes_per_launch": v["bytes_per_launch"], "mean_launch_ms": v["mean_launch_ms"]}
            for k, v in lt["stiffness"].items()}
    if not args.no_batch:
        # 256 tanks of mixed size and order in one lockstep batch, one RK4 step
        # each way, against the per-tank sequential FP64 loop
        del m
        torch.cuda.empty_cache()
        bargs = argparse.Namespace(tanks=256, batch_steps=1, streams=8)
        out["batch_256"] = batch_workload(bargs, modes=("lockstep_fp64", "lockstep_mixed", "sequential_fp64"))
    if not args.no_serve:
        if args.no_batch:
            del m
            torch.cuda.empty_cache()
        out["serving"] = serving(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_budget)
        ncpu = len(os.sched_getaffinity(0))
        out["cpu_baseline_all_threads"] = cpu_baseline(spec, args.cpu_budget / 2, threads=ncpu)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
