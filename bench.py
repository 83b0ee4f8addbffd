"""Benchmark: Laplace-solve throughput of the spectral element free-surface
solver on one MI355X.

Workload (default): the 64x4-quad, P=6, periodic stream-type series tank
(kh = 1, H/L = 90% of the limiting steepness, 20 seeded Fourier modes,
over-integration at Pf = 9, 0.5% filter on the last two modes), advanced by
RK4 steps; every step runs the whole hot path (gradient recovery,
coefficient update, Laplace GMRES solves, vertical-velocity projection,
over-integrated right-hand side, RK4 update, filter) with inputs resident in
HBM.  A step is one RK4 step.

value = Laplace-solve GDOF/s = sum over solves of n_free / sum of solve times.

Prints one JSON line.  --gpus above 1 exits: this build runs on one GPU.
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


def stiffness_bytes_per_elem(P, word=8):
    """Algorithmic HBM bytes of one matrix-free stiffness application per
    element: the geometric-factor stream (3 values per node) plus reading and
    writing each degree of freedom once (P^2/2 owned nodes per element)."""
    Np = (P + 1) * (P + 2) // 2
    return 3 * Np * word + 2 * (P * P / 2.0) * word


def stiffness_flops_per_elem(P):
    Np = (P + 1) * (P + 2) // 2
    return 8 * Np * Np + 6 * Np


def cpu_baseline(spec, budget_s=15.0):
    """The oracle (element matrices -> CSR -> sparse LU) timed on the host for
    a bounded sample of the same workload's Laplace solves."""
    from threadpoolctl import threadpool_limits

    from oracle import laplace as olap
    from oracle import surface as osrf
    from oracle.mesh import Mesh as OMesh
    from paper_1512_02548_amd import workloads as wl

    with threadpool_limits(limits=1):
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
    return dict(value=nfree * count / el / 1e9, unit="GDOF/s", cores=1, kind="oracle",
                sample=f"{count} Laplace solves (assembly + sparse LU) of the initial state, "
                       f"{nfree} free DOF each, {el:.1f} s, BLAS limited to 1 thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rtol", type=float, default=1e-12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

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
    opts = lib.default_opts(rtol=args.rtol, warm_start=1, lookahead=3)
    n_free = m.info.n_free

    def run(steps):
        tsolve, iters, nsolve = 0.0, 0, 0
        for _ in range(steps):
            code, st = m.rk4_step(eta, phi, ws, spec.dt, opts)
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

    # dominant kernel: the matrix-free stiffness apply on this tank's factors
    u = torch.randn(m.n, dtype=torch.float64, device=dev)
    y = torch.empty_like(u)
    reps = 200
    ms = m.apply_timed(lib.SEM_OP_STIFFNESS, u, y, reps)
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
                   "solves": nsolve, "mean_iters": iters / max(nsolve, 1),
                   "solve_time_fraction": tsolve / wall},
        "roofline": {"bound": "hbm", "kernel": "stiffness apply (k_gather STIFF)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "mean_launch_ms": ms,
                     "bytes_per_launch": bytes_launch,
                     "flops_per_launch": stiffness_flops_per_elem(spec.P) * E},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
