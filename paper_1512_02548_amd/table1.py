"""Stability and accuracy ablation of the paper's Table 1 on the GPU.

The kh = 1, H/L = 0.0903 (90% of the limiting steepness) stream-function
wave travels through one wavelength-long periodic tank of 8 elements of
order 6 (here 8 x 1 quads, each cut into two triangles), with the free-surface
right-hand side over-integrated (GLL(2P) nodes) or not, and with the modal
filter (5% off the amplitude of the highest mode once per step) or not, at
T/dt = 40, 80 and 160 time steps per wave period (Sec. 5.1, Table 1).

Each run advances with the library's RK4 step until t/T = 50 or until the
step fails (non-finite values or a water column of non-positive height,
the library's NONFINITE / DOMAIN statuses: the paper's "NaN").  Reported per
run: the step and t/T of failure, the error max_i |eta_i - eta_exact(x_i, t)|
/ H against the exact wave translated by c t at the paper's reporting times
t/T = 1, 1.8, 3.1, 10, 28.2, 50, and the wall time per step over the first
30 steps (the paper's cost per dt is its ratio to the no-filter,
no-over-integration run at the same T/dt).

Usage: python -m paper_1512_02548_amd.table1 [--periods 50] [--out FILE]
"""
import argparse
import json
import sys
import time

import numpy as np

REPORT_TIMES = (1.0, 1.8, 3.1, 10.0, 28.2, 50.0)
COST_STEPS = 30


def run(strategy, steps_per_period, periods=50.0, rtol=1e-12, report_times=REPORT_TIMES, log=None):
    import torch

    from . import lib
    from . import workloads as wl

    spec = wl.table1_spec(steps_per_period, strategy, periods)
    ns = spec.ns
    m = lib.mesh_from_spec(spec, np.ones(ns), np.zeros(ns))
    xs = m.surface_x()
    eta0, phi0, _, _ = wl.stream_series_state(xs, spec)
    dev = torch.device("cuda:0")
    eta = torch.tensor(eta0, device=dev)
    phi = torch.tensor(phi0, device=dev)
    ws = torch.zeros(m.n, dtype=torch.float64, device=dev)
    opts = lib.default_opts(rtol=rtol, warm_start=1, max_iter=2000)
    T = spec.params["period"]
    H = spec.params["HL"] * spec.length
    marks = {int(round(t * steps_per_period)): t for t in report_times if t <= periods}
    out = {"strategy": strategy, "steps_per_period": steps_per_period, "dt": spec.dt, "Pf": spec.Pf,
           "filter": [spec.filter_ic, spec.filter_sigma], "errors": {}, "failed_step": None,
           "failed_t_over_T": None, "status": "OK"}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    t_first = None
    for n in range(1, spec.steps + 1):
        code, _ = m.rk4_step(eta, phi, ws, spec.dt, opts, raise_on_error=False)
        if n == COST_STEPS:
            torch.cuda.synchronize()
            t_first = time.perf_counter() - t0
        if code != lib.SEM_OK:
            out["failed_step"] = n
            out["failed_t_over_T"] = n / steps_per_period
            out["status"] = lib.STATUS_NAMES.get(code, str(code))
            break
        if n in marks:
            ex = wl.stream_series_exact_eta(xs, spec, n * spec.dt)
            e = eta.cpu().numpy()
            out["errors"][f"{marks[n]:g}"] = float(np.max(np.abs(e - ex)) / H)
            if log:
                print(f"# {strategy} T/dt={steps_per_period} t/T={marks[n]:g} error={out['errors'][f'{marks[n]:g}']:.4e}",
                      file=log, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    done = n if out["failed_step"] is None else n - 1
    out["steps_run"] = done
    out["ms_per_step"] = 1e3 * wall / max(n, 1)
    # cost per step over the first steps from the exact wave, before any run
    # has grown far from it (every strategy completes them)
    out["ms_per_step_first"] = 1e3 * t_first / COST_STEPS if t_first is not None else None
    out["period"] = T
    return out


def main(argv=None):
    from . import workloads as wl
    ap = argparse.ArgumentParser()
    ap.add_argument("--periods", type=float, default=50.0)
    ap.add_argument("--steps-per-period", default="40,80,160")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = []
    for spp in (int(v) for v in a.steps_per_period.split(",")):
        base = None
        for strat, _, _ in wl.TABLE1_STRATEGIES:
            r = run(strat, spp, a.periods, log=sys.stderr)
            if base is None:
                base = r["ms_per_step_first"]
            r["cost_per_dt_rel"] = r["ms_per_step_first"] / base if r["ms_per_step_first"] else None
            print(f"# {json.dumps(r)}", file=sys.stderr, flush=True)
            res.append(r)
    text = json.dumps({"table1": res})
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text)


if __name__ == "__main__":
    main()
