"""Continuous-batching server for wave-tank simulation requests.

Each request is a tank (mesh sizes, depth profile, initial surface state) to
be advanced a given number of RK4 steps.  The server

* admits arrived requests while a slot is free and their device footprint
  (workspace + state) fits in the memory budget, in arrival order;
* keeps every admitted tank's mesh, workspace and state resident;
* advances all admitted tanks together, one RK4 step per tick, through the
  library's batch call (lockstep by default: the stage solves of all
  in-flight tanks run as one batched GMRES, every launch covering all tanks);
* admits new tanks and retires finished (or failed) ones only between ticks;
  a retired tank stays in the device batch, switched off by the batch's
  active mask, until the next admission rebuilds the batch (so retirements
  cost no rebuild, and each tick's arrivals share one);
* records per-request latency (arrival to completion) and throughput.

The backend is pluggable: ``GpuBackend`` drives libsem.so; tests substitute a
CPU backend to exercise admission, retirement and failure handling without a
GPU.
"""
import argparse
import json
import sys
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    spec: object                 # workloads.TankSpec
    arrival: float               # seconds after the start of the run
    steps: int
    status: str = "queued"       # queued, running, done, failed
    done_steps: int = 0
    t_admit: float = None
    t_done: float = None
    handle: object = None
    probe: object = None
    footprint: int = 0
    error: str = ""
    result: dict = field(default_factory=dict)

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival


class GpuBackend:
    """Tanks on the GPU through the C ABI; steps are batched across tanks."""

    def __init__(self, nstreams=0, opts=None, device="cuda", tiles=None):
        import torch

        from . import lib
        from . import workloads as wl
        self.torch, self.lib, self.wl = torch, lib, wl
        self.nstreams = nstreams
        self.device = device
        self.opts = opts if opts is not None else lib.default_opts(
            rtol=1e-8, warm_start=1, prec=lib.SEM_PREC_FP32_IR, inner_rtol=1e-5, lookahead=3)
        self._batch = None
        self._members = []        # tanks of the current device batch, in its order
        self._retired = []        # retired members kept alive until the next rebuild
        self.rebuilds = 0
        self.tiles = tiles        # autotuner table (P, nz) -> stiffness tiles per workgroup, or None

    def _tiles(self, spec):
        from . import tune
        return tune.tiles_for(self.tiles, spec)

    def footprint(self, spec):
        ns = spec.ns
        m = self.lib.Mesh(spec.nx, spec.nz, spec.P, spec.length, spec.periodic, np.ones(ns), np.zeros(ns),
                          filter_ic=spec.filter_ic, filter_sigma=spec.filter_sigma, overint=spec.Pf, bind=False,
                          tiles_per_block=self._tiles(spec))
        return int(m.info.workspace_bytes) + 8 * (2 * ns + int(m.n)), m

    def create(self, spec, state_fn, probe=None):
        torch = self.torch
        ns = spec.ns
        # surface x-coordinates come from the mesh; a flat-bed probe mesh is
        # reused when the tank is flat, otherwise rebuilt with its depth
        if probe is None:
            probe = self.lib.Mesh(spec.nx, spec.nz, spec.P, spec.length, spec.periodic, np.ones(ns),
                                  np.zeros(ns), filter_ic=spec.filter_ic, filter_sigma=spec.filter_sigma,
                                  overint=spec.Pf, bind=False, tiles_per_block=self._tiles(spec))
        xs = probe.surface_x()
        eta, phi, h, hx = state_fn(xs, spec)
        if np.all(h == 1.0) and np.all(hx == 0.0):
            m = probe
            m.bind(self.device)
        else:
            m = self.lib.mesh_from_spec(spec, h, hx, device=self.device, tiles_per_block=self._tiles(spec))
        dev = torch.device(self.device)
        tank = dict(mesh=m, spec=spec,
                    eta=torch.tensor(eta, dtype=torch.float64, device=dev),
                    phi=torch.tensor(phi, dtype=torch.float64, device=dev),
                    ws=torch.zeros(m.n, dtype=torch.float64, device=dev))
        return tank

    def step(self, tanks):
        pos = {id(t): i for i, t in enumerate(self._members)}
        if self._batch is None or any(id(t) not in pos for t in tanks):
            # a tank joined: one batch over the running tanks; retired ones go
            self._batch = self.lib.Batch([t["mesh"] for t in tanks], self.nstreams)
            self._members = list(tanks)
            for t in self._retired:
                t.clear()
            self._retired = []
            self.rebuilds += 1
            pos = {id(t): i for i, t in enumerate(self._members)}
        mem = self._members
        want = {id(t) for t in tanks}
        active = [id(t) in want for t in mem]
        code, st, it = self._batch.rk4_step([t["eta"] for t in mem], [t["phi"] for t in mem],
                                            [t["ws"] for t in mem], [t["spec"].dt for t in mem],
                                            active=active, opts=self.opts)
        st = [st[pos[id(t)]] for t in tanks]
        return [s == 0 for s in st], [self.lib.STATUS_NAMES.get(s, str(s)) for s in st]

    def result(self, tank):
        return dict(eta=tank["eta"].cpu().numpy(), phi=tank["phi"].cpu().numpy())

    def release(self, tank):
        if any(t is tank for t in self._members):
            self._retired.append(tank)      # still referenced by the device batch
        else:
            tank.clear()


class Server:
    def __init__(self, backend, state_fn, memory_budget=64 << 30, max_slots=64, clock=None, log=None):
        self.backend = backend
        self.state_fn = state_fn
        self.memory_budget = int(memory_budget)
        self.max_slots = int(max_slots)
        self.clock = clock or time.perf_counter
        self.queue, self.running, self.finished = [], [], []
        self.in_use = 0
        self.tank_steps = 0
        self.ticks = 0
        self.log = log          # optional callable(str): one line per retired request

    def submit(self, req):
        req.footprint, req.probe = self.backend.footprint(req.spec)
        if req.footprint > self.memory_budget:
            req.status, req.error = "failed", "footprint exceeds the memory budget"
            self.finished.append(req)
            return
        self.queue.append(req)

    def _admit(self, now):
        while self.queue and self.queue[0].arrival <= now:
            r = self.queue[0]
            if len(self.running) >= self.max_slots or self.in_use + r.footprint > self.memory_budget:
                break                      # arrival order: wait for memory/slots to free up
            self.queue.pop(0)
            try:
                r.handle = self.backend.create(r.spec, self.state_fn, r.probe)
                r.probe = None
            except Exception as e:         # a tank that cannot be built fails alone
                r.status, r.error, r.t_done = "failed", str(e), now
                self.finished.append(r)
                continue
            r.status, r.t_admit = "running", now
            self.in_use += r.footprint
            self.running.append(r)

    def _retire(self, r, now, ok=True, err=""):
        r.t_done = now
        r.status = "done" if ok else "failed"
        r.error = err
        if ok:
            r.result = self.backend.result(r.handle)
        self.backend.release(r.handle)
        r.handle = None
        self.in_use -= r.footprint
        self.running.remove(r)
        self.finished.append(r)
        if self.log:
            self.log(f"request {r.rid} {r.status} at {now:.2f}s, latency {r.latency:.2f}s {r.error}")

    def run(self, requests, t0=None, realtime=True):
        """Serve requests whose `arrival` times are relative to the start."""
        for r in sorted(requests, key=lambda r: r.arrival):
            self.submit(r)
        start = self.clock() if t0 is None else t0
        virtual = 0.0
        while self.queue or self.running:
            now = (self.clock() - start) if realtime else virtual
            self._admit(now)
            if not self.running:
                # idle until the next arrival
                nxt = self.queue[0].arrival
                if realtime:
                    time.sleep(max(0.0, min(0.05, nxt - now)))
                else:
                    virtual = max(virtual, nxt)
                continue
            t_step = self.clock()
            ok, msg = self.backend.step([r.handle for r in self.running])
            self.ticks += 1
            if not realtime:
                virtual += self.clock() - t_step
            now = (self.clock() - start) if realtime else virtual
            for r, good, m in list(zip(self.running, ok, msg)):
                if not good:
                    self._retire(r, now, ok=False, err=m)
                    continue
                r.done_steps += 1
                self.tank_steps += 1
                if r.done_steps >= r.steps:
                    self._retire(r, now)
        total = (self.clock() - start) if realtime else virtual
        return self.report(total)

    def report(self, total_s):
        lat = np.array([r.latency for r in self.finished if r.status == "done"])
        return dict(requests=len(self.finished), done=int(sum(r.status == "done" for r in self.finished)),
                    failed=int(sum(r.status == "failed" for r in self.finished)),
                    tank_steps=self.tank_steps, seconds=total_s,
                    tank_steps_per_s=self.tank_steps / total_s if total_s > 0 else 0.0,
                    p50_latency_s=float(np.percentile(lat, 50)) if lat.size else None,
                    p99_latency_s=float(np.percentile(lat, 99)) if lat.size else None,
                    ticks=self.ticks)


def make_requests(count, rate, steps, seed=None, bar_fraction=0.5, max_nx=None, filter_modes=3, filter_sigma=0.8):
    """Poisson stream of tanks drawn like the batch workload (exact
    stream-function waves), half over a bar.  Requests filter the top three
    modes by 0.8 per step: with the batch workload's two-mode 0.5% filter the
    growing grid-scale modes of the triangle discretisation end most
    requests within 200 steps (24 of 32 in a measured sample), with this one
    2 of 32."""
    from . import workloads as wl
    kw = {} if seed is None else dict(seed=seed)
    specs = wl.batch_tank_specs(count=count, steps=steps, rtol=1e-8, bar_fraction=bar_fraction,
                                filter_modes=filter_modes, filter_sigma=filter_sigma, **kw)
    if max_nx is not None:
        for s in specs:
            s.nx = min(s.nx, max_nx)
    arr = wl.poisson_arrivals(rate, count)
    return [Request(i, s, float(a), steps) for i, (s, a) in enumerate(zip(specs, arr))]


def main():
    ap = argparse.ArgumentParser(description="serve a Poisson stream of wave-tank requests on one GPU")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=4.0, help="arrivals per second")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--streams", type=int, default=0,
                    help="0: lockstep batch (default); >= 1: per-tank steps on that many streams")
    ap.add_argument("--max-nx", type=int, default=None)
    ap.add_argument("--filter-modes", type=int, default=3)
    ap.add_argument("--filter-sigma", type=float, default=0.8)
    ap.add_argument("--quiet", action="store_true", help="no per-request lines on stderr")
    ap.add_argument("--tune", action="store_true",
                    help="choose the stiffness element tiles with the autotuner first (not timed)")
    ap.add_argument("--sequential-fp64", action="store_true",
                    help="baseline: one tank at a time, plain FP64, arrivals ignored")
    a = ap.parse_args()
    from . import lib
    from . import workloads as wl
    reqs = make_requests(a.requests, a.rate, a.steps, max_nx=a.max_nx, filter_modes=a.filter_modes,
                         filter_sigma=a.filter_sigma)
    log = None if a.quiet else (lambda line: print(line, file=sys.stderr, flush=True))
    if a.sequential_fp64:
        be = GpuBackend(nstreams=1, opts=lib.default_opts(rtol=1e-8, warm_start=1, lookahead=3))
        srv = Server(be, wl.batch_tank_state, max_slots=1, log=log)
    else:
        tiles, trep = None, None
        if a.tune:
            from . import tune
            tiles, trep = tune.tune([r.spec for r in reqs])
        be = GpuBackend(nstreams=a.streams, tiles=tiles)
        srv = Server(be, wl.batch_tank_state, max_slots=a.slots, log=log)
    rep = srv.run(reqs)
    rep.update(mode="sequential_fp64" if a.sequential_fp64 else ("lockstep_mixed" if a.streams == 0 else
                                                                  "concurrent_mixed"), rate=a.rate, steps=a.steps,
               filter=[a.filter_modes, a.filter_sigma], batch_rebuilds=getattr(srv.backend, "rebuilds", None))
    if not a.sequential_fp64 and a.tune:
        rep["autotune"] = trep
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
