"""Autotuner of the stiffness kernel's element tile.

The matrix-core stiffness kernel gives each workgroup a run of whole element
columns, a number of 16-element MFMA tiles (1..4).  The best count depends on
the order P and the layer count nz (tile shape, LDS use, workgroups per CU)
more than on the tank length.  For each (P, nz) class present in a set of
tanks the tuner builds a representative flat tank (the class's median nx)
once per candidate, times the kernel on the device (device events around the
launches), and keeps the fastest.  Meshes built with ``tiles_for(table,
spec)`` use the result; a tank's arithmetic does not depend on the tile
count except for the summation order at shared lines.
"""
import json
import time

import numpy as np

CANDIDATES = (1, 2, 3, 4)


def classes(specs):
    """(P, nz) -> list of nx over the specs."""
    out = {}
    for s in specs:
        out.setdefault((int(s.P), int(s.nz)), []).append(int(s.nx))
    return out


def tune(specs, candidates=CANDIDATES, reps=40, prec=0, device="cuda"):
    """Returns (table, report): table[(P, nz)] = tiles per workgroup."""
    import torch

    from . import lib
    t0 = time.perf_counter()
    table, report = {}, {}
    dt = torch.float64 if prec == 0 else torch.float32
    for (P, nz), nxs in sorted(classes(specs).items()):
        nx = max(2, int(np.median(nxs)))
        ns = nx * P
        times, cols = {}, {}
        for tt in candidates:
            m = lib.Mesh(nx, nz, P, 2 * np.pi, True, np.ones(ns), np.zeros(ns), tiles_per_block=tt, device=device)
            z = torch.zeros(ns, dtype=torch.float64, device=device)
            m.set_surface(z, z)
            u = torch.randn(m.n, dtype=dt, device=device)
            y = torch.empty_like(u)
            m.apply_timed(lib.SEM_OP_STIFFNESS, u, y, 3, prec)          # warm-up
            times[tt] = m.apply_timed(lib.SEM_OP_STIFFNESS, u, y, reps, prec) * 1e3
            cols[tt] = int(m.info.nblocks)
            del m, u, y
        best = min(times, key=times.get)
        table[(P, nz)] = best
        report[f"P{P}_nz{nz}"] = {"nx": nx, "us": {str(k): round(v, 2) for k, v in times.items()},
                                  "workgroups": {str(k): v for k, v in cols.items()}, "best": best}
    report["seconds"] = time.perf_counter() - t0
    return table, report


def tune_batch(specs, state_fn, candidates=CANDIDATES, reps=10, sample=48, seed=7, device="cuda"):
    """Tiles per workgroup chosen in the batched context: a sample of the
    tanks (up to `sample`, spread over the (P, nz) classes) is built once per
    candidate and its batched stiffness launch timed per order with every
    tank live (sem_batch_apply_timed, FP64 and FP32).  The batched launch
    covers all tanks of an order at once, so the choice is per order P and
    applies to every nz.  Returns (table, report) like tune()."""
    import torch

    from . import lib
    t0 = time.perf_counter()
    rng = np.random.default_rng(seed)
    by_class = {}
    for i, s in enumerate(specs):
        by_class.setdefault((int(s.P), int(s.nz)), []).append(i)
    per = max(1, sample // max(1, len(by_class)))
    pick = sorted(j for idx in by_class.values() for j in rng.permutation(idx)[:per])
    orders = sorted({int(specs[i].P) for i in pick})
    times = {P: {} for P in orders}
    for tt in candidates:
        meshes = []
        for i in pick:
            s = specs[i]
            probe = lib.Mesh(s.nx, s.nz, s.P, s.length, s.periodic, np.ones(s.ns), np.zeros(s.ns), bind=False,
                             tiles_per_block=tt)
            _, _, h, hx = state_fn(probe.surface_x(), s)
            meshes.append(lib.Mesh(s.nx, s.nz, s.P, s.length, s.periodic, h, hx, tiles_per_block=tt,
                                   device=device))
        b = lib.Batch(meshes, 0)
        for P in orders:
            times[P][tt] = 1e3 * (b.apply_timed(P, 0, reps) + b.apply_timed(P, 1, reps))
        del b, meshes
        torch.cuda.empty_cache()
    table, report = {}, {}
    for P in orders:
        best = min(times[P], key=times[P].get)
        for (q, nz) in by_class:
            if q == P:
                table[(q, nz)] = best
        report[f"P{P}"] = {"us_fp64_plus_fp32": {str(k): round(v, 2) for k, v in times[P].items()}, "best": best}
    report["tanks_sampled"] = len(pick)
    report["seconds"] = time.perf_counter() - t0
    return table, report


def tiles_for(table, spec):
    """Tiles per workgroup for a spec (0: the library's own choice)."""
    if not table:
        return 0
    return int(table.get((int(spec.P), int(spec.nz)), 0))


def save(table, path):
    with open(path, "w") as f:
        json.dump({f"{P},{nz}": t for (P, nz), t in table.items()}, f, indent=1)


def load(path):
    with open(path) as f:
        raw = json.load(f)
    return {tuple(int(v) for v in k.split(",")): int(t) for k, t in raw.items()}
