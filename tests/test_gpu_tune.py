"""GPU test of the element-tile autotuner: it returns a valid choice per
(P, nz) class, and a tank built with any tile count applies the same
operator (up to the summation order at shared lines)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_autotune_table_and_operator_invariance():
    import torch
    from paper_1512_02548_amd import lib, tune
    from paper_1512_02548_amd import workloads as wl
    specs = wl.batch_tank_specs(count=6, seed=7)
    for s in specs:
        s.nx = min(s.nx, 64)
    table, rep = tune.tune(specs, candidates=(1, 2, 4), reps=5)
    assert set(table) == set(tune.classes(specs))
    assert all(v in (1, 2, 4) for v in table.values())
    assert rep["seconds"] > 0
    # the stiffness apply does not depend on the tile count
    nx, nz, P = 40, 4, 6
    ns = nx * P
    xs = None
    outs = []
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal(nx * P * (P * nz + 1))
    for tt in (1, 2, 3, 4):
        m = lib.Mesh(nx, nz, P, 2 * np.pi, True, np.ones(ns), np.zeros(ns), tiles_per_block=tt)
        if xs is None:
            xs = m.surface_x()
        eta = torch.tensor(0.05 * np.cos(xs), device="cuda")
        etax = torch.tensor(-0.05 * np.sin(xs), device="cuda")
        m.set_surface(eta, etax)
        u = torch.tensor(u0, device="cuda")
        y = torch.empty_like(u)
        m.apply(lib.SEM_OP_STIFFNESS, u, y)
        outs.append(y.cpu().numpy())
    for o in outs[1:]:
        assert np.max(np.abs(o - outs[0])) <= 1e-13 * np.max(np.abs(outs[0]))


def test_batch_context_tuner_and_batched_timing():
    """The batch-context tuner picks one tile count per order from timings
    of the batched launch, and the batched timing hook rejects an order with
    no tank."""
    from paper_1512_02548_amd import lib, tune
    from paper_1512_02548_amd import workloads as wl
    specs = wl.batch_tank_specs(count=12, seed=31)
    for s in specs:
        s.nx = min(s.nx, 64)
        s.params["mwav"] = max(1, s.nx // 8)
        s.length = s.params["mwav"] * 2 * np.pi / s.params["k"]
    table, rep = tune.tune_batch(specs, wl.batch_tank_state, candidates=(1, 4), reps=3, sample=8)
    orders = {P for (P, _) in table}
    assert orders and all(t in (1, 4) for t in table.values())
    for P in orders:
        assert len({t for (q, _), t in table.items() if q == P}) == 1
        assert rep[f"P{P}"]["best"] in (1, 4)
    s = specs[0]
    m = lib.Mesh(s.nx, s.nz, s.P, s.length, True, np.ones(s.ns), np.zeros(s.ns))
    b = lib.Batch([m], 0)
    assert b.apply_timed(s.P, 0, 2) > 0
    other = next(P for P in (4, 6, 8) if P != s.P)
    with pytest.raises(lib.SemError):
        b.apply_timed(other, 0, 2)
