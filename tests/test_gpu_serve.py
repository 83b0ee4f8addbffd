"""GPU tests of batching and serving: a tank's result is the same alone and
in a mix (bitwise: each tank runs the same deterministic kernels), and the
served results match single-tank runs."""
import numpy as np
import pytest

from paper_1512_02548_amd import workloads as wl

pytestmark = pytest.mark.gpu


def small_specs():
    specs = wl.batch_tank_specs(count=6, steps=3, bar_fraction=0.5, seed=99)
    for s in specs:                       # keep the GPU test short
        s.nx = min(s.nx, 24)
        s.length = max(1, s.nx // 8) * 2 * np.pi / s.params["k"]
        s.params["mwav"] = max(1, s.nx // 8)
    return specs


def run_alone(spec, steps, opts):
    import torch
    from paper_1512_02548_amd.serve import GpuBackend
    be = GpuBackend(nstreams=1, opts=opts)
    t = be.create(spec, wl.batch_tank_state)
    for _ in range(steps):
        code, _ = t["mesh"].rk4_step(t["eta"], t["phi"], t["ws"], spec.dt, opts)
    torch.cuda.synchronize()
    return be.result(t)


@pytest.mark.parametrize("prec,nstreams", [(0, 0), (1, 0), (0, 4), (1, 4)])
def test_batch_equals_alone(prec, nstreams):
    from paper_1512_02548_amd import lib
    from paper_1512_02548_amd.serve import GpuBackend
    opts = lib.default_opts(rtol=1e-10, warm_start=1, prec=prec, inner_rtol=1e-3)
    specs = small_specs()
    steps = 3
    alone = [run_alone(s, steps, opts) for s in specs]
    be = GpuBackend(nstreams=nstreams, opts=opts)
    tanks = [be.create(s, wl.batch_tank_state) for s in specs]
    for _ in range(steps):
        ok, msg = be.step(tanks)
        assert all(ok), msg
    for a, t in zip(alone, tanks):
        r = be.result(t)
        assert np.array_equal(r["eta"], a["eta"]) and np.array_equal(r["phi"], a["phi"])


@pytest.mark.parametrize("nstreams", [0, 4])
def test_server_mix_matches_alone(nstreams):
    from paper_1512_02548_amd import lib
    from paper_1512_02548_amd.serve import GpuBackend, Request, Server
    opts = lib.default_opts(rtol=1e-8, warm_start=1, prec=1, inner_rtol=1e-3)
    specs = small_specs()
    reqs = [Request(i, s, arrival=0.02 * i, steps=2 + (i % 3)) for i, s in enumerate(specs)]
    srv = Server(GpuBackend(nstreams=nstreams, opts=opts), wl.batch_tank_state, max_slots=4)
    rep = srv.run(reqs)
    assert rep["done"] == len(specs)
    for r in srv.finished:
        a = run_alone(r.spec, r.steps, opts)
        assert np.array_equal(r.result["eta"], a["eta"]), r.rid
    assert rep["p99_latency_s"] >= rep["p50_latency_s"] > 0


def test_served_results_match_oracle():
    """Requests served together (a bar tank, an eighth-order tank, a
    four-layer tank, arriving while the others run) against the oracle's own
    steps of each tank: FP64 solves to rtol 1e-12, results within 1e-10."""
    from test_gpu_batch import oracle_specs, oracle_steps
    from paper_1512_02548_amd import lib
    from paper_1512_02548_amd.serve import GpuBackend, Request, Server
    opts = lib.default_opts(rtol=1e-12, warm_start=1, max_iter=20000)
    specs = oracle_specs()
    steps = [2, 3, 2]
    reqs = [Request(i, s, arrival=0.01 * i, steps=n) for i, (s, n) in enumerate(zip(specs, steps))]
    srv = Server(GpuBackend(nstreams=0, opts=opts), wl.batch_tank_state, max_slots=4)
    rep = srv.run(reqs)
    assert rep["done"] == len(specs)
    for r in srv.finished:
        e_o, p_o = oracle_steps(r.spec, r.steps)
        assert np.max(np.abs(r.result["eta"] - e_o)) / np.max(np.abs(e_o)) < 1e-10, r.rid
        assert np.max(np.abs(r.result["phi"] - p_o)) / np.max(np.abs(p_o)) < 1e-10, r.rid
