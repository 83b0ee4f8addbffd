"""CPU tests of the serving loop's scheduling with a fake backend: admission
by memory budget and slots in arrival order, retirement, failure isolation,
latency accounting.  The fake backend advances a tiny linear model so that
results are checkable; no GPU and no library calls."""
import numpy as np

from paper_1512_02548_amd.serve import Request, Server


class Spec:
    def __init__(self, size, dt=0.1, poison=False):
        self.size, self.dt, self.poison = size, dt, poison


class FakeBackend:
    def __init__(self):
        self.live = {}
        self.max_live = 0
        self.steps_seen = []

    def footprint(self, spec):
        return spec.size, None

    def create(self, spec, state_fn, probe=None):
        t = dict(spec=spec, y=np.array([1.0, 0.0]))
        self.live[id(t)] = t
        self.max_live = max(self.max_live, len(self.live))
        return t

    def step(self, tanks):
        self.steps_seen.append(len(tanks))
        ok, msg = [], []
        for t in tanks:
            if t["spec"].poison:
                ok.append(False)
                msg.append("NONFINITE")
                continue
            dt = t["spec"].dt
            c, s = np.cos(dt), np.sin(dt)
            t["y"] = np.array([c * t["y"][0] - s * t["y"][1], s * t["y"][0] + c * t["y"][1]])
            ok.append(True)
            msg.append("OK")
        return ok, msg

    def result(self, t):
        return dict(y=t["y"].copy())

    def release(self, t):
        self.live.pop(id(t), None)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.01
        return self.t


def test_admission_budget_slots_and_results():
    be = FakeBackend()
    srv = Server(be, state_fn=None, memory_budget=100, max_slots=3, clock=FakeClock())
    reqs = [Request(i, Spec(size=30 + 10 * (i % 3)), arrival=0.05 * i, steps=5 + i) for i in range(10)]
    rep = srv.run(reqs, realtime=False)
    assert rep["done"] == 10 and rep["failed"] == 0
    assert be.max_live <= 3
    assert max(be.steps_seen) <= 3
    # each result equals the closed form of its own step count (independent of the mix)
    for r in srv.finished:
        ang = r.steps * r.spec.dt
        assert np.allclose(r.result["y"], [np.cos(ang), np.sin(ang)], atol=1e-12)
    assert rep["tank_steps"] == sum(r.steps for r in reqs)
    assert rep["p99_latency_s"] >= rep["p50_latency_s"] > 0
    assert srv.in_use == 0


def test_oversized_and_poisoned_requests_fail_alone():
    be = FakeBackend()
    srv = Server(be, state_fn=None, memory_budget=100, max_slots=4, clock=FakeClock())
    reqs = [Request(0, Spec(50), 0.0, 4), Request(1, Spec(500), 0.0, 4),
            Request(2, Spec(20, poison=True), 0.0, 4), Request(3, Spec(20), 0.0, 4)]
    rep = srv.run(reqs, realtime=False)
    st = {r.rid: r.status for r in srv.finished}
    assert st == {0: "done", 1: "failed", 2: "failed", 3: "done"}
    ang = 4 * 0.1
    for r in srv.finished:
        if r.status == "done":
            assert np.allclose(r.result["y"], [np.cos(ang), np.sin(ang)])
    assert rep["failed"] == 2 and srv.in_use == 0


def test_arrival_order_is_respected_under_memory_pressure():
    be = FakeBackend()
    srv = Server(be, state_fn=None, memory_budget=60, max_slots=8, clock=FakeClock())
    reqs = [Request(0, Spec(50), 0.0, 3), Request(1, Spec(40), 0.0, 3), Request(2, Spec(5), 0.0, 3)]
    srv.run(reqs, realtime=False)
    admits = sorted(srv.finished, key=lambda r: r.t_admit)
    assert [r.rid for r in admits] == [0, 1, 2]
