"""GPU parity of the wave generation and absorption zones (Sec. 2.2) against
the oracle, through sem_set_relaxation and sem_rk4_step_forced."""
import numpy as np
import pytest

from helpers import Pair, cuda, host, rel_err
from oracle.stepper import Tank
from paper_1512_02548_amd import workloads as wl

pytestmark = pytest.mark.gpu


def targets(target, t, dt):
    """[3, 2, ns]: (eta_a, phi~_a) at t, t + dt/2, t + dt."""
    return np.stack([np.stack(target(t + c * dt)) for c in (0.0, 0.5, 1.0)])


@pytest.mark.parametrize("bar", [False, True])
def test_forced_steps_match_oracle(bar):
    """A walled tank with a generation zone (linear wave, ramped in) and an
    absorption zone: 12 forced RK4 steps from rest on the GPU against the
    oracle's, over a flat bed and over a bar, relative 1e-10."""
    spec = wl.relax_tank_spec(nx=24, nz=2, P=4)
    from oracle.mesh import Mesh as OMesh
    om = OMesh(spec.nx, spec.nz, spec.P, spec.length, False)
    xs = om.xs_surf
    h, hx = np.ones_like(xs), np.zeros_like(xs)
    if bar:
        h, hx = wl.trapezoid_bar(xs, spec.length, spec.nx, 1.0, 0.6, 0.4 * spec.length, 1.0, up=5.0, down=5.0)
    pair = Pair(spec.nx, spec.nz, spec.P, spec.length, False, h, hx, Pf=spec.Pf)
    wgt, target = wl.relax_tank_forcing(xs, spec)
    pair.m.set_relaxation(wgt)
    tank = Tank(om, h, hx, Pf=spec.Pf)
    e_t, p_t = cuda(np.zeros(om.ns)), cuda(np.zeros(om.ns))
    ws = cuda(np.zeros(pair.m.n))
    opts = pair.lib.default_opts(rtol=1e-13, warm_start=1)
    e_o, p_o = np.zeros(om.ns), np.zeros(om.ns)
    # start half a period in, so that the ramp is under way and the zone moves
    t = 0.5 * spec.params["period"]
    for _ in range(12):
        pair.m.rk4_step_forced(e_t, p_t, ws, spec.dt, cuda(targets(target, t, spec.dt)), opts)
        e_o, p_o = tank.step(e_o, p_o, spec.dt, t, relax=(wgt, target))
        t += spec.dt
    assert np.max(np.abs(e_o)) > 0.05 * spec.params["H"]
    assert rel_err(host(e_t), e_o) < 1e-10 and rel_err(host(p_t), p_o) < 1e-10


def test_relaxation_argument_checks():
    from paper_1512_02548_amd import lib
    spec = wl.relax_tank_spec(nx=8, nz=1, P=3)
    m = lib.Mesh(spec.nx, spec.nz, spec.P, spec.length, False, np.ones(spec.ns), np.zeros(spec.ns))
    z = cuda(np.zeros(spec.ns))
    ws = cuda(np.zeros(m.n))
    qa = cuda(np.zeros((3, 2, spec.ns)))
    with pytest.raises(lib.SemError):            # no weights yet
        m.rk4_step_forced(z, z.clone(), ws, spec.dt, qa)
    with pytest.raises(lib.SemError):            # weights outside [0, 1]
        m.set_relaxation(np.full(spec.ns, 1.5))
    m.set_relaxation(np.zeros(spec.ns))
    with pytest.raises(lib.SemError):            # batches do not take forced tanks
        lib.Batch([m], 0)
    # zero weights: the forced step is the plain step, bitwise
    e1, p1 = cuda(0.01 * np.cos(np.linspace(0, 3, spec.ns))), cuda(np.zeros(spec.ns))
    e2, p2 = e1.clone(), p1.clone()
    m.rk4_step_forced(e1, p1, ws, spec.dt, qa)
    m.reset_history()
    ws.zero_()
    m.rk4_step(e2, p2, ws, spec.dt)
    assert np.array_equal(host(e1), host(e2)) and np.array_equal(host(p1), host(p2))
