"""GPU parity of vertically clustered meshes and of the volume kinematics
(u, w at every node) against the oracle, and the kinematics of a steep
stream-function wave against the exact wave (Secs. 2, 3.1.3, 4.2, 4.3)."""
import numpy as np
import pytest

from helpers import Pair, cuda, host, rel_err
from oracle import laplace as olap
from oracle import surface as osrf
from oracle.mesh import Mesh as OMesh
from oracle.stepper import Tank
from paper_1512_02548_amd import workloads as wl

pytestmark = pytest.mark.gpu


def cosine_levels(nz):
    """Layer interfaces clustered towards the free surface:
    sigma_j = sin(pi j / (2 nz))."""
    return np.sin(0.5 * np.pi * np.arange(nz + 1) / nz)


def state(xs, L, amp, bar):
    k = 2 * np.pi / L
    eta = amp * np.cos(k * xs) + 0.3 * amp * np.sin(2 * k * xs + 0.4)
    phi = 0.5 * np.sin(k * xs) - 0.2 * np.cos(3 * k * xs)
    h, hx = np.ones_like(xs), np.zeros_like(xs)
    if bar:
        h = 1.0 - 0.4 * np.exp(-((xs - L / 2) / (0.2 * L)) ** 2)
        hx = 0.8 * (xs - L / 2) / (0.2 * L) ** 2 * np.exp(-((xs - L / 2) / (0.2 * L)) ** 2)
    return eta, phi, h, hx


CASES = [
    # nx, nz, P, L, periodic, bar, clustered
    (12, 4, 6, 2 * np.pi, True, False, True),
    (9, 3, 4, 4.0, False, True, True),
    (10, 2, 5, 3.0, True, False, False),
    (7, 3, 8, 2.5, False, True, False),
]


@pytest.mark.parametrize("case", CASES)
def test_kinematics_and_clustered_layers_match_oracle(case):
    nx, nz, P, L, periodic, bar, clustered = case
    lev = cosine_levels(nz) if clustered else None
    xs = OMesh(nx, 1, P, L, periodic).xs_surf
    eta, phi, h, hx = state(xs, L, 0.1, bar)
    pair = Pair(nx, nz, P, L, periodic, h, hx, sigma_levels=lev)
    om, m, lib = pair.om, pair.m, pair.lib
    s1 = osrf.Surface1D(om)
    etax = s1.recover_dx(eta)
    G, d = olap.coefficients(om, eta, etax, h, hx)
    Phi_o = olap.solve_direct(om, olap.stiffness(om, G), phi)
    # the Laplace solve on the (clustered) mesh
    Phi = cuda(np.zeros(m.n))
    m.laplace_solve(cuda(eta), cuda(etax), cuda(phi), Phi, lib.default_opts(rtol=1e-13, max_iter=20000))
    assert rel_err(pair.to_oracle(host(Phi)), Phi_o) < 1e-10
    # u and w in the volume from the oracle's Phi (isolates the projections)
    u, w = cuda(np.zeros(m.n)), cuda(np.zeros(m.n))
    m.recover_kinematics(cuda(pair.to_lib(Phi_o)), cuda(eta), cuda(etax), u, w)
    u_o = osrf.recover_u(om, Phi_o, olap.sigma_x(om, eta, etax, h, hx))
    w_o = osrf.recover_w(om, Phi_o, d)
    assert rel_err(pair.to_oracle(host(u)), u_o) < 1e-11
    assert rel_err(pair.to_oracle(host(w)), w_o) < 1e-11
    # w on the surface is the w~ of the existing recovery
    ws = cuda(np.zeros(m.ns))
    m.gradient_recover(lib.SEM_RECOVER_W, cuda(pair.to_lib(Phi_o)), cuda(eta), ws)
    assert np.array_equal(host(ws), host(w)[m.surface_nodes()])


def test_rk4_steps_on_clustered_layers_match_oracle():
    """Two RK4 steps of a stream-function wave on cosine-clustered layers
    (over-integrated, filtered) against the oracle."""
    spec = wl.stream_series_spec(nx=16, nz=3, P=6)
    lev = cosine_levels(3)
    om = OMesh(spec.nx, spec.nz, spec.P, spec.length, True, sigma_levels=lev)
    eta, phi, h, hx = wl.stream_series_state(om.xs_surf, spec)
    pair = Pair(spec.nx, spec.nz, spec.P, spec.length, True, h, hx, filter_ic=spec.filter_ic,
                filter_sigma=spec.filter_sigma, Pf=spec.Pf, sigma_levels=lev)
    tank = Tank(om, h, hx, Pf=spec.Pf, filt=(spec.filter_ic, spec.filter_sigma))
    e_t, p_t = cuda(eta), cuda(phi)
    ws = cuda(np.zeros(pair.m.n))
    opts = pair.lib.default_opts(rtol=1e-13, warm_start=1)
    e_o, p_o = eta.copy(), phi.copy()
    for _ in range(2):
        pair.m.rk4_step(e_t, p_t, ws, spec.dt, opts)
        e_o, p_o = tank.step(e_o, p_o, spec.dt)
    assert rel_err(host(e_t), e_o) < 1e-10 and rel_err(host(p_t), p_o) < 1e-10


@pytest.mark.parametrize("clustered", [False, True])
def test_stream_function_kinematics(clustered):
    """Kinematics of the kh = 1 wave at 90% of the limiting steepness (the
    paper's Fig. 8 setting: 10 elements of order 6 along one wavelength):
    the Laplace solve from the exact surface potential and the projections
    give u and w at every node within 3% of the wave's crest particle speed
    of the exact values; clustering the layers towards the surface (three
    layers) is at least as accurate as one layer of the same order."""
    from paper_1512_02548_amd import lib
    k, h = 1.0, 1.0
    w = wl.sf_wave(k, h, 0.9 * wl.limiting_steepness(1.0) * 2 * np.pi, None)
    nx, P = 10, 6
    nz = 3 if clustered else 1
    lev = cosine_levels(nz) if clustered else None
    ns = nx * P
    m = lib.Mesh(nx, nz, P, w.wavelength, True, np.ones(ns), np.zeros(ns), sigma_levels=lev)
    xs = m.surface_x()
    eta, phis = w.surface_state(xs)
    om = OMesh(nx, nz, P, w.wavelength, True, sigma_levels=lev)
    etax = osrf.Surface1D(om).recover_dx(eta)
    Phi = cuda(np.zeros(m.n))
    m.laplace_solve(cuda(eta), cuda(etax), cuda(phis), Phi, lib.default_opts(rtol=1e-13, max_iter=20000))
    u, wz = cuda(np.zeros(m.n)), cuda(np.zeros(m.n))
    m.recover_kinematics(Phi, cuda(eta), cuda(etax), u, wz)
    x, s = m.node_coords()
    # physical node depth from the exact surface (the mesh carries its
    # column interpolant, spectrally close)
    z = s * (w.eta(x) + h) - h
    ue, we = w.velocity(x, z)
    scale = np.max(np.abs(ue))
    err = max(np.max(np.abs(host(u) - ue)), np.max(np.abs(host(wz) - we))) / scale
    print(f"\nstream-function kinematics, {'3 clustered layers' if clustered else 'one layer'}: "
          f"max error / max u = {err:.3e}")
    assert err < 3e-2
