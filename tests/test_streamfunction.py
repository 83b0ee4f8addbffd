"""Pins of the stream-function wave generator (CPU): the linear limit, the
second-order Stokes bound harmonic, the third-order deep-water phase speed,
the nonlinear surface conditions between the collocation points, and the
fixed-frame potential that the tanks are started from."""
import numpy as np
import pytest

from paper_1512_02548_amd import streamfunction as sf
from paper_1512_02548_amd.workloads import limiting_steepness

G = 9.81


def harmonics(w, count=4, n=512):
    """Cosine amplitudes E_1..E_count of eta over one wavelength."""
    x = np.arange(n) * w.wavelength / n
    c = np.fft.rfft(w.eta(x)) / n
    return 2 * c.real[1:count + 1], c.real[0]


@pytest.mark.parametrize("kh", [0.5, 1.0, 3.0])
def test_linear_limit(kh):
    """H -> 0: c -> sqrt(g tanh(kh)/k), eta -> H/2 cos kx and the potential
    -> (H/2) c coth(kh) cosh(k(z+h))/cosh(kh) sin kx (Sec. 4.2)."""
    k, h = kh, 1.0
    H = 1e-5 * 2 * np.pi / k           # (kH/2)^2 ~ 1e-9: the nonlinear corrections
    w = sf.solve(k, h, H, N=12)
    c0 = np.sqrt(G * np.tanh(kh) / k)
    assert abs(w.c / c0 - 1) < 1e-8
    assert abs(w.B[0] / (0.5 * H * c0 / np.tanh(kh)) - 1) < 1e-4
    x = np.linspace(0, w.wavelength, 37)
    # the second harmonic, O(kH) relative (largest in shallow water), remains
    assert np.max(np.abs(w.eta(x) - 0.5 * H * np.cos(k * x))) < 1e-3 * H


@pytest.mark.parametrize("kh", [0.8, 1.5])
def test_second_order_bound_harmonic(kh):
    """Stokes' second-order theory: the cos 2kx amplitude of eta equals
    k a^2 cosh(kh) (2 + cosh 2kh) / (4 sinh^3 kh), a the first-harmonic
    amplitude, up to O((ka)^2) relative."""
    k, h = kh, 1.0
    w = sf.solve(k, h, 0.01 / k, N=16)
    E, mean = harmonics(w)
    a = E[0]
    expect = k * a * a * np.cosh(kh) * (2 + np.cosh(2 * kh)) / (4 * np.sinh(kh) ** 3)
    assert abs(E[1] / expect - 1) < 1e-3
    assert abs(mean) < 1e-12


def test_third_order_deep_water_speed():
    """Stokes' third-order dispersion relation in deep water:
    c = sqrt(g/k) (1 + (ka)^2 / 2) with a the first-harmonic amplitude."""
    k, h = 1.0, 10.0
    c0 = np.sqrt(G / k)
    ratios = []
    for ka in (0.02, 0.04):
        w = sf.solve(k, h, 2 * ka / k, N=16)
        a = harmonics(w)[0][0]
        ratios.append((w.c / c0 - 1) / (k * a) ** 2)
    assert all(abs(r - 0.5) < 5e-3 for r in ratios)
    assert abs(ratios[0] - 0.5) < abs(ratios[1] - 0.5)


def test_steep_wave_conditions_between_collocation_points():
    """At 90% of the limiting steepness (kh = 1, H/L = 0.0903, the paper's
    Table 1 wave) the kinematic and dynamic conditions hold between the
    collocation points, spectrally better with more modes."""
    k, h = 1.0, 1.0
    H = 0.9 * limiting_steepness(1.0) * 2 * np.pi
    X = np.linspace(0, np.pi, 301)
    res = []
    for N in (20, 32):
        w = sf.solve(k, h, H, N=N)
        kin, dyn = w.residuals(X)
        assert np.max(np.abs(kin)) < 1e-13
        res.append(np.max(np.abs(dyn)) / w.R)
    assert res[1] < 1e-8 < res[0] < 1e-5
    w = sf.solve_resolved(k, h, H)
    assert np.max(np.abs(w.residuals(X)[1])) / w.R < 5e-9
    # crest-trough height and zero mean level
    x = np.arange(4096) * w.wavelength / 4096
    eta = w.eta(x)
    assert abs(eta.max() - eta.min() - H) < 1e-12
    assert abs(eta.mean()) < 1e-9 * H


def test_fixed_frame_potential_solves_the_free_surface_problem():
    """The potential handed to the tanks satisfies, in the fixed frame, the
    kinematic and dynamic free-surface conditions (eqs. FSeta and FSphi
    written for phi at the surface): eta_t + phi_x eta_x - phi_z = 0 and
    phi_t + |grad phi|^2/2 + g eta = const, with d/dt = -c d/dx for a wave
    of permanent form; and phi is harmonic with no flux through the bed."""
    k, h = 1.0, 1.0
    w = sf.solve_resolved(k, h, 0.6 * limiting_steepness(1.0) * 2 * np.pi)
    x = np.linspace(0.1, 6.0, 23)
    d = 1e-5
    eta = w.eta(x)
    eta_x = (w.eta(x + d) - w.eta(x - d)) / (2 * d)
    u, wz = w.velocity(x, eta)
    kin = -w.c * eta_x + u * eta_x - wz
    assert np.max(np.abs(kin)) < 1e-8
    phi_t = -w.c * u
    bern = phi_t + 0.5 * (u * u + wz * wz) + G * eta
    assert np.max(np.abs(bern - bern.mean())) < 1e-9 * G
    # potential and velocity agree; Laplacian vanishes; no flux at z = -h
    z = -0.4 * np.ones_like(x)
    ux = (w.phi(x + d, z) - w.phi(x - d, z)) / (2 * d)
    uz = (w.phi(x, z + d) - w.phi(x, z - d)) / (2 * d)
    u2, w2 = w.velocity(x, z)
    assert np.max(np.abs(ux - u2)) < 1e-8 and np.max(np.abs(uz - w2)) < 1e-8
    e = 1e-3
    lap = (w.phi(x + e, z) + w.phi(x - e, z) + w.phi(x, z + e) + w.phi(x, z - e) - 4 * w.phi(x, z)) / e ** 2
    assert np.max(np.abs(lap)) < 1e-4
    assert np.max(np.abs(w.velocity(x, -h * np.ones_like(x))[1])) < 1e-14
