"""Seeded synthetic inputs for wave-tank runs.

This module holds no arithmetic of the numerical method: it only draws
parameters and evaluates surface fields (linear waves, exact stream-function
waves, a trapezoidal bar, a JONSWAP-shaped irregular train) at surface
x-coordinates that the caller supplies.  It is shared by the
product path (bench, serving) and by the tests that feed the same arrays to the
CPU oracle.

Workloads (sizes are quads in x by layers in sigma, order P):
  standing_wave    8x2, P=4, periodic, kh=1, H/L=0.001, linear standing wave
  stream_series    64x4, P=6, periodic, kh=1, H/L=0.0903 (90% of limiting),
                   exact stream-function wave of 20 Fourier modes with a seeded
                   crest position, Pf=9, filter last 2 modes 0.5%
  table1           8x1, P=6, periodic, one wavelength of the kh=1, H/L=0.0903
                   stream-function wave; T/dt = 40, 80, 160; filter and
                   over-integration switched on and off
  bar_irregular    2048x8, P=6, walls, L=40h, trapezoidal bar, 64-component
                   JONSWAP-shaped train with kh in [0.5, 3]
  batch_tanks      256 periodic flat tanks with random sizes and orders
  requests         Poisson request stream of tanks drawn like batch_tanks,
                   half of them over a bar
"""
from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

from . import streamfunction as sfw

G_ACC = 9.81
SEED_BASE = 20251512


def omega_linear(k, h, g=G_ACC):
    """Linear dispersion relation omega^2 = g k tanh(kh) (for input generation)."""
    return np.sqrt(g * k * np.tanh(k * h))


def limiting_steepness(kh):
    """H_max/L as a function of kh: 0.1003 at kh = 1 scaled like tanh(kh)
    (calibrated so that 90% gives H/L = 0.0903 at kh = 1)."""
    return 0.1003 * np.tanh(kh) / np.tanh(1.0)


@dataclass
class TankSpec:
    """Everything needed to build one tank and its initial state."""
    nx: int
    nz: int
    P: int
    length: float
    periodic: bool
    Pf: int
    filter_ic: int
    filter_sigma: float
    dt: float
    steps: int
    rtol: float
    g: float = G_ACC
    name: str = ""
    params: dict = field(default_factory=dict)

    @property
    def ns(self):
        return self.P * self.nx + (0 if self.periodic else 1)


def courant_dt(length, nx, P, c, cr=0.5):
    """dt = Cr * (node spacing dX/P) / c."""
    return cr * (length / nx / P) / c


# ------------------------------------------------------------ 8x2 standing wave
def standing_wave_spec():
    k, h = 1.0, 1.0
    L = 2 * np.pi / k
    c = omega_linear(k, h) / k
    return TankSpec(nx=8, nz=2, P=4, length=L, periodic=True, Pf=4, filter_ic=5,
                    filter_sigma=1.0, dt=courant_dt(L, 8, 4, c), steps=10, rtol=1e-12,
                    name="standing_wave_8x2_P4", params=dict(k=k, h=h, H=0.001 * L))


def standing_wave_state(xs, spec, t0_frac=0.125, H=None):
    """Linear standing wave eta = H/2 cos kx cos wt0 and the exact linear
    potential evaluated at z = eta(x), at t0 = T/8."""
    k, h = spec.params["k"], spec.params["h"]
    H = spec.params["H"] if H is None else H
    w = omega_linear(k, h)
    t0 = t0_frac * 2 * np.pi / w
    xs = np.asarray(xs, dtype=float)
    eta = 0.5 * H * np.cos(k * xs) * np.cos(w * t0)
    phi = (-(H * G_ACC / (2 * w)) * np.cosh(k * (eta + h)) / np.cosh(k * h)
           * np.cos(k * xs) * np.sin(w * t0))
    return eta, phi, np.full_like(xs, h), np.zeros_like(xs)


# ------------------------------------------------------ 64x4 stream-type series
def stream_series_spec(nx=64, nz=4, P=6, steps=1000):
    k, h = 1.0, 1.0
    L = 2 * np.pi / k
    c = omega_linear(k, h) / k
    return TankSpec(nx=nx, nz=nz, P=P, length=L, periodic=True, Pf=int(np.ceil(1.5 * P)),
                    filter_ic=P - 1, filter_sigma=0.995, dt=courant_dt(L, nx, P, c),
                    steps=steps, rtol=1e-12, name=f"stream_series_{nx}x{nz}_P{P}",
                    params=dict(k=k, h=h, HL=0.9 * limiting_steepness(k * h), modes=20,
                                seed=SEED_BASE + 2))


@lru_cache(maxsize=512)
def sf_wave(k, h, H, modes=None):
    """Stream-function wave (exact steady wave of permanent form); modes=None
    takes as many Fourier modes as the wave needs."""
    if modes is None:
        return sfw.solve_resolved(k, h, H, g=G_ACC)
    return sfw.solve(k, h, H, N=modes, g=G_ACC)


def sf_crest(seed, wavelength):
    """Seeded crest position in [0, wavelength)."""
    return float(np.random.default_rng(seed).uniform(0.0, wavelength))


def stream_series_state(xs, spec, t=0.0):
    """The exact stream-function wave of the spec (20 Fourier modes) with its
    crest at a seeded position, at time t: (eta, phi~, h, h_x)."""
    p = spec.params
    k, h = p["k"], p["h"]
    w = sf_wave(k, h, p["HL"] * 2 * np.pi / k, p["modes"])
    x0 = sf_crest(p["seed"], w.wavelength)
    xs = np.asarray(xs, dtype=float)
    eta, phi = w.surface_state(xs - x0, t)
    return eta, phi, np.full_like(xs, h), np.zeros_like(xs)


def stream_series_exact_eta(xs, spec, t):
    """Elevation of the spec's exact wave at time t (the reference for
    accuracy measurements)."""
    return stream_series_state(xs, spec, t)[0]


# ------------------------------------------------ Table 1 (filter x over-integration)
TABLE1_STRATEGIES = (
    # (name, filter, over-integration order factor); "top": the paper's 5%
    # off the highest mode; "bubble": every bubble mode (ic = 2) damped at
    # the rate of the still-water growth of the triangle discretisation
    ("no_filter_no_overint", None, 1),
    ("no_filter_overint", None, 2),
    ("filter_no_overint", "top", 1),
    ("filter_overint", "top", 2),
    ("bubble_filter_overint", "bubble", 2),
)
# growth rate (1/s) of the still-water linearised system of the 8x1, P = 6
# triangle tank (kh = 1, h = 1): the rate the bubble filter has to remove
TABLE1_BUBBLE_RATE = 3.5


def table1_spec(steps_per_period, strategy, periods=50.0):
    """One wavelength of the kh = 1, H/L = 0.0903 stream-function wave on 8
    elements of order 6 (one layer), as in the paper's Table 1; the filter
    removes 5% of the amplitude of the highest mode once per step and
    over-integration uses GLL(2P) nodes."""
    name, filt, fac = next(s for s in TABLE1_STRATEGIES if s[0] == strategy)
    k, h, P, nx = 1.0, 1.0, 6, 8
    L = 2 * np.pi / k
    w = sf_wave(k, h, 0.9 * limiting_steepness(k * h) * L, None)
    T = w.period
    dt = T / steps_per_period
    ic, sig = {None: (P + 1, 1.0), "top": (P, 0.95), "bubble": (2, float(np.exp(-TABLE1_BUBBLE_RATE * dt)))}[filt]
    return TankSpec(nx=nx, nz=1, P=P, length=L, periodic=True, Pf=fac * P,
                    filter_ic=ic, filter_sigma=sig,
                    dt=dt, steps=int(round(periods * steps_per_period)), rtol=1e-12,
                    name=f"table1_{strategy}_T{steps_per_period}",
                    params=dict(k=k, h=h, HL=0.9 * limiting_steepness(k * h), modes=None, seed=SEED_BASE + 6,
                                period=T, steps_per_period=steps_per_period, strategy=strategy))


# ---------------------------------------------- 2048x8 bar, irregular waves
def bar_irregular_spec(nx=2048, nz=8, P=6, steps=4):
    L, h0 = 40.0, 1.0
    c = omega_linear(1.0, h0)
    return TankSpec(nx=nx, nz=nz, P=P, length=L, periodic=False, Pf=int(np.ceil(1.5 * P)),
                    filter_ic=P - 1, filter_sigma=0.995, dt=courant_dt(L, nx, P, c),
                    steps=steps, rtol=1e-10, name=f"bar_irregular_{nx}x{nz}_P{P}",
                    params=dict(h0=h0, crest=0.3, seed=SEED_BASE + 3, Hs=0.04,
                                ncomp=64, kmin=0.5, kmax=3.0, kp=1.0, gamma=3.3))


def trapezoid_bar(xs, L, nx, h0, crest, x0, crest_len, up=20.0, down=10.0):
    """Depth of a trapezoidal bar: h0 offshore, rising with slope 1:up to the
    crest depth, flat crest, falling with slope 1:down back to h0.  Corner
    positions snap to element boundaries.  Returns (h, h_x)."""
    dX = L / nx
    rise = h0 - crest
    snap = lambda v: np.round(v / dX) * dX
    xa = snap(x0)
    xb = snap(xa + rise * up)
    xc = snap(xb + crest_len)
    xd = snap(xc + rise * down)
    xs = np.asarray(xs, dtype=float)
    h = np.full_like(xs, h0)
    hx = np.zeros_like(xs)
    m = (xs > xa) & (xs < xb)
    h[m] = h0 - (xs[m] - xa) * rise / (xb - xa)
    hx[m] = -rise / (xb - xa)
    m = (xs >= xb) & (xs <= xc)
    h[m] = crest
    m = (xs > xc) & (xs < xd)
    h[m] = crest + (xs[m] - xc) * rise / (xd - xc)
    hx[m] = rise / (xd - xc)
    return h, hx


def jonswap(omega_, omega_p, gamma=3.3):
    """JONSWAP-shaped spectral density (textbook form, unnormalised)."""
    sig = np.where(omega_ <= omega_p, 0.07, 0.09)
    r = np.exp(-((omega_ - omega_p) ** 2) / (2 * sig ** 2 * omega_p ** 2))
    return omega_ ** -5 * np.exp(-1.25 * (omega_p / omega_) ** 4) * gamma ** r


def bar_irregular_state(xs, spec):
    p = spec.params
    rng = np.random.default_rng(p["seed"])
    x0 = rng.uniform(4.0, 8.0)
    crest_len = rng.uniform(2.0, 6.0)
    h, hx = trapezoid_bar(xs, spec.length, spec.nx, p["h0"], p["crest"], x0, crest_len)
    ks = np.exp(np.linspace(np.log(p["kmin"]), np.log(p["kmax"]), p["ncomp"]))
    om = omega_linear(ks, p["h0"])
    omp = omega_linear(p["kp"], p["h0"])
    dom = np.gradient(om)
    S = jonswap(om, omp, p["gamma"])
    amp = np.sqrt(2 * S * dom)
    phase = rng.uniform(0.0, 2 * np.pi, p["ncomp"])
    # scale to the significant wave height Hs = 4 sqrt(m0)
    m0 = 0.5 * np.sum(amp ** 2)
    amp *= p["Hs"] / (4 * np.sqrt(m0))
    xs = np.asarray(xs, dtype=float)
    arg = ks[:, None] * xs[None, :] - phase[:, None]
    eta = (amp[:, None] * np.cos(arg)).sum(0)
    c = om / ks
    phi = (amp[:, None] * (c / np.tanh(ks * p["h0"]))[:, None] * np.sin(arg)).sum(0)
    # cosine taper to zero within 2 of each wall
    taper = np.ones_like(xs)
    lw, L = 2.0, spec.length
    m = xs < lw
    taper[m] = 0.5 * (1 - np.cos(np.pi * xs[m] / lw))
    m = xs > L - lw
    taper[m] = 0.5 * (1 - np.cos(np.pi * (L - xs[m]) / lw))
    return eta * taper, phi * taper, h, hx


# ------------------------------------------- generation and absorption zones
def relax_weight(xi):
    """1 - gamma over a relaxation zone, xi = 0 at the zone's outer end and 1
    where it meets the interior: 1 - (10 xi^3 - 15 xi^4 + 6 xi^5), which
    falls from 1 to 0 with zero first and second derivatives at both ends."""
    xi = np.clip(xi, 0.0, 1.0)
    return 1.0 - xi ** 3 * (10.0 - 15.0 * xi + 6.0 * xi * xi)


def relax_tank_spec(nx=48, nz=2, P=4, wavelengths=3, periods=4.0):
    """A walled flat tank of `wavelengths` linear waves (kh = 1, H/L = 0.01):
    a generation zone of one wavelength at x = 0 drives the progressive wave,
    an absorption zone of one wavelength at x = L takes it out."""
    k, h = 1.0, 1.0
    lam = 2 * np.pi / k
    L = wavelengths * lam
    c = omega_linear(k, h) / k
    dt = courant_dt(L, nx, P, c)
    T = lam / c
    return TankSpec(nx=nx, nz=nz, P=P, length=L, periodic=False, Pf=int(np.ceil(1.5 * P)),
                    filter_ic=P + 1, filter_sigma=1.0, dt=dt, steps=int(np.ceil(periods * T / dt)), rtol=1e-12,
                    name=f"relax_tank_{nx}x{nz}_P{P}",
                    params=dict(k=k, h=h, H=0.01 * lam, gen_len=lam, abs_len=lam, period=T))


def incident_linear(xs, t, k, h, H):
    """Linear progressive wave of Sec. 4.2 at the surface: (eta, phi~)."""
    w = omega_linear(k, h)
    c = w / k
    eta = 0.5 * H * np.cos(w * t - k * xs)
    phi = -0.5 * H * c * np.cosh(k * (eta + h)) / np.sinh(k * h) * np.sin(w * t - k * xs)
    return eta, phi


def wave_group_state(xs, spec, x0, width=None):
    """A right-going linear wave group centred at x0: the carrier of the
    tank's linear wave under a Gaussian envelope (deep-water-free kh = 1,
    width one wavelength): (eta, phi~)."""
    p = spec.params
    k, h, H = p["k"], p["h"], p["H"]
    width = width or 2 * np.pi / k
    xs = np.asarray(xs, dtype=float)
    env = np.exp(-((xs - x0) / width) ** 2)
    e, ph = incident_linear(xs, 0.0, k, h, H)
    return env * e, env * ph


def relax_tank_forcing(xs, spec, incident=None):
    """(weight, target): weight = 1 - gamma at the surface nodes (generation
    zone at x = 0, absorption zone at x = L, 0 between); target(t) = the
    incident wave (eta_a, phi~_a) in the generation half, 0 in the absorption
    half, ramped in over the first period."""
    p = spec.params
    xs = np.asarray(xs, dtype=float)
    L = spec.length
    wgt = np.zeros_like(xs)
    g = xs < p["gen_len"]
    wgt[g] = relax_weight(xs[g] / p["gen_len"])
    a = xs > L - p["abs_len"]
    wgt[a] = relax_weight((L - xs[a]) / p["abs_len"])
    left = xs < 0.5 * L
    inc = incident or (lambda x, t: incident_linear(x, t, p["k"], p["h"], p["H"]))

    def target(t):
        e, ph = inc(xs, t)
        ramp = min(1.0, t / p["period"])
        ramp = ramp * ramp * (3 - 2 * ramp)
        return np.where(left, ramp * e, 0.0), np.where(left, ramp * ph, 0.0)
    return wgt, target


# ------------------------------------------------------------ batches
def batch_tank_specs(count=256, seed=SEED_BASE + 4, steps=200, rtol=1e-10, bar_fraction=0.0, max_frac=0.9,
                     filter_modes=2, filter_sigma=0.995):
    """Random periodic tanks: nx ~ U{16..1024}, nz ~ U{2,4,8}, P ~ U{4,6,8},
    kh ~ U[0.5, 3], H/L ~ U[0.01, max_frac] of the limiting steepness, about 8
    elements per wavelength (L = m 2 pi / k, m = max(1, nx // 8)); the modal
    filter scales the top `filter_modes` modes by `filter_sigma` once per step."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        nx = int(rng.integers(16, 1025))
        nz = int(rng.choice([2, 4, 8]))
        P = int(rng.choice([4, 6, 8]))
        kh = float(rng.uniform(0.5, 3.0))
        frac = float(rng.uniform(0.01, max_frac))
        bar = bool(rng.uniform() < bar_fraction)
        crest = float(rng.uniform(0.3, 0.6))
        h = 1.0
        k = kh / h
        mwav = max(1, nx // 8)
        L = mwav * 2 * np.pi / k
        c = omega_linear(k, h) / k
        specs.append(TankSpec(nx=nx, nz=nz, P=P, length=L, periodic=True,
                              Pf=int(np.ceil(1.5 * P)), filter_ic=P + 1 - filter_modes, filter_sigma=filter_sigma,
                              dt=courant_dt(L, nx, P, c), steps=steps, rtol=rtol,
                              name=f"tank{i}_{nx}x{nz}_P{P}",
                              params=dict(k=k, h=h, HL=frac * limiting_steepness(kh),
                                          seed=int(rng.integers(0, 2 ** 31)),
                                          mwav=mwav, bar=bar, crest=crest)))
    return specs


def batch_tank_state(xs, spec):
    """The tank's exact stream-function wave (as many modes as it needs),
    crest at a seeded position; optionally a bar scaled into the middle 60%
    of the tank (the wave is then the flat-bed wave of the offshore depth)."""
    p = spec.params
    xs = np.asarray(xs, dtype=float)
    k, h0 = p["k"], p["h"]
    w = sf_wave(k, h0, p["HL"] * 2 * np.pi / k, None)
    eta, phi = w.surface_state(xs - sf_crest(p["seed"], w.wavelength))
    h = np.full_like(xs, h0)
    hx = np.zeros_like(xs)
    if p.get("bar"):
        L = spec.length
        span = 0.6 * L
        rise = h0 - p["crest"]
        # slopes scaled so that the whole bar fits the middle 60%
        total = rise * (20 + 10) + 0.2 * span
        sc = span / total
        h, hx = trapezoid_bar(xs, L, spec.nx, h0, p["crest"], 0.2 * L, 0.2 * span * sc,
                              up=20 * sc, down=10 * sc)
    return eta, phi, h, hx


def poisson_arrivals(rate, count, seed=SEED_BASE + 5):
    """Arrival times of a Poisson process with the given rate (per second)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))
