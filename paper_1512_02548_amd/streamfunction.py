"""Exact steady nonlinear waves by the Fourier stream-function method.

The paper takes its steep-wave initial data and reference solutions from
stream-function theory (Dean 1965): a periodic wave of permanent form on a
flat bed, found numerically as a truncated Fourier series of the stream
function whose coefficients satisfy the nonlinear free-surface conditions at
collocation points (Secs. 4.3 and 5.1, Table 1; Fig. 9).  This module solves
that problem with Newton's method and continuation in wave height, written
from the mathematics of the method (Dean 1965; Rienecker and Fenton 1981),
and evaluates the resulting wave anywhere.  It holds no arithmetic of the
spectral element method: it is an input generator and an exact reference.

Formulation (frame moving with the wave at speed c, y measured up from the
bed, mean depth h, wavenumber k, X = x - c t):

    psi(X, y) = -U y + sum_{j=1..N} B_j sinh(j k y)/cosh(j k h) cos(j k X)

is harmonic and has psi = 0 on the bed.  The free surface y = Y(X) is a
streamline, psi(X, Y) = -Q, and on it Bernoulli's equation holds,
1/2 |grad psi|^2 + g Y = R.  Unknowns: Y at N+1 points X_m = m pi/(N k)
over half a wavelength (the wave is symmetric about its crest at X = 0),
B_1..B_N, U, Q and R.  Two more conditions close the system: the mean of Y
is h (trapezoidal mean over the collocation points) and Y(0) - Y(pi/k) = H.
There is no mean Eulerian current, so c = U (Stokes' first definition).

In the fixed frame the velocity potential is

    phi(x, z, t) = sum_j B_j cosh(j k (z + h))/cosh(j k h) sin(j k (x - c t)),

with z = y - h, so phi is periodic in x and harmonic, with d phi/dz = 0 on
the bed.  The surface elevation at any x solves psi(X, Y) = -Q for Y.
"""
from dataclasses import dataclass

import numpy as np

G_ACC = 9.81


@dataclass
class StreamFunctionWave:
    k: float
    h: float
    H: float
    g: float
    B: np.ndarray           # B_1..B_N
    U: float                # mean speed of the flow in the wave frame (= c)
    Q: float                # volume flux in the wave frame
    R: float                # Bernoulli constant
    Yc: np.ndarray          # surface height above the bed at the collocation points

    @property
    def N(self):
        return len(self.B)

    @property
    def c(self):
        return self.U

    @property
    def period(self):
        return 2 * np.pi / (self.k * self.c)

    @property
    def wavelength(self):
        return 2 * np.pi / self.k

    # ------------------------------------------------------------ fields
    def _j(self):
        return np.arange(1, self.N + 1, dtype=float)

    def _ratio_sinh(self, y):
        """sinh(j k y)/cosh(j k h) for y >= 0, evaluated without overflow."""
        jk = self._j()[:, None] * self.k
        y = np.asarray(y, dtype=float)[None, :]
        return (np.exp(jk * (y - self.h)) - np.exp(-jk * (y + self.h))) / (1.0 + np.exp(-2 * jk * self.h))

    def _ratio_cosh(self, y):
        jk = self._j()[:, None] * self.k
        y = np.asarray(y, dtype=float)[None, :]
        return (np.exp(jk * (y - self.h)) + np.exp(-jk * (y + self.h))) / (1.0 + np.exp(-2 * jk * self.h))

    def psi(self, X, Y):
        X = np.atleast_1d(np.asarray(X, dtype=float))
        Y = np.atleast_1d(np.asarray(Y, dtype=float))
        cosX = np.cos(self._j()[:, None] * self.k * X[None, :])
        return -self.U * Y + (self.B[:, None] * self._ratio_sinh(Y) * cosX).sum(0)

    def velocity_wave_frame(self, X, Y):
        """(u', v') = (d psi/dy, -d psi/dX) in the frame moving with the wave."""
        X = np.atleast_1d(np.asarray(X, dtype=float))
        Y = np.atleast_1d(np.asarray(Y, dtype=float))
        jk = self._j()[:, None] * self.k
        arg = jk * X[None, :]
        u = -self.U + (self.B[:, None] * jk * self._ratio_cosh(Y) * np.cos(arg)).sum(0)
        v = (self.B[:, None] * jk * self._ratio_sinh(Y) * np.sin(arg)).sum(0)
        return u, v

    def surface_height(self, X, tol=1e-14, max_iter=60):
        """Y(X) above the bed: the root of psi(X, Y) + Q = 0 (Newton, starting
        from the cosine interpolant of the collocation values)."""
        X = np.atleast_1d(np.asarray(X, dtype=float))
        N = self.N
        m = np.arange(N + 1)
        # cosine coefficients of the collocation values (trapezoidal rule)
        w = np.ones(N + 1)
        w[0] = w[-1] = 0.5
        E = np.array([2.0 / N * np.sum(w * self.Yc * np.cos(j * m * np.pi / N)) for j in range(N + 1)])
        E[0] *= 0.5
        E[-1] *= 0.5
        Y = (E[:, None] * np.cos(np.arange(N + 1)[:, None] * self.k * X[None, :])).sum(0)
        for _ in range(max_iter):
            f = self.psi(X, Y) + self.Q
            u, _ = self.velocity_wave_frame(X, Y)        # d psi/dy
            dY = -f / u
            Y = Y + dY
            if np.max(np.abs(dY)) < tol * self.h:
                return Y
        raise RuntimeError("surface height did not converge")

    def eta(self, x, t=0.0):
        """Free-surface elevation above the still-water level."""
        return self.surface_height(np.asarray(x, dtype=float) - self.c * t) - self.h

    def phi(self, x, z, t=0.0):
        """Velocity potential in the fixed frame."""
        x = np.atleast_1d(np.asarray(x, dtype=float))
        z = np.atleast_1d(np.asarray(z, dtype=float))
        arg = self._j()[:, None] * self.k * (x - self.c * t)[None, :]
        return (self.B[:, None] * self._ratio_cosh(z + self.h) * np.sin(arg)).sum(0)

    def velocity(self, x, z, t=0.0):
        """(u, w) = grad phi in the fixed frame."""
        x = np.atleast_1d(np.asarray(x, dtype=float))
        z = np.atleast_1d(np.asarray(z, dtype=float))
        jk = self._j()[:, None] * self.k
        arg = jk * (x - self.c * t)[None, :]
        u = (self.B[:, None] * jk * self._ratio_cosh(z + self.h) * np.cos(arg)).sum(0)
        w = (self.B[:, None] * jk * self._ratio_sinh(z + self.h) * np.sin(arg)).sum(0)
        return u, w

    def surface_state(self, x, t=0.0):
        """(eta, phi~) at surface abscissae x: the initial data of a tank."""
        eta = self.eta(x, t)
        return eta, self.phi(x, eta, t)

    def residuals(self, X):
        """Kinematic and dynamic surface conditions at arbitrary X (for checks)."""
        Y = self.surface_height(X)
        u, v = self.velocity_wave_frame(X, Y)
        kin = self.psi(X, Y) + self.Q
        dyn = 0.5 * (u * u + v * v) + self.g * Y - self.R
        return kin, dyn


def _system(z, k, h, H, g, N):
    """Residuals of the collocation system and their Jacobian."""
    Y = z[:N + 1]
    B = z[N + 1:2 * N + 1]
    U, Q, R = z[2 * N + 1:]
    X = np.arange(N + 1) * np.pi / (N * k)
    w = StreamFunctionWave(k, h, H, g, B, U, Q, R, Y)
    jk = w._j()[:, None] * k                    # (N, 1)
    Sh, Ch = w._ratio_sinh(Y), w._ratio_cosh(Y)  # (N, N+1)
    C, Sn = np.cos(jk * X[None, :]), np.sin(jk * X[None, :])
    Bc = B[:, None]
    u = -U + (Bc * jk * Ch * C).sum(0)
    v = (Bc * jk * Sh * Sn).sum(0)
    kin = -U * Y + (Bc * Sh * C).sum(0) + Q
    dyn = 0.5 * (u * u + v * v) + g * Y - R
    mean = (0.5 * Y[0] + Y[1:-1].sum() + 0.5 * Y[-1]) / N - h
    f = np.concatenate([kin, dyn, [mean, Y[0] - Y[-1] - H]])
    n1 = N + 1
    J = np.zeros((2 * n1 + 2, 2 * N + 4))
    du_dY = (Bc * jk * jk * Sh * C).sum(0)
    dv_dY = (Bc * jk * jk * Ch * Sn).sum(0)
    idx = np.arange(n1)
    J[idx, idx] = u
    J[:n1, n1:n1 + N] = (Sh * C).T
    J[:n1, 2 * N + 1] = -Y
    J[:n1, 2 * N + 2] = 1.0
    J[n1 + idx, idx] = u * du_dY + v * dv_dY + g
    J[n1:2 * n1, n1:n1 + N] = (u[None, :] * jk * Ch * C + v[None, :] * jk * Sh * Sn).T
    J[n1:2 * n1, 2 * N + 1] = -u
    J[n1:2 * n1, 2 * N + 3] = -1.0
    wts = np.full(n1, 1.0 / N)
    wts[0] = wts[-1] = 0.5 / N
    J[2 * n1, :n1] = wts
    J[2 * n1 + 1, 0] = 1.0
    J[2 * n1 + 1, N] = -1.0
    return f, J


def _newton(z, args, tol=1e-13, max_iter=50):
    """Newton's method; done when the update or the residual reaches rounding
    level (with many modes in deep water the columns of the high modes are
    nearly zero at the troughs and the Jacobian is ill-conditioned, so the
    update can stall at 1e-9 while the residual is already at 1e-15)."""
    scale = abs(z[-1])                 # the Bernoulli constant, ~ g h
    for _ in range(max_iter):
        f, Jm = _system(z, *args)
        if np.max(np.abs(f)) < 32 * np.finfo(float).eps * scale:
            return z
        step = np.linalg.solve(Jm, -f)
        z = z + step
        if np.max(np.abs(step)) < tol * max(1.0, np.max(np.abs(z))):
            return z
    raise RuntimeError("stream-function Newton iteration did not converge")


def solve(k, h, H, N=20, g=G_ACC, height_steps=None):
    """Steady wave of height H on depth h with wavenumber k, N Fourier modes.
    Continuation in height from the linear wave; returns StreamFunctionWave."""
    if H <= 0:
        raise ValueError("wave height must be positive")
    steps = height_steps or max(4, int(np.ceil(40 * H * k / (2 * np.pi) / 0.1)))
    X = np.arange(N + 1) * np.pi / (N * k)
    c0 = np.sqrt(g * np.tanh(k * h) / k)
    prev = []
    z = None
    for s in range(1, steps + 1):
        Hs = H * s / steps
        if len(prev) >= 2:
            z0 = 2 * prev[-1] - prev[-2]
        elif len(prev) == 1:
            z0 = prev[-1] * 1.0
            z0[:N + 1] = h + (z0[:N + 1] - h) * s / (s - 1)
            z0[N + 1:2 * N + 1] *= s / (s - 1)
        else:
            B = np.zeros(N)
            B[0] = 0.5 * Hs * c0 / np.tanh(k * h)
            z0 = np.concatenate([h + 0.5 * Hs * np.cos(k * X), B, [c0, c0 * h, 0.5 * c0 * c0 + g * h]])
        z = _newton(z0, (k, h, Hs, g, N))
        prev.append(z)
    Y = z[:N + 1]
    return StreamFunctionWave(k, h, H, g, z[N + 1:2 * N + 1].copy(), *z[2 * N + 1:], Y.copy())


def refine(w, N):
    """The same wave with N modes, by Newton's method started from w (its
    surface at the new collocation points, its coefficients padded with
    zeros)."""
    X = np.arange(N + 1) * np.pi / (N * w.k)
    B = np.zeros(N)
    B[:min(N, w.N)] = w.B[:N]
    z0 = np.concatenate([w.surface_height(X), B, [w.U, w.Q, w.R]])
    z = _newton(z0, (w.k, w.h, w.H, w.g, N))
    return StreamFunctionWave(w.k, w.h, w.H, w.g, z[N + 1:2 * N + 1].copy(), *z[2 * N + 1:], z[:N + 1].copy())


def solve_resolved(k, h, H, g=G_ACC, tol=1e-11, sizes=(12, 16, 20, 24, 32, 40, 48, 64)):
    """The wave with the smallest number of modes whose dynamic condition,
    checked between the collocation points, holds to tol relative to the
    Bernoulli constant; if none does, the size with the smallest such
    residual.  (More modes than the wave needs only add columns at rounding
    level and make the collocation system ill-conditioned.)  The first size
    is reached by height continuation, the others start from the previous
    size's wave."""
    best, best_res, w = None, np.inf, None
    for N in sizes:
        try:
            w = solve(k, h, H, N=N, g=g) if w is None else refine(w, N)
        except RuntimeError:
            if w is None:
                continue
            break
        X = np.linspace(0.0, np.pi / k, 4 * N + 1)
        _, dyn = w.residuals(X)
        res = np.max(np.abs(dyn)) / abs(w.R)
        if res < best_res:
            best, best_res = w, res
        if res < tol or res > 10 * best_res:
            break
    if best is None:
        raise RuntimeError("no stream-function solution found")
    return best
