"""Method of lines and time stepping (oracle; test infrastructure).

Sec. 3 (method of lines) turns the free-surface equations into an ODE system
for the nodal eta and phi~.  One evaluation of its right-hand side (one
Runge-Kutta stage) is, in the paper's order:

  1. eta_x, phi~_x by 1D gradient recovery (Sec. 3.1.3),
  2. K from eta, eta_x, h, h_x (Sec. 2) and the Laplace solve for Phi with
     Phi = phi~ on the surface (Sec. 3.1.2),
  3. w~ from the 2D projection M w = S_z Phi (Sec. 3.1.3),
  4. the over-integrated Galerkin right-hand sides and M' solves
     (Secs. 3.1.1, 3.3).

Time integration is the explicit fourth-order Runge-Kutta method of Sec.
3.1.1, read as the classical scheme (nodes 0, 1/2, 1/2, 1; weights
1, 2, 2, 1 over 6).  The modal filter of Sec. 3.4 is applied to eta and phi~
once after every completed step.

Sec. 2.2 (wave generation and absorption zones) adds to the right-hand side
of each surface variable q the penalty source (1 - gamma(x)) tau^-1
(q_a(x, t) - q) with tau equal to the time step; the weights 1 - gamma at
the surface nodes and the target q_a(t) = (eta_a, phi~_a) are inputs.
"""
import numpy as np

from . import laplace as lap
from . import surface as srf


def rk4(f, y, dt):
    """One classical RK4 step for y' = f(y) (any array-valued f)."""
    k1 = f(y)
    k2 = f(y + 0.5 * dt * k1)
    k3 = f(y + 0.5 * dt * k2)
    k4 = f(y + dt * k3)
    return y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def rk4_t(f, y, t, dt):
    """One classical RK4 step for y' = f(y, t)."""
    k1 = f(y, t)
    k2 = f(y + 0.5 * dt * k1, t + 0.5 * dt)
    k3 = f(y + 0.5 * dt * k2, t + 0.5 * dt)
    k4 = f(y + dt * k3, t + dt)
    return y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


class Tank:
    """A wave tank: mesh, still-water depth h and slope h_x at the surface
    nodes, gravity, over-integration order and filter."""

    def __init__(self, mesh, h_s, hx_s, g=9.81, Pf=None, filt=None, sign_w2=+1.0):
        self.mesh = mesh
        self.s1 = srf.Surface1D(mesh)
        self.h = np.asarray(h_s, dtype=float)
        self.hx = np.asarray(hx_s, dtype=float)
        self.g = float(g)
        self.Pf = mesh.P if Pf is None else int(Pf)
        self.filt = filt                   # None or (ic, sigma_f)
        self.Mc = srf.mass2d(mesh)
        # +1: the free-surface equation as in eq. "FSphi".  Tests set -1 to
        # reproduce the sign printed in the semi-discrete system.
        self.sign_w2 = float(sign_w2)

    def stage(self, eta, phi, out=None):
        """Right-hand side (eta_t, phi~_t) of the semi-discrete system."""
        m, s1 = self.mesh, self.s1
        etax = s1.recover_dx(eta)
        phix = s1.recover_dx(phi)
        Phi, G, d = lap.laplace_solve(m, eta, etax, phi, self.h, self.hx)
        w = srf.recover_w(m, Phi, d, self.Mc)[m.surf]
        if self.sign_w2 == 1.0:
            eta_t, phi_t = s1.fs_rhs(eta, etax, phix, w, self.g, self.Pf)
        else:
            eta_t, phi_t = self._fs_rhs_signed(eta, etax, phix, w)
        if out is not None:
            out.update(etax=etax, phix=phix, Phi=Phi, G=G, d=d, w=w, eta_t=eta_t, phi_t=phi_t)
        return eta_t, phi_t

    def _fs_rhs_signed(self, eta, etax, phix, w):
        # right-hand side with the w~^2 term's sign flipped (test use only)
        from .refelem import fine_grid
        I, Mf = fine_grid(self.mesh.P, self.Pf)
        s1 = self.s1
        le, lp = [], []
        for e in range(s1.idx.shape[0]):
            ix = s1.idx[e]
            et, ex, px, ww = (I @ np.asarray(v)[ix] for v in (eta, etax, phix, w))
            le.append(s1.Je * I.T @ Mf @ (-ex * px + ww * (1 + ex * ex)))
            fp = -self.g * et - 0.5 * (px * px + ww * ww * (1 + ex * ex))
            lp.append(s1.Je * I.T @ Mf @ fp)
        return s1.solve_mass(s1.assemble_vec(np.array(le))), s1.solve_mass(s1.assemble_vec(np.array(lp)))

    def step(self, eta, phi, dt, t=0.0, relax=None):
        """One RK4 step of (eta, phi~) followed by the per-element filter.
        relax = (weight, target): weight [ns] holds 1 - gamma(x) at the
        surface nodes, target(t) returns (eta_a, phi~_a) at time t; the
        source weight / dt (q_a - q) joins each stage's right-hand side."""
        ns = self.mesh.ns

        def f(y, ts):
            et, pt = self.stage(y[:ns], y[ns:])
            rhs = np.concatenate([et, pt])
            if relax is not None:
                wgt, target = relax
                ea, pa = target(ts)
                rhs += np.concatenate([wgt, wgt]) / dt * (np.concatenate([ea, pa]) - y)
            return rhs

        y = rk4_t(f, np.concatenate([eta, phi]), t, dt)
        eta, phi = y[:ns], y[ns:]
        if self.filt is not None:
            eta = self.s1.apply_filter(eta, *self.filt)
            phi = self.s1.apply_filter(phi, *self.filt)
        return eta, phi

    def energy(self, eta, phi):
        """Discrete energy 1/2 Phi^T A Phi + 1/2 g eta^T M' eta (kinetic + potential)."""
        m = self.mesh
        etax = self.s1.recover_dx(eta)
        G, d = lap.coefficients(m, eta, etax, self.h, self.hx)
        A = lap.stiffness(m, G)
        Phi = lap.solve_direct(m, A, phi)
        return 0.5 * Phi @ (A @ Phi) + 0.5 * self.g * eta @ (self.s1.Mp @ eta)

    def mass(self, eta):
        return np.ones(self.mesh.ns) @ (self.s1.Mp @ eta)
