"""Closed-form linear-wave solutions (oracle; test infrastructure).

Sec. 4.2 (Linear accuracy and dispersion properties) states the linear
progressive wave and the Stokes dispersion relation c^2 = (g/k) tanh(kh) with
g = 9.81.  The harmonic function cosh(k(z+h))/cosh(kh) sin(kx) satisfies the
Laplace equation and the flat-bed Neumann condition exactly for any free
surface, which makes it a manufactured solution of the sigma-transformed
problem on a deformed surface.
"""
import numpy as np


def omega(k, h, g=9.81):
    """Linear dispersion relation omega^2 = g k tanh(kh)."""
    return np.sqrt(g * k * np.tanh(k * h))


def harmonic_phi(x, z, k, h):
    return np.cosh(k * (z + h)) / np.cosh(k * h) * np.sin(k * x)


def harmonic_w(x, z, k, h):
    """d/dz of harmonic_phi."""
    return k * np.sinh(k * (z + h)) / np.cosh(k * h) * np.sin(k * x)


def progressive(x, z, t, H, k, h, g=9.81):
    """Linear progressive wave of Sec. 4.2: (eta, phi)."""
    w = omega(k, h, g)
    c = w / k
    eta = 0.5 * H * np.cos(w * t - k * x)
    phi = -0.5 * H * c * np.cosh(k * (z + h)) / np.sinh(k * h) * np.sin(w * t - k * x)
    return eta, phi


def standing(x, z, t, H, k, h, g=9.81):
    """Linear standing wave (sum of two opposite progressive waves):
    eta = H/2 cos kx cos wt, phi = -(H g / 2w) cosh k(z+h)/cosh kh cos kx sin wt."""
    w = omega(k, h, g)
    eta = 0.5 * H * np.cos(k * x) * np.cos(w * t)
    phi = -(H * g / (2 * w)) * np.cosh(k * (z + h)) / np.cosh(k * h) * np.cos(k * x) * np.sin(w * t)
    return eta, phi
