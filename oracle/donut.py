"""Exact moments of the donut target of Sec 7 (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline
may import this module.

Target on R^d: f(x) proportional to exp(-(|x|^2 - mu0)^2 / (2 sigma^2)).
In polar form the squared radius u = |x|^2 has density proportional to
exp(-(u - mu0)^2 / (2 sigma^2)) u^(d/2 - 1) on u > 0 (the surface of the
sphere of radius sqrt(u) grows like u^((d-1)/2) and dx = r^(d-1) dr dOmega,
du = 2 r dr), independent of the direction, which is uniform on the sphere.
So, for every coordinate i:

    E[x_i] = 0,  E[1(x_i > 0)] = 1/2           (symmetry x -> -x),
    E[x_i^2] = E[u] / d,                        (E[theta_i^2] = 1/d),
    E[x_i^4] = 3 E[u^2] / (d (d + 2))           (E[theta_i^4] = 3/(d(d+2))),

with E[u], E[u^2] by adaptive quadrature (scipy.integrate.quad).  For d = 2
these are E[u]/2 and 3 E[u^2]/8 (Sec 7 prints mu0^2/2 and 3/8 (mu0^4 +
sigma^2), garbled readings of mu0/2 and 3/8 (mu0^2 + sigma^2) when the
truncation of the radial law is negligible).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate


def radial_moments(d: int, mu0: float, sigma: float):
    """(E[u], E[u^2]) of u = |x|^2 under the donut target in d dimensions."""
    def dens(u, k):
        return np.exp(-(u - mu0) ** 2 / (2 * sigma ** 2)) * u ** (d / 2 - 1) * u ** k
    lo, hi = max(0.0, mu0 - 40 * sigma), mu0 + 40 * sigma
    pts = [min(max(mu0, lo), hi)]
    z = integrate.quad(dens, lo, hi, args=(0,), points=pts, epsabs=0, epsrel=1e-13, limit=500)[0]
    m1 = integrate.quad(dens, lo, hi, args=(1,), points=pts, epsabs=0, epsrel=1e-13, limit=500)[0]
    m2 = integrate.quad(dens, lo, hi, args=(2,), points=pts, epsabs=0, epsrel=1e-13, limit=500)[0]
    return m1 / z, m2 / z


def coordinate_moments(d: int, mu0: float, sigma: float) -> dict:
    """Exact E_pi of h = x_i, x_i^2, x_i^4 and 1(x_i > 0) (same for every i)."""
    Eu, Eu2 = radial_moments(d, mu0, sigma)
    return {"x": 0.0, "x2": Eu / d, "x4": 3.0 * Eu2 / (d * (d + 2)), "pos": 0.5}
