"""Closed-form solutions of the isotropic plane pulse in an infinite
homogeneous slab (one speed, isotropic scattering), used to pin the oracle.

Uncollided flux (c = 0): a unit pulse at x = 0, t = 0 puts the surviving
particles at x = mu v t with mu uniform on [-1, 1], so per source particle
    phi(x, t) = exp(-sigma_t v t) / (2 t)   for |x| < v t,
    J = (x / (v t)) phi,   K = (x / (v t))^2 phi.
Spatial moments for any 0 < c <= 1 follow from the angular-moment equations
of the transport equation (sigma_t = v = 1):
    d/dt int phi = -(1 - c) int phi
    d/dt int K   = -int K + (c / 3) int phi           -> int K = int phi / 3
    d/dt int xJ  = int K - int xJ
    d/dt int x^2 phi = 2 int xJ - (1 - c) int x^2 phi
with the isotropic start int phi = 1, int K = 1/3, int xJ = int x^2 phi = 0.
"""
import math

import numpy as np
from scipy import integrate


def _overlap(a, b, lo, hi):
    return max(a, lo), min(b, hi)


def uncollided_cell_time_avg(a, b, t0, t1, sigma_t, v):
    """Cell [a,b] x step [t0,t1] averages of (phi, J, K), per source particle."""
    def f(t, k):
        if t <= 0.0:
            return 0.0
        lo, hi = _overlap(a, b, -v * t, v * t)
        if hi <= lo:
            return 0.0
        s = math.exp(-sigma_t * v * t) / (2.0 * t)
        if k == 0:
            return s * (hi - lo)
        if k == 1:
            return s * (hi * hi - lo * lo) / (2.0 * v * t)
        return s * (hi ** 3 - lo ** 3) / (3.0 * (v * t) ** 2)
    pts = [t for t in (abs(a) / v, abs(b) / v) if t0 < t < t1]
    out = []
    for k in range(3):
        val, _ = integrate.quad(f, t0, t1, args=(k,), points=pts or None, limit=200,
                                epsabs=1e-14, epsrel=1e-12)
        out.append(val / ((t1 - t0) * (b - a)))
    return out


def uncollided_cell_avg(a, b, t, sigma_t, v):
    """Cell [a,b] averages of (phi, J, K) at time t, per source particle."""
    lo, hi = _overlap(a, b, -v * t, v * t)
    if hi <= lo:
        return [0.0, 0.0, 0.0]
    s = math.exp(-sigma_t * v * t) / (2.0 * t)
    return [s * (hi - lo) / (b - a),
            s * (hi * hi - lo * lo) / (2.0 * v * t) / (b - a),
            s * (hi ** 3 - lo ** 3) / (3.0 * (v * t) ** 2) / (b - a)]


def moments(c, t):
    """(int phi, int K, int xJ, int x^2 phi) at time t for sigma_t = v = 1."""
    m0 = math.exp(-(1.0 - c) * t)
    k = m0 / 3.0
    xj = (m0 - math.exp(-t)) / (3.0 * c)
    x2 = (2.0 / (3.0 * c)) * m0 * (t - (1.0 - math.exp(-c * t)) / c)
    return m0, k, xj, x2


def batch_sigma(per_batch):
    """Standard deviation of the sum over batches, from the batch spread."""
    B = per_batch.shape[0]
    tot = per_batch.sum(0)
    return np.sqrt(B / (B - 1.0) * ((per_batch - tot / B) ** 2).sum(0))
