"""Reference scalar flux of the isotropic plane pulse in an infinite
homogeneous medium (one speed, isotropic scattering, scattering ratio c):
the benchmark solution that the paper's figure of merit FOM_Error measures
the Monte Carlo flux against (Sec. 5.1; Sec. 5, Eq. FOM_error).

A unit pulse at x = 0, t = 0.  With sigma_t = v = 1 (distances in mean free
paths, time in mean free times) and eta = x / t, the flux inside the
light cone |eta| < 1 is the known closed form of the plane-source problem

    phi(x, t) = e^{-t} / (2 t) * [1 + (c t / (4 pi)) (1 - eta^2)
                 * int_0^pi sec^2(u/2) Re( xi^2 exp((c t / 2)(1 - eta^2) xi) ) du],
    xi(u) = (ln q + i u) / (eta + i tan(u/2)),   q = (1 + eta) / (1 - eta),

and zero outside.  The first term is the uncollided flux.  Other sigma_t and
v follow by scaling: phi(x, t) = sigma_t v phi_1(sigma_t x, sigma_t v t).

Everything here is plain numpy quadrature on the host.  It is not part of
the sweep.  Its accuracy is pinned in tests against the exact total weight
and second spatial moment, the c -> 0 limit and the Monte Carlo oracle.
"""
from __future__ import annotations

import numpy as np

_U_NODES = 192


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


_UX, _UW = _gauss(_U_NODES)


def collided_flux(x, t, c):
    """Collided part of phi (sigma_t = v = 1) at points x (array) and time t > 0."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    if c == 0.0 or t <= 0.0:
        return out
    eta = x / t
    m = np.abs(eta) < 1.0
    if not np.any(m):
        return out
    e = eta[m][:, None]
    u = (0.5 * np.pi) * (_UX + 1.0)[None, :]          # Gauss-Legendre nodes on (0, pi)
    wu = (0.5 * np.pi) * _UW[None, :]
    q = (1.0 + e) / (1.0 - e)
    tan_h = np.tan(0.5 * u)
    xi = (np.log(q) + 1j * u) / (e + 1j * tan_h)
    sec2 = 1.0 + tan_h * tan_h
    a = 0.5 * c * t * (1.0 - e * e)
    integrand = sec2 * np.real(xi * xi * np.exp(a * xi))
    integral = (integrand * wu).sum(axis=1)
    pref = np.exp(-t) / (2.0 * t) * (c * t / (4.0 * np.pi)) * (1.0 - eta[m] ** 2)
    out[m] = pref * integral
    return out


def flux(x, t, c):
    """Total phi (sigma_t = v = 1) at points x and time t > 0."""
    x = np.asarray(x, dtype=np.float64)
    unc = np.where(np.abs(x) < t, np.exp(-t) / (2.0 * t), 0.0)
    return unc + collided_flux(x, t, c)


def _uncollided_cell_time(a, b, t0, t1, nt):
    """Cell [a, b] x step [t0, t1] integral of e^{-t}/(2t) 1{|x| < t}
    (sigma_t = v = 1): integral over t of e^{-t}/(2t) |[a,b] n (-t,t)|,
    with Gauss-Legendre pieces split where the overlap length has kinks."""
    cuts = sorted({t0, t1, *[tc for tc in (abs(a), abs(b)) if t0 < tc < t1]})
    gx, gw = _gauss(nt)
    total = 0.0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        tt = 0.5 * (hi - lo) * (gx + 1.0) + lo
        ww = 0.5 * (hi - lo) * gw
        ov = np.clip(np.minimum(b, tt) - np.maximum(a, -tt), 0.0, None)
        total += float(np.sum(ww * np.exp(-tt) / (2.0 * tt) * ov))
    return total


def cell_step_averages(edges, dt, n_steps, c, sigma_t=1.0, v=1.0, nx=12, nt=12):
    """Averages of phi over every cell [edges[i], edges[i+1]] and every time
    step [(n-1) dt, n dt], n = 1..n_steps (what the track-length tally of
    step n estimates per source particle).  Returns [n_steps, I]."""
    edges = np.asarray(edges, dtype=np.float64)
    I = len(edges) - 1
    out = np.zeros((n_steps, I))
    gx, gw = _gauss(nx)
    tx, tw = _gauss(nt)
    s = sigma_t * v
    for n in range(1, n_steps + 1):
        t0, t1 = s * (n - 1) * dt, s * n * dt      # scaled times
        tt = 0.5 * (t1 - t0) * (tx + 1.0) + t0
        ttw = 0.5 * (t1 - t0) * tw
        for i in range(I):
            a, b = sigma_t * edges[i], sigma_t * edges[i + 1]   # scaled positions
            if min(abs(a), abs(b)) >= t1 and a * b > 0:
                continue                                        # not reached yet
            val = _uncollided_cell_time(a, b, t0, t1, nt)
            if c > 0.0:
                for tk, wk in zip(tt, ttw):
                    lo, hi = max(a, -tk), min(b, tk)
                    if hi <= lo:
                        continue
                    xx = 0.5 * (hi - lo) * (gx + 1.0) + lo
                    val += wk * float(np.sum(0.5 * (hi - lo) * gw * collided_flux(xx, tk, c)))
            # Back to physical units: phi = s phi_1; averages over the
            # physical cell and step divide by dx dt = (b - a)(t1 - t0) / (sigma_t s).
            out[n - 1, i] = s * val / ((b - a) * (t1 - t0))
    return out
