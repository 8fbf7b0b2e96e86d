"""Pins at first order in the collisions (not GPU).

First-collided flux: with sigma_t = v = 1 a unit isotropic plane pulse at
x = 0 collides at (x', t') at the rate of its uncollided flux
e^{-t'} / (2 t') on |x'| < t'; a fraction c of the collisions re-emits
isotropically, and a point emission's uncollided flux at distance d after a
time tau is e^{-tau} / (2 tau) for |d| < tau.  So the first-collided flux is

  phi_1(x, t) = (c/4) e^{-t} int_0^t |[-t', t'] n [x - (t - t'), x + (t - t')]|
                                   / (t' (t - t')) dt',

and the collided part of the reference pulse solution must equal phi_1 up
to O(c^2).

At most one collision: over one short step every source particle either
streams (probability e^{-s} of no collision before s), or collides once at
s, re-emits with probability c in a new isotropic direction and streams
for the rest of the step.  Track lengths per cell and the census weight
per cell of these histories are integrals in (s, tau) of the distribution
of mu s + mu' tau, two independent uniform variables, whose distribution
function is piecewise quadratic.  Histories with two or more collisions,
of probability 1 - e^{-dt}(1 + dt), are left out: a bound on their share
is added to the tolerance.
"""
import functools
import math

import numpy as np
import pytest
from scipy import integrate

import closed_forms as CF
from gpu_common import oracle_sim
from oracle import oracle as O
from paper_2512_19925_amd import pulse_reference as P
from paper_2512_19925_amd import workloads as W


# ------------------------------------------------- first-collided flux --
def first_collided(x, t, c):
    def overlap(tp):
        lo = max(-tp, x - (t - tp))
        hi = min(tp, x + (t - tp))
        return max(0.0, hi - lo)

    if abs(x) >= t:
        return 0.0
    kinks = sorted(k for k in ((t - abs(x)) / 2.0, (t + abs(x)) / 2.0) if 0.0 < k < t)
    val, err = integrate.quad(lambda tp: overlap(tp) / (tp * (t - tp)), 0.0, t, points=kinks or None,
                              limit=400, epsabs=0.0, epsrel=1e-12)
    assert err < 1e-9 * max(val, 1e-300)
    return 0.25 * c * math.exp(-t) * val


@pytest.mark.parametrize("x,t", [(0.0, 0.5), (0.3, 1.0), (-1.2, 2.0), (2.5, 3.0), (0.05, 4.0)])
def test_reference_collided_flux_is_first_collided_to_first_order(x, t):
    # The remainder collided - phi_1 is the flux of two or more collisions:
    # positive and of order c^2 (ratio ~4 when c doubles).  A wrong factor
    # in either makes the remainder first order (ratio ~2).
    r = []
    for c in (0.01, 0.02):
        coll = float(P.collided_flux(np.array([x]), t, c)[0])
        f1 = first_collided(x, t, c)
        assert f1 > 0.0
        r.append(coll - f1)
        assert 0.0 < r[-1] < 4.0 * c * f1, (c, coll, f1)
    assert 3.6 < r[1] / r[0] < 4.4, r


def test_first_collided_total_weight():
    # int phi_1 dx = c t e^{-t} (every collision before t re-emits c, and the
    # emitted particles stream without a further collision until t).
    for t in (0.5, 2.0):
        xs, ws = np.polynomial.legendre.leggauss(200)
        # The integrand has kinks where the source interval meets the cone.
        tot = 0.0
        for lo, hi in ((-t, 0.0), (0.0, t)):
            x = 0.5 * (hi - lo) * (xs + 1.0) + lo
            tot += 0.5 * (hi - lo) * sum(w * first_collided(float(xi), t, 1.0) for xi, w in zip(x, ws))
        assert abs(tot / (t * math.exp(-t)) - 1.0) < 1e-4


# --------------------------------------------------- <= 1 collision --
def _px(t, a, b):
    """P(mu t in [a, b]), mu uniform on [-1, 1]."""
    return 0.5 * (np.clip(b / t, -1.0, 1.0) - np.clip(a / t, -1.0, 1.0))


def _sum_cdf(z, s, tau):
    """P(mu s + mu' tau <= z) for independent mu, mu' uniform on [-1, 1]."""
    def r(u):
        return 0.5 * np.maximum(u, 0.0) ** 2
    return (r(z + s + tau) - r(z + s - tau) - r(z - s + tau) + r(z - s - tau)) / (4.0 * s * tau)


@functools.lru_cache(maxsize=None)
def _leggauss(n):
    return np.polynomial.legendre.leggauss(n)


def _gl(lo, hi, n):
    x, w = _leggauss(n)
    return 0.5 * (hi - lo) * (x + 1.0) + lo, 0.5 * (hi - lo) * w


def one_collision_expectations(edges, dt, c, kept_direction=False):
    """Per source particle: track length per cell and census weight per cell
    of the histories with at most one collision (sigma_t = v = 1).
    kept_direction: the same for a scatter that keeps the incoming direction
    (a wrong collision, to show the test's power)."""
    I = len(edges) - 1
    track = np.zeros(I)
    census = np.zeros(I)
    kinks = sorted({abs(e) for e in edges if 0.0 < abs(e) < dt} | {0.0, dt})
    for i in range(I):
        a, b = edges[i], edges[i + 1]
        # Uncollided: the path until the first collision or the step's end.
        for lo, hi in zip(kinks[:-1], kinks[1:]):
            t, w = _gl(lo, hi, 64)
            track[i] += np.sum(w * np.exp(-t) * _px(t, a, b))
        census[i] += math.exp(-dt) * _px(dt, a, b)
        if kept_direction:
            continue
        # One collision at s, re-emission with probability c, then the rest
        # of the step without a further collision.
        s, ws = _gl(0.0, dt, 400)
        u, wu = _gl(0.0, 1.0, 400)
        S = s[:, None]
        tau = (dt - S) * u[None, :]
        wgt = ws[:, None] * (dt - S) * wu[None, :]
        pr = _sum_cdf(b, S, tau) - _sum_cdf(a, S, tau)
        track[i] += c * np.sum(wgt * np.exp(-S - tau) * pr)
        census[i] += c * math.exp(-dt) * np.sum(ws * (_sum_cdf(b, s, dt - s) - _sum_cdf(a, s, dt - s)))
    if kept_direction:
        # A particle that keeps its direction is at mu t at every t: its
        # track and census are the uncollided ones with the no-collision
        # factor of the scattered part added.
        for i in range(I):
            a, b = edges[i], edges[i + 1]
            for lo, hi in zip(kinks[:-1], kinks[1:]):
                t, w = _gl(lo, hi, 64)
                track[i] += c * np.sum(w * t * np.exp(-t) * _px(t, a, b))
            census[i] += c * dt * math.exp(-dt) * _px(dt, a, b)
    return track, census


def test_expectations_add_up():
    # Total track: int_0^dt e^{-t} (1 + c t) dt; total census weight:
    # e^{-dt} (1 + c dt): the <= 1 collision parts of the exact totals.
    dt, c = 0.02, 0.9
    edges = np.linspace(-dt, dt, 9)
    tr, ce = one_collision_expectations(edges, dt, c)
    exact_tr = (1.0 - math.exp(-dt)) + c * (1.0 - math.exp(-dt) * (1.0 + dt))
    assert abs(tr.sum() / exact_tr - 1.0) < 1e-6
    assert abs(ce.sum() / (math.exp(-dt) * (1.0 + c * dt)) - 1.0) < 1e-6
    np.testing.assert_allclose(tr, tr[::-1], rtol=1e-10)
    np.testing.assert_allclose(ce, ce[::-1], rtol=1e-10)


def test_oracle_at_most_one_collision():
    # One step of dt = 0.02 mean free times, c = 0.9, 4e6 particles from the
    # pulse, 8 cells across the reach [-dt, dt] (no particle can leave).
    dt, c, N = 0.02, 0.9, 4_000_000
    w = W.homogeneous("one-collision", -dt, dt, 8, 1.0, c, dt=dt, n_steps=1, n_src=N,
                      n_batches=32, bank_capacity=2 * N, seed=11)
    sim = oracle_sim(w)
    O.run(sim, 1, None)
    cells, bnd = sim.tallies()
    assert np.all(bnd == 0.0)
    edges = w.edges
    ex_tr, ex_ce = one_collision_expectations(edges, dt, c)
    # Left out: the track after a second collision (at most c^2 of the
    # probability of two collisions times the time left) and the census
    # weight of particles that collided twice and survived.
    p2 = 1.0 - math.exp(-dt) * (1.0 + dt)
    bias_tr = c * c * p2 * dt
    bias_ce = c * c * p2
    zs = []
    for k, ex, bias in ((O.T_PHI, ex_tr, bias_tr), (3, ex_ce, bias_ce)):
        per = cells[..., k] / N
        tot = per.sum(0)
        sig = CF.batch_sigma(per)
        assert np.all(sig > 0)
        d = tot - ex
        assert np.all(np.abs(d) < 4.5 * sig + bias), (k, d / sig)
        zs.append(d / sig)
    z = np.concatenate(zs)
    assert float(np.mean(z * z)) < 2.5, z
    # The same data reject a collision that keeps the incoming direction.
    kt, kc = one_collision_expectations(edges, dt, c, kept_direction=True)
    zk = np.concatenate([(cells[..., k].sum(0) / N - ex) / CF.batch_sigma(cells[..., k] / N)
                         for k, ex in ((O.T_PHI, kt), (3, kc))])
    assert float(np.max(np.abs(zk))) > 8.0, zk
