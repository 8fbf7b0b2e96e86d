"""Pins of the oracle's LOSM march and its adjoint gradient (not GPU):
central finite differences (h = 1e-6, FP64) and a fourth-order stencil."""
import numpy as np
import pytest

from oracle import oracle as O


def _problem(I=40, N=10, seed=3):
    rng = np.random.default_rng(seed)
    edges = np.linspace(-2.0, 2.0, I + 1)
    st = rng.uniform(0.5, 2.0, I)
    ss = st * rng.uniform(0.5, 0.95, I)
    x = 0.5 * (edges[1:] + edges[:-1])
    F = np.zeros((N + 1, I + 2))
    for n in range(N + 1):
        F[n, 1:-1] = 0.05 * np.exp(-x ** 2) * np.cos(0.3 * n + x)
        F[n, 0], F[n, -1] = 0.01, -0.02
    P = np.full((N + 1, 2), 0.003)
    phi0 = np.concatenate([[0.0], np.exp(-4 * x ** 2), [0.0]])
    J0 = np.zeros(I + 1)
    J0[1:-1] = 0.1 * np.sin(x[1:] + x[:-1])
    w = np.zeros((N + 1, I + 2))
    w[:, 1 + I // 2: 1 + 3 * I // 4] = 0.05
    w[1:-1] *= 2.0
    return edges, st, ss, F, P, phi0, J0, w


def _G(edges, st, ss, F, P, phi0, J0, w, theta=0.5, v=1.0, dt=0.25):
    phi, J = O.losm_march(edges, st, ss, v, dt, theta, F, P, phi0, J0)
    return float((w * phi).sum())


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_adjoint_gradient_matches_central_differences(theta):
    edges, st, ss, F, P, phi0, J0, w = _problem()
    phi, J = O.losm_march(edges, st, ss, 1.0, 0.25, theta, F, P, phi0, J0)
    gt, gs = O.losm_adjoint(edges, st, ss, 1.0, 0.25, theta, phi, J, w)
    h = 1e-6
    big = max(np.abs(gt).max(), np.abs(gs).max())
    G0 = abs(_G(edges, st, ss, F, P, phi0, J0, w, theta))
    # Central differences carry truncation O(h^2) and roundoff of about
    # eps |G| / h: relative 1e-6 is asked where the component is far above
    # that roundoff, the roundoff bound everywhere.
    round_off = 16 * np.finfo(float).eps * G0 / h
    for i in range(len(st)):
        for arr, g in ((st, gt), (ss, gs)):
            p = arr.copy(); p[i] += h
            m = arr.copy(); m[i] -= h
            if arr is st:
                fd = (_G(edges, p, ss, F, P, phi0, J0, w, theta) - _G(edges, m, ss, F, P, phi0, J0, w, theta)) / (2 * h)
            else:
                fd = (_G(edges, st, p, F, P, phi0, J0, w, theta) - _G(edges, st, m, F, P, phi0, J0, w, theta)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * abs(g[i]) + round_off, (i, fd, g[i], round_off)
            if abs(g[i]) > 1e6 * round_off:
                assert abs(fd - g[i]) <= 2e-6 * abs(g[i]), (i, fd, g[i])


def test_adjoint_fourth_order_stencil_and_sum_identity():
    # Five-point stencil (truncation O(h^4)) along a random direction in both
    # cross sections; and sigma_t, sigma_s moved together (sigma_a fixed)
    # sees only the half-cell cross sections of the first-moment equations.
    edges, st, ss, F, P, phi0, J0, w = _problem(I=30, N=8, seed=5)
    phi, J = O.losm_march(edges, st, ss, 1.0, 0.25, 0.5, F, P, phi0, J0)
    gt, gs = O.losm_adjoint(edges, st, ss, 1.0, 0.25, 0.5, phi, J, w)
    rng = np.random.default_rng(9)
    dt_, ds_ = rng.normal(size=len(st)), rng.normal(size=len(st))
    G = lambda e: _G(edges, st + e * dt_, ss + e * ds_, F, P, phi0, J0, w)
    h = 1e-3
    fd = (-G(2 * h) + 8 * G(h) - 8 * G(-h) + G(-2 * h)) / (12 * h)
    exact = gt @ dt_ + gs @ ds_
    assert abs(fd - exact) <= 1e-9 * (abs(exact) + 1e-12)
    Gs = lambda e: _G(edges, st + e * dt_, ss + e * dt_, F, P, phi0, J0, w)
    fd2 = (-Gs(2 * h) + 8 * Gs(h) - 8 * Gs(-h) + Gs(-2 * h)) / (12 * h)
    assert abs(fd2 - (gt + gs) @ dt_) <= 1e-9 * (abs(fd2) + 1e-12)
