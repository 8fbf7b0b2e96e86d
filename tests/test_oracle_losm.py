"""Pins of the oracle's deterministic pieces: the LOSM step (Sec. 3, Eqs.
losm-disc), the Thomas solve, the moving-average filter (Sec. 4) and the
window centres (Sec. 2, Eq. ww-center).  Not GPU."""
import math

import numpy as np
import pytest

from oracle import oracle as O


# ---------------------------------------------------------------- Thomas --
@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 401])
def test_thomas_matches_dense_solve(n):
    rng = np.random.default_rng(n)
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    b = 2.5 + rng.uniform(0, 1, n)
    d = rng.normal(size=n)
    A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    x = O.thomas(a, b, c, d)
    np.testing.assert_allclose(x, np.linalg.solve(A, d), rtol=1e-13, atol=1e-13)


def test_thomas_zero_pivot_is_an_error():
    with pytest.raises(O.OracleError):
        O.thomas([0, 1.0], [0.0, 1.0], [1.0, 0], [1.0, 1.0])


# ------------------------------------------------- manufactured solution --
# phi = (2 + cos kx) e^{-bt}, J = g sin(kx) e^{-bt}.  The source q and the
# closure F are chosen so that these solve the continuous LOSM equations
# (Eqs. balance, moment) exactly; the BCs give P_L, P_R.
K_, B_, G_ = 2.0, 0.7, 0.3
V_, ST_, SS_ = 1.3, 1.1, 0.6
XA, XB = -1.0, 1.5


def _exact(edges, t):
    sa = ST_ - SS_
    e = math.exp(-B_ * t)
    dx = np.diff(edges)
    avg_cos = (np.sin(K_ * edges[1:]) - np.sin(K_ * edges[:-1])) / (K_ * dx)
    A = G_ * (ST_ - B_ / V_) - K_ / 3.0
    phi_c = e * (2.0 + avg_cos)
    J_e = e * G_ * np.sin(K_ * edges)
    q_c = e * ((-B_ / V_ + sa) * (2.0 + avg_cos) + G_ * K_ * avg_cos)
    F_c = -(A / K_) * e * avg_cos
    F_pt = lambda x: -(A / K_) * e * math.cos(K_ * x)
    phi_pt = lambda x: e * (2.0 + math.cos(K_ * x))
    phi = np.concatenate([[phi_pt(edges[0])], phi_c, [phi_pt(edges[-1])]])
    F = np.concatenate([[F_pt(edges[0])], F_c, [F_pt(edges[-1])]])
    PL = J_e[0] + 0.5 * phi[0]
    PR = 0.5 * phi[-1] - J_e[-1]
    return phi, J_e, F, q_c, PL, PR


def _march(I, nsteps, theta, T=1.0):
    edges = np.linspace(XA, XB, I + 1)
    st = np.full(I, ST_)
    ss = np.full(I, SS_)
    dt = T / nsteps
    phi, J, F, q, _, _ = _exact(edges, 0.0)
    for n in range(1, nsteps + 1):
        phin_ex, Jn_ex, Fn, qn, PL, PR = _exact(edges, n * dt)
        phi, J = O.losm_step(edges, st, ss, V_, dt, theta, phi, J, F, Fn, PL, PR, 0.0, 0.0, q, qn)
        F, q = Fn, qn
    phi_ex, J_ex, *_ = _exact(edges, T)
    return np.abs(phi[1:-1] - phi_ex[1:-1]).max(), np.abs(J - J_ex).max()


def test_losm_crank_nicolson_second_order():
    errs = [_march(I, I // 2, 0.5) for I in (20, 40, 80, 160)]
    ep = np.array([e[0] for e in errs])
    ej = np.array([e[1] for e in errs])
    rate_p = np.log2(ep[:-1] / ep[1:])
    rate_j = np.log2(ej[:-1] / ej[1:])
    assert ep[-1] < 1e-3
    assert rate_p[-1] > 1.8 and rate_j[-1] > 1.8, (ep, ej)


def test_losm_backward_euler_first_order():
    errs = [_march(I, I // 2, 1.0) for I in (20, 40, 80, 160)]
    ep = np.array([e[0] for e in errs])
    rate = np.log2(ep[:-1] / ep[1:])
    assert 0.8 < rate[-1] < 1.3, ep


def test_losm_balance_identity():
    # Summing the balance rows telescopes the edge currents: the discrete
    # particle balance of the whole slab holds for any inputs.
    rng = np.random.default_rng(3)
    I = 37
    edges = np.cumsum(np.concatenate([[-2.0], rng.uniform(0.05, 0.2, I)]))
    st = rng.uniform(0.5, 2.0, I)
    ss = st * rng.uniform(0.1, 0.9, I)
    v, dt, th = 1.7, 0.13, 0.5
    phi_o = rng.uniform(0.1, 1.0, I + 2)
    J_o = rng.normal(size=I + 1) * 0.1
    F_o = rng.normal(size=I + 2) * 0.01
    F_n = rng.normal(size=I + 2) * 0.01
    q_o = rng.uniform(0, 1, I)
    q_n = rng.uniform(0, 1, I)
    phi, J = O.losm_step(edges, st, ss, v, dt, th, phi_o, J_o, F_o, F_n, 0.01, 0.02, 0.0, 0.0, q_o, q_n)
    dx = np.diff(edges)
    sa = st - ss
    lhs = (dx * (phi[1:-1] - phi_o[1:-1])).sum() / (v * dt) + th * (J[-1] - J[0] + (sa * dx * phi[1:-1]).sum())
    rhs = th * (q_n * dx).sum() + (th - 1.0) * (J_o[-1] - J_o[0] + (sa * dx * phi_o[1:-1]).sum() - (q_o * dx).sum())
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + abs(rhs) + 1.0)
    # and the two boundary relations hold
    assert abs(J[0] - (-0.5 * phi[0] + 0.01)) < 1e-14
    assert abs(J[-1] - (0.5 * phi[-1] - 0.02)) < 1e-14


def test_losm_uniform_state_decays_with_rational_factor():
    # No gradients and no closures: every cell follows the theta-rule
    # amplification factor of d phi/dt = -v sigma_a phi, away from the ends.
    I = 400
    edges = np.linspace(-200.0, 200.0, I + 1)
    st, ss = np.full(I, 1.0), np.full(I, 0.75)
    v, dt, th = 2.0, 0.1, 0.5
    phi_o = np.ones(I + 2)
    J_o = np.zeros(I + 1)
    Fz = np.zeros(I + 2)
    phi, J = O.losm_step(edges, st, ss, v, dt, th, phi_o, J_o, Fz, Fz, 0.5, 0.5)
    g = (1.0 / (v * dt) - (1 - th) * 0.25) / (1.0 / (v * dt) + th * 0.25)
    np.testing.assert_allclose(phi[150:250], g, rtol=1e-12)
    np.testing.assert_allclose(J[150:250], 0.0, atol=1e-12)


# ---------------------------------------------------------------- filter --
def test_ma_filter_properties():
    rng = np.random.default_rng(5)
    M, k = 57, 3
    chi = rng.normal(size=M)
    out = O.ma_filter(chi, k)
    # interior: the (2k+1)-point running mean
    run = np.convolve(chi, np.ones(2 * k + 1) / (2 * k + 1), mode="valid")
    np.testing.assert_allclose(out[k:M - k], run, rtol=1e-14, atol=1e-15)
    # ends are not filtered; the base shrinks symmetrically
    assert out[0] == chi[0] and out[-1] == chi[-1]
    assert abs(out[1] - chi[:3].mean()) < 1e-15
    assert abs(out[-3] - chi[-5:].mean()) < 1e-15
    # constants and linear functions are reproduced everywhere
    np.testing.assert_allclose(O.ma_filter(np.full(M, 2.5), k), 2.5, rtol=1e-15)
    lin = 0.3 * np.arange(1, M + 1) - 4.0
    np.testing.assert_allclose(O.ma_filter(lin, k), lin, rtol=1e-13, atol=1e-13)
    # quadratics gain k(k+1)/3 times the curvature in the interior
    quad = np.arange(1, M + 1, dtype=float) ** 2
    np.testing.assert_allclose(O.ma_filter(quad, k)[k:M - k], quad[k:M - k] + k * (k + 1) / 3.0, rtol=1e-13)
    # k = 0 is the identity
    np.testing.assert_array_equal(O.ma_filter(chi, 0), chi)


# --------------------------------------------------------------- windows --
def test_ww_centres():
    phi = np.array([-0.2, 0.0, 0.5, 2.0, 1.0, 1e-9])
    eps, s = 1e-3, 0.37
    ww = O.ww_centres(phi, eps, s)
    assert abs(ww[3] - s) <= 1e-16 * s * 4
    assert ww[0] == eps * s and ww[1] == eps * s  # negative values are clamped
    assert np.all(ww >= eps * s)
    np.testing.assert_allclose((ww / s - eps) / (1 - eps), np.clip(phi, 0, None) / 2.0, rtol=1e-12, atol=1e-15)
    with pytest.raises(O.OracleError):
        O.ww_centres(np.array([-1.0, 0.0]), eps, 1.0)


@pytest.mark.parametrize("M", [7, 64, 201, 400])
def test_fourier_filter_properties(M):
    rng = np.random.default_rng(M)
    x = rng.normal(size=M)
    # Every frequency kept: the identity.
    np.testing.assert_allclose(O.fourier_filter(x, M // 2 + 1), x, rtol=0, atol=1e-12)
    # Only the zero frequency kept: the mean everywhere.
    np.testing.assert_allclose(O.fourier_filter(x, 0), np.full(M, x.mean()), rtol=0, atol=1e-13)
    # The real low pass of numpy's FFT.
    for kappa in (1, 3, M // 4):
        X = np.fft.rfft(x)
        X[kappa + 1:] = 0.0
        np.testing.assert_allclose(O.fourier_filter(x, kappa), np.fft.irfft(X, n=M), rtol=0, atol=1e-12)


def test_fourier_filter_keeps_and_removes_single_modes():
    M = 120
    m = np.arange(1, M + 1)
    low = np.cos(2 * np.pi * 3 * m / M)
    high = 0.5 * np.sin(2 * np.pi * 9 * m / M)
    np.testing.assert_allclose(O.fourier_filter(low + high, 5), low, rtol=0, atol=1e-12)
    np.testing.assert_allclose(O.fourier_filter(low + high, 9), low + high, rtol=0, atol=1e-12)
