"""Pins of the oracle's hand-over from tallies to the HLOSM solve (Sec. 3):
the initial condition and closures it assembles (Eqs. F, F_i-n, ct-mc,
losm-disc-bc, Hpn) and the closure index of the deterministic LOSM march
(Eq. losm-disc).  Not GPU.

The closures are checked against the closed-form uncollided solution
(c = 0), on a mesh of unequal cells whose faces the particles reach, with the
pulse off the centre so that the two faces differ.  Each oracle output is
averaged over independent replicas (different seeds) and compared with the
exact value through its standard error:
  - cell averages of phi at the time layer (Eq. ct-mc) and of
    F = phi/3 - K (Eq. F);
  - edge currents: inside the light cone J = x phi / (v t) is linear in x,
    so the linear interpolation of exact cell averages (weighted by the
    opposite cell's width) is the exact point value;
  - face values (edge-crossing tallies averaged over the step) of phi, F and
    P = phi/2 - |J|, and the boundary currents J_0 = -phi_0/2 + P_L,
    J_I = phi_{I+1}/2 - P_R (Eq. losm-disc-bc);
  - the closures of a fully implicit update after the first chunks of a
    step, scaled by the start weight over the weight swept (Eq. Hpn).
The march is checked against a smooth source-free manufactured solution of
the LOSM equations with time-dependent closures: second-order convergence
for Crank-Nicolson, first order for backward Euler.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O

# ----------------------------------------------------------- c = 0 problem --
# Cells alternate 0.1 and 0.3 wide on [-2, 2]; the pulse sits at 0.45, so the
# right face (1.55 away) starts leaking at t = 1.55 and the left one (2.45
# away) at t = 2.45, both before the last step ends at t = 3.
XS, V, ST, DT, NSTEPS = 0.45, 1.0, 1.0, 0.25, 12
N_SRC, N_REP = 20000, 24
EDGES = np.concatenate([[-2.0], -2.0 + np.cumsum(np.tile([0.1, 0.3], 10))])
EDGES[-1] = 2.0
I_C = len(EDGES) - 1


def _sim(seed, n_chunks=4):
    return O.OracleSim(EDGES, np.full(I_C, ST), np.zeros(I_C), V, DT, NSTEPS, XS, N_SRC,
                       bank_capacity=2 * N_SRC, seed=seed, replica=0, n_batches=8, n_chunks=n_chunks)


def _cell_avg(a, b, t):
    """Cell averages of (phi, J, K) of the uncollided pulse at time t."""
    lo, hi = max(a - XS, -V * t), min(b - XS, V * t)
    if hi <= lo:
        return 0.0, 0.0, 0.0
    s = math.exp(-ST * V * t) / (2.0 * t)
    return (s * (hi - lo) / (b - a), s * (hi * hi - lo * lo) / (2.0 * V * t) / (b - a),
            s * (hi ** 3 - lo ** 3) / (3.0 * (V * t) ** 2) / (b - a))


def _face_avg(x, t0, t1):
    """Step averages over [t0, t1] of (phi, J, P, F) at a face x: one
    direction mu = (x - XS) / (v t) reaches it, with flux exp(-t)/(2t)."""
    d = abs(x - XS)
    ta = max(t0, d / V)
    if ta >= t1:
        return 0.0, 0.0, 0.0, 0.0

    def f(t, k):
        mu = (x - XS) / (V * t)
        s = math.exp(-ST * V * t) / (2.0 * t)
        return (s, mu * s, (0.5 - abs(mu)) * s, (1.0 / 3.0 - mu * mu) * s)[k]
    return tuple(integrate.quad(f, ta, t1, args=(k,), epsabs=1e-15, epsrel=1e-13)[0] / (t1 - t0)
                 for k in range(4))


def _exact_inputs(t_layer, t0, t1):
    """Exact (phi_o, J_o, F_o, P, mask of J_o entries that are exact) for the
    time layer t_layer and faces averaged over the step [t0, t1]."""
    I = I_C
    phi, J, F = np.zeros(I + 2), np.zeros(I + 1), np.zeros(I + 2)
    jmask = np.zeros(I + 1, bool)
    for i in range(I):
        p, _, k = _cell_avg(EDGES[i], EDGES[i + 1], t_layer)
        phi[i + 1] = p
        F[i + 1] = p / 3.0 - k
    inside = [max(abs(EDGES[i] - XS), abs(EDGES[i + 1] - XS)) <= V * t_layer for i in range(I)]
    for i in range(1, I):
        if inside[i - 1] and inside[i]:
            x = EDGES[i] - XS
            J[i] = x / (V * t_layer) * math.exp(-ST * V * t_layer) / (2.0 * t_layer)
            jmask[i] = True
    fl = _face_avg(EDGES[0], t0, t1)
    fr = _face_avg(EDGES[-1], t0, t1)
    phi[0], phi[-1] = fl[0], fr[0]
    F[0], F[-1] = fl[3], fr[3]
    J[0], J[-1] = fl[1], fr[1]
    jmask[0] = jmask[-1] = True
    return phi, J, F, np.array([fl[2], fr[2]]), jmask


def _replica_runs(collect, n_chunks=4):
    """collect(sim, step, chunk) -> dict of arrays, after every chunk of every
    step; returns {(step, chunk, key): array [N_REP, ...]}."""
    out = {}
    for r in range(N_REP):
        sim = _sim(seed=100 + r, n_chunks=n_chunks)
        for n in range(1, NSTEPS + 1):
            for p in range(n_chunks):
                sim.sweep(n, p)
                for k, v in collect(sim, n, p).items():
                    out.setdefault((n, p, k), []).append(v)
        sim.close()
    return {k: np.array(v) for k, v in out.items()}


def _z(samples, exact, mask=None):
    m = samples.mean(0)
    se = samples.std(0, ddof=1) / math.sqrt(samples.shape[0])
    ok = se > 0
    if mask is not None:
        ok &= mask
    # Entries with no spread (cells and faces no particle reaches) must be
    # exactly zero, up to the rounding of the closed form at the front.
    flat = ~(se > 0) & (mask if mask is not None else True)
    assert np.all(np.abs(m[flat] - exact[flat]) <= 1e-12 * (np.abs(exact).max() + 1e-300)), (m[flat], exact[flat])
    return (m[ok] - exact[ok]) / se[ok]


def _check_z(zs, what):
    z = np.concatenate(zs)
    assert len(z) > 50, what
    frac3 = np.mean(np.abs(z) > 3.0)
    assert np.max(np.abs(z)) < 6.0, (what, np.max(np.abs(z)))
    assert frac3 <= 0.03, (what, frac3)
    assert 0.6 < np.mean(z * z) < 1.6, (what, np.mean(z * z))


@pytest.fixture(scope="module")
def semi_runs():
    def collect(sim, n, p):
        if p != sim.n_chunks - 1:
            return {}
        phi_o, J_o, F_o, F_n, P = sim.losm_inputs(implicit=False)
        return {"phi": phi_o, "J": J_o, "F": F_o, "Fn": F_n, "P": P}
    return _replica_runs(collect)


@pytest.fixture(scope="module")
def implicit_runs():
    def collect(sim, n, p):
        if p == sim.n_chunks - 1 or n < 2:
            return {}
        res = sim.losm_inputs(implicit=True)
        assert res is not None
        phi_o, J_o, F_o, F_n, P = res
        return {"phi": phi_o, "J": J_o, "F": F_o, "Fn": F_n, "P": P}
    return _replica_runs(collect)


def test_semi_implicit_inputs_match_closed_form(semi_runs):
    zp, zj, zf, zb = [], [], [], []
    for n in range(2, NSTEPS + 1):
        t = n * DT
        phi, J, F, P, jm = _exact_inputs(t, t - DT, t)
        g = {k: semi_runs[(n, 3, k)] for k in ("phi", "J", "F", "Fn", "P")}
        # the lagged closures of the semi-implicit solve are the time layer's
        np.testing.assert_array_equal(g["Fn"], g["F"])
        zp.append(_z(g["phi"], phi))
        zj.append(_z(g["J"], J, jm))
        zf.append(_z(g["F"], F))
        zb.append(_z(g["P"], P))
    _check_z(zp, "phi")
    _check_z(zj, "J")
    _check_z(zf, "F")
    zb = np.concatenate(zb)
    assert len(zb) >= 8 and np.max(np.abs(zb)) < 4.5, zb


def test_face_closures_distinguish_the_faces(semi_runs):
    # The right face leaks from t = 1.55, the left from t = 2.45: in step 9
    # (t in [2, 2.25]) only the right face has crossings.
    P = semi_runs[(9, 3, "P")].mean(0)
    phi = semi_runs[(9, 3, "phi")].mean(0)
    assert P[0] == 0.0 and phi[0] == 0.0
    assert P[1] != 0.0 and phi[-1] > 0.0


def test_implicit_inputs_match_closed_form(implicit_runs):
    # After chunk p of step n: initial condition of the time layer t^{n-1}
    # (faces of step n-1), closures of t^n from the chunks swept so far,
    # scaled by W_start / W_done.
    zic, zcl = [], []
    for n in range(3, NSTEPS + 1):
        t = n * DT
        phi_o, J_o, F_o, _, jm_o = _exact_inputs(t - DT, t - 2 * DT, t - DT)
        _, _, F_n, P_n, _ = _exact_inputs(t, t - DT, t)
        for p in range(3):
            g = {k: implicit_runs[(n, p, k)] for k in ("phi", "J", "F", "Fn", "P")}
            zic += [_z(g["phi"], phi_o), _z(g["J"], J_o, jm_o), _z(g["F"], F_o)]
            zcl += [_z(g["Fn"], F_n), _z(g["P"], P_n)]
    _check_z(zic, "initial condition")
    _check_z(zcl, "scaled partial closures")


def test_implicit_inputs_need_swept_weight():
    # Chunk membership comes from the particle's own draws: with 4 chunks and
    # a single source particle, some chunk of step 1 holds no start weight.
    sim = O.OracleSim(EDGES, np.full(I_C, ST), np.zeros(I_C), V, DT, 3, XS, 1, bank_capacity=64, seed=1,
                      n_batches=1, n_chunks=8)
    seen_none = seen_some = False
    for p in range(7):
        sim.sweep(1, p)
        r = sim.losm_inputs(implicit=True)
        seen_none |= r is None
        seen_some |= r is not None
    assert seen_none and seen_some


def test_closures_read_equals_semi_implicit_inputs(semi_runs):
    sim = _sim(seed=100)
    for n in range(1, 4):
        for p in range(4):
            sim.sweep(n, p)
    F, P, phi, J = sim.closures()
    np.testing.assert_array_equal(F, semi_runs[(3, 3, "F")][0])
    np.testing.assert_array_equal(P, semi_runs[(3, 3, "P")][0])
    np.testing.assert_array_equal(phi, semi_runs[(3, 3, "phi")][0])
    np.testing.assert_array_equal(J, semi_runs[(3, 3, "J")][0])


def test_solve_is_the_step_of_its_filtered_inputs():
    # The solve runs the pinned LOSM step on the pinned inputs, after the
    # filter of Sec. 4 on F (both levels, cells), phi (cells) and J (edges).
    sim = _sim(seed=7)
    for n in range(1, 3):
        for p in range(4):
            sim.sweep(n, p)
    for filt, k in ((0, 3), (1, 3), (1, 1)):
        phi_o, J_o, F_o, F_n, P = sim.losm_inputs(implicit=False)
        if filt == 1:
            phi_o[1:-1] = O.ma_filter(phi_o[1:-1], k)
            F_o[1:-1] = O.ma_filter(F_o[1:-1], k)
            F_n[1:-1] = O.ma_filter(F_n[1:-1], k)
            J_o = O.ma_filter(J_o, k)
        for theta in (0.5, 1.0):
            want = O.losm_step(EDGES, np.full(I_C, ST), np.zeros(I_C), V, DT, theta, phi_o, J_o, F_o, F_n,
                               P[0], P[1])
            got = sim.solve_losm(O.LosmOpts(theta=theta, filter=filt, ma_k=k), implicit=False,
                                 apply_windows=False)
            np.testing.assert_array_equal(got[0], want[0])
            np.testing.assert_array_equal(got[1], want[1])


# ------------------------------------------- march: manufactured solution --
# phi = e^{-bt}(2 + cos kx) and J = a e^{-bt}(2x + sin(kx)/k) with
# a = b/v - sigma_a solve the balance equation without a source; the first
# moment equation (1/v) J_t + phi_x / 3 + sigma_t J = F_x then fixes
# F = e^{-bt}[beta (x^2 - cos(kx)/k^2) + cos(kx)/3], beta = a (sigma_t - b/v).
# The vacuum-boundary rows take P_L = J(x_0) + phi(x_0)/2 and
# P_R = phi(x_I)/2 - J(x_I) at the new time level.
MK, MB, MV, MST, MSS = 2.0, 1.5, 1.3, 1.1, 0.6
MA_ = MB / MV - (MST - MSS)
MBETA = MA_ * (MST - MB / MV)
MXA, MXB = -1.0, 1.5


def _mms(edges, t):
    e = math.exp(-MB * t)
    a, b = edges[:-1], edges[1:]
    dx = b - a
    s_avg = (np.sin(MK * b) - np.sin(MK * a)) / (MK * dx)
    phi_pt = lambda x: e * (2.0 + math.cos(MK * x))
    F_pt = lambda x: e * (MBETA * (x * x - math.cos(MK * x) / MK ** 2) + math.cos(MK * x) / 3.0)
    phi = np.concatenate([[phi_pt(edges[0])], e * (2.0 + s_avg), [phi_pt(edges[-1])]])
    F_c = e * (MBETA * ((b ** 3 - a ** 3) / (3.0 * dx) - s_avg / MK ** 2) + s_avg / 3.0)
    F = np.concatenate([[F_pt(edges[0])], F_c, [F_pt(edges[-1])]])
    J = MA_ * e * (2.0 * edges + np.sin(MK * edges) / MK)
    P = np.array([J[0] + 0.5 * phi[0], 0.5 * phi[-1] - J[-1]])
    return phi, J, F, P


def _march_error(I, n_steps, theta, T=1.0):
    edges = np.linspace(MXA, MXB, I + 1)
    dt = T / n_steps
    sol = [_mms(edges, n * dt) for n in range(n_steps + 1)]
    F = np.array([s[2] for s in sol])
    P = np.array([s[3] for s in sol])
    phi, J = O.losm_march(edges, np.full(I, MST), np.full(I, MSS), MV, dt, theta, F, P, sol[0][0], sol[0][1])
    return (max(np.abs(phi[n, 1:-1] - sol[n][0][1:-1]).max() for n in range(n_steps + 1)),
            max(np.abs(J[n] - sol[n][1]).max() for n in range(n_steps + 1)))


def test_march_manufactured_crank_nicolson_second_order():
    errs = np.array([_march_error(I, I // 2, 0.5) for I in (20, 40, 80, 160)])
    rates = np.log2(errs[:-1] / errs[1:])
    assert errs[-1, 0] < 2e-4, errs
    assert np.all(rates[-1] > 1.8), (errs, rates)


def test_march_manufactured_backward_euler_first_order():
    errs = np.array([_march_error(I, I // 2, 1.0) for I in (20, 40, 80, 160)])
    rates = np.log2(errs[:-1] / errs[1:])
    assert np.all((rates[-1] > 0.8) & (rates[-1] < 1.3)), (errs, rates)
