"""Pins of the oracle's fission collisions and uniform combing (the paper's
supercritical test problem, Sec. 5.1) against what fixes them independently:
exact equivalence of nu_f = 1 fission with scattering, the exact multiplicity
of integer nu_f, closed-form moments of the pulse with c_eff, the reference
pulse solution at c_eff = 1.1, the defining property of systematic sampling
(every stretch of the laid-out bank gets the floor or the ceiling of its
share of teeth), and the low-order balance with nu_f Sigma_f (Eq. balance)."""
import math

import numpy as np
import pytest

import closed_forms as CF
from gpu_common import oracle_sim
from oracle import oracle as O
from paper_2512_19925_amd import pulse_reference as P
from paper_2512_19925_amd import workloads as W


def _fission(name, x_lo, x_hi, I, ss, sf, nu, **kw):
    st = np.ones(I)
    return W.Workload(name=name, x_lo=x_lo, x_hi=x_hi, n_cells=I, sigma_t=st, sigma_s=st * ss,
                      sigma_f=st * sf, nu_f=nu, **kw)


def _sweep_step(sim, n):
    for p in range(sim.n_chunks):
        sim.sweep(n, p)


# ------------------------------------------------------------- fission --
def test_unit_multiplicity_fission_is_scattering():
    # sigma_s = 0, sigma_f = sigma_t, nu_f = 1: every collision is a fission
    # with floor(1 + xi) = 1 neutron whose direction comes from the same
    # draw a scatter uses, so an analog run is identical to the pure
    # scattering run, tally by tally; the low-order production term
    # nu_f sigma_f equals sigma_s of the scattering run, so the solves agree.
    base = W.homogeneous("c1", -6.0, 6.0, 60, 1.0, 1.0, dt=0.2, n_steps=5, n_src=3000)
    fis = base.with_(sigma_s=np.zeros(60), sigma_f=np.ones(60), nu_f=1.0)
    a, b = oracle_sim(base), oracle_sim(fis)
    for n in range(1, 5):
        _sweep_step(a, n)
        _sweep_step(b, n)
        ta, ba = a.tallies()
        tb, bb = b.tallies()
        assert np.array_equal(ta, tb) and np.array_equal(ba, bb)
        ca, cb = a.counters(), b.counters()
        assert ca["scatters"] == cb["fissions"] == cb["fission_births"] > 0
        assert cb["scatters"] == 0 and ca["fissions"] == 0
        for k in ("segments", "collisions", "census", "leaks", "crossings", "absorptions"):
            assert ca[k] == cb[k]
        opts = O.LosmOpts(theta=0.5)
        pa, ja = a.solve_losm(opts, implicit=False, apply_windows=False)
        pb, jb = b.solve_losm(opts, implicit=False, apply_windows=False)
        assert np.array_equal(pa, pb) and np.array_equal(ja, jb)


@pytest.mark.parametrize("nu", [2.0, 2.3])
def test_fission_multiplicity(nu):
    # floor(nu + xi) neutrons per fission: exactly nu for integer nu, else
    # floor(nu) or floor(nu) + 1 with mean nu.
    w = _fission("mult", -10.0, 10.0, 50, 0.2, 0.5, nu, dt=0.5, n_steps=2, n_src=20000,
                 bank_capacity=200000)
    sim = oracle_sim(w)
    _sweep_step(sim, 1)
    c = sim.counters()
    f, b = c["fissions"], c["fission_births"]
    assert f > 5000
    if nu == 2.0:
        assert b == 2 * f
    else:
        assert 2 * f <= b <= 3 * f
        frac = nu - math.floor(nu)
        assert abs(b / f - nu) < 5 * math.sqrt(frac * (1 - frac) / f)
    assert c["collisions"] == c["scatters"] + c["absorptions"] + c["fissions"]


@pytest.mark.parametrize("ss,sf,nu", [(1 / 3, 1 / 3, 2.3), (0.0, 0.5, 2.0)])
def test_fission_pulse_moments_closed_form(ss, sf, nu):
    # With fission the mean flux obeys the transport equation with the
    # isotropic production (sigma_s + nu sigma_f) phi, so the census moments
    # of the pulse are the closed forms at c_eff = ss + nu sf (here 1.1 and
    # 1.0), over a slab wide enough that nothing leaks.
    c_eff = ss + nu * sf
    w = _fission("mom", -10.0, 10.0, 100, ss, sf, nu, dt=0.25, n_steps=8, n_src=40000,
                 bank_capacity=400000, n_batches=32)
    sim = oracle_sim(w)
    for n in range(1, w.n_steps + 1):
        _sweep_step(sim, n)
        if n % 4:
            continue
        bk = sim.bank(1)
        t = n * w.dt
        ex = dict(zip(("m0", "k", "xj", "x2"), CF.moments(c_eff, t)))
        bat = bk["src"] % w.n_batches
        for name, vals in (("m0", bk["w"]), ("k", bk["w"] * bk["mu"] ** 2),
                           ("xj", bk["w"] * bk["x"] * bk["mu"]), ("x2", bk["w"] * bk["x"] ** 2)):
            per = np.bincount(bat, weights=vals, minlength=w.n_batches)[:, None] / w.n_src
            est = per.sum()
            se = float(CF.batch_sigma(per)[0])
            assert abs(est - ex[name]) < 4.5 * se, (name, t, est, ex[name], se)


def test_fission_flux_agrees_with_the_pulse_solution():
    # Analog oracle run at c_eff = 1.1 (the paper's material): per-cell
    # track-length flux against the reference pulse solution at c = 1.1.
    w = _fission("ref-fis", -3.0, 3.0, 60, 1 / 3, 1 / 3, 2.3, dt=0.1, n_steps=10, n_src=100_000,
                 bank_capacity=600_000, n_batches=32)
    sim = oracle_sim(w)
    ref = P.cell_step_averages(w.edges, w.dt, w.n_steps, 1.1)
    dx = np.diff(w.edges)
    zs = []
    for n in range(1, w.n_steps + 1):
        _sweep_step(sim, n)
        cells, _ = sim.tallies()
        per = cells[..., 0] / (w.n_src * dx[None, :] * w.dt)
        sig = CF.batch_sigma(per)
        m = (ref[n - 1] > 0) & (sig > 0)
        zs.append((per.sum(0)[m] - ref[n - 1][m]) / sig[m])
    z = np.concatenate(zs)
    assert len(z) >= 100   # the cells inside the light cone, summed over the steps
    assert 0.7 < (z ** 2).mean() < 1.4
    assert np.abs(z).max() < 6.0


def test_low_order_balance_includes_fission_production():
    # Eq. balance: the absorption term is (sigma_t - sigma_s - nu_f sigma_f).
    # The semi-implicit solve of a fission problem equals the stand-alone
    # LOSM step with sigma_s + nu_f sigma_f as the production cross section,
    # from the same closures and initial condition.
    w = _fission("lo", -4.0, 4.0, 40, 0.25, 0.3, 2.5, dt=0.2, n_steps=3, n_src=5000, bank_capacity=100000)
    sim = oracle_sim(w)
    _sweep_step(sim, 1)
    F, Pf, phi0, J0 = sim.closures()
    got_phi, got_J = sim.solve_losm(O.LosmOpts(theta=0.5), implicit=False, apply_windows=False)
    sig_lo = w.sigma_s + w.nu_f * w.sigma_f
    phi, J = O.losm_step(w.edges, w.sigma_t, sig_lo, w.speed, w.dt, 0.5, phi0, J0, F, F, Pf[0], Pf[1])
    np.testing.assert_allclose(got_phi, phi, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(got_J, J, rtol=1e-13, atol=1e-15)
    # and not the one without the production term
    phi_s, _ = O.losm_step(w.edges, w.sigma_t, w.sigma_s, w.speed, w.dt, 0.5, phi0, J0, F, F, Pf[0], Pf[1])
    assert np.max(np.abs(phi_s - got_phi)) > 1e-3 * np.max(np.abs(got_phi))


# --------------------------------------------------------------- combing --
def _groups(state):
    """Runs of consecutive equal rows: (first index, length)."""
    out = []
    i = 0
    n = len(state)
    while i < n:
        j = i + 1
        while j < n and np.array_equal(state[j], state[i]):
            j += 1
        out.append((i, j - i))
        i = j
    return out


def _canonical(bk):
    order = np.lexsort((bk["e"], bk["lin"], bk["src"]))
    return {k: v[order] for k, v in bk.items()}


@pytest.mark.parametrize("H", [1000, 3000, 7919])
def test_comb_is_systematic_sampling(H):
    # After a windowed step of varied weights, the comb lays the census out
    # in canonical order (src, lineage, event) and places H equally spaced
    # teeth with one random offset.  Every run of consecutive particles
    # (here: runs of equal state, which split siblings form) then receives
    # floor or ceil of H * (run weight) / W copies, in the same order; each
    # copy has weight W / H and the new identity (k, step, 0), batch k mod B,
    # chunk (k / B) mod n_chunks.
    w = _fission("comb", -6.0, 6.0, 60, 1 / 3, 1 / 3, 2.3, dt=0.5, n_steps=3, n_src=3000, rho=1.25,
                 bank_capacity=200000, n_batches=8, n_chunks=4)
    sim = oracle_sim(w)
    opts = O.LosmOpts(theta=0.5, rho=1.25, filter=1)
    sim.solve_losm(opts, implicit=False)
    for p in range(w.n_chunks):
        sim.sweep(1, p)
        if p < w.n_chunks - 1:
            sim.solve_losm(opts, implicit=True)
    before = _canonical(sim.bank(1))
    assert len(np.unique(before["w"])) > 3   # the windows made the weights differ
    n_before, W_tot = sim.comb(H)
    assert n_before == len(before["w"])
    after = sim.bank(1)
    assert len(after["w"]) == H
    assert abs(W_tot / before["w"].sum() - 1.0) < 1e-9
    assert np.all(after["w"] == after["w"][0])
    assert abs(after["w"][0] * H / W_tot - 1.0) < 1e-15
    assert np.array_equal(after["src"], np.arange(H, dtype=np.uint32))
    assert np.all(after["lin"] == 1) and np.all(after["e"] == 0)
    assert np.array_equal(after["chunk"], (np.arange(H) // w.n_batches) % w.n_chunks)
    st_b = [tuple(r) for r in np.stack([before["x"], before["mu"], before["cell"].astype(float)], 1)]
    st_a = [tuple(r) for r in np.stack([after["x"], after["mu"], after["cell"].astype(float)], 1)]
    # Runs of equal state; a state can recur in runs that are not adjacent
    # (a split parent keeps its own lineage), so the floor/ceil bounds are
    # summed over the runs of each state.
    lo, hi, runs = {}, {}, []
    for i0, ln in _groups(np.array(st_b)):
        share = before["w"][i0:i0 + ln].sum() * H / W_tot
        key = st_b[i0]
        lo[key] = lo.get(key, 0) + math.floor(share - 1e-9)
        hi[key] = hi.get(key, 0) + math.ceil(share + 1e-9)
        runs.append(key)
    got = {}
    for key in st_a:
        got[key] = got.get(key, 0) + 1
    for key in lo:
        assert lo[key] <= got.get(key, 0) <= hi[key], (key, lo[key], got.get(key, 0), hi[key])
    assert set(got) <= set(lo)
    # Copies come in the canonical order of their parents.
    r = 0
    for key in st_a:
        while runs[r] != key:
            r += 1
    ws, wn = sim.state()[2:]
    counts = np.bincount(after["chunk"], minlength=w.n_chunks)
    np.testing.assert_array_equal(wn, counts * after["w"][0])


def test_comb_offsets_are_uniform():
    # The comb's offset xi (slot 7, counter (step, 0, 0, 0)) decides which of
    # two adjacent particles straddling a tooth is copied; over many seeds
    # a particle of share f (0 < f < 1) is copied with probability f.  Here:
    # the census run of the first canonical particle with a fractional
    # share, tallied over seeds.
    hits, exp, var = 0.0, 0.0, 0.0
    for seed in range(1, 121):
        w = _fission("combu", -3.0, 3.0, 30, 1 / 3, 1 / 3, 2.3, dt=0.5, n_steps=2, n_src=300,
                     bank_capacity=20000, n_batches=4, n_chunks=1, seed=seed)
        sim = oracle_sim(w)
        _sweep_step(sim, 1)
        before = _canonical(sim.bank(1))
        _, W_tot = sim.comb(50)
        after = sim.bank(1)
        # The first run of equal state starts the laid-out bank at 0, so it
        # is copied iff the first tooth xi W / 50 falls inside it: with share
        # f < 1, iff xi < f.
        st_b = np.stack([before["x"], before["mu"], before["cell"].astype(float)], 1)
        _, ln = _groups(st_b)[0]
        f = before["w"][:ln].sum() * 50 / W_tot
        if f >= 1.0:
            continue
        got = np.array_equal(np.array([after["x"][0], after["mu"][0], float(after["cell"][0])]), st_b[0])
        hits += float(got)
        exp += f
        var += f * (1 - f)
    assert var > 5.0
    assert abs(hits - exp) < 4.0 * math.sqrt(var)


def test_comb_by_index_is_systematic_sampling_over_particles():
    # Teeth spaced in particle index: every particle of the laid-out census
    # (canonical order) is one unit long, so every run of consecutive
    # particles gets the floor or the ceiling of (run length) H / n copies,
    # in order, and every copy keeps its particle's weight times n / H (its
    # expected weight is its particle's), the weight taken in the comb's
    # integer unit 2^eu (count * largest weight < 2^(53 + eu)).  Fewer and
    # more copies than particles; each copy becomes history k of step 1 as
    # in the other reading.
    w = _fission("combi", -6.0, 6.0, 60, 1 / 3, 1 / 3, 2.3, dt=0.5, n_steps=3, n_src=3000, rho=1.25,
                 bank_capacity=200000, n_batches=8, n_chunks=4)
    for H in (1000, 9000):
        sim = oracle_sim(w)
        sim.set_comb_mode(1)
        opts = O.LosmOpts(theta=0.5, rho=1.25, filter=1)
        sim.solve_losm(opts, implicit=False)
        for p in range(w.n_chunks):
            sim.sweep(1, p)
            if p < w.n_chunks - 1:
                sim.solve_losm(opts, implicit=True)
        before = _canonical(sim.bank(1))
        n = len(before["w"])
        assert len(np.unique(before["w"])) > 3
        n_before, W_tot = sim.comb(H)
        assert n_before == n and abs(W_tot / before["w"].sum() - 1.0) < 1e-12
        after = sim.bank(1)
        assert len(after["w"]) == H
        assert np.array_equal(after["src"], np.arange(H, dtype=np.uint32))
        assert np.all(after["lin"] == 1) and np.all(after["e"] == 0)
        assert np.array_equal(after["chunk"], (np.arange(H) // w.n_batches) % w.n_chunks)
        # Match the copies, in order, to runs of equal state and weight.
        eu = int(np.frexp(before["w"].max())[1]) + int(np.ceil(np.log2(n))) - 53
        w_unit = np.ldexp(np.rint(np.ldexp(before["w"], -eu)), eu)
        assert np.all(np.abs(w_unit / before["w"] - 1.0) < 1e-9)
        key_b = np.stack([before["x"], before["mu"], before["cell"].astype(float), w_unit * (n / H)], 1)
        key_a = np.stack([after["x"], after["mu"], after["cell"].astype(float), after["w"]], 1)
        groups = _groups(key_b)
        pos = 0
        for start, ln in groups:
            share = ln * H / n
            cnt = 0
            while pos < H and np.array_equal(key_a[pos], key_b[start]):
                pos += 1
                cnt += 1
            assert math.floor(share) <= cnt <= math.ceil(share), (start, ln, cnt, share)
        assert pos == H


def test_comb_by_index_keeps_the_weight_on_average():
    # Over many combs (seeds) the total weight after a comb by index equals
    # the census weight before it on average (each particle's expected
    # number of copies is H / n, each copy of weight w n / H).
    ratios = []
    for seed in range(1, 61):
        w = _fission("combw", -3.0, 3.0, 30, 1 / 3, 1 / 3, 2.3, dt=0.5, n_steps=2, n_src=400, rho=1.25,
                     bank_capacity=40000, n_batches=4, n_chunks=2, seed=seed)
        sim = oracle_sim(w)
        sim.set_comb_mode(1)
        opts = O.LosmOpts(theta=0.5, rho=1.25, filter=1)
        sim.solve_losm(opts, implicit=False)
        for p in range(w.n_chunks):
            sim.sweep(1, p)
            if p < w.n_chunks - 1:
                sim.solve_losm(opts, implicit=True)
        _, W_tot = sim.comb(150)
        ratios.append(sim.bank(1)["w"].sum() / W_tot)
    r = np.array(ratios)
    assert r.std() > 0  # the windows made the weights differ, so the total varies
    assert abs(r.mean() - 1.0) < 4.0 * r.std(ddof=1) / math.sqrt(len(r))


def test_comb_keeps_the_paper_problem_bounded():
    # The paper's problem at a tenth of its population: with combing every
    # census holds exactly H particles while the total weight grows.
    w = W.paper_fission(n_src=1000).with_(n_steps=6)
    sim = oracle_sim(w)
    opts = O.LosmOpts(theta=0.5, rho=w.rho, eps_min=w.eps_min, filter=1)
    tot = []
    O.run(sim, w.n_steps, opts, on_step=lambda n, s: tot.append(s.state()[3].sum()), comb=w.comb)
    sim.comb(w.comb)
    assert len(sim.bank(1)["w"]) == w.comb
    assert tot[-1] > tot[0]


@pytest.mark.parametrize("window_scale", [0, 1])
def test_window_scale_readings(window_scale):
    # Eq. ww-center as printed puts the largest centre at exactly 1 and the
    # smallest at eps_min or above; window_scale 0 multiplies the centres by
    # s^n, the census weight per source particle (here grown by fission).
    w = W.paper_fission(n_src=2000).with_(n_steps=4, window_scale=window_scale)
    sim = oracle_sim(w)
    opts = O.LosmOpts(theta=0.5, rho=w.rho, eps_min=w.eps_min, filter=1, window_scale=window_scale)
    for n in (1, 2):
        _sweep_step(sim, n)
    sim.comb(w.comb)
    sim.solve_losm(opts, implicit=False)
    c, u, f = sim.windows()
    s_n = sim.state()[3].sum() / w.n_src
    assert s_n > 1.05            # the population grew
    top = 1.0 if window_scale else s_n
    assert c.max() == pytest.approx(top, rel=1e-15)
    assert c.min() >= w.eps_min * top * (1 - 1e-15)
    np.testing.assert_allclose(u, c * w.rho, rtol=1e-15)
    np.testing.assert_allclose(f, c / w.rho, rtol=1e-15)
