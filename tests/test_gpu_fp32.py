"""FP32 flight arithmetic (positions, directions, distances in FP32; weights,
tallies and the LOSM solve in FP64).  A different rounding gives a different
realisation, so the checks are statistical: every tally within the batch
standard deviation of the closed-form uncollided pulse solution and of the
FP64 oracle."""
import numpy as np
import pytest

import closed_forms as CF
from gpu_common import need_gpu, oracle_opts, oracle_sim, precision_error, say
from oracle import oracle as O
from paper_2512_19925_amd import hww as H
from paper_2512_19925_amd import workloads as W

pytestmark = pytest.mark.gpu


def _z(per_batch_a, per_batch_b=None, exact=None):
    ta = per_batch_a.sum(0)
    sa = CF.batch_sigma(per_batch_a)
    if per_batch_b is not None:
        tb = per_batch_b.sum(0)
        sb = CF.batch_sigma(per_batch_b)
        s = np.sqrt(sa ** 2 + sb ** 2)
        d = ta - tb
    else:
        s, d = sa, ta - exact
    m = s > 0
    return d[m] / s[m]


def test_fp32_uncollided_closed_form():
    need_gpu()
    w = W.homogeneous("fp32-c0", -3.0, 3.0, 60, 1.0, 0.0, dt=0.25, n_steps=8, n_src=200000, rho=2.0,
                      eps_min=0.05, bank_capacity=20_000_000)
    say(f"case {w.name}")
    h = H.Handle(H.spec_from_workload(w, precision=H.HWW_FP32))
    edges = w.edges
    dx = np.diff(edges)
    zs = []

    def on_step(n, hh, _):
        cells = hh.read_tallies(H.TALLY_CELLS)
        t0, t1 = (n - 1) * w.dt, n * w.dt
        ex_t = np.array([CF.uncollided_cell_time_avg(edges[i], edges[i + 1], t0, t1, 1.0, 1.0) for i in range(60)])
        ex_c = np.array([CF.uncollided_cell_avg(edges[i], edges[i + 1], t1, 1.0, 1.0) for i in range(60)])
        for k in range(3):
            zs.append(_z(cells[..., k] / (w.n_src * dx * w.dt), exact=ex_t[:, k]))
            zs.append(_z(cells[..., 3 + k] / (w.n_src * dx), exact=ex_c[:, k]))

    H.run(h, w, on_step=on_step, stats=False)
    z = np.concatenate(zs)
    say(f"  {len(z)} tallies, mean z^2 {np.mean(z ** 2):.3f}, max |z| {np.abs(z).max():.2f}")
    assert len(z) > 500
    assert 0.7 < np.mean(z ** 2) < 1.5
    assert np.abs(z).max() < 6.0


def test_fp32_against_fp64_oracle():
    # Independent seeds: the FP32 GPU run and the FP64 oracle run estimate
    # the same expected tallies of the plain hybrid-WW problem.
    need_gpu()
    w = W.plain_small().with_(n_src=40000, n_steps=10, bank_capacity=2_000_000)
    say(f"case {w.name} fp32 vs fp64 oracle")
    h = H.Handle(H.spec_from_workload(w.with_(seed=7), precision=H.HWW_FP32))
    g_steps = []
    H.run(h, w, on_step=lambda n, hh, _: g_steps.append(hh.read_tallies(H.TALLY_CELLS)), stats=False)
    sim = oracle_sim(w)
    o_steps = []
    O.run(sim, w.n_steps, oracle_opts(w), lambda n, s: o_steps.append(s.tallies()[0].copy()))
    zs = []
    worst_rel = 0.0
    for g, o in zip(g_steps, o_steps):
        for k in range(6):
            zs.append(_z(g[..., k], o[..., k]))
        tg, to = g[..., 0].sum(0), o[..., 0].sum(0)
        m = to > 0.01 * to.max()
        worst_rel = max(worst_rel, float(np.max(np.abs(tg[m] - to[m]) / to[m])))
    z = np.concatenate(zs)
    say(f"  {len(z)} tallies, mean z^2 {np.mean(z ** 2):.3f}, max |z| {np.abs(z).max():.2f}, "
        f"max relative error of track phi (cells above 1% of peak) {worst_rel:.3e}")
    assert len(z) > 300
    assert 0.6 < np.mean(z ** 2) < 1.6
    assert np.abs(z).max() < 6.5


def test_fp32_scattering_moments():
    # Analog FP32 histories: census-bank moments against the closed-form
    # spatial moments of the pulse (c = 0.9, t = 1.5).
    need_gpu()
    w = W.homogeneous("fp32-mom", -20.0, 20.0, 200, 1.0, 0.9, dt=0.1, n_steps=15, n_src=400000,
                      analog=True)
    h = H.Handle(H.spec_from_workload(w, precision=H.HWW_FP32))
    H.run(h, w, stats=False)
    b = h.read_bank(1)
    N = w.n_src
    ex = dict(zip(("m0", "k", "xj", "x2"), CF.moments(0.9, 1.5)))
    vals = {"m0": b["w"], "k": b["w"] * b["mu"] ** 2, "xj": b["w"] * b["x"] * b["mu"], "x2": b["w"] * b["x"] ** 2}
    for name, v in vals.items():
        full = np.zeros(N)
        full[b["src"]] = v
        se = full.std() / np.sqrt(N)
        say(f"  {name}: {full.mean():.6f} vs {ex[name]:.6f} (se {se:.2e})")
        assert abs(full.mean() - ex[name]) < 4.5 * se


@pytest.mark.parametrize("precision", [H.HWW_FP32, H.HWW_FP64])
def test_precision_form_against_the_pulse_solution(precision):
    # The precision form (200 cells on [-20, 20], c = 0.9, 20 steps of 0.1,
    # windows from the LOSM solves) at 1e7 particles: the track-length flux
    # of every reached cell and step against the closed-form pulse solution,
    # within the batch standard deviation.
    need_gpu()
    from paper_2512_19925_amd import pulse_reference as P
    w = W.precision_form()
    say(f"case {w.name} precision {precision}")
    ref = P.cell_step_averages(w.edges, w.dt, w.n_steps, 0.9)
    dx = np.diff(w.edges)
    h = H.Handle(H.spec_from_workload(w, precision=precision))
    zs, rel = [], []

    def on_step(n, hh, _):
        cells = hh.read_tallies(H.TALLY_CELLS)
        per = cells[..., 0] / (w.n_src * dx * w.dt)
        r = ref[n - 1]
        m = r > 1e-3 * r.max()
        zs.append(_z(per[:, m], exact=r[m]))
        rel.append(np.abs(per.sum(0)[m] / r[m] - 1.0))

    H.run(h, w, on_step=on_step, stats=False)
    h.close()
    z = np.concatenate(zs)
    rr = np.concatenate(rel)
    say(f"  {len(z)} cell-steps, mean z^2 {np.mean(z ** 2):.3f}, max |z| {np.abs(z).max():.2f}, "
        f"median relative error {np.median(rr):.2e}, max {rr.max():.2e}")
    # The windows couple the batches (every batch is split and rouletted
    # against windows from the tallies of all), so the batch spread can only
    # overestimate the error of the sum: no lower bound on mean z^2.
    assert len(z) > 150
    assert np.mean(z ** 2) < 1.6
    assert np.abs(z).max() < 5.0


def test_precision_form_against_the_fp64_oracle():
    # The precision form (200 cells on [-20, 20], c = 0.9, 20 steps of 0.1,
    # 1e7 particles, windows from the LOSM solves) in FP32 against the FP64
    # oracle of the same seed, all six tallies of every cell and step.  The
    # two runs draw the same random numbers (24 against 53 bits), so they
    # differ only where rounding changes a decision; each tally's difference
    # must stay within 3 batch standard deviations of the FP64 sum.
    need_gpu()
    import time
    w = W.precision_form()
    say(f"case {w.name}: FP32 GPU against the FP64 oracle, same seed")
    h = H.Handle(H.spec_from_workload(w, precision=H.HWW_FP32))
    g_steps = []
    H.run(h, w, on_step=lambda n, hh, _: g_steps.append(hh.read_tallies(H.TALLY_CELLS)), stats=False)
    h.close()
    t0 = time.time()
    sim = oracle_sim(w)
    o_steps = []
    O.run(sim, w.n_steps, oracle_opts(w), lambda n, s: o_steps.append(s.tallies()[0].copy()))
    say(f"  oracle: {time.time() - t0:.1f} s")
    err = precision_error(g_steps, o_steps)
    for k, e in err.items():
        say(f"  {k:10s}: {e['n']} cell-steps, max |z| {e['max_abs_z']:.3f}, within 3 sigma "
            f"{e['frac_within_3sigma']:.4f}, relative error median {e['median_rel_err']:.2e} "
            f"max {e['max_rel_err']:.2e}")
    for k, e in err.items():
        assert e["n"] >= 200, k  # cells reached (|x| < v t) over the 20 steps
        assert e["max_abs_z"] <= 3.0, k
