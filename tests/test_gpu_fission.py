"""GPU parity of the paper's supercritical test problem (Sec. 5.1): fission
collisions in the HIP sweep and the uniform comb of every census, called
through the C ABI, against the CPU oracle on the same seeded inputs.  FP64
tallies agree to 1e-12 relative per batch and cell, counters exactly, and
census banks as multisets both before and after each comb."""
import numpy as np
import pytest

from gpu_common import (assert_bank_match, assert_bnd_match, assert_tallies_match, need_gpu,
                        oracle_opts, oracle_sim, say)
from paper_2512_19925_amd import hww as H
from paper_2512_19925_amd import workloads as W

pytestmark = pytest.mark.gpu

COUNTERS = ["segments", "collisions", "scatters", "absorptions", "crossings", "leaks", "census",
            "splits", "daughters", "rr_kill", "rr_survive", "histories", "fissions", "fission_births"]


def _run_pair(w, steps=None, analog=False, wait=True):
    need_gpu()
    steps = w.n_steps if steps is None else steps
    say(f"case {w.name}: n_src={w.n_src} I={w.n_cells} nu={w.nu_f} comb={w.comb} steps={steps} analog={analog} "
        f"wait={wait}")
    h = H.Handle(H.spec_from_workload(w))
    sim = oracle_sim(w)
    opts = oracle_opts(w)
    kw = H.losm_kwargs(w)
    worst = 0.0
    for n in range(1, steps + 1):
        if w.comb and n > 1:
            on, ow = sim.comb(w.comb)
            if wait:
                gn, gw = h.comb(w.comb)
                assert gn == on, f"step {n}: census sizes before the comb {gn} vs {on}"
                # The census weights of roulette survivors are window centres,
                # which carry the LOSM solve's rounding (the bank comparison's
                # 1e-12 on weights); the comb's total sums them.
                assert abs(gw / ow - 1.0) < 1e-12, f"step {n}: comb weight {gw} vs {ow}"
            else:
                assert h.comb(w.comb, wait=False) is None
            assert_bank_match(h.read_bank(1), sim.bank(1), what=f"{w.name} comb before step {n}")
        if not analog:
            h.solve_losm(implicit=False, **kw)
            sim.solve_losm(opts, implicit=False)
        for p in range(w.n_chunks):
            st = h.sweep_step(n, p, stats=(p == w.n_chunks - 1))
            sim.sweep(n, p)
            if not analog and p < w.n_chunks - 1:
                h.solve_losm(implicit=True, **kw)
                sim.solve_losm(opts, implicit=True)
        oc = sim.counters()
        assert {k: st[k] for k in COUNTERS} == {k: oc[k] for k in COUNTERS}, f"step {n}: counters"
        g = h.read_tallies(H.TALLY_CELLS)
        o, ob = sim.tallies()
        worst = max(worst, assert_tallies_match(g, o, what=f"{w.name} step {n}"))
        assert_bnd_match(h.read_tallies(H.TALLY_BOUNDARY), ob, what=f"{w.name} step {n}")
        assert np.array_equal(h.read_tallies(H.TALLY_TRACKS), sim.tracks()), f"step {n}: tracks"
        assert_bank_match(h.read_bank(1), sim.bank(1), what=f"{w.name} step {n}")
        if not analog:
            np.testing.assert_allclose(h.read_tallies(H.TALLY_WINDOWS)[0], sim.windows()[0], rtol=1e-12)
    say(f"  max relative tally difference {worst:.2e}; fissions in the last step {st['fissions']}")
    h.close()
    return worst


@pytest.mark.parametrize("by_index", [True, False])
def test_paper_problem_end_to_end(by_index):
    # The paper's problem as specified: 201 cells, c_eff = 1.1, 20 steps of
    # dt = 1, 1e4 histories per step kept by combing, rho = 1.25; the comb's
    # teeth spaced in particle index (the problem's reading) or in weight.
    _run_pair(W.paper_fission().with_(comb_by_index=by_index))


def test_paper_problem_comb_without_wait():
    # The comb only queued (no census size read back): the same realisation
    # as the oracle's, bank for bank and tally for tally.
    _run_pair(W.paper_fission(n_src=4000).with_(name="paper-no-wait", n_steps=8), wait=False)


def test_paper_problem_windows_as_printed():
    # Eq. ww-center as printed (largest centre 1 while the mean weight grows
    # with fission): many more splits at every step start.
    _run_pair(W.paper_fission().with_(name="paper-printed-ww", window_scale=1, n_steps=10))


def test_comb_of_three_histories_after_a_long_one():
    # Three histories: at step 4 one of them has 215 census particles (the
    # work-group sort), and every comb orders fewer histories than the
    # comb's reduction cells: each comb must start from cleared cells.
    w = W.paper_fission(n_src=3).with_(name="three-histories", n_batches=1, n_steps=6, rho=1.25, eps_min=1e-3,
                                       bank_capacity=200_000)
    _run_pair(w)
    _run_pair(w.with_(name="three-histories-no-wait"), wait=False)


def test_fission_analog_without_comb():
    # Integer multiplicity (every fission makes exactly two), no windows, no
    # comb: the population grows freely for a few steps.
    w = W.paper_fission(n_src=3000).with_(name="fis-analog", nu_f=2.0, comb=0, n_steps=4,
                                           bank_capacity=200_000)
    _run_pair(w, analog=True)


def test_fission_with_splitting_daughters():
    # Wide windows of the small problem's kind: splits and fission daughters
    # in the same work-group buffers.
    w = W.paper_fission(n_src=4000).with_(name="fis-split", rho=2.0, eps_min=1e-2, n_steps=6, n_batches=8)
    _run_pair(w)


def test_comb_errors():
    need_gpu()
    w = W.paper_fission(n_src=2000).with_(n_steps=3)
    h = H.Handle(H.spec_from_workload(w))
    with pytest.raises(H.HwwError) as e:       # step 0 is not a finished step of the sweep
        h.comb(2000)
    assert e.value.code == -2
    for p in range(w.n_chunks):
        h.sweep_step(1, p, stats=False)
    with pytest.raises(H.HwwError) as e:
        h.comb(w.capacity() + 1)
    assert e.value.code == -1
    n, W_tot = h.comb(500)
    assert n > 0 and W_tot > 0
    assert len(h.read_bank(1)["w"]) == 500
    h.close()
    plain = H.Handle(H.spec_from_workload(W.plain_small().with_(n_steps=2)))
    for p in range(4):
        plain.sweep_step(1, p, stats=False)
    with pytest.raises(H.HwwError) as e:       # no comb workspace
        plain.comb(100)
    assert e.value.code == -2
    plain.close()
    with pytest.raises(H.HwwError) as e:       # batches take no fission
        H.Batch([H.spec_from_workload(W.paper_fission(n_src=500))])
    assert e.value.code == -1


def _comb_by_definition(bank, n_target, step, seed, replica, B, nc):
    """The comb from its definition, on the host: canonical order, integer
    weights in units of 2^eu, prefix sums, teeth (k + xi) W / n_target.
    Returns (x, mu, cell) of each copy and the copy weight."""
    from oracle import oracle as O
    order = np.lexsort((bank["e"], bank["lin"], bank["src"]))
    w = bank["w"][order]
    n = len(w)
    em = int(np.frexp(w.max())[1])
    ln = int(np.ceil(np.log2(n))) if n > 1 else 0
    eu = em + ln - 53
    wi = np.rint(np.ldexp(w, -eu)).astype(np.uint64)
    q = np.cumsum(wi, dtype=np.uint64)
    W = float(q[-1])
    r = O.philox4x32_10([step, 0, 0, 0], [seed, (replica << 4) | 7])
    xi = O.u53(r[0], r[1])
    delta = W / float(n_target)
    t = (np.arange(n_target, dtype=np.float64) + xi) * delta
    t = np.where(t >= W, W - 1.0, t)
    j = np.searchsorted(q.astype(np.float64), t, side="right")
    par = order[j]
    return bank["x"][par], bank["mu"][par], bank["cell"][par], np.ldexp(W, eu) / n_target


def _comb_by_index_definition(bank, n_target, step, seed, replica):
    """The comb by index from its definition, on the host: canonical order,
    tooth k at position floor((k + xi) n / n_target), each copy with its
    particle's weight in units of 2^eu times n / n_target.  Returns (x, mu,
    cell, w) of each copy and the census weight W (the sum in those units)."""
    from oracle import oracle as O
    order = np.lexsort((bank["e"], bank["lin"], bank["src"]))
    n = len(order)
    w = bank["w"][order]
    eu = int(np.frexp(w.max())[1]) + (int(np.ceil(np.log2(n))) if n > 1 else 0) - 53
    w_unit = np.ldexp(np.rint(np.ldexp(bank["w"], -eu)), eu)
    r = O.philox4x32_10([step, 0, 0, 0], [seed, (replica << 4) | 7])
    xi = O.u53(r[0], r[1])
    delta = n / float(n_target)
    j = np.minimum(((np.arange(n_target, dtype=np.float64) + xi) * delta).astype(np.int64), n - 1)
    par = order[j]
    W = float(np.ldexp(float(np.rint(np.ldexp(bank["w"], -eu)).astype(np.uint64).sum()), eu))
    return bank["x"][par], bank["mu"][par], bank["cell"][par], w_unit[par] * delta, W


@pytest.mark.parametrize("by_index", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_comb_matches_its_definition(precision, by_index):
    # The device comb against the comb written out on the host from the
    # census it combs (FP32 banks included): every copy k, its weight, its
    # identity and its chunk; teeth spaced in weight or in particle index.
    need_gpu()
    w = W.paper_fission(n_src=5000).with_(n_steps=4, n_batches=16, comb_by_index=by_index)
    prec = H.HWW_FP32 if precision == "fp32" else H.HWW_FP64
    h = H.Handle(H.spec_from_workload(w, precision=prec))
    kw = H.losm_kwargs(w)
    for n in (1, 2):
        if n > 1:
            h.comb(w.comb)
        h.solve_losm(implicit=False, **kw)
        for p in range(w.n_chunks):
            h.sweep_step(n, p, stats=False)
            if p < w.n_chunks - 1:
                h.solve_losm(implicit=True, **kw)
    census = h.read_bank(1)
    # Fewer and more copies than particles; the last comb orders 40000
    # histories, so its history counts take the tiled scan.
    for H_t in (3000, 12345, 40000, 7000):
        before = {k: v.copy() for k, v in census.items()}
        n_b, W_tot = h.comb(H_t)
        assert n_b == len(before["w"])
        after = h.read_bank(1)
        o = np.argsort(after["src"])
        after = {k: v[o] for k, v in after.items()}
        assert np.array_equal(after["src"], np.arange(H_t, dtype=np.uint32))
        assert np.all(after["lin"] == 2) and np.all(after["e"] == 0)
        assert np.array_equal(after["chunk"], (np.arange(H_t) // w.n_batches) % w.n_chunks)
        if by_index:
            x, mu, cell, w_c, W_def = _comb_by_index_definition(before, H_t, 2, w.seed, w.replica)
            assert np.array_equal(after["w"], w_c)
            assert W_tot == W_def
        else:
            x, mu, cell, w_out = _comb_by_definition(before, H_t, 2, w.seed, w.replica, w.n_batches,
                                                     w.n_chunks)
            assert np.all(after["w"] == w_out) and abs(W_tot - w_out * H_t) <= 1e-12 * W_tot
        assert np.array_equal(after["x"], x) and np.array_equal(after["mu"], mu)
        assert np.array_equal(after["cell"], cell)
        census = after  # each further comb combs the combed bank
    h.close()


def test_comb_of_an_empty_census():
    # A pure absorber of 100 mean free paths per step: nothing reaches the
    # census (survival e^-100), the comb finds nothing, the census stays
    # empty and the next step sweeps nothing, as in the oracle.
    need_gpu()
    st = np.ones(10)
    w = W.Workload(name="absorb-all", x_lo=-0.5, x_hi=0.5, n_cells=10, sigma_t=st * 100.0, sigma_s=st * 0.0,
                   sigma_f=st * 0.0, nu_f=2.0, speed=1.0, dt=1.0, n_steps=3, n_src=500, comb=500,
                   bank_capacity=20000, n_batches=4)
    h = H.Handle(H.spec_from_workload(w))
    sim = oracle_sim(w)
    for p in range(w.n_chunks):
        h.sweep_step(1, p, stats=False)
        sim.sweep(1, p)
    assert h.comb(500) == (0, 0.0) == sim.comb(500)
    assert len(h.read_bank(1)["w"]) == 0
    for p in range(w.n_chunks):
        st_g = h.sweep_step(2, p)
        sim.sweep(2, p)
    assert st_g["segments"] == 0 == sim.counters()["segments"]
    # Combed without waiting, the empty census leaves an empty combed bank.
    assert h.comb(500, wait=False) is None
    assert len(h.read_bank(1)["w"]) == 0
    for p in range(w.n_chunks):
        st_g = h.sweep_step(3, p)
    assert st_g["segments"] == 0 and st_g["census"] == 0
    h.close()
