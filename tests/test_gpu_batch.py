"""Batched form: many replicas of uneven size in one handle (one persistent
sweep launch per chunk, one batched LOSM launch per solve).  Every replica
keeps its own keying, so each must equal its own oracle run to 1e-12
relative per batch and cell, with exact counters and equal census banks."""
import numpy as np
import pytest

from gpu_common import (assert_bank_match, assert_bnd_match, assert_tallies_match, need_gpu,
                        oracle_opts, oracle_sim, say)
from paper_2512_19925_amd import hww as H
from paper_2512_19925_amd import workloads as W

pytestmark = pytest.mark.gpu

COUNTERS = ["segments", "collisions", "scatters", "absorptions", "crossings", "leaks", "census",
            "splits", "daughters", "rr_kill", "rr_survive", "histories"]


def uneven_replicas(n_steps=5):
    """Replicas that differ in every size the batch handles: cells (odd and
    even, 1 to 300), particles (1 to 20000, so that some replicas have
    several units per batch), batches (1 to 64), cross sections."""
    rng = np.random.default_rng(11)
    shapes = [(200, 20000, 1), (37, 1, 32), (300, 3000, 64), (64, 65, 7), (1, 500, 32), (120, 9000, 2),
              (90, 257, 32), (256, 12000, 3)]
    out = []
    for r, (I, N, B) in enumerate(shapes):
        st = rng.uniform(0.5, 2.0)
        c = rng.uniform(0.3, 0.99)
        half = 4.0 if I > 1 else 0.05
        w = W.homogeneous(f"rep{r}", -half, half, I, st, c, dt=0.1, n_steps=n_steps, n_src=N, rho=5.0,
                          seed=1, replica=r, n_batches=B, filter=1, ma_k=3, bank_capacity=max(8 * N, 4096))
        out.append(w)
    return out


def _kw(w):
    return H.losm_kwargs(w)


def _run_batch_vs_oracle(ws, steps, tune=False, check=None, banks=True):
    need_gpu()
    check = range(len(ws)) if check is None else list(check)
    say(f"batch of {len(ws)} replicas, steps {steps}, checked {list(check)[:12]}")
    bt = H.Batch([H.spec_from_workload(w) for w in ws])
    if tune:
        res = bt.autotune()
        say(f"  tuned: {res}")
    sims = {r: oracle_sim(ws[r]) for r in check}
    opts = {r: oracle_opts(ws[r]) for r in check}
    kw = _kw(ws[0])
    worst = 0.0
    for n in range(1, steps + 1):
        bt.solve_losm(implicit=False, **kw)
        for r in check:
            sims[r].solve_losm(opts[r], implicit=False)
        for p in range(bt.n_chunks):
            st = bt.sweep_step(n, p, stats=(p == bt.n_chunks - 1))
            for r in check:
                sims[r].sweep(n, p)
            if p < bt.n_chunks - 1:
                bt.solve_losm(implicit=True, **kw)
                for r in check:
                    sims[r].solve_losm(opts[r], implicit=True)
        if len(check) == len(ws):
            tot = {k: sum(sims[r].counters()[k] for r in check) for k in COUNTERS}
            assert {k: st[k] for k in COUNTERS} == tot, f"step {n}: counters"
        cells = bt.read_tallies(H.TALLY_CELLS)
        bnd = bt.read_tallies(H.TALLY_BOUNDARY)
        trk = bt.read_tallies(H.TALLY_TRACKS)
        win = bt.read_tallies(H.TALLY_WINDOWS)
        for r in check:
            o, ob = sims[r].tallies()
            what = f"{ws[r].name} step {n}"
            worst = max(worst, assert_tallies_match(cells[r], o, what=what))
            assert_bnd_match(bnd[r], ob, what=what)
            assert np.array_equal(trk[r], sims[r].tracks()), f"{what}: tracks"
            np.testing.assert_allclose(win[r][0], sims[r].windows()[0], rtol=1e-12, err_msg=what)
            if banks:
                assert_bank_match(bt.replica(r).read_bank(1), sims[r].bank(1), what=what)
    say(f"  max relative tally difference {worst:.2e}")
    bt.close()
    return worst


def test_uneven_replicas_match_their_oracles():
    _run_batch_vs_oracle(uneven_replicas(), steps=5)


def test_autotuned_batch_matches_oracles():
    ws = [w.with_(theta=1.0, closure_track=1) for w in uneven_replicas(n_steps=3)]
    _run_batch_vs_oracle(ws, steps=3, tune=True)


def test_autotune_reuses_the_shape_of_a_problem_of_the_same_kind():
    # A second problem of the same kind takes the stored shape without
    # measuring; the shape changes only the summation order of the tallies.
    need_gpu()
    w = W.plain_small().with_(n_src=30_000, n_steps=3)
    h1 = H.Handle(H.spec_from_workload(w))
    r1 = h1.autotune()
    h2 = H.Handle(H.spec_from_workload(w))
    r2 = h2.autotune()
    say(f"  first {r1}, second {r2}")
    assert r2["trials"] == 0
    assert (r2["block"], r2["tile"], r2["grid"]) == (r1["block"], r1["tile"], r1["grid"])
    h3 = H.Handle(H.spec_from_workload(w))  # default shape, not tuned
    out = []
    for h in (h2, h3):
        H.run(h, w, stats=False)
        out.append(h.read_tallies(H.TALLY_CELLS))
        h.close()
    h1.close()
    assert_tallies_match(out[0], out[1], what="tuned against default shape")


def test_batch_fourier_filter_matches_oracles():
    ws = [w.with_(filter=2, kappa=12) for w in uneven_replicas(n_steps=3)]
    _run_batch_vs_oracle(ws, steps=3)


def test_batched_form_sampled_replicas():
    # The 256-replica batched form, three steps; the oracle replays the
    # smallest and largest replicas and a few in between.
    ws = W.batched_replicas(n_steps=3)
    order = np.argsort([w.n_src for w in ws])
    check = sorted({int(order[0]), int(order[1]), int(order[128]), int(order[200]), int(order[-1]),
                    int(np.argmax([w.n_cells for w in ws]))})
    _run_batch_vs_oracle(ws, steps=3, check=check, banks=False)


def test_batch_fp32_equals_single_fp32_handles():
    # FP32 flight arithmetic is identical per particle in both launch forms;
    # only the summation order of the FP64 tallies differs.
    need_gpu()
    ws = uneven_replicas(n_steps=3)[:5]
    bt = H.Batch([H.spec_from_workload(w, precision=H.HWW_FP32) for w in ws])
    hs = [H.Handle(H.spec_from_workload(w, precision=H.HWW_FP32)) for w in ws]
    kw = _kw(ws[0])
    for n in range(1, 4):
        bt.solve_losm(implicit=False, **kw)
        for h in hs:
            h.solve_losm(implicit=False, **kw)
        for p in range(bt.n_chunks):
            bt.sweep_step(n, p, stats=False)
            for h in hs:
                h.sweep_step(n, p, stats=False)
            if p < bt.n_chunks - 1:
                bt.solve_losm(implicit=True, **kw)
                for h in hs:
                    h.solve_losm(implicit=True, **kw)
        cells = bt.read_tallies(H.TALLY_CELLS)
        for r, h in enumerate(hs):
            assert_tallies_match(cells[r], h.read_tallies(H.TALLY_CELLS), what=f"fp32 replica {r} step {n}")
    for h in hs:
        h.close()
    bt.close()


def test_batch_error_paths():
    need_gpu()
    ws = uneven_replicas(n_steps=2)[:3]
    specs = [H.spec_from_workload(w) for w in ws]
    bad = [H.spec_from_workload(ws[0]), H.spec_from_workload(ws[1].with_(n_chunks=3))]
    with pytest.raises(H.HwwError) as e:
        H.Batch(bad)
    assert e.value.code == -1
    bt = H.Batch(specs)
    v = bt.replica(1)
    with pytest.raises(H.HwwError) as e:
        v.sweep_step(1, 0)
    assert e.value.code == -2
    with pytest.raises(H.HwwError) as e:
        bt.replica(3)
    assert e.value.code == -1
    bt.sweep_step(1, 0, stats=True)
    with pytest.raises(H.HwwError) as e:
        bt.autotune()
    assert e.value.code == -2
    bt.close()
