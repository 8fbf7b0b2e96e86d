"""Full-size checks in the launch configuration the benchmark times: the
1000-cell, 1e7-particle problem with 32 batches and three window updates per
step.  With windows fed identically to both sides, the tallies of batch 0
(the histories with src mod 32 = 0, about 3.1e5 of them) are replayed on the
oracle and must match to 1e-12; with the HLOSM windows the method's
invariants are checked at full size."""
import math

import numpy as np
import pytest

import closed_forms as CF
from gpu_common import assert_tallies_match, need_gpu, say
from oracle import oracle as O
from paper_2512_19925_amd import hww as H
from paper_2512_19925_amd import workloads as W

pytestmark = pytest.mark.gpu


def _windows(w):
    xc = 0.5 * (w.edges[1:] + w.edges[:-1])

    def f(n):
        t = n * w.dt
        return np.exp(-0.5 * (xc / (0.2 + 0.7 * t)) ** 2) + 1e-3
    return f


def test_fullsize_batch0_matches_oracle():
    need_gpu()
    w = W.full_scale(c=0.9, rho=5.0)
    steps = 3
    say(f"case {w.name}: n_src={w.n_src}, {steps} steps, fixed windows, oracle replays batch 0")
    h = H.Handle(H.spec_from_workload(w))
    # The source bank holds every history before the batch mask; batch 0 is
    # 1/32 of them, so 1.2 n_src is ample.
    sim = O.OracleSim(w.edges, w.sigma_t, w.sigma_s, w.speed, w.dt, w.n_steps, w.src_x, w.n_src,
                      int(1.2 * w.n_src), w.seed, w.replica, w.n_batches, w.n_chunks)
    mask = np.zeros(w.n_batches, np.uint8)
    mask[0] = 1
    sim.set_batch_mask(mask)
    win = _windows(w)
    for n in range(1, steps + 1):
        h.set_windows(win(n), w.rho)
        sim.set_windows(win(n), w.rho)
        for p in range(w.n_chunks):
            h.sweep_step(n, p, stats=False)
            sim.sweep(n, p)
        g = h.read_tallies(H.TALLY_CELLS)[:1]
        o = sim.tallies()[0][:1]
        worst = assert_tallies_match(g, o, what=f"full-size batch 0 step {n}")
        say(f"  step {n}: batch-0 max relative difference {worst:.2e}")
    h.close()


def test_fullsize_hww_invariants():
    # Full method (HLOSM windows, MA filter) at full size: the census weight
    # follows exp(-(1-c) t) within its batch spread, track and census flux are
    # non-negative, every segment ends in one event, and the population stays
    # within the bank.
    need_gpu()
    w = W.full_scale(c=0.9, rho=5.0)
    steps = 6
    say(f"case {w.name}: HWW invariants over {steps} steps")
    h = H.Handle(H.spec_from_workload(w))
    recs = []

    def on_step(n, hh, st):
        cells = hh.read_tallies(H.TALLY_CELLS)
        s = st[-1]
        recs.append((n, cells, s))

    H.run(h, w, steps=steps, on_step=on_step)
    for n, cells, s in recs:
        t = n * w.dt
        per_batch = cells[..., 3].sum(1) / w.speed / (w.n_src / w.n_batches)  # census weight per source, per batch
        mean = per_batch.mean()
        se = per_batch.std(ddof=1) / math.sqrt(w.n_batches)
        expect = math.exp(-(1 - 0.9) * t)
        say(f"  step {n}: census weight {mean:.6f} +- {se:.1e} vs {expect:.6f}; census {s['census']}")
        assert abs(mean - expect) < 5 * se + 1e-12
        assert np.all(cells[..., 0] >= 0) and np.all(cells[..., 2] >= 0) and np.all(cells[..., 3] >= 0)
        assert s["segments"] == s["census"] + s["crossings"] + s["collisions"] + s["leaks"]
        assert s["collisions"] == s["scatters"] + s["absorptions"]
        assert s["census"] <= w.capacity()
