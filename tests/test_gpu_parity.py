"""GPU parity: the HIP sweep and LOSM solve (called through the C ABI)
against the CPU oracle on the same seeded inputs.  FP64 tallies must agree
to 1e-12 relative per batch and cell (summation order is the only
difference), event counters exactly, census banks as multisets."""
import numpy as np
import pytest

from gpu_common import (assert_bank_match, assert_bnd_match, assert_tallies_match, need_gpu,
                        oracle_opts, oracle_sim, say)
from oracle import oracle as O
from paper_2512_19925_amd import hww as H
from paper_2512_19925_amd import workloads as W

pytestmark = pytest.mark.gpu

COUNTERS = ["segments", "collisions", "scatters", "absorptions", "crossings", "leaks", "census",
            "splits", "daughters", "rr_kill", "rr_survive", "histories"]


def _compare_step(n, h, sim, what, banks=True):
    g = h.read_tallies(H.TALLY_CELLS)
    o, ob = sim.tallies()
    worst = assert_tallies_match(g, o, what=f"{what} step {n}")
    assert_bnd_match(h.read_tallies(H.TALLY_BOUNDARY), ob, what=f"{what} step {n}")
    assert np.array_equal(h.read_tallies(H.TALLY_TRACKS), sim.tracks()), f"{what} step {n}: tracks"
    if banks:
        assert_bank_match(h.read_bank(1), sim.bank(1), what=f"{what} step {n}")
    return worst


def _run_pair(w, steps=None, fixed_windows=None, banks=True, analog=False):
    need_gpu()
    steps = w.n_steps if steps is None else steps
    say(f"case {w.name}: n_src={w.n_src} I={w.n_cells} B={w.n_batches} chunks={w.n_chunks} steps={steps}")
    h = H.Handle(H.spec_from_workload(w))
    sim = oracle_sim(w)
    opts = oracle_opts(w)
    kw = H.losm_kwargs(w)
    worst = 0.0
    for n in range(1, steps + 1):
        if fixed_windows is not None:
            c = fixed_windows(n)
            h.set_windows(c, w.rho)
            sim.set_windows(c, w.rho)
        elif not analog:
            h.solve_losm(implicit=False, **kw)
            sim.solve_losm(opts, implicit=False)
        for p in range(w.n_chunks):
            st = h.sweep_step(n, p, stats=(p == w.n_chunks - 1 or p % 2 == 1))
            sim.sweep(n, p)
            if fixed_windows is None and not analog and not w.lagged and p < w.n_chunks - 1:
                h.solve_losm(implicit=True, **kw)
                sim.solve_losm(opts, implicit=True)
        oc = sim.counters()
        cnt = {k: st[k] for k in COUNTERS}
        assert cnt == {k: oc[k] for k in COUNTERS}, f"step {n}: counters {cnt} vs {oc}"
        worst = max(worst, _compare_step(n, h, sim, w.name, banks=banks))
        if not analog and fixed_windows is None:
            gw = h.read_tallies(H.TALLY_WINDOWS)
            ow = sim.windows()
            if ow is None:  # no windows yet (lagged windows in the first step)
                assert not np.any(gw[0])
            else:
                np.testing.assert_allclose(gw[0], ow[0], rtol=1e-12)
    say(f"  max relative tally difference {worst:.2e}")
    h.close()
    return worst


def test_plain_small_end_to_end():
    # 200 cells, c = 0.9, 20 steps, 1e4 particles, rho = 5, three window
    # updates per step; each side computes its own windows.
    _run_pair(W.plain_small())


def test_filtered_end_to_end():
    _run_pair(W.plain_small().with_(name="plain-ma", filter=1, n_src=5000, n_steps=10))


def test_backward_euler_and_track_closures():
    _run_pair(W.plain_small().with_(name="be-track", theta=1.0, closure_track=1, n_src=4000, n_steps=8))


@pytest.mark.parametrize("tm", [1, 2])
def test_fewer_track_moments(tm):
    # Census closures need only the track-length phi; track_moments 2 keeps
    # K for track-length closures.
    w = W.plain_small().with_(name=f"track-moments-{tm}", n_src=4000, n_steps=6, track_moments=tm,
                              closure_track=1 if tm == 2 else 0)
    _run_pair(w)


def test_track_closures_need_k():
    need_gpu()
    h = H.Handle(H.spec_from_workload(W.plain_small().with_(n_steps=2, track_moments=1)))
    for p in range(4):
        h.sweep_step(1, p, stats=False)
    with pytest.raises(H.HwwError) as e:
        h.solve_losm(implicit=False, closure_track=1)
    assert e.value.code == -1
    h.close()


def test_large_mesh_fallback_paths():
    # 3000 cells: the cell records no longer fit in LDS beside the histogram
    # (global-memory flights), the LOSM working arrays (6 x 3002 doubles
    # beside 6003 unknowns) leave LDS, and each thread has more substitution
    # rows (6) than it keeps in registers (4).
    w = W.homogeneous("large-mesh-3000c", -30.0, 30.0, 3000, 1.0, 0.9, dt=0.1, n_steps=5, n_src=6000,
                      rho=5.0, filter=1, ma_k=3)
    _run_pair(w)


def test_largest_mesh():
    # The largest mesh the LDS histogram takes (3136 cells, 4 chunks), with
    # MA-filtered windows: the maximum size of the sweep's per-work-group
    # state.
    w = W.homogeneous("mesh-3136c", -31.36, 31.36, 3136, 1.0, 0.9, dt=0.1, n_steps=4, n_src=5000,
                      rho=5.0, filter=1, ma_k=3)
    _run_pair(w)


def test_fourier_filtered_end_to_end():
    # Fourier low pass (kappa = 30 of 200 cells) on the closures and the
    # initial condition of every solve.
    _run_pair(W.plain_small().with_(name="plain-fourier", filter=2, kappa=30, n_src=6000, n_steps=10))


def test_lagged_windows_end_to_end():
    # Lagged weight windows: the previous step's track-length flux sets the
    # windows at the start of every step (the first step runs analog).
    # eps_min = 0.05 bounds the splitting where the particles outrun the
    # lagged shape.
    _run_pair(W.plain_small().with_(name="lagged", lagged=True, n_src=6000, n_steps=10, eps_min=0.05,
                                    bank_capacity=60_000))


def test_analog():
    _run_pair(W.plain_small().with_(name="analog", n_src=7777), analog=True)


def _peaked(w):
    xc = 0.5 * (w.edges[1:] + w.edges[:-1])

    def f(n):
        t = n * w.dt
        return np.exp(-0.5 * (xc / (0.3 + t)) ** 2) + 1e-3
    return f


@pytest.mark.parametrize("n_chunks,B", [(1, 1), (3, 7), (8, 64), (4, 32)])
def test_fixed_windows_chunks_batches(n_chunks, B):
    w = W.plain_small().with_(name=f"fixed-c{n_chunks}-b{B}", n_chunks=n_chunks, n_batches=B,
                              n_src=3001, n_steps=6)
    _run_pair(w, fixed_windows=_peaked(w))


@pytest.mark.parametrize("n_src", [1, 63, 65, 257, 1000])
def test_ragged_small_banks(n_src):
    w = W.plain_small().with_(name=f"ragged-{n_src}", n_src=n_src, n_steps=5)
    _run_pair(w)


def test_leakage_small_domain():
    # A 1-mfp slab: particles leak through both faces; the face tallies and
    # P_L, P_R enter the LOSM solve.
    w = W.homogeneous("leak", -0.5, 0.5, 10, 1.0, 0.8, dt=0.2, n_steps=8, n_src=4000, rho=3.0)
    w = w.with_(eps_min=0.05, bank_capacity=400_000)
    _run_pair(w)


def test_single_cell_and_off_edge_source():
    w = W.homogeneous("one-cell", -1.0, 1.0, 1, 2.0, 0.5, dt=0.1, n_steps=6, n_src=2000, src_x=0.3)
    _run_pair(w)
    w = W.homogeneous("off-edge", -3.0, 3.0, 30, 1.0, 0.95, dt=0.05, n_steps=6, n_src=2000, src_x=0.0123,
                    bank_capacity=1_000_000)
    _run_pair(w)


def test_heavy_splitting():
    # Low window floor and narrow windows: many daughters, several daughter
    # generations per chunk.
    w = W.plain_small().with_(name="split-heavy", eps_min=1e-5, rho=1.25, n_src=3000, n_steps=6,
                              bank_capacity=3_000_000)
    _run_pair(w)


def test_empty_source():
    need_gpu()
    w = W.plain_small().with_(name="empty", n_src=0, n_steps=2)
    h = H.Handle(H.spec_from_workload(w))
    h.set_windows(None, 5.0)
    for p in range(w.n_chunks):
        st = h.sweep_step(1, p)
        assert st["segments"] == 0 and st["launches"] == p + 1
    assert np.all(h.read_tallies(H.TALLY_CELLS) == 0.0)


def test_error_paths():
    need_gpu()
    w = W.plain_small().with_(name="errors", n_src=2000, n_steps=3)
    h = H.Handle(H.spec_from_workload(w))
    with pytest.raises(H.HwwError) as e:
        h.sweep_step(2, 0)
    assert e.value.code == -2
    with pytest.raises(H.HwwError) as e:
        h.solve_losm(implicit=True)
    assert e.value.code == -2
    with pytest.raises(H.HwwError) as e:
        h.set_windows(np.full(w.n_cells, -1.0), 5.0)
    assert e.value.code == -5
    h.sweep_step(1, 0)
    with pytest.raises(H.HwwError) as e:
        h.sweep_step(1, 2)
    assert e.value.code == -2
    # A bank too small for the split population: capacity error.
    w2 = W.plain_small().with_(name="overflow", n_src=2000, n_steps=2, bank_capacity=2500)
    h2 = H.Handle(H.spec_from_workload(w2))
    h2.set_windows(np.full(w2.n_cells, 0.25), 2.0)
    with pytest.raises(H.HwwError) as e:
        for p in range(w2.n_chunks):
            h2.sweep_step(1, p)
    assert e.value.code == -3


def test_timing_off_records_nothing_and_changes_nothing():
    # Without the timing events the sweep is the same; kernel_ms stays 0.
    need_gpu()
    w = W.plain_small().with_(name="timing", n_src=3000, n_steps=3)
    sim = oracle_sim(w)
    h = H.Handle(H.spec_from_workload(w))
    h.set_timing(False)
    opts = oracle_opts(w)
    kw = dict(theta=w.theta, filter=w.filter, ma_k=w.ma_k, eps_min=w.eps_min, rho=w.rho,
              closure_track=w.closure_track)
    for n in range(1, 4):
        h.solve_losm(implicit=False, **kw)
        sim.solve_losm(opts, implicit=False)
        for p in range(w.n_chunks):
            st = h.sweep_step(n, p, stats=(p == w.n_chunks - 1))
            sim.sweep(n, p)
            if p < w.n_chunks - 1:
                h.solve_losm(implicit=True, **kw)
                sim.solve_losm(opts, implicit=True)
        assert st["kernel_ms"] == 0.0 and st["launches"] == w.n_chunks
        _compare_step(n, h, sim, w.name)
    tot = h.run_stats()
    assert tot["kernel_ms"] == 0.0 and tot["launches"] == 3 * w.n_chunks
    h.close()
