"""The boundary's normalised tally reads and the adjoint of a given
functional derivative, through the C ABI.

hww_read_tallies(raw = 0) returns the per-batch arrays normalised per source
particle (Eqs. phi-mc, ct-mc); summed over batches they are the estimates the
oracle hands to the LOSM solve (time-layer cells and faces, compared to
1e-12) and, at c = 0, the closed-form step averages of the uncollided pulse
(track-length cells, within 3 sigma).  hww_losm_adjoint(dG_dphi) gives the
gradient of any functional of the march's flux history (Sec. 3 Eq.
losm-disc), against the oracle's adjoint of the same functional."""
import numpy as np
import pytest

import closed_forms as CF
from gpu_common import need_gpu, oracle_opts, oracle_sim, say
from oracle import oracle as O
from paper_2512_19925_amd import hww as H
from paper_2512_19925_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_normalised_reads_match_oracle_inputs():
    need_gpu()
    w = W.plain_small().with_(n_src=20000, n_steps=3)
    say(f"case {w.name}: normalised reads after steps 1-2, {w.n_src} particles")
    h = H.Handle(H.spec_from_workload(w))
    sim = oracle_sim(w)
    opts = oracle_opts(w)
    for n in range(1, 3):
        h.solve_losm(implicit=False, **H.losm_kwargs(w))
        sim.solve_losm(opts, implicit=False)
        for p in range(w.n_chunks):
            h.sweep_step(n, p, stats=False)
            sim.sweep(n, p)
            if p < w.n_chunks - 1:
                h.solve_losm(implicit=True, **H.losm_kwargs(w))
                sim.solve_losm(opts, implicit=True)
        cells = h.read_tallies(H.TALLY_CELLS, raw=False).sum(0)
        bnd = h.read_tallies(H.TALLY_BOUNDARY, raw=False).sum(0)
        phi_o, J_o, F_o, _, P = sim.losm_inputs(implicit=False)
        I = w.n_cells
        scale = np.abs(phi_o).max()
        assert np.max(np.abs(cells[:, 3] - phi_o[1:I + 1])) <= 1e-12 * scale
        assert np.max(np.abs((cells[:, 3] / 3.0 - cells[:, 5]) - F_o[1:I + 1])) <= 1e-12 * scale
        np.testing.assert_allclose(bnd[:, 0], phi_o[[0, I + 1]], rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(bnd[:, 1], P, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(bnd[:, 2], F_o[[0, I + 1]], rtol=1e-12, atol=1e-300)
        # the raw read is unchanged by the normalised one, and the kinds that
        # have no normalisation read the same either way
        raw = h.read_tallies(H.TALLY_CELLS)
        dx = np.diff(w.edges)
        np.testing.assert_allclose(raw[..., 3].sum(0) / (w.n_src * dx), cells[:, 3], rtol=1e-13, atol=0)
        np.testing.assert_array_equal(h.read_tallies(H.TALLY_TRACKS, raw=False), h.read_tallies(H.TALLY_TRACKS))


def test_normalised_track_reads_match_uncollided_pulse():
    # c = 0: the track-length moments over a step are the closed-form step
    # and cell averages of the uncollided pulse.
    need_gpu()
    w = W.homogeneous("uncollided-80c", -4.0, 4.0, 80, 1.0, 0.0, dt=0.25, n_steps=8, n_src=200000)
    say(f"case {w.name}: analog, {w.n_src} particles")
    h = H.Handle(H.spec_from_workload(w.with_(analog=True)))
    edges = w.edges
    zs = []
    for n in range(1, w.n_steps + 1):
        for p in range(w.n_chunks):
            h.sweep_step(n, p, stats=False)
        per = h.read_tallies(H.TALLY_CELLS, raw=False)
        sig = CF.batch_sigma(per[..., :3])
        est = per[..., :3].sum(0)
        t0, t1 = (n - 1) * w.dt, n * w.dt
        for i in range(w.n_cells):
            ex = CF.uncollided_cell_time_avg(edges[i], edges[i + 1], t0, t1, 1.0, 1.0)
            for k in (0, 2):
                if sig[i, k] > 0:
                    zs.append((est[i, k] - ex[k]) / sig[i, k])
                else:
                    assert est[i, k] == 0.0 and abs(ex[k]) < 1e-12
    zs = np.array(zs)
    say(f"  {len(zs)} cells, max |z| {np.abs(zs).max():.2f}, mean z^2 {np.mean(zs ** 2):.2f}")
    assert np.mean(np.abs(zs) > 3) < 0.02 and np.abs(zs).max() < 5.5


def test_adjoint_of_a_given_functional_derivative():
    need_gpu()
    w = W.adjoint_slab(n_src=1000).with_(n_steps=12)
    N = w.n_steps
    I = w.n_cells
    x = 0.5 * (w.edges[1:] + w.edges[:-1])
    F = np.zeros((N + 1, I + 2))
    for n in range(N + 1):
        F[n, 1:-1] = 0.02 * np.exp(-(x / (1 + 0.2 * n)) ** 2)
    P = np.full((N + 1, 2), 1e-4)
    phi0 = np.concatenate([[0.0], np.exp(-x ** 2), [0.0]])
    J0 = np.zeros(I + 1)
    wt = W.adjoint_weights(w, N)
    h = H.Handle(H.spec_from_workload(w))
    h.losm_march(w.sigma_t, w.sigma_s, 0.5, F, P, phi0, J0, wt)
    gt0, gs0 = h.losm_adjoint()
    oph, ojh = O.losm_march(w.edges, w.sigma_t, w.sigma_s, w.speed, w.dt, 0.5, F, P, phi0, J0)
    # twice the weights: exactly twice the gradient (a power-of-two scale)
    gt2, gs2 = h.losm_adjoint(2.0 * wt)
    np.testing.assert_array_equal(gt2, 2.0 * gt0)
    np.testing.assert_array_equal(gs2, 2.0 * gs0)
    # another functional: the sum of phi^2 over cells [300, 400) at the last
    # step, dG/dphi = 2 phi there, against the oracle's adjoint
    d = np.zeros_like(wt)
    d[N, 301:401] = 2.0 * oph[N, 301:401]
    gt, gs = h.losm_adjoint(d)
    ogt, ogs = O.losm_adjoint(w.edges, w.sigma_t, w.sigma_s, w.speed, w.dt, 0.5, oph, ojh, d)
    big = max(np.abs(ogt).max(), np.abs(ogs).max())
    assert big > 0
    assert max(np.abs(gt - ogt).max(), np.abs(gs - ogs).max()) <= 1e-10 * big
    # the march's own weights still apply when no derivative is given
    gt3, gs3 = h.losm_adjoint()
    np.testing.assert_array_equal(gt3, gt0)
    np.testing.assert_array_equal(gs3, gs0)
