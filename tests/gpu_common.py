"""Helpers of the GPU parity tests: run the same workload on the HIP path
(through the C ABI) and on the CPU oracle, and compare."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2512_19925_amd import hww as H


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def oracle_sim(w):
    sim = O.OracleSim(w.edges, w.sigma_t, w.sigma_s, w.speed, w.dt, w.n_steps, w.src_x, w.n_src,
                      w.capacity(), w.seed, w.replica, w.n_batches, w.n_chunks, sigma_f=w.sigma_f,
                      nu_f=w.nu_f, track_moments=w.track_moments)
    sim.set_comb_mode(1 if w.comb_by_index else 0)
    return sim


def oracle_opts(w):
    return O.LosmOpts(theta=w.theta, filter=w.filter, ma_k=w.ma_k, eps_min=w.eps_min, rho=w.rho,
                      closure_track=w.closure_track, kappa=w.kappa, lagged=int(w.lagged),
                      window_scale=int(w.window_scale))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tally_scale(o):
    """Per-entry scale of the 1e-12 relative bound: phi and K against
    themselves, J against phi of the same cell and estimator."""
    a = np.abs(o)
    s = a.copy()
    s[..., 1] = a[..., 0]
    s[..., 4] = a[..., 3]
    return s


def assert_tallies_match(g, o, rtol=1e-12, what=""):
    s = tally_scale(o)
    zero = (o == 0.0)
    assert np.all(g[zero] == 0.0), f"{what}: GPU scored where the oracle did not"
    rel = np.abs(g - o) / np.where(s > 0, s, 1.0)
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= rtol, f"{what}: max relative difference {worst:.3e}"
    return worst


def assert_bnd_match(g, o, rtol=1e-12, what=""):
    s = np.abs(o).max() + 1e-300
    d = np.abs(g - o).max() if o.size else 0.0
    assert d <= rtol * s, f"{what}: boundary tallies differ by {d:.3e}"


def assert_bank_match(gb, ob, what=""):
    """Census banks as multisets keyed by (src, lineage): same members,
    directions and positions (both sides take the same steps, the flight
    logarithm included), weights within the rounding of the window centres
    that roulette sets them to."""
    assert len(gb["src"]) == len(ob["src"]), f"{what}: bank sizes {len(gb['src'])} vs {len(ob['src'])}"
    if len(ob["src"]) == 0:
        return
    kg = np.lexsort((gb["lin"], gb["src"]))
    ko = np.lexsort((ob["lin"], ob["src"]))
    for f in ("src", "lin", "e", "cell", "chunk"):
        assert np.array_equal(gb[f][kg], ob[f][ko]), f"{what}: field {f} differs"
    np.testing.assert_allclose(gb["w"][kg], ob["w"][ko], rtol=1e-12, atol=0, err_msg=what)
    np.testing.assert_array_equal(gb["mu"][kg], ob["mu"][ko], err_msg=what)
    np.testing.assert_array_equal(gb["x"][kg], ob["x"][ko], err_msg=what)


KIND_NAMES = ("track phi", "track J", "track K", "census phi", "census J", "census K")


def precision_error(steps_g, steps_o, floor=1e-3):
    """Error of reduced-precision tallies against FP64 ones of the same seed,
    per tally kind over all cells and steps.  Each step gives [B][I][6] raw
    per-batch sums.  z = (T_g - T_o) / sigma_o with sigma_o the batch
    standard deviation of the FP64 sum (cells where it is 0 are left out of
    z); relative error against |T_o|, J against phi of the same cell and
    estimator, over cells above floor times the step's largest."""
    zs = [[] for _ in range(6)]
    rel = [[] for _ in range(6)]
    for g, o in zip(steps_g, steps_o):
        B = o.shape[0]
        To, Tg = o.sum(0), g.sum(0)
        sig = np.sqrt(B / (B - 1.0) * ((o - To / B) ** 2).sum(0))
        scale = np.abs(To)
        scale[:, 1] = scale[:, 0]
        scale[:, 4] = scale[:, 3]
        for k in range(6):
            m = sig[:, k] > 0
            zs[k].append((Tg[m, k] - To[m, k]) / sig[m, k])
            mr = scale[:, k] > floor * scale[:, k].max() if scale[:, k].max() > 0 else np.zeros(len(To), bool)
            rel[k].append(np.abs(Tg[mr, k] - To[mr, k]) / scale[mr, k])
    out = {}
    for k in range(6):
        z = np.concatenate(zs[k])
        r = np.concatenate(rel[k])
        out[KIND_NAMES[k]] = {"n": int(z.size), "max_abs_z": float(np.abs(z).max()) if z.size else 0.0,
                              "frac_within_3sigma": float(np.mean(np.abs(z) <= 3.0)) if z.size else 1.0,
                              "median_rel_err": float(np.median(r)) if r.size else 0.0,
                              "max_rel_err": float(r.max()) if r.size else 0.0}
    return out
