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
    return O.OracleSim(w.edges, w.sigma_t, w.sigma_s, w.speed, w.dt, w.n_steps, w.src_x, w.n_src,
                       w.capacity(), w.seed, w.replica, w.n_batches, w.n_chunks, sigma_f=w.sigma_f,
                       nu_f=w.nu_f, track_moments=w.track_moments)


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
