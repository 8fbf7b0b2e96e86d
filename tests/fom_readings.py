"""Figure-of-merit readings of the paper's own problem on the CPU oracle.

The paper reports (Sec. 5, FOM comparison) that moving-average filtered
hybrid weight windows improve FOM_Error (Eq. FOM_error) over analog Monte
Carlo by 1.25x on average on its supercritical pulse problem (Sec. 5.1:
fission with c_eff = 1.1, 201 cells, 20 steps of dt = 1, H = 1e4 histories
per step kept by uniform combing, rho = 1.25, eps_min = 1e-3).  Several
steps of that comparison are not fixed by the text; this script runs the
oracle under each reading and prints the FOM ratios to analog:

  comb      'weight': comb teeth spaced in cumulative weight, every copy of
            weight W / H; 'index': teeth spaced in particle index, every copy
            keeping its particle's weight times n / H (Sec. 5.1 names the
            comb only by reference; Sec. 5 remarks that it thins the
            particles of weight near 1 at the source)
  centres   'scaled': window centres of Eq. ww-center times the start weight
            per source particle (reading R13); 'printed': largest centre 1
  error     'step': the track-length flux of the step (Eq. phi-mc) against
            the exact step average; 'layer': the time-layer flux at t^n
            (Eq. ct-mc) against the exact cell average at t^n

The cost of a step (tau^n of Eqs. FOM_sigma, FOM_error) is its number of
flight segments, a serial code's runtime.  FOMs are averaged over the seeds
per step, then the ratio to analog is averaged over the 20 steps, as the
benchmark does on the GPU.

Test infrastructure (it runs the oracle): python tests/fom_readings.py
[--seeds N] [--methods HWW-MA,...]
"""
from __future__ import annotations

import argparse
import itertools
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from gpu_common import oracle_opts, oracle_sim  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2512_19925_amd import pulse_reference as P  # noqa: E402
from paper_2512_19925_amd import workloads as W  # noqa: E402


def cell_layer_averages(edges, t, c, ng=24):
    """Average of the exact flux over every cell at time t (sigma_t = v = 1):
    the uncollided part exactly, the collided part by Gauss-Legendre over
    the part of the cell inside the light cone."""
    gx, gw = np.polynomial.legendre.leggauss(ng)
    out = np.zeros(len(edges) - 1)
    for i, (a, b) in enumerate(zip(edges[:-1], edges[1:])):
        lo, hi = max(a, -t), min(b, t)
        if hi <= lo:
            continue
        val = np.exp(-t) / (2.0 * t) * (hi - lo)
        xx = 0.5 * (hi - lo) * (gx + 1.0) + lo
        val += float(np.sum(0.5 * (hi - lo) * gw * P.collided_flux(xx, t, c)))
        out[i] = val / (b - a)
    return out


def fom_sigma(per_batch):
    B = per_batch.shape[0]
    tot = per_batch.sum(0)
    sig = np.sqrt(B / (B - 1.0) * ((per_batch - tot / B) ** 2).sum(0))
    m = tot > 0
    return 1.0 / np.mean((sig[m] / tot[m]) ** 2) if np.any(m) else 0.0


def fom_error(phi, ref):
    m = ref > 0
    return 1.0 / np.mean(((phi[m] - ref[m]) / ref[m]) ** 2) if np.any(m) else 0.0


METHODS = {
    "analog": dict(analog=True),
    "HWW": dict(filter=0),
    "HWW-MA": dict(),
    "HWW-F": dict(filter=2, kappa=30),
    "LWW": dict(filter=0, lagged=True),
}


def run_method(w, comb_mode, seeds, refs):
    """Per-step FOMs (cost = segments) averaged over the seeds."""
    dx = np.diff(w.edges)
    n = w.n_steps
    acc = {k: np.zeros(n) for k in ("sig", "err_step", "err_layer")}
    segs = 0
    for sd in range(seeds):
        ws = w.with_(seed=1 + sd)
        sim = oracle_sim(ws)
        sim.set_comb_mode(comb_mode)
        rec = []

        def on_step(k, s):
            cells, _ = s.tallies()
            seg = s.counters()["segments"]
            track = cells[..., 0] / (ws.n_src * dx * ws.dt)       # per batch, step average
            layer = cells[..., 3].sum(0) / (ws.n_src * dx)           # time layer at t^n (v w per particle)
            rec.append((seg, fom_sigma(track), fom_error(track.sum(0), refs["step"][k - 1]),
                        fom_error(layer, refs["layer"][k - 1])))

        O.run(sim, ws.n_steps, None if ws.analog else oracle_opts(ws), on_step=on_step, comb=ws.comb)
        for k, (seg, fs, fe_s, fe_l) in enumerate(rec):
            acc["sig"][k] += fs / seg / seeds
            acc["err_step"][k] += fe_s / seg / seeds
            acc["err_layer"][k] += fe_l / seg / seeds
            segs += seg
    acc["segments_per_step"] = segs / (seeds * n)
    return acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=10)
    ap.add_argument("--methods", default="HWW,HWW-MA,HWW-F,LWW")
    args = ap.parse_args()
    base = W.paper_fission()
    c_eff = 1.1
    refs = {"step": P.cell_step_averages(base.edges, base.dt, base.n_steps, c_eff),
            "layer": np.array([cell_layer_averages(base.edges, k * base.dt, c_eff)
                               for k in range(1, base.n_steps + 1)])}
    print(f"paper problem: {base.n_cells} cells, {base.n_steps} steps of dt={base.dt}, H={base.comb}, "
          f"rho={base.rho}, eps_min={base.eps_min}, {args.seeds} seeds; cost = segments of the step")
    print("| comb | centres | method | segments/step vs analog | FOM_sigma | FOM_Error (step) | FOM_Error (layer) |")
    print("|---|---|---|---|---|---|---|")
    for comb_mode, scale in itertools.product((0, 1), (0, 1)):
        w0 = base.with_(window_scale=scale)
        a = run_method(w0.with_(**METHODS["analog"]), comb_mode, args.seeds, refs)
        for name in args.methods.split(","):
            r = run_method(w0.with_(**METHODS[name]), comb_mode, args.seeds, refs)
            ratio = {k: float(np.mean(r[k] / a[k])) for k in ("sig", "err_step", "err_layer")}
            print(f"| {'weight' if comb_mode == 0 else 'index'} | {'scaled' if scale == 0 else 'printed'} | "
                  f"{name} | {r['segments_per_step'] / a['segments_per_step']:.2f} | {ratio['sig']:.2f} | "
                  f"{ratio['err_step']:.2f} | {ratio['err_layer']:.2f} |", flush=True)


if __name__ == "__main__":
    main()
