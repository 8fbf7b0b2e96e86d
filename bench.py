"""Benchmark of the hybrid weight-window sweep on one MI355X.

A step is one time step of the method on the full-scale problem (1000 cells
on [-50, 50], sigma_t = 1, c = 0.9, 1e7 source particles, dt = 0.05,
moving-average filtered HLOSM windows with rho = 5, eps_min = 1e-3 and three
window updates per step): the semi-implicit solve, four chunks of particle
histories with their daughters, and three fully implicit solves.

Prints one JSON line: particle segments/s over the timed steps (inputs
resident in HBM), the sweep kernel's HBM-roofline figures measured with HIP
events on the library's stream, the figure-of-merit gain over the plain
(analog) FP64 sweep of the same problem, the CPU oracle timed on a bounded
sample of the same workload, and three side figures: the batched form (256
uneven replicas, one persistent launch per chunk) against one handle per
replica, the FP32 flight arithmetic against FP64 on the precision form, and
the paper's own supercritical problem (fission, uniform combing) for the
paper's methods against analog.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle segments/s and FOM per time step vs plain FP64 sweep, 1 MI355X"
HBM_PEAK_GBS = 8000.0
# Timed runs of the throughput and roofline passes (after one warm-up run):
# the median is reported.
REPEATS = 5
# HBM traffic of the sweep kernel measured by rocprofv3 on the bench's own
# passes (FETCH_SIZE and WRITE_SIZE, scaled by a plain-copy calibration), as
# a ratio to the algorithmic bytes of the same launches; and its VALU issue
# and lane counters.  Valid only for the kernel sources they were measured on.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sweep_full-1000c-c0.9-rho5_hbm_traffic.md")
VALU_PROFILE = os.path.join(ROOT, "profiles", "sweep_full-1000c-c0.9-rho5_valu.md")
# The sweep kernel's sources and the compiler flags it is built with.
SWEEP_SOURCES = [os.path.join(ROOT, "paper_2512_19925_amd", "csrc", f) for f in ("hww_sweep.hip", "hww_internal.h")] + \
    [os.path.join(ROOT, "paper_2512_19925_amd", "build.py")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=95)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--c", type=float, default=0.9)
    ap.add_argument("--rho", type=float, default=5.0)
    ap.add_argument("--n-src", type=int, default=10_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-analog", action="store_true", help="skip the plain-sweep FOM comparison")
    ap.add_argument("--sweep", action="store_true", help="also run every (c, rho) pair of the workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form figures")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 figures")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's supercritical problem")
    ap.add_argument("--batch-steps", type=int, default=50)
    ap.add_argument("--batch-compare-steps", type=int, default=10,
                    help="steps of the one-handle-per-replica comparison of the batched form (0: skip it)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--out", default=None, help="also write per-step records (JSON) here")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM-counter calibration) and exit")
    return ap.parse_args()


def fom_sigma(cells, n_src, dx, dt):
    """FOM_sigma of the track-length flux (Sec. 5, Eq. FOM_sigma without the
    runtime): 1 / mean over cells with flux of (sigma_i / phi_i)^2, with
    sigma from the spread of the batch sums."""
    per = cells[..., 0] / (n_src * dx[None, :] * dt)
    B = per.shape[0]
    tot = per.sum(0)
    sig = np.sqrt(B / (B - 1.0) * ((per - tot / B) ** 2).sum(0))
    m = tot > 0
    if not np.any(m):
        return 0.0
    return 1.0 / np.mean((sig[m] / tot[m]) ** 2)


def _step(h, w, n, analog, kw, stats):
    if not analog:
        h.solve_losm(implicit=False, **kw)
    st = None
    for p in range(w.n_chunks):
        st = h.sweep_step(n, p, stats=(stats and p == w.n_chunks - 1))
        if not analog and not w.lagged and p < w.n_chunks - 1:
            h.solve_losm(implicit=True, **kw)
    return st


def run_gpu(w, steps_total, warmup, analog, timing=True, tune=False):
    """Timed run: the host queues every step without waiting; one
    synchronisation at each end of the timed region.  Counters and the sweep
    kernels' HIP-event times (timing on) come from the library's run
    totals.  tune: the sweep's launch shape from the library's tuner instead
    of the default one (the tuner times chunk 0 of step 1, where every
    particle still sits at the pulse; on the full-scale problem it picks
    512-particle tiles, which make steps 6-25 8 % slower than the default
    256, so the benchmark keeps the default)."""
    import torch
    from paper_2512_19925_amd import hww as H
    h = H.Handle(H.spec_from_workload(w))
    shape = h.autotune() if tune else None
    h.set_timing(timing)
    kw = H.losm_kwargs(w)
    for n in range(1, warmup + 1):
        _step(h, w, n, analog, kw, stats=False)
    base = h.run_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(warmup + 1, steps_total + 1):
        _step(h, w, n, analog, kw, stats=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot = h.run_stats()
    h.close()
    d = {k: tot[k] - base[k] for k in ("segments", "histories", "census", "daughters", "bytes_moved",
                                       "launches", "kernel_ms")}
    d["wall_s"] = wall
    d["generations"] = tot["generations"]
    d["shape"] = shape
    return d


def fom_error(cells, n_src, dx, dt, ref):
    """FOM_Error without the runtime (Sec. 5, Eq. FOM_error): 1 / mean over
    cells with reference flux of ((phi_mc - phi_ref) / phi_ref)^2; a cell the
    particles have not reached counts as error 1."""
    phi = cells[..., 0].sum(0) / (n_src * dx * dt)
    m = ref > 0
    if not np.any(m):
        return 0.0
    return 1.0 / np.mean(((phi[m] - ref[m]) / ref[m]) ** 2)


def run_fom(w, steps_total, warmup, analog, ref):
    """Per-step pass: tau^n is the wall time of step n (solves, sweeps and the
    wait for them); FOM_sigma^n from the batch spread of the track flux and
    FOM_Error^n from its error against the reference pulse solution ref
    ([steps, I] step and cell averages)."""
    import torch
    from paper_2512_19925_amd import hww as H
    h = H.Handle(H.spec_from_workload(w))
    h.set_timing(False)
    dx = np.diff(w.edges)
    kw = H.losm_kwargs(w)
    foms = []
    torch.cuda.synchronize()
    for n in range(1, steps_total + 1):
        t0 = time.perf_counter()
        _step(h, w, n, analog, kw, stats=True)
        tau = time.perf_counter() - t0
        if n > warmup:
            cells = h.read_tallies(H.TALLY_CELLS)
            foms.append((fom_sigma(cells, w.n_src, dx, w.dt) / tau,
                         fom_error(cells, w.n_src, dx, w.dt, ref[n - 1]) / tau))
    h.close()
    return foms


def sweep_source_hash():
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_figures(path, keys):
    """Figures of a committed rocprofv3 summary (lines 'key: value'), or None
    when the kernel sources differ from the measured ones."""
    try:
        text = open(path).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    if not m_hash or m_hash.group(1) != sweep_source_hash():
        return None
    out = {}
    for k in keys:
        m = re.search(k + r":\s*([0-9.eE+-]+)", text)
        if not m:
            return None
        out[k] = float(m.group(1))
    return out


def host_cpu():
    """CPU model and logical CPU count of the host the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def _batch_steps(bt, steps, kw, first=1):
    for n in range(first, steps + 1):
        bt.solve_losm(implicit=False, **kw)
        for p in range(bt.n_chunks):
            bt.sweep_step(n, p, stats=False)
            if p < bt.n_chunks - 1:
                bt.solve_losm(implicit=True, **kw)


def device_check():
    """The device as the runtime reports it, and the bandwidth of a plain
    device copy (1 GiB read + 1 GiB written, ten copies timed by events on
    the current stream): the measured ceiling beside the published peak."""
    import torch
    pr = torch.cuda.get_device_properties(0)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 10 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"name": pr.name, "arch": pr.gcnArchName, "compute_units": pr.multi_processor_count,
            "hbm_bytes": pr.total_memory, "lds_bytes_per_block": pr.shared_memory_per_block,
            "l2_bytes": pr.L2_cache_size, "copy_GBs": gbs}


def run_batched(steps, compare_steps=10):
    """The batched form: 256 uneven replicas, one persistent sweep launch per
    chunk and one batched LOSM launch per solve, launch shape autotuned.
    Compared with one handle per replica run one after another over the
    first compare_steps steps."""
    import torch
    from paper_2512_19925_amd import hww as H
    from paper_2512_19925_amd import workloads as W
    ws = W.batched_replicas(n_steps=steps)
    w0 = ws[0]
    kw = H.losm_kwargs(w0)
    bt = H.Batch([H.spec_from_workload(w) for w in ws])
    tune = bt.autotune()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _batch_steps(bt, compare_steps, kw)
    torch.cuda.synchronize()
    wall_cmp = time.perf_counter() - t0
    seg_cmp = bt.run_stats()["segments"]
    t1 = time.perf_counter()
    _batch_steps(bt, steps, kw, first=compare_steps + 1)
    torch.cuda.synchronize()
    wall = wall_cmp + (time.perf_counter() - t1)
    st = bt.run_stats()
    bt.close()
    del bt
    torch.cuda.empty_cache()
    # One handle per replica, same steps.
    seg_single, wall_single = 0, 0.0
    for w in (ws if compare_steps > 0 else []):
        h = H.Handle(H.spec_from_workload(w))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in range(1, compare_steps + 1):
            h.solve_losm(implicit=False, **kw)
            for p in range(h.n_chunks):
                h.sweep_step(n, p, stats=False)
                if p < h.n_chunks - 1:
                    h.solve_losm(implicit=True, **kw)
        torch.cuda.synchronize()
        wall_single += time.perf_counter() - t0
        seg_single += h.run_stats()["segments"]
        h.close()
        del h
    torch.cuda.empty_cache()
    return {"workload": f"{len(ws)} replicas, sigma_t~U[0.5,2], c~U[0.3,0.99], cells~logU[100,2000], "
                        f"particles~logU[1e3,1e6] (sum {sum(w.n_src for w in ws)}), [-20,20], dt=0.1, "
                        f"{steps} steps, HWW rho=5 eps_min=1e-3 MA k=3, 3 window updates per step",
            "segments_per_s": st["segments"] / wall, "ms_per_step": wall * 1e3 / steps,
            "kernel_segments_per_s": st["segments"] / (st["kernel_ms"] * 1e-3) if st["kernel_ms"] else None,
            "kernel_achieved_GBs": st["bytes_moved"] / (st["kernel_ms"] * 1e-3) / 1e9 if st["kernel_ms"] else None,
            "kernel_frac_of_hbm_peak": (st["bytes_moved"] / (st["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
                                        if st["kernel_ms"] else None),
            "autotune": tune,
            "steps_1_to_%d" % compare_steps: {
                "batched_segments_per_s": seg_cmp / wall_cmp,
                "one_handle_per_replica_segments_per_s": seg_single / wall_single,
                "speedup": (seg_cmp / wall_cmp) / (seg_single / wall_single)} if compare_steps > 0 else None}


def run_fp32_pair(steps=20, n_src=10_000_000):
    """FP32 against FP64 flight arithmetic on the precision form (the small
    problem's geometry with 1e7 particles), HWW as the small problem."""
    from paper_2512_19925_amd import hww as H
    from paper_2512_19925_amd import workloads as W
    w = W.precision_form(n_src=n_src)
    out = {"workload": f"{w.name}: {w.n_cells} cells on [{w.x_lo},{w.x_hi}], c=0.9, {n_src:.0e} particles, "
                       f"dt={w.dt}, steps 1-{steps}, HWW rho={w.rho} unfiltered"}
    for prec, name in ((H.HWW_FP32, "fp32"), (H.HWW_FP64, "fp64")):
        import torch
        h = H.Handle(H.spec_from_workload(w, precision=prec))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.run(h, w, steps=steps, stats=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = h.run_stats()
        h.close()
        out[f"{name}_segments_per_s"] = st["segments"] / wall
        out[f"{name}_kernel_segments_per_s"] = st["segments"] / (st["kernel_ms"] * 1e-3)
    out["fp32_over_fp64_kernel"] = out["fp32_kernel_segments_per_s"] / out["fp64_kernel_segments_per_s"]
    # Error of the FP32 tallies, every cell and step, against the FP64 path
    # of the same seed (which equals the FP64 oracle within 1e-12 by the
    # parity tests; the oracle at 1e7 particles is run by the test suite).
    steps_t = {}
    for prec in (H.HWW_FP32, H.HWW_FP64):
        h = H.Handle(H.spec_from_workload(w, precision=prec))
        steps_t[prec] = []
        H.run(h, w, steps=steps, stats=False, on_step=lambda n, hh, _: steps_t[prec].append(hh.read_tallies(H.TALLY_CELLS)))
        h.close()
    out["error_vs_fp64"] = precision_error(steps_t[H.HWW_FP32], steps_t[H.HWW_FP64])
    out["error_vs_fp64"]["definition"] = (
        "per tally kind over every cell and step: z = (T32 - T64) / sigma64 with sigma64 the batch standard "
        "deviation of the FP64 sum (cells with sigma64 = 0 left out); relative error |T32 - T64| / |T64| (J: "
        "over phi of the same cell and estimator) over cells above 1e-3 of the step's largest")
    return out


KIND_NAMES = ("track phi", "track J", "track K", "census phi", "census J", "census K")


def precision_error(steps_g, steps_o, floor=1e-3):
    """Reduced-precision tallies against FP64 ones of the same seed: max |z|,
    the fraction within 3 sigma and the median and largest relative error
    per tally kind ([B][I][6] raw per-batch sums per step)."""
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
            top = scale[:, k].max()
            mr = scale[:, k] > floor * top if top > 0 else np.zeros(len(To), bool)
            rel[k].append(np.abs(Tg[mr, k] - To[mr, k]) / scale[mr, k])
    out = {}
    for k in range(6):
        z = np.concatenate(zs[k])
        r = np.concatenate(rel[k])
        out[KIND_NAMES[k]] = {"cell_steps": int(z.size),
                              "max_abs_z": float(np.abs(z).max()) if z.size else 0.0,
                              "frac_within_3sigma": float(np.mean(np.abs(z) <= 3.0)) if z.size else 1.0,
                              "median_rel_err": float(np.median(r)) if r.size else 0.0,
                              "max_rel_err": float(r.max()) if r.size else 0.0}
    return out


def run_methods(total, warmup, n_src, c, rho, ref):
    """The paper's comparison of weight-window methods (Sec. 5) on the
    full-scale workload: HWW without filter, with the moving average (k = 3)
    and with the Fourier filter (kappa = 30), lagged weight windows, each
    against the plain sweep: FOM ratios averaged over the timed steps and
    end-to-end segments/s."""
    from paper_2512_19925_amd import hww as H
    from paper_2512_19925_amd import workloads as W
    w0 = W.full_scale(c=c, rho=rho, n_src=n_src)
    f_a = run_fom(w0.with_(analog=True), total, warmup, analog=True, ref=ref)
    out = {}
    # Lagged windows trail the particle front; the particles that outrun
    # them split the bank past its capacity of 4e7 unless eps_min is raised
    # (eps_min = 0.05 peaks at 7e7 particles, 0.2 at 2.5e7), so LWW runs with
    # eps_min = 0.2.
    # "HWW-MA phi-only": the cheaper closure tallies of census closures, the
    # track-length phi alone per segment instead of phi, J and K.
    for name, w in (("HWW", w0.with_(filter=0)), ("HWW-MA", w0), ("HWW-MA phi-only", w0.with_(track_moments=1)),
                    ("HWW-F", w0.with_(filter=2, kappa=30)),
                    ("LWW eps_min=0.2", w0.with_(filter=0, lagged=True, eps_min=0.2))):
        rec = {}
        try:
            g = run_gpu(w, total, warmup, analog=False, timing=False)
            f_h = run_fom(w, total, warmup, analog=False, ref=ref)
        except H.HwwError as e:
            out[name] = {"error": str(e)}
            continue
        r_sig = [a[0] / b[0] for a, b in zip(f_h, f_a) if b[0] > 0]
        r_err = [a[1] / b[1] for a, b in zip(f_h, f_a) if b[1] > 0]
        rec["segments_per_s"] = g["segments"] / g["wall_s"]
        rec["fom_sigma_over_plain_mean"] = float(np.mean(r_sig)) if r_sig else None
        rec["fom_error_over_plain_mean"] = float(np.mean(r_err)) if r_err else None
        out[name] = rec
        print(json.dumps({name: rec}), file=sys.stderr, flush=True)
    return out


def run_sweep(total, warmup, n_src):
    """Every (c, rho) pair of the full-scale workload: end-to-end segments/s
    and the FOM gains of HWW over the plain sweep of the same c."""
    from paper_2512_19925_amd import hww as H
    from paper_2512_19925_amd import pulse_reference as P
    from paper_2512_19925_amd import workloads as W
    out = []
    for c in W.FULL_SCALE_C:
        w0 = W.full_scale(c=c, n_src=n_src)
        ref = P.cell_step_averages(w0.edges, w0.dt, total, c)
        ana = run_gpu(w0.with_(analog=True), total, warmup, analog=True, timing=False)
        f_a = run_fom(w0.with_(analog=True), total, warmup, analog=True, ref=ref)
        for rho in W.FULL_SCALE_RHO:
            w = W.full_scale(c=c, rho=rho, n_src=n_src)
            rec = {"c": c, "rho": rho, "plain_segments_per_s": ana["segments"] / ana["wall_s"]}
            try:
                g = run_gpu(w, total, warmup, analog=False, timing=False)
                f_h = run_fom(w, total, warmup, analog=False, ref=ref)
            except H.HwwError as e:
                rec["error"] = str(e)
                out.append(rec)
                continue
            r_sig = [a[0] / b[0] for a, b in zip(f_h, f_a) if b[0] > 0]
            r_err = [a[1] / b[1] for a, b in zip(f_h, f_a) if b[1] > 0]
            rec.update({"segments_per_s": g["segments"] / g["wall_s"],
                        "ms_per_step": g["wall_s"] * 1e3 / (total - warmup),
                        "fom_sigma_over_plain_mean": float(np.mean(r_sig)) if r_sig else None,
                        "fom_error_over_plain_mean": float(np.mean(r_err)) if r_err else None})
            out.append(rec)
            print(json.dumps(rec), file=sys.stderr, flush=True)
    return out


def run_paper_problem(seeds=5, window_scale=1, comb_by_index=True):
    """The paper's own supercritical problem (Sec. 5.1: c_eff = 1.1 with
    fission, 201 cells, 20 steps of dt = 1, 1e4 histories per step kept by
    uniform combing, rho = 1.25, eps_min = 1e-3) for the paper's methods:
    analog, HWW, HWW-MA, HWW-F and lagged windows.  Per step: tau^n is the
    wall time of the step (comb, solves, sweeps and the wait for them),
    FOM_sigma^n from the batch spread of the track flux and FOM_Error^n
    against the reference pulse solution at c = 1.1; each FOM is averaged
    over `seeds` seeds before the ratio to analog is taken."""
    import torch
    from paper_2512_19925_amd import hww as H
    from paper_2512_19925_amd import pulse_reference as P
    from paper_2512_19925_amd import workloads as W
    w0 = W.paper_fission().with_(window_scale=window_scale, comb_by_index=comb_by_index)
    ref = P.cell_step_averages(w0.edges, w0.dt, w0.n_steps, 1.1)
    dx = np.diff(w0.edges)
    methods = (("analog", w0.with_(analog=True)), ("HWW", w0.with_(filter=0)), ("HWW-MA", w0),
               ("HWW-F", w0.with_(filter=2, kappa=30)), ("LWW", w0.with_(filter=0, lagged=True)))
    res = {}
    for name, w in methods:
        sig = np.zeros((seeds, w.n_steps))
        err = np.zeros((seeds, w.n_steps))
        sig_w = np.zeros((seeds, w.n_steps))  # cost = segments of the step instead of its wall time
        err_w = np.zeros((seeds, w.n_steps))
        segs, wall, fis = 0, 0.0, 0
        try:
            for sd in range(seeds):
                ws = w.with_(seed=1 + sd)
                h = H.Handle(H.spec_from_workload(ws))
                h.set_timing(False)
                kw = H.losm_kwargs(ws)
                torch.cuda.synchronize()
                for n in range(1, ws.n_steps + 1):
                    t0 = time.perf_counter()
                    if n > 1:
                        h.comb(ws.comb, wait=False)
                    st = _step(h, ws, n, ws.analog, kw, stats=True)
                    tau = time.perf_counter() - t0
                    wall += tau
                    segs += st["segments"]
                    fis += st["fissions"]
                    cells = h.read_tallies(H.TALLY_CELLS)
                    fs = fom_sigma(cells, ws.n_src, dx, ws.dt)
                    fe = fom_error(cells, ws.n_src, dx, ws.dt, ref[n - 1])
                    sig[sd, n - 1], err[sd, n - 1] = fs / tau, fe / tau
                    sig_w[sd, n - 1], err_w[sd, n - 1] = fs / st["segments"], fe / st["segments"]
                h.close()
        except H.HwwError as e:
            res[name] = {"error": str(e)}
            continue
        res[name] = {"sig": sig.mean(0), "err": err.mean(0), "sig_w": sig_w.mean(0), "err_w": err_w.mean(0),
                     "segments_per_s": segs / wall,
                     "ms_per_step": wall * 1e3 / (seeds * w.n_steps), "fissions_per_step": fis / (seeds * w.n_steps)}
    out = {"workload": f"{w0.name}: {w0.n_cells} cells on [{w0.x_lo},{w0.x_hi}], sigma_t=1, sigma_s=sigma_f=1/3, "
                       f"nu_f={w0.nu_f} (c_eff=1.1), v=1, dt={w0.dt}, {w0.n_steps} steps, H={w0.comb} histories "
                       f"per step (uniform comb, teeth spaced in "
                       f"{'particle index' if comb_by_index else 'cumulative weight'}), rho={w0.rho}, "
                       f"eps_min={w0.eps_min}, CN, 3 window updates per "
                       f"step, window centres {'as printed (largest 1)' if window_scale else 'times s^n'}, "
                       f"{seeds} seeds",
           "fom": "per step, tau = step wall time (work_fom: tau = segments of the step); FOM averaged over "
                  "the seeds, ratio to analog averaged over the 20 steps"}
    a = res.get("analog")
    for name, r in res.items():
        if "error" in r:
            out[name] = r
            continue
        rec = {"segments_per_s": r["segments_per_s"], "ms_per_step": r["ms_per_step"],
               "fissions_per_step": r["fissions_per_step"]}
        if a is not None and "error" not in a and name != "analog":
            rec["fom_sigma_over_analog_mean"] = float(np.mean(r["sig"] / a["sig"]))
            rec["fom_error_over_analog_mean"] = float(np.mean(r["err"] / a["err"]))
            rec["fom_sigma_over_analog_steps_4_19"] = [float(r["sig"][3] / a["sig"][3]),
                                                      float(r["sig"][18] / a["sig"][18])]
            # With the cost of a step taken as its segments (a serial code's
            # runtime), not the GPU wall time that launch latency dominates at
            # 1e4 histories.
            rec["work_fom_sigma_over_analog_mean"] = float(np.mean(r["sig_w"] / a["sig_w"]))
            rec["work_fom_error_over_analog_mean"] = float(np.mean(r["err_w"] / a["err_w"]))
        out[name] = rec
    return out


def _oracle_replica(args):
    """One process of the aggregate CPU figure: the bounded oracle sample of
    cpu_baseline with its own replica key."""
    w, n, k, budget_s = args
    from oracle import oracle as O
    ws = w.with_(n_src=n, bank_capacity=4 * n + 4096, replica=k)
    sim = O.OracleSim(ws.edges, ws.sigma_t, ws.sigma_s, ws.speed, ws.dt, ws.n_steps, ws.src_x, ws.n_src,
                      ws.capacity(), ws.seed, ws.replica, ws.n_batches, ws.n_chunks)
    opts = O.LosmOpts(theta=ws.theta, filter=ws.filter, ma_k=ws.ma_k, eps_min=ws.eps_min, rho=ws.rho)
    seg, t0 = 0, time.perf_counter()
    for step in range(1, ws.n_steps + 1):
        sim.solve_losm(opts, implicit=False)
        for p in range(ws.n_chunks):
            sim.sweep(step, p)
            if p < ws.n_chunks - 1:
                sim.solve_losm(opts, implicit=True)
        seg += sim.counters()["segments"]
        if time.perf_counter() - t0 > budget_s:
            break
    return seg, time.perf_counter() - t0


# CPU cores a one-GPU run may use on its host (whatever the host shows).
HOST_CORES_PER_GPU = 16


def cpu_aggregate(w, budget_s, procs=None):
    """The oracle in P independent processes at once, each the bounded
    sample of cpu_baseline under its own replica key, P = the host's CPU
    count, at most the 16 cores a one-GPU run may use: summed segments/s."""
    import multiprocessing as mp
    P = procs or min(os.cpu_count() or 1, HOST_CORES_PER_GPU)
    n = max(w.n_src // 4, 1000)
    with mp.get_context("spawn").Pool(P) as pool:
        res = pool.map(_oracle_replica, [(w, n, k, budget_s) for k in range(P)])
    return {"value": sum(s / t for s, t in res), "unit": "segments/s", "processes": P,
            "cores": P, "host": host_cpu(),
            "sample": f"{P} processes at once (the host's CPU count, at most the {HOST_CORES_PER_GPU} cores "
                      f"of a one-GPU share), each the single-core sample under replica key k = 0..{P - 1}, "
                      f"about {budget_s:.0f} s each"}


def cpu_baseline(w, budget_s):
    """The oracle, as it stands, on a bounded sample: the same problem with
    fewer source particles, as many steps as fit in about budget_s."""
    from oracle import oracle as O
    frac = 4
    n = max(w.n_src // frac, 1000)
    ws = w.with_(n_src=n, bank_capacity=4 * n + 4096)
    sim = O.OracleSim(ws.edges, ws.sigma_t, ws.sigma_s, ws.speed, ws.dt, ws.n_steps, ws.src_x, ws.n_src,
                      ws.capacity(), ws.seed, ws.replica, ws.n_batches, ws.n_chunks)
    opts = O.LosmOpts(theta=ws.theta, filter=ws.filter, ma_k=ws.ma_k, eps_min=ws.eps_min, rho=ws.rho)
    seg = 0
    t0 = time.perf_counter()
    steps = 0
    for step in range(1, ws.n_steps + 1):
        sim.solve_losm(opts, implicit=False)
        for p in range(ws.n_chunks):
            sim.sweep(step, p)
            if p < ws.n_chunks - 1:
                sim.solve_losm(opts, implicit=True)
        seg += sim.counters()["segments"]
        steps = step
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": seg / dt, "unit": "segments/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
            "sample": f"{ws.name} with {n} source particles (1/{frac} of the workload), steps 1-{steps}, "
                      f"{seg} segments in {dt:.1f} s, serial FP64 C oracle"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2512_19925_amd import workloads as W

    if args.calibrate_copy:
        # A plain copy of known size: 1 GiB read + 1 GiB written per dispatch.
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": src.numel() * 8, "bytes_written": dst.numel() * 8}))
        return

    w = W.full_scale(c=args.c, rho=args.rho, n_src=args.n_src)
    total = args.warmup + args.steps
    if total > w.n_steps:
        print(f"warmup + steps must be <= {w.n_steps} time steps of the workload", file=sys.stderr)
        sys.exit(2)
    torch.cuda.init()
    # Throughput pass: no timing events between the launches; one warm-up
    # run, then the median of REPEATS runs (each W untimed steps and K timed
    # ones on a fresh problem).
    run_gpu(w, total, args.warmup, analog=False, timing=False)
    runs = sorted((run_gpu(w, total, args.warmup, analog=False, timing=False) for _ in range(REPEATS)),
                  key=lambda d: d["segments"] / d["wall_s"])
    hww = runs[REPEATS // 2]
    value = hww["segments"] / hww["wall_s"]
    ms_per_step = hww["wall_s"] * 1e3 / args.steps
    # Roofline pass: the same steps with HIP events around every sweep launch
    # on the library's stream; the median run by average launch time.
    tims = sorted((run_gpu(w, total, args.warmup, analog=False, timing=True) for _ in range(REPEATS)),
                  key=lambda d: d["kernel_ms"] / max(d["launches"], 1))
    tim = tims[REPEATS // 2]
    achieved = tim["bytes_moved"] / (tim["kernel_ms"] * 1e-3) / 1e9 if tim["kernel_ms"] > 0 else 0.0
    bytes_per_launch = tim["bytes_moved"] / max(tim["launches"], 1)
    avg_launch_s = tim["kernel_ms"] * 1e-3 / max(tim["launches"], 1)
    dev = device_check()
    traf = profile_figures(TRAFFIC_PROFILE, ["traffic_over_algorithmic"])
    valu = profile_figures(VALU_PROFILE, ["valu_issue_frac", "active_lanes_per_valu", "valu_insts_per_launch"])
    line = {
        "metric": METRIC, "value": value, "unit": "segments/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w.name}: 1D slab, {w.n_cells} cells on [{w.x_lo},{w.x_hi}], sigma_t=1, "
                               f"c={args.c}, v=1, isotropic unit pulse at x=0, {w.n_src:.0e} source "
                               f"particles, dt={w.dt}, steps {args.warmup + 1}-{total} of {w.n_steps}, "
                               f"HWW rho={w.rho} eps_min={w.eps_min}, MA k={w.ma_k} filtered closures, "
                               f"{w.n_chunks - 1} window updates per step",
                   "n_src": w.n_src, "n_cells": w.n_cells, "time_steps": args.steps},
        "kernel_segments_per_s": tim["segments"] / (tim["kernel_ms"] * 1e-3) if tim["kernel_ms"] else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     # Beside the published peak: the measured bandwidth of a
                     # plain device copy on this GPU.
                     "measured_copy_GBs": dev["copy_GBs"], "frac_of_copy": achieved / dev["copy_GBs"],
                     "traffic": traf["traffic_over_algorithmic"] * bytes_per_launch if traf else None,
                     "traffic_over_algorithmic": traf["traffic_over_algorithmic"] if traf else None,
                     "kernel": "sweep_kernel<double, true, false>",
                     "launches": tim["launches"], "avg_launch_ms": avg_launch_s * 1e3,
                     "bytes_per_launch": bytes_per_launch,
                     "runs": REPEATS, "avg_launch_ms_runs": [d["kernel_ms"] / max(d["launches"], 1) for d in tims],
                     # VALU side: wave-instruction issue cycles (4 per wave64
                     # instruction) over the 1024 SIMDs' cycles of the launch,
                     # and active lanes per VALU instruction, from committed
                     # counters of the same command.
                     "valu": ({"issue_frac": valu["valu_issue_frac"],
                               "active_lanes_per_instruction": valu["active_lanes_per_valu"],
                               "lane_frac": valu["active_lanes_per_valu"] / 64.0,
                               "source": os.path.relpath(VALU_PROFILE, ROOT)} if valu else None)},
        "value_runs": [d["segments"] / d["wall_s"] for d in runs],
        "device": dev,
    }
    if not args.no_analog:
        from paper_2512_19925_amd import pulse_reference as P
        ana = run_gpu(w.with_(analog=True), total, args.warmup, analog=True, timing=False)
        ref = P.cell_step_averages(w.edges, w.dt, total, args.c)
        f_h = run_fom(w, total, args.warmup, analog=False, ref=ref)
        f_a = run_fom(w.with_(analog=True), total, args.warmup, analog=True, ref=ref)
        r_sig = [a[0] / b[0] for a, b in zip(f_h, f_a) if b[0] > 0]
        r_err = [a[1] / b[1] for a, b in zip(f_h, f_a) if b[1] > 0]
        line["fom"] = {"kind": "per time step, tau = step wall time; FOM_sigma from the batch spread of the "
                               "track-length flux, FOM_Error against the closed-form pulse solution",
                       "sigma_hww_over_plain_mean": float(np.mean(r_sig)) if r_sig else None,
                       "sigma_hww_over_plain_first_last": [r_sig[0], r_sig[-1]] if r_sig else None,
                       "error_hww_over_plain_mean": float(np.mean(r_err)) if r_err else None,
                       "error_hww_over_plain_first_last": [r_err[0], r_err[-1]] if r_err else None,
                       "plain_segments_per_s": ana["segments"] / ana["wall_s"],
                       "plain_ms_per_step": ana["wall_s"] * 1e3 / args.steps}
        if total < w.n_steps:
            # The windows matter more as the pulse spreads: the same ratios
            # over every step of the run after the warm-up (not timed above).
            ref_all = P.cell_step_averages(w.edges, w.dt, w.n_steps, args.c)
            fa_h = run_fom(w, w.n_steps, args.warmup, analog=False, ref=ref_all)
            fa_a = run_fom(w.with_(analog=True), w.n_steps, args.warmup, analog=True, ref=ref_all)
            ra_sig = [a[0] / b[0] for a, b in zip(fa_h, fa_a) if b[0] > 0]
            ra_err = [a[1] / b[1] for a, b in zip(fa_h, fa_a) if b[1] > 0]
            line["fom"]["whole_run"] = {
                "steps": f"{args.warmup + 1}-{w.n_steps}",
                "sigma_hww_over_plain_mean": float(np.mean(ra_sig)) if ra_sig else None,
                "error_hww_over_plain_mean": float(np.mean(ra_err)) if ra_err else None,
                "sigma_hww_over_plain_first_last": [ra_sig[0], ra_sig[-1]] if ra_sig else None,
                "error_hww_over_plain_first_last": [ra_err[0], ra_err[-1]] if ra_err else None}
        line["methods"] = run_methods(total, args.warmup, args.n_src, args.c, args.rho, ref)
    if args.sweep:
        line["sweep"] = run_sweep(total, args.warmup, args.n_src)
    if not args.no_batch:
        line["batched"] = run_batched(args.batch_steps, args.batch_compare_steps)
    if not args.no_fp32:
        line["fp32"] = run_fp32_pair()
    if not args.no_paper:
        line["paper_problem"] = {"windows_times_s": run_paper_problem(window_scale=0),
                                 "windows_as_printed": run_paper_problem(window_scale=1),
                                 "comb_by_weight": run_paper_problem(window_scale=0, comb_by_index=False)}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        line["cpu_baseline"]["aggregate"] = cpu_aggregate(w, args.cpu_seconds)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"hww": hww, "timed": tim, "line": line}, f, default=float)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
