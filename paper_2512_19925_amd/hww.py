"""Thin ctypes binding of libhww.so (include/hww.h).

Argument marshalling only: every step of the sweep and of the LOSM solve
runs in the HIP kernels of the library.  PyTorch supplies the device
workspace (one uint8 tensor) and the stream.  The binding fails loudly when
the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhww.so")

HWW_OK = 0
ERRORS = {-1: "HWW_E_INVALID_ARG", -2: "HWW_E_STATE", -3: "HWW_E_CAPACITY", -4: "HWW_E_DEVICE",
          -5: "HWW_E_NUMERIC"}
HWW_FP64, HWW_FP32 = 0, 1
TALLY_CELLS, TALLY_BOUNDARY, TALLY_TRACKS, TALLY_PREV_CELLS, TALLY_PREV_BOUNDARY, TALLY_WINDOWS, \
    TALLY_BANK_COUNTS = range(7)

# Every symbol include/hww.h declares.
EXPORTS = ["hww_workspace_bytes", "hww_init_problem", "hww_init_problem_static", "hww_set_windows", "hww_sweep_step",
           "hww_read_run_stats", "hww_comb", "hww_solve_losm", "hww_read_closures", "hww_losm_march", "hww_losm_adjoint",
           "hww_read_tallies", "hww_read_bank", "hww_batch_workspace_bytes", "hww_init_batch",
           "hww_batch_replica", "hww_autotune", "hww_set_timing", "hww_sync", "hww_last_error", "hww_destroy"]


class HwwError(RuntimeError):
    def __init__(self, where, code, text=""):
        super().__init__(f"{where}: {ERRORS.get(code, code)} {text}".strip())
        self.code = code


class Problem(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("edges", C.POINTER(C.c_double)),
                ("sigma_t", C.POINTER(C.c_double)), ("sigma_s", C.POINTER(C.c_double)),
                ("speed", C.c_double), ("dt", C.c_double), ("n_steps", C.c_int32),
                ("src_x", C.c_double), ("n_src", C.c_int64), ("bank_capacity", C.c_int64),
                ("seed", C.c_uint32), ("replica", C.c_uint32), ("n_batches", C.c_int32),
                ("precision", C.c_int32), ("n_chunks", C.c_int32), ("sigma_f", C.POINTER(C.c_double)),
                ("nu_f", C.c_double), ("comb", C.c_int32), ("track_moments", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("segments", "collisions", "scatters", "absorptions",
                                          "crossings", "leaks", "census", "splits", "daughters",
                                          "rr_kill", "rr_survive", "histories", "generations",
                                          "launches")] + \
               [("kernel_ms", C.c_double), ("bytes_moved", C.c_uint64), ("fissions", C.c_uint64),
                ("fission_births", C.c_uint64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class LosmOpts(C.Structure):
    _fields_ = [("theta", C.c_double), ("implicit", C.c_int32), ("filter", C.c_int32),
                ("ma_k", C.c_int32), ("eps_min", C.c_double), ("rho", C.c_double),
                ("closure_track", C.c_int32), ("apply_windows", C.c_int32), ("kappa", C.c_int32),
                ("lagged", C.c_int32), ("window_scale", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("block", C.c_int32), ("tile", C.c_int32), ("grid", C.c_int32), ("trials", C.c_int32),
                ("ms", C.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib():
    """Load libhww.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(python -m paper_2512_19925_amd.build) first")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.hww_workspace_bytes.argtypes = [C.POINTER(Problem)]
        L.hww_workspace_bytes.restype = C.c_int64
        L.hww_init_problem.argtypes = [C.POINTER(Problem), vp, C.c_int64, vp, C.POINTER(vp)]
        L.hww_init_problem_static.argtypes = [C.POINTER(Problem), vp, C.POINTER(vp)]
        L.hww_set_windows.argtypes = [vp, dp, C.c_double]
        L.hww_sweep_step.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(StepStats)]
        L.hww_read_run_stats.argtypes = [vp, C.POINTER(StepStats)]
        L.hww_comb.argtypes = [vp, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.hww_solve_losm.argtypes = [vp, C.POINTER(LosmOpts), dp, dp]
        L.hww_read_tallies.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_int64]
        L.hww_read_closures.argtypes = [vp, dp, dp, dp, dp]
        L.hww_losm_march.argtypes = [vp, dp, dp, C.c_double, C.c_int32] + [dp] * 8
        L.hww_losm_adjoint.argtypes = [vp, dp, dp, dp]
        L.hww_read_bank.argtypes = [vp, C.c_int32, C.c_int64, C.POINTER(C.c_int64)] + [vp] * 8
        L.hww_batch_workspace_bytes.argtypes = [C.POINTER(Problem), C.c_int32]
        L.hww_batch_workspace_bytes.restype = C.c_int64
        L.hww_init_batch.argtypes = [C.POINTER(Problem), C.c_int32, vp, C.c_int64, vp, C.POINTER(vp)]
        L.hww_batch_replica.argtypes = [vp, C.c_int32, C.POINTER(vp)]
        L.hww_autotune.argtypes = [vp, C.POINTER(TuneResult)]
        L.hww_set_timing.argtypes = [vp, C.c_int32]
        L.hww_sync.argtypes = [vp]
        L.hww_last_error.argtypes = [vp]
        L.hww_last_error.restype = C.c_char_p
        L.hww_destroy.argtypes = [vp]
        L.hww_destroy.restype = None
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class ProblemSpec:
    edges: np.ndarray
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    speed: float
    dt: float
    n_steps: int
    src_x: float
    n_src: int
    bank_capacity: int
    seed: int = 1
    replica: int = 0
    n_batches: int = 32
    precision: int = HWW_FP64
    n_chunks: int = 4
    sigma_f: np.ndarray | None = None
    nu_f: float = 0.0
    comb: int = 0
    track_moments: int = 0

    def to_c(self):
        self._keep = [_f64(self.edges), _f64(self.sigma_t), _f64(self.sigma_s),
                      None if self.sigma_f is None else _f64(self.sigma_f)]
        e, st, ss, sf = self._keep
        return Problem(len(st), _dp(e), _dp(st), _dp(ss), float(self.speed), float(self.dt),
                       int(self.n_steps), float(self.src_x), int(self.n_src), int(self.bank_capacity),
                       int(self.seed), int(self.replica), int(self.n_batches), int(self.precision),
                       int(self.n_chunks), _dp(sf), float(self.nu_f), int(self.comb), int(self.track_moments))


def workspace_bytes(spec: ProblemSpec) -> int:
    p = spec.to_c()
    n = lib().hww_workspace_bytes(C.byref(p))
    if n < 0:
        raise HwwError("hww_workspace_bytes", n)
    return int(n)


class Handle:
    """One problem on the GPU.  Owns its torch workspace tensor."""

    @classmethod
    def _view(cls, ptr, spec, owner):
        """Read-only view of one replica of a Batch (owned by the batch)."""
        v = cls.__new__(cls)
        v.spec = spec
        v.I = len(spec.sigma_t)
        v.B = int(spec.n_batches)
        v.n_chunks = int(spec.n_chunks)
        v._h = ptr
        v._owner = owner
        return v

    def __init__(self, spec: ProblemSpec, device="cuda", stream=None, static_workspace=False):
        """static_workspace=True: hww_init_problem_static (the library's
        fixed per-GPU workspace; no device allocation here or there)."""
        import torch
        self.spec = spec
        self.I = len(spec.sigma_t)
        self.B = int(spec.n_batches)
        self.n_chunks = int(spec.n_chunks)
        nbytes = workspace_bytes(spec)
        p = spec.to_c()
        h = C.c_void_p()
        if static_workspace:
            dev = torch.device(device)
            dev = torch.device("cuda", torch.cuda.current_device() if dev.index is None else dev.index)
            self.workspace = None
            self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
            with torch.cuda.device(dev):
                rc = lib().hww_init_problem_static(C.byref(p), C.c_void_p(self.stream.cuda_stream), C.byref(h))
            if rc != HWW_OK:
                raise HwwError("hww_init_problem_static", rc, lib().hww_last_error(None).decode())
            self._h = h
            return
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        rc = lib().hww_init_problem(C.byref(p), C.c_void_p(self.workspace.data_ptr()), nbytes,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != HWW_OK:
            raise HwwError("hww_init_problem", rc, lib().hww_last_error(None).decode())
        self._h = h

    # -- helpers ------------------------------------------------------------
    def _check(self, where, rc):
        if rc != HWW_OK:
            raise HwwError(where, rc, lib().hww_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self._h = None  # a view: the batch owns it
            return
        if getattr(self, "_h", None):
            lib().hww_destroy(self._h)
            self._h = None

    def set_timing(self, on=True):
        """HIP-event timing of every sweep launch (on by default)."""
        self._check("hww_set_timing", lib().hww_set_timing(self._h, int(bool(on))))

    def autotune(self):
        """Pick the fastest sweep launch shape (before the first sweep)."""
        r = TuneResult()
        self._check("hww_autotune", lib().hww_autotune(self._h, C.byref(r)))
        return r.as_dict()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points -------------------------------------------------------
    def set_windows(self, centre, rho):
        if centre is None:
            self._check("hww_set_windows", lib().hww_set_windows(self._h, None, float(rho)))
            return
        c = _f64(centre)
        assert c.shape == (self.I,)
        self._check("hww_set_windows", lib().hww_set_windows(self._h, _dp(c), float(rho)))

    def sweep_step(self, step, chunk, stats=True):
        st = StepStats() if stats else None
        self._check("hww_sweep_step", lib().hww_sweep_step(self._h, int(step), int(chunk),
                                                           C.byref(st) if st is not None else None))
        return st.as_dict() if st is not None else None

    def run_stats(self):
        st = StepStats()
        self._check("hww_read_run_stats", lib().hww_read_run_stats(self._h, C.byref(st)))
        return st.as_dict()

    def comb(self, n_target, wait=True):
        """Uniform comb of the finished step's census into n_target particles;
        returns (census size before, total weight).  With wait=False the
        call only queues the comb (no output, nothing returned; errors show
        at the next call that synchronises)."""
        if not wait:
            self._check("hww_comb", lib().hww_comb(self._h, int(n_target), None, None))
            return None
        nb, wt = C.c_int64(), C.c_double()
        self._check("hww_comb", lib().hww_comb(self._h, int(n_target), C.byref(nb), C.byref(wt)))
        return int(nb.value), float(wt.value)

    def solve_losm(self, theta=0.5, implicit=False, filter=0, ma_k=3, eps_min=1e-3, rho=5.0,
                   closure_track=0, apply_windows=True, want_solution=False, kappa=30, lagged=0,
                   window_scale=0):
        o = LosmOpts(float(theta), int(implicit), int(filter), int(ma_k), float(eps_min), float(rho),
                     int(closure_track), int(apply_windows), int(kappa), int(lagged), int(window_scale))
        phi = np.zeros(self.I + 2) if want_solution else None
        J = np.zeros(self.I + 1) if want_solution else None
        self._check("hww_solve_losm", lib().hww_solve_losm(self._h, C.byref(o), _dp(phi), _dp(J)))
        return (phi, J) if want_solution else None

    def read_tallies(self, kind=TALLY_CELLS, raw=True):
        """Per-batch tally array; raw=False normalises it per source particle."""
        I, B = self.I, self.B
        shapes = {TALLY_CELLS: ((B, I, 6), np.float64), TALLY_BOUNDARY: ((B, 2, 3), np.float64),
                  TALLY_TRACKS: ((I,), np.uint64), TALLY_PREV_CELLS: ((B, I, 6), np.float64),
                  TALLY_PREV_BOUNDARY: ((B, 2, 3), np.float64), TALLY_WINDOWS: ((3, I), np.float64),
                  TALLY_BANK_COUNTS: ((2,), np.uint64)}
        shape, dt = shapes[kind]
        out = np.zeros(shape, dtype=dt)
        self._check("hww_read_tallies", lib().hww_read_tallies(self._h, int(kind), int(bool(raw)), out.ctypes.data,
                                                               out.nbytes))
        return out

    def read_bank(self, which):
        cnt = C.c_int64()
        n = max(int(self.read_tallies(TALLY_BANK_COUNTS)[which]), 1)
        out = {"x": np.zeros(n), "mu": np.zeros(n), "w": np.zeros(n), "src": np.zeros(n, np.uint32),
               "lin": np.zeros(n, np.uint64), "e": np.zeros(n, np.uint32), "cell": np.zeros(n, np.int32),
               "chunk": np.zeros(n, np.int32)}
        self._check("hww_read_bank", lib().hww_read_bank(
            self._h, int(which), n, C.byref(cnt),
            *[out[k].ctypes.data for k in ("x", "mu", "w", "src", "lin", "e", "cell", "chunk")]))
        m = int(cnt.value)
        return {k: v[:m] for k, v in out.items()}

    def read_closures(self):
        """(F, P, phi, J) that the finished step hands to the next."""
        F, P = np.zeros(self.I + 2), np.zeros(2)
        phi, J = np.zeros(self.I + 2), np.zeros(self.I + 1)
        self._check("hww_read_closures", lib().hww_read_closures(self._h, _dp(F), _dp(P), _dp(phi), _dp(J)))
        return F, P, phi, J

    def losm_march(self, sigma_t, sigma_s, theta, F, P, phi0, J0, weights, histories=False):
        st, ss, F, P, phi0, J0, w = map(_f64, (sigma_t, sigma_s, F, P, phi0, J0, weights))
        N = F.shape[0] - 1
        assert st.shape == (self.I,) and ss.shape == (self.I,) and F.shape == (N + 1, self.I + 2)
        assert P.shape == (N + 1, 2) and w.shape == F.shape
        ph = np.zeros((N + 1, self.I + 2)) if histories else None
        jh = np.zeros((N + 1, self.I + 1)) if histories else None
        G = C.c_double()
        self._check("hww_losm_march", lib().hww_losm_march(
            self._h, _dp(st), _dp(ss), float(theta), N, _dp(F), _dp(P), _dp(phi0), _dp(J0), _dp(w),
            _dp(ph), _dp(jh), C.byref(G)))
        return (G.value, ph, jh) if histories else G.value

    def losm_adjoint(self, dG_dphi=None):
        """Gradient of the last march's G (or of the functional whose
        derivative with respect to the flux history is dG_dphi)."""
        gt, gs = np.zeros(self.I), np.zeros(self.I)
        d = None if dG_dphi is None else _f64(dG_dphi)
        self._check("hww_losm_adjoint", lib().hww_losm_adjoint(self._h, _dp(d), _dp(gt), _dp(gs)))
        return gt, gs

    def sync(self):
        self._check("hww_sync", lib().hww_sync(self._h))


class Batch:
    """Many replicas of uneven size in one handle: one persistent sweep launch
    per chunk and one batched LOSM launch per solve for all of them."""

    def __init__(self, specs, device="cuda", stream=None):
        import torch
        self.specs = list(specs)
        self.n = len(self.specs)
        self.I = [len(s.sigma_t) for s in self.specs]
        self.B = [int(s.n_batches) for s in self.specs]
        self.n_chunks = int(self.specs[0].n_chunks)
        self._probs = (Problem * self.n)(*[s.to_c() for s in self.specs])
        nbytes = lib().hww_batch_workspace_bytes(self._probs, self.n)
        if nbytes < 0:
            raise HwwError("hww_batch_workspace_bytes", nbytes)
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        h = C.c_void_p()
        rc = lib().hww_init_batch(self._probs, self.n, C.c_void_p(self.workspace.data_ptr()), int(nbytes),
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != HWW_OK:
            raise HwwError("hww_init_batch", rc, lib().hww_last_error(None).decode())
        self._h = h
        self._views = {}

    def _check(self, where, rc):
        if rc != HWW_OK:
            raise HwwError(where, rc, lib().hww_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            for v in self._views.values():
                v._h = None
            lib().hww_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def replica(self, r) -> Handle:
        """Read-only Handle of replica r (tallies, bank, closures)."""
        if r not in self._views:
            v = C.c_void_p()
            self._check("hww_batch_replica", lib().hww_batch_replica(self._h, int(r), C.byref(v)))
            self._views[r] = Handle._view(v, self.specs[r], self)
        return self._views[r]

    def set_windows(self, centres, rho):
        if centres is None:
            self._check("hww_set_windows", lib().hww_set_windows(self._h, None, float(rho)))
            return
        c = _f64(np.concatenate([np.asarray(x, dtype=np.float64) for x in centres]))
        assert c.shape == (sum(self.I),)
        self._check("hww_set_windows", lib().hww_set_windows(self._h, _dp(c), float(rho)))

    def sweep_step(self, step, chunk, stats=True):
        st = StepStats() if stats else None
        self._check("hww_sweep_step", lib().hww_sweep_step(self._h, int(step), int(chunk),
                                                           C.byref(st) if st is not None else None))
        return st.as_dict() if st is not None else None

    def run_stats(self):
        st = StepStats()
        self._check("hww_read_run_stats", lib().hww_read_run_stats(self._h, C.byref(st)))
        return st.as_dict()

    def solve_losm(self, theta=0.5, implicit=False, filter=0, ma_k=3, eps_min=1e-3, rho=5.0,
                   closure_track=0, apply_windows=True, want_solution=False, kappa=30, lagged=0,
                   window_scale=0):
        o = LosmOpts(float(theta), int(implicit), int(filter), int(ma_k), float(eps_min), float(rho),
                     int(closure_track), int(apply_windows), int(kappa), int(lagged), int(window_scale))
        phi = np.zeros(sum(i + 2 for i in self.I)) if want_solution else None
        J = np.zeros(sum(i + 1 for i in self.I)) if want_solution else None
        self._check("hww_solve_losm", lib().hww_solve_losm(self._h, C.byref(o), _dp(phi), _dp(J)))
        if not want_solution:
            return None
        ps = np.split(phi, np.cumsum([i + 2 for i in self.I])[:-1])
        js = np.split(J, np.cumsum([i + 1 for i in self.I])[:-1])
        return ps, js

    def read_tallies(self, kind=TALLY_CELLS, raw=True):
        """List of per-replica arrays (same shapes as Handle.read_tallies)."""
        def shape(I, B):
            return {TALLY_CELLS: ((B, I, 6), np.float64), TALLY_BOUNDARY: ((B, 2, 3), np.float64),
                    TALLY_TRACKS: ((I,), np.uint64), TALLY_PREV_CELLS: ((B, I, 6), np.float64),
                    TALLY_PREV_BOUNDARY: ((B, 2, 3), np.float64), TALLY_WINDOWS: ((3, I), np.float64),
                    TALLY_BANK_COUNTS: ((2,), np.uint64)}[kind]
        shapes = [shape(I, B) for I, B in zip(self.I, self.B)]
        sizes = [int(np.prod(sh)) * 8 for sh, _ in shapes]
        buf = np.zeros(sum(sizes), dtype=np.uint8)
        self._check("hww_read_tallies", lib().hww_read_tallies(self._h, int(kind), int(bool(raw)), buf.ctypes.data,
                                                               buf.nbytes))
        out, o = [], 0
        for (sh, dt), sz in zip(shapes, sizes):
            out.append(buf[o:o + sz].view(dt).reshape(sh).copy())
            o += sz
        return out

    def set_timing(self, on=True):
        """HIP-event timing of every sweep launch (on by default)."""
        self._check("hww_set_timing", lib().hww_set_timing(self._h, int(bool(on))))

    def autotune(self):
        """Pick the fastest persistent launch shape (before the first sweep)."""
        r = TuneResult()
        self._check("hww_autotune", lib().hww_autotune(self._h, C.byref(r)))
        return r.as_dict()

    def sync(self):
        self._check("hww_sync", lib().hww_sync(self._h))


def spec_from_workload(w, precision=HWW_FP64) -> ProblemSpec:
    """ProblemSpec of a paper_2512_19925_amd.workloads.Workload."""
    return ProblemSpec(edges=w.edges, sigma_t=w.sigma_t, sigma_s=w.sigma_s, speed=w.speed, dt=w.dt,
                       n_steps=w.n_steps, src_x=w.src_x, n_src=w.n_src, bank_capacity=w.capacity(),
                       seed=w.seed, replica=w.replica, n_batches=w.n_batches, precision=precision,
                       n_chunks=w.n_chunks, sigma_f=w.sigma_f, nu_f=w.nu_f,
                       comb=(2 if w.comb_by_index else 1) if w.comb > 0 else 0,
                       track_moments=w.track_moments)


def losm_kwargs(w):
    """solve_losm keywords of a Workload."""
    return dict(theta=w.theta, filter=w.filter, ma_k=w.ma_k, eps_min=w.eps_min, rho=w.rho,
                closure_track=w.closure_track, kappa=w.kappa, lagged=int(w.lagged),
                window_scale=int(w.window_scale))


def run(h: Handle, w, steps=None, on_step=None, analog=None, stats=True):
    """Time loop of the method (Sec. 3): semi-implicit solve at the start of
    each step, then the chunks of histories with a fully implicit solve after
    each chunk but the last; with w.comb, every census but the last is
    combed to that many particles first.  Calls only the C ABI."""
    analog = w.analog if analog is None else analog
    steps = w.n_steps if steps is None else steps
    kw = losm_kwargs(w)
    for n in range(1, steps + 1):
        if w.comb and n > 1:
            h.comb(w.comb, wait=False)
        if not analog:
            h.solve_losm(implicit=False, **kw)
        chunk_stats = []
        for p in range(h.n_chunks):
            chunk_stats.append(h.sweep_step(n, p, stats=stats))
            if not analog and not w.lagged and p < h.n_chunks - 1:
                h.solve_losm(implicit=True, **kw)
        if on_step is not None:
            on_step(n, h, chunk_stats)
