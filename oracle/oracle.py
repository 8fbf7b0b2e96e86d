"""TEST INFRASTRUCTURE ONLY: Python access to the FP64 CPU oracle.

The oracle (``hww_oracle.c``) is a plain serial implementation of the hybrid
weight-window Monte Carlo method (Shaw & Anistratov, arXiv 2512.19925,
Secs. 2-4).  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this module.  It never imports the GPU package;
callers pass plain problem parameters in.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hww_oracle.c")
_LIB = os.path.join(_HERE, "liborc_hww.so")

T_PHI, T_J, T_K, C_PHI, C_J, C_K = range(6)
COUNTER_NAMES = ["segments", "collisions", "scatters", "absorptions", "crossings", "leaks",
                 "census", "splits", "daughters", "rr_kill", "rr_survive", "histories", "fissions",
                 "fission_births"]
N_COUNTERS = 16


def build() -> str:
    """Compile the oracle with gcc (no FMA contraction, plain -O2)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
           "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None
# A copy of the oracle built elsewhere (tests that plant a mistake in the
# oracle's source load their mutated build through this variable).
_LIB_OVERRIDE = os.environ.get("HWW_ORACLE_LIB")


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u53.restype = C.c_double
        L.orc_log.argtypes = [C.c_double]
        L.orc_log.restype = C.c_double
        L.orc_create.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_batch_mask.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_set_windows.argtypes = [C.c_void_p, dp, C.c_double]
        L.orc_sweep_chunk.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.orc_comb.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.orc_set_comb_mode.argtypes = [C.c_void_p, C.c_int32]
        L.orc_solve_losm.argtypes = [C.c_void_p, C.c_void_p, dp, dp]
        L.orc_get_closures.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_losm_inputs.argtypes = [C.c_void_p, C.c_int32, C.c_int32, dp, dp, dp, dp, dp]
        L.orc_get_tallies.argtypes = [C.c_void_p, C.c_int32, dp, dp]
        L.orc_get_counters.argtypes = [C.c_void_p, C.POINTER(C.c_uint64)]
        L.orc_get_tracks.argtypes = [C.c_void_p, C.POINTER(C.c_uint64)]
        L.orc_get_windows.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_get_state.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp, dp]
        L.orc_bank_size.argtypes = [C.c_void_p, C.c_int32]
        L.orc_bank_size.restype = C.c_int64
        L.orc_get_bank.argtypes = [C.c_void_p, C.c_int32] + [C.c_void_p] * 8
        L.orc_losm_step.argtypes = ([C.c_int32, dp, dp, dp, C.c_double, C.c_double, C.c_double]
                                    + [dp] * 4 + [C.c_double] * 4 + [dp] * 4)
        L.orc_thomas.argtypes = [C.c_int32, dp, dp, dp, dp, dp]
        L.orc_losm_march.argtypes = ([C.c_int32, dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_int32]
                                     + [dp] * 6)
        L.orc_losm_adjoint.argtypes = ([C.c_int32, dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_int32]
                                       + [dp] * 5)
        L.orc_ma_filter.argtypes = [dp, C.c_int32, C.c_int32, dp]
        L.orc_fourier_filter.argtypes = [dp, C.c_int32, C.c_int32, dp]
        L.orc_ww_centres.argtypes = [C.c_int32, dp, C.c_double, C.c_double, dp]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, where, rc):
        super().__init__(f"oracle {where} failed with code {rc}")
        self.rc = rc


def _check(where, rc):
    if rc != 0:
        raise OracleError(where, rc)


# --------------------------------------------------------------------------
# Stand-alone pieces
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u53(a, b):
    return lib().orc_u53(int(a) & 0xFFFFFFFF, int(b) & 0xFFFFFFFF)


def log(x):
    """ln x by the oracle's fixed steps (the flight distance's logarithm)."""
    return lib().orc_log(float(x))


def thomas(a, b, c, d):
    a, b, c, d = map(_f64, (a, b, c, d))
    x = np.zeros_like(d)
    _check("thomas", lib().orc_thomas(len(d), _dp(a), _dp(b), _dp(c), _dp(d), _dp(x)))
    return x


def ma_filter(chi, k):
    chi = _f64(chi)
    out = np.zeros_like(chi)
    lib().orc_ma_filter(_dp(chi), len(chi), int(k), _dp(out))
    return out


def fourier_filter(chi, kappa):
    chi = _f64(chi)
    out = np.zeros_like(chi)
    lib().orc_fourier_filter(_dp(chi), len(chi), int(kappa), _dp(out))
    return out


def ww_centres(phi, eps_min, scale=1.0):
    phi = _f64(phi)
    out = np.zeros_like(phi)
    _check("ww_centres", lib().orc_ww_centres(len(phi), _dp(phi), float(eps_min), float(scale), _dp(out)))
    return out


def losm_step(edges, sig_t, sig_s, speed, dt, theta, phi_old, J_old, F_old, F_new,
              PL=0.0, PR=0.0, JL=0.0, JR=0.0, q_old=None, q_new=None):
    edges, sig_t, sig_s = map(_f64, (edges, sig_t, sig_s))
    I = len(sig_t)
    phi_old, J_old, F_old, F_new = map(_f64, (phi_old, J_old, F_old, F_new))
    assert phi_old.shape == (I + 2,) and J_old.shape == (I + 1,)
    assert F_old.shape == (I + 2,) and F_new.shape == (I + 2,)
    q_old = None if q_old is None else _f64(q_old)
    q_new = None if q_new is None else _f64(q_new)
    phi = np.zeros(I + 2)
    J = np.zeros(I + 1)
    _check("losm_step", lib().orc_losm_step(
        I, _dp(edges), _dp(sig_t), _dp(sig_s), float(speed), float(dt), float(theta),
        _dp(phi_old), _dp(J_old), _dp(F_old), _dp(F_new), float(PL), float(PR), float(JL), float(JR),
        _dp(q_old), _dp(q_new), _dp(phi), _dp(J)))
    return phi, J


def losm_march(edges, sig_t, sig_s, speed, dt, theta, F, P, phi0, J0):
    """Fully implicit LOSM march with frozen closures F[n] (I+2), P[n] (2)."""
    edges, sig_t, sig_s, F, P, phi0, J0 = map(_f64, (edges, sig_t, sig_s, F, P, phi0, J0))
    I = len(sig_t)
    N = F.shape[0] - 1
    assert F.shape == (N + 1, I + 2) and P.shape == (N + 1, 2)
    phi = np.zeros((N + 1, I + 2))
    J = np.zeros((N + 1, I + 1))
    _check("losm_march", lib().orc_losm_march(I, _dp(edges), _dp(sig_t), _dp(sig_s), float(speed), float(dt),
                                              float(theta), N, _dp(F), _dp(P), _dp(phi0), _dp(J0), _dp(phi),
                                              _dp(J)))
    return phi, J


def losm_adjoint(edges, sig_t, sig_s, speed, dt, theta, phi_hist, J_hist, weights):
    """Gradient of sum(weights * phi_hist) with respect to sigma_t, sigma_s."""
    edges, sig_t, sig_s, phi_hist, J_hist, weights = map(_f64, (edges, sig_t, sig_s, phi_hist, J_hist, weights))
    I = len(sig_t)
    N = phi_hist.shape[0] - 1
    gt = np.zeros(I)
    gs = np.zeros(I)
    _check("losm_adjoint", lib().orc_losm_adjoint(I, _dp(edges), _dp(sig_t), _dp(sig_s), float(speed), float(dt),
                                                  float(theta), N, _dp(phi_hist), _dp(J_hist), _dp(weights),
                                                  _dp(gt), _dp(gs)))
    return gt, gs


# --------------------------------------------------------------------------
# Simulation
# --------------------------------------------------------------------------
class _Params(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("edges", C.POINTER(C.c_double)),
                ("sigma_t", C.POINTER(C.c_double)), ("sigma_s", C.POINTER(C.c_double)),
                ("speed", C.c_double), ("dt", C.c_double), ("n_steps", C.c_int32),
                ("src_x", C.c_double), ("n_src", C.c_int64), ("bank_capacity", C.c_int64),
                ("seed", C.c_uint32), ("replica", C.c_uint32), ("n_batches", C.c_int32),
                ("n_chunks", C.c_int32), ("sigma_f", C.POINTER(C.c_double)), ("nu_f", C.c_double),
                ("track_moments", C.c_int32)]


class _Opts(C.Structure):
    _fields_ = [("theta", C.c_double), ("implicit", C.c_int32), ("filter", C.c_int32),
                ("ma_k", C.c_int32), ("eps_min", C.c_double), ("rho", C.c_double),
                ("closure_track", C.c_int32), ("apply_windows", C.c_int32), ("kappa", C.c_int32),
                ("lagged", C.c_int32), ("window_scale", C.c_int32)]


@dataclass
class LosmOpts:
    theta: float = 0.5
    filter: int = 0
    ma_k: int = 3
    eps_min: float = 1e-3
    rho: float = 5.0
    closure_track: int = 0
    kappa: int = 30
    lagged: int = 0
    window_scale: int = 0


class OracleSim:
    """One problem on the oracle.  Arguments are plain numbers and arrays."""

    def __init__(self, edges, sigma_t, sigma_s, speed, dt, n_steps, src_x, n_src,
                 bank_capacity=None, seed=1, replica=0, n_batches=32, n_chunks=4, sigma_f=None, nu_f=0.0,
                 track_moments=0):
        self.edges = _f64(edges)
        self.sigma_t = _f64(sigma_t)
        self.sigma_s = _f64(sigma_s)
        self.sigma_f = None if sigma_f is None else _f64(sigma_f)
        self.I = len(self.sigma_t)
        self.B = int(n_batches)
        self.n_chunks = int(n_chunks)
        self.n_src = int(n_src)
        self.speed, self.dt, self.n_steps = float(speed), float(dt), int(n_steps)
        cap = int(bank_capacity) if bank_capacity is not None else max(4 * self.n_src, 1024)
        p = _Params(self.I, _dp(self.edges), _dp(self.sigma_t), _dp(self.sigma_s), self.speed,
                    self.dt, self.n_steps, float(src_x), self.n_src, cap, int(seed), int(replica),
                    self.B, self.n_chunks, _dp(self.sigma_f), float(nu_f), int(track_moments))
        h = C.c_void_p()
        _check("create", lib().orc_create(C.byref(p), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls --------------------------------------------------------------
    def set_batch_mask(self, mask):
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        assert m.shape == (self.B,)
        _check("set_batch_mask", lib().orc_set_batch_mask(self._h, m.ctypes.data))

    def set_windows(self, centre, rho):
        if centre is None:
            _check("set_windows", lib().orc_set_windows(self._h, None, float(rho)))
            return
        c = _f64(centre)
        assert c.shape == (self.I,)
        _check("set_windows", lib().orc_set_windows(self._h, _dp(c), float(rho)))

    def sweep(self, step, chunk):
        _check("sweep", lib().orc_sweep_chunk(self._h, int(step), int(chunk)))

    def comb(self, n_target):
        """Uniform comb of the finished step's census into n_target particles;
        returns (census size before, total weight)."""
        nb, wt = C.c_int64(), C.c_double()
        _check("comb", lib().orc_comb(self._h, int(n_target), C.byref(nb), C.byref(wt)))
        return int(nb.value), float(wt.value)

    def set_comb_mode(self, mode):
        """0: comb teeth spaced in cumulative weight (equal weights after);
        1: spaced in particle index (weights scaled by n / n_target)."""
        _check("set_comb_mode", lib().orc_set_comb_mode(self._h, int(mode)))

    def solve_losm(self, opts: LosmOpts, implicit: bool, apply_windows=True):
        o = _Opts(float(opts.theta), int(implicit), int(opts.filter), int(opts.ma_k),
                  float(opts.eps_min), float(opts.rho), int(opts.closure_track), int(apply_windows),
                  int(opts.kappa), int(opts.lagged), int(opts.window_scale))
        phi = np.zeros(self.I + 2)
        J = np.zeros(self.I + 1)
        _check("solve_losm", lib().orc_solve_losm(self._h, C.byref(o), _dp(phi), _dp(J)))
        return phi, J

    def losm_inputs(self, implicit, closure_track=0):
        """Unfiltered initial condition and closures of the next HLOSM solve:
        (phi_o, J_o, F_o, F_n, P), or None when no start weight has been swept
        yet in the step (implicit solve without closures)."""
        phi_o, J_o = np.zeros(self.I + 2), np.zeros(self.I + 1)
        F_o, F_n, P = np.zeros(self.I + 2), np.zeros(self.I + 2), np.zeros(2)
        rc = lib().orc_losm_inputs(self._h, int(bool(implicit)), int(closure_track), _dp(phi_o), _dp(J_o),
                                   _dp(F_o), _dp(F_n), _dp(P))
        if rc == 1:
            return None
        _check("losm_inputs", rc)
        return phi_o, J_o, F_o, F_n, P

    def closures(self):
        F, P = np.zeros(self.I + 2), np.zeros(2)
        phi, J = np.zeros(self.I + 2), np.zeros(self.I + 1)
        _check("closures", lib().orc_get_closures(self._h, _dp(F), _dp(P), _dp(phi), _dp(J)))
        return F, P, phi, J

    # -- reads --------------------------------------------------------------
    def tallies(self, cur=True):
        cells = np.zeros((self.B, self.I, 6))
        bnd = np.zeros((self.B, 2, 3))
        _check("tallies", lib().orc_get_tallies(self._h, int(bool(cur)), _dp(cells), _dp(bnd)))
        return cells, bnd

    def counters(self):
        out = np.zeros(N_COUNTERS, dtype=np.uint64)
        _check("counters", lib().orc_get_counters(self._h, out.ctypes.data_as(C.POINTER(C.c_uint64))))
        return {n: int(out[i]) for i, n in enumerate(COUNTER_NAMES)}

    def tracks(self):
        out = np.zeros(self.I, dtype=np.uint64)
        _check("tracks", lib().orc_get_tracks(self._h, out.ctypes.data_as(C.POINTER(C.c_uint64))))
        return out

    def windows(self):
        c, u, f = np.zeros(self.I), np.zeros(self.I), np.zeros(self.I)
        rc = lib().orc_get_windows(self._h, _dp(c), _dp(u), _dp(f))
        if rc == 1:
            return None
        _check("windows", rc)
        return c, u, f

    def state(self):
        st, nc = C.c_int32(), C.c_int32()
        ws, wn = np.zeros(self.n_chunks), np.zeros(self.n_chunks)
        _check("state", lib().orc_get_state(self._h, C.byref(st), C.byref(nc), _dp(ws), _dp(wn)))
        return int(st.value), int(nc.value), ws, wn

    def bank(self, which):
        n = int(lib().orc_bank_size(self._h, int(which)))
        out = {
            "x": np.zeros(n), "mu": np.zeros(n), "w": np.zeros(n),
            "src": np.zeros(n, np.uint32), "lin": np.zeros(n, np.uint64),
            "e": np.zeros(n, np.uint32), "cell": np.zeros(n, np.int32), "chunk": np.zeros(n, np.int32),
        }
        _check("bank", lib().orc_get_bank(self._h, int(which), *[out[k].ctypes.data for k in
                                                                 ("x", "mu", "w", "src", "lin", "e", "cell", "chunk")]))
        return out


def run(sim: OracleSim, steps, opts: LosmOpts | None, on_step=None, windows=None, comb=None):
    """Time loop of the method (Sec. 3): at the start of step n the
    semi-implicit HLOSM solve sets the windows; after each of the first
    n_chunks-1 chunks of histories the fully implicit solve updates them.
    ``opts=None`` runs analog (no windows); ``windows`` (a callable n -> centre
    array) feeds fixed windows instead of the HLOSM ones; ``comb`` (a number
    of particles) combs every census but the last one to that size."""
    for n in range(1, steps + 1):
        if comb and n > 1:
            sim.comb(comb)
        if opts is not None and windows is None:
            sim.solve_losm(opts, implicit=False)
        elif windows is not None:
            sim.set_windows(windows(n), opts.rho if opts else 5.0)
        for p in range(sim.n_chunks):
            sim.sweep(n, p)
            if opts is not None and windows is None and not opts.lagged and p < sim.n_chunks - 1:
                sim.solve_losm(opts, implicit=True)
        if on_step is not None:
            on_step(n, sim)
