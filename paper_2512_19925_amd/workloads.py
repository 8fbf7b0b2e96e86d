"""Seeded synthetic workloads of the hybrid weight-window sweep.

This module only builds problem inputs (meshes, cross sections, source and
window parameters).  It holds none of the method's arithmetic, so both the GPU
path and the CPU oracle may be fed from it.

The physics follows the paper's test (Sec. 5.1: infinite homogeneous slab, an
isotropic unit pulse at x = 0 and t = 0, one speed) with the scattering ratios,
meshes and particle counts of the workloads below.  Most are pure scattering
plus absorption (c < 1, no fission), so no population control is needed; the
paper's own supercritical problem (`paper_fission`) adds fission and combs
every census back to a fixed population.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass
class Workload:
    name: str
    x_lo: float
    x_hi: float
    n_cells: int
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    speed: float = 1.0
    dt: float = 0.1
    n_steps: int = 20
    src_x: float = 0.0
    n_src: int = 10_000
    bank_capacity: int = 0
    seed: int = 1
    replica: int = 0
    n_batches: int = 32
    n_chunks: int = 4          # u_ww + 1 (three window updates per step)
    rho: float = 5.0
    eps_min: float = 1e-3
    theta: float = 0.5         # Crank-Nicolson
    filter: int = 0            # 0 none, 1 moving average, 2 Fourier low pass
    ma_k: int = 3
    kappa: int = 30            # Fourier cutoff
    lagged: bool = False       # windows from the previous step's track-length flux (no LOSM)
    closure_track: int = 0
    analog: bool = False
    sigma_f: np.ndarray | None = None  # fission cross sections (None: no fission)
    nu_f: float = 0.0                  # mean neutrons per fission
    comb: int = 0                      # comb every census to this many particles (0: never)
    comb_by_index: bool = False        # comb teeth spaced in particle index (else in cumulative weight)
    window_scale: int = 0              # 1: window centres as printed (largest 1), 0: times s^n
    track_moments: int = 0             # track moments per segment: 0/3 phi, J, K; 2 phi, K; 1 phi

    @property
    def edges(self) -> np.ndarray:
        return np.linspace(self.x_lo, self.x_hi, self.n_cells + 1)

    def capacity(self) -> int:
        return self.bank_capacity if self.bank_capacity > 0 else max(4 * self.n_src, 4096)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def homogeneous(name, x_lo, x_hi, n_cells, sigma_t, c, **kw) -> Workload:
    st = np.full(n_cells, float(sigma_t))
    ss = st * float(c)
    return Workload(name=name, x_lo=x_lo, x_hi=x_hi, n_cells=n_cells, sigma_t=st, sigma_s=ss, **kw)


def plain_small() -> Workload:
    """Plain hybrid-WW FP64 problem: 200 cells on [-20, 20], sigma_t = 1,
    c = 0.9, v = 1, 20 steps of 0.1, 1e4 source particles, window width 5."""
    return homogeneous("plain-200c-1e4", -20.0, 20.0, 200, 1.0, 0.9, dt=0.1, n_steps=20,
                       n_src=10_000, rho=5.0, seed=1)


def full_scale(c: float = 0.9, rho: float = 5.0, n_src: int = 10_000_000) -> Workload:
    """Full-scale FP64 problem: 1000 cells on [-50, 50], 100 steps of 0.05,
    1e7 source particles, moving-average filtered closures, bank <= 4e7."""
    return homogeneous(f"full-1000c-c{c}-rho{rho}", -50.0, 50.0, 1000, 1.0, c, dt=0.05,
                       n_steps=100, n_src=n_src, rho=rho, filter=1, ma_k=3,
                       bank_capacity=max(4 * n_src, 4096), seed=1)


FULL_SCALE_C = (0.5, 0.9, 0.99)
FULL_SCALE_RHO = (2.0, 2.5, 5.0, 10.0)


def paper_fission(n_src: int = 10_000) -> Workload:
    """The paper's supercritical test problem (Sec. 5.1): 201 cells on
    [-20.5, 20.5], sigma_t = 1, sigma_s = sigma_f = 1/3, nu_f = 2.3
    (c_eff = 1.1), v = 1, 20 steps of 1, H^n = 1e4 histories per step kept by
    uniform combing, windows of width 1.25 with eps_min = 1e-3, Crank-Nicolson,
    three window updates per step, moving-average filtered closures (k = 3).
    The bank holds 400 H: unfiltered closures and lagged windows split the
    census at the wave front to about 3e6 particles."""
    I = 201
    st = np.ones(I)
    return Workload(name="paper-fission-201c", x_lo=-20.5, x_hi=20.5, n_cells=I, sigma_t=st,
                    sigma_s=st / 3.0, sigma_f=st / 3.0, nu_f=2.3, speed=1.0, dt=1.0, n_steps=20,
                    n_src=n_src, comb=n_src, comb_by_index=True, rho=1.25, eps_min=1e-3, filter=1, ma_k=3,
                    bank_capacity=max(400 * n_src, 4096), seed=1)


def precision_form(n_src: int = 10_000_000) -> Workload:
    """The small problem's geometry with 1e7 particles (FP32 flight arithmetic)."""
    return plain_small().with_(name="fp32-200c-1e7", n_src=n_src, bank_capacity=4 * n_src)


def batched_replicas(n_replicas: int = 256, seed: int = 1, n_steps: int = 50):
    """Uneven replicas: sigma_t ~ U[0.5, 2], c ~ U[0.3, 0.99],
    cells ~ logU[100, 2000], particles ~ logU[1e3, 1e6]; domain [-20, 20],
    dt = 0.1.  Drawn in that order per replica from default_rng(seed).
    Moving-average filtered closures (k = 3): on meshes this fine the
    unfiltered closures give windows noisy enough to split some banks past
    four times their source size within a few steps."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_replicas):
        st = rng.uniform(0.5, 2.0)
        c = rng.uniform(0.3, 0.99)
        cells = int(round(np.exp(rng.uniform(np.log(100.0), np.log(2000.0)))))
        cells += cells % 2  # keep the pulse on a cell edge, as in the other workloads
        npart = int(round(np.exp(rng.uniform(np.log(1e3), np.log(1e6)))))
        w = homogeneous(f"replica{r}", -20.0, 20.0, cells, st, c, dt=0.1, n_steps=n_steps,
                        n_src=npart, rho=5.0, seed=seed, replica=r, filter=1, ma_k=3,
                        bank_capacity=max(4 * npart, 4096))
        out.append(w)
    return out


def adjoint_slab(seed: int = 1, n_src: int = 1_000_000) -> Workload:
    """Heterogeneous slab: 1000 cells on [-20, 20], per-cell sigma_t ~ U[0.5, 2],
    sigma_s = c sigma_t with c ~ U[0.5, 0.95], 40 steps of 0.25."""
    rng = np.random.default_rng(seed)
    I = 1000
    st = rng.uniform(0.5, 2.0, size=I)
    c = rng.uniform(0.5, 0.95, size=I)
    return Workload(name="adjoint-1000c", x_lo=-20.0, x_hi=20.0, n_cells=I, sigma_t=st,
                    sigma_s=st * c, dt=0.25, n_steps=40, n_src=n_src, rho=5.0,
                    bank_capacity=4 * n_src, seed=seed)


ADJOINT_CELLS = (600, 700)  # functional cells [600, 700)


def adjoint_weights(w: Workload, n_steps: int, cells=ADJOINT_CELLS) -> np.ndarray:
    """Weights of G = sum over cells [lo, hi) of the time integral of phi over
    n_steps steps by the trapezoidal rule: w[n][1 + i] for cell i (the first
    and last phi entries are the face values)."""
    lo, hi = cells
    W = np.zeros((n_steps + 1, w.n_cells + 2))
    W[:, 1 + lo:1 + hi] = w.dt
    W[0] *= 0.5
    W[n_steps] *= 0.5
    return W
