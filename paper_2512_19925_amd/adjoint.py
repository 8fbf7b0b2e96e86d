"""Gradients of an HLOSM flux functional with respect to per-cell cross
sections, as a torch.autograd.Function over the C ABI.

forward: hww_losm_march (deterministic LOSM march with frozen Monte Carlo
closures, on the GPU) returns G = sum w phi.  backward: hww_losm_adjoint
(transposed solves backward in time, on the GPU) returns dG/dsigma_t and
dG/dsigma_s.  Argument marshalling only.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hww as H


class LosmFunctional(torch.autograd.Function):
    """G(sigma_t, sigma_s) for fixed closures, initial condition and weights."""

    @staticmethod
    def forward(ctx, sigma_t, sigma_s, handle: "H.Handle", theta, F, P, phi0, J0, weights):
        st = sigma_t.detach().to("cpu", torch.float64).numpy()
        ss = sigma_s.detach().to("cpu", torch.float64).numpy()
        G = handle.losm_march(st, ss, theta, F, P, phi0, J0, weights)
        ctx.handle = handle
        ctx.march = (st.copy(), ss.copy(), theta, F, P, phi0, J0, weights)
        ctx.march_id = handle.march_count = getattr(handle, "march_count", 0) + 1
        ctx.device, ctx.dtype = sigma_t.device, sigma_t.dtype
        return torch.tensor(G, dtype=torch.float64, device=sigma_t.device)

    @staticmethod
    def backward(ctx, grad_G):
        h = ctx.handle
        if getattr(h, "march_count", 0) != ctx.march_id:
            # Another march ran since this forward: redo ours so that the
            # adjoint sees its own state.
            h.losm_march(*ctx.march)
            h.march_count = ctx.march_id = h.march_count + 1
        gt, gs = h.losm_adjoint()
        g = grad_G.to("cpu", torch.float64)
        to = dict(device=ctx.device, dtype=ctx.dtype)
        return (torch.from_numpy(gt).mul(g).to(**to), torch.from_numpy(gs).mul(g).to(**to),
                None, None, None, None, None, None, None)


def record_closures(h: "H.Handle", w, steps, analog=False):
    """Run the Monte Carlo method for `steps` steps and record the closures
    each finished step hands to the next: F (steps+1, I+2), P (steps+1, 2),
    and the initial condition phi^0, J^0 of the source."""
    F0, P0, phi0, J0 = h.read_closures()
    Fs, Ps = [F0], [P0]

    def on_step(n, hh, _):
        F, P, _phi, _J = hh.read_closures()
        Fs.append(F)
        Ps.append(P)

    H.run(h, w, steps=steps, on_step=on_step, analog=analog, stats=False)
    return np.array(Fs), np.array(Ps), phi0, J0
