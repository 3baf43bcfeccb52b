"""torch.autograd front end of the reverse mode: N coupled steps of a Lattice as
a differentiable function of the initial state and of (gamma, tau, M, kT).

The forward records the run with checkpoints (lbm_record); the backward is the
library's adjoint (lbm_adjoint), which recomputes each segment from its
checkpoint and sweeps it in reverse.  Both run in the HIP kernels; this file
only marshals tensors.
"""
from __future__ import annotations

import torch

from .sim import Lattice


class CoupledSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, r0, v0, params, lattice: Lattice, nsteps: int, every: int):
        p = [float(x) for x in params.detach().cpu().tolist()]
        pd = lattice.pdesc if lattice.n else None
        have = [pd.gamma, lattice.tau, pd.mass, pd.kT] if pd else [p[0], lattice.tau, p[2], p[3]]
        if any(abs(a - b) > 1e-15 * max(1.0, abs(b)) for a, b in zip(p, have)):
            raise ValueError(f"params {p} differ from the lattice's (gamma, tau, M, kT) = {have}")
        lattice.set_populations(f0.detach())
        if lattice.n:
            lattice.r.copy_(r0.detach().reshape(-1, 3))
            lattice.v.copy_(v0.detach().reshape(-1, 3))
        ctx.lattice = lattice
        ctx.tape = lattice.record(nsteps, every)
        fN = lattice.populations()
        if lattice.n:
            rN, vN = lattice.r.clone(), lattice.v.clone()
        else:
            rN = torch.zeros_like(r0, dtype=torch.float64)
            vN = torch.zeros_like(v0, dtype=torch.float64)
        return fN, rN, vN

    @staticmethod
    def backward(ctx, gf, gr, gv):
        g = ctx.lattice.adjoint(ctx.tape, gf, gr, gv)
        return g["pop"], g["r"], g["v"], g["params"], None, None, None


def coupled_steps(lattice: Lattice, f0, r0, v0, params, nsteps: int, every: int = 100):
    """(f^N, r^N, V^N) after nsteps steps from (f0, r0, v0); differentiable in
    f0, r0, v0 and params = tensor([gamma, tau, M, kT]) (which must equal the
    lattice's own parameters: they select the operating point)."""
    return CoupledSteps.apply(f0, r0, v0, params, lattice, int(nsteps), int(every))
