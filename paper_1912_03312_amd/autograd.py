"""torch.autograd wrapper: N REXI steps with gradients w.r.t. psi_0 and V.

Forward: psi_N = R(V)^N psi_0 with R = sum_j w_j (H(V) - s_j)^{-1}
(eq. ``rational-evaluation``), run by the HIP library, keeping psi every
``checkpoint_every`` steps. Backward: per segment, the states are recomputed
from the segment's checkpoint, then ``rexi_step_adjoint`` runs the steps in
reverse:
    gbar_n = R^H gbar_{n+1},   dL/dV += -2 Re sum_j w_j conj(y_j) x_j,
with x_j = (H - s_j)^{-1} psi_n and y_j = (H - conj s_j)^{-1} gbar_{n+1}.

Conventions: for a complex tensor torch passes the gradient 2 dL/d conj(z).
The step map is complex-linear in psi, so psi's gradient passes through the
adjoint as is; the library's dV formula is written for dL/d conj(psi), so
the V gradient is scaled by 1/2. Poles are constants.
"""
from __future__ import annotations

import torch

from . import rexi


class _Propagate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, V, spec, nsteps, every):
        n = psi0.numel()
        h = rexi.setup(spec["n"], spec["lo"], spec["hi"], V.detach().contiguous(), spec["hbar"], spec["mass"],
                       spec["dt"], spec["sigma"], spec["beta"], **spec["opts"])
        cur = psi0.detach().contiguous().clone()
        nxt = torch.empty_like(cur)
        checkpoints = [cur.clone()]
        for k in range(nsteps):
            h.step(cur, nxt, 1, info=False)
            cur, nxt = nxt, cur
            if (k + 1) % every == 0 and k + 1 < nsteps:
                checkpoints.append(cur.clone())
        ctx.h = h
        ctx.nsteps, ctx.every, ctx.n = nsteps, every, n
        ctx.save_for_backward(*checkpoints)
        return cur.clone()

    @staticmethod
    def backward(ctx, gout):
        h = ctx.h
        checkpoints = ctx.saved_tensors
        g = gout.detach().contiguous().to(torch.complex128).clone()
        gnew = torch.empty_like(g)
        dV = torch.zeros(ctx.n, dtype=torch.float64, device=g.device)
        nseg = len(checkpoints)
        for seg in range(nseg - 1, -1, -1):
            start = seg * ctx.every
            stop = min(start + ctx.every, ctx.nsteps)
            states = [checkpoints[seg]]
            cur = checkpoints[seg].clone()
            nxt = torch.empty_like(cur)
            for _ in range(start, stop - 1):
                h.step(cur, nxt, 1, info=False)
                cur, nxt = nxt, cur
                states.append(cur.clone())
            for psi_n in reversed(states):
                h.step_adjoint(psi_n, g, gnew, dV)
                g, gnew = gnew, g
        ctx.h = None
        h.close()
        return g, 0.5 * dV, None, None, None


def propagate(psi0: torch.Tensor, V: torch.Tensor, grid_n, lo, hi, dt: float, sigma, beta, nsteps: int,
              hbar: float = 1.0, mass: float = 1.0, checkpoint_every: int = 5, **opts) -> torch.Tensor:
    """psi_N after ``nsteps`` REXI steps; differentiable w.r.t. ``psi0`` (complex128,
    flat) and ``V`` (float64, flat). Both live on the GPU."""
    spec = dict(n=tuple(grid_n), lo=tuple(lo), hi=tuple(hi), hbar=hbar, mass=mass, dt=dt,
                sigma=sigma, beta=beta, opts=opts)
    return _Propagate.apply(psi0, V, spec, int(nsteps), max(1, int(checkpoint_every)))
