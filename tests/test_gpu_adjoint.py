"""Differentiation through REXI steps: the autograd wrapper and its adjoint.

Workload: 2D 256^2 on [-10, 10]^2, 20 bumps (seed 5), packet (seed 50),
target packet (seed 51), K = 32, dt = 0.5, 20 steps, checkpoints every 5,
L = |<phi, psi_N>_h|^2. Checked against the FP64 oracle's adjoint gradient
(direct solves) and against central finite differences of the GPU forward
along seeded random directions.
"""
import numpy as np
import pytest

from oracle import faber_cf as fcf
from oracle import step as ost
from paper_1912_03312_amd import inputs

from .gpu_util import rel, to_dev

pytestmark = pytest.mark.gpu


def _oracle_grad(g, V, psi0, phi, s, b, dt, nsteps):
    D = ost.DirectStepper(g.n, g.h, V, s, b, dt)
    traj = [psi0.ravel()]
    for _ in range(nsteps):
        traj.append(D.step(traj[-1]).ravel())
    ov = g.cell_volume * np.vdot(phi.ravel(), traj[-1])
    L = abs(ov) ** 2
    gbar = g.cell_volume * ov * phi.ravel()          # dL/d conj(psi_N)
    dV = np.zeros(g.size)
    for n in range(nsteps - 1, -1, -1):
        gbar, dv = D.adjoint(traj[n], gbar)
        gbar = gbar.ravel()
        dV += dv.ravel()
    return L, gbar, dV


@pytest.mark.parametrize("scale,nsteps,solver", [(48, 6, "per_pole"), (None, 20, "per_pole"), (48, 6, "shifted"),
                                                  (None, 20, "shifted")])
def test_autograd_matches_oracle_adjoint(scale, nsteps, solver):
    import torch
    from paper_1912_03312_amd.autograd import propagate
    wl = inputs.workload("2d_adjoint", scale=scale)
    g = wl.grid
    phi = inputs.adjoint_target(g)
    s, b, _ = fcf.faber_cf(wl.K, wl.R1)
    L0, g_ref, dV_ref = _oracle_grad(g, wl.V, wl.psi0, phi, s, b, wl.dt, nsteps)
    psi0 = to_dev(wl.psi0.ravel()).requires_grad_(True)
    V = to_dev(wl.V.ravel()).requires_grad_(True)
    phid = to_dev(phi.ravel())
    out = propagate(psi0, V, g.n, g.lo, g.hi, wl.dt, s, b, nsteps, checkpoint_every=5,
                    tol=1e-12, tol_policy="certified", solver=solver, m=200 if solver == "shifted" else 30)
    ov = g.cell_volume * torch.vdot(phid, out)
    L = (ov.abs() ** 2)
    L.backward()
    torch.cuda.synchronize()
    # torch's gradient of a complex leaf is 2 dL/d conj(psi0)
    e_psi = rel(psi0.grad.cpu().numpy() / 2.0, g_ref)
    e_V = rel(V.grad.cpu().numpy(), dV_ref)
    print("autograd", g.n, nsteps, "L", float(L), L0, "grad psi0", e_psi, "grad V", e_V)
    # the loss carries the forward's own error (iterative solves, amplified by
    # the pole sum over nsteps steps); the gradients carry the same order
    assert abs(float(L) - L0) <= 1e-7 * max(L0, 1e-12)
    assert e_psi <= 1e-7 and e_V <= 1e-7


def test_gradient_vs_central_differences():
    # the full differentiation workload; FD of the GPU forward with h = 1e-6
    import torch
    from paper_1912_03312_amd.autograd import propagate
    wl = inputs.workload("2d_adjoint")
    g = wl.grid
    phi = to_dev(inputs.adjoint_target(g).ravel())
    s, b, d = fcf.faber_cf(wl.K, wl.R1)
    opts = dict(tol=1e-13, tol_policy="certified")

    def loss(psi0, V):
        out = propagate(psi0, V, g.n, g.lo, g.hi, wl.dt, s, b, wl.steps, checkpoint_every=5, **opts)
        return (g.cell_volume * torch.vdot(phi, out)).abs() ** 2

    psi0 = to_dev(wl.psi0.ravel()).requires_grad_(True)
    V = to_dev(wl.V.ravel()).requires_grad_(True)
    L = loss(psi0, V)
    L.backward()
    gV = V.grad.detach()
    gp = psi0.grad.detach()
    rng = np.random.default_rng(52)
    hfd = 1e-6
    # FD noise: the forward's relative error delta (iterative solves at the
    # certified 1e-13 target, amplified by the pole sums of 20 steps; measured
    # ~3e-9 against the direct-solve oracle) enters each loss value, so
    # |fd - exact| <= 2 L delta / h + O(h^2)
    delta = 1e-8
    rows = []
    with torch.no_grad():
        for k in range(8):
            dV = rng.standard_normal(g.size)
            dV /= np.linalg.norm(dV)
            dp = rng.standard_normal(g.size) + 1j * rng.standard_normal(g.size)
            dp /= np.linalg.norm(dp)
            dVd, dpd = to_dev(dV), to_dev(dp)
            fd = float((loss(psi0 + hfd * dpd, V + hfd * dVd) - loss(psi0 - hfd * dpd, V - hfd * dVd)) / (2 * hfd))
            an = float((gV * dVd).sum() + torch.real(torch.vdot(gp, dpd)))
            rows.append((fd, an, abs(fd - an)))
    bar = 2 * float(L) * delta / hfd
    print("FD (fd, analytic, |diff|)", rows, "noise bar", bar, "L", float(L))
    for fd, an, dif in rows:
        assert dif <= bar + 1e-4 * abs(an)
