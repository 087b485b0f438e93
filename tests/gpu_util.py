"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import numpy as np


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_steps(grid, V, psi0, sigma, beta, dt, nsteps, hbar=1.0, mass=1.0, **opt):
    """Run ``nsteps`` single steps through the C ABI; returns (states, infos)."""
    import torch
    from paper_1912_03312_amd import rexi
    Vd = to_dev(np.asarray(V, dtype=np.float64).ravel())
    h = rexi.setup(grid.n, grid.lo, grid.hi, Vd, hbar, mass, dt, sigma, beta, **opt)
    cur = to_dev(np.asarray(psi0, dtype=np.complex128).ravel())
    nxt = torch.empty_like(cur)
    states, infos = [], []
    for _ in range(nsteps):
        infos.append(h.step(cur, nxt, 1))
        torch.cuda.synchronize()
        states.append(nxt.cpu().numpy().reshape(grid.n).copy())
        cur, nxt = nxt, cur
    h.close()
    return states, infos


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
