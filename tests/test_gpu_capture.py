"""Captured (graph-replayed) steps of the shared basis against eager steps.

A capture-safe step reads nothing on the host: its schedule is fixed when it
is recorded. With the tiled Lanczos pass the schedule is one launch per
iteration whose iteration index lives on the device, so that a pause for a
second Gram-Schmidt pass (decided on the device) shifts the later launches;
restart cycles on the shared basis run as a fixed number of cycles, idle for
instances whose poles all met their targets. The same arithmetic runs in the
same order as an eager step with host checks, so every replay must equal the
eager step (and the eager step the oracle).
"""
import numpy as np
import pytest

from oracle import faber_cf as fcf
from oracle import hamiltonian as ham
from oracle import step as ost
from paper_1912_03312_amd import inputs

from .gpu_util import rel, to_dev

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps
_POLES = {}


def poles(K, R1):
    if (K, R1) not in _POLES:
        s, b, _ = fcf.faber_cf(K, R1)
        _POLES[(K, R1)] = (s, b)
    return _POLES[(K, R1)]


@pytest.fixture(scope="module")
def rexi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_03312_amd import rexi as r
    return r


def _replays_equal(h, p0, ref, reps=3):
    import torch
    out = torch.empty_like(p0)
    errs = []
    for rep in range(reps):
        out.zero_()
        h.step(p0, out, 1, info=False)          # the first call records, later calls replay
        torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        errs.append(rel(out.cpu().numpy(), ref.cpu().numpy()))
    return errs


@pytest.mark.parametrize("name,scale,K,R1,opts", [
    ("3d_bumps", 20, 32, 80.0, dict(m=100, tol=1e-10)),
    ("3d_bumps", 16, 64, 180.0, dict(m=100, tol=1e-10, tol_policy="certified")),
    # interior shifts of the double well: long runs with second passes
    ("2d_double_well", 40, 32, 80.0, dict(m=256, tol=1e-9, tile=512)),
])
def test_captured_tiled_schedule_matches_eager(rexi, name, scale, K, R1, opts):
    import torch
    wl = inputs.workload(name, scale=scale)
    g = wl.grid
    s, b = poles(K, R1)
    Vd = to_dev(wl.V.ravel())
    kw = dict(solver="shifted", march_planes=4, march_slots=2, **opts)
    he = rexi.setup(g.n, g.lo, g.hi, Vd, 1.0, 1.0, wl.dt, s, b, **kw)
    hg = rexi.setup(g.n, g.lo, g.hi, Vd, 1.0, 1.0, wl.dt, s, b, capture_safe=1, **kw)
    assert hg.tiling()["march_slots"] == 2
    p0 = to_dev(wl.psi0.ravel())
    ref = torch.empty_like(p0)
    ie = he.step(p0, ref, 1)
    torch.cuda.synchronize()
    errs = _replays_equal(hg, p0, ref)
    print("captured", name, g.n, "eager its", ie["total_iterations"], "second passes", ie["reorth_passes"], errs)
    assert ie["not_converged"] == 0
    assert max(errs) <= 1e-13
    if name == "2d_double_well":
        assert ie["reorth_passes"] >= 1  # the captured schedule took them too
    he.close()
    hg.close()


def _batch(count, sides):
    insts = inputs.batch_instances(count=count, sides=sides) if sides else inputs.batch_instances(count=count)
    grids, Vs, psis, dts, Ks, sig, bet = [], [], [], [], [], [], []
    for it in insts:
        g = it["grid"]
        s, b = poles(it["K"], inputs.R1_PARITY[it["K"]])
        grids.append((g.n, g.lo, g.hi))
        Vs.append(it["V"].ravel())
        psis.append(it["psi0"].ravel())
        dts.append(it["dt"])
        Ks.append(it["K"])
        sig.append(s)
        bet.append(b)
    return insts, grids, Vs, psis, dts, Ks, sig, bet


@pytest.mark.parametrize("slots", [2, 0])
def test_captured_batch_with_restarts(rexi, slots):
    # a basis of 24 vectors is too short for the larger instances: their poles
    # restart on the shared basis inside the captured step (five cycles);
    # every replay equals the eager step, which matches the oracle
    import torch
    insts, grids, Vs, psis, dts, Ks, sig, bet = _batch(6, (12, 17, 24, 31, 40, 47))
    cnt = len(insts)
    kw = dict(solver="shifted", m=24, tol=1e-11, tol_policy="certified", max_cycles=200)
    if slots:
        kw.update(march_planes=4, march_slots=slots)
    args = (grids, to_dev(np.concatenate(Vs)), [1.0] * cnt, [1.0] * cnt, dts, Ks, np.concatenate(sig),
            np.concatenate(bet))
    he = rexi.setup_batch(*args, **kw)
    hg = rexi.setup_batch(*args, capture_safe=1, capture_cycles=6, **kw)
    p0 = to_dev(np.concatenate(psis))
    ref = torch.empty_like(p0)
    ie = he.step(p0, ref, 1)
    torch.cuda.synchronize()
    assert ie["not_converged"] == 0 and 1 < ie["max_cycles_used"] <= 6
    errs = _replays_equal(hg, p0, ref)
    print("captured batch", slots, "cycles", ie["max_cycles_used"], errs)
    assert max(errs) <= 1e-13
    res = ref.cpu().numpy()
    off = 0
    for i, it in enumerate(insts):
        g = it["grid"]
        e = rel(res[off:off + g.size], ost.DirectStepper(g.n, g.h, it["V"], sig[i], bet[i], dts[i]).step(it["psi0"]))
        sj, wj = ost.shifts_and_weights(sig[i], bet[i], dts[i])
        lo, hi = ham.gershgorin(g.n, g.h, it["V"])
        dist = np.abs(np.clip(sj.real, lo, hi) - sj)
        floor = float(np.sum(np.abs(wj) / dist * EPS * (1 + (max(abs(lo), abs(hi)) + np.abs(sj)) / dist)))
        assert e <= max(1e-10, 3 * floor), (i, g.n, e)
        off += g.size
    he.close()
    hg.close()


@pytest.mark.timeout(300)
def test_captured_full_uneven_batch_converges(rexi):
    # the uneven batch at full size (256 instances, 27M points, 7,488 poles) as
    # one captured step with restart cycles: its replays equal the eager step,
    # in which every pole met its target
    import torch
    insts, grids, Vs, psis, dts, Ks, sig, bet = _batch(256, None)
    cnt = len(insts)
    kw = dict(solver="shifted", m=256, tol=1e-10, max_cycles=200)
    args = (grids, to_dev(np.concatenate(Vs)), [1.0] * cnt, [1.0] * cnt, dts, Ks, np.concatenate(sig),
            np.concatenate(bet))
    he = rexi.setup_batch(*args, **kw)
    p0 = to_dev(np.concatenate(psis))
    ref = torch.empty_like(p0)
    ie = he.step(p0, ref, 1)
    torch.cuda.synchronize()
    tiling = he.tiling()
    he.close()
    assert ie["not_converged"] == 0
    hg = rexi.setup_batch(*args, capture_safe=1, capture_cycles=ie["max_cycles_used"] + 2, **kw)
    errs = _replays_equal(hg, p0, ref, reps=2)
    print("captured full batch: cycles", ie["max_cycles_used"], "its", ie["total_iterations"], "tiling", tiling,
          hg.tiling(), errs, flush=True)
    hg.close()
    assert max(errs) <= 1e-13
