"""The allocation-free spectrum estimate against the allocating one.

rexi_estimate_spectrum_noalloc runs the kernels of rexi_estimate_spectrum in
the library's fixed device workspace instead of allocated buffers, so on the
same handle both give the same Ritz values (same kernels, same order: bitwise
equal in practice; the bar is FP64 rounding, 1e-13 of the spectrum's scale).
Two calls in a row, the second on a smaller input, show that what the first
call leaves in the shared workspace does not leak into the second.
"""
import numpy as np
import pytest

from oracle import faber_cf as fcf
from oracle import hamiltonian as ham
from paper_1912_03312_amd import inputs

from .gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _handle(r, grids, seeds):
    s, b, _ = fcf.faber_cf(16, 28.0)
    Vs = [inputs.gaussian_bumps(g, sd).ravel() for g, sd in zip(grids, seeds)]
    if len(grids) == 1:
        g = grids[0]
        return r.setup(g.n, g.lo, g.hi, to_dev(Vs[0]), 1.0, 1.0, 0.01, s, b), Vs
    n = len(grids)
    return r.setup_batch([(g.n, g.lo, g.hi) for g in grids], to_dev(np.concatenate(Vs)), [1.0] * n, [1.0] * n,
                         [0.01] * n, [16] * n, np.concatenate([s] * n), np.concatenate([b] * n)), Vs


def _check(h, grids, Vs, iters):
    lo_a, hi_a = h.estimate_spectrum(iters)
    lo_b, hi_b = h.estimate_spectrum_noalloc(iters)
    for k, (g, V) in enumerate(zip(grids, Vs)):
        glo, ghi = ham.gershgorin(g.n, g.h, V)
        scale = max(abs(glo), abs(ghi))
        print("noalloc", g.n, iters, lo_b[k], lo_a[k], hi_b[k], hi_a[k], flush=True)
        assert abs(lo_b[k] - lo_a[k]) <= 1e-13 * scale
        assert abs(hi_b[k] - hi_a[k]) <= 1e-13 * scale
        # Ritz values lie inside the spectrum bound
        assert glo - 1e-12 * scale <= lo_b[k] <= hi_b[k] <= ghi + 1e-12 * scale


def test_noalloc_spectrum_matches_allocating_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_03312_amd import rexi as r
    # first call: an uneven batch (a 3D and a 2D instance), 40 iterations
    g1 = inputs.Grid((24, 24, 24), (-3.0,) * 3, (4.0,) * 3)
    g2 = inputs.Grid((96, 80), (-5.0, -4.0), (5.0, 4.0))
    h, Vs = _handle(r, [g1, g2], [7, 8])
    _check(h, [g1, g2], Vs, 40)
    h.close()
    # second call: a smaller single instance and fewer iterations
    g3 = inputs.Grid((40, 33), (-5.0, -4.0), (5.0, 4.0))
    h3, V3 = _handle(r, [g3], [9])
    _check(h3, [g3], V3, 20)
    # the allocation-free workspace is bounded: larger requests are refused
    # before anything runs, and bad iteration counts as before
    with pytest.raises(r.RexiError):
        h3.estimate_spectrum_noalloc(0)
    h3.close()
    g4 = inputs.Grid((1024, 1024), (-5.0, -5.0), (5.0, 5.0))
    h4, _ = _handle(r, [g4], [10])
    with pytest.raises(r.RexiError, match="workspace holds"):
        h4.estimate_spectrum_noalloc(20)  # 22 vectors of 16 MiB > 256 MiB
    lo, hi = h4.estimate_spectrum_noalloc(8)  # 10 vectors of 16 MiB fit
    lo_a, hi_a = h4.estimate_spectrum(8)
    assert abs(lo[0] - lo_a[0]) <= 1e-13 * abs(hi_a[0]) and abs(hi[0] - hi_a[0]) <= 1e-13 * abs(hi_a[0])
    h4.close()
