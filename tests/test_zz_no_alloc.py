"""The no-allocation cross-scale entry point (MI355X only): through the
C-ABI it gives the same supports, coefficients, k_used and x-hat, bit for
bit, as cspd_omp_cross_scale on the same inputs, on two calls in a row
(the second smaller, so stale workspace contents from the first are
present), and it rejects a batch whose workspace exceeds its static
scratch before launching anything."""
import numpy as np
import pytest

import gpu_util as G
import synth
from paper_1511_05174_amd import cspd

pytestmark = pytest.mark.gpu


def _np(ts):
    return [t.cpu().numpy() for t in ts]


def _both(plan, w, keep_coarse):
    torch = G.torch_mod()
    y, mask, kf, _ = G.inputs(w)
    ks = w.k_scales
    B = y.shape[0]
    ncoarse = int(sum(ks[:-1]))
    sc_ref = torch.full((B, ncoarse), -7, dtype=torch.int32, device=y.device) if keep_coarse else None
    sc_new = torch.full((B, ncoarse), -9, dtype=torch.int32, device=y.device) if keep_coarse else None
    ref = _np(cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1], support_coarse=sc_ref))
    torch.cuda.synchronize()
    got = _np(cspd.cspd_omp_cross_scale_noalloc(plan, y, mask, ks[:-1], kf, ks[-1], support_coarse=sc_new))
    torch.cuda.synchronize()
    for name, a, b in zip(("support", "coef", "k_used", "xhat"), ref, got):
        assert a.shape == b.shape and np.array_equal(a, b), f"{w.name}: {name} differs (B = {B})"
    if keep_coarse:
        assert np.array_equal(sc_ref.cpu().numpy(), sc_new.cpu().numpy())


@pytest.mark.parametrize("name,b1,b2", [("c2", 8192, 1001), ("c3", 2048, 333), ("c4", 1536, 77)])
def test_noalloc_matches_allocating_call(name, b1, b2):
    w1 = synth.make(name, batch=b1)
    plan = cspd.plan_from_workload(w1)
    print(f"noalloc parity: {name} B = {b1} then {b2}", flush=True)
    _both(plan, w1, keep_coarse=False)
    w2 = synth.make(name, batch=b2, seed=11)
    _both(plan, w2, keep_coarse=False)
    _both(plan, w2, keep_coarse=True)


def test_noalloc_rejects_batches_beyond_the_scratch():
    torch = G.torch_mod()
    w = synth.make("c2", batch=64)
    plan = cspd.plan_from_workload(w)
    ks = w.k_scales
    # 4 (S - 1) + 4 ksum = 20 bytes per patch without the caller's coarse
    # supports: a batch just past the scratch is refused before any launch
    B = cspd.NOALLOC_SCRATCH_BYTES // 20 + 64
    y = torch.zeros((B, w.y.shape[1]), dtype=torch.float32, device="cuda")
    mask = torch.ones((B, w.dims[-1]), dtype=torch.uint8, device="cuda")
    with pytest.raises(cspd.CspdError) as ei:
        cspd.cspd_omp_cross_scale_noalloc(plan, y, mask, ks[:-1], None, ks[-1], want_xhat=False)
    assert ei.value.code == cspd.E_CAPACITY
    assert "scratch" in cspd.cspd_last_error()
