"""lmmew_roi_uptake_noalloc (static device scratch, no allocation) against
lmmew_roi_uptake (a buffer allocated per call), through the C ABI: bitwise
equal sums on two calls in a row, the second smaller than the first, so the
second reads back only what it wrote over the first call's leftovers; sizes
beyond the static scratch are rejected with EINVAL."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _ctx():
    from paper_2305_17111_amd import Context

    p = synth.SysParams(n=16, pix=4.0, ns=8, nb=16, na=16, windows=(synth.EW1, synth.EW2))
    mu, _, _ = synth.phantom_disk2(p)
    return p, Context(p, torch.from_numpy(np.asarray(mu, np.float32)))


def test_noalloc_matches_allocating_entry_point_on_two_calls():
    from paper_2305_17111_amd import LmmewError

    torch.cuda.set_device(0)
    p, ctx = _ctx()
    Q = p.n * p.n
    rng = np.random.default_rng(5)
    try:
        for nc, nk in ((40, 50), (3, 5)):
            lam = torch.from_numpy(rng.gamma(2.0, 1.0, (nc, Q)).astype(np.float32)).cuda()
            masks = torch.from_numpy((rng.random((nk, Q)) < 0.3).astype(np.uint8)).cuda()
            got = ctx.roi_uptake(lam, masks, noalloc=True)
            ref = ctx.roi_uptake(lam, masks)
            assert got.shape == (nc, nk)
            assert np.array_equal(got, ref), np.abs(got - ref).max()
            # and the sums themselves (FP64 on the host)
            want = lam.cpu().numpy().astype(np.float64) @ masks.cpu().numpy().T.astype(np.float64)
            assert np.allclose(got, want, rtol=1e-12, atol=0)
        # beyond the static scratch: rejected before any device work
        lam = torch.zeros((300, Q), device="cuda")
        masks = torch.zeros((300, Q), device="cuda", dtype=torch.uint8)
        with pytest.raises(LmmewError) as ei:
            ctx.roi_uptake(lam, masks, noalloc=True)
        assert ei.value.status == -1 and "exceeds" in str(ei.value)
    finally:
        ctx.close()
