"""pf_plan_autotune: the chosen band height is one of the candidates, the
shared plan is left as it was, and fits with the derived (tuned) plan stay at
parity with the oracle (single and batched launches agree bit for bit)."""
import numpy as np
import pytest

import parity as PT
from depthsynth import frames_for

pytestmark = pytest.mark.gpu

CANDIDATES = {4, 6, 8, 12, 16, 24, 32, 48, 64}


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_autotune_then_parity(gpu, mode):
    import torch
    import paper_2103_06644_amd as pf
    f = frames_for("vga_640x480")[0]
    k = 9
    d = torch.from_numpy(f.depth).cuda()
    plan = pf.get_plan(f.intrinsics, 480, 640, k, mode, "fp64")
    before = plan.tile_h
    chosen = plan.autotune(d)
    print("autotune", mode, "band height", chosen, flush=True)
    assert chosen in CANDIDATES
    assert pf.get_plan(f.intrinsics, 480, 640, k, mode, "fp64") is plan
    assert plan.tile_h == before                     # the shared plan is never written
    tuned = pf.get_plan(f.intrinsics, 480, 640, k, mode, "fp64", band_height=chosen)
    assert tuned.tile_h == chosen
    n, o_, r, s = pf.fit_planes(d, f.intrinsics, k, mode=mode, band_height=chosen)
    torch.cuda.synchronize()
    g = dict(normals=n.cpu().numpy().astype(np.float64), offsets=o_.cpu().numpy().astype(np.float64),
             residuals=r.cpu().numpy().astype(np.float64), status=s.cpu().numpy())
    o = PT.oracle_full(f.depth, f.intrinsics, k, mode)
    PT.assert_parity(PT.check(g, o, mode, f.depth, f.intrinsics))
    single = pf.fit_planes(d, f.intrinsics, k, mode=mode)
    batch = pf.fit_planes_batch([d, d], f.intrinsics, [k, 5], mode=mode)[0]
    for a, b in zip(single, batch):
        assert torch.equal(torch.nan_to_num(a.float(), 7.0), torch.nan_to_num(b.float(), 7.0))
