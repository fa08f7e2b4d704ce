"""pf_plan_autotune: the chosen band height and launch shape are among the
candidates, the shared plan is left as it was, and fits with the derived
(tuned) plan stay at parity with the oracle (single and batched launches agree
bit for bit).  Every launch shape is also held to parity directly."""
import numpy as np
import pytest

import parity as PT
from depthsynth import frames_for

pytestmark = pytest.mark.gpu

CANDIDATES = {4, 6, 8, 12, 16, 20, 24, 32, 48, 64}


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_autotune_then_parity(gpu, mode):
    import torch
    import paper_2103_06644_amd as pf
    f = frames_for("vga_640x480")[0]
    k = 9
    d = torch.from_numpy(f.depth).cuda()
    plan = pf.get_plan(f.intrinsics, 480, 640, k, mode, "fp64")
    before = plan.tile_h
    shape_before = plan.shape
    chosen, shape = plan.autotune(d)
    print("autotune", mode, "band height", chosen, "shape", shape, flush=True)
    assert chosen in CANDIDATES and shape in (0, 1, 2)
    assert pf.get_plan(f.intrinsics, 480, 640, k, mode, "fp64") is plan
    assert plan.tile_h == before and plan.shape == shape_before   # never written
    tuned = pf.get_plan(f.intrinsics, 480, 640, k, mode, "fp64", band_height=chosen, shape=shape)
    assert tuned.tile_h == chosen and tuned.shape == shape
    n, o_, r, s = pf.fit_planes(d, f.intrinsics, k, mode=mode, band_height=chosen, shape=shape)
    torch.cuda.synchronize()
    g = dict(normals=n.cpu().numpy().astype(np.float64), offsets=o_.cpu().numpy().astype(np.float64),
             residuals=r.cpu().numpy().astype(np.float64), status=s.cpu().numpy())
    o = PT.oracle_full(f.depth, f.intrinsics, k, mode)
    PT.assert_parity(PT.check(g, o, mode, f.depth, f.intrinsics))
    single = pf.fit_planes(d, f.intrinsics, k, mode=mode)
    batch = pf.fit_planes_batch([d, d], f.intrinsics, [k, 5], mode=mode)[0]
    for a, b in zip(single, batch):
        assert torch.equal(torch.nan_to_num(a.float(), 7.0), torch.nan_to_num(b.float(), 7.0))


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
@pytest.mark.parametrize("shape,bh", [(0, 4), (1, 12), (2, 8), (2, 24)])
def test_every_shape_at_parity(gpu, mode, shape, bh):
    """Each launch shape (4 x 4 at four or two workgroups per CU, 8 x 8 at
    two) on the 640x480 frame at k = 15 and the 1080p frame's samples."""
    import torch
    import paper_2103_06644_amd as pf
    f = frames_for("vga_640x480")[0]
    k = 15
    d = torch.from_numpy(f.depth).cuda()
    print("[case] shape", shape, "band", bh, mode, flush=True)
    n, o_, r, s = pf.fit_planes(d, f.intrinsics, k, mode=mode, band_height=bh, shape=shape)
    torch.cuda.synchronize()
    g = dict(normals=n.cpu().numpy().astype(np.float64), offsets=o_.cpu().numpy().astype(np.float64),
             residuals=r.cpu().numpy().astype(np.float64), status=s.cpu().numpy())
    o = PT.oracle_full(f.depth, f.intrinsics, k, mode)
    PT.assert_parity(PT.check(g, o, mode, f.depth, f.intrinsics))
    # a batch at this shape equals single calls
    batch = pf.fit_planes_batch([d, d], f.intrinsics, [k, 5], mode=mode, band_heights=bh,
                                shape=shape)[0]
    for x, y in zip((n, o_, r, s), batch):
        assert torch.equal(torch.nan_to_num(x.float(), 7.0), torch.nan_to_num(y.float(), 7.0))


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_shapes_zero_and_one_bit_identical(gpu, mode):
    """Launch shapes 0 and 1 share their tiling (4 x 4) and differ only in
    workgroups per CU, so at one band height their outputs are equal bit for
    bit, and the default plan (shape 1 for implicit, 0 for explicit) equals
    the other shape at its own band height."""
    import torch
    import paper_2103_06644_amd as pf
    f = frames_for("vga_640x480")[0]
    d = torch.from_numpy(f.depth).cuda()
    plan = pf.get_plan(f.intrinsics, 480, 640, 9, mode, "fp64")
    assert plan.shape == (1 if mode == "implicit" else 0)
    outs = {}
    for sh in (0, 1):
        outs[sh] = pf.fit_planes(d, f.intrinsics, 9, mode=mode, band_height=plan.tile_h, shape=sh)
    default = pf.fit_planes(d, f.intrinsics, 9, mode=mode)
    torch.cuda.synchronize()
    for a, b, c in zip(outs[0], outs[1], default):
        assert torch.equal(torch.nan_to_num(a.float(), 7.0), torch.nan_to_num(b.float(), 7.0))
        assert torch.equal(torch.nan_to_num(a.float(), 7.0), torch.nan_to_num(c.float(), 7.0))
