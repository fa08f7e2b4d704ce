"""Disparity input (PF_FLAG_DISPARITY): the frame holds D with 1/Z = D * s.

The oracle has no disparity input: it is given the depth Z = 1 / (D s) computed
in FP64 from the same float32 D, which is the fit the flag defines.  The
backward pass returns dL/dD = dL/dZ * dZ/dD with dZ/dD = -1 / (D^2 s), checked
against the autograd reference on that depth.
"""
import numpy as np
import pytest

import parity as PT
from oracle import grad as og
from depthsynth import frames_for
from parity import crop, upstream
import oracle

pytestmark = pytest.mark.gpu

FB = 525.0 * 0.075          # focal length x baseline of a structured-light sensor
SCALE = 1.0 / FB


def _disp(depth):
    d = np.zeros(depth.shape, np.float32)
    ok = np.isfinite(depth) & (depth > 0)
    d[ok] = (FB / depth[ok].astype(np.float64)).astype(np.float32)
    return d


def _depth_of(d):
    z = np.zeros(d.shape, np.float64)
    ok = d > 0
    z[ok] = 1.0 / (d[ok].astype(np.float64) * SCALE)
    return z


def _gpu(d, intr, k, mode, precision="fp64"):
    import torch
    import paper_2103_06644_amd as pf
    t = torch.from_numpy(d).cuda()
    n, o, r, s = pf.fit_planes(t, intr, k, mode=mode, precision=precision, disparity_scale=SCALE)
    torch.cuda.synchronize()
    return dict(normals=n.cpu().numpy().astype(np.float64), offsets=o.cpu().numpy().astype(np.float64),
                residuals=r.cpu().numpy().astype(np.float64), status=s.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "compensated"])
@pytest.mark.parametrize("mode", ["implicit", "explicit"])
@pytest.mark.parametrize("k", [5, 15])
def test_disparity_parity(gpu, k, mode, precision):
    f = frames_for("vga_640x480")[0]
    d = _disp(f.depth)
    z = _depth_of(d)
    print("[case] disparity", k, mode, precision, flush=True)
    g = _gpu(d, f.intrinsics, k, mode, precision)
    o = oracle.fit_planes(z, f.intrinsics, k, mode)
    rep = PT.check(g, o, mode, z, f.intrinsics)
    print(rep, flush=True)
    PT.assert_parity(rep)


def test_disparity_batch_and_backward(gpu):
    import torch
    import paper_2103_06644_amd as pf
    fr = frames_for("diff_8x640x480", limit=3)
    ds = [torch.from_numpy(_disp(f.depth)).cuda() for f in fr]
    intr = fr[0].intrinsics
    batch = pf.fit_planes_batch(ds, intr, [5, 9, 3], disparity_scale=SCALE)
    # each frame alone at the band height the batch ran it with
    heights = pf.batch_band_heights(ds, intr, [5, 9, 3], disparity_scale=SCALE)
    for i, k in enumerate([5, 9, 3]):
        single = pf.fit_planes(ds[i], intr, k, disparity_scale=SCALE, band_height=heights[i])
        for a, b in zip(batch[i], single):
            assert torch.equal(a, b) or torch.allclose(a, b, equal_nan=True, rtol=0, atol=0)
    # backward: dL/dD against the autograd reference on Z = 1/(D s)
    for mode in ("implicit", "explicit"):
        dcrop = _disp(crop(fr[0], 100, 100, 40, 30)[0])
        intr_c = crop(fr[0], 100, 100, 40, 30)[1]
        z = _depth_of(dcrop)
        o = oracle.fit_planes(z, intr_c, 5, mode)
        gn, gd, gr, _ = upstream(o, 3, mode, depth=z, intr=intr_c)
        gn, gd, gr = (a.astype(np.float32) for a in (gn, gd, gr))
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        g = pf.fit_planes_backward(t(dcrop), intr_c, 5, t(gn), t(gd), t(gr), mode=mode,
                                   disparity_scale=SCALE).cpu().numpy().astype(np.float64)
        ref_z = og.depth_gradient(z, intr_c, 5, mode, gn.astype(np.float64), gd.astype(np.float64),
                                  gr.astype(np.float64))
        dd = dcrop.astype(np.float64)
        ref = np.where(dd > 0, ref_z * (-1.0 / (np.where(dd > 0, dd, 1) ** 2 * SCALE)), 0.0)
        err = np.abs(g - ref).max() / np.abs(ref).max()
        print("disparity backward", mode, err, flush=True)
        assert err <= 2e-6
