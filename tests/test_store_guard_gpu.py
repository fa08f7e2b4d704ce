"""Output stores stay inside their buffers: every output plane is followed by
64 sentinel bytes, and fits at 640x480 and 1920x1080 (explicit mode, whose
runs are stored as float4 vectors and one packed status word, and implicit
mode) plus a mixed batch must leave every sentinel untouched.  Status and
normals at the strip seams (the columns where one workgroup's outputs end and
the next one's begin) must agree with the oracle."""
import numpy as np
import pytest

import oracle
import parity as PT
from depthsynth import frames_for

pytestmark = pytest.mark.gpu

GUARD = 64
SENTINEL = 0xA5


def guarded(torch, shape, dtype, dev):
    """A contiguous tensor of `shape` at the start of a buffer followed by GUARD
    sentinel bytes; returns (view, raw bytes)."""
    nbytes = int(np.prod(shape)) * torch.tensor([], dtype=dtype).element_size()
    raw = torch.full((nbytes + GUARD,), SENTINEL, dtype=torch.uint8, device=dev)
    return raw[:nbytes].view(dtype).view(*shape), raw


def guarded_outs(torch, H, W, dev):
    pairs = [guarded(torch, (3, H, W), torch.float32, dev), guarded(torch, (H, W), torch.float32, dev),
             guarded(torch, (H, W), torch.float32, dev), guarded(torch, (H, W), torch.uint8, dev)]
    return tuple(p[0] for p in pairs), [p[1] for p in pairs]


def assert_guards(torch, raws):
    for raw in raws:
        tail = raw[-GUARD:].cpu().numpy()
        assert (tail == SENTINEL).all(), f"a store ran past the end of its output: {tail}"


def seam_columns(W, k):
    tw_max = ((256 - (k - 1)) // 4) * 4
    n_strips = -(-W // tw_max)
    tile_w = (-(-W // n_strips) + 3) // 4 * 4
    cols = set()
    for s in range(1, n_strips):
        cols.update({s * tile_w - 2, s * tile_w - 1, s * tile_w, s * tile_w + 1})
    cols.update({W - 4, W - 3, W - 2, W - 1})
    return sorted(c for c in cols if 0 <= c < W)


def check_seams(g, f, k, mode):
    H, W = f.depth.shape
    cols = seam_columns(W, k)
    rows = np.arange(0, H, max(1, H // 60))
    ys, xs = [a.ravel() for a in np.meshgrid(rows, cols, indexing="ij")]
    o = oracle.fit_points(f.depth.astype(np.float64), f.intrinsics, k, xs, ys, mode)
    sel = (ys, xs)
    got = dict(normals=g[0].cpu().numpy().astype(np.float64), offsets=g[1].cpu().numpy().astype(np.float64),
               residuals=g[2].cpu().numpy().astype(np.float64), status=g[3].cpu().numpy())
    rep = PT.check(got, o, mode, f.depth, f.intrinsics, sel=sel)
    print("seams", W, k, mode, len(cols), "columns", rep, flush=True)
    PT.assert_parity(rep)


@pytest.mark.parametrize("mode", ["explicit", "implicit"])
@pytest.mark.parametrize("name,k", [("vga_640x480", 9), ("hd_1920x1080", 15)])
def test_stores_stay_in_bounds(gpu, name, k, mode):
    import torch
    import paper_2103_06644_amd as pf
    f = frames_for(name)[0]
    H, W = f.depth.shape
    print("[case] guard", name, k, mode, flush=True)
    d = torch.from_numpy(f.depth).to(gpu)
    outs, raws = guarded_outs(torch, H, W, gpu)
    pf.fit_planes(d, f.intrinsics, k, mode=mode, out=outs)
    torch.cuda.synchronize()
    assert_guards(torch, raws)
    check_seams(outs, f, k, mode)


@pytest.mark.parametrize("mode", ["explicit", "implicit"])
def test_batch_stores_stay_in_bounds(gpu, mode):
    import torch
    import paper_2103_06644_amd as pf
    fv = frames_for("vga_640x480")[0]
    fp = frames_for("plain_160x120")[0]
    frames = [fv, fp, fv, fp]
    ks = [3, 5, 15, 7]
    print("[case] guard batch", mode, flush=True)
    depths = [torch.from_numpy(f.depth).to(gpu) for f in frames]
    all_outs, all_raws = [], []
    for f in frames:
        o, r = guarded_outs(torch, *f.depth.shape, gpu)
        all_outs.append(o)
        all_raws += r
    pf.fit_planes_batch(depths, [f.intrinsics for f in frames], ks, mode=mode, outs=all_outs)
    torch.cuda.synchronize()
    assert_guards(torch, all_raws)
    for f, k, o in zip(frames, ks, all_outs):
        single = pf.fit_planes(torch.from_numpy(f.depth).to(gpu), f.intrinsics, k, mode=mode)
        for a, b in zip(o, single):
            assert torch.equal(torch.nan_to_num(a.float(), 7.0), torch.nan_to_num(b.float(), 7.0))
