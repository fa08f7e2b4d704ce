"""Batched launches: many frames of mixed sizes and window sizes per kernel launch.

Every frame of a batch must come out bit-identical to the same frame fitted
alone at the band height the batch ran it with (each workgroup does the same
arithmetic whatever else shares its launch; pf_batch_band_heights reports the
heights), and sampled pixels must match the FP64 oracle.  The batch here is a
cut-down version of the 64-frame mixed workload (more than 32 frames, so it
spans two launches)."""
import numpy as np
import pytest

import oracle
import parity as PT
from depthsynth import CONFIGS
from depthsynth.configs import frame_for

pytestmark = pytest.mark.gpu


def _batch_frames(n):
    specs = CONFIGS["batch_mixed_64"]["frames"]
    # interleave sizes: take every frame of the recipe whose index is in a spread set
    idx = sorted(set(np.linspace(0, len(specs) - 1, n).astype(int)))
    return [frame_for(specs[i]) for i in idx]


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_batch_matches_single_and_oracle(gpu, mode):
    import torch
    import paper_2103_06644_amd as pf
    frames = _batch_frames(40)
    assert len(frames) > 32
    print("[case] batch", mode, len(frames), flush=True)
    depths = [torch.from_numpy(f.depth).cuda() for f in frames]
    intr = [f.intrinsics for f in frames]
    ks = [f.window for f in frames]
    outs = pf.fit_planes_batch(depths, intr, ks, mode=mode)
    torch.cuda.synchronize()
    heights = pf.batch_band_heights(depths, intr, ks, mode=mode)
    rng = np.random.Generator(np.random.PCG64(9))
    for i, f in enumerate(frames):
        single = pf.fit_planes(depths[i], intr[i], ks[i], mode=mode, band_height=heights[i])
        torch.cuda.synchronize()
        for a, b in zip(outs[i], single):
            assert torch.equal(torch.nan_to_num(a.float(), nan=-7.0),
                               torch.nan_to_num(b.float(), nan=-7.0)), f"frame {i}"
        if i % 8 == 0:
            H, W = f.depth.shape
            ys = rng.integers(0, H, 3000)
            xs = rng.integers(0, W, 3000)
            o = oracle.fit_points(f.depth.astype(np.float64), f.intrinsics, ks[i], xs, ys, mode)
            g = dict(normals=outs[i][0].cpu().numpy().astype(np.float64),
                     offsets=outs[i][1].cpu().numpy().astype(np.float64),
                     residuals=outs[i][2].cpu().numpy().astype(np.float64),
                     status=outs[i][3].cpu().numpy())
            PT.assert_parity(PT.check(g, o, mode, f.depth, f.intrinsics, sel=(ys, xs)))


def test_batch_with_masks_and_mixed_none(gpu):
    import torch
    import paper_2103_06644_amd as pf
    frames = _batch_frames(6)
    depths = [torch.from_numpy(f.depth).cuda() for f in frames]
    masks = []
    for i, f in enumerate(frames):
        if i % 2:
            m = np.ones(f.depth.shape, np.uint8)
            m[10:20, 30:50] = 0
            masks.append(torch.from_numpy(m).cuda())
        else:
            masks.append(None)
    outs = pf.fit_planes_batch(depths, [f.intrinsics for f in frames], [f.window for f in frames],
                               masks, mode="implicit")
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        mk = None if masks[i] is None else masks[i].cpu().numpy()
        o = oracle.fit_planes(f.depth.astype(np.float64), f.intrinsics, f.window, "implicit",
                              mask=mk)
        g = dict(normals=outs[i][0].cpu().numpy().astype(np.float64),
                 offsets=outs[i][1].cpu().numpy().astype(np.float64),
                 residuals=outs[i][2].cpu().numpy().astype(np.float64),
                 status=outs[i][3].cpu().numpy())
        PT.assert_parity(PT.check(g, o, "implicit", f.depth, f.intrinsics))


@pytest.mark.parametrize("mode,precision", [("implicit", "fp64"), ("explicit", "fp64"),
                                            ("implicit", "compensated")])
def test_queued_batch_matches_chunked(gpu, mode, precision):
    """The persistent queued launch (all 64 frames of the mixed workload in one
    fit launch) is bit-identical to the chunked launches, hence to single-frame
    calls; oracle samples on a few frames."""
    import torch
    import paper_2103_06644_amd as pf
    frames = _batch_frames(64)
    print("[case] queued batch", mode, precision, len(frames), flush=True)
    depths = [torch.from_numpy(f.depth).cuda() for f in frames]
    intr = [f.intrinsics for f in frames]
    ks = [f.window for f in frames]
    a = pf.fit_planes_batch(depths, intr, ks, mode=mode, precision=precision)
    b = pf.fit_planes_batch(depths, intr, ks, mode=mode, precision=precision, queued=True)
    torch.cuda.synchronize()
    for i in range(len(frames)):
        for x, y in zip(a[i], b[i]):
            assert torch.equal(torch.nan_to_num(x.float(), nan=-7.0),
                               torch.nan_to_num(y.float(), nan=-7.0)), f"frame {i}"
    rng = np.random.Generator(np.random.PCG64(19))
    for i in (0, 31, 63):
        f = frames[i]
        H, W = f.depth.shape
        ys, xs = rng.integers(0, H, 2000), rng.integers(0, W, 2000)
        o = oracle.fit_points(f.depth.astype(np.float64), f.intrinsics, ks[i], xs, ys, mode)
        g = dict(normals=b[i][0].cpu().numpy().astype(np.float64),
                 offsets=b[i][1].cpu().numpy().astype(np.float64),
                 residuals=b[i][2].cpu().numpy().astype(np.float64), status=b[i][3].cpu().numpy())
        PT.assert_parity(PT.check(g, o, mode, f.depth, f.intrinsics, sel=(ys, xs)))


def test_queued_batch_graph_replays(gpu):
    """A queued batch captured in a HIP graph: every replay (with eager work and
    synchronisations between replays) equals the eager result, since each replay
    rewrites the job table and resets the queue counter with kernel nodes."""
    import torch
    import paper_2103_06644_amd as pf
    frames = _batch_frames(40)
    depths = [torch.from_numpy(f.depth).cuda() for f in frames]
    intr = [f.intrinsics for f in frames]
    ks = [f.window for f in frames]
    outs = [(torch.empty((3,) + f.depth.shape, device="cuda"), torch.empty(f.depth.shape, device="cuda"),
             torch.empty(f.depth.shape, device="cuda"),
             torch.empty(f.depth.shape, dtype=torch.uint8, device="cuda")) for f in frames]
    ws = torch.empty(pf.batch_workspace_bytes(len(frames)), dtype=torch.uint8, device="cuda")
    ref = pf.fit_planes_batch(depths, intr, ks, queued=True, workspace=ws)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):   # warm-up on the capture stream
        pf.fit_planes_batch(depths, intr, ks, outs=outs, queued=True, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pf.fit_planes_batch(depths, intr, ks, outs=outs, queued=True, workspace=ws)
    for rep in range(4):
        for o in outs:
            for t in o:
                t.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(frames)):
            for x, y in zip(outs[i], ref[i]):
                assert torch.equal(torch.nan_to_num(x.float(), nan=-7.0),
                                   torch.nan_to_num(y.float(), nan=-7.0)), f"replay {rep} frame {i}"
