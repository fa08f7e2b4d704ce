"""The allocation-free queued batch (pf_fit_planes_batch_queued_noalloc), called
through the C ABI, against the queued batch with a caller's workspace: two
calls in a row, the second with fewer and smaller frames, each bit-identical
to the workspace entry point's output (the static scratch keeps the previous
call's table, which the second call must fully replace)."""
import ctypes

import numpy as np
import pytest

import parity as PT
from depthsynth import CONFIGS
from depthsynth.configs import frame_for

pytestmark = pytest.mark.gpu


def _frames(idx):
    specs = CONFIGS["batch_mixed_64"]["frames"]
    return [frame_for(specs[i]) for i in idx]


def _same(a, b):
    import torch
    return all(torch.equal(torch.nan_to_num(x.float(), nan=-7.0), torch.nan_to_num(y.float(), nan=-7.0))
               for oa, ob in zip(a, b) for x, y in zip(oa, ob))


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_noalloc_matches_workspace_queue(gpu, mode):
    import torch
    import paper_2103_06644_amd as pf
    lib = pf.load_library()
    assert lib.pf_batch_noalloc_max_frames() == 256
    # both calls take the queue (more than 32 frames); the second has fewer and
    # smaller frames (320x240 and 640x480 only), so its job table and item
    # count are smaller than what the scratch still holds from the first
    calls = [list(range(0, 64, 2)) + [1, 3, 33, 57, 61, 63, 40, 41, 43, 45, 47, 49, 51, 53, 55, 59],
             list(range(1, 56, 2)) + [0, 2, 4, 6, 8, 10]]
    for c, idx in enumerate(calls):
        frames = _frames(idx)
        print("[case] no-alloc queued batch", mode, "call", c, len(frames), "frames", flush=True)
        depths = [torch.from_numpy(f.depth).cuda() for f in frames]
        intr = [f.intrinsics for f in frames]
        ks = [f.window for f in frames]
        ref = pf.fit_planes_batch(depths, intr, ks, mode=mode, queued=True)
        got = pf.fit_planes_batch(depths, intr, ks, mode=mode, queued=True, workspace="static")
        torch.cuda.synchronize()
        assert _same(ref, got), f"call {c}"
        # and against the oracle on samples of the first frame
        f = frames[0]
        rng = np.random.Generator(np.random.PCG64(3 + c))
        H, W = f.depth.shape
        ys, xs = rng.integers(0, H, 1500), rng.integers(0, W, 1500)
        import oracle
        o = oracle.fit_points(f.depth.astype(np.float64), f.intrinsics, ks[0], xs, ys, mode)
        g = dict(normals=got[0][0].cpu().numpy().astype(np.float64),
                 offsets=got[0][1].cpu().numpy().astype(np.float64),
                 residuals=got[0][2].cpu().numpy().astype(np.float64), status=got[0][3].cpu().numpy())
        PT.assert_parity(PT.check(g, o, mode, f.depth, f.intrinsics, sel=(ys, xs)))


def test_noalloc_rejects_too_many_frames(gpu):
    """257 frames: refused on the host before anything is enqueued."""
    import paper_2103_06644_amd as pf
    from paper_2103_06644_amd._binding import _FrameIO
    lib = pf.load_library()
    plan = pf.get_plan((525.0, 525.0, 31.5, 23.5), 48, 64, 5)
    n = 257
    handles = (ctypes.c_void_p * n)(*([plan.handle.value] * n))
    fake = 0x10000
    ios = (_FrameIO * n)(*[_FrameIO(fake, 64, None, 0, fake, fake, fake, None) for _ in range(n)])
    assert lib.pf_fit_planes_batch_queued_noalloc(handles, ios, n, None) == 7
