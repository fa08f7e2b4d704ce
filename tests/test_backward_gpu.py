"""GPU parity of the adjoint (pf_fit_planes_backward) against the FP64
references: the PyTorch-autograd reference of oracle/grad.py element by
element, central finite differences of the C oracle, and the same references
at sampled pixels of full 640x480 frames with the differentiation workload's
loss  L = sum W (1 - n . t) + 0.1 r.

Upstream gradients are kept to well-posed windows (valid, implicit kappa below
1e3, offset away from the sign flip d = 0): elsewhere the outputs are not
differentiable or their derivatives are dominated by conditioning, and the
comparison would measure the reference's FD step rather than the kernel.
"""
import numpy as np
import pytest

import oracle
import parity as PT
from parity import crop, loss_oracle, upstream
from oracle import grad as og
from depthsynth import diff_loss_inputs, frames_for

pytestmark = pytest.mark.gpu

GRAD_RTOL = 2e-6  # |gpu - reference| <= GRAD_RTOL * max |reference| per case

_cache = {}


def _frames():
    if "f" not in _cache:
        _cache["f"] = frames_for("diff_8x640x480", limit=4)
    return _cache["f"]


def gpu_backward(z, intr, k, mode, gn=None, gd=None, gr=None, mask=None):
    import torch
    import paper_2103_06644_amd as pf
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    m = None if mask is None else torch.from_numpy(mask.astype(np.uint8)).to(dev)
    out = pf.fit_planes_backward(t(z), intr, k, t(gn), t(gd), t(gr), m, mode=mode)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def f32_up(gn, gd, gr):
    return (gn.astype(np.float32).astype(np.float64), gd.astype(np.float32).astype(np.float64),
            gr.astype(np.float32).astype(np.float64))


CROPS = [  # (frame, x0, y0, w, h, k)
    (0, 100, 100, 40, 30, 5), (1, 20, 380, 64, 48, 9), (2, 300, 40, 300, 37, 15),
    (3, 600, 0, 40, 44, 3), (0, 0, 0, 33, 41, 9), (1, 250, 250, 90, 70, 7),
]


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
@pytest.mark.parametrize("case", range(len(CROPS)))
def test_backward_matches_autograd_reference(gpu, mode, case):
    fi, x0, y0, w, h, k = CROPS[case]
    print("[case] backward crop", mode, CROPS[case], flush=True)
    z, intr = crop(_frames()[fi], x0, y0, w, h)
    z32 = z.astype(np.float32).astype(np.float64)
    o = oracle.fit_planes(z32, intr, k, mode)
    gn, gd, gr, keep = upstream(o, 100 + case, mode, depth=z32, intr=intr)
    gn, gd, gr = f32_up(gn, gd, gr)
    g = gpu_backward(z32, intr, k, mode, gn, gd, gr)
    ref = og.depth_gradient(z32, intr, k, mode, gn, gd, gr)
    scale = np.abs(ref).max()
    err = np.abs(g - ref)
    print("  keep", int(keep.sum()), "max |g - ref| / max |ref| =", err.max() / scale, flush=True)
    assert scale > 0
    assert np.all(np.isfinite(g))
    assert err.max() <= GRAD_RTOL * scale
    assert np.all(g[~(z32 > 0)] == 0.0)


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_backward_matches_finite_differences(gpu, mode):
    """Independent of the autograd reference: central differences of the C
    oracle's outputs at every pixel of a small crop (step 1e-6 Z)."""
    k = 5
    z, intr = crop(_frames()[0], 100, 100, 18, 14)
    z = z.astype(np.float32).astype(np.float64)
    z[3, 4] = np.nan
    o = oracle.fit_planes(z, intr, k, mode)
    gn, gd, gr, keep = upstream(o, 7, mode, depth=z, intr=intr)
    gn, gd, gr = f32_up(gn, gd, gr)
    g = gpu_backward(z, intr, k, mode, gn, gd, gr)
    fd = np.zeros_like(z)
    for (y, x), zz in np.ndenumerate(z):
        if not np.isfinite(zz):
            continue
        hh = 1e-6 * zz
        zp, zm = z.copy(), z.copy()
        zp[y, x] += hh
        zm[y, x] -= hh
        fd[y, x] = (loss_oracle(zp, intr, k, mode, gn, gd, gr)
                    - loss_oracle(zm, intr, k, mode, gn, gd, gr)) / (2 * hh)
    scale = np.abs(fd).max()
    err = np.abs(g - fd)
    print(mode, "max |g - fd| / max |fd| =", err.max() / scale, flush=True)
    assert err.max() <= 1e-5 * scale
    assert g[3, 4] == 0.0


def _diff_upstream(f, k, mode, seed):
    """The differentiation workload's loss L = sum W (1 - n . t) + 0.1 r, with W
    zeroed outside well-posed windows (decided by the oracle)."""
    H, W = f.depth.shape
    wts, tgt = diff_loss_inputs(H, W, seed)
    o = PT.oracle_full(f.depth, f.intrinsics, k, mode)
    keep = o["status"] == 0
    if mode == "implicit":
        keep &= o["kappa"] < 1e3
    pc = PT.centre_distance(f.depth, f.intrinsics)
    keep &= np.abs(o["offsets"]) > 0.02 * pc
    wk = np.where(keep, wts, 0.0)
    gn = -wk[None] * tgt
    gd = np.zeros((H, W))
    gr = 0.1 * wk
    return f32_up(gn, gd, gr)


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_backward_full_frame_sampled(gpu, mode):
    """Full 640x480 frames, k = 9, in the launch configuration of the bench:
    dL/dZ at 300 seeded pixels per frame against the autograd reference run on
    the (4r+1)^2 neighbourhood that decides it (every window containing the
    pixel lies inside it), plus image corners and edges."""
    k, r = 9, 4
    for fi, f in enumerate(_frames()[:2]):
        print("[case] backward full frame", mode, fi, flush=True)
        H, W = f.depth.shape
        gn, gd, gr = _diff_upstream(f, k, mode, 6000 + fi)
        g = gpu_backward(f.depth.astype(np.float64), f.intrinsics, k, mode, gn, gd, gr)
        assert np.all(np.isfinite(g))
        rng = np.random.Generator(np.random.PCG64(31 + fi))
        pts = list(zip(rng.integers(0, H, 300), rng.integers(0, W, 300)))
        pts += [(0, 0), (H - 1, W - 1), (0, W - 1), (H - 1, 0), (r, r), (H // 2, 2 * r)]
        fx, fy, cx, cy = f.intrinsics
        worst = 0.0
        for (y, x) in pts:
            ya, yb_ = max(0, y - 2 * r), min(H, y + 2 * r + 1)
            xa, xb = max(0, x - 2 * r), min(W, x + 2 * r + 1)
            zc = f.depth[ya:yb_, xa:xb].astype(np.float64)
            ic = (fx, fy, cx - xa, cy - ya)
            ref = og.depth_gradient(zc, ic, k, mode, gn[:, ya:yb_, xa:xb], gd[ya:yb_, xa:xb],
                                    gr[ya:yb_, xa:xb])[y - ya, x - xa]
            # per-pixel scale: the sum of the magnitudes it is made of is not
            # available, so use the frame's gradient scale
            worst = max(worst, abs(g[y, x] - ref))
        scale = np.abs(g).max()
        print("  max |g - ref| / max |g| =", worst / scale, flush=True)
        assert worst <= GRAD_RTOL * scale


def test_autograd_wrapper_matches_direct_call(gpu):
    import torch
    import paper_2103_06644_amd as pf
    f = _frames()[0]
    k = 9
    dev = torch.device("cuda:0")
    H, W = f.depth.shape
    wts, tgt = diff_loss_inputs(H, W, 6000)
    z = torch.from_numpy(f.depth).to(dev).requires_grad_(True)
    wt = torch.from_numpy(wts.astype(np.float32)).to(dev)
    tt = torch.from_numpy(tgt.astype(np.float32)).to(dev)
    n, d, r, st = pf.fit_planes_differentiable(z, f.intrinsics, k)
    ok = (st == 0).float()
    loss = torch.where(st == 0, wt * (1 - (n * tt).sum(0)) + 0.1 * r, torch.zeros_like(r)).sum()
    loss.backward()
    gn = (-(wt * ok)[None] * tt).contiguous()
    gr = (0.1 * ok).contiguous()
    direct = pf.fit_planes_backward(z.detach(), f.intrinsics, k, gn, None, gr)
    torch.cuda.synchronize()
    a, b = z.grad.cpu().numpy(), direct.cpu().numpy()
    assert np.all(np.isfinite(a))
    assert np.allclose(a, b, rtol=1e-6, atol=1e-6 * np.abs(b).max())


def test_backward_edge_cases(gpu):
    import torch
    import paper_2103_06644_amd as pf
    f = _frames()[1]
    k = 7
    z, intr = crop(f, 200, 120, 50, 40)
    z = z.astype(np.float32).astype(np.float64)
    o = oracle.fit_planes(z, intr, k, "implicit")
    gn, gd, gr, keep = upstream(o, 5, "implicit", depth=z, intr=intr)
    gn, gd, gr = f32_up(gn, gd, gr)
    # no upstream gradient at all: zero everywhere
    assert np.all(gpu_backward(z, intr, k, "implicit") == 0.0)
    # NaN upstream at invalid windows is ignored
    base = gpu_backward(z, intr, k, "implicit", gn, gd, gr)
    inval = o["status"] != 0
    gn2, gd2 = gn.copy(), gd.copy()
    gn2[:, inval] = np.nan
    gd2[inval] = np.nan
    assert np.array_equal(gpu_backward(z, intr, k, "implicit", gn2, gd2, gr), base)
    # a masked pixel is the same as a hole
    mask = np.ones(z.shape, bool)
    mask[20, 25] = False
    zh = z.copy()
    zh[20, 25] = np.nan
    oh = oracle.fit_planes(zh, intr, k, "implicit")
    gnh, gdh, grh, _ = upstream(oh, 5, "implicit", depth=z, intr=intr)
    gnh, gdh, grh = f32_up(gnh, gdh, grh)
    gm = gpu_backward(z, intr, k, "implicit", gnh, gdh, grh, mask=mask)
    gh = gpu_backward(zh, intr, k, "implicit", gnh, gdh, grh)
    assert np.array_equal(gm, gh)
    assert gm[20, 25] == 0.0
    ref = og.depth_gradient(zh, intr, k, "implicit", gnh, gdh, grh)
    assert np.abs(gm - ref).max() <= GRAD_RTOL * np.abs(ref).max()
    # all-invalid frame and a frame exactly one window large
    zero = np.zeros((16, 16))
    assert np.all(gpu_backward(zero, intr, 5, "explicit", np.ones((3, 16, 16)), np.ones((16, 16)),
                               np.ones((16, 16))) == 0.0)
    zt, it = crop(f, 210, 130, k, k)
    zt = zt.astype(np.float32).astype(np.float64)
    ot = oracle.fit_planes(zt, it, k, "explicit")
    assert (ot["status"] == 0).sum() == 1
    gt = gpu_backward(zt, it, k, "explicit", np.ones((3, k, k)), np.ones((k, k)), np.ones((k, k)))
    rt = og.depth_gradient(zt, it, k, "explicit", np.ones((3, k, k)), np.ones((k, k)),
                           np.ones((k, k)))
    assert np.abs(gt - rt).max() <= GRAD_RTOL * np.abs(rt).max()
    # argument errors surface as exceptions before anything is enqueued
    dev = torch.device("cuda:0")
    zt_d = torch.from_numpy(z.astype(np.float32)).to(dev)
    with pytest.raises(ValueError):
        pf.fit_planes_backward(zt_d, intr, k, torch.zeros((3, 5, 5), device=dev))


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_backward_batch_matches_single_calls(gpu, mode):
    """Frames of mixed size, k and mask in one batched backward: bit-identical
    to one call per frame (same kernels, same per-job arithmetic), and the
    second group of 32 frames lands in its own launch pair."""
    import torch
    import paper_2103_06644_amd as pf
    dev = torch.device("cuda:0")
    fr = _frames()
    specs = [(0, 0, 0, 640, 480, 9), (1, 10, 20, 300, 200, 5), (2, 100, 50, 64, 48, 15),
             (3, 0, 0, 33, 41, 3), (0, 200, 100, 250, 120, 7)]
    specs = (specs * 7)[:34]  # 34 frames: two launch pairs
    depths, intrs, ks, gns, grs, masks = [], [], [], [], [], []
    rng = np.random.Generator(np.random.PCG64(12))
    for i, (fi, x0, y0, w, h, k) in enumerate(specs):
        z, intr = crop(fr[fi], x0, y0, w, h)
        depths.append(torch.from_numpy(z.astype(np.float32)).to(dev))
        intrs.append(intr)
        ks.append(k)
        gns.append(torch.from_numpy(rng.standard_normal((3, h, w)).astype(np.float32)).to(dev))
        grs.append(None if i % 3 == 0 else
                   torch.from_numpy(rng.standard_normal((h, w)).astype(np.float32)).to(dev))
        masks.append(None if i % 2 == 0 else
                     torch.from_numpy((rng.random((h, w)) > 0.02).astype(np.uint8)).to(dev))
    print("[case] backward batch", mode, len(specs), flush=True)
    batch = pf.fit_planes_backward_batch(depths, intrs, ks, gns, None, grs, masks, mode=mode)
    torch.cuda.synchronize()
    for i in range(len(specs)):
        single = pf.fit_planes_backward(depths[i], intrs[i], ks[i], gns[i], None, grs[i], masks[i],
                                        mode=mode)
        torch.cuda.synchronize()
        a, b = batch[i].cpu().numpy(), single.cpu().numpy()
        assert np.array_equal(a, b, equal_nan=True), (i, specs[i])


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_backward_fd_1e4_on_32x24(gpu, mode):
    """The differentiation workload's own check on the GPU adjoint: central
    differences of the C oracle with a 1e-4 m step (FP64) at every pixel of a
    32 x 24 crop, k = 9, for L = sum W (1 - n . t) + 0.1 r.  Bar: the central
    difference's truncation error (Richardson estimate against a 5e-5 m step)
    plus GRAD_RTOL of the largest derivative; the extrapolated difference within
    1e-5."""
    from test_oracle_grad import c5_upstream
    k = 9
    z, intr = crop(_frames()[0], 300, 200, 32, 24)
    z = z.astype(np.float32).astype(np.float64)
    o = oracle.fit_planes(z, intr, k, mode)
    if mode == "explicit":
        o.pop("kappa")
    gn, gd, gr, keep = c5_upstream(o, z, intr, 6000)
    gn, gd, gr = f32_up(gn, gd, gr)
    print("[case] backward fd 1e-4 32x24", mode, flush=True)
    g = gpu_backward(z, intr, k, mode, gn, gd, gr)

    def fd(h):
        out = np.zeros_like(z)
        for (y, x), zz in np.ndenumerate(z):
            zp, zm = z.copy(), z.copy()
            zp[y, x] += h
            zm[y, x] -= h
            out[y, x] = (loss_oracle(zp, intr, k, mode, gn, gd, gr)
                         - loss_oracle(zm, intr, k, mode, gn, gd, gr)) / (2 * h)
        return out

    f1, f2 = fd(1e-4), fd(5e-5)
    trunc = np.abs(f1 - f2) * 4.0 / 3.0
    scale = np.abs(f1).max()
    err = np.abs(g - f1)
    print(mode, "max |gpu - fd(1e-4)| / max |fd| =", err.max() / scale, flush=True)
    assert np.all(err <= 1.5 * trunc + GRAD_RTOL * scale)
    assert np.abs(g - (4 * f2 - f1) / 3).max() <= 1e-5 * scale
