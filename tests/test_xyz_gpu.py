"""GPU parity of the standard XYZ formulation (pf_fit_planes_xyz, Eq. 3-9)
against the oracle's unweighted XYZ fits, element by element.

Normals, offsets, validity and status are compared with the parity bar of the
RGBD path.  The residual of this entry point is the RMS point-to-plane
distance in the depth unit; its expected value is computed here by brute force
over each window's back-projected points from the oracle's plane.
"""
import numpy as np
import pytest

import oracle
import parity as PT
from depthsynth import frames_for

pytestmark = pytest.mark.gpu

_cache = {}


def _frame(name):
    if name not in _cache:
        _cache[name] = frames_for(name)[0]
    return _cache[name]


def gpu_fit_xyz(depth_np, intrinsics, k, mode, mask_np=None, kappa_flag=0.0):
    import torch
    import paper_2103_06644_amd as pf
    d = torch.from_numpy(np.ascontiguousarray(depth_np, np.float32)).cuda()
    m = None if mask_np is None else torch.from_numpy(np.ascontiguousarray(mask_np, np.uint8)).cuda()
    n, o, r, s = pf.fit_planes_xyz(d, intrinsics, k, m, mode=mode, kappa_flag=kappa_flag)
    torch.cuda.synchronize()
    return dict(normals=n.cpu().numpy().astype(np.float64), offsets=o.cpu().numpy().astype(np.float64),
                residuals=r.cpu().numpy().astype(np.float64), status=s.cpu().numpy())


def metric_residual(depth, intrinsics, k, normals, offsets, ys, xs):
    """RMS over each selected window of n . P_i + d (P_i back-projected, Eq. 1)."""
    fx, fy, cx, cy = intrinsics
    H, W = depth.shape
    r = k // 2
    out = np.full(len(ys), np.nan)
    dy, dx = np.mgrid[-r:r + 1, -r:r + 1]
    for i, (y, x) in enumerate(zip(ys, xs)):
        if y < r or x < r or y >= H - r or x >= W - r:
            continue
        yy, xx = y + dy, x + dx
        z = depth[yy, xx].astype(np.float64)
        P = np.stack([(xx - cx) / fx * z, (yy - cy) / fy * z, z])
        e = np.tensordot(normals[:, i], P, axes=1) + offsets[i]
        out[i] = np.sqrt(np.mean(e * e))
    return out


def _check_residuals(g, o, f, k, n=3000, seed=5):
    H, W = f.depth.shape
    rng = np.random.Generator(np.random.PCG64(seed + k))
    ys, xs = rng.integers(0, H, n), rng.integers(0, W, n)
    ok = o["status"][ys, xs] == 0
    ys, xs = ys[ok], xs[ok]
    exp = metric_residual(f.depth, f.intrinsics, k, o["normals"][:, ys, xs], o["offsets"][ys, xs],
                          ys, xs)
    got = g["residuals"][ys, xs]
    bad = np.abs(got - exp) > 1e-4 * exp + 1e-9
    assert not bad.any(), (int(bad.sum()), got[bad][:5], exp[bad][:5])


def _compare(g, o, f, k, mode, sel=None):
    oo = dict(o)
    oo["residuals"] = g["residuals"] if sel is None else g["residuals"][sel]  # checked separately
    return PT.check(g, oo, mode, f.depth, f.intrinsics, sel=sel)


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
@pytest.mark.parametrize("name,k", [("plain_160x120", 5), ("vga_640x480", 3), ("vga_640x480", 9),
                                    ("vga_640x480", 15)])
def test_xyz_parity_full_frames(gpu, name, k, mode):
    print("[case] xyz", name, k, mode, flush=True)
    f = _frame(name)
    g = gpu_fit_xyz(f.depth, f.intrinsics, k, mode)
    o = PT.oracle_full(f.depth, f.intrinsics, k, "xyz_" + mode)
    rep = _compare(g, o, f, k, mode)
    print(rep, flush=True)
    PT.assert_parity(rep)
    _check_residuals(g, o, f, k)


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_xyz_parity_hd_sampled(gpu, mode):
    f = _frame("hd_1920x1080")
    k = 15
    print("[case] xyz hd", mode, flush=True)
    g = gpu_fit_xyz(f.depth, f.intrinsics, k, mode)
    H, W = f.depth.shape
    rng = np.random.Generator(np.random.PCG64(99))
    ys, xs = rng.integers(0, H, 8000), rng.integers(0, W, 8000)
    o = oracle.fit_points(f.depth.astype(np.float64), f.intrinsics, k, xs, ys, "xyz_" + mode)
    rep = _compare(g, o, f, k, mode, sel=(ys, xs))
    print(rep, flush=True)
    PT.assert_parity(rep)


def test_xyz_mask_and_edges(gpu):
    f = _frame("vga_640x480")
    k = 7
    rng = np.random.Generator(np.random.PCG64(3))
    mask = (rng.random(f.depth.shape) > 0.01).astype(np.uint8)
    for mode in ("implicit", "explicit"):
        g = gpu_fit_xyz(f.depth, f.intrinsics, k, mode, mask_np=mask)
        o = PT.oracle_full(f.depth, f.intrinsics, k, "xyz_" + mode, mask=mask)
        PT.assert_parity(_compare(g, o, f, k, mode))
    # a frame exactly one window large, and an all-invalid one
    z = f.depth[100:107, 200:207]
    intr = (f.intrinsics[0], f.intrinsics[1], f.intrinsics[2] - 200, f.intrinsics[3] - 100)
    g = gpu_fit_xyz(z, intr, 7, "implicit")
    o = oracle.fit_planes(z.astype(np.float64), intr, 7, "xyz_implicit")
    assert np.array_equal((g["status"] & 1) == 0, o["status"] == 0)
    g0 = gpu_fit_xyz(np.zeros((20, 30), np.float32), intr, 5, "explicit")
    assert np.all(g0["status"] == 1) and np.all(np.isnan(g0["normals"]))


def test_xyz_kappa_flag(gpu):
    f = _frame("vga_640x480")
    k = 5
    g = gpu_fit_xyz(f.depth, f.intrinsics, k, "implicit", kappa_flag=50.0)
    o = PT.oracle_full(f.depth, f.intrinsics, k, "xyz_implicit")
    v = o["status"] == 0
    clear = v & ((o["kappa"] < 40) | (o["kappa"] > 60))   # away from the threshold
    assert np.array_equal((g["status"][clear] & 2) != 0, o["kappa"][clear] > 50)
