"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Both sides read the same seeded float32 depth frame.  Validity must agree on
every window; normals, offsets and residuals must agree within the stated
tolerances on every valid window (implicit: every window whose oracle
eigen-condition kappa is at most the gate).  The HD frame is checked on a
seeded sample of pixels plus one full crop, in the launch configuration the
benchmark times (the whole frame is fitted on the GPU).
"""
import numpy as np
import pytest

import oracle
import parity as PT
from depthsynth import camera_for, exact_plane_depth, frames_for
from oracle_pins import EXACT_PLANES, tie_break_frame

pytestmark = pytest.mark.gpu

_frames = {}


def frame(name):
    if name not in _frames:
        _frames[name] = frames_for(name)[0]
    return _frames[name]


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
@pytest.mark.parametrize("k", [3, 5, 15])
def test_exact_planes(gpu, mode, k):
    cam = camera_for(200, 150, 150.0, 160.0, 99.3, 75.1)
    intr = (cam.fx, cam.fy, cam.cx, cam.cy)
    for n, d in EXACT_PLANES:
        n = np.asarray(n) / np.linalg.norm(n)
        z = exact_plane_depth(cam, n, d).astype(np.float32)
        z[~np.isfinite(z)] = 0.0
        _say("exact plane", n, d, k, mode)
        g = PT.gpu_fit(z, intr, k, mode)
        o = oracle.fit_planes(z.astype(np.float64), intr, k, mode)
        rep = PT.check(g, o, mode, z, intr)
        PT.assert_parity(rep)
        # float32 depth of an exact plane: residual at the level of its rounding
        v = o["status"] == 0
        assert np.nanmax(g["residuals"][v]) < 1e-6
        # and the true plane, to the accuracy float32 depth allows
        ang = PT.angle(g["normals"][:, v], n[:, None] * np.ones((1, v.sum())))
        assert ang.max() < 2e-3 / k


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_parity_plain_160x120(gpu, mode):
    f = frame("plain_160x120")
    _say("plain_160x120", mode)
    g = PT.gpu_fit(f.depth, f.intrinsics, 5, mode)
    o = PT.oracle_full(f.depth, f.intrinsics, 5, mode)
    rep = PT.check(g, o, mode, f.depth, f.intrinsics)
    print(rep)
    PT.assert_parity(rep)


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
@pytest.mark.parametrize("k", [3, 5, 9, 15])
def test_parity_vga(gpu, mode, k):
    f = frame("vga_640x480")
    _say("vga_640x480", mode, k)
    g = PT.gpu_fit(f.depth, f.intrinsics, k, mode)
    o = PT.oracle_full(f.depth, f.intrinsics, k, mode)
    rep = PT.check(g, o, mode, f.depth, f.intrinsics)
    print(rep)
    PT.assert_parity(rep)


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
@pytest.mark.parametrize("k", [15, 31])
def test_parity_hd_sampled(gpu, mode, k):
    f = frame("hd_1920x1080")
    H, W = f.depth.shape
    _say("hd_1920x1080", mode, k)
    g = PT.gpu_fit(f.depth, f.intrinsics, k, mode)
    rng = np.random.Generator(np.random.PCG64(100 + k))
    ys = rng.integers(0, H, 12000)
    xs = rng.integers(0, W, 12000)
    # plus a full 48x48 crop at a strip/band seam region, and the image corners
    cy, cx = np.mgrid[500:548, 230:278]
    ys = np.concatenate([ys, cy.ravel(), [0, 0, H - 1, H - 1]])
    xs = np.concatenate([xs, cx.ravel(), [0, W - 1, 0, W - 1]])
    o = oracle.fit_points(f.depth.astype(np.float64), f.intrinsics, k, xs, ys, mode)
    rep = PT.check(g, o, mode, f.depth, f.intrinsics, sel=(ys, xs))
    print(rep)
    PT.assert_parity(rep)


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_fp32_path_validity_and_error_report(gpu, mode):
    """The plain FP32 path is the throughput reference: validity is exact (integer
    counts), its errors against the oracle are reported, not gated."""
    f = frame("vga_640x480")
    for k in (5, 15):
        g = PT.gpu_fit(f.depth, f.intrinsics, k, mode, precision="fp32")
        o = PT.oracle_full(f.depth, f.intrinsics, k, mode)
        rep = PT.check(g, o, mode, f.depth, f.intrinsics)
        print("fp32", mode, k, rep)
        assert rep["invalid_nan"]


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_depth_scaling_bitwise(gpu, mode):
    """Every operation is homogeneous in w = 1/Z: scaling depth by 2^j leaves normals and
    residuals bit-identical and scales offsets by exactly 2^j.  The extreme scales put the
    0.5-6 m frame at 2-23 mm and at 64-768 m, near both ends of the supported depth range
    (1e-3 .. 1e3), so no intermediate of the FP64 sums or solves over- or underflows there."""
    f = frame("vga_640x480")
    base = PT.gpu_fit(f.depth, f.intrinsics, 9, mode)
    for j in (-8, -3, 4, 7):
        _say("depth scale", mode, j)
        s = np.float32(2.0 ** j)
        g = PT.gpu_fit(f.depth * s, f.intrinsics, 9, mode)
        v = (base["status"] & 1) == 0
        assert np.array_equal(g["status"], base["status"])
        assert np.array_equal(g["normals"][:, v], base["normals"][:, v])
        assert np.array_equal(g["residuals"][v], base["residuals"][v])
        assert np.array_equal(g["offsets"][v], base["offsets"][v] * float(s))


def test_determinism(gpu):
    f = frame("vga_640x480")
    a = PT.gpu_fit(f.depth, f.intrinsics, 5, "implicit")
    b = PT.gpu_fit(f.depth, f.intrinsics, 5, "implicit")
    for key in a:
        assert np.array_equal(a[key], b[key], equal_nan=True)


def test_robust_inputs_and_mask(gpu):
    f = frame("plain_160x120")
    z = f.depth.copy()
    z[10, 10] = np.nan
    z[20, 30] = np.inf
    z[40, 50] = -2.0
    z[60, 70] = -0.0
    mask = np.ones(z.shape, np.uint8)
    mask[80:83, 90:92] = 0
    for mode in ("implicit", "explicit"):
        _say("robust", mode)
        g = PT.gpu_fit(z, f.intrinsics, 5, mode, mask_np=mask)
        o = oracle.fit_planes(z.astype(np.float64), f.intrinsics, 5, mode, mask=mask)
        PT.assert_parity(PT.check(g, o, mode, z, f.intrinsics))


def test_all_invalid_and_tiny_frames(gpu):
    intr = (10.0, 10.0, 1.0, 1.0)
    z = np.zeros((40, 40), np.float32)
    g = PT.gpu_fit(z, intr, 3, "implicit")
    assert (g["status"] == 1).all() and np.isnan(g["offsets"]).all()
    # H = W = k: exactly one valid window
    for k in (3, 7, 63):
        cam = camera_for(k, k, 20.0)
        zz = exact_plane_depth(cam, np.array([0.1, 0.2, -0.97]) / np.linalg.norm([0.1, 0.2, -0.97]), 1.0)
        zz = zz.astype(np.float32)
        for mode in ("implicit", "explicit"):
            g = PT.gpu_fit(zz, (cam.fx, cam.fy, cam.cx, cam.cy), k, mode)
            o = oracle.fit_planes(zz.astype(np.float64), (cam.fx, cam.fy, cam.cx, cam.cy), k, mode)
            assert int((g["status"] == 0).sum()) == 1
            PT.assert_parity(PT.check(g, o, mode, zz, (cam.fx, cam.fy, cam.cx, cam.cy)))


def test_pitched_depth_and_ragged_widths(gpu):
    """Depth as a view into a wider buffer (row pitch > W), widths that leave ragged
    last strips, heights that leave ragged last bands."""
    import torch
    import paper_2103_06644_amd as pf
    for (h, w, k) in [(479, 611, 5), (300, 257, 9), (97, 1000, 31), (250, 249, 7)]:
        src = frame("vga_640x480" if w <= 640 else "hd_1920x1080").depth
        sub = np.ascontiguousarray(src[:h, :w])
        wide = torch.zeros((h, w + 37), dtype=torch.float32, device="cuda")
        wide[:, 5:5 + w] = torch.from_numpy(sub).cuda()
        view = wide[:, 5:5 + w]
        intr = (525.0, 525.0, (w - 1) / 2, (h - 1) / 2)
        for mode in ("implicit", "explicit"):
            _say("pitched", h, w, k, mode)
            n, o_, r, s = pf.fit_planes(view, intr, k, mode=mode)
            torch.cuda.synchronize()
            g = dict(normals=n.cpu().numpy().astype(np.float64),
                     offsets=o_.cpu().numpy().astype(np.float64),
                     residuals=r.cpu().numpy().astype(np.float64), status=s.cpu().numpy())
            o = oracle.fit_planes(sub.astype(np.float64), intr, k, mode)
            PT.assert_parity(PT.check(g, o, mode, sub, intr))


def test_kappa_flag_marks_ill_conditioned(gpu):
    f = frame("vga_640x480")
    g = PT.gpu_fit(f.depth, f.intrinsics, 3, "implicit", kappa_flag=1e4)
    o = PT.oracle_full(f.depth, f.intrinsics, 3, "implicit")
    v = o["status"] == 0
    flagged = (g["status"] & 2) != 0
    assert not flagged[~v].any()
    # the GPU's kappa estimate tracks the oracle's: decisively conditioned windows agree
    assert not flagged[v & (o["kappa"] < 1e3)].any()
    assert flagged[v & (o["kappa"] > 1e5)].all()


@pytest.mark.parametrize("fx,fy,want", [(64.0, 32.0, (-1.0, 0.0, 0.0)), (32.0, 64.0, (0.0, -1.0, 0.0))])
def test_orientation_tie_break(gpu, fx, fy, want):
    """A window whose best plane passes through the camera centre (d = 0): the
    normal's sign is settled by the tie-break (first non-zero of n_z, n_y, n_x
    negative), as in the oracle.  The 5 x 5 symmetric pattern of depths 1/2
    and 1 sits in a 32-pixel-wide frame of unit depth; every integrand and sum
    is a short dyadic number, so the window's moments are exact on both sides
    and d comes out exactly 0."""
    import paper_2103_06644_amd as pf
    import torch
    pat, _ = tie_break_frame(fx, fy)
    z = np.ones((5, 32), np.float32)
    z[:, 13:18] = pat
    intr = (fx, fy, 15.0, 2.0)
    _say("tie-break", fx, fy)
    g = PT.gpu_fit(z, intr, 5, "implicit")
    o = oracle.fit_planes(z.astype(np.float64), intr, 5, "implicit")
    assert o["status"][2, 15] == 0 and o["offsets"][2, 15] == 0.0
    assert np.array_equal(o["normals"][:, 2, 15], np.array(want))
    assert g["status"][2, 15] == 0
    assert np.array_equal(g["normals"][:, 2, 15], np.array(want)), g["normals"][:, 2, 15]
    assert g["offsets"][2, 15] == 0.0
    # every window of the middle row sees a frame that is symmetric in y, so
    # its plane passes through (or within rounding of) the camera centre; where
    # the oracle's d is only rounding, the sign of (n, d) is not determined by
    # the data and is compared up to sign; everything else is held to parity
    pc = PT.centre_distance(z, intr)
    tie = (o["status"] == 0) & (np.abs(o["offsets"]) <= 1e-9 * pc)
    tie[2, 15] = False
    if tie.any():
        gn, on = g["normals"][:, tie], o["normals"][:, tie]
        ang = PT.angle(gn / np.linalg.norm(gn, axis=0), on)
        assert np.minimum(ang, np.pi - ang).max() <= PT.ANGLE_TOL
        assert np.abs(g["offsets"][tie]).max() <= 1e-6 * pc[tie].max()
    rest = dict(g)
    rest["status"] = g["status"].copy()
    o2 = {key: v.copy() for key, v in o.items()}
    o2["status"][tie] = 1
    rest["status"][tie] = 1
    rest["normals"] = g["normals"].copy()
    rest["normals"][:, tie] = np.nan
    rest["offsets"] = g["offsets"].copy()
    rest["offsets"][tie] = np.nan
    PT.assert_parity(PT.check(rest, o2, "implicit", z, intr))
