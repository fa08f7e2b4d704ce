"""Pins of the oracle's literal implicit mode (constraint |(a, b, c, d)| = 1 as
Sec. II-A states it): numpy's eigh of the 4x4 scatter of Eq. 14, exact planes,
and the depth-unit dependence that motivates the |(a, b, c)| = 1 reading."""
import numpy as np

import oracle
from depthsynth import camera_for, exact_plane_depth, frames_for
from oracle_pins import EXACT_PLANES, angle


def test_literal_matches_numpy_eigh():
    f = frames_for("plain_160x120")[0]
    z = f.depth.astype(np.float64)
    fx, fy, cx, cy = f.intrinsics
    k = 7
    rng = np.random.Generator(np.random.PCG64(6))
    xs, ys = rng.integers(3, 157, 400), rng.integers(3, 117, 400)
    o = oracle.fit_points(z, f.intrinsics, k, xs, ys, "implicit_literal")
    checked = 0
    for i, (x0, y0) in enumerate(zip(xs, ys)):
        if o["status"][i]:
            continue
        yy, xx = np.mgrid[y0 - 3:y0 + 4, x0 - 3:x0 + 4]
        zz = z[yy, xx].ravel()
        M = np.stack([((xx - cx) / fx).ravel(), ((yy - cy) / fy).ravel(), np.ones(k * k), 1 / zz], 1)
        ev, V = np.linalg.eigh(M.T @ M)
        a = V[:, 0]
        n = a[:3] / np.linalg.norm(a[:3])
        d = a[3] / np.linalg.norm(a[:3])
        if d < 0:
            n, d = -n, -d
        kap = ev[3] / (ev[1] - ev[0])
        assert angle(o["normals"][:, i:i + 1], n[:, None])[0] <= 1e-13 * kap + 1e-12
        assert abs(o["offsets"][i] - d) <= (1e-13 * kap + 1e-12) * max(d, 1.0)
        assert abs(o["kappa"][i] / kap - 1) <= 1e-6
        checked += 1
    assert checked > 100


def test_literal_exact_planes():
    cam = camera_for(48, 40, 40.0, 44.0, 23.2, 19.7)
    intr = (cam.fx, cam.fy, cam.cx, cam.cy)
    for n, d in EXACT_PLANES:
        n = np.asarray(n, np.float64) / np.linalg.norm(n)
        z = exact_plane_depth(cam, n, d)
        o = oracle.fit_planes(z, intr, 5, "implicit_literal")
        v = o["status"] == 0
        assert v.sum() >= 10
        assert angle(o["normals"][:, v], n[:, None]).max() <= 1e-8
        assert np.abs(o["offsets"][v] / d - 1).max() <= 1e-8


def test_literal_depends_on_the_depth_unit_and_unit_normal_fit_does_not():
    f = frames_for("vga_640x480")[0]
    z = f.depth.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(2))
    xs, ys = rng.integers(10, 630, 2000), rng.integers(10, 470, 2000)
    ref = oracle.fit_points(z, f.intrinsics, 9, xs, ys, "implicit")
    v = (ref["status"] == 0) & (ref["kappa"] < 1e4)   # well-conditioned windows
    assert v.sum() > 500
    for mode, changes in (("implicit_literal", True), ("implicit", False)):
        a = oracle.fit_points(z, f.intrinsics, 9, xs, ys, mode)
        b = oracle.fit_points(z * 1000.0, f.intrinsics, 9, xs, ys, mode)  # metres -> millimetres
        dev = angle(a["normals"][:, v], b["normals"][:, v])
        if changes:
            assert np.median(dev) > 1e-6
        else:
            assert dev.max() < 1e-9
            assert np.allclose(b["offsets"][v], 1000.0 * a["offsets"][v], rtol=1e-9)
