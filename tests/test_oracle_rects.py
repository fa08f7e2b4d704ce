"""Pins of the oracle's fits to arbitrary rectangles (CPU only).

A k x k rectangle is the k x k window (bit-identical); exact planes are
recovered from non-square rectangles; the explicit fit equals numpy's least
squares and the implicit fit the smallest eigenvector of the Schur complement
of the literal 4x4 scatter of Eq. 14 built here; the validity rule holds.
"""
import numpy as np
import pytest

import oracle
from depthsynth import camera_for, exact_plane_depth, frames_for
from oracle_pins import EXACT_PLANES, angle

SHAPES = [(2, 7), (13, 4), (40, 25), (2, 2), (31, 31)]


@pytest.mark.parametrize("mode", ["implicit", "explicit", "xyz_implicit", "xyz_explicit"])
def test_square_rect_is_the_window(mode):
    f = frames_for("plain_160x120")[0]
    z = f.depth.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(4))
    for k in (3, 5, 9):
        xs, ys = rng.integers(0, 160, 300), rng.integers(0, 120, 300)
        o = oracle.fit_points(z, f.intrinsics, k, xs, ys, mode)
        rects = np.stack([xs - k // 2, ys - k // 2, np.full(300, k), np.full(300, k)], 1)
        r = oracle.fit_rects(z, f.intrinsics, rects, mode)
        for key in ("normals", "offsets", "residuals", "status"):
            assert np.array_equal(o[key], r[key], equal_nan=True), (k, key)


def test_exact_planes_on_rectangles():
    cam = camera_for(64, 48, 50.0, 47.0, 30.3, 21.6)
    intr = (cam.fx, cam.fy, cam.cx, cam.cy)
    for n, d in EXACT_PLANES:
        n = np.asarray(n, np.float64) / np.linalg.norm(n)
        z = exact_plane_depth(cam, n, d)
        rects = np.array([(x0, y0, w, h) for (w, h) in SHAPES
                          for (x0, y0) in [(0, 0), (64 - w, 48 - h), (17, 9), (32 - w // 2, 24 - h // 2)]
                          if x0 + w <= 64 and y0 + h <= 48], np.int32)
        seen = np.array([bool((np.isfinite(z[y:y + h, x:x + w]) & (z[y:y + h, x:x + w] > 0)).all())
                         for (x, y, w, h) in rects])   # the plane covers the whole rectangle
        assert seen.sum() >= 3
        for mode in ("implicit", "explicit", "xyz_implicit", "xyz_explicit"):
            o = oracle.fit_rects(z, intr, rects, mode)
            v = o["status"] == 0
            assert np.array_equal(v, seen), mode
            o = {key: val[..., v] for key, val in o.items()}
            assert angle(o["normals"], n[:, None]).max() <= 1e-9, mode
            assert np.abs(o["offsets"] / d - 1).max() <= 1e-9, mode
            assert o["residuals"].max() <= 1e-9, mode


def _design(z, intr, rect):
    fx, fy, cx, cy = intr
    x0, y0, w, h = rect
    yy, xx = np.mgrid[y0:y0 + h, x0:x0 + w]
    zz = z[y0:y0 + h, x0:x0 + w].ravel()
    u = ((xx - cx) / fx).ravel()
    v = ((yy - cy) / fy).ravel()
    return u, v, 1.0 / zz


def test_rect_fits_match_library_routines():
    f = frames_for("vga_640x480")[0]
    z = f.depth.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(8))
    rects = []
    while len(rects) < 60:
        w, h = int(rng.integers(2, 60)), int(rng.integers(2, 60))
        x0, y0 = int(rng.integers(0, 640 - w)), int(rng.integers(0, 480 - h))
        if (z[y0:y0 + h, x0:x0 + w] > 0).all():
            rects.append((x0, y0, w, h))
    rects = np.array(rects, np.int32)
    oe = oracle.fit_rects(z, f.intrinsics, rects, "explicit")
    oi = oracle.fit_rects(z, f.intrinsics, rects, "implicit")
    for i, rect in enumerate(rects):
        u, v, w = _design(z, f.intrinsics, rect)
        A = np.stack([u, v, np.ones_like(u)], 1)
        alpha = np.linalg.lstsq(A, w, rcond=None)[0]
        n_e = -alpha / np.linalg.norm(alpha)
        assert angle(oe["normals"][:, i:i + 1], n_e[:, None])[0] <= 1e-7
        assert abs(oe["offsets"][i] * np.linalg.norm(alpha) - 1) <= 1e-7
        # literal Eq. 14 scatter of [u, v, 1, w], d eliminated
        M = np.stack([u, v, np.ones_like(u), w], 1)
        S = M.T @ M
        C = S[:3, :3] - np.outer(S[:3, 3], S[:3, 3]) / S[3, 3]
        ev, V = np.linalg.eigh(C)
        n_i = V[:, 0]
        d_i = -(S[:3, 3] @ n_i) / S[3, 3]
        if d_i < 0:
            n_i, d_i = -n_i, -d_i
        kappa = ev[2] / (ev[1] - ev[0])
        if kappa < 1e6:
            assert angle(oi["normals"][:, i:i + 1], n_i[:, None])[0] <= 1e-9 * max(kappa, 1) + 1e-12
            assert abs(oi["offsets"][i] - d_i) <= 1e-8 * d_i + 1e-12


def test_rect_validity_rule():
    f = frames_for("vga_640x480")[0]
    z = f.depth.astype(np.float64)
    rects = np.array([(-1, 0, 5, 5), (0, -1, 5, 5), (636, 0, 5, 5), (0, 476, 5, 5), (10, 10, 1, 5),
                      (10, 10, 5, 1), (10, 10, 0, 0), (0, 0, 640, 480)], np.int32)
    o = oracle.fit_rects(z, f.intrinsics, rects, "implicit")
    assert np.all(o["status"] == 1)            # out of the image, too thin, or holes inside
    assert np.all(np.isnan(o["normals"]))
    # a rectangle over a hole is invalid, the same rectangle beside it is not
    ys, xs = np.nonzero(z == 0)
    y, x = int(ys[len(ys) // 2]), int(xs[len(xs) // 2])
    o2 = oracle.fit_rects(z, f.intrinsics, np.array([(x - 1, y - 1, 3, 3)], np.int32), "explicit")
    assert o2["status"][0] == 1
