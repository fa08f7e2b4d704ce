"""Pins of the oracle's partial windows (fits from the valid pixels of a window
when at least min_valid of them exist and they are not collinear).  CPU only."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from depthsynth import frames_for
from oracle_pins import angle


def _frame():
    return frames_for("vga_640x480")[0]


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_min_valid_k2_is_the_full_window_rule(mode):
    f = frames_for("plain_160x120")[0]
    z = f.depth.astype(np.float64)
    a = oracle.fit_planes(z, f.intrinsics, 5, mode)
    b = oracle.fit_planes(z, f.intrinsics, 5, mode, min_valid=25)
    for key in ("normals", "offsets", "residuals", "status"):
        assert np.array_equal(a[key], b[key], equal_nan=True), key


def test_partial_validity_count_rule():
    """Windows are fitted iff at least min_valid pixels are valid (a box count of
    the valid mask, pixels outside the image counting as invalid); the
    collinear exception does not arise on this frame for min_valid >= 10."""
    f = _frame()
    z = f.depth.astype(np.float64)
    k, mv = 9, 40
    o = oracle.fit_planes(z, f.intrinsics, k, "explicit", min_valid=mv)
    valid = (z > 0).astype(np.int64)
    counts = ndimage.correlate(valid, np.ones((k, k), np.int64), mode="constant", cval=0)
    assert np.array_equal(o["status"] == 0, counts >= mv)


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_partial_fits_match_library_routines(mode):
    """On windows with holes: numpy least squares (explicit) and the smallest
    eigenvector of the Schur complement of the literal Eq. 14 scatter built
    over the valid pixels only (implicit)."""
    f = _frame()
    z = f.depth.astype(np.float64)
    fx, fy, cx, cy = f.intrinsics
    k, r, mv = 9, 4, 30
    H, W = z.shape
    o = oracle.fit_planes(z, f.intrinsics, k, mode, min_valid=mv)
    holes = (z == 0)
    partial = (o["status"] == 0) & (ndimage.maximum_filter(holes, size=k, mode="constant") |
                                    (np.arange(W)[None, :] < r) | (np.arange(H)[:, None] < r))
    ys, xs = np.nonzero(partial)
    rng = np.random.Generator(np.random.PCG64(1))
    pick = rng.choice(len(ys), 300, replace=False)
    for y0, x0 in zip(ys[pick], xs[pick]):
        yy, xx = np.mgrid[y0 - r:y0 + r + 1, x0 - r:x0 + r + 1]
        inside = (yy >= 0) & (xx >= 0) & (yy < H) & (xx < W)
        yy, xx = yy[inside], xx[inside]
        zz = z[yy, xx]
        ok = zz > 0
        yy, xx, zz = yy[ok], xx[ok], zz[ok]
        assert len(zz) >= mv
        u, v, w = (xx - cx) / fx, (yy - cy) / fy, 1 / zz
        if mode == "explicit":
            alpha = np.linalg.lstsq(np.stack([u, v, np.ones_like(u)], 1), w, rcond=None)[0]
            n = -alpha / np.linalg.norm(alpha)
            d = 1 / np.linalg.norm(alpha)
            tol = 1e-8
        else:
            M = np.stack([u, v, np.ones_like(u), w], 1)
            S = M.T @ M
            C = S[:3, :3] - np.outer(S[:3, 3], S[:3, 3]) / S[3, 3]
            ev, V = np.linalg.eigh(C)
            n = V[:, 0]
            d = -(S[:3, 3] @ n) / S[3, 3]
            if d < 0:
                n, d = -n, -d
            tol = 1e-10 * ev[2] / (ev[1] - ev[0]) + 1e-10
        got = o["normals"][:, y0, x0]
        assert angle(got[:, None], n[:, None])[0] <= tol
        assert abs(o["offsets"][y0, x0] - d) <= 1e-8 * d
        e = np.stack([u, v, np.ones_like(u)], 1) @ got + o["offsets"][y0, x0] * w
        assert abs(o["residuals"][y0, x0] - np.sqrt(np.mean(e * e))) <= 1e-12


def test_collinear_valid_pixels_are_not_fitted():
    f = frames_for("plain_160x120")[0]
    z = np.zeros_like(f.depth, dtype=np.float64)
    z[60, 40:60] = 2.0                 # one valid row only
    z[30:40, 100] = 1.5                # one valid column only
    z[80, 10:20] = 1.0
    z[81, 15] = 1.0                    # plus one pixel off that row
    o = oracle.fit_planes(z, f.intrinsics, 7, "implicit", min_valid=5)
    assert np.all(o["status"][55:66, 40:60] == 1)
    assert np.all(o["status"][25:45, 95:106] == 1)
    assert o["status"][80, 15] == 0
    assert oracle.fit_planes(z, f.intrinsics, 7, "explicit", min_valid=5)["status"][80, 15] == 0
