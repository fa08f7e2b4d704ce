"""FP64 CPU oracle for the per-pixel RGBD plane fit (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the HIP product path, and it shares no
code with it.  See pfo_oracle.h for the definitions it implements.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

IMPLICIT = 0
EXPLICIT = 1
IMPLICIT_SCATTER = 2
EXPLICIT_NORMALEQ = 3
XYZ_IMPLICIT = 4
XYZ_EXPLICIT = 5
IMPLICIT_LITERAL = 6

_MODES = {"implicit": IMPLICIT, "explicit": EXPLICIT, "implicit_scatter": IMPLICIT_SCATTER,
          "explicit_normaleq": EXPLICIT_NORMALEQ, "xyz_implicit": XYZ_IMPLICIT,
          "xyz_explicit": XYZ_EXPLICIT, "implicit_literal": IMPLICIT_LITERAL}

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _build.LIB.endswith("libpfo_oracle.so") and os.path.dirname(_build.LIB) == _build.HERE and (
            not os.path.exists(_build.LIB)
            or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    i64, i32, d = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.pfo_fit_planes.argtypes = [_dp, i64, i64, _u8p, d, d, d, d, i32, i32, i32,
                                   _dp, _dp, _dp, _dp, _u8p]
    lib.pfo_fit_planes.restype = ctypes.c_int
    lib.pfo_fit_points.argtypes = [_dp, i64, i64, _u8p, d, d, d, d, i32, i32, _i64p, _i64p,
                                   i64, i32, _dp, _dp, _dp, _dp, _u8p]
    lib.pfo_fit_points.restype = ctypes.c_int
    lib.pfo_fit_planes_partial.argtypes = [_dp, i64, i64, _u8p, d, d, d, d, i32, i32, i32, i32,
                                           _dp, _dp, _dp, _dp, _u8p]
    lib.pfo_fit_planes_partial.restype = ctypes.c_int
    lib.pfo_fit_points_partial.argtypes = [_dp, i64, i64, _u8p, d, d, d, d, i32, i32, i32,
                                           _i64p, _i64p, i64, i32, _dp, _dp, _dp, _dp, _u8p]
    lib.pfo_fit_points_partial.restype = ctypes.c_int
    lib.pfo_fit_rects.argtypes = [_dp, i64, i64, _u8p, d, d, d, d,
                                  ctypes.POINTER(ctypes.c_int32), i64, i32, i32, _dp, _dp, _dp,
                                  _dp, _u8p]
    lib.pfo_fit_rects.restype = ctypes.c_int
    lib.pfo_camera_moments.argtypes = [d, d, d, d, i32, i64, i64, _dp]
    lib.pfo_camera_moments.restype = None
    lib.pfo_window_sums.argtypes = [_dp, i64, i64, _u8p, d, d, d, d, i32, _dp]
    lib.pfo_window_sums.restype = None
    lib.pfo_integral_images.argtypes = [_dp, i64, i64, _u8p, d, d, d, d, _dp]
    lib.pfo_integral_images.restype = None
    lib.pfo_fit_planes_integral.argtypes = [_dp, i64, i64, _u8p, d, d, d, d, i32, i32,
                                            _dp, _dp, _dp, _u8p]
    lib.pfo_fit_planes_integral.restype = ctypes.c_int
    lib.pfo_jacobi3.argtypes = [_dp, _dp, _dp]
    lib.pfo_jacobi3.restype = None
    _lib = lib
    return lib


class using_library:
    """Temporarily route every wrapper call through another build of the oracle
    (used by the tests that check the pins reject deliberately broken builds)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = _lib
        _lib = None
        saved_lib = _build.LIB
        _build.LIB = self.path
        try:
            _load()
        finally:
            _build.LIB = saved_lib
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _prep(depth, mask):
    depth = np.ascontiguousarray(depth, dtype=np.float64)
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mask.shape == depth.shape
    return depth, mask


def _mode(mode):
    return _MODES[mode] if isinstance(mode, str) else int(mode)


def fit_planes(depth, intrinsics, k, mode="implicit", mask=None, threads=0, min_valid=None):
    """Per-pixel k x k window fits over the whole frame (partial windows with at
    least min_valid valid pixels when min_valid is given).

    Returns a dict of FP64 arrays: normals [3,H,W], offsets [H,W], residuals [H,W],
    kappa [H,W] and status uint8 [H,W] (1 = invalid window)."""
    depth, mask = _prep(depth, mask)
    H, W = depth.shape
    fx, fy, cx, cy = map(float, intrinsics)
    out = dict(normals=np.empty((3, H, W)), offsets=np.empty((H, W)),
               residuals=np.empty((H, W)), kappa=np.empty((H, W)),
               status=np.empty((H, W), np.uint8))
    outs = (_ptr(out["normals"]), _ptr(out["offsets"]), _ptr(out["residuals"]),
            _ptr(out["kappa"]), _ptr(out["status"], _u8p))
    if min_valid is None:
        rc = _load().pfo_fit_planes(_ptr(depth), H, W, _ptr(mask, _u8p), fx, fy, cx, cy, int(k),
                                    _mode(mode), int(threads), *outs)
    else:
        rc = _load().pfo_fit_planes_partial(_ptr(depth), H, W, _ptr(mask, _u8p), fx, fy, cx, cy,
                                            int(k), _mode(mode), int(min_valid), int(threads),
                                            *outs)
    if rc != 0:
        raise ValueError("oracle: bad arguments")
    return out


def fit_points(depth, intrinsics, k, xs, ys, mode="implicit", mask=None, threads=0,
               min_valid=None):
    """Fits at the window centres (xs[i], ys[i]) only; arrays of length len(xs)."""
    depth, mask = _prep(depth, mask)
    H, W = depth.shape
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    n = xs.size
    fx, fy, cx, cy = map(float, intrinsics)
    out = dict(normals=np.empty((3, n)), offsets=np.empty(n), residuals=np.empty(n),
               kappa=np.empty(n), status=np.empty(n, np.uint8))
    outs = (_ptr(out["normals"]), _ptr(out["offsets"]), _ptr(out["residuals"]),
            _ptr(out["kappa"]), _ptr(out["status"], _u8p))
    if min_valid is None:
        rc = _load().pfo_fit_points(_ptr(depth), H, W, _ptr(mask, _u8p), fx, fy, cx, cy, int(k),
                                    _mode(mode), _ptr(xs, _i64p), _ptr(ys, _i64p), n,
                                    int(threads), *outs)
    else:
        rc = _load().pfo_fit_points_partial(_ptr(depth), H, W, _ptr(mask, _u8p), fx, fy, cx, cy,
                                            int(k), _mode(mode), int(min_valid), _ptr(xs, _i64p),
                                            _ptr(ys, _i64p), n, int(threads), *outs)
    if rc != 0:
        raise ValueError("oracle: bad arguments")
    return out


def fit_rects(depth, intrinsics, rects, mode="implicit", mask=None, threads=0):
    """Fits to rectangles rects [n, 4] = (x0, y0, w, h); arrays of length n."""
    depth, mask = _prep(depth, mask)
    H, W = depth.shape
    rects = np.ascontiguousarray(rects, dtype=np.int32).reshape(-1, 4)
    n = rects.shape[0]
    fx, fy, cx, cy = map(float, intrinsics)
    out = dict(normals=np.empty((3, n)), offsets=np.empty(n), residuals=np.empty(n),
               kappa=np.empty(n), status=np.empty(n, np.uint8))
    rc = _load().pfo_fit_rects(_ptr(depth), H, W, _ptr(mask, _u8p), fx, fy, cx, cy,
                               rects.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n,
                               _mode(mode), int(threads), _ptr(out["normals"]),
                               _ptr(out["offsets"]), _ptr(out["residuals"]),
                               _ptr(out["kappa"]), _ptr(out["status"], _u8p))
    if rc != 0:
        raise ValueError("oracle: bad arguments")
    return out


def camera_moments(intrinsics, k, x0, y0):
    """[sum u^2, sum u v, sum u, sum v^2, sum v, N] over the window at (x0, y0)."""
    out = np.empty(6)
    fx, fy, cx, cy = map(float, intrinsics)
    _load().pfo_camera_moments(fx, fy, cx, cy, int(k), int(x0), int(y0), _ptr(out))
    return out


def window_sums(depth, intrinsics, k, mask=None):
    """Direct window sums [sum w, sum u w, sum v w, sum w^2, count] -> [5,H,W]."""
    depth, mask = _prep(depth, mask)
    H, W = depth.shape
    out = np.empty((5, H, W))
    fx, fy, cx, cy = map(float, intrinsics)
    _load().pfo_window_sums(_ptr(depth), H, W, _ptr(mask, _u8p), fx, fy, cx, cy, int(k),
                            _ptr(out))
    return out


def integral_images(depth, intrinsics, mask=None):
    """FP64 integral images of the five integrands -> [5, H+1, W+1]."""
    depth, mask = _prep(depth, mask)
    H, W = depth.shape
    out = np.empty((5, H + 1, W + 1))
    fx, fy, cx, cy = map(float, intrinsics)
    _load().pfo_integral_images(_ptr(depth), H, W, _ptr(mask, _u8p), fx, fy, cx, cy, _ptr(out))
    return out


def fit_planes_integral(depth, intrinsics, k, mode="implicit", mask=None):
    """The paper's integral-image method in FP64 (uncentred sums as written)."""
    depth, mask = _prep(depth, mask)
    H, W = depth.shape
    fx, fy, cx, cy = map(float, intrinsics)
    out = dict(normals=np.empty((3, H, W)), offsets=np.empty((H, W)),
               residuals=np.empty((H, W)), status=np.empty((H, W), np.uint8))
    rc = _load().pfo_fit_planes_integral(_ptr(depth), H, W, _ptr(mask, _u8p), fx, fy, cx, cy,
                                         int(k), _mode(mode), _ptr(out["normals"]),
                                         _ptr(out["offsets"]), _ptr(out["residuals"]),
                                         _ptr(out["status"], _u8p))
    if rc != 0:
        raise ValueError("oracle: bad arguments")
    return out


def jacobi3(a):
    """Eigen-decomposition of a symmetric 3x3: (ascending eigenvalues, eigenvector columns)."""
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(9)
    ev, V = np.empty(3), np.empty(9)
    _load().pfo_jacobi3(_ptr(a), _ptr(ev), _ptr(V))
    return ev, V.reshape(3, 3)
