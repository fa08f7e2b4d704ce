"""ctypes binding of libplanefit.so (argument marshalling only).

Every step of the fit runs in the HIP kernels of the library; this module only
checks tensor shapes and devices, allocates the outputs through torch and
passes raw device pointers and the current HIP stream across the C ABI
declared in include/planefit.h.  If the library is missing the calls raise:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplanefit.so")

PF_OK = 0
STATUS_NAMES = {0: "PF_OK", 1: "PF_ERR_NULL", 2: "PF_ERR_SHAPE", 3: "PF_ERR_WINDOW",
                4: "PF_ERR_INTRINSICS", 5: "PF_ERR_PITCH", 6: "PF_ERR_ALIGNMENT",
                7: "PF_ERR_WORKSPACE", 8: "PF_ERR_UNSUPPORTED", 9: "PF_ERR_HIP"}
MODES = {"implicit": 0, "explicit": 1, "implicit_literal": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "compensated": 2}
FLAG_DISPARITY = 1

# status byte bits written per pixel
STATUS_INVALID = 1
STATUS_ILL_CONDITIONED = 2
STATUS_FP64_SOLVE = 4


class PlanefitError(RuntimeError):
    """A pf_* call failed; .code holds the pf_status value."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class PlanefitArgumentError(PlanefitError, ValueError):
    pass


class _Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


class _FrameIO(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("depth_pitch", ctypes.c_int64),
                ("mask", ctypes.c_void_p), ("mask_pitch", ctypes.c_int64),
                ("normals", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("residuals", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class _BackwardIO(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("depth_pitch", ctypes.c_int64),
                ("mask", ctypes.c_void_p), ("mask_pitch", ctypes.c_int64),
                ("grad_normals", ctypes.c_void_p), ("grad_offsets", ctypes.c_void_p),
                ("grad_residuals", ctypes.c_void_p), ("grad_depth", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("kappa_flag", ctypes.c_double), ("kappa_fp64", ctypes.c_double),
                ("disparity_scale", ctypes.c_double), ("min_valid", ctypes.c_int32)]


_lib = None
_lib_lock = threading.Lock()

EXPORTS = ("pf_plan_create", "pf_plan_destroy", "pf_plan_workspace_bytes", "pf_plan_autotune",
           "pf_plan_band_height", "pf_plan_derive", "pf_plan_shape",
           "pf_plan_camera_moments", "pf_fit_planes", "pf_fit_planes_batch",
           "pf_batch_workspace_bytes", "pf_fit_planes_batch_queued",
           "pf_fit_planes_batch_queued_noalloc", "pf_batch_noalloc_max_frames",
           "pf_batch_band_heights",
           "pf_backward_workspace_bytes", "pf_fit_planes_backward",
           "pf_fit_planes_backward_batch", "pf_fit_planes_xyz",
           "pf_integral_workspace_bytes", "pf_integral_images", "pf_fit_rects",
           "pf_status_string", "pf_last_hip_error")


def load_library(path: str | None = None):
    """Load libplanefit.so (built by paper_2103_06644_amd.build); raises if absent."""
    global _lib
    with _lib_lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(f"planefit HIP library not built: {p} is missing "
                               "(run `python -m paper_2103_06644_amd.build`)")
        lib = ctypes.CDLL(p)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.pf_plan_create.argtypes = [ctypes.POINTER(_Intrinsics), i64, i64,
                                       ctypes.POINTER(_Params), ctypes.POINTER(vp)]
        lib.pf_plan_create.restype = i32
        lib.pf_plan_destroy.argtypes = [vp]
        lib.pf_plan_destroy.restype = None
        lib.pf_plan_workspace_bytes.argtypes = [vp]
        lib.pf_plan_workspace_bytes.restype = ctypes.c_size_t
        lib.pf_plan_camera_moments.argtypes = [vp, i64, i64, ctypes.POINTER(ctypes.c_double)]
        lib.pf_plan_camera_moments.restype = i32
        lib.pf_fit_planes.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp,
                                      ctypes.c_size_t, vp]
        lib.pf_fit_planes.restype = i32
        lib.pf_fit_planes_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_FrameIO), i32, vp]
        lib.pf_fit_planes_batch.restype = i32
        lib.pf_batch_workspace_bytes.argtypes = [i32]
        lib.pf_batch_workspace_bytes.restype = ctypes.c_size_t
        lib.pf_fit_planes_batch_queued.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_FrameIO), i32,
                                                   vp, ctypes.c_size_t, vp]
        lib.pf_fit_planes_batch_queued.restype = i32
        lib.pf_fit_planes_batch_queued_noalloc.argtypes = [ctypes.POINTER(vp),
                                                           ctypes.POINTER(_FrameIO), i32, vp]
        lib.pf_fit_planes_batch_queued_noalloc.restype = i32
        lib.pf_batch_noalloc_max_frames.argtypes = []
        lib.pf_batch_noalloc_max_frames.restype = i32
        lib.pf_batch_band_heights.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32)]
        lib.pf_batch_band_heights.restype = i32
        lib.pf_plan_band_height.argtypes = [vp]
        lib.pf_plan_band_height.restype = i32
        lib.pf_plan_autotune.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp,
                                         ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.pf_plan_autotune.restype = i32
        lib.pf_plan_derive.argtypes = [vp, i32, i32, ctypes.POINTER(vp)]
        lib.pf_plan_derive.restype = i32
        lib.pf_plan_shape.argtypes = [vp]
        lib.pf_plan_shape.restype = i32
        lib.pf_backward_workspace_bytes.argtypes = [vp]
        lib.pf_backward_workspace_bytes.restype = ctypes.c_size_t
        lib.pf_fit_planes_backward.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp,
                                               ctypes.c_size_t, vp]
        lib.pf_fit_planes_backward.restype = i32
        lib.pf_fit_planes_backward_batch.argtypes = [ctypes.POINTER(vp),
                                                     ctypes.POINTER(_BackwardIO), i32, vp,
                                                     ctypes.c_size_t, vp]
        lib.pf_fit_planes_backward_batch.restype = i32
        lib.pf_integral_workspace_bytes.argtypes = [vp]
        lib.pf_integral_workspace_bytes.restype = ctypes.c_size_t
        lib.pf_integral_images.argtypes = [vp, vp, i64, vp, i64, vp, ctypes.c_size_t, vp]
        lib.pf_integral_images.restype = i32
        lib.pf_fit_rects.argtypes = [vp, vp, ctypes.c_size_t, vp, i64, vp, vp, vp, vp, vp]
        lib.pf_fit_rects.restype = i32
        lib.pf_fit_planes_xyz.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp]
        lib.pf_fit_planes_xyz.restype = i32
        lib.pf_status_string.argtypes = [i32]
        lib.pf_status_string.restype = ctypes.c_char_p
        lib.pf_last_hip_error.argtypes = []
        lib.pf_last_hip_error.restype = ctypes.c_int
        if path is None:
            _lib = lib
        return lib


def status_string(code: int) -> str:
    return load_library().pf_status_string(int(code)).decode()


def _check(code: int):
    if code == PF_OK:
        return
    lib = load_library()
    msg = lib.pf_status_string(code).decode()
    if code == 9:
        raise PlanefitError(code, f"{msg} (hipError_t {lib.pf_last_hip_error()})")
    raise PlanefitArgumentError(code, msg)


class Plan:
    """A pf_plan: camera + frame size + window + mode + precision (host-only object)."""

    def __init__(self, intrinsics, height: int, width: int, window: int,
                 mode: str = "implicit", precision: str = "fp64", kappa_flag: float = 0.0,
                 flags: int = 0, kappa_fp64: float = 0.0, disparity_scale: float = 0.0,
                 min_valid: int = 0):
        lib = load_library()
        fx, fy, cx, cy = (float(v) for v in intrinsics)
        if mode not in MODES:
            raise ValueError(f"mode must be one of {sorted(MODES)}")
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        self._intr = _Intrinsics(fx, fy, cx, cy)
        self._params = _Params(int(window), MODES[mode], PRECISIONS[precision], int(flags),
                               float(kappa_flag), float(kappa_fp64), float(disparity_scale),
                               int(min_valid))
        h = ctypes.c_void_p()
        _check(lib.pf_plan_create(ctypes.byref(self._intr), int(height), int(width),
                                  ctypes.byref(self._params), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.intrinsics = (fx, fy, cx, cy)
        self.height, self.width, self.window = int(height), int(width), int(window)
        self.mode, self.precision, self.kappa_flag = mode, precision, float(kappa_flag)

    @property
    def handle(self):
        return self._h

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.pf_plan_workspace_bytes(self._h))

    @property
    def backward_workspace_bytes(self) -> int:
        return int(self._lib.pf_backward_workspace_bytes(self._h))

    def derive(self, band_height: int = 0, shape: int = -1) -> "Plan":
        """A new plan equal to this one except for its launch shape: band height
        (0 = the rule for the shape) and shape (-1 = keep) (pf_plan_derive);
        this plan is not changed."""
        h = ctypes.c_void_p()
        _check(self._lib.pf_plan_derive(self._h, int(band_height), int(shape), ctypes.byref(h)))
        p = Plan.__new__(Plan)
        p._intr, p._params, p._h, p._lib = self._intr, self._params, h, self._lib
        p.intrinsics, p.height, p.width, p.window = (self.intrinsics, self.height, self.width,
                                                     self.window)
        p.mode, p.precision, p.kappa_flag = self.mode, self.precision, self.kappa_flag
        return p

    def autotune(self, depth, valid_mask=None, stream=None):
        """Time this plan's launch on `depth` (float32 [H, W] on the GPU) for
        every launch shape and band height it offers (pf_plan_autotune) and
        return the fastest as (band_height, shape).  The plan itself is not
        changed: apply the result with derive() or the band_height / shape
        arguments of fit_planes.  Blocks until the timing launches have run."""
        import torch
        _check_depth(torch, depth)
        if tuple(depth.shape) != (self.height, self.width):
            raise ValueError("depth must match the plan's frame size")
        dev = depth.device
        H, W = self.height, self.width
        mptr, mpitch = _mask_arg(torch, valid_mask, depth)
        outs = (torch.empty((3, H, W), dtype=torch.float32, device=dev),
                torch.empty((H, W), dtype=torch.float32, device=dev),
                torch.empty((H, W), dtype=torch.float32, device=dev),
                torch.empty((H, W), dtype=torch.uint8, device=dev))
        chosen, shape = ctypes.c_int32(0), ctypes.c_int32(0)
        with _on_device(torch, dev):
            code = self._lib.pf_plan_autotune(
                self._h, ctypes.c_void_p(depth.data_ptr()), depth.stride(0),
                ctypes.c_void_p(mptr) if mptr else None, mpitch,
                *[ctypes.c_void_p(t.data_ptr()) for t in outs],
                _stream_handle(torch, dev, stream), ctypes.byref(chosen), ctypes.byref(shape))
        _check(code)
        return int(chosen.value), int(shape.value)

    @property
    def shape(self) -> int:
        """Launch shape of this plan's launches (pf_plan_shape)."""
        return int(self._lib.pf_plan_shape(self._h))

    @property
    def tile_h(self) -> int:
        """Output rows per workgroup (band height) of this plan's launches."""
        return int(self._lib.pf_plan_band_height(self._h))

    def camera_moments(self, x0: int, y0: int):
        out = (ctypes.c_double * 6)()
        _check(self._lib.pf_plan_camera_moments(self._h, int(x0), int(y0), out))
        return list(out)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pf_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_plan_cache: dict = {}
_plan_cache_lock = threading.Lock()


def get_plan(intrinsics, height, width, window, mode="implicit", precision="fp64",
             kappa_flag=0.0, disparity_scale=None, min_valid=None, band_height=None,
             shape=None) -> Plan:
    """Cached plan; disparity_scale (1/Z = D * scale) selects disparity input,
    min_valid partial windows, band_height / shape a launch shape other than the
    built-in one (a derived plan, cached under its own key; an explicit band
    height is never raised by the batch planner, see batch_band_heights)."""
    ds = 0.0 if disparity_scale is None else float(disparity_scale)
    mv = 0 if min_valid is None else int(min_valid)
    key = (tuple(float(v) for v in intrinsics), int(height), int(width), int(window), mode,
           precision, float(kappa_flag), ds, mv)
    with _plan_cache_lock:
        p = _plan_cache.get(key)
        if p is None:
            p = Plan(intrinsics, height, width, window, mode, precision, kappa_flag,
                     flags=FLAG_DISPARITY if disparity_scale is not None else 0,
                     disparity_scale=ds, min_valid=mv)
            _plan_cache[key] = p
        bh = 0 if band_height is None else int(band_height)
        sh = -1 if shape is None else int(shape)
        # a band height given explicitly, even the default rule's, is kept by
        # batch launches (a derived plan); 0 leaves it to the batch planner
        if bh == 0 and (sh == -1 or sh == p.shape):
            return p
        dkey = key + (bh, sh)
        d = _plan_cache.get(dkey)
        if d is None:
            d = p.derive(bh, sh)
            _plan_cache[dkey] = d
        return d


def _stream_handle(torch, device, stream):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(int(stream.cuda_stream))


class _on_device:
    """Make `dev` current for the call only when it is not already (cheap path)."""

    def __init__(self, torch, dev):
        self.torch, self.dev, self.ctx = torch, dev, None

    def __enter__(self):
        idx = self.dev.index if self.dev.index is not None else 0
        if self.torch.cuda.current_device() != idx:
            self.ctx = self.torch.cuda.device(self.dev)
            self.ctx.__enter__()
        return self

    def __exit__(self, *exc):
        if self.ctx is not None:
            self.ctx.__exit__(*exc)
        return False


def fit_planes(depth, intrinsics, window: int, valid_mask=None, *, mode: str = "implicit",
               precision: str = "fp64", kappa_flag: float = 0.0, out=None, stream=None,
               disparity_scale=None, min_valid=None, band_height=None, shape=None):
    """Per-pixel plane fits of a depth frame on the GPU.

    depth       float32 tensor [H, W] on a HIP device (unit stride along W)
    intrinsics  (fx, fy, cx, cy) in pixels
    window      odd window size k
    valid_mask  optional uint8/bool tensor [H, W] on the same device (0 = invalid)
    out         optional (normals [3,H,W], offsets [H,W], residuals [H,W], status [H,W])
    disparity_scale  if given, `depth` holds disparity D with 1/Z = D * disparity_scale
    min_valid   if given (3 <= min_valid < k*k), partial windows: a window is fitted
                from its valid pixels when at least min_valid are valid
    band_height, shape  output rows per workgroup and launch shape (e.g. from
                Plan.autotune); None = the plan's built-in launch shape
    Returns (normals, offsets, residuals, status), enqueued on the current stream.
    """
    import torch
    if depth.dim() != 2 or depth.dtype != torch.float32 or depth.device.type != "cuda":
        raise ValueError("depth must be a float32 [H, W] tensor on a HIP device")
    if depth.stride(1) != 1:
        raise ValueError("depth must have unit stride along W")
    H, W = depth.shape
    plan = get_plan(intrinsics, H, W, window, mode, precision, kappa_flag, disparity_scale,
                    min_valid, band_height, shape)
    dev = depth.device
    mptr, mpitch = None, 0
    if valid_mask is not None:
        if valid_mask.shape != depth.shape or valid_mask.device != dev:
            raise ValueError("valid_mask must match depth's shape and device")
        if valid_mask.dtype == torch.bool:
            valid_mask = valid_mask.view(torch.uint8)
        if valid_mask.dtype != torch.uint8 or valid_mask.stride(1) != 1:
            raise ValueError("valid_mask must be uint8/bool with unit stride along W")
        mptr, mpitch = valid_mask.data_ptr(), valid_mask.stride(0)
    if out is None:
        normals = torch.empty((3, H, W), dtype=torch.float32, device=dev)
        offsets = torch.empty((H, W), dtype=torch.float32, device=dev)
        residuals = torch.empty((H, W), dtype=torch.float32, device=dev)
        status = torch.empty((H, W), dtype=torch.uint8, device=dev)
    else:
        _check_outs(torch, out, H, W, dev)
        normals, offsets, residuals, status = out
    ws = plan.workspace_bytes
    work = torch.empty(ws, dtype=torch.uint8, device=dev) if ws else None
    with _on_device(torch, dev):
        code = plan._lib.pf_fit_planes(
            plan.handle, ctypes.c_void_p(depth.data_ptr()), depth.stride(0),
            ctypes.c_void_p(mptr) if mptr else None, mpitch,
            ctypes.c_void_p(normals.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
            ctypes.c_void_p(residuals.data_ptr()), ctypes.c_void_p(status.data_ptr()),
            ctypes.c_void_p(work.data_ptr()) if work is not None else None, ws,
            _stream_handle(torch, dev, stream))
    _check(code)
    return normals, offsets, residuals, status


def fit_planes_xyz(depth, intrinsics, window: int, valid_mask=None, *, mode: str = "implicit",
                   kappa_flag: float = 0.0, out=None, stream=None):
    """The standard XYZ formulation of the same per-pixel fits (nine
    depth-dependent window sums instead of four), for comparison; FP64.
    Same arguments and outputs as fit_planes, except that residuals are RMS
    point-to-plane distances in the depth unit."""
    import torch
    _check_depth(torch, depth)
    H, W = depth.shape
    dev = depth.device
    plan = get_plan(intrinsics, H, W, window, mode, "fp64", kappa_flag)
    mptr, mpitch = _mask_arg(torch, valid_mask, depth)
    if out is None:
        out = (torch.empty((3, H, W), dtype=torch.float32, device=dev),
               torch.empty((H, W), dtype=torch.float32, device=dev),
               torch.empty((H, W), dtype=torch.float32, device=dev),
               torch.empty((H, W), dtype=torch.uint8, device=dev))
    _check_outs(torch, out, H, W, dev)
    normals, offsets, residuals, status = out
    with _on_device(torch, dev):
        code = plan._lib.pf_fit_planes_xyz(
            plan.handle, ctypes.c_void_p(depth.data_ptr()), depth.stride(0),
            ctypes.c_void_p(mptr) if mptr else None, mpitch,
            ctypes.c_void_p(normals.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
            ctypes.c_void_p(residuals.data_ptr()), ctypes.c_void_p(status.data_ptr()),
            _stream_handle(torch, dev, stream))
    _check(code)
    return normals, offsets, residuals, status


def integral_images(depth, intrinsics, valid_mask=None, *, mode="implicit", kappa_flag=0.0,
                    workspace=None, stream=None):
    """FP64 integral images of one frame on the GPU (Sec. II-C), for
    fit_rects.  Returns the workspace tensor that holds them."""
    import torch
    _check_depth(torch, depth)
    H, W = depth.shape
    dev = depth.device
    plan = get_plan(intrinsics, H, W, 3 if min(H, W) >= 3 else 1, mode, "fp64", kappa_flag)
    need = int(plan._lib.pf_integral_workspace_bytes(plan.handle))
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    mptr, mpitch = _mask_arg(torch, valid_mask, depth)
    with _on_device(torch, dev):
        code = plan._lib.pf_integral_images(
            plan.handle, ctypes.c_void_p(depth.data_ptr()), depth.stride(0),
            ctypes.c_void_p(mptr) if mptr else None, mpitch,
            ctypes.c_void_p(workspace.data_ptr()), need, _stream_handle(torch, dev, stream))
    _check(code)
    return workspace


def fit_rects(workspace, frame_shape, intrinsics, rects, *, mode="implicit", kappa_flag=0.0,
              out=None, stream=None):
    """Plane fits to rectangles rects (int32 [n, 4] = x0, y0, w, h, on the
    device) from the integral images in `workspace` (see integral_images).
    Returns (normals [3, n], offsets [n], residuals [n], status [n])."""
    import torch
    H, W = (int(v) for v in frame_shape)
    dev = workspace.device
    if rects.dtype != torch.int32 or rects.dim() != 2 or rects.shape[1] != 4 or \
            not rects.is_contiguous() or rects.device != dev:
        raise ValueError("rects must be a contiguous int32 [n, 4] tensor on the workspace's device")
    n = rects.shape[0]
    plan = get_plan(intrinsics, H, W, 3 if min(H, W) >= 3 else 1, mode, "fp64", kappa_flag)
    need = int(plan._lib.pf_integral_workspace_bytes(plan.handle))
    have = workspace.numel() * workspace.element_size()
    if not workspace.is_contiguous() or have < need:
        raise ValueError(f"workspace must be contiguous and hold the integral images of a "
                         f"{H}x{W} frame ({need} bytes; got {have})")
    if out is None:
        out = (torch.empty((3, n), dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.uint8, device=dev))
    if len(out) != 4:
        raise ValueError("out must be (normals, offsets, residuals, status)")
    for t, shp, dt in zip(out, ((3, n), (n,), (n,), (n,)),
                          (torch.float32, torch.float32, torch.float32, torch.uint8)):
        if tuple(t.shape) != shp or t.dtype != dt or not t.is_contiguous() or t.device != dev:
            raise ValueError("out tensors must be contiguous, on the workspace's device, with "
                             "shapes [3,n], [n], [n], [n] (float32 x3, uint8)")
    normals, offsets, residuals, status = out
    if n == 0:
        return out
    with _on_device(torch, dev):
        code = plan._lib.pf_fit_rects(
            plan.handle, ctypes.c_void_p(workspace.data_ptr()), have,
            ctypes.c_void_p(rects.data_ptr()),
            n, ctypes.c_void_p(normals.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
            ctypes.c_void_p(residuals.data_ptr()), ctypes.c_void_p(status.data_ptr()),
            _stream_handle(torch, dev, stream))
    _check(code)
    return out


def _check_outs(torch, out, H, W, dev):
    """out = (normals [3,H,W], offsets [H,W], residuals [H,W], status [H,W]):
    float32 / uint8, contiguous, on `dev` (the kernels write these shapes)."""
    if len(out) != 4:
        raise ValueError("out must be (normals, offsets, residuals, status)")
    for t, shp, dt in zip(out, ((3, H, W), (H, W), (H, W), (H, W)),
                          (torch.float32, torch.float32, torch.float32, torch.uint8)):
        if tuple(t.shape) != shp or t.dtype != dt or not t.is_contiguous() or t.device != dev:
            raise ValueError("out tensors must be contiguous, on depth's device, with "
                             "shapes [3,H,W], [H,W], [H,W], [H,W] (float32 x3, uint8)")


def _check_depth(torch, depth):
    if depth.dim() != 2 or depth.dtype != torch.float32 or depth.device.type != "cuda":
        raise ValueError("depth must be a float32 [H, W] tensor on a HIP device")
    if depth.stride(1) != 1:
        raise ValueError("depth must have unit stride along W")


def _mask_arg(torch, valid_mask, depth):
    if valid_mask is None:
        return None, 0
    if valid_mask.shape != depth.shape or valid_mask.device != depth.device:
        raise ValueError("valid_mask must match depth's shape and device")
    if valid_mask.dtype == torch.bool:
        valid_mask = valid_mask.view(torch.uint8)
    if valid_mask.dtype != torch.uint8 or valid_mask.stride(1) != 1:
        raise ValueError("valid_mask must be uint8/bool with unit stride along W")
    return valid_mask.data_ptr(), valid_mask.stride(0)


def fit_planes_batch(depths, intrinsics, windows, valid_masks=None, *, mode="implicit",
                     precision="fp64", kappa_flag=0.0, outs=None, stream=None,
                     disparity_scale=None, min_valid=None, queued=False, workspace=None,
                     band_heights=None, shape=None):
    """Per-pixel plane fits of several frames (any sizes, per-frame window sizes)
    in as few kernel launches as possible: up to 32 frames per launch, or with
    queued=True all frames in one persistent launch fed by a work queue
    (pf_fit_planes_batch_queued; `workspace` optionally a uint8 device tensor of
    at least pf_batch_workspace_bytes(n) bytes, 256-byte aligned, else one is
    allocated).  workspace="static" uses the library's own static device
    scratch instead (pf_fit_planes_batch_queued_noalloc: no device allocation;
    at most pf_batch_noalloc_max_frames() frames; calls on one GPU must not
    overlap in time).

    depths       list of float32 [H_i, W_i] tensors on one HIP device
    intrinsics   one (fx, fy, cx, cy) for all frames, or a list of them
    windows      one odd k for all frames, or a list of them
    valid_masks  None or a list of (uint8/bool tensor or None)
    min_valid    None, one value for all frames, or a list of them (partial
                 windows; the frames must be all partial or all full-window)
    band_heights None, one band height for all frames, or a list of them (e.g.
                 each frame's Plan.autotune result); shape: one launch shape
                 for all frames (None = the plans' own, which must agree)
    outs         optional list of (normals, offsets, residuals, status) per frame
    Returns the list of (normals, offsets, residuals, status).
    """
    import torch
    n = len(depths)
    if n == 0:
        return []
    masks = list(valid_masks) if valid_masks is not None else [None] * n
    if len(masks) != n:
        raise ValueError("per-frame argument lists must have one entry per frame")
    for d in depths:
        _check_depth(torch, d)
    plans = _batch_plans([tuple(d.shape) for d in depths], intrinsics, windows, mode, precision,
                         kappa_flag, disparity_scale, min_valid, band_heights, shape)
    dev = depths[0].device
    ios, results, keep = (_FrameIO * n)(), [], []
    for i, d in enumerate(depths):
        if d.device != dev:
            raise ValueError("all frames must be on one device")
        H, W = d.shape
        mptr, mpitch = _mask_arg(torch, masks[i], d)
        if outs is None:
            o = (torch.empty((3, H, W), dtype=torch.float32, device=dev),
                 torch.empty((H, W), dtype=torch.float32, device=dev),
                 torch.empty((H, W), dtype=torch.float32, device=dev),
                 torch.empty((H, W), dtype=torch.uint8, device=dev))
        else:
            o = outs[i]
            _check_outs(torch, o, H, W, dev)
        results.append(o)
        ios[i] = _FrameIO(d.data_ptr(), d.stride(0), mptr, mpitch, o[0].data_ptr(),
                          o[1].data_ptr(), o[2].data_ptr(), o[3].data_ptr())
    handles = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    lib = load_library()
    with _on_device(torch, dev):
        if queued and isinstance(workspace, str):
            if workspace != "static":
                raise ValueError('workspace must be a device tensor, None or "static"')
            code = lib.pf_fit_planes_batch_queued_noalloc(handles, ios, n,
                                                          _stream_handle(torch, dev, stream))
        elif queued:
            need = int(lib.pf_batch_workspace_bytes(n))
            if workspace is None:
                workspace = torch.empty(need, dtype=torch.uint8, device=dev)
            have = workspace.numel() * workspace.element_size()
            if workspace.device != dev or not workspace.is_contiguous() or have < need:
                raise ValueError(f"workspace must be a contiguous device tensor of >= {need} bytes")
            code = lib.pf_fit_planes_batch_queued(handles, ios, n,
                                                  ctypes.c_void_p(workspace.data_ptr()), have,
                                                  _stream_handle(torch, dev, stream))
        else:
            code = lib.pf_fit_planes_batch(handles, ios, n, _stream_handle(torch, dev, stream))
    _check(code)
    return results


def _batch_plans(shapes, intrinsics, windows, mode, precision, kappa_flag, disparity_scale,
                 min_valid, band_heights, shape):
    """The plans of a batch of frames of the given (H, W) shapes."""
    n = len(shapes)
    intr = list(intrinsics) if isinstance(intrinsics[0], (tuple, list)) else [intrinsics] * n
    ks = list(windows) if isinstance(windows, (tuple, list)) else [windows] * n
    mvs = list(min_valid) if isinstance(min_valid, (tuple, list)) else [min_valid] * n
    bhs = list(band_heights) if isinstance(band_heights, (tuple, list)) else [band_heights] * n
    if not (len(intr) == len(ks) == len(mvs) == len(bhs) == n):
        raise ValueError("per-frame argument lists must have one entry per frame")
    return [get_plan(intr[i], H, W, ks[i], mode, precision, kappa_flag, disparity_scale,
                     mvs[i], bhs[i], shape) for i, (H, W) in enumerate(shapes)]


def batch_band_heights(shapes, intrinsics, windows, *, mode="implicit", precision="fp64",
                       kappa_flag=0.0, disparity_scale=None, min_valid=None, band_heights=None,
                       shape=None):
    """Band heights (output rows per workgroup) that fit_planes_batch would run
    each frame of a batch with (pf_batch_band_heights): frames of the given
    (H, W) shapes (or depth tensors), other arguments as in fit_planes_batch.
    Fitting a frame alone with band_height set to its entry reproduces its batch
    outputs bit for bit.  Host only."""
    shapes = [tuple(x.shape) if hasattr(x, "shape") else tuple(x) for x in shapes]
    n = len(shapes)
    if n == 0:
        return []
    plans = _batch_plans(shapes, intrinsics, windows, mode, precision, kappa_flag,
                         disparity_scale, min_valid, band_heights, shape)
    handles = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    out = (ctypes.c_int32 * n)()
    _check(load_library().pf_batch_band_heights(handles, n, out))
    return list(out)


def batch_workspace_bytes(n: int) -> int:
    """Bytes of device workspace a queued batch of n frames needs."""
    return int(load_library().pf_batch_workspace_bytes(int(n)))


def fit_planes_backward(depth, intrinsics, window: int, grad_normals=None, grad_offsets=None,
                        grad_residuals=None, valid_mask=None, *, mode: str = "implicit",
                        out=None, stream=None, disparity_scale=None):
    """Gradient of a scalar loss with respect to the depth image, given the
    loss's gradients with respect to the outputs of fit_planes (each optional,
    float32 [3,H,W] / [H,W] / [H,W] on depth's device).  Differentiated in FP64
    on the GPU; returns dL/dZ as float32 [H, W]."""
    import torch
    _check_depth(torch, depth)
    H, W = depth.shape
    dev = depth.device
    plan = get_plan(intrinsics, H, W, window, mode, "fp64", 0.0, disparity_scale)
    mptr, mpitch = _mask_arg(torch, valid_mask, depth)
    ptrs = []
    for g, shp in ((grad_normals, (3, H, W)), (grad_offsets, (H, W)), (grad_residuals, (H, W))):
        if g is None:
            ptrs.append(None)
            continue
        if (tuple(g.shape) != shp or g.dtype != torch.float32 or not g.is_contiguous()
                or g.device != dev):
            raise ValueError(f"output gradients must be contiguous float32 {shp} on depth's device")
        ptrs.append(ctypes.c_void_p(g.data_ptr()))
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=dev)
    elif (tuple(out.shape) != (H, W) or out.dtype != torch.float32 or not out.is_contiguous()
          or out.device != dev):
        raise ValueError("out must be a contiguous float32 [H, W] tensor on depth's device")
    ws = plan.backward_workspace_bytes
    work = torch.empty(ws, dtype=torch.uint8, device=dev)
    with _on_device(torch, dev):
        code = plan._lib.pf_fit_planes_backward(
            plan.handle, ctypes.c_void_p(depth.data_ptr()), depth.stride(0),
            ctypes.c_void_p(mptr) if mptr else None, mpitch, ptrs[0], ptrs[1], ptrs[2],
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(work.data_ptr()), ws,
            _stream_handle(torch, dev, stream))
    _check(code)
    return out


def _grad_arg(torch, g, shp, dev):
    if g is None:
        return None
    if (tuple(g.shape) != shp or g.dtype != torch.float32 or not g.is_contiguous()
            or g.device != dev):
        raise ValueError(f"output gradients must be contiguous float32 {shp} on depth's device")
    return g.data_ptr()


def fit_planes_backward_batch(depths, intrinsics, windows, grad_normals=None, grad_offsets=None,
                              grad_residuals=None, valid_masks=None, *, mode="implicit",
                              outs=None, stream=None, disparity_scale=None):
    """The backward pass of several frames (any sizes, per-frame k) in two
    launches per 32 frames.  Per-frame lists of output gradients (entries or
    whole lists may be None); returns the list of dL/dZ tensors."""
    import torch
    n = len(depths)
    if n == 0:
        return []
    intr = list(intrinsics) if isinstance(intrinsics[0], (tuple, list)) else [intrinsics] * n
    ks = list(windows) if isinstance(windows, (tuple, list)) else [windows] * n
    lists = [list(x) if x is not None else [None] * n
             for x in (grad_normals, grad_offsets, grad_residuals, valid_masks)]
    if not all(len(x) == n for x in [intr, ks] + lists):
        raise ValueError("per-frame argument lists must have one entry per frame")
    dev = depths[0].device
    plans, ios, results = [], (_BackwardIO * n)(), []
    ws = 0
    for i, d in enumerate(depths):
        _check_depth(torch, d)
        if d.device != dev:
            raise ValueError("all frames must be on one device")
        H, W = d.shape
        p = get_plan(intr[i], H, W, ks[i], mode, "fp64", 0.0, disparity_scale)
        plans.append(p)
        ws += p.backward_workspace_bytes
        mptr, mpitch = _mask_arg(torch, lists[3][i], d)
        out = torch.empty((H, W), dtype=torch.float32, device=dev) if outs is None else outs[i]
        if (tuple(out.shape) != (H, W) or out.dtype != torch.float32 or not out.is_contiguous()
                or out.device != dev):
            raise ValueError("outs must be contiguous float32 [H, W] tensors on depth's device")
        results.append(out)
        ios[i] = _BackwardIO(d.data_ptr(), d.stride(0), mptr, mpitch,
                             _grad_arg(torch, lists[0][i], (3, H, W), dev),
                             _grad_arg(torch, lists[1][i], (H, W), dev),
                             _grad_arg(torch, lists[2][i], (H, W), dev), out.data_ptr())
    work = torch.empty(ws, dtype=torch.uint8, device=dev)
    handles = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    lib = load_library()
    with _on_device(torch, dev):
        code = lib.pf_fit_planes_backward_batch(handles, ios, n, ctypes.c_void_p(work.data_ptr()),
                                                ws, _stream_handle(torch, dev, stream))
    _check(code)
    return results


def _autograd_function():
    import torch

    class FitPlanesFunction(torch.autograd.Function):
        """fit_planes as a differentiable op: forward in the requested
        precision, backward in FP64 through pf_fit_planes_backward."""

        @staticmethod
        def forward(ctx, depth, intrinsics, window, valid_mask, mode, precision):
            n, d, r, st = fit_planes(depth, intrinsics, window, valid_mask, mode=mode,
                                     precision=precision)
            ctx.save_for_backward(depth, valid_mask if valid_mask is not None else depth.new_empty(0))
            ctx.has_mask = valid_mask is not None
            ctx.cfg = (tuple(intrinsics), window, mode)
            ctx.mark_non_differentiable(st)
            return n, d, r, st

        @staticmethod
        def backward(ctx, gn, gd, gr, gst):
            depth, mask = ctx.saved_tensors
            intr, k, mode = ctx.cfg
            prep = lambda g: None if g is None else g.contiguous()
            dz = fit_planes_backward(depth, intr, k, prep(gn), prep(gd), prep(gr),
                                     mask if ctx.has_mask else None, mode=mode)
            return dz, None, None, None, None, None

    return FitPlanesFunction


_fn_cache = []


def fit_planes_differentiable(depth, intrinsics, window: int, valid_mask=None, *,
                              mode: str = "implicit", precision: str = "fp64"):
    """fit_planes with autograd support with respect to `depth`.  Gradients at
    invalid windows are ignored (their outputs are NaN: mask them out of the
    loss, e.g. with torch.where on the status), as are gradients at windows
    whose smallest eigenvalue is repeated."""
    if not _fn_cache:
        _fn_cache.append(_autograd_function())
    return _fn_cache[0].apply(depth, tuple(float(v) for v in intrinsics), int(window),
                              valid_mask, mode, precision)
