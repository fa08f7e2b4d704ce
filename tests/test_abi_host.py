"""Host-only checks of the C ABI (no GPU needed): the library loads and exports
every function include/planefit.h declares, argument validation returns the
documented codes before anything is enqueued, and the plan's closed-form
camera-only moments match the oracle's brute-force window sums."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2103_06644_amd as pf
from paper_2103_06644_amd._binding import _Intrinsics, _Params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "planefit.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = pf.load_library()
    names = declared_functions()
    assert len(names) >= 7
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pf.EXPORTS)


def _create(intr=(525.0, 525.0, 319.5, 239.5), H=480, W=640, k=5, mode=0, prec=0, flags=0,
            kappa=0.0, mv=0):
    lib = pf.load_library()
    h = ctypes.c_void_p()
    code = lib.pf_plan_create(ctypes.byref(_Intrinsics(*intr)), H, W,
                              ctypes.byref(_Params(k, mode, prec, flags, kappa, 0.0, 0.0, mv)),
                              ctypes.byref(h))
    return code, h


@pytest.mark.parametrize("kw,code", [
    (dict(k=4), 3), (dict(k=1), 3), (dict(k=65), 3), (dict(H=4, W=640, k=5), 3),
    (dict(H=0), 2), (dict(W=-3), 2), (dict(H=70000), 2),
    (dict(intr=(0.0, 525.0, 1.0, 1.0)), 4), (dict(intr=(525.0, float("nan"), 1.0, 1.0)), 4),
    (dict(intr=(525.0, 525.0, float("inf"), 1.0)), 4),
    (dict(mode=3), 8), (dict(mode=2, prec=1), 8), (dict(mv=10), 0), (dict(mv=2), 8), (dict(mv=-1), 8),
    (dict(mv=10, prec=2), 8), (dict(mv=10, mode=2), 8), (dict(mv=25, prec=2), 0), (dict(mode=2, kappa=5.0), 8), (dict(mode=2), 0),
    (dict(prec=7), 8), (dict(flags=2), 8), (dict(flags=1), 8), (dict(kappa=-1.0), 8),
    (dict(prec=2), 0),
    (dict(), 0), (dict(H=63, W=63, k=63), 0), (dict(mode=1, prec=1, kappa=1e6), 0),
])
def test_plan_validation(kw, code):
    got, h = _create(**kw)
    assert got == code, pf.status_string(got)
    if code == 0:
        assert h.value
        pf.load_library().pf_plan_destroy(h)
    else:
        assert not h.value


def test_plan_create_null_arguments():
    lib = pf.load_library()
    h = ctypes.c_void_p()
    assert lib.pf_plan_create(None, 10, 10, ctypes.byref(_Params(3, 0, 0, 0, 0.0, 0.0)),
                              ctypes.byref(h)) == 1
    assert lib.pf_plan_create(ctypes.byref(_Intrinsics(1, 1, 1, 1)), 10, 10, None,
                              ctypes.byref(h)) == 1
    lib.pf_plan_destroy(None)


def test_fit_argument_checks_return_before_launch():
    """Only error paths: every call below must be rejected on the host."""
    lib = pf.load_library()
    code, plan = _create(H=48, W=64, k=5)
    assert code == 0
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: the checks return first
    odd = ctypes.c_void_p(0x10001)
    V = ctypes.c_void_p
    call = lambda *a: lib.pf_fit_planes(*a)
    assert call(None, fake, 64, None, 0, fake, fake, fake, None, None, 0, None) == 1
    assert call(plan, None, 64, None, 0, fake, fake, fake, None, None, 0, None) == 1
    assert call(plan, fake, 64, None, 0, None, fake, fake, None, None, 0, None) == 1
    assert call(plan, fake, 63, None, 0, fake, fake, fake, None, None, 0, None) == 5
    assert call(plan, fake, 64, fake, 10, fake, fake, fake, None, None, 0, None) == 5
    assert call(plan, odd, 64, None, 0, fake, fake, fake, None, None, 0, None) == 6
    assert call(plan, fake, 64, None, 0, fake, odd, fake, None, None, 0, None) == 6
    lib.pf_plan_destroy(plan)


def test_status_strings():
    for c in range(10):
        s = pf.status_string(c)
        assert isinstance(s, str) and s
    assert pf.load_library().pf_last_hip_error() == 0


def test_workspace_is_zero_for_fused_path():
    p = pf.Plan((525, 525, 319.5, 239.5), 480, 640, 9)
    assert p.workspace_bytes == 0


@pytest.mark.parametrize("k", [3, 5, 9, 15, 31, 63])
def test_camera_moments_match_oracle_brute_force(k):
    """Row a1: the plan's closed-form camera-only moments equal the oracle's
    brute-force sums of u^2, uv, u, v^2, v, 1 over the window."""
    for intr in [(525.0, 525.0, 319.5, 239.5), (131.25, 140.0, 79.5, 59.5),
                 (1050.0, 1050.0, 959.5, 539.5)]:
        p = pf.Plan(intr, 1080, 1920, k)
        for (x0, y0) in [(0, 0), (k // 2, k // 2), (321, 17), (1919, 1079), (960, 540)]:
            a = np.array(p.camera_moments(x0, y0))
            b = oracle.camera_moments(intr, k, x0, y0)
            scale = np.maximum(np.abs(b), 1.0)
            assert np.all(np.abs(a - b) <= 1e-12 * scale * k * k), (k, intr, x0, y0, a, b)


def test_binding_rejects_bad_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        pf.fit_planes(torch.zeros((8, 8)), (1, 1, 1, 1), 3)  # CPU tensor


def test_batch_argument_checks_return_before_launch():
    from paper_2103_06644_amd._binding import _FrameIO
    lib = pf.load_library()
    c1, p1 = _create(H=48, W=64, k=5, mode=0)
    c2, p2 = _create(H=48, W=64, k=5, mode=1)
    assert c1 == 0 and c2 == 0
    fake = 0x10000
    io = (_FrameIO * 2)(_FrameIO(fake, 64, None, 0, fake, fake, fake, None),
                        _FrameIO(fake, 64, None, 0, fake, fake, fake, None))
    plans = (ctypes.c_void_p * 2)(p1.value, p2.value)
    assert lib.pf_fit_planes_batch(plans, io, 0, None) == 0          # empty batch: no-op
    assert lib.pf_fit_planes_batch(None, io, 2, None) == 1
    assert lib.pf_fit_planes_batch(plans, io, -1, None) == 2
    assert lib.pf_fit_planes_batch(plans, io, 2, None) == 8          # mixed modes
    io[1].depth_pitch = 10
    plans2 = (ctypes.c_void_p * 2)(p1.value, p1.value)
    assert lib.pf_fit_planes_batch(plans2, io, 2, None) == 5         # bad pitch in frame 1
    io[1].depth_pitch = 64
    io[1].normals = None
    assert lib.pf_fit_planes_batch(plans2, io, 2, None) == 1         # NULL output in frame 1
    # partial-window plans batch with each other (any min_valid), not with full-window ones
    # (frame 2's NULL output stops the call on the host should the check let frame 1 pass)
    c3, p3 = _create(H=48, W=64, k=5, mode=0, mv=12)
    assert c3 == 0
    io3 = (_FrameIO * 3)(*[_FrameIO(fake, 64, None, 0, fake, fake, fake, None) for _ in range(3)])
    io3[2].normals = None
    plans3 = (ctypes.c_void_p * 3)(p3.value, p1.value, p3.value)
    assert lib.pf_fit_planes_batch(plans3, io3, 3, None) == 8        # partial with full-window
    lib.pf_plan_destroy(p1)
    lib.pf_plan_destroy(p2)
    lib.pf_plan_destroy(p3)


def test_backward_argument_checks_return_before_launch():
    """Only error paths of pf_fit_planes_backward: all rejected on the host."""
    lib = pf.load_library()
    code, plan = _create(H=48, W=64, k=5)
    assert code == 0
    need = lib.pf_backward_workspace_bytes(plan)
    assert need == 32 * 48 * 64
    assert lib.pf_backward_workspace_bytes(None) == 0
    fake = ctypes.c_void_p(0x10000)
    odd = ctypes.c_void_p(0x10004)   # 4-byte but not 8-byte aligned
    odd1 = ctypes.c_void_p(0x10001)
    call = lambda *a: lib.pf_fit_planes_backward(*a)
    assert call(None, fake, 64, None, 0, None, None, None, fake, fake, need, None) == 1
    assert call(plan, None, 64, None, 0, None, None, None, fake, fake, need, None) == 1
    assert call(plan, fake, 64, None, 0, None, None, None, None, fake, need, None) == 1
    assert call(plan, fake, 63, None, 0, None, None, None, fake, fake, need, None) == 5
    assert call(plan, fake, 64, fake, 3, None, None, None, fake, fake, need, None) == 5
    assert call(plan, odd1, 64, None, 0, None, None, None, fake, fake, need, None) == 6
    assert call(plan, fake, 64, None, 0, odd1, None, None, fake, fake, need, None) == 6
    assert call(plan, fake, 64, None, 0, None, None, None, fake, None, need, None) == 7
    assert call(plan, fake, 64, None, 0, None, None, None, fake, fake, need - 1, None) == 7
    assert call(plan, fake, 64, None, 0, None, None, None, fake, odd, need, None) == 7
    lib.pf_plan_destroy(plan)


def test_xyz_argument_checks_return_before_launch():
    lib = pf.load_library()
    code, plan = _create(H=48, W=64, k=5)
    code32, plan32 = _create(H=48, W=64, k=5, prec=1)
    assert code == 0 and code32 == 0
    fake = ctypes.c_void_p(0x10000)
    odd = ctypes.c_void_p(0x10001)
    call = lambda *a: lib.pf_fit_planes_xyz(*a)
    assert call(None, fake, 64, None, 0, fake, fake, fake, None, None) == 1
    assert call(plan, fake, 64, None, 0, None, fake, fake, None, None) == 1
    assert call(plan32, fake, 64, None, 0, fake, fake, fake, None, None) == 8
    assert call(plan, fake, 60, None, 0, fake, fake, fake, None, None) == 5
    assert call(plan, odd, 64, None, 0, fake, fake, fake, None, None) == 6
    lib.pf_plan_destroy(plan)
    lib.pf_plan_destroy(plan32)


def test_backward_batch_argument_checks_return_before_launch():
    from paper_2103_06644_amd._binding import _BackwardIO
    lib = pf.load_library()
    c1, p1 = _create(H=48, W=64, k=5, mode=0)
    c2, p2 = _create(H=48, W=64, k=5, mode=1)
    assert c1 == 0 and c2 == 0
    fake = 0x10000
    need = 2 * lib.pf_backward_workspace_bytes(p1)
    io = (_BackwardIO * 2)(_BackwardIO(fake, 64, None, 0, None, None, None, fake),
                           _BackwardIO(fake, 64, None, 0, None, None, None, fake))
    same = (ctypes.c_void_p * 2)(p1.value, p1.value)
    mixed = (ctypes.c_void_p * 2)(p1.value, p2.value)
    ws = ctypes.c_void_p(0x20000)
    call = lib.pf_fit_planes_backward_batch
    assert call(same, io, 0, None, 0, None) == 0                  # empty: no-op
    assert call(None, io, 2, ws, need, None) == 1
    assert call(same, io, -1, ws, need, None) == 2
    assert call(mixed, io, 2, ws, need, None) == 8                # mixed modes
    assert call(same, io, 2, ws, need - 8, None) == 7             # workspace for one frame only
    assert call(same, io, 2, None, need, None) == 7
    io[1].depth_pitch = 10
    assert call(same, io, 2, ws, need, None) == 5
    io[1].depth_pitch = 64
    io[1].grad_depth = None
    assert call(same, io, 2, ws, need, None) == 1
    lib.pf_plan_destroy(p1)
    lib.pf_plan_destroy(p2)


def test_rect_argument_checks_return_before_launch():
    lib = pf.load_library()
    code, plan = _create(H=48, W=64, k=5)
    assert code == 0
    need = lib.pf_integral_workspace_bytes(plan)
    # header, five (H+1) x (W+1) planes, column totals of 3 bands of 16 rows,
    # row totals of 1 strip of 256 columns, and the 4 waves' row totals of
    # each of the 3 tiles
    assert need == 8 * (32 + 5 * 49 * 65 + 5 * 3 * 64 + 5 * 1 * 48 + 3 * 1 * 16 * 4 * 5)
    fake = ctypes.c_void_p(0x10000)
    odd = ctypes.c_void_p(0x10004)
    assert lib.pf_integral_images(None, fake, 64, None, 0, fake, need, None) == 1
    assert lib.pf_integral_images(plan, fake, 63, None, 0, fake, need, None) == 5
    assert lib.pf_integral_images(plan, fake, 64, None, 0, fake, need - 1, None) == 7
    assert lib.pf_integral_images(plan, fake, 64, None, 0, odd, need, None) == 7
    assert lib.pf_fit_rects(plan, fake, need, fake, 0, fake, fake, fake, None, None) == 0  # no-op
    assert lib.pf_fit_rects(plan, fake, need, fake, -1, fake, fake, fake, None, None) == 2
    assert lib.pf_fit_rects(plan, None, need, fake, 3, fake, fake, fake, None, None) == 1
    assert lib.pf_fit_rects(plan, fake, need, fake, 3, ctypes.c_void_p(0x10001), fake, fake,
                            None, None) == 6
    # a workspace sized for a smaller frame is refused before anything is read
    assert lib.pf_fit_rects(plan, fake, need - 8, fake, 3, fake, fake, fake, None, None) == 7
    lib.pf_plan_destroy(plan)


def test_disparity_flag_validation():
    lib = pf.load_library()
    for scale, code in ((1.0 / 40.0, 0), (0.0, 8), (-1.0, 8), (float("inf"), 8), (float("nan"), 8)):
        h = ctypes.c_void_p()
        got = lib.pf_plan_create(ctypes.byref(_Intrinsics(525.0, 525.0, 319.5, 239.5)), 48, 64,
                                 ctypes.byref(_Params(5, 0, 0, 1, 0.0, 0.0, scale)), ctypes.byref(h))
        assert got == code, (scale, got)
        if h.value:
            fake = ctypes.c_void_p(0x10000)
            # the XYZ and rectangle paths take depth only
            assert lib.pf_fit_planes_xyz(h, fake, 64, None, 0, fake, fake, fake, None, None) == 8
            assert lib.pf_integral_images(h, fake, 64, None, 0, fake, 1 << 30, None) == 8
            lib.pf_plan_destroy(h)


def test_autotune_argument_checks_return_before_launch():
    lib = pf.load_library()
    code, plan = _create(H=48, W=64, k=5)
    assert code == 0
    fake = ctypes.c_void_p(0x10000)
    chosen, shape = ctypes.c_int32(-1), ctypes.c_int32(-1)
    args = (ctypes.byref(chosen), ctypes.byref(shape))
    assert lib.pf_plan_autotune(None, fake, 64, None, 0, fake, fake, fake, None, None, *args) == 1
    assert lib.pf_plan_autotune(plan, None, 64, None, 0, fake, fake, fake, None, None, *args) == 1
    assert lib.pf_plan_autotune(plan, fake, 60, None, 0, fake, fake, fake, None, None, *args) == 5
    assert chosen.value == -1 and shape.value == -1   # untouched: nothing was launched
    lib.pf_plan_destroy(plan)


@pytest.mark.parametrize("H,W,k,mode,rows", [
    (480, 640, 9, "implicit", 4),      # 3 strips x 480 rows fit one round at the 4-row minimum
    (480, 640, 9, "explicit", 4),      # the 4-row minimum
    (1080, 1920, 15, "implicit", 12),  # 8 strips: 9 rows for one round, rounded up to whole 4-row rounds
    (1080, 1920, 15, "explicit", 12),  # 9 rows -> 12
    (1080, 1920, 31, "explicit", 12),
    (1080, 1920, 31, "implicit", 12),  # 9 strips: 10 rows -> 12
    (720, 1280, 5, "implicit", 8),     # 6 strips: 5 rows -> 8
    (30, 40, 3, "implicit", 4),
    (6, 40, 3, "explicit", 4),
    (3, 40, 3, "explicit", 3),         # never taller than the frame
])
def test_default_band_height_is_whole_rounds(H, W, k, mode, rows):
    """The plan's band height: one round of 1,024 workgroups (four per CU on 256
    CUs, whatever the launch shape's occupancy), at least 4 rows, rounded up to a
    multiple of the kernel's 4-row round and capped at the frame height.  The default launch shape is two workgroups per CU for
    the FP64 implicit fit and four otherwise."""
    p = pf.Plan((525.0, 525.0, W / 2 - 0.5, H / 2 - 0.5), H, W, k, mode)
    assert p.tile_h == rows
    assert p.shape == (1 if mode == "implicit" else 0)


def test_derive_leaves_the_plan_alone():
    """pf_plan_derive makes a new plan with another band height; the source
    plan (shared by every caller of the Python cache) is never written."""
    lib = pf.load_library()
    code, plan = _create(H=480, W=640, k=9)
    assert code == 0
    before = lib.pf_plan_band_height(plan)
    out = ctypes.c_void_p()
    assert lib.pf_plan_derive(plan, 12, -1, ctypes.byref(out)) == 0
    assert lib.pf_plan_band_height(out) == 12
    assert lib.pf_plan_band_height(plan) == before
    assert lib.pf_plan_shape(out) == lib.pf_plan_shape(plan) == 1   # FP64 implicit default
    big = ctypes.c_void_p()
    assert lib.pf_plan_derive(plan, 100000, 2, ctypes.byref(big)) == 0
    assert lib.pf_plan_band_height(big) == 480              # clamped to the frame
    assert lib.pf_plan_shape(big) == 2 and lib.pf_plan_shape(plan) == 1
    rule = ctypes.c_void_p()
    assert lib.pf_plan_derive(plan, 0, 1, ctypes.byref(rule)) == 0   # the shape's own rule
    assert lib.pf_plan_band_height(rule) >= 4
    bad = ctypes.c_void_p(1)
    assert lib.pf_plan_derive(plan, -1, -1, ctypes.byref(bad)) == 2
    assert bad.value is None
    assert lib.pf_plan_derive(plan, 8, 3, ctypes.byref(bad)) == 8
    assert lib.pf_plan_derive(None, 8, -1, ctypes.byref(bad)) == 1
    # shapes 1 and 2 only for FP64 full-window implicit / explicit plans
    code, p32 = _create(H=480, W=640, k=9, prec=1)
    assert lib.pf_plan_derive(p32, 8, 2, ctypes.byref(bad)) == 8
    code, pex = _create(H=480, W=640, k=9, mode=1)
    assert lib.pf_plan_shape(pex) == 0                      # FP64 explicit default
    for h in (out, big, rule, plan, p32, pex):
        lib.pf_plan_destroy(h)


def _groups(H, W, k, th):
    tw_max = ((256 - (k - 1)) // 4) * 4
    return -(-W // tw_max) * -(-H // th)


def test_batch_band_heights():
    """The batch planner (pf_batch_band_heights; host only, 256 CUs here and on
    MI355X): a batch of more workgroups than four per CU gets taller bands,
    largest windows first (equal windows: lowest band first), one 4-row round at
    a time up to 12 rows, until it fits; explicit heights and 8-row-round shapes
    are kept; a frame alone keeps the default rule's height."""
    intr = (525.0, 525.0, 319.5, 239.5)
    vga4 = [(480, 640)] * 4
    for mode in ("implicit", "explicit"):
        # 640x480 at k = 3, 5, 9, 15: 4 x 360 workgroups -> 1020 <= 1024
        h = pf.batch_band_heights(vga4, intr, [3, 5, 9, 15], mode=mode)
        assert h == [4, 4, 8, 12]
        assert sum(_groups(480, 640, k, t) for k, t in zip([3, 5, 9, 15], h)) <= 1024
        # the caller's order does not matter, only the windows
        assert pf.batch_band_heights(vga4, intr, [15, 3, 9, 5], mode=mode) == [12, 4, 8, 4]
        # ties: the lowest band first, then the first frame
        assert pf.batch_band_heights(vga4, intr, [9, 9, 9, 9], mode=mode) == [8, 8, 8, 4]
    # heights given explicitly are kept, even the default rule's own
    assert pf.batch_band_heights(vga4, intr, [3, 5, 9, 15], band_heights=4) == [4, 4, 4, 4]
    assert pf.batch_band_heights(vga4, intr, [3, 5, 9, 15],
                                 band_heights=[None, None, 4, None]) == [4, 8, 4, 12]
    # the 8 x 8 shape (8-row rounds) keeps its own rule, and so do the FP32,
    # compensated, partial-window and literal fits
    assert pf.batch_band_heights(vga4, intr, [3, 5, 9, 15], shape=2) == [8, 8, 8, 8]
    for kw in (dict(precision="fp32"), dict(precision="compensated"), dict(min_valid=5),
               dict(mode="implicit_literal")):
        assert pf.batch_band_heights(vga4, intr, [3, 5, 9, 15], **kw) == [4, 4, 4, 4], kw
    # alone, or a batch that fits: the default rule
    assert pf.batch_band_heights([(480, 640)], intr, [15]) == [4]
    assert pf.batch_band_heights([(480, 640)] * 2, intr, [15, 3]) == [4, 4]
    assert pf.batch_band_heights([(1080, 1920)], intr, [31]) == [12]
    # a large batch: every frame at the 12-row cap, still more than the slots
    sizes = [(240, 320)] * 24 + [(480, 640)] * 32 + [(720, 1280)] * 8
    ks = [3, 5, 7, 9, 15] * 12 + [3, 5, 7, 9]
    h = pf.batch_band_heights(sizes, intr, ks)
    assert h == [12] * 64
    # a frame shorter than the cap stops at its own height, and the planner
    # stops once the batch fits (300 x 6 workgroups, 3 fewer per raised frame)
    h = pf.batch_band_heights([(6, 640)] * 300, intr, [3] * 300)
    assert h == [6] * 259 + [4] * 41
    assert sum(_groups(6, 640, 3, t) for t in h) == 1023
    assert pf.batch_band_heights([], intr, 5) == []
    lib = pf.load_library()
    out = (ctypes.c_int32 * 1)()
    assert lib.pf_batch_band_heights(None, 1, out) == 1
    assert lib.pf_batch_band_heights(None, -1, out) == 2
    assert lib.pf_batch_band_heights(None, 0, None) == 0


def test_output_tensor_checks():
    """The binding refuses out tensors of the wrong shape, dtype, layout or
    device before any pointer reaches the library (the kernels write the
    plan's [3,H,W] / [H,W] shapes whatever they are given)."""
    import torch
    from paper_2103_06644_amd._binding import _check_outs
    H, W, dev = 6, 8, torch.device("cpu")
    good = (torch.empty(3, H, W), torch.empty(H, W), torch.empty(H, W),
            torch.empty(H, W, dtype=torch.uint8))
    _check_outs(torch, good, H, W, dev)
    bad = [
        (torch.empty(3, H, W + 1),) + good[1:],                       # shape
        good[:1] + (torch.empty(H, W, dtype=torch.float64),) + good[2:],  # dtype
        good[:2] + (torch.empty(W, H).t(),) + good[3:],               # not contiguous
        good[:3] + (torch.empty(H, W),),                              # status dtype
        good[:3],                                                     # missing tensor
    ]
    for b in bad:
        with pytest.raises(ValueError):
            _check_outs(torch, b, H, W, dev)
    with pytest.raises(ValueError):
        _check_outs(torch, good, H, W, torch.device("meta"))          # device
