"""The five synthetic workloads the plane-fitting path is measured and tested on.

Each entry is a recipe for seeded frames; `frames_for(name)` renders them.

* plain_160x120  - one 160x120 frame, f = 131.25, 3 planes at 0.5-4 m,
                   5 % invalid pixels in 4x4 blobs, window k = 5.
* vga_640x480    - one 640x480 frame, f = 525, 8 planes + 3 spheres
                   (radius 0.2-0.8 m) at 0.5-6 m, 10 % invalid in square blobs
                   of side 2-12, windows k in {3, 5, 9, 15}.
* hd_1920x1080   - one 1920x1080 frame, f = 1050, depth 0.3-10 m, edge-on
                   planes covering 20 % of the pixels, no holes, k in {15, 31}.
* batch_mixed_64 - 64 frames: 24 at 320x240, 32 at 640x480, 8 at 1280x720,
                   f = 525 * W / 640, per-frame k drawn from {3, 5, 7, 9, 15}.
* diff_8x640x480 - 8 frames at 640x480 with k = 9, plus seeded loss weights
                   and target normals for the differentiation workload.

The scene statistics follow the paper's synthetic protocol (Sec. III):
rays through pixel centres, plane intersections, noise along the measurement
direction with sigma_Z = 1.425e-3 Z^2 (Eq. 2).
"""
from __future__ import annotations

import numpy as np

from .scenes import camera_for, make_frame

VGA_SCENE = dict(n_planes=8, n_spheres=3, zmin=0.5, zmax=6.0, hole_fraction=0.10,
                 hole_sizes=tuple(range(2, 13)))

CONFIGS = {
    "plain_160x120": dict(
        frames=[dict(width=160, height=120, fx=131.25, seed=1, window=5,
                     scene=dict(n_planes=3, n_spheres=0, zmin=0.5, zmax=4.0,
                                hole_fraction=0.05, hole_sizes=(4,)))],
        windows=(5,),
    ),
    "vga_640x480": dict(
        frames=[dict(width=640, height=480, fx=525.0, seed=2, window=None, scene=VGA_SCENE)],
        windows=(3, 5, 9, 15),
    ),
    "hd_1920x1080": dict(
        frames=[dict(width=1920, height=1080, fx=1050.0, seed=3, window=None,
                     scene=dict(n_planes=8, n_spheres=3, zmin=0.3, zmax=10.0,
                                hole_fraction=0.0, grazing_fraction=0.20))],
        windows=(15, 31),
    ),
    "diff_8x640x480": dict(
        frames=[dict(width=640, height=480, fx=525.0, seed=5000 + i, window=9, scene=VGA_SCENE)
                for i in range(8)],
        windows=(9,),
    ),
}


def _batch_mixed_frames():
    sizes = [(320, 240)] * 24 + [(640, 480)] * 32 + [(1280, 720)] * 8
    ks = (3, 5, 7, 9, 15)
    out = []
    for i, (w, h) in enumerate(sizes):
        rng = np.random.Generator(np.random.PCG64(4000 + i))
        k = int(ks[rng.integers(len(ks))])
        out.append(dict(width=w, height=h, fx=525.0 * w / 640.0, seed=4000 + i,
                        window=k, scene=VGA_SCENE))
    return out


CONFIGS["batch_mixed_64"] = dict(frames=_batch_mixed_frames(), windows=(3, 5, 7, 9, 15))


def frame_for(spec: dict):
    cam = camera_for(spec["width"], spec["height"], spec["fx"])
    return make_frame(cam, spec["seed"], window=spec.get("window"), **spec["scene"])


def frames_for(name: str, limit: int | None = None):
    """Render the frames of workload `name` (optionally only the first `limit`)."""
    specs = CONFIGS[name]["frames"]
    if limit is not None:
        specs = specs[:limit]
    return [frame_for(s) for s in specs]


def diff_loss_inputs(height: int, width: int, seed: int):
    """Seeded per-pixel loss weights w ~ U[0, 1] and target normals uniform on the
    sphere for the differentiation workload (loss = sum w (1 - n.n_t) + 0.1 r)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.uniform(0.0, 1.0, size=(height, width))
    t = rng.standard_normal((3, height, width))
    t /= np.linalg.norm(t, axis=0, keepdims=True)
    return w, t
