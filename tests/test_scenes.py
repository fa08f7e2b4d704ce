"""Properties of the seeded input generator (CPU only)."""
import numpy as np

from depthsynth import CONFIGS, camera_for, exact_plane_depth, frames_for
from depthsynth.configs import diff_loss_inputs
from depthsynth.scenes import add_kinect_noise, punch_holes


def test_same_seed_same_bytes():
    a = frames_for("plain_160x120")[0]
    b = frames_for("plain_160x120")[0]
    assert a.depth.tobytes() == b.depth.tobytes()
    assert a.depth.dtype == np.float32


def test_noise_follows_kinect_model():
    rng = np.random.Generator(np.random.PCG64(7))
    z = np.full((400, 400), 2.5)
    zn = add_kinect_noise(z, rng)
    s = np.std((zn - z) / z ** 2)
    assert abs(s / 1.425e-3 - 1) < 0.02


def test_hole_fractions_and_blob_sizes():
    f1 = frames_for("plain_160x120")[0]
    assert 0.05 <= f1.meta["invalid_fraction"] < 0.05 + 16 / (160 * 120)
    assert (f1.depth[f1.holes] == 0).all() and (f1.depth[~f1.holes] > 0).all()
    rng = np.random.Generator(np.random.PCG64(3))
    h = punch_holes((100, 120), rng, 0.1, range(2, 13))
    assert 0.1 <= h.mean() < 0.1 + 144 / 12000


def test_grazing_fraction_hd():
    f = frames_for("hd_1920x1080")[0]
    assert abs(f.meta["grazing_fraction"] - 0.20) <= 0.01
    assert f.meta["invalid_fraction"] == 0.0
    d = f.depth
    assert d.min() >= 0.3 * (1 - 0.05) and d.max() <= 10.0 * 1.2


def test_ground_truth_normals_face_camera():
    f = frames_for("vga_640x480")[0]
    rx, ry = f.camera.rays()
    ndr = f.normal_gt[0] * rx + f.normal_gt[1] * ry + f.normal_gt[2]
    assert (ndr <= 1e-12).all()
    assert np.allclose(np.linalg.norm(f.normal_gt, axis=0), 1.0)


def test_exact_plane_depth_closed_form():
    cam = camera_for(32, 24, 30.0)
    n = np.array([0.3, -0.2, -0.9]) / np.linalg.norm([0.3, -0.2, -0.9])
    z = exact_plane_depth(cam, n, 1.5)
    rx, ry = cam.rays()
    P = np.stack([rx * z, ry * z, z])
    assert np.abs(np.einsum("i,ihw->hw", n, P) + 1.5).max() < 1e-14


def test_config_recipes():
    assert set(CONFIGS) == {"plain_160x120", "vga_640x480", "hd_1920x1080", "batch_mixed_64",
                            "diff_8x640x480"}
    frames = CONFIGS["batch_mixed_64"]["frames"]
    assert len(frames) == 64
    sizes = [(f["width"], f["height"]) for f in frames]
    assert sizes.count((320, 240)) == 24 and sizes.count((640, 480)) == 32
    assert sizes.count((1280, 720)) == 8
    assert all(f["window"] in (3, 5, 7, 9, 15) for f in frames)
    w, t = diff_loss_inputs(24, 32, 5000)
    assert w.min() >= 0 and w.max() <= 1
    assert np.allclose(np.linalg.norm(t, axis=0), 1.0)
