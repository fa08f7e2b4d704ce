"""Scene rendering for synthetic RGBD depth frames.

The protocol follows the paper's synthetic-data experiment (Sec. III): a
virtual pinhole camera casts one ray through the centre of every pixel, the
rays are intersected with 3D primitives, and the hit points are perturbed
along the ray (in depth) with Gaussian noise whose standard deviation is the
Kinect model of Eq. (2), sigma_Z = 1.425e-3 * Z^2 metres.

Conventions
-----------
* Pixel (x, y) has its centre at integer coordinates; the ray through it is
  r = ((x - cx)/fx, (y - cy)/fy, 1) (Eq. 1 with delta = 0), so a point at
  depth Z on that ray is P = Z * r.
* A plane is {P : n.P + d = 0} with unit n and d > 0 (it faces the camera).
* Invalid pixels carry depth 0 (the sensor convention for "no return").
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KINECT_SIGMA_COEFF = 1.425e-3  # sigma_Z / Z^2 in 1/m, Eq. (2)


@dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def rays(self):
        """Per-pixel ray directions (rx, ry) with rz = 1, float64, shape [H, W]."""
        x = (np.arange(self.width, dtype=np.float64) - self.cx) / self.fx
        y = (np.arange(self.height, dtype=np.float64) - self.cy) / self.fy
        rx, ry = np.meshgrid(x, y)
        return rx, ry


@dataclass
class Frame:
    """One rendered frame plus its ground truth."""
    camera: Camera
    depth: np.ndarray            # float32 [H, W], metres, 0 = invalid
    depth_clean: np.ndarray      # float64 [H, W], noise-free z-buffer (before holes)
    normal_gt: np.ndarray        # float64 [3, H, W], unit normal of the visible primitive
    prim_id: np.ndarray          # int32 [H, W], 0 = background, 1.. = primitives
    holes: np.ndarray            # bool [H, W], pixels punched to Z = 0
    seed: int
    window: int | None = None
    meta: dict = field(default_factory=dict)

    @property
    def intrinsics(self):
        c = self.camera
        return (c.fx, c.fy, c.cx, c.cy)


def camera_for(width: int, height: int, fx: float, fy: float | None = None,
               cx: float | None = None, cy: float | None = None) -> Camera:
    fy = fx if fy is None else fy
    cx = (width - 1) / 2.0 if cx is None else cx
    cy = (height - 1) / 2.0 if cy is None else cy
    return Camera(width, height, float(fx), float(fy), float(cx), float(cy))


def exact_plane_depth(cam: Camera, n, d) -> np.ndarray:
    """Noise-free depth of the plane n.P + d = 0 at every pixel (float64).

    Pixels whose ray misses the plane in front of the camera get NaN.
    """
    n = np.asarray(n, dtype=np.float64)
    rx, ry = cam.rays()
    ndr = n[0] * rx + n[1] * ry + n[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        z = -float(d) / ndr
    z[~(z > 0)] = np.nan
    return z


def _random_unit(rng, size=None):
    v = rng.standard_normal(3 if size is None else (size, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _random_facing_plane(rng, cam: Camera, zmin: float, zmax: float):
    """Normal uniform on the camera-facing hemisphere, anchored on a random pixel ray.

    Returns (n, d, anchor): the plane n.P + d = 0 passes through `anchor`."""
    while True:
        n = _random_unit(rng)
        if n[2] > 0:
            n = -n
        ax = rng.uniform(0, cam.width - 1)
        ay = rng.uniform(0, cam.height - 1)
        r = np.array([(ax - cam.cx) / cam.fx, (ay - cam.cy) / cam.fy, 1.0])
        a = rng.uniform(zmin, zmax) * r
        d = -float(n @ a)
        if d > 0:
            return n, d, a


def _grazing_plane(rng, cam: Camera):
    """A plane seen edge-on along a band of rays through a random pixel:
    the anchor ray makes |n . r_hat| = g with g in [0.02, 0.08], and the plane
    passes 0.15-0.6 m from the camera centre."""
    ax = rng.uniform(0, cam.width - 1)
    ay = rng.uniform(0, cam.height - 1)
    r = np.array([(ax - cam.cx) / cam.fx, (ay - cam.cy) / cam.fy, 1.0])
    rh = r / np.linalg.norm(r)
    g = rng.uniform(0.02, 0.08)
    t = _random_unit(rng)
    t = t - (t @ rh) * rh
    t /= np.linalg.norm(t)
    n = -g * rh + np.sqrt(1.0 - g * g) * t
    d = rng.uniform(0.15, 0.6)
    return n, d


def _plane_hits(rx, ry, n, d, zmin, zmax, anchor=None, radius=None, max_cos=None):
    """Depth of the plane n.P + d = 0 along every ray (inf where not drawn).

    With `anchor`/`radius` the plane is a disk of that radius around the anchor;
    with `max_cos` only rays with |n . r_hat| < max_cos see it (an edge-on strip)."""
    ndr = n[0] * rx + n[1] * ry + n[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        z = -d / ndr
    ok = (ndr < 0) & (z >= zmin) & (z <= zmax)
    if radius is not None:
        dx, dy, dz = z * rx - anchor[0], z * ry - anchor[1], z - anchor[2]
        ok &= dx * dx + dy * dy + dz * dz <= radius * radius
    if max_cos is not None:
        ok &= -ndr < max_cos * np.sqrt(rx * rx + ry * ry + 1.0)
    return np.where(ok, z, np.inf)


def _sphere_hits(rx, ry, c, radius, zmin, zmax):
    a = rx * rx + ry * ry + 1.0
    b = rx * c[0] + ry * c[1] + c[2]
    cc = float(c @ c) - radius * radius
    disc = b * b - a * cc
    with np.errstate(invalid="ignore"):
        z = (b - np.sqrt(disc)) / a
    ok = (disc >= 0) & (z >= zmin) & (z <= zmax)
    return np.where(ok, z, np.inf)


def _grazing_fraction(normal_gt, rx, ry, valid):
    rn = np.sqrt(rx * rx + ry * ry + 1.0)
    cosv = np.abs(normal_gt[0] * rx + normal_gt[1] * ry + normal_gt[2]) / rn
    return float(np.mean((cosv < 0.1) & valid))


def render_scene(cam: Camera, rng, *, n_planes: int, n_spheres: int = 0,
                 zmin: float, zmax: float, sphere_radius=(0.2, 0.8),
                 patch_radius=(0.2, 0.8), grazing_fraction: float | None = None):
    """Z-buffer planar patches and spheres; returns (depth float64, normal_gt, prim_id, meta).

    Planes are drawn as disks around their anchor point whose radius is a
    fraction `patch_radius` of the anchor depth (so each covers a sizeable part
    of the image without hiding every other primitive); pixels no primitive
    covers see a fronto-parallel background at `zmax`."""
    rx, ry = cam.rays()
    H, W = rx.shape
    zbuf = np.full((H, W), np.inf)
    pid = np.zeros((H, W), np.int32)
    normals = np.zeros((3, H, W))
    prims = []

    def add_plane(z, n, pidx):
        closer = z < zbuf
        zbuf[closer] = z[closer]
        pid[closer] = pidx
        for c in range(3):
            normals[c][closer] = n[c]

    for _ in range(n_planes):
        n, d, a = _random_facing_plane(rng, cam, zmin, zmax)
        radius = rng.uniform(*patch_radius) * a[2]
        prims.append(("plane", n, d, a, radius))
        add_plane(_plane_hits(rx, ry, n, d, zmin, zmax, anchor=a, radius=radius), n, len(prims))

    for _ in range(n_spheres):
        radius = rng.uniform(*sphere_radius)
        ax = rng.uniform(0, cam.width - 1)
        ay = rng.uniform(0, cam.height - 1)
        r = np.array([(ax - cam.cx) / cam.fx, (ay - cam.cy) / cam.fy, 1.0])
        zc = rng.uniform(zmin + radius, zmax - radius)
        c = zc * r
        prims.append(("sphere", c, radius))
        z = _sphere_hits(rx, ry, c, radius, zmin, zmax)
        closer = z < zbuf
        zbuf[closer] = z[closer]
        pid[closer] = len(prims)
        px, py, pz = z * rx - c[0], z * ry - c[1], z - c[2]
        normals[0][closer] = (px / radius)[closer]
        normals[1][closer] = (py / radius)[closer]
        normals[2][closer] = (pz / radius)[closer]

    meta = {"n_planes": n_planes, "n_spheres": n_spheres, "n_grazing": 0}
    if grazing_fraction is not None:
        # Add edge-on planes one at a time until the visible fraction of pixels
        # whose ground-truth normal makes |n . r_hat| < 0.1 reaches the target
        # (+/- 1 percentage point); an overshooting plane is rejected.
        lo, hi = grazing_fraction - 0.01, grazing_fraction + 0.01
        for _ in range(400):
            bg = ~np.isfinite(zbuf)
            tmp_n = normals.copy()
            tmp_n[2][bg] = -1.0
            frac = _grazing_fraction(tmp_n, rx, ry, np.ones_like(bg))
            if frac >= lo:
                break
            n, d = _grazing_plane(rng, cam)
            z = _plane_hits(rx, ry, n, d, zmin, zmax, max_cos=0.12)
            closer = z < zbuf
            for c in range(3):
                tmp_n[c][closer] = n[c]
            if _grazing_fraction(tmp_n, rx, ry, np.ones_like(bg)) > hi:
                continue
            prims.append(("grazing", n, d))
            add_plane(z, n, len(prims))
            meta["n_grazing"] += 1

    bg = ~np.isfinite(zbuf)
    zbuf[bg] = zmax
    normals[0][bg] = 0.0
    normals[1][bg] = 0.0
    normals[2][bg] = -1.0
    pid[bg] = 0
    meta["grazing_fraction"] = _grazing_fraction(normals, rx, ry, np.ones_like(bg))
    meta["primitives"] = prims
    return zbuf, normals, pid, meta


def add_kinect_noise(z, rng, coeff: float = KINECT_SIGMA_COEFF):
    """Perturb depth along the ray: Z += coeff * Z^2 * N(0, 1) (Eq. 2)."""
    return z + coeff * z * z * rng.standard_normal(z.shape)


def punch_holes(shape, rng, fraction: float, sizes):
    """Square blobs of Z = 0, placed uniformly (overlap allowed) until the
    invalid fraction first reaches `fraction`. `sizes` is a list of side lengths
    drawn uniformly."""
    H, W = shape
    holes = np.zeros(shape, bool)
    target = fraction * H * W
    count = 0
    sizes = list(sizes)
    while count < target:
        s = int(sizes[rng.integers(len(sizes))])
        s = min(s, H, W)
        y = int(rng.integers(0, H - s + 1))
        x = int(rng.integers(0, W - s + 1))
        blk = holes[y:y + s, x:x + s]
        count += int(s * s - blk.sum())
        blk[...] = True
    return holes


def make_frame(cam: Camera, seed: int, *, n_planes: int, n_spheres: int = 0,
               zmin: float, zmax: float, hole_fraction: float = 0.0,
               hole_sizes=(4,), grazing_fraction: float | None = None,
               noise: bool = True, window: int | None = None) -> Frame:
    rng = np.random.Generator(np.random.PCG64(seed))
    z, normals, pid, meta = render_scene(cam, rng, n_planes=n_planes, n_spheres=n_spheres,
                                         zmin=zmin, zmax=zmax,
                                         grazing_fraction=grazing_fraction)
    zn = add_kinect_noise(z, rng) if noise else z.copy()
    holes = punch_holes(z.shape, rng, hole_fraction, hole_sizes) if hole_fraction > 0 \
        else np.zeros(z.shape, bool)
    depth = zn.astype(np.float32)
    depth[holes] = 0.0
    meta["invalid_fraction"] = float(holes.mean())
    return Frame(cam, depth, z, normals, pid, holes, seed, window, meta)
