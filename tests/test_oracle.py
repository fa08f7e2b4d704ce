"""Pins of the FP64 oracle (CPU only).

The oracle is checked against closed forms, library routines, the definition
of the objective, brute force and invariants (tests/oracle_pins.py), never
against the HIP path.  The mutation test rebuilds the oracle from its source
with one planted mistake at a time and asserts that some pin rejects it.
"""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest
from scipy.ndimage import minimum_filter

import oracle
import oracle_pins as P
from depthsynth import camera_for, exact_plane_depth, frames_for


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    fails = pin()
    assert not fails, "\n".join(fails[:10])


def test_jacobi_matches_numpy_eigh():
    rng = np.random.Generator(np.random.PCG64(0))
    for t in range(300):
        a = rng.standard_normal((3, 3))
        a = a + a.T
        if t % 3 == 0:   # clustered spectra
            q = np.linalg.qr(rng.standard_normal((3, 3)))[0]
            a = q @ np.diag([1.0, 1.0 + 1e-7, 3.0]) @ q.T
        ev, V = oracle.jacobi3(a)
        ref = np.linalg.eigvalsh(a)
        assert np.allclose(ev, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        assert np.allclose(V.T @ V, np.eye(3), atol=1e-13)
        assert np.allclose(a @ V, V * ev, atol=1e-12 * np.abs(ref).max())


def test_validity_rule_matches_brute_force_mask():
    f = frames_for("plain_160x120")[0]
    z = f.depth.astype(np.float64)
    z[3, 7] = np.nan
    z[50, 60] = np.inf
    z[80, 100] = -1.0
    mask = np.ones(z.shape, np.uint8)
    mask[20:22, 30:33] = 0
    for k in (3, 5):
        o = oracle.fit_planes(z, f.intrinsics, k, "implicit", mask=mask)
        good = np.isfinite(z) & (z > 0) & (mask != 0)
        r = k // 2
        want = minimum_filter(good.astype(np.uint8), size=k, mode="constant", cval=0) == 1
        assert np.array_equal(o["status"] == 0, want)
        inv = o["status"] == 1
        assert np.isnan(o["normals"][:, inv]).all() and np.isnan(o["offsets"][inv]).all()
        assert np.isfinite(o["normals"][:, ~inv]).all()
        # border windows are never valid
        assert inv[:r].all() and inv[-r:].all() and inv[:, :r].all() and inv[:, -r:].all()


def test_unit_normals_and_orientation():
    f = frames_for("plain_160x120")[0]
    for m in ("implicit", "explicit"):
        o = oracle.fit_planes(f.depth, f.intrinsics, 5, m)
        v = o["status"] == 0
        nrm = np.linalg.norm(o["normals"][:, v], axis=0)
        assert np.abs(nrm - 1).max() < 1e-14
        assert (o["offsets"][v] >= 0).all()


def test_implicit_paths_agree_on_noisy_frame():
    """Weighted PCA (two-pass) and the Eq. 14 scatter route give the same plane."""
    f = frames_for("plain_160x120")[0]
    a = oracle.fit_planes(f.depth, f.intrinsics, 5, "implicit")
    b = oracle.fit_planes(f.depth, f.intrinsics, 5, "implicit_scatter")
    v = (a["status"] == 0) & (a["kappa"] < 1e4)
    ang = P.angle(a["normals"][:, v], b["normals"][:, v])
    # the one-pass scatter loses digits to cancellation: error grows like eps*kappa*(u^2/spread)
    assert ang.max() < 1e-6
    assert np.median(ang) < 1e-9


def test_rgbd_fit_differs_from_unweighted_xyz_fit():
    """The RGBD implicit fit is the 1/Z^2-weighted estimator, not classic PCA: on noisy
    data the two estimators differ (so a parity check can tell which one it got)."""
    f = frames_for("vga_640x480")[0]
    a = oracle.fit_planes(f.depth, f.intrinsics, 5, "implicit", threads=4)
    b = oracle.fit_planes(f.depth, f.intrinsics, 5, "xyz_implicit", threads=4)
    v = (a["status"] == 0) & (a["kappa"] < 1e3)
    ang = P.angle(a["normals"][:, v], b["normals"][:, v])
    assert np.median(ang) > 1e-6


def test_fit_points_matches_fit_planes():
    f = frames_for("plain_160x120")[0]
    full = oracle.fit_planes(f.depth, f.intrinsics, 5, "implicit")
    rng = np.random.Generator(np.random.PCG64(1))
    xs = rng.integers(0, 160, 50)
    ys = rng.integers(0, 120, 50)
    pts = oracle.fit_points(f.depth, f.intrinsics, 5, xs, ys, "implicit")
    assert np.array_equal(pts["status"], full["status"][ys, xs])
    v = pts["status"] == 0
    assert np.array_equal(pts["normals"][:, v], full["normals"][:, ys[v], xs[v]])


def test_bad_arguments_raise():
    z = np.ones((8, 8))
    with pytest.raises(ValueError):
        oracle.fit_planes(z, (1, 1, 1, 1), 4)
    with pytest.raises(ValueError):
        oracle.fit_planes(z, (1, 1, 1, 1), 3, mode=9)


# ---------------------------------------------------------------------------
# Planted mistakes: each must be caught by at least one pin.
# ---------------------------------------------------------------------------
MUTATIONS = {
    "cx_sign": ("X[n] = ((double)x - cam->cx) * z / cam->fx;",
                "X[n] = ((double)x + cam->cx) * z / cam->fx;"),
    "fy_swapped_for_fx": ("Y[n] = ((double)y - cam->cy) * z / cam->fy;",
                          "Y[n] = ((double)y - cam->cy) * z / cam->fx;"),
    "weight_1_over_z": ("double w = weighted ? 1.0 / (Z[i] * Z[i]) : 1.0;\n    sw += w;",
                        "double w = weighted ? 1.0 / Z[i] : 1.0;\n    sw += w;"),
    "dropped_intercept_term": ("alpha[2] = mw - alpha[0] * mu - alpha[1] * mv;",
                               "alpha[2] = mw - alpha[0] * mu;"),
    "offset_not_inverted": ("f->d = 1.0 / s;", "f->d = s;"),
    "rotation_transposed": ("J[p][p] = c; J[p][q] = s; J[q][p] = -s; J[q][q] = c;",
                            "J[p][p] = c; J[p][q] = -s; J[q][p] = s; J[q][q] = c;"),
    "largest_eigvec": ("double n[3] = {V[0], V[3], V[6]};\n  unit_from(n, f->n);\n  f->d = -(f->n[0] * c[0]",
                       "double n[3] = {V[2], V[5], V[8]};\n  unit_from(n, f->n);\n  f->d = -(f->n[0] * c[0]"),
    "centroid_unweighted_z": ("c[2] += w * Z[i];", "c[2] += Z[i];"),
    "kappa_l3_over_l2": ("? ev[2] / (ev[1] - ev[0]) : INFINITY;", "? ev[2] / ev[1] : INFINITY;"),
    "tie_break_dropped": ("  else if (f->n[2] != 0.0)\n    flip = f->n[2] > 0.0;\n"
                          "  else if (f->n[1] != 0.0)\n    flip = f->n[1] > 0.0;\n"
                          "  else\n    flip = f->n[0] > 0.0;",
                          "  else\n    flip = 0;"),
    "xyz_implicit_weighted": ("case PFO_XYZ_IMPLICIT: fit_implicit_pca(X, Y, Z, N, 0, &f);",
                              "case PFO_XYZ_IMPLICIT: fit_implicit_pca(X, Y, Z, N, 1, &f);"),
    "xyz_explicit_dropped_y": ("double c = mz - a * mx - b * my;", "double c = mz - a * mx;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    here = os.path.dirname(oracle.__file__)
    src = open(os.path.join(here, "pfo_oracle.c")).read()
    old, new = MUTATIONS[name]
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    src = src.replace(old, new)
    (tmp_path / "pfo_oracle.h").write_text(open(os.path.join(here, "pfo_oracle.h")).read())
    (tmp_path / "pfo_oracle.c").write_text(src)
    lib = str(tmp_path / "libmut.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                    str(tmp_path / "pfo_oracle.c"), "-o", lib, "-lm"], check=True)
    caught = []
    with oracle.using_library(lib):
        for pin in P.ALL_PINS:
            try:
                if pin():
                    caught.append(pin.__name__)
            except Exception as e:  # a crash in a pin also rejects the build
                caught.append(f"{pin.__name__} ({type(e).__name__})")
            if caught:
                break
    assert caught, f"no pin rejected the planted mistake {name}"
