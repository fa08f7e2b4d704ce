"""Checks that pin the FP64 oracle to facts other than itself.

Each function returns a list of failure strings (empty = the pin holds), so the
same checks serve tests/test_oracle.py and the mutation test, which rebuilds
the oracle with a planted mistake and asserts some pin rejects it.

The facts used:
  * closed forms: depth of a known plane (Eq. 1 intersected with n.P + d = 0)
    and the camera-only window moments in centred coordinates;
  * library routines on tiny windows: numpy.linalg.lstsq for the explicit
    fit (Eq. 15) and numpy.linalg.svd for the constrained implicit fit;
  * the definition of the objective, minimised by scipy.optimize;
  * brute-force window sums vs four-corner sums of integral images (Sec. II-C);
  * invariants: power-of-two and general depth scaling, image flips;
  * exact symmetry: a window whose best plane passes through the camera
    centre, for the orientation tie-break.
"""
from __future__ import annotations

import numpy as np

import oracle
from depthsynth import camera_for, exact_plane_depth, frames_for


def angle(a, b):
    """Angle between unit vectors stored along axis 0 (sign-sensitive)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    cr = np.cross(a, b, axis=0)
    return np.arctan2(np.linalg.norm(cr, axis=0), np.sum(a * b, axis=0))


EXACT_PLANES = [
    # (normal, offset) of n.P + d = 0; the normal faces the camera (d > 0)
    ((0.0, 0.0, -1.0), 2.0),                      # fronto-parallel
    ((0.3, -0.2, -0.9), 1.5),                     # generic tilt
    ((np.sin(np.pi / 3), 0.0, -np.cos(np.pi / 3)), 1.2),   # 60 degrees
    ((0.0, -0.998749217771909, -0.05), 0.8),      # grazing at the optical axis
    ((0.1, 0.2, -0.97), 0.05),                    # 5 cm from the camera centre
]


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def pin_exact_planes(ks=(3, 5, 7), modes=None, tol=1e-9):
    modes = modes or ["implicit", "explicit", "implicit_scatter", "explicit_normaleq",
                      "xyz_implicit", "xyz_explicit"]
    cam = camera_for(48, 40, 40.0, 44.0, 23.2, 19.7)
    intr = (cam.fx, cam.fy, cam.cx, cam.cy)
    fails = []
    for n, d in EXACT_PLANES:
        n = _unit(n)
        z = exact_plane_depth(cam, n, d)
        for k in ks:
            for m in modes:
                o = oracle.fit_planes(z, intr, k, m)
                v = o["status"] == 0
                if v.sum() < 10:
                    fails.append(f"exact plane {n},{d} k={k} {m}: only {v.sum()} valid windows")
                    continue
                ang = angle(o["normals"][:, v], n[:, None]).max()
                derr = np.abs(o["offsets"][v] / d - 1).max()
                res = o["residuals"][v].max()
                if not (ang <= tol and derr <= tol and res <= tol):
                    fails.append(f"exact plane {n},{d} k={k} {m}: angle {ang:.2e} "
                                 f"offset {derr:.2e} residual {res:.2e}")
    return fails


def pin_camera_moments(tol=1e-12):
    fails = []
    for (fx, fy, cx, cy) in [(525.0, 525.0, 319.5, 239.5), (131.25, 140.0, 79.5, 59.5)]:
        for k in (3, 5, 9, 15, 31):
            N = k * k
            S2 = k * k * (k * k - 1) / 12.0
            for (x0, y0) in [(0, 0), (100, 37), (-5, 400), (639, 479)]:
                uc, vc = (x0 - cx) / fx, (y0 - cy) / fy
                want = np.array([N * uc * uc + S2 / fx ** 2, N * uc * vc, N * uc,
                                 N * vc * vc + S2 / fy ** 2, N * vc, N])
                got = oracle.camera_moments((fx, fy, cx, cy), k, x0, y0)
                rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
                rel[np.abs(want) < 1e-9] = np.abs(got - want)[np.abs(want) < 1e-9]
                if rel.max() > tol:
                    fails.append(f"camera moments k={k} at {(x0, y0)}: {got} vs {want}")
    return fails


def _tiny_frames():
    rng = np.random.Generator(np.random.PCG64(11))
    out = []
    for (W, H) in [(7, 5), (9, 11), (16, 12)]:
        cam = camera_for(W, H, 12.0, 13.0)
        n = _unit([0.2, -0.3, -0.9])
        z = exact_plane_depth(cam, n, 1.0)
        z = z + 1.425e-3 * z * z * rng.standard_normal(z.shape)
        z[rng.random(z.shape) < 0.08] = 0.0
        out.append((cam, z))
    return out


def pin_integral_vs_direct(tol=1e-12):
    fails = []
    for cam, z in _tiny_frames():
        intr = (cam.fx, cam.fy, cam.cx, cam.cy)
        H, W = z.shape
        I = oracle.integral_images(z, intr)
        for k in (3, 5):
            r = k // 2
            direct = oracle.window_sums(z, intr, k)
            for y0 in range(r, H - r):
                for x0 in range(r, W - r):
                    ya, yb, xa, xb = y0 - r, y0 + r + 1, x0 - r, x0 + r + 1
                    s = I[:, yb, xb] - I[:, ya, xb] - I[:, yb, xa] + I[:, ya, xa]
                    dd = direct[:, y0, x0]
                    if np.abs(s - dd).max() > tol * max(1.0, np.abs(dd).max()):
                        fails.append(f"box sum {W}x{H} k={k} at {(x0, y0)}: {s} vs {dd}")
    return fails


def pin_integral_method_fit(tol=1e-8):
    """The paper's integral-image fit agrees with the brute-force fit."""
    fails = []
    for cam, z in _tiny_frames():
        intr = (cam.fx, cam.fy, cam.cx, cam.cy)
        for k in (3, 5):
            for m in ("implicit", "explicit"):
                a = oracle.fit_planes(z, intr, k, m)
                b = oracle.fit_planes_integral(z, intr, k, m)
                if not np.array_equal(a["status"], b["status"]):
                    fails.append(f"integral-method validity differs {z.shape} k={k} {m}")
                    continue
                v = a["status"] == 0
                if m == "implicit":
                    v &= a["kappa"] < 1e3
                if v.any():
                    ang = angle(a["normals"][:, v], b["normals"][:, v]).max()
                    if ang > tol:
                        fails.append(f"integral-method fit {z.shape} k={k} {m}: angle {ang:.2e}")
    return fails


def _window_design(z, cam, k, x0, y0):
    """Rows m_i = (tan th_x, tan th_y, 1) from pixel coordinates (Eq. 10) and w_i = 1/Z_i."""
    r = k // 2
    ys, xs = np.mgrid[y0 - r:y0 + r + 1, x0 - r:x0 + r + 1]
    zz = z[ys, xs].ravel()
    u = ((xs.ravel() - cam.cx) / cam.fx)
    v = ((ys.ravel() - cam.cy) / cam.fy)
    m = np.stack([u, v, np.ones_like(u)], 1)
    return m, 1.0 / zz, zz


def _noisy_windows(count=40, seed=5):
    f = frames_for("plain_160x120")[0]
    cam = f.camera
    z = f.depth.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    o = oracle.fit_planes(z, f.intrinsics, 5, "implicit")
    cand = np.argwhere((o["status"] == 0) & (o["kappa"] < 1e3))
    pick = cand[rng.choice(len(cand), size=count, replace=False)]
    return cam, z, [(int(x), int(y)) for y, x in pick]


def pin_library_routines(k=5, tol_ang=1e-9, tol_off=1e-9):
    """Explicit fit vs numpy lstsq; implicit fit vs numpy svd of the design with the
    disparity column projected out (the |n| = 1 constrained minimiser)."""
    cam, z, pts = _noisy_windows()
    intr = (cam.fx, cam.fy, cam.cx, cam.cy)
    xs = np.array([p[0] for p in pts])
    ys = np.array([p[1] for p in pts])
    oe = oracle.fit_points(z, intr, k, xs, ys, "explicit")
    oi = oracle.fit_points(z, intr, k, xs, ys, "implicit")
    fails = []
    for i, (x0, y0) in enumerate(pts):
        m, w, zz = _window_design(z, cam, k, x0, y0)
        alpha = np.linalg.lstsq(m, w, rcond=None)[0]
        n_e = -alpha / np.linalg.norm(alpha)
        d_e = 1.0 / np.linalg.norm(alpha)
        ang = angle(oe["normals"][:, i], n_e)
        if ang > tol_ang or abs(oe["offsets"][i] / d_e - 1) > tol_off:
            fails.append(f"explicit vs lstsq at {(x0, y0)}: angle {ang:.2e}")
        wn = w / np.linalg.norm(w)
        B = m - np.outer(wn, wn @ m)
        n_i = np.linalg.svd(B)[2][-1]
        d_i = -(w @ m @ n_i) / (w @ w)
        if d_i < 0:
            n_i, d_i = -n_i, -d_i
        ang = angle(oi["normals"][:, i], n_i)
        res = np.sqrt(np.mean((m @ n_i + d_i * w) ** 2))
        if ang > tol_ang * max(1.0, oi["kappa"][i]) or abs(oi["offsets"][i] / d_i - 1) > tol_off * max(1.0, oi["kappa"][i]):
            fails.append(f"implicit vs svd at {(x0, y0)}: angle {ang:.2e}")
        if abs(oi["residuals"][i] - res) > 1e-9 * max(res, 1e-12):
            fails.append(f"implicit residual vs svd at {(x0, y0)}: {oi['residuals'][i]} vs {res}")
    return fails


def pin_objective_minimum(k=5, n_windows=6):
    """scipy.optimize on the raw objective sum((n.P_i + d)/Z_i)^2 over unit n and d
    never finds a lower value than the oracle's implicit fit."""
    from scipy.optimize import minimize
    cam, z, pts = _noisy_windows(count=n_windows, seed=9)
    intr = (cam.fx, cam.fy, cam.cx, cam.cy)
    xs = np.array([p[0] for p in pts])
    ys = np.array([p[1] for p in pts])
    oi = oracle.fit_points(z, intr, k, xs, ys, "implicit")
    fails = []
    for i, (x0, y0) in enumerate(pts):
        r = k // 2
        yy, xx = np.mgrid[y0 - r:y0 + r + 1, x0 - r:x0 + r + 1]
        Z = z[yy, xx].ravel()
        P = np.stack([(xx.ravel() - cam.cx) * Z / cam.fx, (yy.ravel() - cam.cy) * Z / cam.fy, Z], 1)

        def obj(p):
            th, ph, d = p
            n = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
            return np.sum(((P @ n + d) / Z) ** 2)

        n0 = oi["normals"][:, i]
        e0 = obj([np.arccos(np.clip(n0[2], -1, 1)), np.arctan2(n0[1], n0[0]), oi["offsets"][i]])
        best = np.inf
        for start in ([2.8, 0.3, 1.0], [2.5, -2.0, 2.0], [3.0, 1.5, 0.5]):
            res = minimize(obj, start, method="Nelder-Mead",
                           options=dict(xatol=1e-12, fatol=1e-18, maxiter=20000, maxfev=40000))
            best = min(best, res.fun)
        if best < e0 * (1 - 1e-7) - 1e-18:
            fails.append(f"optimiser beat the oracle at {(x0, y0)}: {best} < {e0}")
        # KKT: small rotations of n with d re-optimised never lower the objective
        rng = np.random.Generator(np.random.PCG64(i))
        for _ in range(8):
            t = rng.standard_normal(3)
            t -= (t @ n0) * n0
            t /= np.linalg.norm(t)
            n1 = np.cos(1e-4) * n0 + np.sin(1e-4) * t
            w2 = 1.0 / Z ** 2
            d1 = -np.sum(w2 * (P @ n1)) / np.sum(w2)
            if np.sum(((P @ n1 + d1) / Z) ** 2) < e0 * (1 - 1e-9):
                fails.append(f"perturbed normal lowered the objective at {(x0, y0)}")
    return fails


def pin_invariants(k=5):
    f = frames_for("plain_160x120")[0]
    z = f.depth.astype(np.float64)
    fx, fy, cx, cy = f.intrinsics
    H, W = z.shape
    fails = []
    for m in ("implicit", "explicit"):
        base = oracle.fit_planes(z, f.intrinsics, k, m)
        v = base["status"] == 0
        if m == "implicit":
            v &= base["kappa"] < 1e4
        for s in (2.0 ** -3, 2.0 ** 5, 1.37):
            o = oracle.fit_planes(z * s, f.intrinsics, k, m)
            ang = angle(o["normals"][:, v], base["normals"][:, v]).max()
            derr = np.abs(o["offsets"][v] / (s * base["offsets"][v]) - 1).max()
            rerr = np.abs(o["residuals"][v] - base["residuals"][v]).max()
            if ang > 1e-10 or derr > 1e-10 or rerr > 1e-12:
                fails.append(f"depth scale {s} {m}: angle {ang:.2e} offset {derr:.2e} res {rerr:.2e}")
        # left-right flip with cx -> W-1-cx negates n_x
        o = oracle.fit_planes(z[:, ::-1], (fx, fy, W - 1 - cx, cy), k, m)
        nf = o["normals"][:, :, ::-1].copy()
        nf[0] = -nf[0]
        ang = angle(nf[:, v], base["normals"][:, v]).max()
        if ang > 1e-10:
            fails.append(f"left-right flip {m}: angle {ang:.2e}")
        o = oracle.fit_planes(z[::-1, :], (fx, fy, cx, H - 1 - cy), k, m)
        nf = o["normals"][:, ::-1, :].copy()
        nf[1] = -nf[1]
        ang = angle(nf[:, v], base["normals"][:, v]).max()
        if ang > 1e-10:
            fails.append(f"up-down flip {m}: angle {ang:.2e}")
    return fails


def pin_explicit_orthogonality(k=5):
    """The explicit residual vector alpha.m_i - w_i is orthogonal to the regressors."""
    cam, z, pts = _noisy_windows(count=20, seed=3)
    intr = (cam.fx, cam.fy, cam.cx, cam.cy)
    xs = np.array([p[0] for p in pts])
    ys = np.array([p[1] for p in pts])
    oe = oracle.fit_points(z, intr, k, xs, ys, "explicit")
    fails = []
    for i, (x0, y0) in enumerate(pts):
        m, w, _ = _window_design(z, cam, k, x0, y0)
        alpha = -oe["normals"][:, i] / oe["offsets"][i]
        e = m @ alpha - w
        g = m.T @ e
        if np.abs(g).max() > 1e-10 * np.abs(m.T @ w).max():
            fails.append(f"explicit normal equations violated at {(x0, y0)}: {g}")
    return fails


def pin_kappa(k=5, tol=1e-9):
    """kappa = l3 / (l2 - l1) of the implicit 3x3 (the gate of the parity tests)
    against numpy.linalg.eigvalsh of B^T B, B = m - w (w^T m) / (w^T w): the
    design with the disparity direction projected out, whose Gram matrix is
    the 1/Z^2-weighted covariance of the back-projected points."""
    cam, z, pts = _noisy_windows(count=48, seed=21)
    intr = (cam.fx, cam.fy, cam.cx, cam.cy)
    xs = np.array([p[0] for p in pts])
    ys = np.array([p[1] for p in pts])
    oi = oracle.fit_points(z, intr, k, xs, ys, "implicit")
    fails = []
    for i, (x0, y0) in enumerate(pts):
        m, w, _ = _window_design(z, cam, k, x0, y0)
        B = m - np.outer(w, w @ m) / (w @ w)
        l1, l2, l3 = np.linalg.eigvalsh(B.T @ B)
        want = l3 / (l2 - l1)
        if abs(oi["kappa"][i] / want - 1) > tol:
            fails.append(f"kappa at {(x0, y0)}: {oi['kappa'][i]!r} vs eigvalsh {want!r}")
    return fails


def pin_xyz_library_routines(k=5, tol=1e-9):
    """The standard XYZ fits (Eq. 3-9) on noisy windows: explicit against
    numpy lstsq of Z on (X, Y, 1), implicit against the smallest right singular
    vector of the centred points (unweighted PCA, |n| = 1); both oriented d >= 0."""
    cam, z, pts = _noisy_windows(count=40, seed=17)
    intr = (cam.fx, cam.fy, cam.cx, cam.cy)
    xs = np.array([p[0] for p in pts])
    ys = np.array([p[1] for p in pts])
    oe = oracle.fit_points(z, intr, k, xs, ys, "xyz_explicit")
    oi = oracle.fit_points(z, intr, k, xs, ys, "xyz_implicit")
    fails = []
    for i, (x0, y0) in enumerate(pts):
        m, _, zz = _window_design(z, cam, k, x0, y0)
        P = m * zz[:, None]                        # back-projected points (Eq. 1)
        a, b, c = np.linalg.lstsq(np.stack([P[:, 0], P[:, 1], np.ones(len(zz))], 1), P[:, 2],
                                  rcond=None)[0]
        s_ = np.sqrt(a * a + b * b + 1.0)
        n_e, d_e = np.array([a, b, -1.0]) / s_, c / s_
        if d_e < 0:
            n_e, d_e = -n_e, -d_e
        ang = angle(oe["normals"][:, i], n_e)
        if ang > tol or abs(oe["offsets"][i] / d_e - 1) > tol:
            fails.append(f"xyz explicit vs lstsq at {(x0, y0)}: angle {ang:.2e}, "
                         f"offset {oe['offsets'][i]} vs {d_e}")
        cen = P.mean(0)
        n_i = np.linalg.svd(P - cen)[2][-1]
        d_i = -n_i @ cen
        if d_i < 0:
            n_i, d_i = -n_i, -d_i
        kap = max(1.0, oi["kappa"][i])
        ang = angle(oi["normals"][:, i], n_i)
        if ang > tol * kap or abs(oi["offsets"][i] / d_i - 1) > tol * kap:
            fails.append(f"xyz implicit vs svd at {(x0, y0)}: angle {ang:.2e}, "
                         f"offset {oi['offsets'][i]} vs {d_i}")
    return fails


def tie_break_frame(fx, fy):
    """A 5 x 5 depth frame whose one full window is centred on the optical axis
    (c = (2, 2)), with depths 1/2 and 1 placed with mirror symmetry in x and
    y: 13 pixels at 1/2 (centre, the four diagonal neighbours, the four
    corners, the two ends of the middle row and of the middle column) and 12
    at 1.  Every integrand is a short dyadic number, so every sum is exact.
    By symmetry the 1/Z^2-weighted centroid lies on the optical axis and the
    weighted covariance is diagonal; its x and y entries are the camera-only
    sums S2/fx^2, S2/fy^2 (S2 = 50) and its z entry is about 2.4, so the
    best plane is X = 0 (fx > fy) or Y = 0 (fx < fy): a plane through the
    camera centre, d = 0."""
    z = np.ones((5, 5))
    for dy, dx in [(0, 0), (-1, -1), (-1, 1), (1, -1), (1, 1), (-2, -2), (-2, 2), (2, -2),
                   (2, 2), (0, -2), (0, 2), (-2, 0), (2, 0)]:
        z[2 + dy, 2 + dx] = 0.5
    return z, (float(fx), float(fy), 2.0, 2.0)


def pin_orientation_tie_break():
    """d = 0 leaves the sign of the eigenvector (Sec. I-C) to the tie-break:
    the first non-zero of n_z, n_y, n_x is negative.  On the symmetric frame
    the exact answer is n = (-1, 0, 0) for fx > fy and (0, -1, 0) for fx < fy,
    with d exactly 0 (and not -0)."""
    fails = []
    for (fx, fy), want in (((64.0, 32.0), (-1.0, 0.0, 0.0)), ((32.0, 64.0), (0.0, -1.0, 0.0))):
        z, intr = tie_break_frame(fx, fy)
        for mode in ("implicit", "implicit_scatter"):
            o = oracle.fit_points(z, intr, 5, np.array([2]), np.array([2]), mode)
            n, d = o["normals"][:, 0], o["offsets"][0]
            if o["status"][0] != 0 or not np.array_equal(n, np.array(want)) or d != 0.0 \
                    or np.signbit(d):
                fails.append(f"tie-break fx={fx} fy={fy} {mode}: n={n} d={d!r}, want {want}, 0")
    return fails


ALL_PINS = [pin_exact_planes, pin_camera_moments, pin_integral_vs_direct,
            pin_integral_method_fit, pin_library_routines, pin_objective_minimum,
            pin_invariants, pin_explicit_orthogonality, pin_kappa, pin_xyz_library_routines,
            pin_orientation_tie_break]
