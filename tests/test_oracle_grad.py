"""Pins of the FP64 autograd reference of the fit's depth gradient (CPU only).

The reference (oracle/grad.py, plain PyTorch autograd) is checked against two
things it shares no code with: its forward outputs against the C oracle's, and
its gradient against central finite differences of the C oracle's outputs.
"""
import numpy as np
import pytest

import oracle
from oracle import grad as og
from depthsynth import frames_for
from parity import crop, loss_oracle, upstream

_cache = {}


def _frame():
    if "f" not in _cache:
        _cache["f"] = frames_for("diff_8x640x480", limit=1)[0]
    return _cache["f"]


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_reference_forward_matches_c_oracle(mode):
    z, intr = crop(_frame(), 100, 100, 26, 21)
    z[5, 7] = 0.0
    k = 5
    import torch
    n, d, r, valid = og.fit_outputs(torch.tensor(z), intr, k, mode)
    o = oracle.fit_planes(z, intr, k, mode)
    v = valid.numpy()
    assert np.array_equal(v, o["status"] == 0)
    cosang = np.clip(np.abs((n.numpy()[:, v] * o["normals"][:, v]).sum(0)), 0, 1)
    assert np.all(np.arccos(cosang) < 1e-7)
    assert np.allclose(n.numpy()[:, v], o["normals"][:, v], atol=1e-7)
    assert np.allclose(d.numpy()[v], o["offsets"][v], rtol=1e-9, atol=1e-12)
    assert np.allclose(r.numpy()[v], o["residuals"][v], rtol=1e-7, atol=1e-13)


@pytest.mark.parametrize("mode,k,where", [("implicit", 5, (100, 100)), ("explicit", 5, (100, 100)),
                                           ("implicit", 3, (40, 400)), ("explicit", 7, (500, 60))])
def test_reference_gradient_matches_finite_differences(mode, k, where):
    """Central differences of the C oracle's weighted outputs, step 1e-6 Z."""
    z, intr = crop(_frame(), where[0], where[1], 18, 14)
    z[3, 4] = np.nan  # a hole: its windows drop out, its own gradient is 0
    o = oracle.fit_planes(z, intr, k, mode)
    gn, gd, gr, keep = upstream(o, 11 + k, mode, depth=z, intr=intr)
    assert keep.sum() >= 20
    g = og.depth_gradient(z, intr, k, mode, gn, gd, gr)
    fd = np.zeros_like(z)
    for (y, x), zz in np.ndenumerate(z):
        if not np.isfinite(zz):
            continue
        h = 1e-6 * zz
        zp, zm = z.copy(), z.copy()
        zp[y, x] += h
        zm[y, x] -= h
        fd[y, x] = (loss_oracle(zp, intr, k, mode, gn, gd, gr)
                    - loss_oracle(zm, intr, k, mode, gn, gd, gr)) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 0
    err = np.abs(g - fd)
    print(mode, k, "max |g - fd| / max |fd| =", err.max() / scale)
    assert err.max() <= 1e-5 * scale, (err.max(), scale)
    assert g[3, 4] == 0.0


def c5_upstream(o, z, intr, seed):
    """The differentiation workload's loss on a crop, L = sum W (1 - n . t) +
    0.1 r (seeded W ~ U[0, 1], t uniform on the sphere), restricted to
    well-posed windows (valid, implicit kappa below 1e3, offset away from the
    sign flip d = 0): dL/dn = -W t, dL/dr = 0.1 W."""
    from depthsynth import diff_loss_inputs
    H, W = z.shape
    wts, tgt = diff_loss_inputs(H, W, seed)
    _, _, _, keep = upstream(o, seed, "implicit" if "kappa" in o else "explicit", depth=z, intr=intr)
    wk = np.where(keep, wts, 0.0)
    return -wk[None] * tgt, np.zeros((H, W)), 0.1 * wk, keep


@pytest.mark.parametrize("mode", ["implicit", "explicit"])
def test_reference_gradient_fd_1e4_on_32x24(mode):
    """The configuration's own check: central differences with a step of
    1e-4 m (FP64) at every pixel of a 32 x 24 crop, k = 9, for the
    differentiation workload's loss.  The step is not small against the
    curvature of the loss, so the bar is the central difference's truncation
    error, estimated by Richardson extrapolation against a 5e-5 m step, plus
    1e-7 of the largest derivative."""
    z, intr = crop(_frame(), 300, 200, 32, 24)
    k = 9
    o = oracle.fit_planes(z, intr, k, mode)
    if mode == "explicit":
        o.pop("kappa")
    gn, gd, gr, keep = c5_upstream(o, z, intr, 6000)
    assert keep.sum() >= 50
    g = og.depth_gradient(z, intr, k, mode, gn, gd, gr)

    def fd(h):
        out = np.zeros_like(z)
        for (y, x), zz in np.ndenumerate(z):
            zp, zm = z.copy(), z.copy()
            zp[y, x] += h
            zm[y, x] -= h
            out[y, x] = (loss_oracle(zp, intr, k, mode, gn, gd, gr)
                         - loss_oracle(zm, intr, k, mode, gn, gd, gr)) / (2 * h)
        return out

    f1, f2 = fd(1e-4), fd(5e-5)
    trunc = np.abs(f1 - f2) * 4.0 / 3.0       # O(h^2) error of the 1e-4 m step
    scale = np.abs(f1).max()
    err = np.abs(g - f1)
    print(mode, "max |g - fd(1e-4)| / max |fd| =", err.max() / scale,
          "max truncation estimate / max |fd| =", trunc.max() / scale)
    assert np.all(err <= 1.5 * trunc + 1e-7 * scale)
    # and the extrapolated difference (error O(h^4)) agrees far more closely
    rich = (4 * f2 - f1) / 3
    assert np.abs(g - rich).max() <= 1e-5 * scale
