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
