"""GPU parity of the literal implicit mode (PF_IMPLICIT_LITERAL: constraint
|(a, b, c, d)| = 1 as Sec. II-A states it, smallest eigenvector of the 4x4
scatter of Eq. 14) against the oracle's literal mode, element by element,
gated where the 4x4's kappa = l4 / (l2 - l1) is at most 1e6."""
import numpy as np
import pytest

import oracle
import parity as PT
from depthsynth import frames_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,k", [("plain_160x120", 5), ("vga_640x480", 5), ("vga_640x480", 9),
                                    ("vga_640x480", 15)])
def test_literal_parity(gpu, name, k):
    f = frames_for(name)[0]
    print("[case] literal", name, k, flush=True)
    g = PT.gpu_fit(f.depth, f.intrinsics, k, "implicit_literal")
    o = PT.oracle_full(f.depth, f.intrinsics, k, "implicit_literal")
    rep = PT.check(g, o, "implicit", f.depth, f.intrinsics)
    print(rep, flush=True)
    PT.assert_parity(rep)


def test_literal_hd_sampled_and_unit_dependence(gpu):
    import torch
    import paper_2103_06644_amd as pf
    f = frames_for("hd_1920x1080")[0]
    k = 15
    g = PT.gpu_fit(f.depth, f.intrinsics, k, "implicit_literal")
    rng = np.random.Generator(np.random.PCG64(41))
    ys, xs = rng.integers(0, 1080, 6000), rng.integers(0, 1920, 6000)
    o = oracle.fit_points(f.depth.astype(np.float64), f.intrinsics, k, xs, ys, "implicit_literal")
    rep = PT.check(g, o, "implicit", f.depth, f.intrinsics, sel=(ys, xs))
    print(rep, flush=True)
    PT.assert_parity(rep)
    # the literal fit changes with the depth unit, the unit-normal fit does not
    z = f.depth[:240, :320].copy()
    intr = f.intrinsics
    a = PT.gpu_fit(z, intr, 9, "implicit_literal")
    b = PT.gpu_fit(z * np.float32(1000.0), intr, 9, "implicit_literal")
    v = (a["status"] & 1) == 0
    assert np.median(PT.angle(a["normals"][:, v], b["normals"][:, v])) > 1e-6
    # other entry points refuse the mode
    d = torch.from_numpy(z).cuda()
    with pytest.raises(pf.PlanefitError):
        pf.fit_planes_xyz(d, intr, 9, mode="implicit_literal")
    with pytest.raises(pf.PlanefitError):
        pf.fit_planes(d, intr, 9, mode="implicit_literal", precision="fp32")
