"""Host emulation of the fused kernel's output index map (no GPU): for the
launch geometry a plan chooses, every output pixel is written by exactly one
thread of one workgroup, and no store (scalar, float4 run or packed status
word) touches a byte at or past the end of its plane.

The emulation follows the kernel's own arithmetic: strip = wg % n_strips,
band = wg / n_strips, rounds of ROWS rows, runs of RUN outputs per thread, and
the vectorised run store taken only when the whole run lies in the strip and
in the row."""
import numpy as np
import pytest

import paper_2103_06644_amd as pf

BLOCK = 256
SHAPES = {0: (4, 4), 1: (4, 4), 2: (8, 8)}   # launch shape -> (rows per round, run)


def geometry(H, W, k, mode, shape=None, band_height=None):
    """(tile_w, n_strips, tile_h, n_bands, shape) as the plan computes them."""
    tw_max = ((BLOCK - (k - 1)) // 4) * 4
    n_strips = -(-W // tw_max)
    tile_w = (-(-W // n_strips) + 3) // 4 * 4
    p = pf.Plan((525.0, 525.0, W / 2 - 0.5, H / 2 - 0.5), H, W, k, mode)
    if shape is not None or band_height is not None:
        p = p.derive(band_height or 0, -1 if shape is None else shape)
    tile_h = p.tile_h
    return tile_w, n_strips, tile_h, -(-H // tile_h), p.shape


def emulate(H, W, k, mode, vec_store, shape=None, band_height=None):
    """Bytes written per status position and per float position (one plane)."""
    tile_w, n_strips, tile_h, n_bands, shp = geometry(H, W, k, mode, shape, band_height)
    ROWS, RUN = SHAPES[shp]
    assert tile_w + k - 1 <= BLOCK
    hits = np.zeros(H * W + 64, np.int32)        # +64: room to catch an overrun
    for wg in range(n_strips * n_bands):
        strip, band = wg % n_strips, wg // n_strips
        ox0 = strip * tile_w
        yb = band * tile_h
        ye = min(yb + tile_h, H)
        for yg in range(yb, ye, ROWS):
            nr = min(ROWS, ye - yg)
            for tid in range(BLOCK):
                hj, run = tid // (BLOCK // RUN), tid % (BLOCK // RUN)
                o0 = run * RUN
                o1 = min(o0 + RUN, tile_w)
                if hj >= nr or o0 >= o1:
                    continue
                y0 = yg + hj
                x0 = ox0 + o0
                p = y0 * W + x0
                if mode == "explicit" and vec_store and o0 + RUN <= o1 and x0 + RUN <= W:
                    hits[p:p + RUN] += 1              # float4 runs and one status word
                else:
                    for q in range(RUN):
                        if o0 + q < o1 and x0 + q < W:
                            hits[p + q] += 1
    return hits


@pytest.mark.parametrize("H,W,k,mode", [
    (480, 640, 3, "explicit"), (480, 640, 15, "explicit"), (1080, 1920, 15, "explicit"),
    (1080, 1920, 31, "explicit"), (120, 160, 5, "explicit"), (37, 93, 7, "explicit"),
    (480, 640, 9, "implicit"), (1080, 1920, 31, "implicit"), (37, 93, 7, "implicit"),
    (63, 63, 63, "implicit"), (720, 1280, 63, "explicit"),
])
def test_every_pixel_written_once_and_nothing_past_the_end(H, W, k, mode):
    vec = (W % 4 == 0)
    hits = emulate(H, W, k, mode, vec)
    assert np.all(hits[:H * W] == 1), np.unique(hits[:H * W], return_counts=True)
    assert not hits[H * W:].any()


@pytest.mark.parametrize("shape,bh", [(1, 12), (2, 8), (2, 24), (2, 0), (0, 6)])
@pytest.mark.parametrize("H,W,k,mode", [(480, 640, 15, "explicit"), (1080, 1920, 31, "implicit"),
                                        (37, 92, 7, "explicit"), (120, 160, 5, "implicit")])
def test_every_shape_writes_each_pixel_once(H, W, k, mode, shape, bh):
    vec = (W % 4 == 0)
    hits = emulate(H, W, k, mode, vec, shape, bh)
    assert np.all(hits[:H * W] == 1), np.unique(hits[:H * W], return_counts=True)
    assert not hits[H * W:].any()
