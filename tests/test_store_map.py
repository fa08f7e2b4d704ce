"""Host emulation of the fused kernel's output index map (no GPU): for the
launch geometry a plan chooses, every output pixel is written by exactly one
thread of one workgroup, no store (scalar, 16-byte group or packed status word)
lands outside its plane, and the horizontal phase's LDS reads stay inside the
column-sum rows.

The emulation follows the kernel's own arithmetic: strip = wg % n_strips,
band = wg / n_strips, rounds of ROWS rows, runs of RUN outputs per thread.
Forward launches run every lane: a lane past the strip recomputes the strip's
last run, and a store is kept only when its element offset, taken from the
wave's first row of the round, lies in the wave's buffer range (its rows of
the frame), which the hardware enforces by dropping the rest; the kernel sends
a pixel outside the strip, the frame or the band a drop offset instead.

Implicit fits with runs of four pack each wave's windows before solving: the
windows with a full valid count take slots 0 .. nfit-1 in column order, every
other window of the wave the slots after them (also in column order), each
slot keeping its column; slot s is then solved (below nfit) and stored by lane
s % 64 in round s / 64, dropped when its column lies past the row's range.
Which windows are valid depends on the depth, so the emulation draws it at
random."""
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


PITCH = 296                                    # LDS row pitch (16-byte records) of the column sums
SUB = {4: 74, 8: 37}                          # LDS layout (i % RUN) * SUB + i / RUN
DROP = 0x80000000


RECORD = 16                                    # bytes per LDS record
SLOT_SUB = 66                                  # packed slot s: record (s % 4) * SLOT_SUB + s / 4


def emulate_packed(hits, W, ox0, tile_w, yg, nr, rng, p_fit):
    """One round of the packed implicit store path (runs of four: wave = row)."""
    for hj in range(4):
        cols = min(tile_w, W - ox0) if hj < nr else 0
        keep = 4 * np.arange(64)[None, :] + np.arange(4)[:, None] < cols
        fit = keep & (rng.random((4, 64)) < p_fit)
        nfit = int(fit.sum())
        # the packed row: slot s in record s of the row (two 16-byte records in
        # FP64), the slots' column bytes in the records after slot 255
        assert (PITCH - BLOCK) * RECORD >= BLOCK
        col = np.full(BLOCK, -1)
        lanes = np.arange(64)
        # valid windows of the lower lanes (the sum over the run of each
        # window's mbcnt), and this lane's valid windows before window q
        below = np.cumsum(fit.sum(axis=0)) - fit.sum(axis=0)
        mine = np.zeros(64, int)
        for q in range(4):
            slots = np.where(fit[q], below + mine, nfit + (4 * lanes - below) + (q - mine))
            assert (col[slots] == -1).all()
            col[slots] = 4 * lanes + q
            mine += fit[q]
        sf, sr = nfit, BLOCK
        assert sf == nfit and sr == BLOCK and (col >= 0).all()
        assert (col < 256).all()                              # kept in one byte
        # the slots below nfit hold exactly the valid windows, each kind in
        # column order
        assert sorted(col[:nfit]) == sorted((4 * lanes[None, :] + np.arange(4)[:, None])[fit])
        assert (np.diff(col[:nfit]) > 0).all() and (np.diff(col[nfit:]) > 0).all()
        # slot s lives in record (s % 4) * SLOT_SUB + s / 4, below the bytes
        # of the slots' columns
        rec = (np.arange(BLOCK) % 4) * SLOT_SUB + np.arange(BLOCK) // 4
        assert len(set(rec)) == BLOCK and rec.max() < 4 * SLOT_SUB
        assert 4 * SLOT_SUB * RECORD + BLOCK <= PITCH * RECORD
        # round s // 64, lane s % 64 stores slot s; a column past the row's
        # range (past the strip, the frame or the band) is dropped
        c = col[col < cols]
        np.add.at(hits, (yg + hj) * W + ox0 + c, 1)


def emulate(H, W, k, mode, vec_store, shape=None, band_height=None, p_fit=None, seed=0):
    """Writes per output position (one plane; +64 positions to catch an overrun)."""
    tile_w, n_strips, tile_h, n_bands, shp = geometry(H, W, k, mode, shape, band_height)
    ROWS, RUN = SHAPES[shp]
    lanes_per_row = BLOCK // RUN
    rows_per_wave = 64 // lanes_per_row
    assert tile_w + k - 1 <= BLOCK
    hits = np.zeros(H * W + 64, np.int32)
    packed = mode == "implicit" and RUN == 4
    rng = np.random.default_rng(seed)
    for wg in range(n_strips * n_bands):
        strip, band = wg % n_strips, wg // n_strips
        ox0 = strip * tile_w
        yb = band * tile_h
        ye = min(yb + tile_h, H)
        for yg in range(yb, ye, ROWS):
            nr = min(ROWS, ye - yg)
            if packed:
                emulate_packed(hits, W, ox0, tile_w, yg, nr, rng, 0.6 if p_fit is None else p_fit)
                continue
            for tid in range(BLOCK):
                hj, run = tid // lanes_per_row, tid % lanes_per_row
                h0 = (tid // 64 * 64) // lanes_per_row        # the wave's first row
                o0s = run * RUN
                o0 = min(o0s, (tile_w - 1) // RUN * RUN)      # the run this lane computes
                # LDS reads: columns o0 .. o0 + RUN - 1 + k - 1 of row hj
                i_max = o0 + RUN - 1 + k - 1
                assert (RUN - 1) * SUB[RUN] + i_max // RUN < PITCH
                base_row = min(yg + h0, H - 1)
                rng = rows_per_wave * W                       # the wave's buffer range (elements)
                cols = min(tile_w, W - ox0) if hj < nr else 0
                base = (hj - h0) * W

                def at(c):
                    return base + c if c < cols else DROP

                if mode == "explicit" and vec_store:
                    for h in range(RUN // 4):
                        e = at(o0s + 4 * h)
                        if e != DROP:
                            assert e % 4 == 0 and e + 4 <= rng
                            g = base_row * W + ox0 + e
                            hits[g:g + 4] += 1
                else:
                    for q in range(RUN):
                        e = at(o0s + q)
                        if e != DROP:
                            assert e < rng
                            hits[base_row * W + ox0 + e] += 1
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


@pytest.mark.parametrize("p_fit", [0.0, 0.3, 1.0])
@pytest.mark.parametrize("H,W,k", [(37, 93, 7), (120, 160, 5), (63, 63, 63)])
def test_packed_implicit_writes_each_pixel_once(H, W, k, p_fit):
    """Any pattern of valid windows (none, some, all): every in-frame pixel is
    stored once, from its own slot, and nothing else is."""
    for shape, bh in ((0, None), (1, 6), (0, 5)):
        hits = emulate(H, W, k, "implicit", W % 4 == 0, shape, bh, p_fit=p_fit, seed=k)
        assert np.all(hits[:H * W] == 1), np.unique(hits[:H * W], return_counts=True)
        assert not hits[H * W:].any()


def test_column_record_writes_spread_over_the_banks():
    """The vertical phase writes column tid's 16-byte record at (tid % RUN) * SUB
    + tid / RUN: the eight lanes one LDS cycle serves (128 bytes) land on eight
    different 16-byte bank groups, for both tilings."""
    for run in (4, 8):
        for first in range(0, 64, 8):
            groups = {(((t % run) * SUB[run] + t // run) * RECORD) % 128 // 16
                      for t in range(first, first + 8)}
            assert len(groups) == 8, (run, first, groups)


def test_packed_slot_records_spread_over_the_banks():
    """A dense row writes slot 4 * lane + q from lane `lane` (consecutive
    records for consecutive lanes) and reads slots s0 + lane: both accesses of
    eight consecutive lanes fall on eight different 16-byte bank groups."""
    rec = lambda s: (s % 4) * SLOT_SUB + s // 4
    for first in range(0, 64, 8):
        for q in range(4):
            w = {(rec(4 * L + q) * RECORD) % 128 // 16 for L in range(first, first + 8)}
            assert len(w) == 8
        for s0 in range(0, 256, 64):
            r = {(rec(s0 + L) * RECORD) % 128 // 16 for L in range(first, first + 8)}
            assert len(r) == 8
