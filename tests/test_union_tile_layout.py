"""Host checks of the union product's LDS tile addressing (kern_batch.hip, k_baxpy).

The B operand of the int8 matrix-core step is built from a block-shared tile of the
step's 64 union columns (column c at byte c * XSB, XSB = RB + 16, rows contiguous) with
gfx950's transposing 8-byte LDS read.  Its lane layout was measured on the GPU with an
in-bounds probe: in each group of 16 lanes, byte b of the result of lane 16 g + 8 e + j
is byte j of the 8 bytes that lane 16 g + 2 b + e read.  These tests emulate that
layout and check, for every block shape the launches use, that the kernel's addresses
give every lane (row m = lane % 16, tile kb = lane / 16) the bytes of row m for columns
16 kb + 8 h .. + 7 in order, stay inside the tile, keep 8-byte alignment, and hit 16
distinct bank pairs per group of 16 lanes.  (The GPU tests check the product itself.)
"""
import itertools

import pytest

PAD = 16   # kXTilePad: LDS bytes after each tile column


def tr8_read(mem, addrs):
    """Emulated ds_read_b64_tr_b8 of a wavefront: addrs[L] is lane L's address."""
    got = [[mem[a + j] for j in range(8)] for a in addrs]
    out = []
    for lane in range(64):
        g, e, j = lane >> 4, (lane >> 3) & 1, lane & 7
        out.append([got[16 * g + 2 * b + e][j] for b in range(8)])
    return out


def lane_address(lane, h, rt, rw, xsb):
    """The byte address k_baxpy passes for lane `lane`, half h, row tile rt, wave rows rw."""
    kb = lane >> 4
    return rw + (16 * kb + 8 * h + ((lane >> 1) & 7)) * xsb + 8 * (lane & 1) + 16 * rt


# (RT, WPB) of the launches: 16-, 8- and 4-wavefront blocks, 1 to 4 row tiles
SHAPES = [(2, 16), (1, 16), (4, 8), (2, 8), (1, 8), (4, 4), (2, 4), (1, 4)]


@pytest.mark.parametrize("rt_count,wpb", SHAPES)
def test_transposing_reads_deliver_the_b_operand(rt_count, wpb):
    rb = 16 * rt_count * wpb
    assert 1024 % rb == 0
    xsb = rb + PAD
    size = 64 * xsb
    mem = {}
    for c in range(64):
        for r in range(rb):
            mem[c * xsb + r] = (c, r)
    for wv in range(wpb):
        rw = wv * 16 * rt_count
        for rt, h in itertools.product(range(rt_count), range(2)):
            addrs = [lane_address(lane, h, rt, rw, xsb) for lane in range(64)]
            assert all(a % 8 == 0 and 0 <= a and a + 8 <= size for a in addrs)
            out = tr8_read(mem, addrs)
            for lane in range(64):
                m, kb = lane & 15, lane >> 4
                want = [(16 * kb + 8 * h + b, rw + 16 * rt + m) for b in range(8)]
                assert out[lane] == want, (rt_count, wpb, wv, rt, h, lane)


@pytest.mark.parametrize("rt_count,wpb", SHAPES)
def test_transposing_reads_are_bank_conflict_free_per_16_lanes(rt_count, wpb):
    xsb = 16 * rt_count * wpb + PAD
    for wv in range(wpb):
        rw = wv * 16 * rt_count
        for rt, h in itertools.product(range(rt_count), range(2)):
            for g0 in range(0, 64, 16):
                banks = set()
                for lane in range(g0, g0 + 16):
                    a = lane_address(lane, h, rt, rw, xsb)
                    banks.update(((a // 4) % 64, (a // 4 + 1) % 64))
                assert len(banks) == 32


def test_tile_stores_cover_every_row_of_every_column_once():
    """Thread t stores 16-byte pieces of column t / WPB at 16 (t % WPB) + 16 WPB rt."""
    for rt_count, wpb in SHAPES:
        rb = 16 * rt_count * wpb
        xsb = rb + PAD
        seen = {}
        for t in range(64 * wpb):
            xc, xj = t // wpb, t % wpb
            for rt in range(rt_count):
                off = xc * xsb + 16 * xj + 16 * wpb * rt
                assert off % 16 == 0
                for k in range(16):
                    seen[off + k] = seen.get(off + k, 0) + 1
        want = {c * xsb + r for c in range(64) for r in range(rb)}
        assert set(seen) == want and all(v == 1 for v in seen.values())
