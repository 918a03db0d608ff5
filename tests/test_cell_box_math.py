"""The packed-cell box test of the render kernels, as integer arithmetic.

A cell is packed as x | y << 11 | z << 22 with guard bits 10, 21 and 31; a box
is held as the two words G - lo and G - (hi + 1) (G = the guard mask).  A cell
c lies in the box exactly when every guard of c + (G - lo) is set and every
guard of c + (G - (hi + 1)) is clear, and neither addition carries out of its
32-bit word, so two cells packed in 64 bits can be tested with two 64-bit
additions.  These checks run the same arithmetic in Python integers against
the direct per-axis comparison, on every cell of small grids and on random
cells of the largest grid the packing allows (1023 x 1023 x 511), including
the dead cell (every field at its maximum) and empty boxes.
"""
import numpy as np
import pytest

G = (1 << 10) | (1 << 21) | (1 << 31)
ONES = 1 | (1 << 11) | (1 << 22)
MAX_XY, MAX_Z = 1023, 511
DEAD = 0x3FF | (0x3FF << 11) | (0x1FF << 22)
M32 = (1 << 32) - 1


def pack(x, y, z):
    return x | (y << 11) | (z << 22)


def box_words(lo, hi):
    empty = any(l > h for l, h in zip(lo, hi)) or hi[0] >= MAX_XY or hi[1] >= MAX_XY or hi[2] >= MAX_Z
    plo = DEAD if empty else pack(*lo)
    phi = 0 if empty else pack(*hi)
    return (G - plo) & M32, (G - (phi + ONES)) & M32


def guards(a, b):
    return (a & ~b & G) == G


def in_box(c, glo, ghi):
    a, b = c + glo, c + ghi
    assert a <= M32 and b <= M32          # no carry leaves the word
    return guards(a, b)


def in_box2(c0, c1, glo, ghi):
    c2 = c0 | (c1 << 32)
    a = (c2 + (glo | (glo << 32))) & ((1 << 64) - 1)
    b = (c2 + (ghi | (ghi << 32))) & ((1 << 64) - 1)
    return guards(a & M32, b & M32), guards(a >> 32, b >> 32)


def direct(cell, lo, hi):
    return all(l <= c <= h for c, l, h in zip(cell, lo, hi))


@pytest.mark.parametrize("dims", [(5, 4, 3), (9, 2, 7)])
def test_every_cell_of_small_grids(dims):
    rng = np.random.default_rng(11)
    cells = [(x, y, z) for x in range(dims[0]) for y in range(dims[1]) for z in range(dims[2])]
    for _ in range(60):
        lo = [int(rng.integers(0, d)) for d in dims]
        hi = [int(rng.integers(l, d)) for l, d in zip(lo, dims)]
        glo, ghi = box_words(lo, hi)
        for cell in cells:
            assert in_box(pack(*cell), glo, ghi) == direct(cell, lo, hi), (lo, hi, cell)
        assert not in_box(DEAD, glo, ghi)


def test_random_cells_of_the_largest_grid_and_pairs():
    rng = np.random.default_rng(12)
    caps = (MAX_XY, MAX_XY, MAX_Z)
    for _ in range(400):
        lo = [int(rng.integers(0, c)) for c in caps]
        hi = [int(rng.integers(l, c)) for l, c in zip(lo, caps)]
        glo, ghi = box_words(lo, hi)
        # cells around the box's faces, its corners and anywhere in the grid
        pts = []
        for _ in range(24):
            pts.append(tuple(int(np.clip(rng.integers(l - 2, h + 3), 0, c - 1)) for l, h, c in zip(lo, hi, caps)))
            pts.append(tuple(int(rng.integers(0, c)) for c in caps))
        pts += [tuple(lo), tuple(hi), (0, 0, 0), (caps[0] - 1, caps[1] - 1, caps[2] - 1)]
        for i in range(0, len(pts) - 1, 2):
            c0, c1 = pack(*pts[i]), pack(*pts[i + 1])
            m0, m1 = in_box2(c0, c1, glo, ghi)
            assert m0 == direct(pts[i], lo, hi) == in_box(c0, glo, ghi)
            assert m1 == direct(pts[i + 1], lo, hi) == in_box(c1, glo, ghi)
        assert in_box2(DEAD, DEAD, glo, ghi) == (False, False)


def test_empty_boxes_hold_no_cell():
    for lo, hi in [((3, 3, 3), (2, 5, 5)), ((0, 0, 0), (MAX_XY, 4, 4)), ((0, 0, 0), (4, 4, MAX_Z))]:
        glo, ghi = box_words(lo, hi)
        for cell in [(0, 0, 0), (3, 3, 3), (2, 4, 4), (MAX_XY - 1, MAX_XY - 1, MAX_Z - 1)]:
            assert not in_box(pack(*cell), glo, ghi)
        assert not in_box(DEAD, glo, ghi)
