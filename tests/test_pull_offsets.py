"""Host check of the closure kernel's 32-bit pull offsets.

The kernel forms the byte offset of each pull as a per-lane base plus
wave-uniform neighbour deltas selected by per-lane face masks, modulo 2^32;
the 64-bit form selects the source block per lane and takes the slot's
block-interleaved index.  Both are restated here from their definitions (a
pull of direction c at lane (x, y, z) of a 4^3 block reads (x, y, z) - c,
wrapping into the face, edge or corner neighbour block it crosses into) and
compared for every D3Q19 direction and lane, with random neighbour blocks and
block indices up to the 4 GiB limit of the 32-bit form.
"""
import numpy as np
import pytest

Q = 19
MASK = (1 << 32) - 1


def lattice(orc):
    c, _, _ = orc.lattice(19)
    return [tuple(int(v) for v in ci) for ci in c]


def dir_of(c, v):
    return c.index(v)


def slot_64(c, i, lane, own, nbv):
    """Source slot as the block-selecting form takes it."""
    cx, cy, cz = c[i]
    lx, ly, lz = lane & 3, (lane >> 2) & 3, lane >> 4
    ox = cx != 0 and lx == (0 if cx > 0 else 3)
    oy = cy != 0 and ly == (0 if cy > 0 else 3)
    oz = cz != 0 and lz == (0 if cz > 0 else 3)
    b = own
    if ox: b = nbv[dir_of(c, (-cx, 0, 0)) - 1]
    if oy: b = nbv[dir_of(c, (0, -cy, 0)) - 1]
    if oz: b = nbv[dir_of(c, (0, 0, -cz)) - 1]
    if ox and oy: b = nbv[dir_of(c, (-cx, -cy, 0)) - 1]
    if ox and oz: b = nbv[dir_of(c, (-cx, 0, -cz)) - 1]
    if oy and oz: b = nbv[dir_of(c, (0, -cy, -cz)) - 1]
    local = ((lx - cx) & 3) | (((ly - cy) & 3) << 2) | (((lz - cz) & 3) << 4)
    return b * 64 + local


def bytes_64(c, i, lane, own, nbv, s):
    slot = slot_64(c, i, lane, own, nbv)
    return (((slot >> 6) * Q + i) * 64 + (slot & 63)) * s


def bytes_32(c, i, lane, own, nbv, s):
    """The kernel's 32-bit form."""
    cx, cy, cz = c[i]
    qs = Q * 64 * s
    lx, ly, lz = lane & 3, (lane >> 2) & 3, lane >> 4
    m = lambda cond: MASK if cond else 0
    fx = m(lx == (0 if cx > 0 else 3)) if cx else 0
    fy = m(ly == (0 if cy > 0 else 3)) if cy else 0
    fz = m(lz == (0 if cz > 0 else 3)) if cz else 0
    delta = lambda d, wrap: (nbv[d - 1] * qs - own * qs + wrap * s) & MASK
    base = (lane * s + own * qs) & MASK
    off = (base + (64 * i - (cx + 4 * cy + 16 * cz)) * s) & MASK
    dx = dy = dz = 0
    if cx:
        dx = delta(dir_of(c, (-cx, 0, 0)), 4 * cx)
        off += fx & dx
    if cy:
        dy = delta(dir_of(c, (0, -cy, 0)), 16 * cy)
        off += fy & dy
    if cz:
        dz = delta(dir_of(c, (0, 0, -cz)), 64 * cz)
        off += fz & dz
    if cx and cy:
        off += (fx & fy) & ((delta(dir_of(c, (-cx, -cy, 0)), 4 * cx + 16 * cy) - dx - dy) & MASK)
    if cx and cz:
        off += (fx & fz) & ((delta(dir_of(c, (-cx, 0, -cz)), 4 * cx + 64 * cz) - dx - dz) & MASK)
    if cy and cz:
        off += (fy & fz) & ((delta(dir_of(c, (0, -cy, -cz)), 16 * cy + 64 * cz) - dy - dz) & MASK)
    return off & MASK


@pytest.mark.parametrize("s", [4, 2])
def test_32bit_pull_offsets_equal_slot_arithmetic(orc, s):
    c = lattice(orc)
    rng = np.random.default_rng(2503 + s)
    nb_max = (1 << 32) // (Q * 64 * s)  # blocks of the largest buffer the 32-bit form serves
    for trial in range(40):
        own = int(rng.integers(0, nb_max)) if trial % 4 else int(rng.integers(0, 64))
        nbv = [int(v) for v in rng.integers(0, nb_max, Q - 1)]
        for i in range(1, Q):
            for lane in range(64):
                want = bytes_64(c, i, lane, own, nbv, s)
                assert want < (1 << 32)
                assert bytes_32(c, i, lane, own, nbv, s) == want, (trial, i, lane)
