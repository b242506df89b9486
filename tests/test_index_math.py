"""CPU checks of the hidden-layer kernels' index arithmetic (cnn_kernels.hip).

The kernels replace 32-bit divisions by constants with 24-bit reciprocal
multiplies (Div24: x / D as (x * ceil(2^20 / D)) >> 20) and load each
work-group's input tile in steps of whole pixels.  These tests replay that
arithmetic in Python, with the 24-bit multiplies' wrap-around, and compare it
with the plain divisions it replaces, for every channel width, split mode,
tile shape and wave count the kernels are built for and tiles at every grid
edge.  The GPU tests check the kernels' outputs; these check the scheme.
"""
import pytest

S = 20  # Div24's shift


def u24(a, b):
    return ((a & 0xFFFFFF) * (b & 0xFFFFFF)) & 0xFFFFFFFF


def s24(a, b):
    def sx(v):
        v &= 0xFFFFFF
        return v - (1 << 24) if v & 0x800000 else v
    r = (sx(a) * sx(b)) & 0xFFFFFFFF
    return r - (1 << 32) if r & 0x80000000 else r


def div24(x, d):
    return u24(x, ((1 << S) + d - 1) // d) >> S


CONFIGS = [(C, split, th, tw, nw) for C in (16, 32, 48, 64) for split in (False, True)
           for th, tw in ((8, 32), (16, 16)) for nw in (4, 6)]


def tile_geometry(C, split, th, tw):
    ps = 2 * C + 8 if split else C + 8      # LDS pixel stride (elements)
    sp = ps // 8                            # 16-byte slots per pixel
    tpix = (th + 2) * (tw + 2)
    data = (2 if split else 1) * (C // 8)   # slots that hold data (the rest is pad)
    return ps, sp, tpix, data, tw + 2


@pytest.mark.parametrize("C,split,th,tw,nw", CONFIGS)
def test_tile_load_steps_fill_every_slot_once(C, split, th, tw, nw):
    """Every data slot of the input tile gets the bytes the old per-slot
    divisions named (same plane, same byte offset), exactly once, and no pad
    slot is written."""
    nt = 64 * nw
    _, sp, tpix, data, rw = tile_geometry(C, split, th, tw)
    nslot = tpix * sp
    dp = nt // sp
    step = dp * sp
    for n in (32, 64, 1024):
        ln = n.bit_length() - 1
        for y0, x0 in ((0, 0), (0, n - tw), (n - th, 0), (n - th, n - tw), (th, tw)):
            want = {}
            for sl in range(nslot):
                pp, j = divmod(sl, sp)
                if j >= data:
                    continue
                lo = split and j >= C // 8
                c8 = j - C // 8 if lo else j
                ty, tx = divmod(pp, rw)
                gy, gx = (y0 + ty - 1) & (n - 1), (x0 + tx - 1) & (n - 1)
                want[sl] = (bool(lo), 2 * ((gy * n + gx) * C + c8 * 8))
            got = {}
            for w0 in range(0, nt, 64):
                for lane in range(64):
                    q = w0 + lane
                    pp = div24(q, sp)
                    j = q - s24(pp, sp)
                    ty = div24(pp, rw)
                    tx = pp - s24(ty, rw)
                    lo = split and j >= C // 8
                    c16 = (j - C // 8 if lo else j) * 16
                    live = q < step and j < data
                    for s0 in range(0, nslot, step):
                        if live and q < nslot - s0:
                            gy, gx = (y0 - 1 + ty) & (n - 1), (x0 - 1 + tx) & (n - 1)
                            off = (u24((gy << ln) | gx, 2 * C) + c16) & 0xFFFFFFFF
                            slot = s0 + q
                            assert slot not in got
                            got[slot] = (bool(lo), off)
                        tx += dp % rw
                        ty += dp // rw
                        if tx >= rw:
                            tx -= rw
                            ty += 1
            assert got == want


@pytest.mark.parametrize("C,split,th,tw", sorted({c[:4] for c in CONFIGS}))
def test_first_layer_items(C, split, th, tw):
    """The first layer's item -> (pixel, channel group) -> (row, column),
    state-patch and LDS indices match the plain divisions."""
    ps, _, tpix, _, rw = tile_geometry(C, split, th, tw)
    uw = tw + 4
    for item in range(tpix * (C // 8)):
        px, c8 = divmod(item, C // 8)
        ty, tx = divmod(px, rw)
        want = [(ty + tp // 3) * uw + tx + tp % 3 for tp in range(9)] + [px * ps + c8 * 8]
        px2 = div24(item, C // 8)
        c82 = item - s24(px2, C // 8)
        ty2 = div24(px2, rw)
        tx2 = px2 - s24(ty2, rw)
        ub = s24(ty2, uw) + tx2
        got = [ub + (tp // 3) * uw + tp % 3 for tp in range(9)] + [s24(px2, ps) + c82 * 8]
        assert got == want


def test_div24_range_check_catches_a_short_reciprocal():
    """The compile-time exactness check is not vacuous: a reciprocal rounded
    down instead of up gives wrong quotients on the kernels' ranges."""
    bad = [x for x in range(5000) if (u24(x, (1 << S) // 13) >> S) != x // 13]
    assert bad
    assert all(div24(x, 13) == x // 13 for x in range(5000))
