"""Host-side checks of the arithmetic the register mini-map kernel relies on
(no GPU): its lane-to-row layout and its fixed-point row carry.

Lane t of a 768-lane workgroup owns column t % w and rows r0 = t // w,
r0 + R, r0 + 2R, ... (R = 768 // w) of the cell's h*d rows; row r sits at
y = r % h, z = r // h.  Each step adds R rows: dz = R // h planes and dy =
R % h rows, plus one more plane when y passes h.  The kernel finds that carry
as the carry-out of a 32-bit add: y is held as y * K with K = ceil(2^32 / h)
and each step adds dy * K.  These tests walk the same arithmetic in Python
integers and compare every step with the direct division r // h, r % h.
"""
import numpy as np

LANES = 768


def _walk_ok(w, h, d):
    """True when the fixed-point carry equals the y wrap for every lane and
    every slot that holds a row of a w x h x d cell."""
    R = LANES // w
    nrows = h * d
    if h == 1:
        return True  # dy = 0: no step ever wraps
    K = ((1 << 32) + h - 1) // h
    dz, dy = divmod(R, h)
    r0 = np.arange(min(R, nrows), dtype=np.int64)
    nvalid = (nrows - r0 + R - 1) // R
    y = (r0 % h) * K % (1 << 32)
    z_fixed = r0 // h
    for j in range(1, int(nvalid.max())):
        live = j < nvalid
        s = y + dy * K
        carry = s >> 32
        y = s & 0xFFFFFFFF
        z_fixed = z_fixed + dz + carry
        r = r0 + j * R
        if not np.array_equal(z_fixed[live], (r // h)[live]):
            return False
    return True


def test_fixed_point_carry_matches_division_on_every_layout():
    """Every cell shape the register path takes (w <= 768, at most 64 slots a
    lane: h*d <= 64 * (768 // w)), on a grid of widths and heights."""
    bad = []
    widths = list(range(1, 33)) + [40, 48, 64, 100, 128, 200, 256, 384, 500, 767, 768]
    for w in widths:
        R = LANES // w
        for h in list(range(1, 40)) + [64, 97, 128, 255, 256, 500, 1000, 4096, 12288, 49152]:
            maxd = (64 * R) // h
            if maxd < 1:
                continue
            for d in sorted({1, 2, maxd // 2 or 1, maxd}):
                if not _walk_ok(w, h, d):
                    bad.append((w, h, d))
    assert not bad, bad[:10]


def test_carry_bound_on_the_largest_cells():
    """The carry stays exact while (planes in the cell) * (h*K - 2^32) < K:
    with h*d <= 64 * 768 rows that holds for every h (the kernel's bound)."""
    for h in range(2, 64 * LANES + 1, 97):
        K = ((1 << 32) + h - 1) // h
        e = h * K - (1 << 32)
        d_max = (64 * LANES) // h
        assert d_max * e < K, (h, d_max, e, K)
