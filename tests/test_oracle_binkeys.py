"""CPU check of the bin-key definition against its defining property, by brute force.

A point's key names the tile that holds the first cell of its kernel window: with
u = theta n1 / 2 pi and v = phi n2 / 2 pi (single-rounded FP64 products), the window
is the w consecutive cells c with u - w/2 <= c < u + w/2 along theta (likewise along
phi, cyclically over n2 cells), and the key is (row tile of its first row cell relative to
a_min) * ntile2 + (column tile of its first column cell mod n2).  Here the first cell
is found by scanning integers with exact rational arithmetic, independently of the
ceil-based formula, and the key is rebuilt from it; points on cell boundaries,
at the poles and across phi = 0 are included.  The cell-order key adds the first
cell's place inside its tile (row-major)."""
import math
from fractions import Fraction

import numpy as np

import oracle


def first_cell(x: float, w: int) -> int:
    """Smallest integer c with c >= x - w/2, i.e. the first cell of the window
    x - w/2 <= c < x + w/2 (x exact as the FP64 value it is)."""
    lo = Fraction(x) - Fraction(w, 2)
    c = math.floor(float(lo)) - 2
    while Fraction(c) < lo:
        c += 1
    assert Fraction(c - 1) < lo <= Fraction(c)
    # the window's last cell lies below x + w/2, the next one does not
    assert Fraction(c + w - 1) < Fraction(x) + Fraction(w, 2) <= Fraction(c + w)
    return c


def test_bin_keys_window_starts_in_its_tile():
    rng = np.random.default_rng(5)
    n1, n2, t1, t2 = 96, 160, 16, 32
    for w in (4, 7, 8, 12, 15):
        a_min = -(w // 2) - 1
        ntile2 = (n2 + t2 - 1) // t2
        th = np.concatenate([rng.uniform(0, math.pi, 300), [0.0, math.pi, math.pi / 2]])
        ph = np.concatenate([rng.uniform(0, 2 * math.pi, 300), [0.0, 2 * math.pi - 1e-15, 1e-300]])
        # points whose u or v sits exactly on a cell edge (x - w/2 an integer) or a
        # half-cell
        k = rng.integers(0, n1 // 2, 40)
        th = np.concatenate([th, (k + (w % 2) * 0.5) * (2 * math.pi / n1)])
        ph = np.concatenate([ph, rng.uniform(0, 2 * math.pi, 40)])
        keys = oracle.bin_keys(th, ph, n1, n2, w, a_min, t1, t2, ntile2)
        ckeys = oracle.bin_keys(th, ph, n1, n2, w, a_min, t1, t2, ntile2, cells=True)
        c1 = np.float64(n1) / (np.float64(2.0) * np.float64(np.pi))
        c2 = np.float64(n2) / (np.float64(2.0) * np.float64(np.pi))
        for i in range(th.size):
            u = float(np.float64(th[i]) * c1)
            v = float(np.float64(ph[i]) * c2)
            a0, b0 = first_cell(u, w), first_cell(v, w)
            row, col = (a0 - a_min) // t1, (b0 % n2) // t2
            assert 0 <= a0 - a_min and 0 <= col < ntile2
            assert keys[i] == row * ntile2 + col, (w, i, th[i], ph[i], keys[i], row, col)
            # cell order: the tile, then the first cell's row and column inside it.  The
            # FP64 formula's first cell equals the exact one except where u - w/2 or
            # v - w/2 rounds onto an integer (phi = 1e-300 here), one cell lower.
            half = np.float64(w) * np.float64(0.5)
            af = int(np.ceil(np.float64(u) - half))
            bf = int(np.ceil(np.float64(v) - half))
            for e, f, x in ((a0, af, u), (b0, bf, v)):
                assert e == f or (e - f == 1 and float(np.float64(x) - half) == f), (w, i, e, f)
            assert ckeys[i] == keys[i] * t1 * t2 + ((af - a_min) % t1) * t2 + (bf % n2) % t2
