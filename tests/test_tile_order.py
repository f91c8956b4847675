"""The banded tile order shared by every tile sweep and its refinement pass
(qk_tile_coords), restated index for index: bands of B tile rows, column by
column within a band (symmetric tasks: the upper triangle, diagonal
included). For every band height the autotuner may pick, the map from the
task-local tile number to (tile row, tile column) must be a bijection onto
the task's tiles, with the double-precision band inversion corrected to the
exact band by its integer loops."""
import math

import numpy as np
import pytest


def tile_coords(symmetric, tiles_r, tiles_c, B, lt):
    if not symmetric:
        nr, nc = tiles_r, tiles_c
        band = lt // (B * nc)
        l = lt - band * (B * nc)
        r0 = band * B
        h = min(nr - r0, B)
        return r0 + l % h, l // h
    n = tiles_c
    nb = (n + B - 1) // B
    before = lambda r: B * n * r + (B * r - B * B * r * r) // 2
    bq = float(B) * float(n) + 0.5 * float(B)
    disc = bq * bq - 2.0 * float(B * B) * float(lt)
    R = int((bq - math.sqrt(max(disc, 0.0))) / float(B * B))
    R = min(max(R, 0), nb - 1)
    while R > 0 and before(R) > lt:
        R -= 1
    while R + 1 < nb and before(R + 1) <= lt:
        R += 1
    l = lt - before(R)
    r0 = B * R
    h = min(n - r0, B)
    part = h * (h - 1) // 2
    if l < part:
        c = 0
        while (c + 1) * (c + 2) // 2 <= l:
            c += 1
        return r0 + (l - c * (c + 1) // 2), r0 + c
    l2 = l - part
    return r0 + l2 % h, r0 + h - 1 + l2 // h


@pytest.mark.parametrize("B", [1, 2, 3, 4, 8, 16])
@pytest.mark.parametrize("n", [1, 2, 5, 16, 37, 63, 250])
def test_symmetric_order_is_a_bijection(B, n):
    tot = n * (n + 1) // 2
    seen = set()
    for lt in range(tot):
        ti, tj = tile_coords(True, n, n, B, lt)
        assert 0 <= ti <= tj < n
        seen.add((ti, tj))
    assert len(seen) == tot


@pytest.mark.parametrize("B", [1, 2, 4, 8])
@pytest.mark.parametrize("nr,nc", [(1, 1), (3, 7), (63, 250), (250, 63)])
def test_rectangular_order_is_a_bijection(B, nr, nc):
    seen = set()
    for lt in range(nr * nc):
        ti, tj = tile_coords(False, nr, nc, B, lt)
        assert 0 <= ti < nr and 0 <= tj < nc
        seen.add((ti, tj))
    assert len(seen) == nr * nc


def test_band_four_is_the_previous_closed_form():
    """B = 4 reproduces the fixed order the kernels used before the band was
    a parameter: full bands before band R hold 4 n R - 8 R^2 + 2 R tiles."""
    n = 250
    for R in range(0, 62):
        B = 4
        assert B * n * R + (B * R - B * B * R * R) // 2 == 4 * n * R - 8 * R * R + 2 * R


def test_large_symmetric_task_band_starts():
    """Every band start of a 4000-tile-row task maps to the band's diagonal
    tile (the inversion near the end of the triangle, where the discriminant
    is smallest)."""
    n = 4000
    for B in (2, 4, 8):
        before = lambda r: B * n * r + (B * r - B * B * r * r) // 2
        for R in range(0, (n + B - 1) // B):
            assert tile_coords(True, n, n, B, before(R)) == (B * R, B * R)
