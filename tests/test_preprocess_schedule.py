"""The rotation schedule of the device's Jacobi eigensolver (pre-processing,
Section II-A's PCA), restated from its rule: m (even) players, round r
pairs player 0 with 1 + r and, for i >= 1, 1 + (r + i) mod (m - 1) with
1 + (r - i) mod (m - 1). Every round must be a perfect matching (the
rotations of a round act on disjoint index pairs, so they commute and one
launch applies them all), and m - 1 rounds must meet every pair once (a
full cyclic sweep). Odd sizes add a padding player that never rotates."""
import pytest


def rr_pair(r, i, m):
    P = m - 1
    if i == 0:
        p, q = 0, 1 + r
    else:
        u, v = r + i, r - i + P
        if u >= P:
            u -= P
        if v >= P:
            v -= P
        p, q = 1 + u, 1 + v
    return (p, q) if p < q else (q, p)


@pytest.mark.parametrize("d", [2, 3, 4, 7, 16, 63, 64, 784])
def test_rounds_are_matchings_and_a_sweep_meets_every_pair(d):
    m = d + (d & 1)
    met = set()
    for r in range(m - 1):
        seen = set()
        for i in range(m // 2):
            p, q = rr_pair(r, i, m)
            assert 0 <= p < q < m
            assert p not in seen and q not in seen
            seen |= {p, q}
            met.add((p, q))
        assert len(seen) == m
    assert len(met) == m * (m - 1) // 2
