"""The column schedule of the large-bond build's Jacobi rounds (workgroup
kernel for bond bounds 32 and 64), restated from its rule: after a round,
slot 0 keeps its first column, slot 1 takes slot 0's second column, slot
p >= 2 takes slot p-1's first column, slot p < P-1 takes slot p+1's second
column and the last slot takes its own first column. One sweep is C - 1
rounds over C = 2P columns. The kernel needs every pair of columns to meet
exactly once per sweep (a one-sided Jacobi sweep) and every column to be
back in its starting slot at the end (singular values and factors are read
from the starting layout)."""
import pytest


def move(slots):
    P = len(slots)
    out = []
    for p in range(P):
        first = slots[0][0] if p == 0 else (slots[0][1] if p == 1 else slots[p - 1][0])
        second = slots[p][0] if p == P - 1 else slots[p + 1][1]
        out.append((first, second))
    return out


@pytest.mark.parametrize("P", list(range(1, 65)))
def test_round_robin_meets_every_pair_once_and_returns(P):
    C = 2 * P
    start = [(p, C - 1 - p) for p in range(P)]
    cur, met = start, set()
    for _ in range(C - 1):
        for a, b in cur:
            assert a != b
            key = (min(a, b), max(a, b))
            assert key not in met
            met.add(key)
        if P >= 2:
            cur = move(cur)
    assert len(met) == C * (C - 1) // 2
    assert cur == start
