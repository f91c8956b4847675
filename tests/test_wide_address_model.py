"""Host model of every memory access and barrier of the large-bond sweeps.

The complex-FP32 matrix-core sweep for padded bonds 8..64
(`sweep_wide_kernel<T>`), the FP64 per-pair sweep its refinement runs
(`sweep_big_list_kernel<T>`, the same `sweep_pair<T>` body as
`sweep_big_kernel<T>`) and the pair numbering they share (`qk_pair_of`,
`qk_pair_lookup`) are restated here index for index, for every thread of a
workgroup, at the bond dimensions 8, 16, 32, 64 and at the task shapes the
GPU tests and the bond-64 benchmark leg launch. Each model enumerates the
offsets the kernel forms and asserts that:

- every global read and write falls inside the buffer the host allocated
  (site tensors [nq][n][2][T][T], packed FP32 at 3 floats per element or
  FP64 complex; features n x ld; outputs rows x ld; the refinement list of
  pairs + 1 int64 words whose last word holds the int32 count);
- every LDS index falls inside its array, and the workgroup's LDS fits the
  160 KB of a CU at the residency the launch bounds ask for;
- every thread of a workgroup reaches the same sequence of barriers (the
  barrier count is computed per thread from the control flow);
- the pair numbering is a bijection onto the pair set (the upper triangle
  for symmetric tasks) at every size the 32-bit pair count admits.

The kernels' float arithmetic is not modelled: only indices.
"""
import math

import numpy as np
import pytest

PACK = 3          # floats per packed FP32 complex element (-Im, Re, Im)
LDS_PER_CU = 160 * 1024


# ----------------------------------------------------------------- pair map

def pair_of(sym, na, nb, l):
    """qk_pair_of: local pair l -> (i, j); the double-precision inversion of
    the triangle count with the kernel's two correction loops."""
    if not sym:
        i = l // nb
        return i, l - i * nb
    n = na
    b2 = 2.0 * float(n) + 1.0
    r = int((b2 - math.sqrt(b2 * b2 - 8.0 * float(l))) * 0.5)
    r = min(max(r, 0), n - 1)
    before = lambda q: q * n - q * (q - 1) // 2
    while r > 0 and before(r) > l:
        r -= 1
    while r + 1 < n and before(r + 1) <= l:
        r += 1
    return r, r + (l - before(r))


def pair_of_vec(n, ls):
    """Vectorised copy of the symmetric branch (numpy float64 sqrt is the
    correctly rounded IEEE square root, as the device's)."""
    ls = np.asarray(ls, dtype=np.int64)
    b2 = 2.0 * float(n) + 1.0
    r = ((b2 - np.sqrt(b2 * b2 - 8.0 * ls.astype(np.float64))) * 0.5).astype(np.int64)
    r = np.clip(r, 0, n - 1)
    before = lambda q: q * n - q * (q - 1) // 2
    for _ in range(4):  # the correction loops move r by at most a step here
        down = (r > 0) & (before(r) > ls)
        r = np.where(down, r - 1, r)
        up = (r + 1 < n) & (before(r + 1) <= ls)
        r = np.where(up, r + 1, r)
    assert not np.any((r > 0) & (before(r) > ls))
    assert not np.any((r + 1 < n) & (before(r + 1) <= ls))
    return r, r + (ls - before(r))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 9, 16, 37, 250, 1000, 4000])
def test_pair_numbering_is_a_bijection_onto_the_triangle(n):
    tot = n * (n + 1) // 2
    i, j = pair_of_vec(n, np.arange(tot))
    assert np.all((0 <= i) & (i <= j) & (j < n))
    seen = np.zeros((n, n), dtype=np.int8)
    np.add.at(seen, (i, j), 1)
    assert np.array_equal(seen, np.triu(np.ones((n, n), dtype=np.int8)))
    for l in (0, tot // 3, tot - 1):  # scalar copy agrees with the vector one
        assert pair_of(True, n, n, l) == (int(i[l]), int(j[l]))


@pytest.mark.parametrize("n", [65535, 65536, 65537])
def test_pair_numbering_near_the_32_bit_pair_limit(n):
    """The wide launcher rejects more than 2^31 - 1 pairs; up to there the
    sqrt inversion with its corrections lands on the right row (checked on
    every row start and end, and on random pairs)."""
    tot = n * (n + 1) // 2
    rows = np.arange(n, dtype=np.int64)
    starts = rows * n - rows * (rows - 1) // 2
    for ls, want_i, want_j in ((starts, rows, rows), (starts + (n - 1 - rows), rows,
                                                       np.full(n, n - 1))):
        i, j = pair_of_vec(n, ls)
        assert np.array_equal(i, want_i) and np.array_equal(j, want_j)
    ls = np.random.default_rng(n).integers(0, tot, 200000)
    i, j = pair_of_vec(n, ls)
    assert np.all((0 <= i) & (i <= j) & (j < n))
    assert np.array_equal(i * n - i * (i - 1) // 2 + (j - i), ls)


def test_pair_lookup_over_a_task_table():
    """qk_pair_lookup walks the running pair counts of the table's tasks."""
    tasks = [(True, 9, 9), (False, 5, 9), (False, 9, 9), (True, 1, 1)]
    begin = [0]
    for sym, na, nb in tasks:
        begin.append(begin[-1] + (na * (na + 1) // 2 if sym else na * nb))
    seen = set()
    for p in range(begin[-1]):
        k = 0
        while k + 1 < len(tasks) and begin[k + 1] <= p:
            k += 1
        sym, na, nb = tasks[k]
        i, j = pair_of(sym, na, nb, p - begin[k])
        assert 0 <= i < na and 0 <= j < nb and (not sym or j >= i)
        seen.add((k, i, j))
    assert len(seen) == begin[-1]


# -------------------------------------------------------- wide sweep model

def wide_shape(T):
    TP = 16 if T < 16 else T
    NB = TP // 16
    return TP, NB, 64 * NB


def wide_lds_bytes(T):
    """WideSmem<T>: g[NB][NB][4][64] float2, b[TP][TP + 4] float2, red[NB]
    float, d2[NB] double (8-byte alignment of the double array)."""
    TP, NB, _ = wide_shape(T)
    g = NB * NB * 4 * 64 * 8
    b = TP * (TP + 4) * 8
    red = NB * 4
    off = g + b + red
    off = (off + 7) // 8 * 8
    return off + NB * 8


def wide_pair_accesses(T, nq, na, nb, i, j, fuse, ld_xr, ld_xc):
    """Every offset one pair's workgroup forms in wide_pair<T>, per thread.
    Returns the extreme offsets per buffer and the per-thread barrier counts."""
    TP, NB, nthr = wide_shape(T)
    kS = T * T * PACK
    kSlot = 2 * kS
    tid = np.arange(nthr)
    lane, w = tid & 63, tid >> 6
    g, c = lane >> 4, lane & 15
    lo, hi = {}, {}

    def note(buf, offs):
        offs = np.asarray(offs)
        if offs.size == 0:
            return
        lo[buf] = min(lo.get(buf, np.inf), int(offs.min()))
        hi[buf] = max(hi.get(buf, -np.inf), int(offs.max()))

    kper = (T * T + nthr - 1) // nthr
    barriers = np.zeros(nthr, dtype=np.int64)
    # BStage::load of B^s of site k (elements tid + nthr m below T*T; floats 1, 2)
    def bstage(k, s):
        for m in range(kper):
            e = tid + nthr * m
            ok = (T * T % nthr == 0) | (e < T * T)
            base = (k * nb + j) * kSlot + s * kS + e[ok] * PACK
            note("tb", base + 1)
            note("tb", base + 2)
            # BStage::store into sm.b[e / T][e % T]
            note("lds_b_row", e[ok] // T)
            note("lds_b_col", e[ok] % T)

    bstage(0, 0)
    rows_kb = [16 * kb + 4 * g + r for kb in range(NB) for r in range(4)]
    for k in range(nq):
        for s in range(2):
            barriers += 1                       # B^s staged
            if s == 0:
                bstage(k, 1)
            elif k + 1 < nq:
                bstage(k + 1, 0)
            if s == 0 and k > 0 and k % 8 == 0:
                note("lds_red", np.arange(NB))  # sm.red[0 .. NB)
            for row in rows_kb:                 # R: sm.b[row][16 q + c]
                note("lds_b_row", row)
                for q in range(NB):
                    note("lds_b_col", 16 * q + c)
            for q in range(NB):                 # G^s to sm.g[w][q][r][lane]
                for r in range(4):
                    note("lds_g", ((w * NB + q) * 4 + r) * 64 + lane)
            barriers += 1                       # G^s visible
            for kb in range(NB):                # L: A^s element (row, 16 w + c)
                for r in range(4):
                    row = 16 * kb + 4 * g + r
                    col = 16 * w + c
                    live = (row < T) & (col < T) if T < 16 else np.ones(nthr, bool)
                    base = (k * na + i) * kSlot + s * kS + (row * T + col)[live] * PACK
                    for f in range(3):
                        note("ta", base + f)
                    for q in range(NB):
                        note("lds_g", ((kb * NB + q) * 4 + r) * 64 + lane)
        if k % 8 == 7:
            note("lds_red", w[lane == 0])
    if fuse:
        for f0 in range(0, nq, nthr):
            f = tid + f0
            f = f[f < nq]
            note("xr", i * ld_xr + f)
            note("xc", j * ld_xc + f)
        note("lds_d2", w[lane == 0])
        barriers += 1
        note("lds_d2", np.arange(NB))
    barriers += 1                               # end of pair
    return lo, hi, barriers


# The shapes the GPU tests and the bond-64 leg launch: (T, nq, tasks) with a
# task (symmetric, na, nb, fuse).
WIDE_CASES = [
    (8, 8, [(True, 9, 9, True), (False, 5, 9, False), (False, 9, 9, False)]),
    (16, 10, [(True, 9, 9, True), (False, 5, 9, False), (False, 9, 9, False)]),
    (32, 12, [(True, 9, 9, True), (False, 5, 9, False), (False, 9, 9, False)]),
    (64, 14, [(True, 9, 9, True), (False, 5, 9, False), (False, 9, 9, False)]),
    (64, 40, [(True, 9, 9, True), (False, 5, 9, False), (False, 9, 9, False)]),
    (64, 784, [(False, 4, 8, False), (True, 8, 8, False)]),
    (64, 784, [(False, 32, 64, False)]),
]


def sample_pairs(sym, na, nb):
    tot = na * (na + 1) // 2 if sym else na * nb
    ls = sorted(set([0, 1, tot // 2, tot - 2, tot - 1]) & set(range(tot)))
    return [pair_of(sym, na, nb, l) for l in ls]


@pytest.mark.parametrize("T,nq,tasks", WIDE_CASES)
def test_wide_sweep_accesses_in_bounds(T, nq, tasks):
    TP, NB, nthr = wide_shape(T)
    per_cu = {8: 16, 16: 16, 32: 8, 64: 2}[T]
    assert wide_lds_bytes(T) * min(per_cu, 2 if T == 64 else per_cu) <= LDS_PER_CU
    assert T != 64 or 2 * wide_lds_bytes(64) <= LDS_PER_CU
    slot_floats = 2 * T * T * PACK
    for sym, na, nb, fuse in tasks:
        pairs = sample_pairs(sym, na, nb)
        if nq <= 16:  # small shapes: every pair
            tot = na * (na + 1) // 2 if sym else na * nb
            pairs = [pair_of(sym, na, nb, l) for l in range(tot)]
        ld_xr = ld_xc = nq
        for i, j in pairs:
            assert 0 <= i < na and 0 <= j < nb
            lo, hi, bar = wide_pair_accesses(T, nq if nq <= 16 else 17, na, nb, i, j, fuse,
                                             ld_xr, ld_xc)
            # longer chains are modelled on 17 sites (every branch of the site loop:
            # the rescale period, the last-site prefetch guard) and the
            # site-dependent offsets are checked at the last site below
            assert np.all(bar == bar[0]), "barrier count differs between threads"
            n_sites = nq if nq <= 16 else 17
            assert lo["tb"] >= 0 and hi["tb"] < n_sites * nb * slot_floats
            assert lo["ta"] >= 0 and hi["ta"] < n_sites * na * slot_floats
            assert lo["lds_b_row"] >= 0 and hi["lds_b_row"] < TP
            assert lo["lds_b_col"] >= 0 and hi["lds_b_col"] < TP + 4
            assert lo["lds_g"] >= 0 and hi["lds_g"] < NB * NB * 4 * 64
            if n_sites > 8:
                assert lo["lds_red"] >= 0 and hi["lds_red"] < NB
            if fuse:
                assert lo["xr"] >= 0 and hi["xr"] < na * ld_xr
                assert lo["xc"] >= 0 and hi["xc"] < nb * ld_xc
                assert hi["lds_d2"] < NB
            # last site of the full length: the largest site offsets
            kl = nq - 1
            assert ((kl * nb + j) * slot_floats + slot_floats - 1) < nq * nb * slot_floats
            assert ((kl * na + i) * slot_floats + slot_floats - 1) < nq * na * slot_floats
            # outputs (i, j) and, for symmetric tasks, (j, i) in rows x ld
            assert i * nb + j < na * nb and (not sym or j * nb + i < na * nb)


@pytest.mark.parametrize("T", [8, 16, 32, 64])
def test_wide_refinement_list_bounds(T):
    """The list holds at most one entry per pair (each pair's single thread 0
    appends itself at most once), so atomicAdd's slot stays below the pair
    count; the count word sits in the extra int64 after the list."""
    for sym, na, nb in ((True, 9, 9), (False, 5, 9), (False, 32, 64), (True, 8, 8)):
        tot = na * (na + 1) // 2 if sym else na * nb
        appended = np.arange(tot)  # the worst case: every pair above tau
        assert appended.max() < tot
        list_words = tot + 1
        assert tot * 8 + 4 <= list_words * 8  # count (int32) inside the last word


# ----------------------------------------------------- FP64 per-pair model

def big_shape(T):
    KR = 4 if T == 64 else (1 if T == 8 else 2)
    KC = 1 if T == 8 else 2
    GR, GC = T // KR, T // KC
    per_cu = 1 if T == 64 else (4 if T == 32 else 16)
    return KR, KC, GR, GC, GR * GC, T + 1, per_cu


@pytest.mark.parametrize("T", [8, 16, 32, 64])
def test_big_pair_sweep_accesses_in_bounds(T):
    KR, KC, GR, GC, nthr, P, per_cu = big_shape(T)
    lds = 2 * T * P * 16 + (nthr // 64) * 8
    assert lds <= 64 * 1024 or per_cu * lds <= LDS_PER_CU
    assert per_cu * lds <= LDS_PER_CU
    tid = np.arange(nthr)
    r0 = (tid // GC) * KR
    c0 = (tid % GC) * KC
    TT = T * T
    # E and G^s: rows r0 + x < T, columns b < T or c0 + y < T, pitch P
    rows = (r0[:, None] + np.arange(KR)[None, :]).ravel()
    cols = (c0[:, None] + np.arange(KC)[None, :]).ravel()
    assert rows.max() < T and cols.max() < T
    assert rows.max() * P + (T - 1) < T * P and (T - 1) * P + cols.max() < T * P
    # every (r0 + x, c0 + y) of E' is written by exactly one thread
    cover = np.zeros((T, T), dtype=np.int64)
    for x in range(KR):
        for y in range(KC):
            np.add.at(cover, (r0 + x, c0 + y), 1)
    assert np.all(cover == 1)
    # site reads A[s TT + a T + r0 + x], B[s TT + b T + c0 + y] inside a slot
    assert (TT + (T - 1) * T + rows.max()) < 2 * TT
    assert (TT + (T - 1) * T + cols.max()) < 2 * TT
    # the reduction slots: one per wavefront
    assert (nthr - 1) >> 6 < max(nthr // 64, 1)
    # barriers: per site 2 per s + 1 (max) + 1 (E written), per pair + 1 or 2
    # (fuse) + 1; no barrier sits under a thread-dependent branch
    assert nthr % 64 == 0


def test_big_list_kernel_reads_only_listed_pairs():
    """sweep_big_list_kernel reads *count once, walks q < count by grid
    stride, and looks up list[q]: a pair number below the table's total, so
    its task and (i, j) are those the matrix-core pass wrote."""
    for sym, na, nb in ((True, 9, 9), (False, 32, 64)):
        tot = na * (na + 1) // 2 if sym else na * nb
        listed = np.random.default_rng(1).permutation(tot)[: tot // 3]
        for q in range(len(listed)):
            i, j = pair_of(sym, na, nb, int(listed[q]))
            assert 0 <= i < na and 0 <= j < nb
