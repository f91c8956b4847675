"""The benchmark's algorithmic FLOP count (the numerator of its roofline
fraction) against closed forms. Per pair, sum over sites k of
16 (chi^A_k chi^B_k chi^B_{k+1} + chi^A_{k+1} chi^A_k chi^B_{k+1}) real FLOP
on realized bonds (one complex MAC = 8 real FLOP; Eqs. (9), (10) as two
matrix products per physical index). For the 2-layer circuit the bonds are
1, 2, 4, ..., 4, 2, 1, which gives 2048 (d - 4) + 1728 per pair for d >= 4."""
import numpy as np
import pytest

import bench


def two_layer_bonds(d):
    return np.array([min(2 ** k, 2 ** (d - k), 4) for k in range(d + 1)], dtype=np.int32)


@pytest.mark.parametrize("d", [4, 5, 8, 64, 784])
def test_two_layer_closed_form(d):
    chi = two_layer_bonds(d)[None, :]
    assert bench.algorithmic_flops(chi, chi, False) == 2048 * (d - 4) + 1728


def test_brute_force_and_symmetric_count():
    rng = np.random.default_rng(5)
    d = 9
    A = rng.integers(1, 5, size=(3, d + 1))
    B = rng.integers(1, 5, size=(4, d + 1))
    A[:, 0] = A[:, -1] = B[:, 0] = B[:, -1] = 1

    def pair(a, b):
        return sum(16 * (a[k] * b[k] * b[k + 1] + a[k + 1] * a[k] * b[k + 1]) for k in range(d))

    full = sum(pair(a, b) for a in A for b in B)
    assert bench.algorithmic_flops(A, B, False) == full
    # symmetric: the upper triangle with its diagonal
    tri = sum(pair(A[i], A[j]) for i in range(3) for j in range(i, 3))
    assert bench.algorithmic_flops(A, A, True) == tri


def test_bond_64_profile():
    """784 sites with bonds min(2^k, 2^(784-k), 64): the per-pair figure the
    bond-64 sweep leg divides by."""
    d = 784
    chi = np.array([min(2 ** min(k, 30), 2 ** min(d - k, 30), 64) for k in range(d + 1)])[None]
    assert bench.algorithmic_flops(chi, chi, False) == 6483195584


def test_pathsum_flop_count():
    """The path-sum's FLOP per pair, counted from its operations: at L = 2
    each bond applies 12 butterflies (3 lines x 4 state pairs; 4 sums, 2
    products, 4 FMAs = 14 FLOP) and one shared-line phase (a complex product,
    6), each site 7 complex products of the weight (6 each; the first site
    skips the bond); at L = 1, 1 butterfly, the phase and 3 weight products."""
    from bench import pathsum_flops
    assert pathsum_flops(784, 2, 1) == 783 * (12 * 14 + 6 + 7 * 6) + 42
    assert pathsum_flops(784, 1, 1) == 783 * (14 + 6 + 3 * 6) + 18
    assert pathsum_flops(1, 2, 10) == 420.0
    # L = 3: 80 butterflies, the phase, q^3 / r^3, 16 cross products, 32 states
    assert pathsum_flops(3, 3, 1) == 2 * (80 * 14 + 6 + 52 * 6) + 52 * 6


def test_launch_shape_from_the_tuning_table():
    """The headline's launch shape is read from the tuning entry of its bond
    bound and qubit bucket (ceil(log2 784) = 10), only when that entry was
    tuned for the form that runs; otherwise the library defaults (2, 4)."""
    table = "2 1 5 1 4 0.07\n4 9 5 2 2 2.3\n4 10 5 1 8 3.46\n4 10 0 2 4 9.0\n"
    assert bench.launch_shape(table, 4, 784, 5) == (1, 8)
    assert bench.launch_shape(table, 4, 512, 5) == (2, 2)
    assert bench.launch_shape(table, 4, 784, 1) == (2, 4)
    assert bench.launch_shape("", 4, 784, 5) == (2, 4)
    assert bench.launch_shape(table, 2, 2, 5) == (1, 4)


def test_traffic_is_reported_only_for_its_source_and_launch_shape(monkeypatch, tmp_path):
    import hashlib
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel")
    h = hashlib.sha256(b"kernel").hexdigest()[:16]
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC", {
        "a": {"source": "k.hip", "sha256_prefix": h, "bytes": 5.0, "shape": (1, 8)},
        "b": {"source": "k.hip", "sha256_prefix": h, "bytes": 7.0},
        "c": {"source": "k.hip", "sha256_prefix": "0" * 16, "bytes": 9.0}})
    assert bench.traffic_for("a", (1, 8)) == 5.0
    assert bench.traffic_for("a", (2, 4)) is None
    assert bench.traffic_for("a") is None
    assert bench.traffic_for("b") == 7.0
    assert bench.traffic_for("c") is None
    assert bench.traffic_for("missing") is None


def test_all_pairs_gap_counts_unique_pairs_only():
    """The chosen-vs-plain comparison covers the train upper triangle (with
    the diagonal) and every test row; the lower train triangle (a mirror) is
    ignored, and two -inf logs (an exactly zero amplitude) count as equal."""
    torch = pytest.importorskip("torch")
    ntr, nte = 5, 3
    z = lambda r, c: torch.zeros((r, c), dtype=torch.float64)
    plain = {"ln": z(ntr, ntr), "kq": z(ntr, ntr), "k": z(ntr, ntr)}
    plain_te = {"ln": z(nte, ntr), "kq": z(nte, ntr), "k": z(nte, ntr)}
    ch = {k: (v.clone(), plain_te[k].clone()) for k, v in plain.items()}
    ch["ln"][0][3, 1] = 5.0          # lower triangle: not a unique pair
    ch["ln"][0][1, 3] = 2e-3         # upper triangle
    ch["ln"][0][2, 2] = 5e-4         # diagonal
    ch["ln"][1][2, 4] = -3e-3        # test row
    ch["ln"][0][0, 4] = -float("inf")
    plain["ln"][0, 4] = -float("inf")
    ch["kq"][1][0, 0] = 1e-7
    ch["k"][0][4, 4] = 2e-6
    res = bench.all_pairs_gap(ch, plain, plain_te, ntr)
    assert res["max_abs_dln"] == pytest.approx(3e-3)
    assert res["pairs_above_ln_gate_1e-3"] == 2
    assert res["pairs_above_ln_1e-4"] == 3
    assert res["max_abs_dkq"] == pytest.approx(1e-7)
    assert res["max_abs_dk"] == pytest.approx(2e-6)
