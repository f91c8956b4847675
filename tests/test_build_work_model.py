"""The host model of the build's one-sided Jacobi rule (tests/build_work_model.py)
computes what a one-sided Jacobi must: the singular values of LAPACK's SVD,
on random complex matrices of the merged shapes (square, tall, wide, odd
column counts, rank-deficient); its sweep counts are small for a matrix
that is already column-orthogonal and grow for a dense one; and the FLOP
tally of a step is the stated formula."""
import numpy as np
import pytest

from tests.build_work_model import jacobi_model, round_robin_rounds, step_flop


@pytest.mark.parametrize("R,C", [(8, 8), (16, 8), (8, 16), (32, 32), (12, 7), (64, 64)])
def test_singular_values_match_lapack(R, C):
    rng = np.random.default_rng(R * 100 + C)
    X = rng.normal(size=(R, C)) + 1j * rng.normal(size=(R, C))
    sv, sweeps, rot = jacobi_model(X)
    ref = np.linalg.svd(X, compute_uv=False)
    assert np.allclose(sv[: len(ref)], ref, rtol=1e-12, atol=1e-12 * ref[0])
    assert 2 <= sweeps < 40 and rot > 0


def test_rank_deficient_columns_stay_at_zero():
    rng = np.random.default_rng(7)
    B = rng.normal(size=(16, 4)) + 1j * rng.normal(size=(16, 4))
    X = B @ (rng.normal(size=(4, 12)) + 1j * rng.normal(size=(4, 12)))
    sv, _, _ = jacobi_model(X)
    ref = np.linalg.svd(X, compute_uv=False)
    assert np.allclose(sv[:4], ref[:4], rtol=1e-11)
    assert (sv[4:] < 1e-10 * sv[0]).all()


def test_orthogonal_columns_need_one_sweep():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(32, 16)) + 1j * rng.normal(size=(32, 16)))
    _, sweeps, rot = jacobi_model(Q * np.arange(1, 17))
    assert sweeps == 1 and rot == 0


@pytest.mark.parametrize("C", [2, 4, 10, 128])
def test_rounds_cover_every_pair_once(C):
    met = set()
    for ip, iq in round_robin_rounds(C):
        for a, b in zip(ip, iq):
            key = (min(a, b), max(a, b))
            assert a != b and key not in met
            met.add(key)
    assert len(met) == C * (C - 1) // 2


def test_step_flop_formula():
    R, C, m, keep, S, rot = 128, 128, 64, 64, 3, 1000
    assert step_flop(R, C, m, keep, S, rot) == (
        8 * R * C * m + S * (C * (C - 1) // 2) * 16 * R + rot * 14 * R + 8 * keep * R * C)


def test_qr_preconditioned_jacobi_keeps_the_singular_values():
    """Jacobi on R^H after a QR with column pivoting (once, or with a second
    QR) has the singular values of the original matrix, and on a strongly
    graded matrix needs fewer sweeps than Jacobi on the matrix itself."""
    pytest.importorskip("scipy")
    from tests.build_work_model import preconditioned_jacobi
    rng = np.random.default_rng(11)
    U, _ = np.linalg.qr(rng.normal(size=(48, 48)) + 1j * rng.normal(size=(48, 48)))
    V, _ = np.linalg.qr(rng.normal(size=(48, 48)) + 1j * rng.normal(size=(48, 48)))
    s = 10.0 ** -np.linspace(0, 10, 48)
    X = (U * s) @ V.conj().T
    ref = np.linalg.svd(X, compute_uv=False)
    _, plain, _ = jacobi_model(X)
    for twice in (False, True):
        sv, sweeps, _ = preconditioned_jacobi(X, twice)
        assert np.allclose(sv[:24], ref[:24], rtol=0, atol=1e-13 * ref[0])
        assert sweeps < plain
