"""Pins of the oracle's block-structured entanglers (Section II-C: single-
qubit encoding layers interleaved with locally restricted, block-structured
entangling layers; a block product state). With blocks of B consecutive
qubits the RZZ chain keeps only the pairs inside a block, so the state is a
tensor product of the blocks' states and the kernel of Eq. (7) factorises:

    K(x, y) = prod_blocks K_chain(x_block, y_block)

with K_chain the open-chain kernel of each block on its own qubits. That
identity is checked against statevectors computed block by block (an
independent construction: separate small registers, no gate skipping), and
the oracle's MPS and path-sum routes are checked against the full
statevector with blocks. The MPS bonds at block boundaries are 1."""
import numpy as np
import pytest

from oracle import circuit, mps, pathsum, statevector as sv
from synthdata import gen_clusters


def blocks_of(n, B):
    return [list(range(s, min(s + B, n))) for s in range(0, n, B)]


def product_kernel(x, y, L, B):
    k = 1.0
    for blk in blocks_of(len(x), B):
        k *= sv.kernel_overlap(x[blk], y[blk], L, True)
    return k


@pytest.mark.parametrize("B", [2, 3, 4, 5])
@pytest.mark.parametrize("L", [1, 2, 3])
def test_statevector_with_blocks_factorises(B, L):
    X, _ = gen_clusters(4, 10, 700 + B + L)
    for i in range(4):
        for j in range(4):
            full = sv.kernel_overlap(X[i], X[j], L, B)
            prod = product_kernel(X[i], X[j], L, B)
            assert abs(full - prod) <= 1e-13 * max(1.0, prod)


def test_block_mask():
    assert circuit.entangler_mask(7, 3).tolist() == [True, True, False, True, True, False]
    assert circuit.entangler_mask(5, True).all() and not circuit.entangler_mask(5, False).any()
    assert circuit.entangler_mask(5, 5).all()   # one block over all qubits = the chain
    assert circuit.entangler_mask(5, 9).all()


def test_a_block_as_large_as_the_register_is_the_chain():
    X, _ = gen_clusters(3, 9, 77)
    for i in range(3):
        for j in range(3):
            assert abs(sv.kernel_overlap(X[i], X[j], 2, 9) - sv.kernel_overlap(X[i], X[j], 2, True)) < 1e-14


@pytest.mark.parametrize("n,B,L", [(10, 2, 2), (10, 3, 2), (11, 4, 3), (12, 5, 2), (12, 6, 4)])
def test_mps_route_with_blocks_equals_statevector(n, B, L):
    X, _ = gen_clusters(5, n, 800 + n + B)
    P = mps.pad_batch(mps.build_batch(X, L, 64, 1e-10, entangle=B))
    K, _ = mps.gram(P, P)
    ref = sv.gram(X, X, L, B)
    assert np.max(np.abs(K - ref)) < 1e-12


@pytest.mark.parametrize("n,B,L", [(10, 2, 1), (10, 3, 2), (10, 4, 3)])
def test_pathsum_with_blocks_equals_statevector(n, B, L):
    X, _ = gen_clusters(5, n, 900 + n + B)
    pairs = [(i, j) for i in range(5) for j in range(5)]
    ln = pathsum.ln_kernel_pairs(X, X, L, pairs, entangle=B)
    ref = np.array([np.log(sv.kernel_overlap(X[i], X[j], L, B)) for i, j in pairs])
    assert np.max(np.abs(ln - ref)) < 1e-10


@pytest.mark.parametrize("n,B,L", [(12, 4, 2), (13, 5, 3), (16, 8, 4)])
def test_bond_profile_of_block_product_states(n, B, L):
    """Bond k (between qubits k-1 and k) is 1 at block boundaries (k a
    multiple of B) and at most 2^min(L, c, B - c) inside a block, where c is
    the number of the block's qubits left of the cut."""
    X, _ = gen_clusters(3, n, 1000 + n)
    for x in X:
        _, chis = mps.build_mps(x, L, 64, 1e-10, entangle=B)
        for k in range(1, n):
            c = k % B
            if c == 0:
                assert chis[k] == 1, (k, chis)
            else:
                b_len = min(B, n - (k - c))
                assert chis[k] <= 2 ** min(L, c, b_len - c), (k, chis)
        assert max(chis) > 1


def test_planted_block_boundary_off_by_one_is_caught():
    """A mask that cuts after qubit k with k % B == 0 (one pair too early)
    is a different circuit: the factorisation pin sees it."""
    X, _ = gen_clusters(2, 10, 31)
    B, L = 3, 2
    wrong = np.array([k % B != 0 for k in range(9)])

    def state_with(x, mask):
        th = circuit.rzz_angles(x)
        psi = sv.zero_state(len(x))
        for _ in range(L):
            for k in range(len(x)):
                psi = sv._apply(psi, (k,), circuit.HADAMARD)
            for k in range(len(x)):
                psi = sv._apply(psi, (k,), circuit.rz(2.0 * x[k]))
            for k in range(len(x) - 1):
                if mask[k]:
                    psi = sv._apply(psi, (k, k + 1), circuit.rzz(th[k]))
        return psi.ravel()

    bad = abs(np.vdot(state_with(X[0], wrong), state_with(X[1], wrong))) ** 2
    good = product_kernel(X[0], X[1], L, B)
    assert abs(bad - good) > 1e-6 * good
