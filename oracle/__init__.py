"""Plain FP64 CPU oracle for the quantum-classical dual kernel.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this
package: only the test suite, the smoke check and the benchmark's CPU
baseline use it. It shares no code, header, table or helper with the HIP
library; the two meet only through the seeded arrays of ``synthdata``.

What it computes (paper: "Scalable Tensor Network Simulation for
Quantum-Classical Dual Kernel"):

* the feature state |psi(x)> = U(x)|0...0> of Eq. (6), for the benchmark
  encoding circuit (per layer: H on every qubit, RZ(2 x_k) on qubit k, then
  an open nearest-neighbour RZZ(2 (pi - x_k)(pi - x_{k+1})) chain; repeated
  L times) -- ``circuit``;
* the quantum kernel K_q = |<psi(x)|psi(y)>|^2 of Eq. (7), and the
  compute-uncompute amplitude of Eqs. (8)-(10), by brute-force statevector
  on up to ~16 qubits -- ``statevector``;
* the entangler-free closed forms (a product of per-qubit overlaps) --
  ``closed_form``;
* an exact path-sum transfer chain over computational-basis histories, for
  any qubit count and up to three layers -- ``pathsum``;
* the MPS simulation: per-sample TEBD build (entangler chains swept in
  alternating directions, SVD bond truncation at the orthogonality centre),
  and the pairwise transfer-matrix overlap sweep with power-of-two
  rescaling -- ``mps``;
* the RBF kernel of Eq. (3), the linear mix of Eq. (11) and the SVM
  decision values of Eqs. (4), (5) on kernel rows -- ``classical``;
* SVM training on a precomputed kernel: the dual of Eqs. (1)-(2) by
  sequential minimal optimisation with second-order pair selection, the
  bias of Eq. (5), and one-against-one voting -- ``svm``;
* kernel invariants and the tolerance gates used by the parity tests --
  ``checks``;
* the pre-processing of Section II-A: z-score, PCA to n components,
  min-max scaling -- ``preprocess``.

Pins (what ties each function to something other than itself) are listed in
the test-suite docstrings. ``mps.build_mps`` in the truncating regime
(chi_max below the exact bond dimension) is pinned only on <= 20 qubits
(including the 8-layer, chi_max 64 schedule of the truncating workload)
through the discarded-weight bound against exact statevectors; beyond that
it is parity unpinned (its own step-by-step replay is the reference).
"""
from . import circuit, statevector, closed_form, pathsum, mps, classical, checks, svm, preprocess  # noqa: F401
