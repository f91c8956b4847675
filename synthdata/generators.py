"""Seeded synthetic stand-ins for the paper's inputs.

The paper feeds Fashion-MNIST images (28x28 grayscale, flattened to 784
features, 10 classes; Section II-A) through standardisation, PCA and min-max
scaling. That dataset is not available here, so two generators produce inputs
of the same shapes and value ranges:

* ``gen_clusters``: 10 Gaussian class clusters in [0, pi]^d (means drawn from
  U[0.5, 2.6], sigma 0.3, clipped to [0, pi]).
* ``gen_images``: 28x28 "images", one smooth random field per class (a
  Gaussian-filtered white-noise field, min-max scaled to [0, 1]) plus 0.02
  pixel noise, clipped to [0, 1], scaled by pi and flattened row-major.

Labels are ``i mod 10``. The train rows come first, then the test rows, all
from one draw of the class means. Every draw uses ``numpy.random.default_rng``
(PCG64) with the seed listed in ``CONFIGS``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_CLASSES = 10


def gen_clusters(n: int, d: int, seed, n_classes: int = N_CLASSES,
                 mu_low: float = 0.5, mu_high: float = 2.6,
                 sigma: float = 0.3):
    """Return (x, labels): x is (n, d) float64 in [0, pi], labels i mod 10.

    Draw order: class means (n_classes x d) first, then the (n x d) noise.
    """
    rng = np.random.default_rng(seed)
    mu = rng.uniform(mu_low, mu_high, size=(n_classes, d))
    labels = np.arange(n) % n_classes
    noise = rng.standard_normal((n, d))
    x = np.clip(mu[labels] + sigma * noise, 0.0, math.pi)
    return np.ascontiguousarray(x, dtype=np.float64), labels


def gen_images(n: int, seed, side: int = 28, smooth_px: float = 3.0,
               pixel_noise: float = 0.02, n_classes: int = N_CLASSES):
    """Return (x, labels): x is (n, side*side) float64 in [0, pi].

    Draw order: one (side x side) white-noise field per class, then the
    (n x side*side) pixel noise.
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    fields = np.empty((n_classes, side, side))
    for c in range(n_classes):
        f = gaussian_filter(rng.standard_normal((side, side)), sigma=smooth_px,
                            mode="wrap")
        lo, hi = f.min(), f.max()
        fields[c] = (f - lo) / (hi - lo)
    labels = np.arange(n) % n_classes
    noise = rng.standard_normal((n, side * side))
    x = np.clip(fields.reshape(n_classes, -1)[labels] + pixel_noise * noise,
                0.0, 1.0) * math.pi
    return np.ascontiguousarray(x, dtype=np.float64), labels


def gen_requests(seed, rate_per_s: float, duration_s: float,
                 dims=(16, 64, 256, 784), max_rows: int = 64):
    """Open-loop Poisson request stream.

    Returns a list of dicts with keys ``t`` (arrival offset in seconds),
    ``d`` (feature dimension), ``n_rows`` (1..max_rows) and ``w`` (mixing
    weight in [0, 1]). Draw order per request: inter-arrival gap, d index,
    row count, w.
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        out.append({
            "t": t,
            "d": int(dims[rng.integers(len(dims))]),
            "n_rows": int(rng.integers(1, max_rows + 1)),
            "w": float(rng.uniform(0.0, 1.0)),
        })
    return out


def gen_isometry_mps(n: int, nq: int, chi_max: int, seed, distinct_interior: int = 16):
    """Random left-canonical MPS with the widest bond profile a chi_max cap
    allows: chi_k = min(2^k, 2^(nq - k), chi_max). Timing and invariant
    inputs for the overlap sweep at large bond dimensions; they stand for no
    circuit.

    Returns (chi, tensors) in the library's import layout: chi int32
    (n, nq + 1), tensors complex128 [nq][n][2][T][T] with T = chi_max and
    tensors[k, i, s, a, b] = A_i^s[a][b] of site k. Each site tensor is the Q
    factor of a complex Gaussian (2 chi_l) x chi_r matrix, row s chi_l + a
    holding A^s[a][:], so sum_s A^{s dagger} A^s = I and every state has
    unit norm. Sites with chi_l = chi_r = chi_max cycle through
    ``distinct_interior`` draws per sample (saves host time at nq = 784).
    Draw order: per sample, the distinct interior draws, then every other
    site left to right.
    """
    rng = np.random.default_rng(seed)
    T = chi_max
    chi = np.array([min(2 ** min(k, 30), 2 ** min(nq - k, 30), chi_max)
                    for k in range(nq + 1)], dtype=np.int32)

    def draw(cl, cr):
        m = rng.standard_normal((2 * cl, cr)) + 1j * rng.standard_normal((2 * cl, cr))
        q, _ = np.linalg.qr(m)
        return q.reshape(2, cl, cr)

    tens = np.zeros((nq, n, 2, T, T), dtype=np.complex128)
    for i in range(n):
        inner = [draw(T, T) for _ in range(distinct_interior)]
        u = 0
        for k in range(nq):
            cl, cr = int(chi[k]), int(chi[k + 1])
            if cl == T and cr == T:
                tens[k, i] = inner[u % distinct_interior]
                u += 1
            else:
                tens[k, i, :, :cl, :cr] = draw(cl, cr)
    return np.tile(chi, (n, 1)), tens


@dataclass(frozen=True)
class Config:
    name: str
    generator: str          # "clusters" or "images"
    n_train: int
    n_test: int
    d: int
    n_layers: int
    chi_max: int
    cutoff: float
    w: float = 0.5
    seed: object = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)


def _c4_seeds():
    return np.random.SeedSequence(4).spawn(10)


C4_DIMS = (2, 4, 8, 16, 32, 64, 128, 256, 512, 784)
C5_DIMS = (16, 64, 256, 784)

CONFIGS = {
    # 200 samples x 8 features, 1 layer, no binding truncation, complex128.
    "C1": Config("C1", "clusters", 200, 0, 8, 1, 16, 1e-10, seed=1),
    # 2000 train + 500 test, 64 features, 2 layers, chi_max 32.
    "C2": Config("C2", "clusters", 2000, 500, 64, 2, 32, 1e-10, seed=2),
    # 4000 train + 1000 test 28x28 images, 2 layers, chi_max 64.
    "C3": Config("C3", "images", 4000, 1000, 784, 2, 64, 1e-10, seed=3),
    # 10 feature dimensions, 1000 samples each, one launch; chi_max per d.
    "C4": Config("C4", "clusters", 1000, 0, 0, 2, 64, 1e-10, seed=4,
                 extra={"dims": C4_DIMS}),
    # serving: 5000 support samples per d, Poisson requests.
    "C5": Config("C5", "clusters", 5000, 0, 0, 2, 64, 1e-10, seed=5,
                 extra={"dims": C5_DIMS, "rate": 200.0, "stream_seed": 55}),
    # truncating regime: 1000 train + 250 test images, 8 layers, chi_max 64
    # (the bonds would reach 2^8 without the cap).
    "S1": Config("S1", "images", 1000, 250, 784, 8, 64, 1e-10, seed=6),
}


def config_inputs(name: str, d: int | None = None, n_train: int | None = None,
                  n_test: int | None = None):
    """Inputs for a named configuration: returns (x_train, x_test, labels).

    ``n_train``/``n_test`` may shrink a config (same seed, same generator).
    The generators fill their noise arrays row by row, so a shrunk draw is a
    row prefix of the full draw: train rows are rows [0, n_train), test rows
    are rows [n_train, n_train + n_test).
    For C4/C5 pass ``d``; each d gets its own spawned seed.
    """
    c = CONFIGS[name]
    ntr = c.n_train if n_train is None else n_train
    nte = c.n_test if n_test is None else n_test
    if name == "C4":
        seeds = _c4_seeds()
        seed = seeds[C4_DIMS.index(d)]
        dd = d
    elif name == "C5":
        seeds = np.random.SeedSequence(5).spawn(len(C5_DIMS))
        seed = seeds[C5_DIMS.index(d)]
        dd = d
    else:
        seed = c.seed
        dd = c.d
    if c.generator == "images":
        x, lab = gen_images(ntr + nte, seed)
    else:
        x, lab = gen_clusters(ntr + nte, dd, seed)
    return x[:ntr], x[ntr:], lab


def chi_cap(name: str, d: int) -> int:
    """Bond-dimension cap of a config (C4 uses min(2^(d/2), 64))."""
    if name == "C4":
        return int(min(2 ** (d // 2), 64))
    return CONFIGS[name].chi_max
