"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds no arithmetic of the transform itself: only workload
definitions (lattice sizes, batch sizes), seeded random signals and the
analysis windows that the workloads name.  Both the oracle (``oracle/``) and
the GPU tests/benchmark draw their inputs from here so that the two sides see
bit-identical data; neither side imports the other.

All generators return NumPy arrays in complex128 (or float64 for real
signals).  A single-precision run rounds these arrays to complex64 and the
oracle is then fed the rounded values upcast back to complex128.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

SEED_BASE = 13074569


@dataclasses.dataclass(frozen=True)
class Workload:
    """One transform configuration: signal length L, time step a, M channels,
    lattice offset lambda1/lambda2 (the relative shear of the lattice normal
    form, Section 2.1) and the batch size."""

    name: str
    L: int
    a: int
    M: int
    lam1: int
    lam2: int
    batch: int
    real_signal: bool = False

    @property
    def N(self) -> int:
        return self.L // self.a

    @property
    def b(self) -> int:
        return self.L // self.M

    @property
    def coeffs_per_signal(self) -> int:
        return self.M * self.N


# Quincunx lattice on a short signal: every stage can be checked exhaustively.
SMALL = Workload("small-L144-a6-M12-q12", 144, 6, 12, 1, 2, 1)
# The throughput workload: 64 signals of 2^18 samples, redundancy 8.
LARGE = Workload("quincunx-L262144-a64-M512-B64", 262144, 64, 512, 1, 2, 64)
# Long real signals on a lambda = 1/4 lattice.
PRECISION = Workload("chirps-L1048576-a128-M1024-l14-B16", 1048576, 128, 1024, 1, 4, 16, True)
# The differentiation workload.
GRADIENT = Workload("grad-L65536-a32-M256-B32", 65536, 32, 256, 1, 2, 32)

# The request mix of the serving workload.
SERVE_LENGTHS = (36864, 73728, 147456, 294912)
SERVE_AM = ((32, 256), (64, 512))
SERVE_LAMBDAS = ((1, 2), (1, 3), (2, 3))
SERVE_REQUESTS = 10000


def seed_for(config_index: int, signal_index: int) -> int:
    return SEED_BASE + 1000 * config_index + signal_index


def complex_normal(L: int, seed: int) -> np.ndarray:
    """i.i.d. circular complex normal CN(0,1): real and imaginary parts each
    N(0, 1/2)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(L)
    im = rng.standard_normal(L)
    return (re + 1j * im) * math.sqrt(0.5)


def complex_normal_batch(B: int, L: int, config_index: int, first: int = 0) -> np.ndarray:
    out = np.empty((B, L), dtype=np.complex128)
    for i in range(B):
        out[i] = complex_normal(L, seed_for(config_index, first + i))
    return out


def chirp_mixture(L: int, seed: int, n_chirps: int = 8, snr_db: float = 20.0) -> np.ndarray:
    """Real signal: a sum of linear chirps with seeded start/end frequencies
    (cycles per sample in [0, 1/2)) and phases, plus white Gaussian noise at
    the given SNR."""
    rng = np.random.default_rng(seed)
    f0 = rng.uniform(0.0, 0.5, n_chirps)
    f1 = rng.uniform(0.0, 0.5, n_chirps)
    ph = rng.uniform(0.0, 1.0, n_chirps)
    l = np.arange(L, dtype=np.float64)
    x = np.zeros(L)
    for i in range(n_chirps):
        x += np.cos(2 * np.pi * (ph[i] + f0[i] * l + (f1[i] - f0[i]) * l * l / (2.0 * L)))
    sigma2 = float(np.mean(x * x)) / (10.0 ** (snr_db / 10.0))
    x += rng.standard_normal(L) * math.sqrt(sigma2)
    return x


def gaussian_window(L: int, a: int, M: int) -> np.ndarray:
    """Full-length periodic Gaussian exp(-pi d(l)^2/(a M)), d(l) = min(l, L-l),
    normalised to unit l2 norm (complex128)."""
    l = np.arange(L)
    d = np.minimum(l, L - l).astype(np.float64)
    g = np.exp(-np.pi * d * d / (a * M))
    g /= np.linalg.norm(g)
    return g.astype(np.complex128)


def hann_window(L: int, Lg: int = 2048) -> np.ndarray:
    """Periodic Hann window of length Lg centred at l = 0 (signed positions
    -Lg/2 .. Lg/2-1), zero-padded to L, unit l2 norm (complex128)."""
    if Lg > L or Lg % 2:
        raise ValueError("Hann length must be even and at most L")
    g = np.zeros(L)
    j = np.arange(-Lg // 2, Lg // 2)
    g[j % L] = 0.5 * (1.0 + np.cos(2 * np.pi * j / Lg))
    g /= np.linalg.norm(g)
    return g.astype(np.complex128)


def round_to(x: np.ndarray, single: bool) -> np.ndarray:
    """Round to the precision of a run; the oracle then receives the rounded
    values upcast to double."""
    if single:
        if np.iscomplexobj(x):
            return x.astype(np.complex64).astype(np.complex128)
        return x.astype(np.float32).astype(np.float64)
    return x


def serving_plans() -> List[Tuple[int, int, int, int, int]]:
    """The 24 (L, a, M, lam1, lam2) plans of the serving mix."""
    plans = []
    for L in SERVE_LENGTHS:
        for a, M in SERVE_AM:
            for l1, l2 in SERVE_LAMBDAS:
                plans.append((L, a, M, l1, l2))
    return plans


# Fig. 2 shapes (Section 4.4): L = lcm(a, M) 2520 for these (a, M), and
# lambda = 1/lambda2 for lambda2 = 1..10 (lambda2 = 1 is the separable 0/1).
CROSSOVER_AM = ((32, 64), (40, 60), (60, 80))


def crossover_lattices() -> List[Tuple[int, int, int, int, int]]:
    """The 30 (L, a, M, lam1, lam2) lattices of the crossover experiment;
    2520 = lcm(1, ..., 10) makes every lambda2 feasible."""
    out = []
    for a, M in CROSSOVER_AM:
        L = a * M // math.gcd(a, M) * 2520
        for lam2 in range(1, 11):
            out.append((L, a, M, 1 if lam2 > 1 else 0, lam2))
    return out


def crossover_batch(L: int) -> int:
    """Signals per batch of the crossover experiment: about 2^22 samples."""
    return max(1, (1 << 22) // L)


def serving_requests(n: int = SERVE_REQUESTS, seed: int = seed_for(5, 0)):
    """Seeded request stream: for each request a plan index (uniform over the
    24 plans) and a signal seed."""
    rng = np.random.default_rng(seed)
    plans = serving_plans()
    idx = rng.integers(0, len(plans), n)
    return [(int(i), plans[int(i)], seed_for(5, 1 + k)) for k, i in enumerate(idx)]


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
