"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws numbers; it contains none of the solver's arithmetic.
Layout: band-major ``bands`` of shape (2k+1, n) with ``bands[d + k, i] = A[i, i+d]``
and right-hand sides of shape (n, m), row-major.

Draw order (identical for every consumer):
  1. all 2k+1 diagonals as U[-1, 1];
  2. entries outside the matrix (i + d outside [0, n)) set to zero;
  3. the main diagonal overwritten by the dominance rule;
  4. the right-hand sides, N(0, 1).

Dominance rules
  ``strict``  a_ii = 2k + 1 + |u_ii|            (strictly dominant)
  ``weak``    a_ii = 1.05 * sum_{j != i} |a_ij|  (weakly dominant)
  ``theta``   a_ii = theta * sum_{j != i} |a_ij|  (non-dominant for theta < 1)
"""
from dataclasses import dataclass

import numpy as np


def make_band(n, k, seed=0, rule="strict", theta=1.05, rng=None):
    rng = np.random.default_rng(seed) if rng is None else rng
    bands = rng.uniform(-1.0, 1.0, size=(2 * k + 1, n))
    for d in range(-k, k + 1):
        if d < 0:
            bands[d + k, : -d] = 0.0
        elif d > 0:
            bands[d + k, n - d:] = 0.0
    if rule == "strict":
        bands[k] = 2 * k + 1 + np.abs(bands[k])
    elif rule in ("weak", "theta"):
        off = np.abs(bands).sum(axis=0) - np.abs(bands[k])
        bands[k] = (1.05 if rule == "weak" else theta) * off
    else:
        raise ValueError(rule)
    return bands


def make_rhs(n, m, rng):
    return rng.standard_normal(size=(n, m))


def make_problem(n, k, m, seed=0, rule="strict", theta=1.05):
    """(bands, f) drawn in the fixed order above from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    bands = make_band(n, k, rule=rule, theta=theta, rng=rng)
    return bands, make_rhs(n, m, rng)


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    k: int
    p: int
    r: int
    m: int
    rule: str
    seed: int = 0


# The five workloads of the method's evaluation plan, at full size.
SMALL_EXACT = Workload("n4096_k8_p4_r8_m1_strict", 4096, 8, 4, 8, 1, "strict")
LARGE = Workload("n4194304_k32_p1024_m16_weak", 1 << 22, 32, 1024, 8, 16, "weak")
GRAD = Workload("n1048576_k16_p256_r8_m1_strict", 1 << 20, 16, 256, 8, 1, "strict")


def batched_systems(count=4096, seed=0):
    """Per-system (n, k, r, nrhs, seed) for the batched workload: n log-uniform in
    [2^10, 2^16], k uniform over {4, 16, 64}, r = k / 2, nrhs uniform in [1, 32];
    system s draws from default_rng([seed, s])."""
    out = []
    for s in range(count):
        rng = np.random.default_rng([seed, s])
        n = int(round(2.0 ** rng.uniform(10.0, 16.0)))
        k = int(rng.choice([4, 16, 64]))
        m = int(rng.integers(1, 33))
        out.append((n, k, k // 2, m, (seed, s)))
    return out


def gaussian_test_matrices(p, k, ell, seed=0):
    """Gaussian test matrices of the randomized spike SVD, shape (p, 2, k, ell):
    [j, 0] for the spike V_j, [j, 1] for W_j, entries N(0, 1) from
    default_rng([seed, 7])."""
    return np.random.default_rng([seed, 7]).standard_normal((p, 2, k, ell))
