"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random positions and charges and records the run
parameters of each workload.  It holds none of the Spectral Ewald arithmetic:
no window, no grid, no Green's function, no parameter rule.

Positions are uniform in the cubic box [0, L)^3 (the box of the paper's problem
statement, Section 2) in float64.  Charges follow one of the paper's
distributions (Section 7: uniform in [-1, 1]) or the configurations' own
(+-1 with exact neutrality; standard normal re-centred to zero sum).
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 171204732


def positions(rng: np.random.Generator, n: int, L: float) -> np.ndarray:
    """n points uniform in [0, L)^3, float64, shape (n, 3)."""
    x = rng.random((n, 3)) * L
    # guard the open upper end against rounding of r*L up to L
    np.minimum(x, np.nextafter(L, 0.0), out=x)
    return x


def charges(rng: np.random.Generator, n: int, kind: str) -> np.ndarray:
    """Charges of one of the kinds used by the workloads, float64, shape (n,).

    kind:
      "pm1"     exactly n/2 charges +1 and n/2 charges -1 in random order (n even)
      "normal"  standard normal, re-centred so that the sum is zero
      "uniform" uniform in [-1, 1], re-centred so that the sum is zero
      "raw_uniform" uniform in [-1, 1], not re-centred
    """
    if kind == "pm1":
        if n % 2:
            raise ValueError("pm1 charges need an even n")
        q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
        rng.shuffle(q)
        return q
    if kind == "normal":
        q = rng.standard_normal(n)
        return q - q.mean()
    if kind == "uniform":
        q = rng.uniform(-1.0, 1.0, n)
        return q - q.mean()
    if kind == "raw_uniform":
        return rng.uniform(-1.0, 1.0, n)
    raise ValueError(f"unknown charge kind {kind!r}")


def system(n: int, L: float, seed: int, kind: str = "pm1"):
    """(x, q) for one system drawn from its own seeded generator."""
    rng = np.random.default_rng(seed)
    x = positions(rng, n, L)
    q = charges(rng, n, kind)
    return x, q


# The five benchmark configurations.  xi is fixed here as a number; the rule
# that produced it (the k-space truncation estimate capped by the error
# pollution bound) lives in the oracle and the planner, and a test re-derives
# these values from the oracle.
CONFIGS = {
    "C1_3P": dict(D=3, N=1000, L=1.0, M=32, P=8, window="gaussian", xi=13.18,
                  charges="pm1", seed=SEED_BASE + 0, prec="f64"),
    "C2_0P": dict(D=0, N=20000, L=1.0, M=64, P=8, window="pkb", xi=22.56,
                  charges="pm1", seed=SEED_BASE + 1, prec="f32"),
    "C3_2P": dict(D=2, N=100000, L=1.0, M=96, P=8, window="pkb", xi=33.84,
                  charges="pm1", seed=SEED_BASE + 2, prec="f32"),
    "C4_1P": dict(D=1, N=1000000, L=1.0, M=160, P=8, window="pkb", xi=56.40,
                  charges="normal", seed=SEED_BASE + 3, prec="f32"),
}


# The batched configuration: 256 independent systems from batch_draw(), each
# with xi = 1.2 N^(1/3) / L, PKB window P = 10, grid from a 1e-7 relative
# tolerance, FP32.  P = 10 because forces must meet 1e-6 rms as well: with
# P = 8 the window alone leaves relative force errors near 1e-6 (the grid is
# then set by the error-pollution bound, and refining it does not help).
BATCH = dict(n_sys=256, seed=SEED_BASE + 4, P=10, window="pkb", tol_rel=1e-7, xi_coef=1.2, prec="f32",
             charges="pm1")


def batch_xi(N: int, L: float, coef: float = 1.2) -> float:
    """xi = coef * N^(1/3) / L: the splitting parameter of a batch system."""
    return coef * N ** (1.0 / 3.0) / L


def batch_systems(n_sys: int | None = None):
    """(list of system dicts with D, N, L, seed, xi, x, q) of the batched workload."""
    n = BATCH["n_sys"] if n_sys is None else n_sys
    out = []
    for s in batch_draw(n, BATCH["seed"]):
        x, q = system(s["N"], s["L"], s["seed"], BATCH["charges"])
        out.append(dict(s, xi=batch_xi(s["N"], s["L"], BATCH["xi_coef"]), x=x, q=q))
    return out


def config_system(name: str):
    c = CONFIGS[name]
    return system(c["N"], c["L"], c["seed"], c["charges"])


def batch_draw(n_sys: int = 256, seed: int = SEED_BASE + 4):
    """Draw the batched workload: n_sys independent systems.

    N is log-uniform in [500, 50000] rounded down to even, L uniform in
    [0.5, 2], the periodicity uniform over {3, 2, 1, 0}; charges +-1 neutral.
    Returns a list of dicts with keys D, N, L, seed (each system has its own
    seed so that any one of them can be regenerated alone).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_sys):
        n = int(math.floor(math.exp(rng.uniform(math.log(500), math.log(50000)))))
        n -= n % 2
        L = float(rng.uniform(0.5, 2.0))
        D = int(rng.choice([3, 2, 1, 0]))
        out.append(dict(D=D, N=n, L=L, seed=seed * 1000 + i))
    return out
