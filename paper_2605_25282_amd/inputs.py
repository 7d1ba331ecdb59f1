"""Seeded synthetic inputs shared by the HIP path, its tests and the benchmark.

This module holds no arithmetic of the method.  It only draws the random
variables of the initial measure and names the workloads:

* ``kl_coefficients`` draws the coefficients Y_k, Z_k ~ U(-1, 1) of the
  Karhunen-Loeve inlet perturbation (eq:karhunenExp, Sec. 2.3) for a range of
  realizations.  Realization m's coefficients depend on (seed, m) only, so
  ensembles drawn in batches, or restricted to a prefix, see the same samples
  (the nested sample sets of Sec. 3.1).
* The generator is the SplitMix64 output function of Steele, Lea and Flood
  ("Fast splittable pseudorandom number generators", OOPSLA 2014) used in
  counter mode: draw n of a stream with seed s is mix(s + (n + 1) * G) with
  G = 0x9E3779B97F4A7C15, i.e. the n-th output of a SplitMix64 generator
  seeded with s.  Draw n = m * 2K + c feeds coefficient c of realization m;
  its top 53 bits give a uniform u in [0, 1) and the coefficient is 2u - 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MUL1 = np.uint64(0xBF58476D1CE4E5B9)
_MUL2 = np.uint64(0x94D049BB133111EB)


def splitmix64(state: np.ndarray) -> np.ndarray:
    """SplitMix64 output (mixing) function applied elementwise to uint64 states."""
    z = np.asarray(state, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _MUL1
        z = (z ^ (z >> np.uint64(27))) * _MUL2
    return z ^ (z >> np.uint64(31))


def stream(seed: int, counters: np.ndarray) -> np.ndarray:
    """Outputs number ``counters`` (0-based) of a SplitMix64 stream seeded with ``seed``."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        st = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GOLDEN
    return splitmix64(st)


def kl_coefficients(seed: int, first: int, count: int, modes: int = 10) -> np.ndarray:
    """Coefficients for realizations first .. first+count-1, shape (count, 2*modes),
    float64 in [-1, 1).  Column 2(k-1) is Y_k, column 2(k-1)+1 is Z_k."""
    m = np.arange(first, first + count, dtype=np.uint64)[:, None]
    c = np.arange(2 * modes, dtype=np.uint64)[None, :]
    z = stream(seed, m * np.uint64(2 * modes) + c)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def random_fields(seed: int, shape, low: float = 0.1, high: float = 10.0) -> np.ndarray:
    """Seeded positive test fields (for statistics kernels), float64 in [low, high)."""
    n = int(np.prod(shape))
    z = stream(seed, np.arange(n, dtype=np.uint64))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (low + (high - low) * u).reshape(shape)


@dataclass(frozen=True)
class JetWorkload:
    """One Mach-2000 jet ensemble configuration on the domain
    [0, x_len] x [y_min, y_min + ny*dx] with square cells."""
    name: str
    nx: int
    ny: int
    m: int
    t_final: float
    x_len: float = 1.0
    y_min: float = -0.25

    @property
    def dx(self) -> float:
        return self.x_len / self.nx


# The Mach-2000 jet ensembles measured and tested here (domain [0,1]x[-0.25,0.25]).
WORKLOADS = {
    "jet128": JetWorkload("jet128", 128, 64, 8, 1e-4),
    "jet640": JetWorkload("jet640", 640, 320, 64, 1e-3),
    "jet1280": JetWorkload("jet1280", 1280, 640, 256, 1e-3),
    "jet320": JetWorkload("jet320", 320, 160, 128, 1e-3),
    "jet5056": JetWorkload("jet5056", 5056, 2528, 1000, 1e-3),
}

# The paper's own study (Sec. 3.3): domain [0, 2.5] x [-1, 1], four nested grids,
# M = 1000, statistics at t = 0.0005 k, k = 1..7.
PAPER_GRIDS = {
    f"paper{nx}": JetWorkload(f"paper{nx}", nx, nx * 4 // 5, 1000, 0.0035, x_len=2.5, y_min=-1.0)
    for nx in (500, 1000, 2000, 4000)
}
PAPER_CHECKPOINTS = tuple(0.0005 * k for k in range(1, 8))

DEFAULT_SEED = 2605
