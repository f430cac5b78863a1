"""Seeded synthetic inputs for PTHR runs: couplings, temperature grids and the
named workloads.

This module holds none of the method's arithmetic; the GPU library, the tests
and the benchmark all draw their inputs from it.

* Couplings (paper Sec. 2): J_ij ~ N(0, 1), one value per bond, stored as
  ``J[s][d][i]`` for the bond joining site ``i = x + L*(y + L*z)`` and
  ``i + e_d``.  Every sample has its own numpy generator seeded with
  ``(seed, global sample id)``, so any subset of a large batch can be
  regenerated on its own.
* Temperatures (paper App. A.2): ``n_temps`` values uniformly spaced between
  ``t_min`` and ``t_max``, both included.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def couplings(L: int, n_samples: int, seed: int = 1, first_sample: int = 0,
              dtype=np.float64) -> np.ndarray:
    """Gaussian couplings [n_samples][3][L^3] for samples first_sample.. ."""
    V = L ** 3
    out = np.empty((n_samples, 3, V), dtype=np.float64)
    for s in range(n_samples):
        rng = np.random.default_rng([seed, first_sample + s])
        out[s] = rng.standard_normal((3, V))
    return out.astype(dtype, copy=False)


def temperatures(t_min: float, t_max: float, n_temps: int) -> np.ndarray:
    """Uniform grid with both endpoints included; the last value is t_max exactly."""
    step = (t_max - t_min) / (n_temps - 1)
    T = np.array([t_min + k * step for k in range(n_temps)], dtype=np.float64)
    T[-1] = t_max
    return T


@dataclass
class Workload:
    name: str
    L: int
    n_samples: int
    n_replicas: int
    n_temps: int
    t_min: float
    t_max: float
    n_reservoir: int
    precision: str            # "fp64" or "fp32"
    emcs_total: float         # length of the full run, in EMCS
    sweeps_per_emcs: int = 10
    er_sweeps_per_emcs: int = 240
    t_acu: float = 1.0
    seed: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def V(self) -> int:
        return self.L ** 3

    def temperatures(self) -> np.ndarray:
        return temperatures(self.t_min, self.t_max, self.n_temps)

    def couplings(self, n_samples: int | None = None, first_sample: int = 0) -> np.ndarray:
        n = self.n_samples if n_samples is None else n_samples
        return couplings(self.L, n, self.seed, first_sample)


# The five workloads the method is exercised on (sizes from the paper's setting:
# Gaussian couplings, uniform temperature grids, 4 reservoir clones per replica
# group swept 960/4 = 240 times per EMCS).
WORKLOADS = {
    "l4_single": Workload("l4_single", 4, 1, 2, 8, 0.5, 1.6, 0, "fp64", 1e4),
    "l8_fp64": Workload("l8_fp64", 8, 256, 4, 20, 0.3, 1.6, 4, "fp64", 1e5),
    "l12_fp64": Workload("l12_fp64", 12, 512, 4, 28, 0.2, 1.6, 4, "fp64", 1e6),
    "l12_fp32": Workload("l12_fp32", 12, 512, 4, 28, 0.2, 1.6, 4, "fp32", 1e6),
    "l16_fp32": Workload("l16_fp32", 16, 1024, 4, 36, 0.2, 1.6, 4, "fp32", 1e7),
}

# Mixed-size batch: L in {8,...,16} with n_temps growing linearly from 16 to 36.
MIXED_BATCH = [
    Workload(f"mixed_l{L}", L, S, 4, NT, 0.2, 1.6, 4, "fp32", 1e7)
    for L, S, NT in ((8, 512, 16), (10, 384, 21), (12, 256, 26), (14, 192, 31), (16, 128, 36))
]
