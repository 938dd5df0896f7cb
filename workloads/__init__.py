"""Seeded synthetic inputs shared by the test oracle and the device path.

This module holds no arithmetic of the method: it only draws random numbers
from fixed seeds and names the workloads (chain length, field strength,
boundary condition, Krylov dimension, time step).  Both the oracle and the
device path receive the same arrays from here and do all physics themselves.

The paper's workloads are synthetic model instances (Sec. 4: a Neel initial
state on a clean or quasiperiodic chain; Sec. 5: L=28 at half filling evolved
to t=100), so nothing here stands in for an external dataset.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Inverse golden ratio, the quasiperiodicity of the on-site field (Sec. 2,
# "Models").  A model parameter, passed to both sides as a plain number.
BETA_GOLDEN = (math.sqrt(5.0) - 1.0) / 2.0


def phases(n: int, seed: int = 0) -> np.ndarray:
    """n phases phi ~ U[0, 2*pi) from numpy's PCG64 generator with `seed`."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * math.pi, n)


def random_complex(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """n complex numbers with independent standard-normal real/imag parts."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return z.astype(dtype)


def random_fields(L: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """L uniform fields in [-scale, scale): an arbitrary (non-quasiperiodic) field set."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, L)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One named model instance and its time grid."""
    name: str
    L: int
    h: float
    pbc: bool
    m: int
    dt: float
    t_end: float
    jxy: float = 1.0
    jz: float = 1.0
    n_phases: int = 1
    seed: int = 0

    @property
    def n_up(self) -> int:
        return self.L // 2

    def phis(self) -> np.ndarray:
        return phases(self.n_phases, self.seed)


# The small periodic chain the oracle finishes in seconds (L=16, h=1.5, m=30,
# dt=0.1 to t=10), the mid-size chain (L=24), the metric chain (L=28, periodic,
# h=1.5, m=30, dt=0.1; the paper's strong-scaling size of Sec. 5), the batched
# L=20 set, the gradient chain and the large L=30 chain.
WORKLOADS = {
    "xxz_L16_pbc": Workload("xxz_L16_pbc", 16, 1.5, True, 30, 0.1, 10.0),
    "xxz_L24_obc": Workload("xxz_L24_obc", 24, 1.0, False, 30, 0.1, 100.0),
    "xxz_L24_pbc": Workload("xxz_L24_pbc", 24, 1.0, True, 30, 0.1, 100.0),
    "xxz_L28_pbc": Workload("xxz_L28_pbc", 28, 1.5, True, 30, 0.1, 100.0),
    "xxz_L20_batch64": Workload("xxz_L20_batch64", 20, 2.0, True, 30, 0.1, 50.0, n_phases=64),
    "xxz_L20_grad": Workload("xxz_L20_grad", 20, 1.5, True, 30, 0.1, 5.0),
    "xxz_L30_pbc": Workload("xxz_L30_pbc", 30, 2.0, True, 20, 0.05, 100.0),
}


def log_times(t_min: float = 1e-2, t_max: float = 100.0, n: int = 200) -> np.ndarray:
    """Log-spaced output times used for the mid-size chain."""
    return np.logspace(math.log10(t_min), math.log10(t_max), n)
