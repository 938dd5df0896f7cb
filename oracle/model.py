"""Model definition (Sec. 2, "Models", Eq. (1)) -- oracle, test infrastructure.

Readings taken here (the paper writes Eq. (1) for hard-core bosons with
hopping t, repulsion V and field h*cos(2*pi*beta*i + phi)*n_i):

* Spin language.  n_i = S^z_i + 1/2 and c_i^dagger = S^+_i turn Eq. (1) into
  an XXZ chain  H = sum_b [ (jxy/2)(S^+_a S^-_c + h.c.) + jz S^z_a S^z_c ]
  + sum_i h_i S^z_i  with t = jxy/2, V = jz.  With periodic bonds the
  linear terms that V*n*n leaves behind add up to V*S^z_total, a constant in
  a fixed particle-number sector; with open bonds the two end fields shift
  by -V/2.  Either way (jxy, jz, h[]) expresses the paper's model.
* The on-site sum of Eq. (1) is read as running over all L sites.
* Site i (1-based, as in the cosine) is bit i-1 of the state integer; the
  Neel state "(...010101)" of Sec. 4 has bits 0, 2, 4, ... set.
* Periodic boundary conditions (used in Sec. 4) add the bond (L, 1), i.e.
  bits (L-1, 0).  The bond list is the literal sum over i = 1..L of the pair
  (i, i+1 mod L), so a 2-site ring carries its single pair twice.
* The hopping sign is +jxy/2 as in Eq. (1) (+t).
"""
from __future__ import annotations

import math

import numpy as np


def fields(L: int, h: float, beta: float, phi: float) -> np.ndarray:
    """On-site fields h_i = h*cos(2*pi*beta*i + phi), i = 1..L (Eq. (1)).

    Element i-1 of the result is the field on site i (bit i-1).
    """
    i = np.arange(1, L + 1, dtype=np.float64)
    return h * np.cos(2.0 * math.pi * beta * i + phi)


def bonds(L: int, pbc: bool) -> list[tuple[int, int]]:
    """Nearest-neighbour bonds as (bit, bit) pairs.

    Open chain: (0,1), (1,2), ..., (L-2, L-1) -- the i = 1..L-1 sums of Eq. (1).
    Periodic chain: additionally (L-1, 0).
    """
    out = [(i, i + 1) for i in range(L - 1)]
    if pbc and L >= 2:
        out.append((L - 1, 0))
    return out


def neel_state(L: int) -> int:
    """The Neel state (...010101) of Sec. 4: bits 0, 2, 4, ... set."""
    s = 0
    for b in range(0, L, 2):
        s |= 1 << b
    return s


def z_values(states: np.ndarray, L: int) -> np.ndarray:
    """S^z eigenvalues bit_i - 1/2 for every state (rows) and site (columns)."""
    states = np.asarray(states, dtype=np.int64)
    bits = (states[:, None] >> np.arange(L, dtype=np.int64)[None, :]) & 1
    return bits.astype(np.float64) - 0.5
