"""Closed form of the survival amplitude without zz coupling -- oracle, test infrastructure.

With V = jz = 0 (the free-particle limit named in Sec. 2), the Jordan-Wigner
transformation maps the hard-core bosons of Eq. (1) on N particles to free
fermions with the L x L single-particle Hamiltonian
    h1[i,i] = h_i,   h1[i,j] = jxy/2 for every bond (i,j),
where the bond closing a ring picks up the sign (-1)^(N-1) from the fermionic
string.  A basis state with occupied sites `occ` is a Slater determinant, so
    A(t) = det( exp(-i h1 t)[occ, occ] ),   F(t) = |A(t)|^2.
The constant -1/2 * sum_i h_i of the S^z reading is a global phase and drops
out of F.  This closed form works at any L (cost O(L^3) per time).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import model as _model


def single_particle_h(L: int, N: int, pbc: bool, jxy: float, h: np.ndarray) -> np.ndarray:
    h1 = np.diag(np.asarray(h, dtype=np.float64)).astype(np.float64)
    for a, c in _model.bonds(L, pbc):
        val = 0.5 * jxy
        if pbc and (a, c) == (L - 1, 0):
            val *= (-1.0) ** (N - 1)
        h1[a, c] += val
        h1[c, a] += val
    return h1


def survival_amplitude(L: int, N: int, pbc: bool, jxy: float, h: np.ndarray, state: int, times) -> np.ndarray:
    """A(t) for the basis state `state` (N set bits) at every t in `times`."""
    occ = [b for b in range(L) if (state >> b) & 1]
    if len(occ) != N:
        raise ValueError("state has wrong particle number")
    w, U = sla.eigh(single_particle_h(L, N, pbc, jxy, h))
    out = []
    for t in np.atleast_1d(np.asarray(times, dtype=np.float64)):
        G = (U * np.exp(-1j * w * t)[None, :]) @ U.T
        out.append(np.linalg.det(G[np.ix_(occ, occ)]))
    return np.array(out)


def survival_probability(L: int, N: int, pbc: bool, jxy: float, h: np.ndarray, state: int, times) -> np.ndarray:
    return np.abs(survival_amplitude(L, N, pbc, jxy, h, state, times)) ** 2
