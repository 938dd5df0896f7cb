"""Mid-size exact propagation through a library routine -- oracle, test infrastructure.

Same definition as `oracle.exact` (psi(t) = exp(-iHt) psi(0), Sec. 2 Eq. (3)),
evaluated without diagonalising: scipy.sparse.linalg.expm_multiply implements
the truncated-Taylor algorithm with scaling of Al-Mohy and Higham (2011) and
reaches double-precision accuracy for the action of the exponential.  Used for
sectors too large for a dense eigendecomposition (L = 18..24 and sampled
checks above).  H is kept as complex128 CSR so every call works in one dtype.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def evolve(Hcsr, psi0: np.ndarray, times) -> np.ndarray:
    """psi at each of the ascending `times` (first may be 0); shape (T, D)."""
    H = Hcsr.astype(np.complex128)
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    out = []
    t_prev = 0.0
    for t in np.atleast_1d(np.asarray(times, dtype=np.float64)):
        dt = t - t_prev
        if dt < 0:
            raise ValueError("times must ascend")
        if dt > 0:
            psi = spla.expm_multiply(-1j * dt * H, psi)
        out.append(psi.copy())
        t_prev = t
    return np.array(out)


def survival_probability(Hcsr, r0: int, times) -> np.ndarray:
    """F(t) = |psi(t)[r0]|^2 for psi(0) = e_r0."""
    D = Hcsr.shape[0]
    psi0 = np.zeros(D, dtype=np.complex128)
    psi0[r0] = 1.0
    H = Hcsr.astype(np.complex128)
    psi = psi0
    out = []
    t_prev = 0.0
    for t in np.atleast_1d(np.asarray(times, dtype=np.float64)):
        dt = t - t_prev
        if dt > 0:
            psi = spla.expm_multiply(-1j * dt * H, psi)
        out.append(abs(psi[r0]) ** 2)
        t_prev = t
    return np.array(out)
