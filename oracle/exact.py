"""Exact propagation by full diagonalisation (Sec. 2, Eqs. (2)-(3); Sec. 4,
survival probability F(t)) -- oracle, test infrastructure.

psi(t) = exp(-i H t) psi(0) with hbar = 1.  For the real symmetric H of the
model, H = U diag(w) U^T with real orthogonal U, so
    psi(t) = U ( exp(-i w t) * (U^T psi(0)) ).
The survival amplitude of Sec. 4 is A(t) = <psi(0)| exp(-iHt) |psi(0)> and the
survival (return) probability is F(t) = |A(t)|^2.  For psi(0) = e_r0 (a basis
state such as the Neel state) A(t) = sum_n U[r0,n]^2 exp(-i w_n t).

This is the route the paper avoids for large systems (Sec. 1-2); here it is
the plain definition the Krylov path is checked against at small L.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def eig(H: np.ndarray):
    """Eigenvalues w (ascending) and orthonormal eigenvectors U of real symmetric H."""
    return sla.eigh(H)


def evolve(H: np.ndarray, psi0: np.ndarray, times, eigsys=None) -> np.ndarray:
    """psi(t) for each t in `times`; result shape (len(times), D), complex128."""
    w, U = eig(H) if eigsys is None else eigsys
    coef = U.T @ np.asarray(psi0, dtype=np.complex128)
    times = np.atleast_1d(np.asarray(times, dtype=np.float64))
    phases = np.exp(-1j * np.outer(times, w))            # (T, D)
    return (phases * coef[None, :]) @ U.T


def survival_amplitude(H: np.ndarray, r0: int, times, eigsys=None) -> np.ndarray:
    """A(t) = <e_r0| exp(-iHt) |e_r0> = sum_n U[r0,n]^2 exp(-i w_n t)."""
    w, U = eig(H) if eigsys is None else eigsys
    c2 = U[r0, :] ** 2
    times = np.atleast_1d(np.asarray(times, dtype=np.float64))
    return np.exp(-1j * np.outer(times, w)) @ c2


def survival_probability(H: np.ndarray, r0: int, times, eigsys=None) -> np.ndarray:
    """F(t) = |A(t)|^2 (Sec. 4)."""
    return np.abs(survival_amplitude(H, r0, times, eigsys)) ** 2


def overlap_probability(psi0: np.ndarray, psi: np.ndarray) -> float:
    """|<psi0|psi>|^2 for a general (normalised) initial state."""
    return float(abs(np.vdot(psi0, psi)) ** 2)


def autocorrelation(times: np.ndarray, F: np.ndarray) -> np.ndarray:
    """C(t) = (1/t) * integral_0^t F(t') dt' (Sec. 4) by the trapezoid rule on
    the given grid, which must start at t = 0 (C(0) is taken as F(0))."""
    times = np.asarray(times, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    if times[0] != 0.0:
        raise ValueError("grid must start at t=0")
    integ = np.concatenate([[0.0], np.cumsum(0.5 * (F[1:] + F[:-1]) * np.diff(times))])
    out = np.empty_like(F)
    out[0] = F[0]
    out[1:] = integ[1:] / times[1:]
    return out


def autocorrelation_exact(H: np.ndarray, psi0: np.ndarray, times, eigsys=None) -> np.ndarray:
    """C(t) = (1/t) * integral_0^t |<psi0| exp(-iHt') |psi0>|^2 dt' (Sec. 4) in
    closed form.  With w_n = |<n|psi0>|^2 over the eigenvectors of H,
    |A(t')|^2 = sum_{n,m} w_n w_m exp(-i (E_n - E_m) t'), whose time average
    over [0, t] is sum_{n,m} w_n w_m sin((E_n - E_m) t) / ((E_n - E_m) t)
    (the imaginary parts cancel between (n, m) and (m, n)); the limit t -> 0
    is (sum_n w_n)^2."""
    w, U = eig(H) if eigsys is None else eigsys
    c = U.T @ np.asarray(psi0, dtype=np.complex128)
    wn = np.abs(c) ** 2
    times = np.atleast_1d(np.asarray(times, dtype=np.float64))
    dE = w[:, None] - w[None, :]
    out = np.empty(len(times))
    for k, t in enumerate(times):
        # np.sinc(x) = sin(pi x) / (pi x)
        out[k] = float(wn @ np.sinc(dE * t / np.pi) @ wn)
    return out
