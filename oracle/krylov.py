"""Krylov subspace propagation as Sec. 2 ("Krylov subspace methods") describes it
-- oracle, test infrastructure.

For an initial state psi0 and Krylov dimension m:
  * the Krylov space K_m = span{psi0, H psi0, ..., H^(m-1) psi0} is spanned by
    orthonormal columns V_m, built by the Arnoldi process (each new H v_j is
    orthogonalised against all previous columns, modified Gram-Schmidt);
  * the projected matrix is A_m = V_m^dagger H V_m (upper Hessenberg; the
    transpose in the paper is read as the conjugate transpose, which is the
    same for the real H of Eq. (1) but keeps complex psi0 correct);
  * psi(t) is approximated by ||psi0|| V_m exp(-i t A_m) e_1;
  * the small exponential is evaluated by a Pade approximant (scipy's expm:
    diagonal Pade with scaling and squaring).
If the Arnoldi recurrence produces a zero new direction (the Krylov space is
invariant under H) it stops with m_used < m, and the result is then exact.

The a-posteriori error estimate returned with each step is
h_{m+1,m} * |[exp(-i t A_m)]_{m,1}| * ||psi0|| (Saad 1992), the quantity the
time-stepping codes the paper cites (Expokit) use.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


def arnoldi(matvec, psi0: np.ndarray, m: int, breakdown_rtol: float = 1e-12):
    """Arnoldi decomposition of K_m(H, psi0).

    Returns (V, A, beta0, h_next, m_used): V is D x m_used with orthonormal
    columns, A is m_used x m_used, beta0 = ||psi0||, h_next = the norm of the
    residual direction after the last column (0 at breakdown).
    """
    psi0 = np.asarray(psi0, dtype=np.complex128)
    beta0 = float(np.linalg.norm(psi0))
    if beta0 == 0.0:
        raise ValueError("zero initial vector")
    D = psi0.shape[0]
    V = np.zeros((D, m + 1), dtype=np.complex128)
    A = np.zeros((m + 1, m), dtype=np.complex128)
    V[:, 0] = psi0 / beta0
    m_used = m
    h_next = 0.0
    scale = 0.0
    for j in range(m):
        w = np.asarray(matvec(V[:, j]), dtype=np.complex128)
        for i in range(j + 1):
            A[i, j] = np.vdot(V[:, i], w)
            w = w - A[i, j] * V[:, i]
        h_next = float(np.linalg.norm(w))
        scale = max(scale, float(np.max(np.abs(A[: j + 1, j]))), h_next)
        A[j + 1, j] = h_next
        if h_next <= breakdown_rtol * scale:
            m_used = j + 1
            h_next = 0.0
            break
        V[:, j + 1] = w / h_next
    return V[:, :m_used], A[:m_used, :m_used], beta0, h_next, m_used


def expm_step(matvec, psi: np.ndarray, dt: float, m: int, breakdown_rtol: float = 1e-12):
    """One Krylov step psi -> exp(-i dt H) psi.

    Returns (psi_new, info) with info = dict(m_used, err_est, beta0, A).
    """
    V, A, beta0, h_next, m_used = arnoldi(matvec, psi, m, breakdown_rtol)
    E = sla.expm(-1j * dt * A)
    psi_new = beta0 * (V @ E[:, 0])
    err = beta0 * h_next * abs(E[m_used - 1, 0])
    return psi_new, dict(m_used=m_used, err_est=err, beta0=beta0, A=A)


def evolve(matvec, psi0: np.ndarray, dt: float, n_steps: int, m: int, r0: int | None = None):
    """Fixed-step Krylov evolution; returns (psi_final, F) where F[k] is the
    survival probability |<psi0|psi(k dt)>|^2 after step k (k = 1..n_steps),
    or |psi[r0]|^2 when r0 is given (psi0 = e_r0)."""
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    F = np.empty(n_steps)
    for k in range(n_steps):
        psi, _ = expm_step(matvec, psi, dt, m)
        F[k] = abs(psi[r0]) ** 2 if r0 is not None else abs(np.vdot(psi0, psi)) ** 2
    return psi, F


def error_bound(m: int, t: float, normA: float) -> float:
    """The a-priori bound shape quoted in Sec. 2 for the Krylov error,
    e^(m - t||A||) (t||A|| / m)^m, evaluated as a number (no hidden constant)."""
    x = t * normA
    if x == 0.0:
        return 0.0
    return math.exp(m - x + m * math.log(x / m))
