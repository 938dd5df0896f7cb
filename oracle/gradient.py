"""Derivative of the survival probability with respect to every on-site field
-- oracle, test infrastructure.

F(T) = |A(T)|^2 with A(T) = <e_r0| exp(-iHT) |e_r0> (Sec. 4).  The field h_i
enters H through h_i * Z_i with Z_i = diag(bit_i - 1/2) (Eq. (1) in the spin
reading).  In the eigenbasis H = U diag(w) U^T the derivative of the matrix
exponential is the Daleckii-Krein formula
    d exp(-iHT) / dh_i = U [ (U^T Z_i U) o G ] U^T,
    G_jk = (exp(-i w_j T) - exp(-i w_k T)) / (w_j - w_k),   G_jj = -i T exp(-i w_j T),
so with c = U[r0, :]
    dA/dh_i = sum_jk c_j c_k (U^T Z_i U)_jk G_jk = sum_r z_i(r) q_r,
    q_r = sum_jk M_rj G_jk M_rk,  M = U diag(c),
and dF/dh_i = 2 Re( conj(A) dA/dh_i ).
"""
from __future__ import annotations

import numpy as np

from . import basis as _basis
from . import exact as _exact
from . import hamiltonian as _ham
from . import model as _model


def dF_dh(L: int, N: int, pbc: bool, jxy: float, jz: float, h: np.ndarray, r0: int, T: float,
          degeneracy_tol: float = 1e-10):
    """Returns (F(T), dF/dh as an array of length L) by Daleckii-Krein."""
    H = _ham.build_dense(L, N, pbc, jxy, jz, h)
    w, U = _exact.eig(H)
    c = U[r0, :]
    e = np.exp(-1j * w * T)
    dw = w[:, None] - w[None, :]
    close = np.abs(dw) < degeneracy_tol
    G = np.where(close, -1j * T * e[:, None], (e[:, None] - e[None, :]) / np.where(close, 1.0, dw))
    A = np.sum(c * c * e)
    M = U * c[None, :]
    q = np.sum((M @ G) * M, axis=1)                      # q_r
    z = _model.z_values(_basis.sector_states(L, N), L)   # (D, L)
    dA = z.T @ q
    dF = 2.0 * np.real(np.conj(A) * dA)
    return float(abs(A) ** 2), dF


def dF_dh_finite_difference(L: int, N: int, pbc: bool, jxy: float, jz: float, h: np.ndarray,
                            r0: int, T: float, eps: float = 1e-6, propagate=None,
                            indices=None) -> np.ndarray:
    """Central differences (F(h + eps e_i) - F(h - eps e_i)) / (2 eps).

    `propagate(h) -> F(T)` may be supplied (e.g. a mid-size propagator); the
    default diagonalises the dense H.  `indices` restricts the result to the
    listed fields (in that order); the default is all L of them.
    """
    h = np.asarray(h, dtype=np.float64)

    def F_of(hh):
        if propagate is not None:
            return propagate(hh)
        H = _ham.build_dense(L, N, pbc, jxy, jz, hh)
        return float(_exact.survival_probability(H, r0, [T])[0])

    idx = list(range(L)) if indices is None else [int(i) for i in indices]
    out = np.empty(len(idx))
    for n, i in enumerate(idx):
        hp = h.copy(); hp[i] += eps
        hm = h.copy(); hm[i] -= eps
        out[n] = (F_of(hp) - F_of(hm)) / (2 * eps)
    return out
