"""Hamiltonian rows from bit operations and binary lookup (Sec. 3, "Hamiltonian
matrix construction") -- oracle, test infrastructure.

For a state s the Hamiltonian of Eq. (1), in the spin reading of
`oracle.model`, gives
  * a diagonal entry  jz * sum_b z_a z_c + sum_i h_i z_i,  z = bit - 1/2;
  * for every bond whose two bits differ, the entry jxy/2 in the column of the
    state with both bits flipped, found by binary lookup in the sorted basis.
Counting those columns per row is the exact preallocation of Sec. 3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis as _basis
from . import model as _model


def diagonal(states: np.ndarray, L: int, pbc: bool, jz: float, h: np.ndarray) -> np.ndarray:
    """Diagonal of H for the given states (float64).

    `h` is one field set of shape (L,) -> result (rows,), or B field sets of
    shape (B, L) -> result (rows, B).
    """
    z = _model.z_values(states, L)
    h = np.asarray(h, dtype=np.float64)
    zz = np.zeros(len(z))
    for a, c in _model.bonds(L, pbc):
        zz = zz + jz * z[:, a] * z[:, c]
    if h.ndim == 1:
        return z @ h + zz
    return z @ h.T + zz[:, None]


def hop_amplitude(jxy: float) -> float:
    """Off-diagonal entry of a bond whose two bits differ: (jxy/2) <..|S+S- + h.c.|..> = jxy/2."""
    return 0.5 * jxy


def hop_targets(states: np.ndarray, L: int, pbc: bool):
    """Per bond: (mask of rows whose bond bits differ, flipped states)."""
    states = np.asarray(states, dtype=np.int64)
    out = []
    for a, c in _model.bonds(L, pbc):
        ba = (states >> a) & 1
        bc = (states >> c) & 1
        anti = ba != bc
        flipped = states ^ ((1 << a) | (1 << c))
        out.append((anti, flipped))
    return out


def nnz_per_row(L: int, N: int, pbc: bool, rows: np.ndarray | None = None) -> np.ndarray:
    """Off-diagonal entries per row (the counting pass for exact preallocation).

    A bond listed twice (2-site ring) counts twice, since it is summed twice.
    """
    b = _basis.sector_states(L, N)
    st = b if rows is None else b[np.asarray(rows)]
    cnt = np.zeros(len(st), dtype=np.int64)
    for anti, _ in hop_targets(st, L, pbc):
        cnt += anti
    return cnt


def build_csr(L: int, N: int, pbc: bool, jxy: float, jz: float, h: np.ndarray,
              rows: np.ndarray | None = None, dtype=np.float64) -> sp.csr_matrix:
    """H (or the listed rows of H) as a scipy CSR matrix of shape (rows, D).

    Duplicate (row, col) pairs -- only possible on a 2-site ring -- are summed.
    """
    b = _basis.sector_states(L, N)
    D = len(b)
    row_ids = np.arange(D, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    st = b[row_ids]
    nr = len(st)
    local = np.arange(nr, dtype=np.int64)
    r_list = [local]
    c_list = [row_ids]
    v_list = [diagonal(st, L, pbc, jz, h)]
    for anti, flipped in hop_targets(st, L, pbc):
        cols = _basis.lookup(b, flipped[anti])
        if np.any(cols < 0):
            raise AssertionError("hop left the sector")
        r_list.append(local[anti])
        c_list.append(cols)
        v_list.append(np.full(cols.shape, hop_amplitude(jxy)))
    H = sp.coo_matrix((np.concatenate(v_list), (np.concatenate(r_list), np.concatenate(c_list))),
                      shape=(nr, D), dtype=np.float64).tocsr()
    H.sum_duplicates()
    return H.astype(dtype)


def build_dense(L: int, N: int, pbc: bool, jxy: float, jz: float, h: np.ndarray) -> np.ndarray:
    """Dense H (small sectors only)."""
    if _basis.sector_dim(L, N) > 20000:
        raise ValueError("dense H only for D <= 20000")
    return build_csr(L, N, pbc, jxy, jz, h).toarray()


def apply_rows(L: int, N: int, pbc: bool, jxy: float, jz: float, h: np.ndarray,
               x: np.ndarray, rows: np.ndarray, basis: np.ndarray | None = None) -> np.ndarray:
    """(H x)[rows], computed row by row from the rule above.

    `x` is the full input vector (or a [D, B] block); `basis` may be passed to
    avoid rebuilding the sorted state list for large L.
    """
    b = _basis.sector_states(L, N) if basis is None else basis
    rows = np.asarray(rows, dtype=np.int64)
    st = b[rows]
    x = np.asarray(x)
    d = diagonal(st, L, pbc, jz, h)          # (rows,) or (rows, B)
    if d.ndim == 1:
        d = d[:, None]
    y = (d * x[rows].reshape(len(rows), -1)).astype(np.complex128)
    for anti, flipped in hop_targets(st, L, pbc):
        if not np.any(anti):
            continue
        cols = _basis.lookup(b, flipped[anti])
        y[anti] += hop_amplitude(jxy) * x[cols].reshape(len(cols), -1)
    return y.reshape((len(rows),) + x.shape[1:])
