"""Integer-encoded sorted basis (Sec. 2 "Basis representation"; Sec. 3,
Algorithms 2 and 3) -- oracle, test infrastructure.

A basis state of N particles on L sites is the integer whose set bits are the
occupied sites; the basis of the sector is the ascending list of all such
integers, of length D = L!/(N!(L-N)!) (Sec. 2).  Row r of every vector and of
the Hamiltonian belongs to the r-th integer of that list.
"""
from __future__ import annotations

from itertools import combinations
from math import comb

import numpy as np


def sector_dim(L: int, N: int) -> int:
    """D = L! / (N! (L-N)!)  (Sec. 2, "Basis representation")."""
    return comb(L, N)


def sector_states(L: int, N: int) -> np.ndarray:
    """All integers in [0, 2^L) with exactly N set bits, ascending (int64).

    This is the plain definition of the basis.  Up to L = 30 it scans the full
    2^L range in chunks and keeps the integers whose popcount is N; above, it
    forms the integer of every N-subset of the L bit positions and sorts them
    (the same set, for sectors too large to scan; L <= 63 so that int64 holds
    every state).
    """
    if not (0 <= N <= L <= 63):
        raise ValueError("need 0 <= N <= L <= 63")
    if L > 30:
        if comb(L, N) > 50_000_000:
            raise ValueError("sector too large for the oracle")
        vals = sorted(sum(1 << p for p in c) for c in combinations(range(L), N))
        return np.array(vals, dtype=np.int64)
    chunk = 1 << 22
    parts = []
    for lo in range(0, 1 << L, chunk):
        v = np.arange(lo, min(lo + chunk, 1 << L), dtype=np.int64)
        keep = np.bitwise_count(v) == N
        parts.append(v[keep])
    return np.concatenate(parts) if parts else np.zeros(0, np.int64)


def smallest_int(N: int) -> int:
    """Smallest integer of the sector: the N lowest bits set (Sec. 3)."""
    return (1 << N) - 1


def next_bit_permutation(v: int) -> int:
    """One step of Algorithm 2: the next larger integer with the same popcount.

    t sets the lowest clear bit above the lowest run of ones and clears that
    run; the ones of the run, less one, are then refilled at the bottom.  The
    paper writes the refill with an exact division of the lowest set bits of
    t and v (both powers of two).
    """
    t = (v | (v - 1)) + 1
    return t | ((((t & -t) // (v & -v)) >> 1) - 1)


def basis_alg2(L: int, N: int, start_state: int | None = None, count: int | None = None) -> list[int]:
    """Sequential basis construction of Algorithm 2 (or of a section, Algorithm 3).

    Starting from `start_state` (default smallest_int(N)), apply the next bit
    permutation count-1 times (default: the whole sector).
    """
    if N == 0:
        return [0]
    v = smallest_int(N) if start_state is None else start_state
    if count is None:
        count = sector_dim(L, N)
    out = [v]
    for _ in range(count - 1):
        v = next_bit_permutation(v)
        out.append(v)
    return out


def first_int(L: int, N: int, start: int) -> int:
    """The `start`-th state of the sorted basis, i.e. Algorithm 3's first_int().

    Built from the combinatorial counting that the sorted order implies: going
    from the top bit down, the number of sector states whose remaining k set
    bits all lie below position p is C(p, k); if the index left over is at
    least that, bit p must be set.
    """
    if not 0 <= start < sector_dim(L, N):
        raise ValueError("start out of range")
    s, r, k = 0, start, N
    for p in range(L - 1, -1, -1):
        if k == 0:
            break
        c = comb(p, k)
        if r >= c:
            s |= 1 << p
            r -= c
            k -= 1
    return s


def distribution(D: int, nprocs: int, rank: int) -> tuple[int, int, int]:
    """Balanced block-row partition of D rows over nprocs ranks, the
    distribution of Algorithm 1: every rank gets floor(D / nprocs) rows and
    the first D mod nprocs ranks one more, in rank order.  Returns
    (nlocal, start, end) of `rank`."""
    q, r = divmod(D, nprocs)
    nlocal = q + (1 if rank < r else 0)
    start = rank * q + min(rank, r)
    return nlocal, start, start + nlocal


def lookup(basis: np.ndarray, states) -> np.ndarray:
    """Row index of each state by binary search of the sorted basis (Sec. 3,
    "Hamiltonian matrix construction"); -1 where the state is not in the basis."""
    states = np.asarray(states, dtype=np.int64)
    idx = np.searchsorted(basis, states)
    idx_c = np.minimum(idx, len(basis) - 1)
    found = (idx < len(basis)) & (basis[idx_c] == states)
    return np.where(found, idx, -1).astype(np.int64)
