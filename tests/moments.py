"""Short-time Taylor expansion of exp(-iHt) between two basis states, from
the oracle's definition of H (test helper; not collected by pytest).

With v_a = H^a e_s held sparsely on the states reached after a hops (the
oracle's diagonal and hop targets applied to those states only), and H real
symmetric,
    <s| exp(-iHt) |n> = sum_k (-i t)^k / k! <H^a e_s, H^b e_n>,  a + b = k,
exact up to the Taylor remainder, which the Gershgorin bound G of H bounds by
e^{tG} (tG)^{K+1} / (K+1)!.  The number of states reached grows like L^a, so
nine hops stay within a few million states even at L = 30.
"""
import math

import numpy as np

from oracle import hamiltonian as OH


def sparse_apply(states, vals, L, pbc, jxy, jz, h):
    """(H v) for a sparse v given by sorted states and their values."""
    out_s = [states]
    out_v = [OH.diagonal(states, L, pbc, jz, h) * vals]
    g = OH.hop_amplitude(jxy)
    for anti, flipped in OH.hop_targets(states, L, pbc):
        out_s.append(flipped[anti])
        out_v.append(g * vals[anti])
    s = np.concatenate(out_s)
    u, inv = np.unique(s, return_inverse=True)
    return u, np.bincount(inv, weights=np.concatenate(out_v), minlength=len(u))


def powers(state, n, L, pbc, jxy, jz, h):
    """[H^a e_state for a = 0..n] as (sorted states, values) pairs."""
    out = [(np.array([state], dtype=np.int64), np.array([1.0]))]
    for _ in range(n):
        out.append(sparse_apply(*out[-1], L, pbc, jxy, jz, h))
    return out


def sdot(a, b):
    """Inner product of two sparse real vectors."""
    _, ia, ib = np.intersect1d(a[0], b[0], assume_unique=True, return_indices=True)
    return float(np.dot(a[1][ia], b[1][ib]))


def taylor_amplitude(ps, pn, t, K):
    """sum_{k <= K} (-i t)^k / k! <H^a e_s, H^b e_n> (a + b = k) from the powers
    of both ends; needs K <= (len(ps) - 1) + (len(pn) - 1)."""
    half = len(pn) - 1
    if K > half + len(ps) - 1:
        raise ValueError("not enough powers for this order")
    amp = 0j
    for k in range(K + 1):
        a = max(0, k - half)
        amp += (-1j * t) ** k / math.factorial(k) * sdot(ps[a], pn[k - a])
    return amp


def remainder_bound(L, pbc, jxy, jz, h, t, K):
    """e^{tG} (tG)^{K+1} / (K+1)! with G = jz n_b / 4 + sum |h_i| / 2 + n_b jxy / 2,
    n_b the number of bonds (a Gershgorin bound of the norm of H)."""
    nb = L if pbc else L - 1
    G = abs(jz) * nb / 4.0 + float(np.sum(np.abs(h))) / 2.0 + nb * abs(jxy) / 2.0
    x = t * G
    return math.exp(x) * x ** (K + 1) / math.factorial(K + 1)
