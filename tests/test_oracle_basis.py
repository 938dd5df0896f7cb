"""Pins of the oracle's basis against the paper's printed values and plain counting."""
from math import comb

import numpy as np
import pytest

from conftest import read_golden
from oracle import basis as B
from oracle import model as M


def test_paper_example_L4_N2():
    want = [int(r[0]) for r in read_golden("basis_L4_N2.txt")]
    assert B.sector_states(4, 2).tolist() == want
    assert B.basis_alg2(4, 2) == want


@pytest.mark.parametrize("L,N,D", [(int(a), int(b), int(c)) for a, b, c in read_golden("dims_exact.txt")])
def test_exact_dims_printed_in_paper(L, N, D):
    assert B.sector_dim(L, N) == D


@pytest.mark.parametrize("row", read_golden("table1_dims.txt"))
def test_table1(row):
    L, N, D3, mem = int(row[0]), int(row[1]), float(row[2]), float(row[3])
    D = B.sector_dim(L, N)
    assert float(f"{D:.2e}") == pytest.approx(D3)
    # 8-byte integers per state, decimal GB; the table rounds to ~1%.
    assert 8 * D / 1e9 == pytest.approx(mem, rel=0.01)


def test_count_by_scan_matches_binomial():
    for L in range(1, 17):
        for N in range(0, L + 1):
            st = B.sector_states(L, N)
            assert len(st) == comb(L, N)
            assert np.all(np.diff(st) > 0)
            assert np.all(np.bitwise_count(st) == N)


def test_alg2_matches_scan():
    for L in range(2, 15):
        for N in range(1, L + 1):
            assert B.basis_alg2(L, N) == B.sector_states(L, N).tolist()


def test_alg2_single_steps():
    # next bit permutation of a few hand-checked integers
    assert B.next_bit_permutation(0b0011) == 0b0101
    assert B.next_bit_permutation(0b0110) == 0b1001
    assert B.next_bit_permutation(0b1011) == 0b1101
    assert B.next_bit_permutation(0b0111000) == 0b1000011


def test_first_int_is_kth_state():
    for L, N in [(10, 5), (12, 3), (9, 9), (8, 1)]:
        st = B.sector_states(L, N)
        for k in range(len(st)):
            assert B.first_int(L, N, k) == st[k]


def test_sections_alg1_alg3_rebuild_basis():
    # Algorithm 1 partition + Algorithm 3 per-section construction cover the basis
    L, N = 12, 6
    full = B.sector_states(L, N).tolist()
    D = len(full)
    for P in [1, 3, 7, 16]:
        got = []
        ends = []
        for rank in range(P):
            nlocal, start, end = B.distribution(D, P, rank)
            ends.append((start, end))
            if nlocal:
                got += B.basis_alg2(L, N, B.first_int(L, N, start), nlocal)
        assert got == full
        assert ends[0][0] == 0 and ends[-1][1] == D
        assert all(ends[i][1] == ends[i + 1][0] for i in range(P - 1))
        sizes = [e - s for s, e in ends]
        assert max(sizes) - min(sizes) <= 1 and sizes[0] == max(sizes)


def test_lookup_bijection_and_misses():
    st = B.sector_states(10, 4)
    assert np.array_equal(B.lookup(st, st), np.arange(len(st)))
    other = B.sector_states(10, 5)
    assert np.all(B.lookup(st, other) == -1)
    assert B.lookup(st, [0, 1 << 11])[0] == -1


def test_neel_state():
    assert M.neel_state(4) == 0b0101
    assert M.neel_state(16) == 21845
    assert M.neel_state(28) == (4 ** 14 - 1) // 3


def test_bonds():
    assert M.bonds(4, False) == [(0, 1), (1, 2), (2, 3)]
    assert M.bonds(4, True) == [(0, 1), (1, 2), (2, 3), (3, 0)]
    assert len(M.bonds(2, True)) == 2     # the literal sum over i = 1..L on a 2-site ring


def test_fields_special_beta():
    # beta = 1/2 makes the cosine alternate: h*cos(pi*i + phi) = h*(-1)^i*cos(phi)
    f = M.fields(6, 2.0, 0.5, 0.3)
    assert np.allclose(f, 2.0 * np.cos(0.3) * np.array([-1, 1, -1, 1, -1, 1]))
    # beta = 1 makes it uniform
    assert np.allclose(M.fields(5, 1.5, 1.0, 0.7), 1.5 * np.cos(0.7))


def test_large_sector_enumeration():
    # the subset route used above L = 30 against the full scan on sectors both
    # can list, then the count and order at L = 55 and L = 63
    from itertools import combinations
    for L, N in [(20, 3), (22, 11), (24, 1), (24, 23)]:
        scan = B.sector_states(L, N)
        sub = np.array(sorted(sum(1 << p for p in c) for c in combinations(range(L), N)), dtype=np.int64)
        assert np.array_equal(scan, sub)
    for L, N in [(55, 3), (63, 2), (40, 5)]:
        st = B.sector_states(L, N)
        assert len(st) == B.sector_dim(L, N)
        assert np.all(np.diff(st) > 0)
        assert np.all(np.bitwise_count(st) == N)
        assert st[0] == (1 << N) - 1 and st[-1] == ((1 << N) - 1) << (L - N)
        # Alg. 3's first_int and Alg. 2's walk agree with the list
        for r in (0, 1, len(st) // 3, len(st) - 1):
            assert B.first_int(L, N, r) == st[r]
        assert B.basis_alg2(L, N, start_state=int(st[5]), count=50) == [int(v) for v in st[5:55]]
