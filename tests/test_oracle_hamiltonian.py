"""Pins of the oracle's Hamiltonian against closed forms that fix each term."""
import numpy as np
import pytest

from oracle import basis as B
from oracle import exact as X
from oracle import hamiltonian as Hm
from oracle import model as M
from workloads import random_complex, random_fields


def test_real_symmetric():
    for L, pbc in [(8, False), (8, True), (10, True)]:
        H = Hm.build_dense(L, L // 2, pbc, 1.0, 0.7, random_fields(L, 1))
        assert np.isrealobj(H)
        assert np.array_equal(H, H.T)


def test_heisenberg_ring_L4_spectrum():
    # 4-site Heisenberg ring sum S_i.S_{i+1} = (S1+S3).(S2+S4): Sz=0 levels
    # 1/2[S(S+1) - SA(SA+1) - SB(SB+1)] = {-2, -1, 0, 0, 0, 1}.
    H = Hm.build_dense(4, 2, True, 1.0, 1.0, np.zeros(4))
    assert np.allclose(np.linalg.eigvalsh(H), [-2, -1, 0, 0, 0, 1], atol=1e-13)


def test_heisenberg_ring_L2_doubled_bond():
    # 2-site ring: the pair is summed twice, H = 2 S1.S2 -> singlet -3/2, triplet(m=0) 1/2
    H = Hm.build_dense(2, 1, True, 1.0, 1.0, np.zeros(2))
    assert np.allclose(np.linalg.eigvalsh(H), [-1.5, 0.5], atol=1e-14)


def test_two_level_amplitude():
    # L=2 open, one particle: H = [[e1, g], [g, e2]], g = jxy/2,
    # e1 = -jz/4 + (h1-h2)/2 (site 1 occupied), e2 = -jz/4 - (h1-h2)/2.
    jxy, jz, h = 0.8, 0.6, np.array([0.9, -0.4])
    H = Hm.build_dense(2, 1, False, jxy, jz, h)
    t = np.linspace(0, 7, 29)
    A = X.survival_amplitude(H, 0, t)
    d = h[0] - h[1]
    Om = np.sqrt(d * d + jxy * jxy)
    want = np.exp(1j * jz / 4 * t) * (np.cos(Om * t / 2) - 1j * d / Om * np.sin(Om * t / 2))
    assert np.allclose(A, want, atol=1e-14)
    P = 1 - (jxy / Om) ** 2 * np.sin(Om * t / 2) ** 2
    assert np.allclose(np.abs(A) ** 2, P, atol=1e-14)


@pytest.mark.parametrize("L,pbc", [(8, True), (8, False), (10, True), (12, False)])
def test_neel_energy_and_first_lanczos_norm(L, pbc):
    jxy, jz = 1.3, 0.9
    h = random_fields(L, 5)
    st = B.sector_states(L, L // 2)
    r0 = int(B.lookup(st, [M.neel_state(L)])[0])
    H = Hm.build_csr(L, L // 2, pbc, jxy, jz, h)
    nb = L if pbc else L - 1
    sign = np.array([1 if i % 2 == 1 else -1 for i in range(1, L + 1)])   # site 1 occupied
    E0 = -jz * nb / 4 + 0.5 * np.sum(sign * h)
    e = np.zeros(len(st)); e[r0] = 1
    He = H @ e
    assert He[r0] == pytest.approx(E0, abs=1e-13)
    beta0 = np.linalg.norm(He - E0 * e)
    assert beta0 == pytest.approx(0.5 * jxy * np.sqrt(nb), abs=1e-13)
    # every Neel bond is anti-aligned: nb off-diagonal entries in that row
    assert Hm.nnz_per_row(L, L // 2, pbc, [r0])[0] == nb


def test_apply_rows_matches_matrix():
    L, pbc = 12, True
    h = random_fields(L, 2)
    H = Hm.build_csr(L, 6, pbc, 1.0, 1.0, h)
    x = random_complex(H.shape[0], 3)
    rows = np.array([0, 5, 17, 400, H.shape[0] - 1])
    assert np.allclose(Hm.apply_rows(L, 6, pbc, 1.0, 1.0, h, x, rows), (H @ x)[rows], atol=1e-13)


def test_apply_rows_batched_fields():
    L, pbc, Bn = 10, True, 3
    hs = np.stack([random_fields(L, s) for s in range(Bn)])
    D = B.sector_dim(L, 5)
    X2 = np.stack([random_complex(D, 10 + s) for s in range(Bn)], axis=1)   # [D][B]
    rows = np.arange(D)
    Y = Hm.apply_rows(L, 5, pbc, 1.0, 1.0, hs, X2, rows)
    for s in range(Bn):
        H = Hm.build_csr(L, 5, pbc, 1.0, 1.0, hs[s])
        assert np.allclose(Y[:, s], H @ X2[:, s], atol=1e-13)


def test_row_counts_average():
    # Average off-diagonal entries per row at half filling: each bond is
    # anti-aligned in a fraction N(L-N)/(L(L-1))*2 of the states.
    L, N = 12, 6
    for pbc in (False, True):
        nb = L if pbc else L - 1
        avg = Hm.nnz_per_row(L, N, pbc).mean()
        assert avg == pytest.approx(nb * 2 * N * (L - N) / (L * (L - 1)))


def test_hopping_sign_on_odd_ring():
    # A 3-site ring is not bipartite, so the sign of the hopping is visible in
    # the spectrum: one particle with +jxy/2 on each bond has levels
    # {jxy, -jxy/2, -jxy/2} (Eq. (1) with +t).
    jxy = 1.4
    H = Hm.build_dense(3, 1, True, jxy, 0.0, np.zeros(3))
    assert np.allclose(np.linalg.eigvalsh(H), [-jxy / 2, -jxy / 2, jxy], atol=1e-14)


def test_mean_offdiagonal_count_and_table3_memory_law():
    # Sec. 3's exact preallocation counts, per row, the bonds whose two bits
    # differ.  At half filling on a ring their mean is L^2 / (2 (L - 1)) (each
    # of the L bonds differs with probability 2 N (L - N) / (L (L - 1))); the
    # oracle's counts must reproduce it exactly at small L.
    from math import comb

    from conftest import read_golden
    for L in (8, 10, 12, 14, 16):
        N = L // 2
        cnt = Hm.nnz_per_row(L, N, True)
        assert cnt.sum() * 2 * (L - 1) == L * L * comb(L, N)
        cnt_obc = Hm.nnz_per_row(L, N, False)
        assert cnt_obc.sum() * 2 * (L - 1) == L * (L - 1) * comb(L, N)
    # Sec. 5, Table III: the estimated matrix memory grows like the number of
    # stored entries D (1 + L^2 / (2 (L - 1))): bytes per stored entry stay
    # within a few per cent of each other from L = 28 to 38 (the table prints
    # two to four significant figures).
    per_entry = []
    for L, D, mem_gb, _ in read_golden("table3_memory.txt"):
        L = int(L)
        assert abs(comb(L, L // 2) / float(D) - 1) < 0.006
        entries = comb(L, L // 2) * (1 + L * L / (2 * (L - 1)))
        per_entry.append(float(mem_gb) * 1e9 / entries)
    assert max(per_entry) / min(per_entry) < 1.03, per_entry
