"""Plants plausible mistakes in the oracle (on the CPU only) and checks that
the pins in the other oracle tests catch each of them."""
import numpy as np
import pytest

import test_oracle_basis as TB
import test_oracle_gradient as TG
import test_oracle_hamiltonian as TH
import test_oracle_propagation as TP
from oracle import basis as B
from oracle import exact as X
from oracle import gradient as G
from oracle import hamiltonian as Hm
from oracle import krylov as K
from oracle import model as M

_orig_bonds = M.bonds
_orig_fields = M.fields
_orig_diagonal = Hm.diagonal
_orig_hop = Hm.hop_targets
_orig_evolve = X.evolve
_orig_amp = X.survival_amplitude
_orig_nbp = B.next_bit_permutation
_orig_first = B.first_int
_orig_states = B.sector_states
_orig_acx = X.autocorrelation_exact
_orig_dF = G.dF_dh
_orig_bound = K.error_bound


def _fails(*checks):
    """True when at least one of the pin checks raises AssertionError."""
    for c in checks:
        try:
            c()
        except AssertionError:
            return True
    return False


def _no_wrap(L, pbc):
    return _orig_bonds(L, False)


def _field_shift(L, h, beta, phi):
    return _orig_fields(L + 1, h, beta, phi)[1:]


def _half_jz(states, L, pbc, jz, h):
    return _orig_diagonal(states, L, pbc, 0.5 * jz, h)


def _field_sign(states, L, pbc, jz, h):
    zz = _orig_diagonal(states, L, pbc, jz, np.zeros_like(np.asarray(h)))
    return zz - (_orig_diagonal(states, L, pbc, 0.0, h))


def _reversed_time(H, psi0, times, eigsys=None):
    return _orig_evolve(H, psi0, -np.asarray(times, dtype=float), eigsys)


def _transposed_U(H, psi0, times, eigsys=None):
    w, U = X.eig(H) if eigsys is None else eigsys
    coef = U @ np.asarray(psi0, dtype=np.complex128)
    ph = np.exp(-1j * np.outer(np.atleast_1d(times), w))
    return (ph * coef[None, :]) @ U.T


def _bad_nbp(v):
    t = (v | (v - 1)) + 1
    return t | ((((t & -t) // (v & -v)) >> 2) - 1)


def _bad_first(L, N, start):
    return _orig_first(L, N, max(start - 1, 0)) if start == 3 else _orig_first(L, N, start)


def _sinc_without_time(H, psi0, times, eigsys=None):
    # the time average taken as sin(dE t) / dE instead of sin(dE t) / (dE t)
    t = np.atleast_1d(np.asarray(times, dtype=float))
    return _orig_acx(H, psi0, times, eigsys) * np.where(t > 1.0, t, 1.0)


def _acx_diagonal_only(H, psi0, times, eigsys=None):
    # only the n == m terms: the long-time limit at every time
    w, U = X.eig(H) if eigsys is None else eigsys
    wn = np.abs(U.T @ np.asarray(psi0, dtype=np.complex128)) ** 2
    return np.full(len(np.atleast_1d(times)), float(np.sum(wn ** 2)))


def _subsets_shifted(L, N):
    # bit positions 1..L instead of 0..L-1 above the scan range
    if L <= 30:
        return _orig_states(L, N)
    from itertools import combinations
    return np.array(sorted(sum(1 << p for p in c) for c in combinations(range(1, L + 1), N)), dtype=np.int64)


def _dF_half(*args, **kw):
    # 2 Re(conj(A) dA) taken without the factor 2
    F, g = _orig_dF(*args, **kw)
    return F, 0.5 * g


def _dF_sites_reversed(*args, **kw):
    # derivative assigned to the mirrored site
    F, g = _orig_dF(*args, **kw)
    return F, g[::-1].copy()


def _bound_sign_flipped(m, t, normA):
    # e^(m + x) instead of e^(m - x): an overestimate everywhere
    x = t * normA
    return _orig_bound(m, t, normA) * np.exp(2 * x) if x > 0 else 0.0


def _bound_extra_e(m, t, normA):
    return np.e * _orig_bound(m, t, normA)


def _bound_power_m_minus_1(m, t, normA):
    # (x / m)^(m - 1) instead of (x / m)^m
    x = t * normA
    return _orig_bound(m, t, normA) * m / x if x > 0 else 0.0


def _hop_full(jxy):
    return jxy


def _hop_negative(jxy):
    return -0.5 * jxy


PLANTS = {
    "hopping jxy instead of jxy/2": [(Hm, "hop_amplitude", _hop_full)],
    "hopping sign flipped": [(Hm, "hop_amplitude", _hop_negative)],
    "dropped wrap bond": [(M, "bonds", _no_wrap)],
    "field on the wrong site": [(M, "fields", _field_shift)],
    "zz coupling halved": [(Hm, "diagonal", _half_jz)],
    "field sign flipped": [(Hm, "diagonal", _field_sign)],
    "time runs backwards": [(X, "evolve", _reversed_time)],
    "transposed eigenvectors": [(X, "evolve", _transposed_U)],
    "wrong refill shift in Algorithm 2": [(B, "next_bit_permutation", _bad_nbp)],
    "off-by-one section start": [(B, "first_int", _bad_first)],
    "autocorrelation without the 1/t": [(X, "autocorrelation_exact", _sinc_without_time)],
    "autocorrelation keeps only n == m": [(X, "autocorrelation_exact", _acx_diagonal_only)],
    "large sectors on shifted bits": [(B, "sector_states", _subsets_shifted)],
    "gradient without the factor 2": [(G, "dF_dh", _dF_half)],
    "gradient on mirrored sites": [(G, "dF_dh", _dF_sites_reversed)],
    "error bound with the exponent's sign flipped": [(K, "error_bound", _bound_sign_flipped)],
    "error bound with an extra factor e": [(K, "error_bound", _bound_extra_e)],
    "error bound with power m - 1": [(K, "error_bound", _bound_power_m_minus_1)],
}

CHECKS = [
    TB.test_paper_example_L4_N2, TB.test_alg2_matches_scan, TB.test_first_int_is_kth_state,
    TB.test_sections_alg1_alg3_rebuild_basis,
    TH.test_heisenberg_ring_L4_spectrum, TH.test_two_level_amplitude,
    lambda: TH.test_neel_energy_and_first_lanczos_norm(8, True),
    TH.test_hopping_sign_on_odd_ring,
    lambda: TP.test_free_fermion_determinant_matches_dense(8, True),
    TP.test_norm_energy_conservation_and_time_reversal, TP.test_expm_multiply_matches_dense,
    TP.test_krylov_converged_matches_exact,
    lambda: TB.test_fields_special_beta(),
    TP.test_autocorrelation_exact_two_level_closed_form, TP.test_autocorrelation_exact_limits_and_trapezoid,
    TB.test_large_sector_enumeration,
    lambda: TG.test_daleckii_krein_vs_finite_differences(True), TG.test_gradient_sums_to_zero,
    TP.test_error_bound_is_tight_at_the_edge_of_its_regime,
]


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    for mod, attr, fn in PLANTS[name]:
        monkeypatch.setattr(mod, attr, fn)
    assert _fails(*CHECKS), f"no pin caught: {name}"


def test_unplanted_oracle_passes_all_checks():
    assert not _fails(*CHECKS)
