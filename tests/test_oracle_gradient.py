"""Pins of the oracle's field gradient: finite differences, a sum rule and a symmetry."""
import numpy as np
import pytest

from oracle import basis as B
from oracle import gradient as G
from oracle import model as M
from workloads import BETA_GOLDEN


def _r0(L):
    st = B.sector_states(L, L // 2)
    return int(B.lookup(st, [M.neel_state(L)])[0])


@pytest.mark.parametrize("pbc", [True, False])
def test_daleckii_krein_vs_finite_differences(pbc):
    L = 8
    h = M.fields(L, 1.5, BETA_GOLDEN, 1.1)
    F, g = G.dF_dh(L, L // 2, pbc, 1.0, 1.0, h, _r0(L), 2.5)
    g_fd = G.dF_dh_finite_difference(L, L // 2, pbc, 1.0, 1.0, h, _r0(L), 2.5, eps=1e-5)
    assert np.max(np.abs(g - g_fd)) < 1e-8
    assert 0 < F < 1


def test_gradient_sums_to_zero():
    # a uniform field couples to S^z_total, which is constant in the sector
    L = 10
    h = M.fields(L, 1.5, BETA_GOLDEN, 0.3)
    _, g = G.dF_dh(L, L // 2, True, 1.0, 1.0, h, _r0(L), 5.0)
    assert abs(g.sum()) < 1e-12
    assert np.max(np.abs(g)) > 1e-3


def test_clean_ring_sublattice_pattern():
    # h = 0 ring: translation by two sites maps the Neel state to itself, so
    # dF/dh_i depends only on the sublattice, and the sum rule makes the two
    # values opposite.
    L = 8
    _, g = G.dF_dh(L, L // 2, True, 1.0, 1.0, np.zeros(L), _r0(L), 1.7)
    assert np.allclose(g[0::2], g[0], atol=1e-12)
    assert np.allclose(g[1::2], -g[0], atol=1e-12)
    assert abs(g[0]) > 1e-4


def test_finite_differences_through_expm_multiply_and_richardson():
    # the route of the L = 20 golden values: F from the mid-size propagator
    # (expm_multiply on the CSR H), central differences at eps and eps / 2
    # combined by one Richardson step, against the Daleckii-Krein derivative
    from oracle import hamiltonian as OH
    from oracle import midsize as OMS
    L, T = 10, 2.0
    h = M.fields(L, 1.5, BETA_GOLDEN, 0.7)
    r0 = _r0(L)

    def F(hh):
        return float(OMS.survival_probability(OH.build_csr(L, L // 2, True, 1.0, 1.0, hh), r0, [T])[0])

    _, g = G.dF_dh(L, L // 2, True, 1.0, 1.0, h, r0, T)
    idx = [0, 3, 7]
    d1 = G.dF_dh_finite_difference(L, L // 2, True, 1.0, 1.0, h, r0, T, eps=1e-3, propagate=F, indices=idx)
    d2 = G.dF_dh_finite_difference(L, L // 2, True, 1.0, 1.0, h, r0, T, eps=5e-4, propagate=F, indices=idx)
    rich = (4.0 * d2 - d1) / 3.0
    assert np.max(np.abs(d1 - g[idx])) < 1e-5          # O(eps^2) truncation visible
    assert np.max(np.abs(rich - g[idx])) < 1e-9          # removed by the Richardson step
