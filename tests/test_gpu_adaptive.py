"""GPU tests of adaptive time stepping with error control (the step-size
rule of Expokit, which the paper's runs use through SLEPc with a
tolerance): results against the oracle's exact propagation at small and
mid-size L, the effect of the tolerance, batches, complex64 storage and the
argument checks."""
import math

import numpy as np
import pytest
import torch

import paper_1704_02770_amd as qk
from gpu_util import max_rel, neel_row, say, to_host
from oracle import exact as OX
from oracle import hamiltonian as OH
from oracle import model as OM
from workloads import BETA_GOLDEN, phases

pytestmark = pytest.mark.gpu


def _setup(L, pbc=True, h=1.5, Bn=1, m=12, dtype=torch.complex128):
    b = qk.qk_basis_build(L, L // 2)
    if Bn == 1:
        hf = OM.fields(L, h, BETA_GOLDEN, phases(1, 0)[0])
    else:
        hf = np.stack([OM.fields(L, h, BETA_GOLDEN, p) for p in phases(Bn, 4)])
    H = qk.qk_ham_create(b, 1.0, 1.0, pbc, hf)
    k = qk.qk_krylov_create(H, m, dtype)
    D = qk.qk_basis_dim(b)
    r0 = neel_row(L)
    psi = torch.zeros((D, Bn) if Bn > 1 else D, dtype=dtype, device="cuda")
    psi[r0] = 1.0
    return b, H, k, psi, r0, hf


def _exact(L, pbc, hf, r0, t):
    Hd = OH.build_dense(L, L // 2, pbc, 1.0, 1.0, hf)
    e0 = np.zeros(len(Hd), complex)
    e0[r0] = 1.0
    return OX.evolve(Hd, e0, [t])[0]


@pytest.mark.parametrize("L,pbc,m,tol", [(10, True, 10, 1e-10), (12, False, 12, 1e-9), (12, True, 16, 1e-12)])
def test_adaptive_vs_exact(L, pbc, m, tol):
    t = 5.0
    b, H, k, psi, r0, hf = _setup(L, pbc, m=m)
    say("adaptive", L, pbc, m, tol)
    info = qk.qk_krylov_evolve(k, psi, t, tol, dt_init=1.0)
    ref = _exact(L, pbc, hf, r0, t)
    err = np.linalg.norm(to_host(psi) - ref)
    say("  steps", info["steps"], "dt", info["dt_min"], info["dt_max"], "err", err, "est", info["err_sum"])
    assert info["steps"] >= 2
    assert err < 20 * tol * t
    assert abs(torch.linalg.vector_norm(psi).item() - 1.0) < 1e-12
    # one fixed step over the whole interval with the same m is far off
    b2, H2, k2, psi2, _, _ = _setup(L, pbc, m=m)
    qk.qk_krylov_expm_step(k2, psi2, t)
    assert np.linalg.norm(to_host(psi2) - ref) > 1e3 * err


def test_tolerance_controls_steps_and_error():
    L, t = 12, 4.0
    res = {}
    for tol in (1e-5, 1e-8, 1e-11):
        b, H, k, psi, r0, hf = _setup(L, m=10)
        info = qk.qk_krylov_evolve(k, psi, t, tol, dt_init=0.5)
        res[tol] = (info["steps"], np.linalg.norm(to_host(psi) - _exact(L, True, hf, r0, t)))
        say("tol", tol, res[tol])
        assert res[tol][1] < 20 * tol * t
    assert res[1e-5][0] < res[1e-8][0] < res[1e-11][0]


def test_adaptive_blocked_path_vs_expm_multiply():
    from oracle import midsize as OMS
    L, t, tol = 20, 2.0, 1e-10
    b, H, k, psi, r0, hf = _setup(L, m=20)
    say("adaptive blocked", L)
    info = qk.qk_krylov_evolve(k, psi, t, tol, dt_init=0.5)
    P = abs(psi[r0].item()) ** 2
    Hc = OH.build_csr(L, L // 2, True, 1.0, 1.0, hf)
    F = OMS.survival_probability(Hc, r0, [t])[0]
    say("  steps", info["steps"], "dP", P - F)
    assert abs(P - F) < 1e-9


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_adaptive_batch(dtype):
    L, Bn, t = 12, 4, 3.0
    tol = 1e-10 if dtype == torch.complex128 else 1e-6
    b, H, k, psi, r0, hs = _setup(L, Bn=Bn, m=12, dtype=dtype)
    say("adaptive batch", dtype)
    info = qk.qk_krylov_evolve(k, psi, t, tol, dt_init=1.0)
    assert info["steps"] >= 2
    bound = 20 * tol * t if dtype == torch.complex128 else 1e-5
    for i in range(Bn):
        ref = _exact(L, True, hs[i], r0, t)
        got = to_host(psi[:, i].contiguous()).astype(np.complex128)
        assert np.linalg.norm(got - ref) < bound


def test_adaptive_zero_time_and_invalid_arguments():
    b, H, k, psi, r0, hf = _setup(10, m=8)
    before = to_host(psi).copy()
    info = qk.qk_krylov_evolve(k, psi, 0.0, 1e-8)
    assert info["steps"] == 0 and np.array_equal(to_host(psi), before)
    for kw in (dict(tol=0.0), dict(tol=-1.0), dict(tol=float("nan")), dict(tol=1e-8, dt_init=0.0),
               dict(tol=1e-8, dt_max=-1.0), dict(tol=1e-8, max_steps=0)):
        with pytest.raises(qk.QkError):
            qk.qk_krylov_evolve(k, psi, 1.0, **kw)
    with pytest.raises(qk.QkError):
        qk.qk_krylov_evolve(k, psi, -1.0, 1e-8)
    # too few steps allowed for the requested accuracy
    with pytest.raises(qk.QkError):
        qk.qk_krylov_evolve(k, psi, 50.0, 1e-12, dt_init=1.0, max_steps=2)
