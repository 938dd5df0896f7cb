"""GPU tests of general particle-number sectors with 64-bit states (L > 32 at
low density, as in the paper's L = 55 runs of Sec. 4): the basis bit-exact,
ranks, y = H x (matrix-free rows and CSR, both dtypes, batches) against the
oracle, Krylov propagation against the free-fermion closed form and dense
propagation, and the adjoint gradient."""
import math

import numpy as np
import pytest
import torch

import paper_1704_02770_amd as qk
from gpu_util import max_rel, say, to_dev, to_host
from oracle import basis as OB
from oracle import exact as OX
from oracle import freefermion as OF
from oracle import gradient as OG
from oracle import hamiltonian as OH
from oracle import model as OM
from workloads import BETA_GOLDEN, phases, random_complex, random_fields

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-13, torch.complex64: 2e-6}


def _states(b):
    return to_host(qk.qk_basis_states(b)).view(np.uint64)


@pytest.mark.parametrize("L,N", [(33, 3), (40, 4), (55, 3), (63, 2), (64, 2), (64, 3)])
def test_wide_basis(L, N):
    say("wide basis", L, N)
    b = qk.qk_basis_build(L, N)
    D = qk.qk_basis_dim(b)
    assert D == math.comb(L, N)
    st = _states(b)
    # D distinct ascending L-bit integers of popcount N: exactly the sector
    assert len(st) == D and np.all(st[1:] > st[:-1])
    assert np.all(np.bitwise_count(st) == N)
    if L < 64:
        assert np.all(st >> np.uint64(L) == 0)
        assert np.array_equal(st.astype(np.int64), OB.sector_states(L, N))
    rows = np.array([0, 1, D // 2, D - 1])
    assert np.array_equal(qk.qk_basis_rank(b, st[rows]), rows)
    assert qk.qk_basis_rank(b, [np.uint64(1) << np.uint64(L - 1)])[0] == -1   # popcount 1 != N


def test_wide_basis_limits():
    with pytest.raises(qk.QkError):
        qk.qk_basis_build(65, 2)
    with pytest.raises(qk.QkError):
        qk.qk_basis_build(64, 32)   # C(64, 32) is not below 2^32


@pytest.mark.parametrize("mode", [qk.QK_MATFREE, qk.QK_CSR])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("L,N,pbc,Bn", [(40, 3, True, 1), (55, 3, False, 1), (63, 2, True, 3), (36, 4, True, 2)])
def test_wide_hv(L, N, pbc, Bn, mode, dtype):
    hs = np.stack([random_fields(L, 60 + i) for i in range(Bn)]) if Bn > 1 else random_fields(L, 60)
    b = qk.qk_basis_build(L, N)
    D = qk.qk_basis_dim(b)
    say("wide hv", L, N, pbc, Bn, mode, dtype)
    H = qk.qk_ham_create(b, 1.0, 0.6, pbc, hs, mode)
    X = random_complex(D * Bn, 70).reshape(D, Bn) if Bn > 1 else random_complex(D, 70)
    xd = to_dev(X, dtype)
    y = to_host(qk.qk_ham_apply(H, xd))
    Xc = to_host(xd).astype(np.complex128)
    if Bn == 1:
        ref = OH.build_csr(L, N, pbc, 1.0, 0.6, hs) @ Xc
    else:
        st = OB.sector_states(L, N)
        H0 = OH.build_csr(L, N, pbc, 1.0, 0.6, np.zeros(L))
        dfield = OH.diagonal(st, L, pbc, 0.6, hs) - OH.diagonal(st, L, pbc, 0.6, np.zeros(L))[:, None]
        ref = H0 @ Xc + dfield * Xc
    assert max_rel(y, ref) < TOL[dtype] * 4


@pytest.mark.parametrize("L,N,h", [(55, 1, 1.0), (55, 1, 2.5), (55, 3, 2.0), (64, 2, 1.0)])
def test_wide_krylov_free_fermions(L, N, h):
    # one particle (the paper's non-interacting runs at L = 55): the zz term is
    # a constant, so the closed form holds for jz = 1; several particles use jz = 0
    jz = 1.0 if N == 1 else 0.0
    b = qk.qk_basis_build(L, N)
    D = qk.qk_basis_dim(b)
    hf = OM.fields(L, h, BETA_GOLDEN, float(phases(1, 0)[0]))
    H = qk.qk_ham_create(b, 1.0, jz, True, hf)
    s0 = sum(1 << (j * (L // N)) for j in range(N))   # evenly spaced particles
    r0 = int(qk.qk_basis_rank(b, [s0])[0])
    psi = torch.zeros(D, dtype=torch.complex128, device="cuda")
    psi[r0] = 1.0
    k = qk.qk_krylov_create(H, 30)
    dt, steps = 0.25, 40
    P = torch.empty(steps, dtype=torch.float64, device="cuda")
    say("wide krylov free fermions", L, N, h)
    for s in range(steps):
        qk.qk_krylov_expm_step(k, psi, dt)
        qk.qk_return_prob(b, psi, r0=r0, out=P[s:s + 1])
    t = dt * np.arange(1, steps + 1)
    ref = OF.survival_probability(L, N, True, 1.0, hf, s0, t)
    assert np.max(np.abs(to_host(P) - ref)) < 1e-10


def test_wide_krylov_interacting_vs_dense():
    L, N = 40, 2
    b = qk.qk_basis_build(L, N)
    D = qk.qk_basis_dim(b)
    hf = OM.fields(L, 1.5, BETA_GOLDEN, 0.3)
    H = qk.qk_ham_create(b, 1.0, 1.0, True, hf)
    Hd = OH.build_dense(L, N, True, 1.0, 1.0, hf)
    r0 = 17
    psi = torch.zeros(D, dtype=torch.complex128, device="cuda")
    psi[r0] = 1.0
    k = qk.qk_krylov_create(H, 30)
    say("wide krylov dense")
    for _ in range(20):
        qk.qk_krylov_expm_step(k, psi, 0.1)
    e0 = np.zeros(D, complex)
    e0[r0] = 1
    assert np.linalg.norm(to_host(psi) - OX.evolve(Hd, e0, [2.0])[0]) < 1e-10


def test_wide_gradient_vs_daleckii_krein():
    L, N, T, n = 40, 2, 2.0, 20
    b = qk.qk_basis_build(L, N)
    hf = OM.fields(L, 2.0, BETA_GOLDEN, 0.8)
    H = qk.qk_ham_create(b, 1.0, 1.0, True, hf)
    k = qk.qk_krylov_create(H, 24)
    r0 = 101
    say("wide gradient")
    F, g = qk.qk_grad_return_prob(k, r0, T, n)
    F_ref, g_ref = OG.dF_dh(L, N, True, 1.0, 1.0, hf, r0, T)
    assert abs(F - F_ref) < 1e-10
    assert np.max(np.abs(g - g_ref)) < 1e-9 * max(1.0, np.max(np.abs(g_ref)))
