"""Handle memory from a caller's allocator (qk_set_allocator).

torch's caching allocator gives bitwise the results of hipMalloc, its
accounting sees the workspaces and gets them back on destroy; an allocator
that runs dry is reported as QK_ENOMEM and every block it did hand out comes
back (no leak on any failure point).
"""
import gc

import numpy as np
import pytest
import torch

import paper_1704_02770_amd as qk
from gpu_util import neel_row, say
from workloads import BETA_GOLDEN, phases

pytestmark = pytest.mark.gpu

L = 20   # blocked H-pass (L >= 18): its tables come from the allocator too


@pytest.fixture(autouse=True)
def _default_allocator_after():
    yield
    qk.qk_set_allocator()


def _handles(mode=qk.QK_MATFREE, reorth=0):
    b = H = k = None
    try:
        b = qk.qk_basis_build(L, L // 2)
        h = qk.qk_fields_quasiperiodic(L, 1.5, BETA_GOLDEN, phases(1, 0))
        H = qk.qk_ham_create(b, 1.0, 1.0, True, h, mode=mode)
        k = qk.qk_krylov_create(H, 30, torch.complex128, reorth)
        return b, H, k
    except Exception:
        for x in (k, H, b):
            if x is not None:
                x.close()
        raise


def _evolve(k, D, r0, n=5):
    psi = torch.zeros(D, dtype=torch.complex128, device="cuda")
    psi[r0] = 1.0
    for _ in range(n):
        qk.qk_krylov_expm_step(k, psi, 0.1)
    torch.cuda.synchronize()
    return psi


def _close(*hs):
    for x in hs:
        x.close()


@pytest.mark.parametrize("mode,reorth", [(qk.QK_MATFREE, 0), (qk.QK_CSR, 2)])
def test_torch_allocator_bitwise_and_accounting(mode, reorth):
    r0 = neel_row(L)
    say("allocator default", L, mode, reorth)
    b, H, k = _handles(mode, reorth)
    D = qk.qk_basis_dim(b)
    ref = _evolve(k, D, r0)
    g_ref = qk.qk_grad_return_prob(k, r0, 1.0, 10, 3)
    psi0 = torch.roll(ref, 7).contiguous()   # general initial state: stream-ordered temporary
    P_ref = qk.qk_return_prob(b, ref, psi0=psi0).cpu()
    _close(k, H, b)

    say("allocator torch", L, mode, reorth)
    psi = torch.zeros(D, dtype=torch.complex128, device="cuda")
    psi[r0] = 1.0
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    qk.use_torch_allocator()
    b, H, k = _handles(mode, reorth)
    qk.qk_set_allocator()   # handles keep the allocator they were created with
    m1 = torch.cuda.memory_allocated()
    assert m1 - m0 >= 30 * D * 16 + 4 * D   # Krylov basis + the sorted states
    for _ in range(5):
        qk.qk_krylov_expm_step(k, psi, 0.1)
    torch.cuda.synchronize()
    assert torch.equal(psi, ref)
    g = qk.qk_grad_return_prob(k, r0, 1.0, 10, 3)   # temporaries through the allocator
    assert g[0] == g_ref[0] and np.array_equal(g[1], g_ref[1])
    assert torch.cuda.memory_allocated() == m1
    P = qk.qk_return_prob(b, psi, psi0=psi0).cpu()
    assert torch.equal(P, P_ref)
    assert torch.cuda.memory_allocated() == m1
    _close(k, H, b)
    assert torch.cuda.memory_allocated() == m0


def test_exhausted_allocator_reports_enomem_without_leak():
    live = {}
    calls = {"n": 0, "limit": 0}

    def alloc(n, stream):
        if calls["n"] >= calls["limit"]:
            return 0
        calls["n"] += 1
        p = torch.cuda.caching_allocator_alloc(n, stream=stream or None)
        live[p] = n
        return p

    def release(p, stream):
        del live[p]
        torch.cuda.caching_allocator_delete(p)

    r0 = neel_row(L)
    # count the blocks a full set of handles plus one gradient call takes
    qk.qk_set_allocator(alloc, release)
    calls["limit"] = 1 << 30
    b, H, k = _handles()
    need = calls["n"]
    _close(k, H, b)
    assert not live and need >= 10
    # fail at every allocation in turn
    for limit in range(need):
        say("allocator limit", limit, "of", need)
        calls["n"], calls["limit"] = 0, limit
        with pytest.raises(qk.QkError) as ei:
            _handles()
        assert ei.value.status == qk.QK_ENOMEM
        assert not live, (limit, live)
    # a gradient call whose temporaries cannot be had fails cleanly and the
    # workspace still works afterwards
    calls["n"], calls["limit"] = 0, need
    b, H, k = _handles()
    n_handles = len(live)
    with pytest.raises(qk.QkError) as ei:
        qk.qk_grad_return_prob(k, r0, 1.0, 10, 3)
    assert ei.value.status == qk.QK_ENOMEM and len(live) == n_handles
    psi = _evolve(k, qk.qk_basis_dim(b), r0, 1)
    assert abs(float(torch.linalg.vector_norm(psi)) - 1.0) < 1e-12
    _close(k, H, b)
    assert not live


def _batch_run(dt=0.1, steps=5):
    """Two workspaces (L = 20 complex64 with two phases, L = 18 complex128) in one
    graph-driven batch; returns P and the handles to close."""
    hs = []
    b1 = qk.qk_basis_build(20, 10)
    H1 = qk.qk_ham_create(b1, 1.0, 1.0, True, qk.qk_fields_quasiperiodic(20, 2.0, BETA_GOLDEN, phases(2, 3)))
    k1 = qk.qk_krylov_create(H1, 30, torch.complex64)
    b2 = qk.qk_basis_build(18, 9)
    H2 = qk.qk_ham_create(b2, 1.0, 1.0, False, qk.qk_fields_quasiperiodic(18, 2.0, BETA_GOLDEN, phases(1, 4)))
    k2 = qk.qk_krylov_create(H2, 30, torch.complex128)
    hs += [k1, H1, b1, k2, H2, b2]
    r1, r2 = neel_row(20), neel_row(18)
    p1 = torch.zeros(qk.qk_basis_dim(b1) * 2, dtype=torch.complex64, device="cuda")
    p1[2 * r1] = 1.0
    p1[2 * r1 + 1] = 1.0
    p2 = torch.zeros(qk.qk_basis_dim(b2), dtype=torch.complex128, device="cuda")
    p2[r2] = 1.0
    bt = qk.qk_batch_create([k1, k2], [p1, p2], [r1, r2])
    hs.insert(0, bt)
    P = qk.qk_batch_run(bt, dt, steps, use_graph=True).cpu()
    torch.cuda.synchronize()
    return P, hs


def test_batch_autotune_and_side_stream_through_torch_allocator(tmp_path):
    say("allocator batch default")
    P_ref, hs = _batch_run()
    _close(*hs)
    del hs
    gc.collect()
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    qk.use_torch_allocator()
    say("allocator batch torch")
    P, hs = _batch_run()
    assert torch.equal(P, P_ref)
    assert torch.cuda.memory_allocated() > m0
    _close(*hs)
    del hs                      # the batch wrapper keeps its state vectors alive
    gc.collect()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == m0

    # autotuner scratch and a stream-ordered temporary on a side stream
    say("allocator autotune torch")
    b, H, k = _handles()
    D = qk.qk_basis_dim(b)
    psi = _evolve(k, D, neel_row(L), 2)
    psi0 = torch.roll(psi, 3).contiguous()
    P_cur = qk.qk_return_prob(b, psi, psi0=psi0).cpu()
    torch.cuda.synchronize()
    m1 = torch.cuda.memory_allocated()
    shape = qk.qk_krylov_autotune(k, 0.1, cache_path=str(tmp_path / "shapes.json"))
    assert shape["blocked_wgs_per_cu"] >= 0
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == m1
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        qk.qk_return_prob(b, psi, psi0=psi0, out=out, stream=side)
    side.synchronize()
    assert torch.equal(out.cpu(), P_cur)
    del out
    _close(k, H, b)
