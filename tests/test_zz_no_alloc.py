"""The allocation-free survival probability (qk_return_prob_noalloc), called
through the C ABI, against qk_return_prob (Sec. 4's F = |<psi0|psi>|^2) on
two calls in a row, the second with a smaller input: the same kernels on the
same data, so the results agree bitwise; the reference call draws its
temporary from a counting allocator, the allocation-free call draws nothing."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_1704_02770_amd as qk
from paper_1704_02770_amd._native import lib
from gpu_util import say, to_host
from workloads import random_complex

pytestmark = pytest.mark.gpu


def _states(D, B, seed, dtype):
    z = random_complex(D * B, seed).reshape(D, B)
    z = z / np.linalg.norm(z, axis=0)
    t = torch.from_numpy(np.ascontiguousarray(z if B > 1 else z[:, 0]))
    return t.to(device="cuda", dtype=dtype), z


def _noalloc(b, r0, psi0, psi, batch, out):
    st = lib.qk_return_prob_noalloc(b.ptr, r0, None if psi0 is None else psi0.data_ptr(), psi.data_ptr(),
                                    qk.dtype_code(psi), batch, out.data_ptr(),
                                    torch.cuda.current_stream().cuda_stream)
    return st


@pytest.fixture(autouse=True)
def _default_allocator_after():
    yield
    qk.qk_set_allocator()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_noalloc_matches_return_prob_twice(dtype):
    calls = {"n": 0}

    def alloc(n, stream):
        calls["n"] += 1
        return torch.cuda.caching_allocator_alloc(n, stream=stream or None)

    # two calls in a row: a larger input (L = 18, 8 columns), then a smaller one (L = 12, 2 columns)
    for L, B, seed in ((18, 8, 3), (12, 2, 4)):
        qk.qk_set_allocator(alloc, lambda p, stream: torch.cuda.caching_allocator_delete(p))
        b = qk.qk_basis_build(L, L // 2)
        qk.qk_set_allocator()
        D = qk.qk_basis_dim(b)
        psi0, z0 = _states(D, B, seed, dtype)
        psi, z1 = _states(D, B, seed + 100, dtype)
        ref = torch.empty(B, dtype=torch.float64, device="cuda")
        got = torch.full((B,), -1.0, dtype=torch.float64, device="cuda")
        say("no-alloc return_prob", L, B, dtype)
        n0 = calls["n"]
        qk.qk_return_prob(b, psi, psi0=psi0, batch=B, out=ref)
        torch.cuda.synchronize()
        assert calls["n"] == n0 + 1          # the reference drew its temporary
        assert _noalloc(b, -1, psi0, psi, B, got) == 0
        torch.cuda.synchronize()
        assert calls["n"] == n0 + 1          # the allocation-free call drew nothing
        r, g = to_host(ref), to_host(got)
        assert np.array_equal(r, g), (r, g)
        # and against the overlap computed on the host from the same values
        a = to_host(psi0).astype(np.complex128).reshape(D, B)
        c = to_host(psi).astype(np.complex128).reshape(D, B)
        host = np.abs(np.sum(np.conj(a) * c, axis=0)) ** 2
        tol = 1e-13 if dtype == torch.complex128 else 1e-6
        assert np.max(np.abs(g - host)) < tol
        # basis-state form (psi0 = NULL): one element per column
        r0 = 5
        assert _noalloc(b, r0, None, psi, B, got) == 0
        assert np.allclose(to_host(got), np.abs(c[r0]) ** 2, rtol=1e-6 if dtype == torch.complex64 else 1e-14,
                           atol=0)
        b.close()


def test_noalloc_rejects_bad_arguments():
    b = qk.qk_basis_build(10, 5)
    D = qk.qk_basis_dim(b)
    psi = torch.zeros(D, dtype=torch.complex128, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    say("no-alloc invalid arguments")
    assert _noalloc(b, -1, psi, psi, 65, out) == qk.QK_EINVAL
    assert _noalloc(b, D, None, psi, 1, out) == qk.QK_EINVAL
    st = lib.qk_return_prob_noalloc(b.ptr, 0, None, psi.data_ptr(), 7, 1, out.data_ptr(), None)
    assert st == qk.QK_EINVAL
    assert b"dtype" in lib.qk_last_error()
    b.close()
