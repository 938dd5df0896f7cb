"""The C ABI without a GPU: the library loads, exports every symbol that
include/qk.h declares, and rejects bad arguments before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qk.h")
LIB = os.path.join(ROOT, "paper_1704_02770_amd", "libqkrylov.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libqkrylov.so not built (run python paper_1704_02770_amd/build.py)")


def header_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qk_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_core_calls():
    syms = header_symbols()
    for name in ["qk_basis_build", "qk_ham_apply", "qk_krylov_expm_step", "qk_return_prob"]:
        assert name in syms


def test_library_exports_every_header_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (qk_[a-z0-9_]+)\b", out))
    missing = [s for s in header_symbols() if s not in exported]
    assert not missing, missing
    # nothing beyond the header is exported under the qk_ prefix
    assert exported <= set(header_symbols())


def test_binding_covers_every_symbol():
    import paper_1704_02770_amd as qk
    from paper_1704_02770_amd import _native
    assert set(_native.SIGNATURES) == set(header_symbols())
    for s in header_symbols():
        if s.endswith("_destroy") or s == "qk_last_error":
            continue
        assert hasattr(qk, s), s


def test_version_and_validation_without_device():
    import paper_1704_02770_amd as qk
    from paper_1704_02770_amd._native import lib
    assert qk.qk_abi_version() == 2
    out = C.c_void_p()
    assert lib.qk_basis_build(65, 2, None, C.byref(out)) == qk.QK_EINVAL
    assert b"L must be" in lib.qk_last_error()
    # C(40, 20) > 2^32: 64-bit states are supported, but not sectors that large
    assert lib.qk_basis_build(40, 20, None, C.byref(out)) == qk.QK_EUNSUPPORTED
    assert b"below 2^32" in lib.qk_last_error()
    assert lib.qk_basis_build(1, 1, None, C.byref(out)) == qk.QK_EINVAL
    assert lib.qk_basis_build(8, 0, None, C.byref(out)) == qk.QK_EINVAL
    assert lib.qk_basis_build(8, 8, None, C.byref(out)) == qk.QK_EINVAL
    assert lib.qk_basis_build(8, 4, None, None) == qk.QK_EINVAL
    assert lib.qk_ham_apply(None, None, None, 0, None) == qk.QK_EINVAL
    assert lib.qk_krylov_create(None, 30, 0, 0, C.byref(out)) == qk.QK_EINVAL
    assert lib.qk_krylov_expm_step(None, None, 0.1, None, None) == qk.QK_EINVAL
    assert lib.qk_return_prob(None, 0, None, None, 0, 1, None, None) == qk.QK_EINVAL
    D = C.c_int64()
    assert lib.qk_basis_dim(None, C.byref(D)) == qk.QK_EINVAL
    lib.qk_basis_destroy(None)
    lib.qk_ham_destroy(None)
    lib.qk_krylov_destroy(None)


def test_fields_host_function():
    # host-side field generation of Eq. (1); checked against the definition
    import paper_1704_02770_amd as qk
    from oracle import model
    from workloads import BETA_GOLDEN, phases
    phi = phases(3, 0)
    got = qk.qk_fields_quasiperiodic(28, 1.5, BETA_GOLDEN, phi)
    for b in range(3):
        assert np.allclose(got[b], model.fields(28, 1.5, BETA_GOLDEN, phi[b]), rtol=0, atol=1e-14)
    with pytest.raises(qk.QkError):
        qk.qk_fields_quasiperiodic(0, 1.0, 0.5, [0.0])
    with pytest.raises(qk.QkError):
        qk.qk_fields_quasiperiodic(8, float("nan"), 0.5, [0.0])


def test_set_allocator_validation():
    import paper_1704_02770_amd as qk
    from paper_1704_02770_amd import _native
    from paper_1704_02770_amd._native import lib
    calls = []
    fa = _native.ALLOC_FN(lambda n, s, c: calls.append(n))
    fr = _native.RELEASE_FN(lambda p, s, c: calls.append(p))
    none_a, none_r = C.cast(None, _native.ALLOC_FN), C.cast(None, _native.RELEASE_FN)
    assert lib.qk_set_allocator(fa, none_r, None) == qk.QK_EINVAL
    assert b"both" in lib.qk_last_error()
    assert lib.qk_set_allocator(none_a, fr, None) == qk.QK_EINVAL
    assert lib.qk_set_allocator(fa, fr, None) == qk.QK_OK
    # a rejected create allocates nothing
    out = C.c_void_p()
    assert lib.qk_basis_build(65, 2, None, C.byref(out)) == qk.QK_EINVAL
    assert lib.qk_set_allocator(none_a, none_r, None) == qk.QK_OK
    assert calls == []
    with pytest.raises(ValueError):
        qk.qk_set_allocator(alloc=lambda n, s: 0)
    qk.qk_set_allocator()


def test_argument_validation_property():
    # random arguments at the boundary: every call returns a status from the
    # documented set (no crash, no exception), and invalid shapes are EINVAL
    # or EUNSUPPORTED before any device work (here there is no device at all)
    from hypothesis import given, settings
    from hypothesis import strategies as st
    import paper_1704_02770_amd as qk
    from paper_1704_02770_amd._native import lib
    from math import comb

    @settings(max_examples=300, deadline=None)
    @given(L=st.integers(-4, 72), n=st.integers(-4, 72))
    def basis(L, n):
        out = C.c_void_p()
        if 2 <= L <= 64 and 0 < n < L and 1e6 < comb(L, n) < 0xFFFFFFFF:
            return   # a valid sector too large to build in a unit test where a device exists
        s = lib.qk_basis_build(L, n, None, C.byref(out))
        if L < 2 or L > 64 or n <= 0 or n >= L:
            assert s == qk.QK_EINVAL
        elif comb(L, n) >= 0xFFFFFFFF:
            assert s == qk.QK_EUNSUPPORTED
        else:
            assert s in (qk.QK_OK, qk.QK_EHIP, qk.QK_ENOMEM)
            if s == qk.QK_OK:
                lib.qk_basis_destroy(out)

    @settings(max_examples=200, deadline=None)
    @given(L=st.integers(-2, 70), h=st.floats(allow_nan=True, allow_infinity=True),
           beta=st.floats(-2, 2), nphi=st.integers(0, 3))
    def fields(L, h, beta, nphi):
        phi = np.zeros(max(nphi, 1))
        out = np.zeros((max(nphi, 1), max(L, 1)))
        s = lib.qk_fields_quasiperiodic(L, h, beta, phi.ctypes.data_as(C.POINTER(C.c_double)), nphi,
                                        out.ctypes.data_as(C.POINTER(C.c_double)))
        ok = 1 <= L <= 64 and nphi >= 1 and np.isfinite(h)
        assert s == (qk.QK_OK if ok else qk.QK_EINVAL)

    basis()
    fields()
