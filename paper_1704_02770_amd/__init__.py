"""Python binding of libqkrylov (include/qk.h): Krylov time evolution of a
spin-1/2 XXZ chain with on-site fields on an MI355X (arXiv:1704.02770).

Every function here has the name of the C entry point it calls and only
marshals arguments: torch tensors supply device memory (their data pointers)
and streams (torch's current HIP stream); all computation runs in the HIP
kernels of the library.  Failures raise QkError with the library's message.
"""
from __future__ import annotations

import ctypes as C
import sys

import numpy as np
import torch

from . import _native
from ._native import AdaptInfo, AdaptParams, HamParams, KernelTime, LaunchShape, StepInfo, lib

QK_OK, QK_EINVAL, QK_ENOMEM, QK_EHIP, QK_EUNSUPPORTED, QK_ENUMERIC = range(6)
QK_C128, QK_C64 = 0, 1
QK_MATFREE, QK_CSR, QK_MATFREE_ROWS = 0, 1, 2

_DTYPE = {torch.complex128: QK_C128, torch.complex64: QK_C64}
TORCH_DTYPE = {QK_C128: torch.complex128, QK_C64: torch.complex64}


class QkError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.qk_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")


def _check(status: int, where: str) -> None:
    if status != QK_OK:
        raise QkError(status, where)


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dptr(t: torch.Tensor) -> C.c_void_p:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def dtype_code(t: torch.Tensor) -> int:
    try:
        return _DTYPE[t.dtype]
    except KeyError:
        raise ValueError(f"unsupported dtype {t.dtype}") from None


class _Handle:
    """Owns one library handle; released by the matching *_destroy."""
    _destroy = None

    def __init__(self, ptr: C.c_void_p, keep=()):
        self.ptr = ptr
        self._keep = keep   # objects that must outlive this handle

    def close(self):
        if self.ptr is not None and self.ptr.value:
            type(self)._destroy(self.ptr)
        self.ptr = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the process is about to release the device
        # anyway, and a destroy could call back into a Python allocator that
        # is already torn down (the check is bound at definition time, since
        # module globals may already be cleared then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Basis(_Handle):
    _destroy = staticmethod(lib.qk_basis_destroy)


class Ham(_Handle):
    _destroy = staticmethod(lib.qk_ham_destroy)


class Krylov(_Handle):
    _destroy = staticmethod(lib.qk_krylov_destroy)


class Batch(_Handle):
    _destroy = staticmethod(lib.qk_batch_destroy)


# every callback pair ever registered stays referenced: handles created with
# it keep calling it until they are destroyed
_allocator_refs = []


def qk_set_allocator(alloc=None, release=None) -> None:
    """Device memory of handles created from now on comes from
    alloc(nbytes, stream) -> int pointer (0 on failure) and returns through
    release(pointer, stream); stream is the raw HIP stream (an int) a
    temporary is ordered on, or 0 for memory that may be used on any stream
    (released only after the device work on it has finished).  Both None
    restores hipMalloc / hipFree.  Existing handles keep their allocator."""
    if alloc is None and release is None:
        _check(lib.qk_set_allocator(C.cast(None, _native.ALLOC_FN), C.cast(None, _native.RELEASE_FN), None),
               "qk_set_allocator")
        return
    if alloc is None or release is None:
        raise ValueError("alloc and release must both be given")

    def _alloc(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0))) or None
        except Exception:   # reported by the library as QK_ENOMEM
            return None

    def _release(ptr, stream, ctx):
        try:
            release(int(ptr), int(stream or 0))
        except Exception:   # nothing can be reported through a release; the block stays allocated
            pass

    fa, fr = _native.ALLOC_FN(_alloc), _native.RELEASE_FN(_release)
    _allocator_refs.append((fa, fr))
    _check(lib.qk_set_allocator(fa, fr, None), "qk_set_allocator")


def use_torch_allocator() -> None:
    """Handles created from now on take their device memory from torch's
    caching allocator (torch.cuda.memory_allocated counts it)."""
    def alloc(n, stream):
        # a block used on any stream is released after a synchronisation, so
        # the stream torch files it under does not matter
        return torch.cuda.caching_allocator_alloc(n, stream=stream or None)

    qk_set_allocator(alloc, lambda p, stream: torch.cuda.caching_allocator_delete(p))


def qk_abi_version() -> int:
    return int(lib.qk_abi_version())


def qk_fields_quasiperiodic(L: int, h: float, beta: float, phi) -> np.ndarray:
    """Fields h*cos(2*pi*beta*i + phi_b), i = 1..L, for every phase: shape (batch, L)."""
    phi = np.ascontiguousarray(np.atleast_1d(phi), dtype=np.float64)
    out = np.empty((len(phi), L), dtype=np.float64)
    _check(lib.qk_fields_quasiperiodic(L, h, beta, phi.ctypes.data_as(C.POINTER(C.c_double)), len(phi),
                                       out.ctypes.data_as(C.POINTER(C.c_double))), "qk_fields_quasiperiodic")
    return out


def qk_basis_build(L: int, n_up: int, stream=None) -> Basis:
    out = C.c_void_p()
    _check(lib.qk_basis_build(L, n_up, _stream(stream), C.byref(out)), "qk_basis_build")
    return Basis(out)


def qk_basis_dim(b: Basis) -> int:
    D = C.c_int64()
    _check(lib.qk_basis_dim(b.ptr, C.byref(D)), "qk_basis_dim")
    return D.value


def qk_basis_shape(b: Basis) -> tuple[int, int]:
    L, N = C.c_int32(), C.c_int32()
    _check(lib.qk_basis_shape(b.ptr, C.byref(L), C.byref(N)), "qk_basis_shape")
    return L.value, N.value


def qk_basis_states(b: Basis, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The sorted states as a device tensor holding their bit patterns: int32
    (uint32 patterns) for L <= 32, int64 (uint64 patterns) for L > 32."""
    D = qk_basis_dim(b)
    L, _ = qk_basis_shape(b)
    width = 8 if L > 32 else 4
    if out is None:
        out = torch.empty(D, dtype=torch.int64 if width == 8 else torch.int32, device="cuda")
    if out.numel() != D or out.element_size() != width:
        raise ValueError(f"out must hold D {8 * width}-bit integers")
    _check(lib.qk_basis_states(b.ptr, _dptr(out), _stream(stream)), "qk_basis_states")
    return out


def qk_basis_rank(b: Basis, states) -> np.ndarray:
    st = np.ascontiguousarray(np.atleast_1d(states), dtype=np.uint64)
    idx = np.empty(len(st), dtype=np.int64)
    _check(lib.qk_basis_rank(b.ptr, st.ctypes.data_as(C.POINTER(C.c_uint64)), len(st),
                             idx.ctypes.data_as(C.POINTER(C.c_int64))), "qk_basis_rank")
    return idx


def qk_ham_create(b: Basis, jxy: float, jz: float, pbc: bool, fields, mode: int = QK_MATFREE,
                  stream=None) -> Ham:
    """fields: (L,) or (batch, L) host array of on-site fields."""
    f = np.ascontiguousarray(np.atleast_2d(np.asarray(fields, dtype=np.float64)))
    p = HamParams(float(jxy), float(jz), int(bool(pbc)), int(mode))
    out = C.c_void_p()
    _check(lib.qk_ham_create(b.ptr, C.byref(p), f.ctypes.data_as(C.POINTER(C.c_double)), f.shape[0],
                             _stream(stream), C.byref(out)), "qk_ham_create")
    H = Ham(out, keep=(b,))
    H.L = qk_basis_shape(b)[0]
    return H


def qk_ham_set_fields(H: Ham, fields, stream=None) -> None:
    f = np.ascontiguousarray(np.atleast_2d(np.asarray(fields, dtype=np.float64)))
    _check(lib.qk_ham_set_fields(H.ptr, f.ctypes.data_as(C.POINTER(C.c_double)), f.shape[0], _stream(stream)),
           "qk_ham_set_fields")


def qk_ham_get_fields(H: Ham) -> np.ndarray:
    """The current field sets, shape (batch, L) (host copy)."""
    _, Bn, _ = qk_ham_shape(H)
    out = np.empty((Bn, H.L), dtype=np.float64)
    _check(lib.qk_ham_get_fields(H.ptr, out.ctypes.data_as(C.POINTER(C.c_double)), Bn), "qk_ham_get_fields")
    return out


def qk_ham_shape(H: Ham) -> tuple[int, int, int]:
    D, Bn, mode = C.c_int64(), C.c_int32(), C.c_int32()
    _check(lib.qk_ham_shape(H.ptr, C.byref(D), C.byref(Bn), C.byref(mode)), "qk_ham_shape")
    return D.value, Bn.value, mode.value


def _check_vec(H_or_D, t: torch.Tensor, batch: int, name: str):
    D = H_or_D
    if t.numel() != D * batch:
        raise ValueError(f"{name} must hold D*batch = {D * batch} elements, got {t.numel()}")


def qk_ham_apply(H: Ham, x: torch.Tensor, y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """y = H x; x is (D,) or (D, batch) complex128/complex64 on the device."""
    D, Bn, _ = qk_ham_shape(H)
    _check_vec(D, x, Bn, "x")
    if y is None:
        y = torch.empty_like(x)
    if y.dtype != x.dtype:
        raise ValueError("x and y dtypes differ")
    _check_vec(D, y, Bn, "y")
    _check(lib.qk_ham_apply(H.ptr, _dptr(x), _dptr(y), dtype_code(x), _stream(stream)), "qk_ham_apply")
    return y


def qk_krylov_create(H: Ham, m: int, dtype=torch.complex128, reorth: int = 0) -> Krylov:
    out = C.c_void_p()
    code = _DTYPE[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
    _check(lib.qk_krylov_create(H.ptr, m, code, reorth, C.byref(out)), "qk_krylov_create")
    k = Krylov(out, keep=(H,))
    k.m, k.dtype, k.H = m, code, H
    return k


def qk_krylov_expm_step(k: Krylov, psi: torch.Tensor, dt: float, stream=None, info: bool = False):
    """psi <- exp(-i dt H) psi in place.  With info=True waits and returns a
    list of dicts (m_used, status, err_est, beta0), one per batch item."""
    D, Bn, _ = qk_ham_shape(k.H)
    _check_vec(D, psi, Bn, "psi")
    if dtype_code(psi) != k.dtype:
        raise ValueError("psi dtype differs from the workspace dtype")
    if not info:
        _check(lib.qk_krylov_expm_step(k.ptr, _dptr(psi), float(dt), _stream(stream), None), "qk_krylov_expm_step")
        return None
    arr = (StepInfo * Bn)()
    st = lib.qk_krylov_expm_step(k.ptr, _dptr(psi), float(dt), _stream(stream), arr)
    res = [dict(m_used=a.m_used, status=a.status, err_est=a.err_est, beta0=a.beta0) for a in arr]
    if st not in (QK_OK, QK_ENUMERIC):
        _check(st, "qk_krylov_expm_step")
    return res


def qk_krylov_evolve(k: Krylov, psi: torch.Tensor, t: float, tol: float, dt_init: float = 0.1,
                     dt_max: float = 1e30, max_steps: int = 1000000, stream=None) -> dict:
    """psi <- exp(-i t H) psi in place by adaptive Krylov steps with error
    control (tol per unit time).  Returns steps, dt_min, dt_max, err_sum."""
    D, Bn, _ = qk_ham_shape(k.H)
    _check_vec(D, psi, Bn, "psi")
    if dtype_code(psi) != k.dtype:
        raise ValueError("psi dtype differs from the workspace dtype")
    prm = AdaptParams(float(tol), float(dt_init), float(dt_max), int(max_steps))
    inf = AdaptInfo()
    _check(lib.qk_krylov_evolve(k.ptr, _dptr(psi), float(t), C.byref(prm), _stream(stream), C.byref(inf)),
           "qk_krylov_evolve")
    return dict(steps=inf.steps, dt_min=inf.dt_min, dt_max=inf.dt_max, err_sum=inf.err_sum)


def qk_krylov_coefficients(k: Krylov, item: int = 0):
    """(alpha, beta, m_used) of the last completed step for one batch item."""
    a = np.zeros(k.m)
    b = np.zeros(k.m)
    mu = C.c_int32()
    _check(lib.qk_krylov_coefficients(k.ptr, item, a.ctypes.data_as(C.POINTER(C.c_double)),
                                      b.ctypes.data_as(C.POINTER(C.c_double)), C.byref(mu)),
           "qk_krylov_coefficients")
    return a[: mu.value], b[: mu.value], mu.value


KERNEL_KINDS = ("lanczos_h", "lanczos_update", "small_expm", "combine", "prepass")


def qk_krylov_profile(k: Krylov, enable: bool = True) -> None:
    """Start (totals reset) or stop HIP-event timing of every kernel of later steps."""
    _check(lib.qk_krylov_profile(k.ptr, int(bool(enable))), "qk_krylov_profile")


def qk_krylov_profile_read(k: Krylov) -> dict:
    """{kind: (milliseconds summed, launches)} since profiling was enabled (waits)."""
    arr = (KernelTime * len(KERNEL_KINDS))()
    _check(lib.qk_krylov_profile_read(k.ptr, arr), "qk_krylov_profile_read")
    return {name: (arr[i].ms_total, arr[i].launches) for i, name in enumerate(KERNEL_KINDS)}


def _shape_dict(sh: LaunchShape) -> dict:
    return dict(threads=sh.threads, blocks_per_cu=sh.blocks_per_cu, blocked_wgs_per_cu=sh.blocked_wgs_per_cu,
                blocked_llo=sh.blocked_llo)


def qk_krylov_set_shape(k: Krylov, threads: int = 0, blocks_per_cu: int = 0, blocked_wgs_per_cu: int = 0,
                        blocked_llo: int = 0) -> None:
    """blocked_llo != 0 rebuilds the block tables of the workspace's Hamiltonian."""
    sh = LaunchShape(threads, blocks_per_cu, blocked_wgs_per_cu, blocked_llo)
    _check(lib.qk_krylov_set_shape(k.ptr, C.byref(sh)), "qk_krylov_set_shape")


def qk_krylov_get_shape(k: Krylov) -> dict:
    sh = LaunchShape()
    _check(lib.qk_krylov_get_shape(k.ptr, C.byref(sh)), "qk_krylov_get_shape")
    return _shape_dict(sh)


def qk_krylov_autotune(k: Krylov, dt: float, cache_path: str | None = None, stream=None) -> dict:
    """Times launch shapes for one step of this workspace and applies the
    fastest (looked up in / stored to the JSON file `cache_path`)."""
    sh = LaunchShape()
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib.qk_krylov_autotune(k.ptr, float(dt), path, _stream(stream), C.byref(sh)), "qk_krylov_autotune")
    return _shape_dict(sh)


def qk_batch_create(ks, psis, r0s) -> Batch:
    """Groups workspaces with their state vectors and initial basis rows
    (r0 < 0: the vector as given is the initial state; its overlap is recorded)."""
    n = len(ks)
    if not (len(psis) == len(r0s) == n):
        raise ValueError("ks, psis and r0s must have the same length")
    for k, p in zip(ks, psis):
        D, Bn, _ = qk_ham_shape(k.H)
        _check_vec(D, p, Bn, "psi")
        if dtype_code(p) != k.dtype:
            raise ValueError("psi dtype differs from its workspace")
    karr = (C.c_void_p * n)(*[k.ptr.value for k in ks])
    parr = (C.c_void_p * n)(*[p.data_ptr() for p in psis])
    rarr = (C.c_int64 * n)(*[int(r) for r in r0s])
    out = C.c_void_p()
    _check(lib.qk_batch_create(karr, parr, rarr, n, C.byref(out)), "qk_batch_create")
    return Batch(out, keep=(tuple(ks), tuple(psis)))


def qk_batch_items(b: Batch) -> int:
    n = C.c_int32()
    _check(lib.qk_batch_items(b.ptr, C.byref(n)), "qk_batch_items")
    return n.value


def _graph_mode(use_graph) -> int:
    """0 (direct launches), 1 (graph of one branch per workspace) or 2 (graph of
    the persistent step kernel); a bool means 0 or 1."""
    if isinstance(use_graph, bool):
        return int(use_graph)
    m = int(use_graph)
    if m not in (0, 1, 2):
        raise ValueError("use_graph must be 0, 1 or 2")
    return m


def qk_batch_run(b: Batch, dt: float, n_steps: int, use_graph: bool | int = True, out: torch.Tensor | None = None,
                 stream=None) -> torch.Tensor:
    """n_steps steps of every workspace; returns the device tensor P[n_steps, items].
    use_graph: 0/False direct launches, 1/True one graph branch per workspace,
    2 the persistent step kernel (one launch per step, captured in a graph)."""
    items = qk_batch_items(b)
    if out is None:
        out = torch.empty((n_steps, items), dtype=torch.float64, device="cuda")
    if out.numel() < n_steps * items or out.dtype != torch.float64:
        raise ValueError("out must be a float64 tensor of n_steps * items entries")
    _check(lib.qk_batch_run(b.ptr, float(dt), int(n_steps), _graph_mode(use_graph), _dptr(out), _stream(stream)),
           "qk_batch_run")
    return out


def qk_batch_run_autocorr(b: Batch, dt: float, n_steps: int, use_graph: bool | int = True,
                          out: torch.Tensor | None = None,
                          out_c: torch.Tensor | None = None, stream=None):
    """As qk_batch_run, plus the temporal autocorrelation C(t) of every item
    after every step; returns the device tensors (P, C), each [n_steps, items]."""
    items = qk_batch_items(b)
    if out is None:
        out = torch.empty((n_steps, items), dtype=torch.float64, device="cuda")
    if out_c is None:
        out_c = torch.empty((n_steps, items), dtype=torch.float64, device="cuda")
    for t in (out, out_c):
        if t.numel() < n_steps * items or t.dtype != torch.float64:
            raise ValueError("out and out_c must be float64 tensors of n_steps * items entries")
    _check(lib.qk_batch_run_autocorr(b.ptr, float(dt), int(n_steps), _graph_mode(use_graph), _dptr(out), _dptr(out_c),
                                     _stream(stream)), "qk_batch_run_autocorr")
    return out, out_c


def qk_grad_return_prob(k: Krylov, r0: int, T: float, n_steps: int, ckpt_every: int = 1, stream=None):
    """(F(T), dF/dh as a numpy array of length L) for the initial basis state r0;
    forward states are kept every ckpt_every steps."""
    L = k.H.L
    F = C.c_double()
    g = np.zeros(L)
    _check(lib.qk_grad_return_prob(k.ptr, int(r0), float(T), int(n_steps), int(ckpt_every), C.byref(F),
                                   g.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)), "qk_grad_return_prob")
    return F.value, g


def qk_return_prob(b: Basis, psi: torch.Tensor, r0: int = -1, psi0: torch.Tensor | None = None,
                   batch: int = 1, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """|<psi0|psi>|^2 per batch item into a device float64 tensor (asynchronous)."""
    if out is None:
        out = torch.empty(batch, dtype=torch.float64, device=psi.device)
    p0 = None if psi0 is None else _dptr(psi0)
    if psi0 is not None and psi0.dtype != psi.dtype:
        raise ValueError("psi0 and psi dtypes differ")
    _check(lib.qk_return_prob(b.ptr, int(r0), p0, _dptr(psi), dtype_code(psi), batch, _dptr(out),
                              _stream(stream)), "qk_return_prob")
    return out


def qk_return_prob_noalloc(b: Basis, psi: torch.Tensor, out: torch.Tensor, r0: int = -1,
                           psi0: torch.Tensor | None = None, batch: int = 1, stream=None) -> torch.Tensor:
    """qk_return_prob without any device allocation: the caller supplies `out`
    (float64, `batch` entries); the overlap's partial sums use the library's
    fixed per-GPU scratch array, so calls overlapping on one GPU race."""
    p0 = None if psi0 is None else _dptr(psi0)
    if psi0 is not None and psi0.dtype != psi.dtype:
        raise ValueError("psi0 and psi dtypes differ")
    _check(lib.qk_return_prob_noalloc(b.ptr, int(r0), p0, _dptr(psi), dtype_code(psi), batch, _dptr(out),
                                      _stream(stream)), "qk_return_prob_noalloc")
    return out


__all__ = [n for n in dir() if n.startswith("qk_")] + ["QkError", "Basis", "Ham", "Krylov", "Batch", "use_torch_allocator"]
