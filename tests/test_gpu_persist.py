"""GPU tests of the persistent batched step (qk_batch_run with use_graph = 2):
one kernel launch per step advances every workspace of a batch, records P and
advances C(t).  It runs the same kernel bodies on the same grids as the plain
launches, so its results must equal theirs bit for bit; through them it is
tied to the oracle (the mixed workload's oracle values are checked in
test_gpu_batch.py against the graph of plain launches, and here the persistent
step against that graph)."""
import numpy as np
import pytest
import torch

import paper_1704_02770_amd as qk
from gpu_util import neel_row, say, to_host
from oracle import exact as OX
from oracle import hamiltonian as OH
from oracle import model as OM
from workloads import BETA_GOLDEN, phases, random_complex

pytestmark = pytest.mark.gpu


def _ws(L, Bn, dtype, h=2.0, seed=0, m=30, reorth=0, mode=None):
    b = qk.qk_basis_build(L, L // 2)
    phi = phases(Bn, seed)
    hf = np.stack([OM.fields(L, h, BETA_GOLDEN, p) for p in phi])
    H = qk.qk_ham_create(b, 1.0, 1.0, True, hf) if mode is None else qk.qk_ham_create(b, 1.0, 1.0, True, hf, mode)
    k = qk.qk_krylov_create(H, m, dtype, reorth=reorth)
    D = qk.qk_basis_dim(b)
    r0 = neel_row(L)
    psi = torch.zeros((D, Bn) if Bn > 1 else D, dtype=dtype, device="cuda")
    psi[r0] = 1.0
    return dict(b=b, H=H, k=k, psi=psi, r0=r0, hf=hf, L=L, B=Bn, D=D)


def _random_states(D, Bn, seed, dtype):
    z = random_complex(D * Bn, seed).reshape(D, Bn) if Bn > 1 else random_complex(D, seed)
    z = z / np.linalg.norm(z, axis=0)
    return torch.from_numpy(np.ascontiguousarray(z)).to(device="cuda", dtype=dtype)


def _run_modes(make, steps, dt, modes=(0, 1, 2), autocorr=False, chunks=1):
    """P (and C) and the final vectors of the same batch run in each mode."""
    out = {}
    for mode in modes:
        ws, psis, r0s = make()
        bt = qk.qk_batch_create([w["k"] for w in ws], psis, r0s)
        say("batch mode", mode, "steps", steps, "in", chunks, "calls")
        Ps, Cs = [], []
        per = steps // chunks
        for c in range(chunks):
            n = per if c + 1 < chunks else steps - per * (chunks - 1)
            if autocorr:
                P, C = qk.qk_batch_run_autocorr(bt, dt, n, use_graph=mode)
                Cs.append(to_host(C).copy())
            else:
                P = qk.qk_batch_run(bt, dt, n, use_graph=mode)
            Ps.append(to_host(P).copy())
            # eager work of the program between calls
            assert np.isfinite(torch.randn(1000, device="cuda").sum().item())
        out[mode] = (np.concatenate(Ps), np.concatenate(Cs) if autocorr else None,
                     [to_host(p).copy() for p in psis])
        del bt
    return out


def _assert_same(out, modes=(0, 1, 2)):
    P0, C0, v0 = out[modes[0]]
    for mode in modes[1:]:
        P, C, v = out[mode]
        assert np.array_equal(P, P0), f"mode {mode}: max |dP| {np.max(np.abs(P - P0))}"
        if C0 is not None:
            assert np.array_equal(C, C0)
        for a, b in zip(v, v0):
            assert np.array_equal(a, b)


def test_persistent_small_batch_first():
    # two small workspaces (row form, one and four columns), three steps one
    # call at a time: the smallest persistent launches, bitwise against the
    # plain launches
    dtype = torch.complex128

    def make():
        ws = [_ws(10, 1, dtype, seed=81, m=12), _ws(12, 4, dtype, seed=82, m=12)]
        return ws, [w["psi"] for w in ws], [w["r0"] for w in ws]

    _assert_same(_run_modes(make, 3, 0.1, chunks=3))


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_persistent_mixed_lengths_bitwise(dtype):
    # the mixed workload's shape: 64 phases of L=20 (batched blocked H-pass
    # with partial-sum totals) and single chains L=16 (row form), 18, 20, 22
    # (one-phase blocked kernel with 9, 10, 11 low bits), 25 steps
    spec = [(20, 64), (16, 1), (18, 1), (20, 1), (22, 1)]

    def make():
        ws = [_ws(L, Bn, dtype, seed=i) for i, (L, Bn) in enumerate(spec)]
        return ws, [w["psi"] for w in ws], [w["r0"] for w in ws]

    out = _run_modes(make, 25, 0.1)
    _assert_same(out)
    assert out[2][0].shape == (25, 68)


def test_persistent_random_states_autocorr_reorth_vs_oracle():
    # basis-state and random initial states (overlap records), local
    # reorthogonalisation, a batch of 8 (totals passes) and a batch of 2 at
    # L = 18 (batched blocked kernel without totals), P and C(t) over three
    # calls; bitwise against the plain launches, and the small chains against
    # the oracle's exact P and its trapezoid average
    dtype, dt, steps = torch.complex128, 0.05, 60
    init = {}

    def make():
        wa = _ws(12, 8, dtype, h=1.5, seed=41, m=24, reorth=1)
        wb = _ws(10, 2, dtype, h=3.0, seed=42, m=24)
        wc = _ws(18, 2, dtype, h=2.0, seed=43, m=20)
        pb = _random_states(wb["D"], 2, 51, dtype)
        init["b"] = to_host(pb).copy()
        init["wa"], init["wb"] = wa, wb
        return [wa, wb, wc], [wa["psi"], pb, wc["psi"]], [wa["r0"], -1, wc["r0"]]

    out = _run_modes(make, steps, dt, autocorr=True, chunks=3)
    _assert_same(out)
    P, C, _ = out[2]
    t = dt * np.arange(0, steps + 1)
    cases = [(12, init["wa"]["hf"][i], None, i) for i in range(8)] + \
            [(10, init["wb"]["hf"][i], init["b"][:, i], 8 + i) for i in range(2)]
    for L, hf, p0, col in cases:
        Hd = OH.build_dense(L, L // 2, True, 1.0, 1.0, hf)
        if p0 is None:
            p0 = np.zeros(len(Hd), complex)
            p0[neel_row(L)] = 1.0
        Pt = np.array([OX.overlap_probability(p0, v) for v in OX.evolve(Hd, p0, t)])
        assert np.max(np.abs(P[:, col] - Pt[1:])) < 1e-10
        assert np.max(np.abs(C[:, col] - OX.autocorrelation(t, Pt)[1:])) < 1e-10


def test_persistent_row_form_and_csr():
    # Hamiltonians without block tables: matrix-free rows and CSR, one dtype
    dtype = torch.complex64

    def make():
        ws = [_ws(18, 1, dtype, seed=61, mode=qk.QK_MATFREE_ROWS), _ws(14, 4, dtype, seed=62, mode=qk.QK_CSR)]
        return ws, [w["psi"] for w in ws], [w["r0"] for w in ws]

    _assert_same(_run_modes(make, 12, 0.1))


def test_persistent_rejects_what_it_does_not_cover():
    w1 = _ws(12, 1, torch.complex128, seed=71)
    w2 = _ws(12, 1, torch.complex64, seed=72)
    w3 = _ws(12, 1, torch.complex128, seed=73, reorth=2)
    out = torch.full((2, 2), -7.0, dtype=torch.float64, device="cuda")
    for pair in ((w1, w2), (w1, w3)):
        bt = qk.qk_batch_create([w["k"] for w in pair], [w["psi"] for w in pair], [w["r0"] for w in pair])
        with pytest.raises(qk.QkError):
            qk.qk_batch_run(bt, 0.1, 2, use_graph=2, out=out)
    assert np.all(to_host(out) == -7.0)   # nothing was enqueued
    # after a refusal the same batch still runs in the other modes
    bt = qk.qk_batch_create([w1["k"], w3["k"]], [w1["psi"], w3["psi"]], [w1["r0"], w3["r0"]])
    with pytest.raises(qk.QkError):
        qk.qk_batch_run(bt, 0.1, 2, use_graph=2, out=out)
    P = to_host(qk.qk_batch_run(bt, 0.1, 2, use_graph=1))
    assert np.all(np.isfinite(P)) and P.shape == (2, 2)
    with pytest.raises(ValueError):
        qk.qk_batch_run(bt, 0.1, 2, use_graph=3)


def test_persistent_full_size_l28_bitwise():
    # an L = 28 complex64 workspace (321 MB vectors: non-temporal update and
    # combination, the 11-low-bit blocked H-pass on its full grid) batched
    # with an L = 16 chain, two steps, persistent against the graph of plain
    # launches
    dtype = torch.complex64

    def make():
        ws = [_ws(28, 1, dtype, h=1.5, seed=91, m=30), _ws(16, 1, dtype, seed=92, m=30)]
        return ws, [w["psi"] for w in ws], [w["r0"] for w in ws]

    out = _run_modes(make, 2, 0.1, modes=(1, 2))
    _assert_same(out, modes=(1, 2))
    torch.cuda.empty_cache()
