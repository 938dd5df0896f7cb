#!/usr/bin/env python3
"""Krylov time-evolution benchmark on one MI355X.

Workload: spin-1/2 XXZ ring L=28 in the Sz=0 sector (D = 40,116,600; the
strong-scaling system of the paper's Sec. 5), J = Delta = 1, quasiperiodic
fields h_i = 1.5 cos(2 pi beta i + phi) with beta the inverse golden ratio and
phi from numpy's default_rng(0), Neel initial state, Krylov dimension m = 30,
dt = 0.1.  A step is one Krylov step psi <- exp(-i dt H) psi (m Lanczos
iterations, the projected exponential, the combination) followed by the
survival probability.  Inputs are synthetic and resident in HBM before the
timed region starts.

Forms: plain complex128 (the headline `value`), complex64 storage, and a
batch of 8 phases in complex64 ([D][8] layout); `adaptive` runs the same
complex128 chain from the Neel state to t = 100 with error-controlled steps
(tolerance 1e-7 per unit time), the evolution the paper times in Sec. 5, and
reports its step count and wall time; `mixed` times the batched workload of
64 phases of the L = 20 ring plus single rings of L = 16, 18, 20, 22 (h = 2,
complex64, one hipGraph replay per step, and in the default launch shape the
graph of plain launches against the persistent step kernel); `large` times Krylov steps of the
L = 30 ring (m = 20, dt = 0.05, complex128 and complex64).  Every rate is the
median of --repeats timed runs of exactly --steps steps.  Also reported: standalone
y = H x throughput (algorithmic bytes 2 s D per call), a device-copy ceiling,
the roofline of the dominant kernel from HIP events recorded on the step's
stream, and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Krylov steps/sec + achieved HBM GB/s of H·v at L=28 Sz=0, plain FP64 vs batched/FP32"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_lanczos_h_L28.json")
# sources of the blocked H-pass kernel; stored counter bytes are used only
# while these files are unchanged
KERNEL_SRCS = [os.path.join(ROOT, "paper_1704_02770_amd", "csrc", f)
               for f in ("qk_blocked.hip", "qk_blocked_bodies.h", "qk_blocked.h", "qk_device.h")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=28)
    ap.add_argument("--m", type=int, default=30)
    ap.add_argument("--dt", type=float, default=0.1)
    ap.add_argument("--h", type=float, default=1.5)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--forms", default="fp64,fp32,batched,adaptive,mixed,large")
    ap.add_argument("--repeats", type=int, default=5, help="timed runs of --steps steps per form (median reported)")
    ap.add_argument("--mixed-steps", type=int, default=50, help="steps of the mixed batched workload per timed run")
    ap.add_argument("--large-steps", type=int, default=5, help="steps of the L = 30 form per timed run")
    ap.add_argument("--adaptive-t", type=float, default=100.0)
    ap.add_argument("--adaptive-tol", type=float, default=1e-7)
    ap.add_argument("--hv-reps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes instead of running the library's autotuner per form")
    ap.add_argument("--no-aux", action="store_true", help="skip the set-up, CSR and overlap timings")
    ap.add_argument("--csr-L", type=int, default=22, help="chain length of the CSR-versus-matrix-free H x timing")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--cpu-table", action="store_true",
                    help="time the CPU oracle at several sizes on this host (no GPU) and print one JSON line")
    args = ap.parse_args()
    problems = []
    if args.steps < 1 or args.warmup < 0 or args.hv_reps < 1 or args.repeats < 1:
        problems.append("--steps, --repeats and --hv-reps must be >= 1 and --warmup >= 0")
    if args.L < 4 or args.L > 32 or args.L % 2:
        problems.append("--L must be even, 4 <= L <= 32 (the Sz = 0 sector)")
    if args.m < 1 or args.m > 64 or not math.isfinite(args.dt) or args.dt <= 0:
        problems.append("--m must be in [1, 64] and --dt positive")
    if args.batch < 2 or args.batch > 64 or args.batch & (args.batch - 1):
        problems.append("--batch must be a power of two in [2, 64]")
    if problems:
        ap.error("; ".join(problems))
    return args


def source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def run_form(qk, torch, b, fields, m, dt, dtype, steps, warmup, r0, repeats, pbc=True, tune=True):
    """Times `steps` Krylov steps (+ survival probability) after `warmup`:
    one run with HIP events around every kernel (per-kernel times), then
    `repeats` runs without events, each bracketed by device synchronisation;
    the rate is the median of the latter.  With `tune` the library's
    autotuner picks the workspace's launch shape and block decomposition
    first (outside the timed runs)."""
    D = qk.qk_basis_dim(b)
    B = fields.shape[0]
    H = qk.qk_ham_create(b, 1.0, 1.0, pbc, fields)
    k = qk.qk_krylov_create(H, m, dtype)
    shape = qk.qk_krylov_autotune(k, dt) if tune else qk.qk_krylov_get_shape(k)
    psi = torch.zeros((D, B) if B > 1 else D, dtype=dtype, device="cuda")
    psi[r0] = 1.0
    P = torch.empty((steps + warmup, B), dtype=torch.float64, device="cuda")
    for s in range(warmup):
        qk.qk_krylov_expm_step(k, psi, dt)
        qk.qk_return_prob(b, psi, r0=r0, batch=B, out=P[s])
    torch.cuda.synchronize()
    # HIP events bracket every kernel launch on the same stream
    qk.qk_krylov_profile(k, True)
    torch.cuda.synchronize()
    for s in range(steps):
        qk.qk_krylov_expm_step(k, psi, dt)
        qk.qk_return_prob(b, psi, r0=r0, batch=B, out=P[warmup + s])
    torch.cuda.synchronize()
    prof = qk.qk_krylov_profile_read(k)
    qk.qk_krylov_profile(k, False)
    secs = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            qk.qk_krylov_expm_step(k, psi, dt)
            qk.qk_return_prob(b, psi, r0=r0, batch=B, out=P[warmup + s])
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
    info = qk.qk_krylov_expm_step(k, psi, dt, info=True)
    norm = torch.linalg.vector_norm(psi.reshape(D, B).to(torch.complex128), dim=0).cpu().tolist()
    out = dict(sec=statistics.median(secs), sec_all=secs, prof=prof, shape=shape, m_used=[i["m_used"] for i in info],
               err_est=max(i["err_est"] for i in info), P_last=P[warmup + steps - 1].cpu().tolist(),
               norm_drift=max(abs(x - 1.0) for x in norm))
    del k, H, psi
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def run_mixed(qk, torch, steps, warmup, repeats, m=30, dt=0.1, h=2.0, tune=True):
    """The batched workload: 64 phases of the L = 20 ring and single rings of
    L = 16, 18, 20, 22 (h = 2, Neel state, complex64 vectors, FP64 Lanczos
    coefficients), one hipGraph replay per step for all of them; also the
    64-phase workspace's kernels timed alone with HIP events (eager steps)."""
    from workloads import BETA_GOLDEN, phases
    spec = [(20, 64, 0), (16, 1, 1), (18, 1, 2), (20, 1, 3), (22, 1, 4)]
    hold, ks, psis, r0s = [], [], [], []
    for L, Bn, seed in spec:
        b = qk.qk_basis_build(L, L // 2)
        f = qk.qk_fields_quasiperiodic(L, h, BETA_GOLDEN, phases(Bn, seed))
        H = qk.qk_ham_create(b, 1.0, 1.0, True, f)
        k = qk.qk_krylov_create(H, m, torch.complex64)
        if tune:
            qk.qk_krylov_autotune(k, dt)
        D = qk.qk_basis_dim(b)
        r0 = int(qk.qk_basis_rank(b, [sum(1 << i for i in range(0, L, 2))])[0])
        psi = torch.zeros((D, Bn) if Bn > 1 else D, dtype=torch.complex64, device="cuda")
        psi[r0] = 1.0
        hold.append((b, H))
        ks.append(k)
        psis.append(psi)
        r0s.append(r0)
    bt = qk.qk_batch_create(ks, psis, r0s)
    items = qk.qk_batch_items(bt)
    out = torch.empty((steps, items), dtype=torch.float64, device="cuda")
    if warmup:
        qk.qk_batch_run(bt, dt, warmup, use_graph=True)
    secs = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qk.qk_batch_run(bt, dt, steps, use_graph=True, out=out)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
    sec = statistics.median(secs)
    # the same members in the default launch shape, one hipGraph of plain
    # launches per step against one persistent kernel per step (the
    # persistent step takes 256-thread row-streaming blocks)
    for k in ks:
        qk.qk_krylov_set_shape(k)
    default = {}
    for mode in (1, 2):
        qk.qk_batch_run(bt, dt, max(warmup, 1), use_graph=mode)
        ms = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            qk.qk_batch_run(bt, dt, steps, use_graph=mode, out=out)
            torch.cuda.synchronize()
            ms.append(time.perf_counter() - t0)
        default[mode] = statistics.median(ms)
    # kernels of the 64-phase L = 20 workspace alone (eager steps with events)
    k64, psi64 = ks[0], psis[0]
    qk.qk_krylov_profile(k64, True)
    for _ in range(steps):
        qk.qk_krylov_expm_step(k64, psi64, dt)
    torch.cuda.synchronize()
    prof = qk.qk_krylov_profile_read(k64)
    qk.qk_krylov_profile(k64, False)
    D20 = qk.qk_basis_dim(hold[0][0])
    res = dict(items=items, steps=steps, sec=sec, sec_all=secs, phase_steps_per_s=items * steps / sec,
               steps_per_s=steps / sec, prof64=prof, D20=D20, sec_graph_default=default[1],
               sec_persistent=default[2])
    bt.close()
    del ks, psis, hold
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def run_large(qk, torch, args, L=30, m=20, dt=0.5, h=2.0):
    """Krylov steps of the L = 30 ring (D = 155,117,520; h = 2, Neel state,
    m = 20, dt = 0.5) in complex128 and in complex64 storage, the Krylov basis
    resident in HBM."""
    from workloads import BETA_GOLDEN, phases
    b = qk.qk_basis_build(L, L // 2)
    D = qk.qk_basis_dim(b)
    f = qk.qk_fields_quasiperiodic(L, h, BETA_GOLDEN, phases(1, 0))
    r0 = int(qk.qk_basis_rank(b, [sum(1 << i for i in range(0, L, 2))])[0])
    out = dict(workload=f"XXZ ring L={L} Sz=0 (D={D}), J=Delta=1, h={h} quasiperiodic, Neel state, m={m}, dt={dt}")
    for name, dtype, s in (("fp64", torch.complex128, 16), ("fp32", torch.complex64, 8)):
        log("large", name)
        r = run_form(qk, torch, b, f, m, dt, dtype, args.large_steps, 1, r0, args.repeats, tune=not args.no_tune)
        out[name] = dict(steps_per_s=round(args.large_steps / r["sec"], 3),
                         ms_per_step=round(1e3 * r["sec"] / args.large_steps, 2),
                         ms_per_step_runs=[round(1e3 * x / args.large_steps, 2) for x in r["sec_all"]],
                         roofline=hpass_roofline(r["prof"], m, D, 1, s, None),
                         m_used=r["m_used"], err_est=r["err_est"], norm_drift=r["norm_drift"], P_last=r["P_last"])
    b.close()
    torch.cuda.empty_cache()
    return out


def hpass_roofline(prof, m, D, B, s, traffic):
    """Roofline entry of the H-pass (the dominant kernel): algorithmic bytes
    per step are (3m - 1) s D B (iteration 0 reads u_0 and writes w; later
    iterations also read u_{j-1}), divided by the HIP-event time of its m
    launches."""
    ms_h, n_h = prof["lanczos_h"]
    bytes_launch = (3 * m - 1) * s * D * B / m
    achieved = bytes_launch * n_h / (ms_h / 1e3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(achieved / PEAK_HBM_GBS, 4), traffic=traffic,
                bytes_per_launch_avg=bytes_launch, ms_per_launch_avg=ms_h / max(n_h, 1))


def host_cpu():
    """Model name and usable thread count of the host."""
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def run_adaptive(qk, torch, b, fields, m, r0, t_end, tol):
    """Adaptive stepping with error control from the Neel state to t_end
    (complex128), timed; also the same interval in fixed steps of 0.1."""
    D = qk.qk_basis_dim(b)
    H = qk.qk_ham_create(b, 1.0, 1.0, True, fields)
    k = qk.qk_krylov_create(H, m, torch.complex128)
    psi = torch.zeros(D, dtype=torch.complex128, device="cuda")
    psi[r0] = 1.0
    qk.qk_krylov_evolve(k, psi, 0.1, tol, dt_init=0.1)   # warm-up
    psi.zero_()
    psi[r0] = 1.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = qk.qk_krylov_evolve(k, psi, t_end, tol, dt_init=0.1)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    P = abs(psi[r0].item()) ** 2
    del k, H, psi
    torch.cuda.empty_cache()
    return dict(t_end=t_end, tol=tol, m=m, sec=round(sec, 4), steps=info["steps"], dt_min=info["dt_min"],
                dt_max=info["dt_max"], err_est_sum=info["err_sum"], P_end=P,
                time_units_per_s=round(t_end / sec, 3))


def hv_throughput(qk, torch, b, fields, dtype, reps):
    D = qk.qk_basis_dim(b)
    H = qk.qk_ham_create(b, 1.0, 1.0, True, fields)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(D, dtype=dtype, device="cuda", generator=g)
    y = torch.empty_like(x)
    qk.qk_ham_apply(H, x, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        qk.qk_ham_apply(H, x, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    s = x.element_size()
    # copy ceiling on the same vector size
    y.copy_(x)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(reps):
        y.copy_(x)
    c1.record()
    torch.cuda.synchronize()
    cms = c0.elapsed_time(c1) / reps
    del H, x, y
    torch.cuda.empty_cache()
    return dict(ms=ms, GBps=2 * s * D / ms / 1e6, copy_GBps=2 * s * D / cms / 1e6)


def _apply_ms(qk, torch, H, D, dtype, reps):
    g = torch.Generator(device="cuda").manual_seed(1)
    x = torch.randn(D, dtype=dtype, device="cuda", generator=g)
    y = torch.empty_like(x)
    qk.qk_ham_apply(H, x, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        qk.qk_ham_apply(H, x, y)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def aux_timings(qk, torch, L, fields1, b, csr_L, h):
    """Outside the timed steps: building the sector basis and the blocked
    Hamiltonian tables at L (wall clock, both calls are synchronous); y = H x
    through the CSR variant against the matrix-free kernel at csr_L; the
    survival probability of a general (dense) initial state at L."""
    from workloads import BETA_GOLDEN, phases
    out = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b2 = qk.qk_basis_build(L, L // 2)
    torch.cuda.synchronize()
    out["basis_build_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    b2.close()
    t0 = time.perf_counter()
    H = qk.qk_ham_create(b, 1.0, 1.0, True, fields1)
    torch.cuda.synchronize()
    out["ham_create_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    H.close()
    bc = qk.qk_basis_build(csr_L, csr_L // 2)
    Dc = qk.qk_basis_dim(bc)
    fc = qk.qk_fields_quasiperiodic(csr_L, h, BETA_GOLDEN, phases(1, 0))
    t0 = time.perf_counter()
    Hc = qk.qk_ham_create(bc, 1.0, 1.0, True, fc, mode=qk.QK_CSR)
    torch.cuda.synchronize()
    csr_build = (time.perf_counter() - t0) * 1e3
    Hm = qk.qk_ham_create(bc, 1.0, 1.0, True, fc)
    ms_csr = _apply_ms(qk, torch, Hc, Dc, torch.complex128, 50)
    ms_mf = _apply_ms(qk, torch, Hm, Dc, torch.complex128, 50)
    out["csr_vs_matfree"] = dict(L=csr_L, D=Dc, csr_build_ms=round(csr_build, 2), csr_hx_ms=round(ms_csr, 4),
                                 matfree_hx_ms=round(ms_mf, 4),
                                 csr_hx_GBps_algorithmic=round(32 * Dc / ms_csr / 1e6, 1))
    Hc.close()
    Hm.close()
    bc.close()
    D = qk.qk_basis_dim(b)
    g = torch.Generator(device="cuda").manual_seed(2)
    psi0 = torch.randn(D, dtype=torch.complex128, device="cuda", generator=g)
    psi = torch.randn(D, dtype=torch.complex128, device="cuda", generator=g)
    P = torch.empty(1, dtype=torch.float64, device="cuda")
    qk.qk_return_prob(b, psi, psi0=psi0, out=P)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        qk.qk_return_prob(b, psi, psi0=psi0, out=P)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    out["return_prob_general_state"] = dict(ms=round(ms, 4), GBps_algorithmic=round(32 * D / ms / 1e6, 1))
    del psi0, psi, P
    torch.cuda.empty_cache()
    # adjoint gradient dF/dh_i: the gradient workload (L = 20, T = 5 in 50
    # steps, m = 30) and five steps of the L chain; the handles and the call's
    # temporaries (checkpoints, the kept Krylov bases) come from torch's
    # caching allocator, and a first identical call fills its cache, so the
    # timed call measures the steady state of repeated gradient calls
    qk.use_torch_allocator()
    for Lg, T, n in ((20, 5.0, 50), (L, 0.5, 5)):
        bg = qk.qk_basis_build(Lg, Lg // 2)
        fg = qk.qk_fields_quasiperiodic(Lg, 1.5, BETA_GOLDEN, phases(1, 0))
        Hg = qk.qk_ham_create(bg, 1.0, 1.0, True, fg)
        kg = qk.qk_krylov_create(Hg, 30, torch.complex128)
        rg = int(qk.qk_basis_rank(bg, [sum(1 << i for i in range(0, Lg, 2))])[0])
        qk.qk_grad_return_prob(kg, rg, T, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F, dF = qk.qk_grad_return_prob(kg, rg, T, n)
        sec = time.perf_counter() - t0
        # the forward step of the same workspace (launch shape as created)
        psi = torch.zeros(qk.qk_basis_dim(bg), dtype=torch.complex128, device="cuda")
        psi[rg] = 1.0
        qk.qk_krylov_expm_step(kg, psi, T / n)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(3):
            qk.qk_krylov_expm_step(kg, psi, T / n)
        torch.cuda.synchronize()
        fwd = (time.perf_counter() - t1) / 3
        del psi
        out[f"gradient_L{Lg}"] = dict(T=T, steps=n, m=30, seconds=round(sec, 4), ms_per_step=round(1e3 * sec / n, 3),
                                       forward_ms_per_step=round(1e3 * fwd, 3),
                                       forward_steps_per_gradient_step=round(sec / n / fwd, 3),
                                       F=round(F, 12), max_abs_dFdh=round(float(max(abs(dF))), 9))
        kg.close()
        Hg.close()
        bg.close()
        torch.cuda.empty_cache()
    qk.qk_set_allocator()
    return out


def cpu_baseline(L, m, fields, pbc, target_s):
    """The oracle's Krylov step (Arnoldi with modified Gram-Schmidt, scipy CSR
    matvec) timed on the host on a bounded sample of the same L=28 workload:
    the CSR matvec on a seeded sample of rows (scaled to all D rows) and the
    oracle's vector operations on full-length vectors."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import basis as OB
    from oracle import hamiltonian as OH

    N = L // 2
    with threadpool_limits(limits=1):
        t_b0 = time.perf_counter()
        basis = OB.sector_states(L, N)
        t_basis = time.perf_counter() - t_b0
        D = len(basis)
        rng = np.random.default_rng(0)
        R = 20000
        Hs = OH.build_csr(L, N, pbc, 1.0, 1.0, fields, rows=np.sort(rng.choice(D, R, replace=False)))
        x = (rng.standard_normal(D) + 1j * rng.standard_normal(D)).astype(np.complex128)
        Hc = Hs.astype(np.complex128)
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 0.35 * target_s:
            Hc @ x
            reps += 1
        t_rows = (time.perf_counter() - t0) / reps
        t_hv = t_rows * D / R
        y = x.copy()
        def timeit(fn, n=2):
            fn()
            a = time.perf_counter()
            for _ in range(n):
                fn()
            return (time.perf_counter() - a) / n
        t_dot = timeit(lambda: np.vdot(x, y))
        t_axpy = timeit(lambda: np.subtract(y, 0.5 * x, out=y))
        t_norm = timeit(lambda: np.linalg.norm(y))
    # one oracle step: m matvecs; at iteration j, j+1 (vdot + axpy) pairs, a
    # norm and a scaling; the final combination V @ c costs about m axpys
    t_step = m * t_hv + sum((j + 1) * (t_dot + t_axpy) for j in range(m)) + m * (t_norm + t_axpy) + m * t_axpy
    return dict(value=1.0 / t_step, unit="steps/s", cores=1, kind="oracle",
                sample=(f"oracle Krylov step at L={L} (D={D}), m={m}: scipy CSR matvec of the oracle's H "
                        f"timed on {R} seeded rows and scaled by D/{R} ({t_hv:.2f} s per full H*x); numpy "
                        f"vdot/axpy/norm timed on full-length complex128 vectors; one host thread; "
                        f"basis build {t_basis:.1f} s not counted"),
                t_hv_s=t_hv, t_vec_s=dict(dot=t_dot, axpy=t_axpy, norm=t_norm))


def cpu_table(h):
    """The oracle timed on this host at the sizes of the workloads: dense
    eigendecomposition (L = 12, 14 on one thread and on all cores; L = 16 on
    all cores), the CSR H*x of the oracle's H (L = 20, 24 in full; L = 28 on
    a row sample), expm_multiply propagation of the L = 16 workload to t = 10,
    and the equivalent Krylov-step rate at L = 20/24/28 (m = 30)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import basis as OB
    from oracle import exact as OX
    from oracle import hamiltonian as OH
    from oracle import midsize as OM
    from oracle import model as OMo
    from workloads import BETA_GOLDEN, phases

    cores = os.cpu_count() or 1
    phi = float(phases(1, 0)[0])
    out = dict(cores_available=cores, dense_eigh_s={}, csr_hx_s={}, krylov_steps_per_s={})
    for L, threads in ((12, 1), (12, cores), (14, 1), (14, cores), (16, cores)):
        f = OMo.fields(L, h, BETA_GOLDEN, phi)
        Hd = OH.build_dense(L, L // 2, True, 1.0, 1.0, f)
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            OX.eig(Hd)
            out["dense_eigh_s"][f"L{L}_threads{threads}"] = round(time.perf_counter() - t0, 3)
        log("dense", L, threads, out["dense_eigh_s"][f"L{L}_threads{threads}"])
    with threadpool_limits(limits=1):
        for L in (20, 24):
            f = OMo.fields(L, h, BETA_GOLDEN, phi)
            t0 = time.perf_counter()
            Hc = OH.build_csr(L, L // 2, True, 1.0, 1.0, f).astype(np.complex128)
            t_build = time.perf_counter() - t0
            x = np.random.default_rng(0).standard_normal(Hc.shape[0]).astype(np.complex128)
            Hc @ x
            t0 = time.perf_counter()
            for _ in range(3):
                Hc @ x
            t_hv = (time.perf_counter() - t0) / 3
            out["csr_hx_s"][f"L{L}"] = dict(build=round(t_build, 3), hx=round(t_hv, 4), D=int(Hc.shape[0]))
            log("csr", L, t_build, t_hv)
        f16 = OMo.fields(16, h, BETA_GOLDEN, phi)
        H16 = OH.build_csr(16, 8, True, 1.0, 1.0, f16)
        r0 = int(OB.lookup(OB.sector_states(16, 8), [OMo.neel_state(16)])[0])
        t0 = time.perf_counter()
        OM.survival_probability(H16, r0, np.linspace(0.0, 10.0, 101))
        out["expm_multiply_L16_t10_s"] = round(time.perf_counter() - t0, 3)
    # a Krylov step as the oracle runs it: m matvecs; at iteration j, j + 1
    # (vdot + axpy) pairs of the Gram-Schmidt, a norm and a scaling; the
    # combination about m more axpys (vector passes timed on one thread)
    m = 30
    with threadpool_limits(limits=1):
        for L in (20, 24):
            c = out["csr_hx_s"][f"L{L}"]
            x = np.ones(c["D"], dtype=np.complex128)
            y = x.copy()
            t0 = time.perf_counter()
            for _ in range(5):
                np.vdot(x, y)
                np.subtract(y, 0.5 * x, out=y)
            t_pair = (time.perf_counter() - t0) / 5
            t_step = m * c["hx"] + sum(j + 1 for j in range(m)) * t_pair + 2 * m * t_pair
            out["krylov_steps_per_s"][f"L{L}"] = round(1.0 / t_step, 3)
    b28 = cpu_baseline(28, 30, OMo.fields(28, h, BETA_GOLDEN, phi), True, 15.0)
    out["csr_hx_s"]["L28_sampled"] = dict(hx=round(b28["t_hv_s"], 3), D=40116600)
    out["krylov_steps_per_s"]["L28"] = round(b28["value"], 5)
    return out


def main():
    args = parse()
    if args.cpu_table:
        print(json.dumps(dict(kind="oracle", host_cpu_table=cpu_table(args.h))), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent phases or a row-sharded L would each need their own process).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1704_02770_amd as qk
    from workloads import BETA_GOLDEN, phases

    L, N, m, dt = args.L, args.L // 2, args.m, args.dt
    log(f"L={L} m={m} dt={dt} steps={args.steps} warmup={args.warmup}")
    phi = phases(1, 0)
    fields1 = qk.qk_fields_quasiperiodic(L, args.h, BETA_GOLDEN, phi)
    b = qk.qk_basis_build(L, N)
    D = qk.qk_basis_dim(b)
    neel = sum(1 << i for i in range(0, L, 2))
    r0 = int(qk.qk_basis_rank(b, [neel])[0])
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]

    res = {}
    hv = {}
    adaptive = mixed = large = None
    log("H*x throughput")
    hv["fp64"] = hv_throughput(qk, torch, b, fields1, torch.complex128, args.hv_reps)
    hv["fp32"] = hv_throughput(qk, torch, b, fields1, torch.complex64, args.hv_reps)
    aux = None
    if not args.no_aux:
        log("set-up, CSR and overlap timings")
        aux = aux_timings(qk, torch, L, fields1, b, args.csr_L, args.h)
    for f in forms:
        log("form", f)
        if f == "fp64":
            res[f] = run_form(qk, torch, b, fields1, m, dt, torch.complex128, args.steps, args.warmup, r0, args.repeats,
                              tune=not args.no_tune)
        elif f == "fp32":
            res[f] = run_form(qk, torch, b, fields1, m, dt, torch.complex64, args.steps, args.warmup, r0, args.repeats,
                              tune=not args.no_tune)
        elif f == "batched":
            fb = qk.qk_fields_quasiperiodic(L, args.h, BETA_GOLDEN, phases(args.batch, 0))
            res[f] = run_form(qk, torch, b, fb, m, dt, torch.complex64, args.steps, args.warmup, r0, args.repeats,
                              tune=not args.no_tune)
        elif f == "adaptive":
            adaptive = run_adaptive(qk, torch, b, fields1, m, r0, args.adaptive_t, args.adaptive_tol)
        elif f == "mixed":
            mixed = run_mixed(qk, torch, args.mixed_steps, 2, args.repeats, tune=not args.no_tune)
        elif f == "large":
            large = run_large(qk, torch, args)
        else:
            raise SystemExit(f"unknown form {f}")

    if not res:
        raise SystemExit("at least one of the forms fp64, fp32, batched is needed")
    head_form = "fp64" if "fp64" in res else next(iter(res))
    head = res[head_form]
    steps = args.steps
    value = steps / head["sec"]
    B_head = args.batch if head_form == "batched" else 1
    traffic = None
    if head_form == "fp64" and os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_source_sha256") == source_sha() and tr.get("m") == m and tr.get("L") == L:
            traffic = tr.get("bytes_per_launch")
    roof = hpass_roofline(head["prof"], m, D, B_head, 16 if head_form == "fp64" else 8, traffic)
    roof["kernel"] = ("H-pass of the Lanczos iteration, w = a H u_j - b u_{j-1} with its dot products "
                      + {"fp64": "(k_blk<double,11,true>, the blocked matrix-free kernel used for L >= 18)",
                         "fp32": "(k_blk<float,11,true>, complex64 storage)",
                         "batched": f"(k_blkb<float,true>, {args.batch} phases in complex64)"}[head_form])
    roof["form"] = head_form

    def form_summary(r, B, s, m_, D_, steps_):
        sec = r["sec"]
        kernels = {kname: dict(ms_per_launch=ms / max(n, 1), launches=n) for kname, (ms, n) in r["prof"].items()}
        step_bytes = (7 * m_ - 1) * s * D_ * B
        return dict(steps_per_s=round(steps_ / sec, 3), phase_steps_per_s=round(B * steps_ / sec, 3),
                    ms_per_step=round(1e3 * sec / steps_, 3),
                    ms_per_step_runs=[round(1e3 * x / steps_, 3) for x in r["sec_all"]],
                    step_algorithmic_GBps=round(step_bytes * steps_ / sec / 1e9, 1), kernels=kernels,
                    roofline=hpass_roofline(r["prof"], m_, D_, B, s, None), launch_shape=r["shape"],
                    m_used=r["m_used"], err_est=r["err_est"], norm_drift=r["norm_drift"], P_last=r["P_last"])

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * head["sec"] / steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"XXZ ring L={L} Sz=0 (D={D}), J=Delta=1, h=1.5 quasiperiodic, phi=default_rng(0), "
                               f"Neel initial state, Lanczos m={m}, dt={dt}, complex128",
                   "L": L, "D": D, "m": m, "dt": dt, "h": args.h, "pbc": True, "phi": float(phi[0]),
                   "parallelism": "single GPU"},
        "roofline": roof,
        "hv": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in hv.items()},
        "hv_fp64_GBps": round(hv["fp64"]["GBps"], 1),
        "hv_fp32_GBps": round(hv["fp32"]["GBps"], 1),
        "forms": {},
    }
    for f, r in res.items():
        B = args.batch if f == "batched" else 1
        s = 16 if f == "fp64" else 8
        out["forms"][f] = form_summary(r, B, s, m, D, steps)
    if adaptive is not None:
        out["adaptive"] = adaptive
    if mixed is not None:
        out["mixed"] = dict(
            workload="64 phases of the L=20 ring (D=184756) + rings L=16,18,20,22 (one phase each), h=2, "
                     "J=Delta=1, Neel state, m=30, dt=0.1, complex64 vectors, FP64 Lanczos coefficients; "
                     "all members advanced by one hipGraph replay per step",
            items=mixed["items"], steps=mixed["steps"], phase_steps_per_s=round(mixed["phase_steps_per_s"], 1),
            steps_per_s=round(mixed["steps_per_s"], 2), ms_per_step=round(1e3 * mixed["sec"] / mixed["steps"], 3),
            ms_per_step_runs=[round(1e3 * x / mixed["steps"], 3) for x in mixed["sec_all"]],
            default_shape=dict(
                graph_ms_per_step=round(1e3 * mixed["sec_graph_default"] / mixed["steps"], 3),
                persistent_ms_per_step=round(1e3 * mixed["sec_persistent"] / mixed["steps"], 3),
                persistent_phase_steps_per_s=round(mixed["items"] * mixed["steps"] / mixed["sec_persistent"], 1),
                note="the members in the default launch shape: one hipGraph of plain launches per step "
                     "against one persistent kernel per step (qk_batch_run use_graph=2; same bits)"),
            roofline_L20x64=hpass_roofline(mixed["prof64"], 30, mixed["D20"], 64, 8, None),
            kernels_L20x64={kname: dict(ms_per_launch=ms_ / max(n_, 1), launches=n_)
                            for kname, (ms_, n_) in mixed["prof64"].items()})
    if large is not None:
        out["large"] = large
    if aux is not None:
        out["aux"] = aux
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cb = cpu_baseline(L, m, fields1[0], True, args.cpu_seconds)
        out["cpu_baseline"] = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in cb.items()
                               if k in ("value", "unit", "cores", "kind", "sample")}
        model, avail = host_cpu()
        out["cpu_baseline"]["host_cpu"] = model
        out["cpu_baseline"]["host_threads_available"] = avail
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
