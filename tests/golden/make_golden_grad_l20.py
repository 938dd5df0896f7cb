"""Writes tests/golden/grad_l20_richardson.txt: the derivative of the survival
probability F(T) = |<Neel| exp(-iHT) |Neel>|^2 with respect to every on-site
field h_i of the L=20 ring (Sz=0, D = 184,756; J = Delta = 1,
h_i = 1.5 cos(2 pi beta i + phi), phi = default_rng(0).uniform(0, 2 pi), T = 5).

F is evaluated by the oracle alone (its CSR Hamiltonian and scipy's
expm_multiply, oracle.midsize) and differentiated by the oracle's central
differences (oracle.gradient.dF_dh_finite_difference) at two step sizes,
eps = 1e-3 and 5e-4, combined by one Richardson step
    R = (4 D(eps/2) - D(eps)) / 3,
which cancels the eps^2 term of the central difference.  The remaining
truncation is of order eps^4 T^5 / 120 (about 3e-11 here) and the rounding
of F contributes about 1e-15 / eps.  Both D(eps) and D(eps/2) are stored, so
the test can state the spread.  The 20 fields run in parallel processes.
Run from the repository root:  python tests/golden/make_golden_grad_l20.py [workers]
"""
import os

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import multiprocessing as mp   # noqa: E402
import sys                      # noqa: E402
import time                     # noqa: E402

import numpy as np              # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import basis as OB          # noqa: E402
from oracle import gradient as OG       # noqa: E402
from oracle import hamiltonian as OH    # noqa: E402
from oracle import midsize as OMS       # noqa: E402
from oracle import model as OM          # noqa: E402
from workloads import BETA_GOLDEN, WORKLOADS   # noqa: E402

W = WORKLOADS["xxz_L20_grad"]
EPS = (1e-3, 5e-4)


def _setup():
    L = W.L
    st = OB.sector_states(L, L // 2)
    r0 = int(OB.lookup(st, [OM.neel_state(L)])[0])
    hf = OM.fields(L, W.h, BETA_GOLDEN, float(W.phis()[0]))
    return L, r0, hf


def _F(hh):
    L, r0, _ = _setup()
    H = OH.build_csr(L, L // 2, W.pbc, W.jxy, W.jz, hh)
    return float(OMS.survival_probability(H, r0, [W.t_end])[0])


def _one_field(i):
    """Central differences of F along field i at both step sizes."""
    t0 = time.time()
    L, r0, hf = _setup()
    out = [float(OG.dF_dh_finite_difference(L, L // 2, W.pbc, W.jxy, W.jz, hf, r0, W.t_end, eps=eps,
                                            propagate=_F, indices=[i])[0]) for eps in EPS]
    print(f"field {i}: {time.time() - t0:.1f} s", flush=True)
    return out


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    L, r0, hf = _setup()
    with mp.Pool(workers) as pool:
        F0 = pool.apply_async(_F, (hf,))
        rows = pool.map(_one_field, range(L), chunksize=1)
        F0 = F0.get()
    D1 = np.array([r[0] for r in rows], dtype=np.float64)
    D2 = np.array([r[1] for r in rows], dtype=np.float64)
    R = (4.0 * D2 - D1) / 3.0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_l20_richardson.txt")
    with open(out, "w") as f:
        f.write("# dF(T)/dh_i of the Neel survival probability, L=20 ring, J=Delta=1, h=1.5, T=5,\n")
        f.write(f"# phi={float(W.phis()[0])!r} (default_rng(0)); written by tests/golden/make_golden_grad_l20.py\n")
        f.write("# from the oracle (expm_multiply F, central differences at eps=1e-3 and 5e-4, one Richardson step).\n")
        f.write(f"# F(T) = {float(F0)!r}\n")
        f.write("# columns: i  R_i  D_i(1e-3)  D_i(5e-4)\n")
        f.write(f"F {float(F0)!r}\n")
        for i in range(L):
            f.write(f"{i} {float(R[i])!r} {float(D1[i])!r} {float(D2[i])!r}\n")


if __name__ == "__main__":
    main()
