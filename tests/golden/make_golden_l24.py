"""Writes tests/golden/l24_log_times.txt: the survival probability of the
Neel state on the L=24 chain (Sz=0, D = 2,704,156; J = Delta = 1, fields
h cos(2 pi beta i + phi), phi = default_rng(0).uniform(0, 2 pi)) for
h in {0, 1, 3}, open and periodic bonds, at all 200 log-spaced output times
10^-2 .. 10^2.

Every value comes from the oracle alone: its sorted basis, its CSR Hamiltonian
and scipy's expm_multiply (oracle.midsize), step by step between output times.
The six cases run in parallel processes, one host thread each (one to two
hours of wall time on an 8-core host).
Run from the repository root:  python tests/golden/make_golden_l24.py
"""
import os

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import multiprocessing as mp   # noqa: E402
import sys                      # noqa: E402
import time                     # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import basis as OB          # noqa: E402
from oracle import hamiltonian as OH    # noqa: E402
from oracle import midsize as OMS       # noqa: E402
from oracle import model as OM          # noqa: E402
from workloads import BETA_GOLDEN, log_times, phases   # noqa: E402

L = 24
CASES = [(pbc, h) for pbc in (False, True) for h in (0.0, 1.0, 3.0)]


def _case(args):
    pbc, h = args
    t0 = time.time()
    times = log_times()
    phi = float(phases(1, 0)[0])
    st = OB.sector_states(L, L // 2)
    r0 = int(OB.lookup(st, [OM.neel_state(L)])[0])
    hf = OM.fields(L, h, BETA_GOLDEN, phi)
    H = OH.build_csr(L, L // 2, pbc, 1.0, 1.0, hf)
    P = OMS.survival_probability(H, r0, times)
    print(f"pbc={pbc} h={h}: {time.time() - t0:.1f} s", flush=True)
    return int(pbc), h, P


def main():
    times = log_times()
    phi = float(phases(1, 0)[0])
    with mp.Pool(len(CASES)) as pool:
        rows = pool.map(_case, CASES)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "l24_log_times.txt")
    with open(out, "w") as f:
        f.write("# Survival probability of the Neel state, L=24 Sz=0, J=Delta=1, beta=(sqrt5-1)/2,\n")
        f.write(f"# phi={phi!r} (default_rng(0)), written by tests/golden/make_golden_l24.py from the oracle\n")
        f.write("# (Sec. 4's F(t); exact propagation by expm_multiply).  Line 1 of data: times;\n")
        f.write("# then one line per case: pbc h P(t_1) ... P(t_n)\n")
        f.write(" ".join(repr(float(t)) for t in times) + "\n")
        for pbc, h, P in rows:
            f.write(f"{pbc} {h!r} " + " ".join(repr(float(p)) for p in P) + "\n")


if __name__ == "__main__":
    main()
