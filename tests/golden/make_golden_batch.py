"""Writes tests/golden/batch_mixed_t50.txt: the survival probability of the
Neel state for every member of the mixed batched workload, at t = 1, 2, ..., 50:

* 64 phases phi = default_rng(0).uniform(0, 2 pi, 64) of the L=20 ring
  (Sz=0, D = 184,756);
* single rings of L = 16, 18, 20, 22 with phi = default_rng(s).uniform(0, 2 pi)
  for s = 1, 2, 3, 4;

all with J = Delta = 1, fields h cos(2 pi beta i + phi), h = 2 (Sec. 4's
quasiperiodic chains, evolved from the Neel state).

Every value comes from the oracle alone: its sorted basis, its CSR Hamiltonian
and scipy's expm_multiply (oracle.midsize) from one output time to the next.
The members run in parallel processes, one host thread each.
Run from the repository root:  python tests/golden/make_golden_batch.py [workers]
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
from oracle import hamiltonian as OH    # noqa: E402
from oracle import midsize as OMS       # noqa: E402
from oracle import model as OM          # noqa: E402
from workloads import BETA_GOLDEN, phases   # noqa: E402

H_FIELD = 2.0
TIMES = np.arange(1, 51, dtype=np.float64)


def members():
    """(L, phi) of every member in batch order."""
    out = [(20, float(p)) for p in phases(64, 0)]
    for s, L in enumerate((16, 18, 20, 22), start=1):
        out.append((L, float(phases(1, s)[0])))
    return out


def _member(args):
    L, phi = args
    t0 = time.time()
    st = OB.sector_states(L, L // 2)
    r0 = int(OB.lookup(st, [OM.neel_state(L)])[0])
    H = OH.build_csr(L, L // 2, True, 1.0, 1.0, OM.fields(L, H_FIELD, BETA_GOLDEN, phi))
    P = OMS.survival_probability(H, r0, TIMES)
    print(f"L={L} phi={phi:.6f}: {time.time() - t0:.1f} s", flush=True)
    return P


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    mem = members()
    with mp.Pool(workers) as pool:
        rows = pool.map(_member, mem, chunksize=1)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_mixed_t50.txt")
    with open(out, "w") as f:
        f.write("# Survival probability of the Neel state on periodic chains, J=Delta=1, h=2, beta=(sqrt5-1)/2:\n")
        f.write("# 64 phases of L=20 (default_rng(0)), then L=16/18/20/22 with phases from default_rng(1..4).\n")
        f.write("# Written by tests/golden/make_golden_batch.py from the oracle (Sec. 4's F(t); exact\n")
        f.write("# propagation by expm_multiply).  Line 1 of data: times; then one line per member: L phi P(t)...\n")
        f.write(" ".join(repr(float(t)) for t in TIMES) + "\n")
        for (L, phi), P in zip(mem, rows):
            f.write(f"{L} {phi!r} " + " ".join(repr(float(p)) for p in P) + "\n")


if __name__ == "__main__":
    main()
