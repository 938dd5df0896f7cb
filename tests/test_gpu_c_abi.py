"""The C ABI used from plain C (tests/c_abi/qk_demo.c: include/qk.h, the HIP
runtime and nothing else), against the oracle's dense propagation: the
survival probability of the Neel state of an L=12 ring, ten Krylov steps."""
import os
import subprocess

import numpy as np
import pytest

from gpu_util import say
from oracle import basis as OB
from oracle import exact as OX
from oracle import hamiltonian as OH
from oracle import model as OM
from workloads import BETA_GOLDEN

pytestmark = pytest.mark.gpu

DEMO = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "qk_demo")


def test_c_program_matches_dense_propagation():
    assert os.path.exists(DEMO), "tests/c_abi/qk_demo is built by paper_1704_02770_amd/build.py"
    L, h, phi, m, dt, n = 12, 1.5, 0.4, 30, 0.1, 10
    say("C demo", L)
    r = subprocess.run([DEMO, str(L), str(h), str(phi), str(m), str(dt), str(n)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    rows = np.array([[float(x) for x in ln.split()] for ln in r.stdout.strip().splitlines()])
    assert rows.shape == (n, 2)
    H = OH.build_dense(L, L // 2, True, 1.0, 1.0, OM.fields(L, h, BETA_GOLDEN, phi))
    r0 = int(OB.lookup(OB.sector_states(L, L // 2), [OM.neel_state(L)])[0])
    P = OX.survival_probability(H, r0, rows[:, 0])
    assert np.max(np.abs(rows[:, 1] - P)) < 1e-10
    # a bad argument is reported with the library's message and a non-zero exit
    bad = subprocess.run([DEMO, "12", "1.5", "0.4", "65", "0.1", "1"], capture_output=True, text=True, timeout=60)
    assert bad.returncode == 1 and "qk_krylov_create failed with status 1" in bad.stderr, bad.stderr
