"""The C ABI used from plain C (tests/c_abi/lid_cavity.c: include/lbm.h and
liblbm.so only, the library's own device memory, the null stream), run as a
child process; its macroscopic fields against the FP64 oracle, and its
batch (a pressure-driven duct and a lid cavity, one with a step budget)
bit-identical to single runs, checked by the program itself."""
import os
import subprocess

import numpy as np
import pytest

from oracle import runner as R

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_plain_c_lid_cavity_matches_oracle(tmp_path):
    exe = os.path.join(HERE, "c_abi", "lid_cavity")
    assert os.path.exists(exe), "build it with __graft_entry__.build()"
    out = tmp_path / "fields.bin"
    run = subprocess.run([exe, str(out)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    print(run.stdout.strip())
    assert "bit-identical to single runs" in run.stdout
    assert "duct t=17, cavity t=12" in run.stdout
    nx, ny, nz, N = 12, 10, 8, 12 * 10 * 8
    data = np.fromfile(out, dtype=np.float64)
    assert data.size == 4 * N
    p, u = data[:N].reshape(nz, ny, nx), data[N:].reshape(3, nz, ny, nx)
    s = [1.0, 1.19, 1.0, 1.2, 1.0, 1.2, 1.0, 1.2, 1.6, 1.6, 1.6, 1.6, 1.6, 0.98]
    pr = R.problem(14, nx, ny, nz, s, faces=("wall",) * 6, wall_u={"+z": (0.06, 0.0, 0.0)},
                   F0=(1e-5, 0.0, -2e-5))
    f = R.run(pr, R.init_eq(pr, 0, p0=0.002, u0=(0.01, -0.005, 0.0)), 0, 25)
    pr_, ur = R.macros(pr, f, 25)
    assert np.max(np.abs(u - ur)) <= 1e-14
    assert np.max(np.abs(p - pr_)) <= 1e-14
    mass = float(run.stdout.split("mass=")[1].split()[0])
    assert abs(mass - float(np.sum(f))) <= 1e-12 * abs(float(np.sum(f)))
