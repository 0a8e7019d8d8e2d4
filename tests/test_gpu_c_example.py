"""The C ABI from C: paper_1405_6162_amd/csrc/lb_example.c drives a binary
spinodal quench through include/lb.h with HIP runtime memory and a stream of
its own (no Python in the process); its final moments must equal the
oracle's."""

import os
import subprocess

import numpy as np
import pytest

from oracle import lb_oracle as O

pytestmark = pytest.mark.gpu

EXAMPLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1405_6162_amd", "_lib",
                       "lb_example")


def test_c_example_matches_oracle(tmp_path):
    assert os.path.exists(EXAMPLE), "lb_example not built (python -m paper_1405_6162_amd.build)"
    nx, ny, nz, steps = 24, 20, 18, 30
    out = tmp_path / "moments.bin"
    print("case c example", nx, ny, nz, steps, flush=True)
    res = subprocess.run([EXAMPLE, str(nx), str(ny), str(nz), str(steps), str(out)], capture_output=True,
                         text=True, timeout=120)
    print(res.stdout, res.stderr, flush=True)
    assert res.returncode == 0
    n = nx * ny * nz
    got = np.fromfile(out, dtype=np.float64)
    assert got.size == 5 * n
    rho, u, phi = got[:n].reshape(nz, ny, nx), got[n:4 * n].reshape(3, nz, ny, nx), got[4 * n:].reshape(nz, ny, nx)
    z = np.arange(nz).reshape(-1, 1, 1)
    y = np.arange(ny).reshape(1, -1, 1)
    x = np.arange(nx).reshape(1, 1, -1)
    phi0 = 0.05 * np.sin(2 * np.pi * (x / nx + 2.0 * y / ny)) * np.cos(2 * np.pi * 3.0 * z / nz)
    phi0 = np.broadcast_to(phi0, (nz, ny, nx)).copy()
    prm = O.Params()
    f, g = O.step_binary(*O.init_binary(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)), phi0, prm), prm, steps)
    uref, rref = O.velocity(f)
    rel = lambda a, b: np.abs(a - b).max() / np.abs(b).max()
    assert rel(rho, rref) < 1e-12
    assert rel(u, uref) < 1e-10          # u starts at zero: relative to a field of order 1e-6
    assert rel(phi, O.order_parameter(g)) < 1e-12
