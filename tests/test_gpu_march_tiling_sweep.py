"""The single-pass march in each of its launch shapes.

The march picks its tile per storage and lattice (64 x 8; in FP32 and FP16
128 x 4 where nx mod 128 is 0 or above 64) and its chunks per lattice: depth
64 where that gives more than 512 blocks (two per CU), else as many chunks
as fill 512 blocks (at least nz/64, at most nz/16, rounded up).  Where the
block count is a multiple of 8 (blocks remapped to XCDs in contiguous runs)
the chunks split nz evenly, else all but the last take the full depth.  The
lattices below were chosen so that every combination runs, each ragged in x
and y:

| lattice          | FP64: tile, blocks, chunks    | FP32/FP16: tile, blocks, chunks |
|------------------|-------------------------------|---------------------------------|
| 195 x 252 x 17   | 64 x 8, 256, even 8/9         | 128 x 4, 252, 9 + 8             |
| 282 x 205 x 17   | 64 x 8, 260, 9 + 8            | 64 x 8, 260, 9 + 8              |
| 211 x 255 x 17   | 64 x 8, 256, even 8/9         | 128 x 4, 256, even 8/9          |
| 257 x 319 x 34   | 64 x 8, 400, even 17          | 64 x 8, 400, even 17            |
| 68 x 266 x 164   | 64 x 8, 476, 6 x 24 + 20      | 128 x 4, 469, 6 x 24 + 20       |
| 262 x 322 x 35   | 64 x 8, 410, 18 + 17          | 64 x 8, 410, 18 + 17            |
| 262 x 318 x 66   | 64 x 8, 400, even 33          | 64 x 8, 400, even 33            |
| 326 x 289 x 65   | 64 x 8, 444, 33 + 32          | 128 x 4, 438, 33 + 32           |
| 65 x 1025 x 66   | 64 x 8, 516, 64 + 2           | 128 x 4, 514, 64 + 2            |
| 65 x 1037 x 66   | 64 x 8, 520, even 33          | 128 x 4, 520, even 33           |

In every storage the march and the two-pass step (phi pass + fused
collide, whose launch shape is fixed) give the same bits after three steps;
both are compared with the oracle elsewhere.
"""

import pytest
import torch

from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = [(195, 252, 17), (282, 205, 17), (211, 255, 17), (257, 319, 34), (68, 266, 164), (262, 322, 35),
          (262, 318, 66), (326, 289, 65), (65, 1025, 66), (65, 1037, 66)]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("nx,ny,nz", SHAPES)
def test_march_launch_shapes_equal_two_pass(lbgpu, storage, nx, ny, nz):
    print("case binary %dx%dx%d %s x3: march vs two-pass" % (nx, ny, nz, storage), flush=True)
    code = {"f64": lbgpu.LB_F64, "f32": lbgpu.LB_F32, "f16": lbgpu.LB_F16}[storage]
    rho, _u, phi = inputs.spinodal_quench(nx, ny, nz, seed=71, phi_max=0.3)
    _r, u = inputs.single_fluid_random(nx, ny, nz, seed=72, u_max=0.01)
    states = {}
    for path, step in (("march", lbgpu.LB_STEP_MARCH), ("two_pass", lbgpu.LB_STEP_TWO_PASS)):
        lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, storage=code, phi0=float(phi.mean()),
                            binary_step=step)
        lat.init_equilibrium(rho, u, phi)
        lat.step(3)
        states[path] = lat.get_state()
        lat.close()
    for a, b in zip(states["march"], states["two_pass"]):
        assert torch.equal(a, b)
