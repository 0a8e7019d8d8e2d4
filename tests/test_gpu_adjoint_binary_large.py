"""The binary adjoint on a lattice whose arrays exceed 4 GiB.

Below 4 GiB per array of 19 directions the local adjoint kernel addresses
each array from one base with 32-bit byte offsets; above (here 320 x 320 x
280 = 28.7 M sites, 4.36 GB per array) it takes one 64-bit base per
direction.  The state and the seeds are a 10^3 pattern repeated over the
large lattice, so the adjoint must repeat it too:

- one adjoint step (BGK, TRT, MRT; state direct or pulled from the
  post-collision fields): every value of lambda_f^n and lambda_g^n equals,
  bit for bit, the 10^3 lattice's value at the same place in the pattern
  (the per-site arithmetic is the same, only the addressing differs), and
  the parameter sums equal the 10^3 lattice's times the number of copies;
- a 2-step rollout and its backward (the segment sweep, BGK) with a loss
  summed over sites: dL/dphi0 repeats the 10^3 pattern within 1e-12.
"""

import numpy as np
import pytest
import torch

from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu

T = 10                          # the repeated pattern, T^3
REP = (28, 32, 32)              # copies along z, y, x: 280 x 320 x 320
BIG = tuple(T * r for r in REP)
COPIES = REP[0] * REP[1] * REP[2]
TRT = dict(tau_minus=1.3)
MRT = dict(tau_minus=1.3, tau_bulk=1.4, tau_ghost_even=0.85, tau_ghost_odd=1.15)


def _tile(a):
    """Repeat a (..., T, T, T) array over the large lattice, on the GPU."""
    t = torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    lead = t.dim() - 3
    return t.repeat(*([1] * lead), *REP).contiguous()


def _lattice(lbgpu, shape, coll):
    nz, ny, nx = shape
    kw = {}
    if coll == "trt":
        kw = dict(collision=lbgpu.LB_TRT, **TRT)
    elif coll == "mrt":
        kw = dict(collision=lbgpu.LB_MRT, **MRT)
    return lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, tau_f=0.9, kappa=0.05, mobility=0.3, **kw)


def _small_state(lbgpu, coll):
    """A binary state off equilibrium on the T^3 pattern, after one step, and
    its post-collision fields (the pulled form of the same state)."""
    rho, _u, phi = inputs.spinodal_quench(T, T, T, seed=51, phi_max=0.3)
    _r, u = inputs.single_fluid_random(T, T, T, seed=52, u_max=0.02)
    lat = _lattice(lbgpu, (T, T, T), coll)
    lat.init_equilibrium(rho, u, phi)
    lat.step(1)
    f, g = (a.clone() for a in lat.get_state())
    lat.collide()
    pf, pg = (a.clone() for a in lat.get_state())      # post-collision, before propagation
    lat.close()
    return f, g, pf, pg


def _adjoint_step(lbgpu, lat, f, g, lf1, lg1, pending, ng):
    lf, lg = torch.empty_like(lf1), torch.empty_like(lg1)
    grads = torch.zeros(ng, dtype=torch.float64, device="cuda")
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_adjoint_step_binary(lat.ctx, f, g, lf1, lg1, lf, lg, grads, pending=pending)
    torch.cuda.synchronize()
    return lf, lg, grads


@pytest.mark.parametrize("pending", [False, True])
@pytest.mark.parametrize("coll", ["bgk", "trt", "mrt"])
def test_large_adjoint_step_repeats_the_pattern(lbgpu, coll, pending):
    print("case binary adjoint step %s %s on %s (arrays above 4 GiB)" % (coll, "pending" if pending else "direct",
                                                                          "x".join(map(str, BIG))), flush=True)
    ng = {"bgk": 3, "trt": 4, "mrt": 7}[coll]
    f, g, pf, pg = _small_state(lbgpu, coll)
    given = (pf, pg) if pending else (f, g)
    rng = np.random.default_rng(53)
    lf1, lg1 = (torch.as_tensor(rng.standard_normal((19, T, T, T)), device="cuda") for _ in range(2))
    small = _lattice(lbgpu, (T, T, T), coll)
    s_lf, s_lg, s_gr = _adjoint_step(lbgpu, small, given[0], given[1], lf1, lg1, pending, ng)
    small.close()
    big = _lattice(lbgpu, BIG, coll)
    assert 19 * BIG[0] * BIG[1] * BIG[2] * 8 > 1 << 32
    b_lf, b_lg, b_gr = _adjoint_step(lbgpu, big, _tile(given[0].cpu().numpy()), _tile(given[1].cpu().numpy()),
                                     _tile(lf1.cpu().numpy()), _tile(lg1.cpu().numpy()), pending, ng)
    big.close()
    for name, b, s in (("lambda_f", b_lf, s_lf), ("lambda_g", b_lg, s_lg)):
        want = s.repeat(1, *REP)
        assert torch.equal(b, want), name
    s_gr, b_gr = s_gr.cpu().numpy() * COPIES, b_gr.cpu().numpy()
    np.testing.assert_allclose(b_gr, s_gr, rtol=1e-11, atol=0)


def test_large_rollout_gradient_repeats_the_pattern(lbgpu):
    """Forward steps, recording and the segment sweep of the backward on the
    large lattice, against the same rollout on the pattern."""
    from paper_1405_6162_amd.adjoint import rollout_binary, velocity_table
    print("case binary rollout 2 steps + backward on %s (arrays above 4 GiB)" % "x".join(map(str, BIG)),
          flush=True)
    rho, _u, phi = inputs.spinodal_quench(T, T, T, seed=54, phi_max=0.3)
    _r, u = inputs.single_fluid_random(T, T, T, seed=55, u_max=0.02)

    def loss(f, g):
        c = velocity_table(f.device, f.dtype)
        r = f.sum(0)
        v = torch.stack([(c[:, a].reshape(-1, 1, 1, 1) * f).sum(0) for a in range(3)]) / r
        p = g.sum(0)
        return ((v * v).sum(0) + p * p).sum()

    def grad(shape, fields):
        lat = _lattice(lbgpu, shape, "bgk")
        r0, u0, p0 = fields
        p0 = p0.clone().requires_grad_(True)
        L = loss(*rollout_binary(r0, u0, p0, lat, 2, 2))
        L.backward()
        torch.cuda.synchronize()
        lat.close()
        return p0.grad

    small = grad((T, T, T), tuple(torch.as_tensor(a, device="cuda") for a in (rho, u, phi)))
    big = grad(BIG, (_tile(rho), _tile(u), _tile(phi)))
    want = small.repeat(*REP)
    err = float((big - want).abs().max() / want.abs().max())
    print("large rollout dL/dphi0 against the pattern: %.2e" % err, flush=True)
    assert err <= 1e-12
