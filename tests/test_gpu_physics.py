"""Physics of the binary fluid at sizes the oracle cannot run, checked
against laws that hold at any size: a droplet of radius R at rest obeys the
Laplace law, a pressure jump Delta[rho c_s^2 + p0(phi)] = 2 sigma / R with
p0 = A/2 phi^2 + 3B/4 phi^4 the bulk part of the chemical stress, and the
Gibbs-Thomson shift of both bulk phases, mu = sigma / R on either side
(Delta phi = 2 between the bulk values).  sigma = sqrt(-8 kappa A^3 / 9 B^2)
is the surface tension of the continuum phi^4 interface; on the lattice,
with an interface only xi = sqrt(-2 kappa / A) = 1.13 sites wide, the
effective tension is 11% lower, and 5% lower at xi = 2.26, so that
constant is checked loosely and the 1/R law tightly."""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

A, B, KAPPA = -0.0625, 0.0625, 0.04
SIGMA = np.sqrt(-8 * KAPPA * A ** 3 / (9 * B ** 2))
XI = np.sqrt(-2 * KAPPA / A)


def p0(p):
    return 0.5 * A * p ** 2 + 0.75 * B * p ** 4


def _droplet(lbgpu, L, R, steps):
    """Pressure jump times R, the droplet radius, and mu inside / outside
    after `steps` steps from a tanh droplet whose bulk values start at the
    Gibbs-Thomson shift."""
    d = dict(dtype=torch.float64, device="cuda")
    z, y, x = torch.meshgrid(*(torch.arange(L, **d) for _ in range(3)), indexing="ij")
    r = torch.sqrt((x - L / 2 + 0.5) ** 2 + (y - L / 2 + 0.5) ** 2 + (z - L / 2 + 0.5) ** 2)
    shift = SIGMA / (R * (A + 3 * B))
    phi = (shift - torch.tanh((r - R) / XI)).contiguous()
    lat = lbgpu.Lattice(L, L, L, model=lbgpu.LB_BINARY, A=A, B=B, kappa=KAPPA)
    lat.init_equilibrium(torch.ones_like(phi), torch.zeros((3,) + phi.shape, **d), phi)
    lat.step(steps)
    rho, _u, ph = lat.moments()
    inner, outer = r < R / 2, r > (R + L / 2) / 2 + 2
    pin, pout = float(ph[inner].mean()), float(ph[outer].mean())
    rt = (3 * float(((ph - pout) / (pin - pout)).sum()) / (4 * np.pi)) ** (1 / 3)
    dp = float(rho[inner].mean() - rho[outer].mean()) / 3 + p0(pin) - p0(pout)
    mu = lambda p: A * p + B * p ** 3
    stats = lat.field_stats().cpu().numpy()
    lat.close()
    assert np.isfinite(stats).all()
    return dp * rt, rt, mu(pin), mu(pout)


def test_laplace_law_and_gibbs_thomson(lbgpu):
    rows = []
    for L, R in ((64, 12.0), (64, 16.0), (96, 24.0)):
        print("case droplet L=%d R=%.0f" % (L, R), flush=True)
        dpR, rt, mu_in, mu_out = _droplet(lbgpu, L, R, 4000)
        print("  Delta p R / 2 sigma = %.4f, R = %.3f, mu R / sigma = %.3f (in), %.3f (out)"
              % (dpR / (2 * SIGMA), rt, mu_in * rt / SIGMA, mu_out * rt / SIGMA), flush=True)
        rows.append((dpR, rt, mu_in, mu_out))
    dpR = np.array([r[0] for r in rows])
    # the Laplace law: Delta p proportional to 1/R
    assert dpR.max() / dpR.min() - 1 < 0.015
    # the effective tension of the 1.13-site interface
    assert 0.85 < dpR.mean() / (2 * SIGMA) < 1.0
    for _dp, rt, mu_in, mu_out in rows:
        # equal chemical potentials across the interface, both near sigma / R
        assert abs(mu_in - mu_out) < 0.1 * SIGMA / rt
        assert abs(0.5 * (mu_in + mu_out) * rt / SIGMA - 1) < 0.1
