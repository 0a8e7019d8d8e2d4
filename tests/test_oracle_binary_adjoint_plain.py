"""The binary-fluid adjoint against its definition.

`adjoint_step_binary` (and `adjoint_init_binary`) are hand-derived closed
forms: weighted sums of the post-collision adjoints, sensitivities to phi,
grad phi and lap phi, and the transposed stencils.  The GPU kernels follow
the same derivation, so agreement between the two says nothing about the
derivation itself.  Here the closed form is checked on EVERY component, and
on every parameter gradient, against the definition of the reverse step,
lambda^n = J^T lambda^{n+1} with J the Jacobian of one whole step built
column by column from the plain forward (`adjoint_step_binary_plain`), for
BGK, TRT and MRT relaxation of f.  The definition itself is pinned first by
central differences of the real forward, which use no complex arithmetic.
"""

import functools

import numpy as np
import pytest

from oracle import lb_oracle as O
from paper_1405_6162_amd import inputs

NX, NY, NZ = 5, 4, 3
TRT_TAUS = (0.9, 1.3, 0.9, 0.9, 1.3)           # even groups at tau+, odd (flux, odd ghosts) at tau-
MRT_TAUS = (0.9, 1.3, 1.4, 0.85, 1.15)
TAUS = {"bgk": None, "trt": TRT_TAUS, "mrt": MRT_TAUS}


def _prm(coll):
    t = TAUS[coll]
    return O.Params(tau_f=0.9 if t is None else t[0], kappa=0.05, mobility=0.3)


def _state(coll, nx=NX, ny=NY, nz=NZ):
    """A binary state off equilibrium: non-uniform rho, random u, phi up to
    0.3, one step of the collision under test."""
    rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=11, phi_max=0.3)
    _r, u = inputs.single_fluid_random(nx, ny, nz, seed=12, u_max=0.02)
    rho = rho + 0.01 * np.cos(2 * np.pi * np.arange(nx) / nx)
    prm = _prm(coll)
    f, g = O.init_binary(rho, u, phi, prm)
    t = TAUS[coll]
    return O.step_binary(f, g, prm, 1) if t is None else O.step_binary_mrt(f, g, prm, t, 1)


def _adjoints(shape, seed=13):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape), rng.standard_normal(shape)


@functools.lru_cache(maxsize=None)
def _plain(coll):
    f, g = _state(coll)
    lf1, lg1 = _adjoints(f.shape)
    return O.adjoint_step_binary_plain(f, g, lf1, lg1, _prm(coll), TAUS[coll])


def test_step_jacobian_matches_central_differences():
    """J v against [step(x + eps v) - step(x - eps v)] / (2 eps) in real
    arithmetic for random directions v (the truncation error is
    O(eps^2 |F'''|), far below the tolerance)."""
    nx, ny, nz = 3, 4, 3
    for coll in ("bgk", "mrt"):
        f, g = _state(coll, nx, ny, nz)
        prm, t = _prm(coll), TAUS[coll]
        J = O.binary_step_jacobian(f, g, prm, t)
        x = np.concatenate([f.ravel(), g.ravel()])
        half = x.size // 2
        rng = np.random.default_rng(14)
        eps = 1e-5
        for _ in range(3):
            v = rng.standard_normal(x.size)

            def F(y):
                a, b = (O.step_binary(y[:half].reshape(f.shape), y[half:].reshape(g.shape), prm, 1) if t is None
                        else O.step_binary_mrt(y[:half].reshape(f.shape), y[half:].reshape(g.shape), prm, t, 1))
                return np.concatenate([a.ravel(), b.ravel()])
            fd = (F(x + eps * v) - F(x - eps * v)) / (2 * eps)
            jv = J @ v
            assert np.abs(jv - fd).max() <= 1e-7 * np.abs(jv).max(), coll


def test_step_jacobian_domain_of_dependence():
    """The step's domain of dependence: a value at s after the step came
    from s - c_i, whose collision read phi at its six neighbours, so every
    nonzero of J links sites at most one velocity (|c|_1 <= 2) plus one
    stencil hop apart: at most 2 per axis and 3 in all (periodic)."""
    nx, ny, nz = 5, 4, 3
    f, g = _state("bgk", nx, ny, nz)
    J = O.binary_step_jacobian(f, g, _prm("bgk"))
    n = nx * ny * nz
    coords = np.array([(s % nx, (s // nx) % ny, s // (nx * ny)) for s in range(n)])
    ext = np.array([nx, ny, nz])

    def dist(a, b):                   # periodic L-infinity distance per axis
        d = np.abs(coords[a] - coords[b])
        return np.minimum(d, ext - d)
    Js = np.abs(J).reshape(2, 19, n, 2, 19, n)
    for s_in in (0, 17, n - 1):
        out_sites = np.flatnonzero(Js[:, :, :, :, :, s_in].max(axis=(0, 1, 3, 4)) > 0)
        for s_out in out_sites:
            d = dist(s_out, s_in)
            # a value moves at most one hop per axis; phi's stencil adds one
            assert (d <= 2).all() and d.sum() <= 3, (s_in, s_out, d)


@pytest.mark.parametrize("coll", ["bgk", "trt", "mrt"])
def test_closed_form_adjoint_equals_definition(coll):
    """Every component of lf^n and lg^n, and every parameter gradient."""
    f, g = _state(coll)
    lf1, lg1 = _adjoints(f.shape)
    prm, t = _prm(coll), TAUS[coll]
    pf, pg, pgr = _plain(coll)
    cf, cg, cgr = O.adjoint_step_binary(f, g, lf1, lg1, prm, t)
    assert np.abs(cf - pf).max() <= 1e-12 * np.abs(pf).max()
    assert np.abs(cg - pg).max() <= 1e-12 * np.abs(pg).max()
    # the closed form returns d/d omega (omega = 1/tau) and tau_g = M / Gamma + 1/2
    want = {"kappa": cgr["kappa"], "mobility": -cgr["omega_g"] / prm.tau_g ** 2 / prm.gamma}
    if t is None:
        want["tau_f"] = -cgr["omega_f"] / prm.tau_f ** 2
    else:
        for name, tk in zip(O.MRT_RATES, t):
            want["tau_" + name] = -cgr["omega_" + name] / tk ** 2
    assert set(want) == set(pgr)
    for name, w in want.items():
        assert abs(w - pgr[name]) <= 1e-12 * max(abs(pgr[name]), 1e-3), name


def test_closed_form_init_adjoint_equals_definition():
    nx, ny, nz = 4, 3, 5
    prm = O.Params(kappa=0.03)
    rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=15, phi_max=0.3)
    _r, u = inputs.single_fluid_random(nx, ny, nz, seed=16, u_max=0.02)
    rho = rho + 0.01 * np.sin(2 * np.pi * np.arange(nx) / nx)
    lf0, lg0 = _adjoints((19, nz, ny, nx), seed=17)
    want = O.adjoint_init_binary_plain(rho, u, phi, lf0, lg0, prm)
    got = O.adjoint_init_binary(rho, u, phi, lf0, lg0, prm)
    for name, w, c in zip(("phi", "rho", "u"), want[:3], got[:3]):
        assert np.abs(c - w).max() <= 1e-12 * np.abs(w).max(), name
    assert abs(got[3] - want[3]) <= 1e-12 * abs(want[3])


def test_definition_detects_a_dropped_term():
    """The comparison has teeth: a closed form with the stencil transpose's
    Laplacian part dropped fails it."""
    f, g = _state("bgk")
    lf1, lg1 = _adjoints(f.shape)
    prm = _prm("bgk")
    pf, pg, _ = _plain("bgk")
    orig = O.stencil_transpose
    try:
        O.stencil_transpose = lambda a_phi, a_G, a_lap: orig(a_phi, a_G, 0.0 * a_lap)
        cf, cg, _ = O.adjoint_step_binary(f, g, lf1, lg1, prm)
    finally:
        O.stencil_transpose = orig
    assert np.abs(cg - pg).max() > 1e-6 * np.abs(pg).max()
