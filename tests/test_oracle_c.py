"""The two CPU references against each other: the C ABI implemented in plain
C on host pointers (oracle/lb_oracle.c) and the numpy reference
(oracle/lb_oracle.py, pinned on its own by tests/test_oracle_pins.py).  They
share no code; agreement to rounding pins the C reference."""

import numpy as np
import pytest

from oracle import c_backend as C
from oracle import lb_oracle as O
from paper_1405_6162_amd import inputs


@pytest.fixture(scope="module", autouse=True)
def built():
    from oracle import build
    build.build()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("nx,ny,nz", [(4, 4, 4), (5, 6, 7), (1, 1, 3), (7, 3, 2)])
def test_single_fluid(nx, ny, nz):
    rho, u = inputs.single_fluid_random(nx, ny, nz, seed=1)
    lat = C.CLattice(nx, ny, nz, tau_f=0.8)
    lat.init_equilibrium(rho, u)
    ref = O.init_single(rho, u)
    assert rel(lat.state()[0], ref) < 1e-15
    lat.collide()
    ref = O.collide_single(ref, 0.8)
    assert rel(lat.state()[0], ref) < 1e-14
    lat.propagate()
    ref = O.propagate(ref)
    np.testing.assert_array_equal(lat.state()[0], ref)          # a permutation: exact
    lat.step(6)
    ref = O.step_single(ref, 0.8, 6)
    assert rel(lat.state()[0], ref) < 1e-13
    r, uu, _ = lat.moments()
    uref, rref = O.velocity(ref)
    assert rel(r, rref) < 1e-13 and rel(uu, uref) < 1e-12
    np.testing.assert_allclose(lat.sums(), O.conserved_sums(ref), rtol=1e-13, atol=1e-13)
    lat.close()


@pytest.mark.parametrize("nx,ny,nz", [(4, 4, 4), (6, 5, 7), (3, 1, 4)])
def test_binary_fluid(nx, ny, nz):
    prm = O.Params(tau_f=0.9, kappa=0.05, mobility=0.3)
    rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=2, phi_max=0.3)
    _r, u = inputs.single_fluid_random(nx, ny, nz, seed=3, u_max=0.01)
    lat = C.CLattice(nx, ny, nz, model=1, tau_f=prm.tau_f, kappa=prm.kappa, mobility=prm.mobility)
    lat.init_equilibrium(rho, u, phi)
    rf, rg = O.init_binary(rho, u, phi, prm)
    f, g = lat.state()
    assert rel(f, rf) < 1e-14 and rel(g, rg) < 1e-14
    lat.step(5)
    rf, rg = O.step_binary(rf, rg, prm, 5)
    f, g = lat.state()
    assert rel(f, rf) < 1e-13 and rel(g, rg) < 1e-13
    _r2, _u2, ph = lat.moments()
    assert rel(ph, O.order_parameter(rg)) < 1e-13
    lat.close()


def test_set_state_then_collide_off_equilibrium():
    nx, ny, nz = 5, 4, 3
    prm = O.Params()
    rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=4, phi_max=0.3)
    f, g = O.step_binary(*O.init_binary(rho, u, phi, prm), prm, 1)
    lat = C.CLattice(nx, ny, nz, model=1)
    lat.set_state(f, g)
    lat.collide()
    rf, rg = O.collide_binary(f, g, prm)
    cf, cg = lat.state()
    assert rel(cf, rf) < 1e-14 and rel(cg, rg) < 1e-14


def test_refusals():
    with pytest.raises(ValueError):
        C.CLattice(4, 4, 4, storage=1)                 # reduced precision: not in this reference
    with pytest.raises(ValueError):
        C.CLattice(4, 4, 4, tau_f=0.5)
    with pytest.raises(ValueError):
        C.CLattice(0, 4, 4)


@pytest.mark.parametrize("model", [0, 1])
def test_thread_count_does_not_change_a_bit(model):
    """The site loops are shared among OpenMP threads; every value is the same
    expression on any thread and the conserved sums are serial, so 1, 3 and
    8 threads give identical states, moments and sums."""
    nx, ny, nz = 9, 7, 11
    out = []
    for threads in (1, 3, 8):
        C.set_threads(threads)
        lat = C.CLattice(nx, ny, nz, model=model, tau_f=0.9)
        if model:
            lat.init_equilibrium(*inputs.spinodal_quench(nx, ny, nz, seed=3, phi_max=0.2))
        else:
            lat.init_equilibrium(*inputs.single_fluid_random(nx, ny, nz, seed=3))
        lat.step(4)
        f, g = lat.state()
        rho, u, phi = lat.moments()
        out.append((f, g, rho, u, phi, lat.sums()))
        lat.close()
    C.set_threads(0)
    for other in out[1:]:
        for a, b in zip(out[0], other):
            if a is not None:
                assert np.array_equal(a, b)
