"""GPU (HIP, through the C ABI) against the FP64 CPU oracle, element by element.

Tolerance for FP64: 1e-12 relative, measured as max |gpu - oracle| divided by
max |oracle| of the same field (distributions, rho, u, phi separately).  The
two sides differ only in the order of rounding, so the observed gap is a few
1e-16; 1e-12 leaves room for the amplification of unstable binary dynamics
over 100 steps.
"""

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def relerr(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return float(np.abs(a - ref).max() / (scale if scale > 0 else 1.0))


def params_of(prm):
    return dict(tau_f=prm.tau_f, A=prm.A, B=prm.B, kappa=prm.kappa, mobility=prm.mobility,
                gamma=prm.gamma)


def single_case(nx, ny, nz, seed=0):
    rho, u = inputs.single_fluid_random(nx, ny, nz, seed=seed)
    return rho, u


def binary_case(nx, ny, nz, seed=0, phi_max=0.05, u_max=0.0):
    rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=seed, phi_max=phi_max)
    if u_max:
        _r, u = inputs.single_fluid_random(nx, ny, nz, seed=seed + 7, u_max=u_max)
    return rho, u, phi


def cpu(t):
    return t.detach().cpu().numpy() if t is not None else None


# Several tiles and ragged tails in x (64-wide tiles) and y (4-high tiles),
# and z extents below, at and above the single-pass kernel's chunks of 8
# (FP64) and 16 planes (37 = 16 + 16 + 5 = 4 x 8 + 5, 17 = 16 + 1 = 2 x 8 + 1).
SIZES = [(4, 4, 4), (16, 16, 16), (5, 6, 7), (67, 9, 5), (4, 8, 12), (1, 1, 3), (130, 3, 2),
         (5, 6, 37), (70, 5, 17),
         (1, 1, 1), (3, 1, 1), (1, 7, 1), (2, 2, 2), (64, 4, 16)]      # one site; single-extent axes; whole tiles


@pytest.mark.parametrize("nx,ny,nz", SIZES)
@pytest.mark.parametrize("nsteps", [1, 10])
def test_single_fluid_steps(lbgpu, nx, ny, nz, nsteps):
    print("case single", nx, ny, nz, nsteps, flush=True)
    tau = 0.8
    rho, u = single_case(nx, ny, nz, seed=1)
    lat = lbgpu.Lattice(nx, ny, nz, tau_f=tau)
    lat.init_equilibrium(rho, u)
    f0, _ = lat.get_state()
    ref0 = O.init_single(rho, u)
    assert relerr(cpu(f0), ref0) < TOL64
    lat.step(nsteps)
    f, _ = lat.get_state()
    r, uu, _ = lat.moments()
    ref = O.step_single(ref0, tau, nsteps)
    uref, rref = O.velocity(ref)
    assert relerr(cpu(f), ref) < TOL64
    assert relerr(cpu(r), rref) < TOL64
    assert relerr(cpu(uu), uref) < TOL64
    lat.close()


STEP_KERNELS = {"march": 1, "two_pass": 2}       # LB_STEP_MARCH, LB_STEP_TWO_PASS: both forced at every size


@pytest.mark.parametrize("path", sorted(STEP_KERNELS))
@pytest.mark.parametrize("nx,ny,nz", SIZES)
@pytest.mark.parametrize("nsteps", [1, 10])
def test_binary_fluid_steps(lbgpu, nx, ny, nz, nsteps, path):
    print("case binary", nx, ny, nz, nsteps, path, flush=True)
    prm = O.Params()
    rho, u, phi = binary_case(nx, ny, nz, seed=2, phi_max=0.3, u_max=0.01)
    lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, binary_step=STEP_KERNELS[path], **params_of(prm))
    lat.init_equilibrium(rho, u, phi)
    f0, g0 = lat.get_state()
    rf0, rg0 = O.init_binary(rho, u, phi, prm)
    assert relerr(cpu(f0), rf0) < TOL64
    assert relerr(cpu(g0), rg0) < TOL64
    lat.step(nsteps)
    f, g = lat.get_state()
    r, uu, ph = lat.moments()
    rf, rg = O.step_binary(rf0, rg0, prm, nsteps)
    uref, rref = O.velocity(rf)
    assert relerr(cpu(f), rf) < TOL64
    assert relerr(cpu(g), rg) < TOL64
    assert relerr(cpu(r), rref) < TOL64
    assert relerr(cpu(uu), uref) < TOL64
    assert relerr(cpu(ph), O.order_parameter(rg)) < TOL64
    lat.close()


def test_single_fluid_c1_config(lbgpu):
    """16^3, tau = 1, rho = 1 + 0.01 N(0,1), u ~ U(-0.01, 0.01), 10 steps, seed 0."""
    rho, u = inputs.single_fluid_random(16, 16, 16, seed=0)
    lat = lbgpu.Lattice(16, 16, 16, tau_f=1.0)
    lat.init_equilibrium(rho, u)
    lat.step(10)
    f, _ = lat.get_state()
    ref = O.step_single(O.init_single(rho, u), 1.0, 10)
    assert relerr(cpu(f), ref) < TOL64
    r, uu, _ = lat.moments()
    uref, rref = O.velocity(ref)
    assert relerr(cpu(uu), uref) < TOL64 and relerr(cpu(r), rref) < TOL64


@pytest.mark.parametrize("model", ["single", "binary"])
def test_collide_and_propagate_separately(lbgpu, model):
    """lb_collide / lb_propagate on every state representation against the
    oracle's separate phases, including collide-collide and
    propagate-propagate sequences."""
    nx, ny, nz = 7, 6, 5
    prm = O.Params(tau_f=0.9)
    if model == "single":
        rho, u = single_case(nx, ny, nz, seed=3)
        lat = lbgpu.Lattice(nx, ny, nz, tau_f=prm.tau_f)
        lat.init_equilibrium(rho, u)
        ref = [O.init_single(rho, u)]
        collide = lambda s: [O.collide_single(s[0], prm.tau_f)]
    else:
        rho, u, phi = binary_case(nx, ny, nz, seed=3, phi_max=0.4, u_max=0.02)
        lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, **params_of(prm))
        lat.init_equilibrium(rho, u, phi)
        ref = list(O.init_binary(rho, u, phi, prm))
        collide = lambda s: list(O.collide_binary(s[0], s[1], prm))
    propagate = lambda s: [O.propagate(a) for a in s]
    seq = ["c", "p", "s", "c", "c", "p", "p", "s", "p", "c", "s", "s"]
    for op in seq:
        if op == "c":
            lat.collide()
            ref = collide(ref)
        elif op == "p":
            lat.propagate()
            ref = propagate(ref)
        else:
            lat.step(1)
            ref = propagate(collide(ref))
        st = [a for a in lat.get_state() if a is not None]
        for a, b in zip(st, ref):
            assert relerr(cpu(a), b) < TOL64, op
        r, uu, _ = lat.moments()
        uref, rref = O.velocity(ref[0])
        assert relerr(cpu(r), rref) < TOL64 and relerr(cpu(uu), uref) < TOL64


def test_set_state_round_trip_and_continue(lbgpu):
    nx, ny, nz = 9, 5, 4
    prm = O.Params()
    rho, u, phi = binary_case(nx, ny, nz, seed=4, phi_max=0.5)
    rf, rg = O.init_binary(rho, u, phi, prm)
    rng = np.random.default_rng(5)
    rf = rf + 1e-3 * rng.standard_normal(rf.shape) * O.W[:, None, None, None]
    lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, **params_of(prm))
    lat.set_state(rf, rg)
    f, g = lat.get_state()
    assert np.array_equal(cpu(f), rf) and np.array_equal(cpu(g), rg)
    lat.step(3)
    f, g = lat.get_state()
    ef, eg = O.step_binary(rf, rg, prm, 3)
    assert relerr(cpu(f), ef) < TOL64 and relerr(cpu(g), eg) < TOL64


@pytest.mark.parametrize("model", ["single", "binary"])
def test_conserved_sums(lbgpu, model):
    nx, ny, nz = 33, 10, 6
    prm = O.Params()
    if model == "single":
        rho, u = single_case(nx, ny, nz, seed=6)
        lat = lbgpu.Lattice(nx, ny, nz)
        lat.init_equilibrium(rho, u)
        ref = (O.init_single(rho, u), None)
    else:
        rho, u, phi = binary_case(nx, ny, nz, seed=6, phi_max=0.3, u_max=0.01)
        lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, **params_of(prm))
        lat.init_equilibrium(rho, u, phi)
        ref = O.init_binary(rho, u, phi, prm)
    s0 = cpu(lat.conserved_sums())
    want = O.conserved_sums(*ref)
    scale = np.array([want[0], 1, 1, 1, 1]) * np.abs(ref[0]).max()
    assert (np.abs(s0 - want) <= 1e-13 * nx * ny * nz * np.abs(scale)).all()
    lat.step(20)
    s1 = cpu(lat.conserved_sums())
    # collision and streaming conserve every sum: drift is rounding only
    assert abs(s1[0] - s0[0]) <= 1e-13 * abs(s0[0])
    assert (np.abs(s1[1:4] - s0[1:4]) <= 1e-14 * abs(s0[0])).all()
    if model == "binary":
        assert abs(s1[4] - s0[4]) <= 1e-14 * nx * ny * nz
    # bitwise reproducible
    assert np.array_equal(cpu(lat.conserved_sums()), s1)


def test_binary_128_bench_config_last_step(lbgpu):
    """The benchmark workload (128^3 binary, FP64, spinodal quench, 100 steps)
    in the benchmark's launch configuration: the oracle recomputes the 100th
    step from the GPU's state after 99 steps, every site; mass and phi are
    conserved over the whole run."""
    n, prm = 128, O.Params()
    rho, u, phi = inputs.spinodal_quench(n, n, n, seed=0)
    lat = lbgpu.Lattice(n, n, n, model=lbgpu.LB_BINARY, **params_of(prm))
    lat.init_equilibrium(rho, u, phi)
    s0 = cpu(lat.conserved_sums())
    lat.step(99)
    f99, g99 = (cpu(a) for a in lat.get_state())
    lat.step(1)
    f100, g100 = (cpu(a) for a in lat.get_state())
    s1 = cpu(lat.conserved_sums())
    ef, eg = O.step_binary(f99, g99, prm, 1)
    assert relerr(f100, ef) < TOL64
    assert relerr(g100, eg) < TOL64
    assert abs(s1[0] - s0[0]) <= 1e-12 * abs(s0[0])
    assert abs(s1[4] - s0[4]) <= 1e-12 * n ** 3 * 0.05
    # the quench is unstable: the band of modes with linear growth rate
    # sigma(k) = M k_h^2 (-A - kappa k_h^2) near its maximum 0.011/step has
    # gained power (x7 in the linear regime) while the white-noise total decays
    k = 2 * np.pi * np.fft.fftfreq(n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    kh2 = 2 * (3 - np.cos(kx) - np.cos(ky) - np.cos(kz))
    sigma = prm.mobility * kh2 * (-prm.A - prm.kappa * kh2)
    band = sigma > 0.009
    p0 = (np.abs(np.fft.fftn(phi)) ** 2)[band].sum()
    p1 = (np.abs(np.fft.fftn(O.order_parameter(g100))) ** 2)[band].sum()
    assert p1 > 3.0 * p0


def test_binary_128_first_steps_vs_oracle_run(lbgpu):
    """Same workload, 3 steps from the initial condition, all on both sides."""
    n, prm = 128, O.Params()
    rho, u, phi = inputs.spinodal_quench(n, n, n, seed=0)
    lat = lbgpu.Lattice(n, n, n, model=lbgpu.LB_BINARY, **params_of(prm))
    lat.init_equilibrium(rho, u, phi)
    lat.step(3)
    f, g = (cpu(a) for a in lat.get_state())
    ef, eg = O.step_binary(*O.init_binary(rho, u, phi, prm), prm, 3)
    assert relerr(f, ef) < TOL64 and relerr(g, eg) < TOL64


@pytest.mark.parametrize("vvl", [2, 4])
@pytest.mark.parametrize("nx,ny,nz", [(67, 9, 5), (5, 6, 37), (16, 16, 16)])
def test_sites_per_lane(lbgpu, vvl, nx, ny, nz):
    """2 and 4 sites per lane along z (ragged in z for nz = 5, 37): the
    single-fluid step and the binary collide-only path (phi kernel + LDS
    stencil collision) against the oracle."""
    print("case vvl", vvl, nx, ny, nz, flush=True)
    rho, u = single_case(nx, ny, nz, seed=11)
    lat = lbgpu.Lattice(nx, ny, nz, tau_f=0.8, vvl=vvl)
    lat.init_equilibrium(rho, u)
    lat.step(3)
    assert relerr(cpu(lat.get_state()[0]), O.step_single(O.init_single(rho, u), 0.8, 3)) < TOL64
    prm = O.Params()
    rho, u, phi = binary_case(nx, ny, nz, seed=12, phi_max=0.3, u_max=0.01)
    lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, vvl=vvl, **params_of(prm))
    lat.init_equilibrium(rho, u, phi)
    lat.collide()
    rf, rg = O.collide_binary(*O.init_binary(rho, u, phi, prm), prm)
    f, g = (cpu(a) for a in lat.get_state())
    assert relerr(f, rf) < TOL64 and relerr(g, rg) < TOL64


@pytest.mark.parametrize("nx,ny,nz", [(4, 4, 4), (67, 9, 5), (5, 6, 37)])
@pytest.mark.parametrize("vvl", [1, 2])
def test_trt_single_fluid(lbgpu, nx, ny, nz, vvl):
    """Two-relaxation-time collision against the oracle: fused steps and the
    stand-alone collide-only path."""
    print("case trt", nx, ny, nz, vvl, flush=True)
    tp, tm = 0.8, 1.3
    rho, u = single_case(nx, ny, nz, seed=13)
    lat = lbgpu.Lattice(nx, ny, nz, tau_f=tp, collision=lbgpu.LB_TRT, tau_minus=tm, vvl=vvl)
    lat.init_equilibrium(rho, u)
    ref = O.init_single(rho, u)
    lat.collide()
    ref = O.collide_single_trt(ref, tp, tm)
    assert relerr(cpu(lat.get_state()[0]), ref) < TOL64
    lat.propagate()
    lat.step(4)
    ref = O.step_single_trt(O.propagate(ref), tp, tm, 4)
    assert relerr(cpu(lat.get_state()[0]), ref) < TOL64


MRT_TAUS = (0.8, 1.1, 1.4, 0.9, 1.2)          # shear, flux (tau_minus), bulk, ghost_even, ghost_odd


def _mrt_lattice(lbgpu, nx, ny, nz, taus, **kw):
    ts, tq, tb, tge, tgo = taus
    return lbgpu.Lattice(nx, ny, nz, tau_f=ts, collision=lbgpu.LB_MRT, tau_minus=tq, tau_bulk=tb,
                         tau_ghost_even=tge, tau_ghost_odd=tgo, **kw)


@pytest.mark.parametrize("nx,ny,nz,vvl", [(16, 16, 16, 1), (5, 6, 37, 1), (70, 5, 17, 2), (12, 10, 9, 4)])
def test_mrt_single_fluid(lbgpu, nx, ny, nz, vvl):
    """Multiple-relaxation-time collision against the oracle: collide-only and
    fused steps."""
    print("case mrt", nx, ny, nz, vvl, flush=True)
    rho, u = single_case(nx, ny, nz, seed=17)
    lat = _mrt_lattice(lbgpu, nx, ny, nz, MRT_TAUS, vvl=vvl)
    rng = np.random.default_rng(20)                  # off equilibrium, so every moment has something to relax
    ref = O.init_single(rho, u) * (1 + 1e-3 * rng.standard_normal((19, nz, ny, nx)))
    lat.set_state(ref)
    lat.collide()
    ref = O.collide_single_mrt(ref, MRT_TAUS)
    assert relerr(cpu(lat.get_state()[0]), ref) < TOL64
    lat.propagate()
    lat.step(4)
    ref = O.step_single_mrt(O.propagate(ref), MRT_TAUS, 4)
    assert relerr(cpu(lat.get_state()[0]), ref) < TOL64


def test_mrt_reduces_to_trt_on_gpu(lbgpu):
    """With tau_bulk = tau_ghost_even = tau_f and tau_ghost_odd = tau_minus the
    MRT kernel gives the TRT kernel's result (to rounding)."""
    n = 17
    rho, u = single_case(n, n, n, seed=18)
    a = _mrt_lattice(lbgpu, n, n, n, (0.8, 1.3, 0.8, 0.8, 1.3))
    b = lbgpu.Lattice(n, n, n, tau_f=0.8, collision=lbgpu.LB_TRT, tau_minus=1.3)
    for lat in (a, b):
        lat.init_equilibrium(rho, u)
        lat.step(5)
    fa, fb = cpu(a.get_state()[0]), cpu(b.get_state()[0])
    assert relerr(fa, fb) < 1e-14


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f16", 5e-2)])
def test_mrt_reduced_precision(lbgpu, storage, tol):
    """MRT in deviation storage: velocity within the storage's tolerance of the
    FP64 oracle after 10 steps."""
    n = 16
    code = {"f32": lbgpu.LB_F32, "f16": lbgpu.LB_F16}[storage]
    rho, u = single_case(n, n, n, seed=19)
    lat = _mrt_lattice(lbgpu, n, n, n, MRT_TAUS, storage=code)
    lat.init_equilibrium(rho, u)
    lat.step(10)
    _r, ug, _p = (cpu(t) for t in lat.moments())
    uref, _rr = O.velocity(O.step_single_mrt(O.init_single(rho, u), MRT_TAUS, 10))
    assert relerr(ug, uref) < tol


@pytest.mark.parametrize("path", sorted(STEP_KERNELS))
@pytest.mark.parametrize("coll", ["trt", "mrt"])
@pytest.mark.parametrize("nx,ny,nz", [(16, 16, 16), (5, 6, 37), (70, 5, 17)])
def test_binary_trt_mrt(lbgpu, coll, nx, ny, nz, path):
    """Binary fluid with f relaxing by TRT or MRT: the collide of a direct
    state, then steps by the single-pass march or the two-pass step, against
    the oracle."""
    print("case binary", coll, nx, ny, nz, path, flush=True)
    prm = O.Params(tau_f=0.8)
    taus = (0.8, 1.25, 1.4, 0.9, 1.2) if coll == "mrt" else (0.8, 1.25, 0.8, 0.8, 1.25)
    kw = dict(collision=lbgpu.LB_MRT if coll == "mrt" else lbgpu.LB_TRT, tau_minus=taus[1])
    if coll == "mrt":
        kw.update(tau_bulk=taus[2], tau_ghost_even=taus[3], tau_ghost_odd=taus[4])
    rho, u, phi = binary_case(nx, ny, nz, seed=21, phi_max=0.3, u_max=0.01)
    lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, binary_step=STEP_KERNELS[path], **params_of(prm), **kw)
    f, g = O.step_binary(*O.init_binary(rho, u, phi, prm), prm, 1)      # off equilibrium
    lat.set_state(f, g)
    lat.collide()
    rf, rg = O.collide_binary_mrt(f, g, prm, taus)
    sf, sg = (cpu(a) for a in lat.get_state())
    assert relerr(sf, rf) < TOL64 and relerr(sg, rg) < TOL64
    lat.propagate()
    lat.step(4)
    rf, rg = O.step_binary_mrt(O.propagate(rf), O.propagate(rg), prm, taus, 4)
    sf, sg = (cpu(a) for a in lat.get_state())
    assert relerr(sf, rf) < TOL64 and relerr(sg, rg) < TOL64


@pytest.mark.parametrize("storage,tol", [("f32", 2e-4), ("f16", 0.3)])
def test_binary_mrt_reduced_precision(lbgpu, storage, tol):
    n = 16
    prm = O.Params()
    taus = (1.0, 1.25, 1.4, 0.9, 1.2)
    code = {"f32": lbgpu.LB_F32, "f16": lbgpu.LB_F16}[storage]
    rho, u, phi = binary_case(n, n, n, seed=22, phi_max=0.3, u_max=0.01)
    lat = lbgpu.Lattice(n, n, n, model=lbgpu.LB_BINARY, storage=code, phi0=float(phi.mean()),
                        collision=lbgpu.LB_MRT, tau_minus=1.25, tau_bulk=1.4, tau_ghost_even=0.9, tau_ghost_odd=1.2)
    lat.init_equilibrium(rho, u, phi)
    lat.step(10)
    _r, ug, pg = (cpu(t) for t in lat.moments())
    rf, rg = O.step_binary_mrt(*O.init_binary(rho, u, phi, prm), prm, taus, 10)
    uref, _rr = O.velocity(rf)
    assert relerr(ug, uref) < tol and relerr(pg, O.order_parameter(rg)) < tol


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("coll", ["bgk", "mrt"])
@pytest.mark.parametrize("nx,ny,nz", [(5, 6, 7), (67, 9, 21), (64, 8, 33)])
def test_binary_step_kernels_agree_bitwise(lbgpu, storage, coll, nx, ny, nz):
    """The single-pass march and the two-pass step sum phi in the same order
    and share the collision, so the states they produce are the same bits,
    in every storage and collision; LB_STEP_AUTO is one of the two."""
    code = {"f64": lbgpu.LB_F64, "f32": lbgpu.LB_F32, "f16": lbgpu.LB_F16}[storage]
    kw = dict(collision=lbgpu.LB_MRT, tau_minus=1.25, tau_bulk=1.4, tau_ghost_even=0.9,
              tau_ghost_odd=1.2) if coll == "mrt" else {}
    rho, u, phi = binary_case(nx, ny, nz, seed=31, phi_max=0.3, u_max=0.01)
    states = {}
    for path, step in (("march", 1), ("two_pass", 2), ("auto", 0)):
        lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, storage=code, phi0=float(phi.mean()),
                            binary_step=step, **kw)
        lat.init_equilibrium(rho, u, phi)
        lat.step(7)
        states[path] = lat.get_state()
        lat.close()
    for a, b in zip(states["march"], states["two_pass"]):
        assert torch.equal(a, b)
    for a, b in zip(states["march"], states["auto"]):
        assert torch.equal(a, b)
