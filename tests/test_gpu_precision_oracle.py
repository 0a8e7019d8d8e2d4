"""GPU runs at the benchmarked sizes against the FP64 oracle from the same
initial state, per moment: the plain C reference (oracle/lb_oracle.c, FP64
loops on all host cores, bitwise independent of the thread count) runs the
whole lattice alongside.

- the 128^3 binary FP64 spinodal quench, 100 steps end to end: f, g, rho
  and phi equal the oracle's within 1e-12 (u in lattice units, see there);
- binary FP32 storage at 64^3 after 1 and 10 steps: velocity within 1e-6 of
  the oracle, the short-horizon claim of the FP32 path (over hundreds of
  steps the unstable modes of the quench amplify any rounding, the oracle's
  own included);
- the 96^3 sub-run of the 384^3 FP16 workload: 1000 steps in FP64, FP32 and
  FP16-deviation storage against the oracle: per-moment errors printed,
  FP64 gated by its rounding floor, the reduced storages by the coarsening
  length and interface density of phi and by mass drift.

Error metric: max |q - q_ref| / max |q_ref| for q in rho, u (all three
components together) and phi.
"""

import numpy as np
import pytest

from oracle import c_backend as C
from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu


def relerr(a, ref):
    return float(np.abs(np.asarray(a) - ref).max() / np.abs(ref).max())


def _oracle_moments(n, steps, seed=0):
    C.set_threads(0)
    rho, u, phi = inputs.spinodal_quench(n, n, n, seed=seed)
    ref = C.CLattice(n, n, n, model=1)
    ref.init_equilibrium(rho, u, phi)
    done = 0
    out = {}
    for k in sorted(steps):
        ref.step(k - done)
        done = k
        out[k] = ref.moments()
    ref.close()
    return (rho, u, phi), out


def _gpu(lbgpu, fields, storage):
    rho, u, phi = fields
    n = phi.shape[0]
    lat = lbgpu.Lattice(n, n, n, model=lbgpu.LB_BINARY, storage=storage, rho0=1.0, phi0=float(phi.mean()))
    lat.init_equilibrium(rho, u, phi)
    return lat


def _errors(lat, ref):
    r, u, p = (a.cpu().numpy() for a in lat.moments())
    return {"rho": relerr(r, ref[0]), "u": relerr(u, ref[1]), "phi": relerr(p, ref[2])}


def test_binary_128_fp64_100_steps_end_to_end(lbgpu):
    """f and g within 1e-12 of the oracle's, relative to their largest
    value, and so rho and phi.  u = j / rho is small in a quench that starts
    at rest (max |u| ~ 1e-4 here), so its error is gated in lattice units
    (the scale of c_i, where rounding of the O(1) populations lives) and
    only reported relative to max |u|."""
    print("case binary 128^3 FP64 x100 vs C oracle", flush=True)
    n = 128
    C.set_threads(0)
    rho, u, phi = inputs.spinodal_quench(n, n, n, seed=0)
    ref = C.CLattice(n, n, n, model=1)
    ref.init_equilibrium(rho, u, phi)
    ref.step(100)
    fo, go = ref.state()
    r0, u0, p0 = ref.moments()
    ref.close()
    lat = _gpu(lbgpu, (rho, u, phi), lbgpu.LB_F64)
    lat.step(100)
    f, g = (a.cpu().numpy() for a in lat.get_state())
    r, v, p = (a.cpu().numpy() for a in lat.moments())
    lat.close()
    ef, eg, er, ep = relerr(f, fo), relerr(g, go), relerr(r, r0), relerr(p, p0)
    du = float(np.abs(v - u0).max())
    print("binary 128^3 FP64 x100 vs oracle: f %.2e g %.2e rho %.2e phi %.2e | u %.2e absolute, %.2e relative to "
          "max |u| = %.2e" % (ef, eg, er, ep, du, du / np.abs(u0).max(), np.abs(u0).max()), flush=True)
    assert max(ef, eg, er, ep) <= 1e-12
    assert du <= 1e-14


def test_binary_fp32_velocity_short_horizon_64(lbgpu):
    print("case binary 64^3 FP32 x1, x10 vs C oracle", flush=True)
    fields, ref = _oracle_moments(64, [1, 10])
    lat = _gpu(lbgpu, fields, lbgpu.LB_F32)
    errs = {}
    done = 0
    for k in (1, 10):
        lat.step(k - done)
        done = k
        errs[k] = _errors(lat, ref[k])
        print("binary 64^3 FP32 x%d vs oracle: rho %.2e u %.2e phi %.2e"
              % (k, errs[k]["rho"], errs[k]["u"], errs[k]["phi"]), flush=True)
    lat.close()
    for k in (1, 10):
        assert errs[k]["u"] <= 1e-6, k
        assert errs[k]["rho"] <= 1e-7 and errs[k]["phi"] <= 1e-6, k


def _coarsening_length(phi):
    S = np.abs(np.fft.fftn(phi)) ** 2
    ks = [2 * np.pi * np.fft.fftfreq(m) for m in phi.shape]
    kz, ky, kx = np.meshgrid(*ks, indexing="ij")
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    S[0, 0, 0] = 0
    return float(2 * np.pi * S.sum() / (k * S).sum())


def _interface_density(phi):
    return float(sum((phi * np.roll(phi, 1, axis=a) < 0).mean() for a in range(3)) / 3)


def test_binary_96_sub_run_1000_steps(lbgpu):
    """The 96^3 sub-run: FP64, FP32 and FP16-deviation storage after 1000
    steps against the FP64 oracle."""
    print("case binary 96^3 x1000 FP64/FP32/FP16 vs C oracle", flush=True)
    n, steps = 96, 1000
    fields, ref = _oracle_moments(n, [steps])
    r_ref, u_ref, p_ref = ref[steps]
    L_ref, I_ref = _coarsening_length(p_ref), _interface_density(p_ref)
    print("oracle 96^3 x1000: coarsening length %.4f interface density %.5f" % (L_ref, I_ref), flush=True)
    res = {}
    for name, code in (("f64", lbgpu.LB_F64), ("f32", lbgpu.LB_F32), ("f16", lbgpu.LB_F16)):
        lat = _gpu(lbgpu, fields, code)
        s0 = lat.conserved_sums().cpu().numpy()
        lat.step(steps)
        s1 = lat.conserved_sums().cpu().numpy()
        e = _errors(lat, ref[steps])
        p = lat.moments()[2].cpu().numpy()
        lat.close()
        e["L"] = abs(_coarsening_length(p) / L_ref - 1)
        e["I"] = abs(_interface_density(p) / I_ref - 1)
        e["mass"] = abs(s1[0] - s0[0]) / abs(s0[0])
        res[name] = e
        print("%s 96^3 x1000 vs oracle: rho %.2e u %.2e phi %.2e | coarsening length %.2e interface density %.2e "
              "(relative) | mass drift %.2e" % (name, e["rho"], e["u"], e["phi"], e["L"], e["I"], e["mass"]),
              flush=True)
    # FP64: rounding order only, grown by the unstable modes over 1000 steps
    # (measured 1e-13 on phi); FP32 keeps the statistics to a few 1e-6,
    # FP16 deviations to about 1e-3.
    assert res["f64"]["phi"] <= 1e-11 and res["f64"]["u"] <= 1e-11 and res["f64"]["rho"] <= 1e-13
    assert res["f32"]["L"] <= 1e-4 and res["f32"]["I"] <= 1e-4
    assert res["f16"]["L"] <= 1e-2 and res["f16"]["I"] <= 1e-2
    for name in ("f32", "f16"):
        assert res[name]["mass"] <= 1e-6, name
