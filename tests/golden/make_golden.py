"""Writes the stored expected values under tests/golden/ from the oracle
alone (oracle/lb_oracle.py and the seeded inputs; nothing from the GPU
library).  The paper prints no worked example, so these fixtures are the
oracle's own results on tiny seeded cases (two forward runs and one binary
adjoint step with f relaxing in moment space), kept so that a later change
of the oracle's arithmetic shows up as a failing test.

    python tests/golden/make_golden.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lb_oracle as O  # noqa: E402
from paper_1405_6162_amd import inputs  # noqa: E402

CASES = {
    # name: (model, (nx, ny, nz), steps, seed)
    "single_4x4x4_3steps": ("single", (4, 4, 4), 3, 7),
    "binary_5x4x3_2steps": ("binary", (5, 4, 3), 2, 8),
    # one MRT step of the seeded binary state, then one adjoint step with
    # seeded standard-normal adjoints (seed + 1): dL/df^n and dL/dg^n
    "binary_mrt_adjoint_5x4x3": ("binary_mrt_adjoint", (5, 4, 3), 1, 9),
}

# relaxation times of f for the moment-space case: shear, flux, bulk,
# even ghosts, odd ghosts
MRT_TAUS = (0.9, 1.3, 1.4, 0.85, 1.15)


def adjoint_inputs(shape, steps, seed):
    """(f, g, lambda_f, lambda_g) of the moment-space adjoint case."""
    nx, ny, nz = shape
    prm = O.Params(tau_f=MRT_TAUS[0])
    rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=seed, phi_max=0.3)
    f, g = O.step_binary_mrt(*O.init_binary(rho, u, phi, prm), prm, MRT_TAUS, steps)
    rng = np.random.default_rng(seed + 1)
    return f, g, rng.standard_normal(f.shape), rng.standard_normal(g.shape)


def compute(model, shape, steps, seed):
    """The case's state after `steps` steps, as one (k, 19, nz, ny, nx) array
    (k = 1 single fluid: f; k = 2 binary: f, g; for the adjoint case the
    adjoints dL/df, dL/dg one step earlier)."""
    nx, ny, nz = shape
    if model == "single":
        rho, u = inputs.single_fluid_random(nx, ny, nz, seed=seed)
        f = O.step_single(O.init_single(rho, u), 1.0, steps)
        return f[None]
    if model == "binary_mrt_adjoint":
        f, g, lf, lg = adjoint_inputs(shape, steps, seed)
        lf_n, lg_n, _grads = O.adjoint_step_binary(f, g, lf, lg, O.Params(tau_f=MRT_TAUS[0]), MRT_TAUS)
        return np.stack([lf_n, lg_n])
    prm = O.Params()
    rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=seed, phi_max=0.3)
    f, g = O.step_binary(*O.init_binary(rho, u, phi, prm), prm, steps)
    return np.stack([f, g])


# the library's order of the binary MRT rate sums: d/d omega of the shear
# (tau_f), of g (tau_g), of kappa, then flux, bulk, even ghosts, odd ghosts
MRT_GRAD_NAMES = ("omega_shear", "omega_g", "kappa", "omega_flux", "omega_bulk", "omega_ghost_even",
                  "omega_ghost_odd")


def adjoint_grads(shape, steps, seed):
    """The seven parameter sums of the binary MRT adjoint step, in the
    library's order."""
    f, g, lf, lg = adjoint_inputs(shape, steps, seed)
    _lf, _lg, grads = O.adjoint_step_binary(f, g, lf, lg, O.Params(tau_f=MRT_TAUS[0]), MRT_TAUS)
    return np.array([grads[k] for k in MRT_GRAD_NAMES])


def path(name):
    return os.path.join(HERE, name + ".txt")


def grads_path(name):
    return os.path.join(HERE, name + "_grads.txt")


def main():
    for name, (model, shape, steps, seed) in CASES.items():
        a = compute(model, shape, steps, seed)
        what = ("%s fluid, lattice %s (nx, ny, nz), %d steps from the seeded initial state (seed %d)"
                % (model, shape, steps, seed))
        if model == "binary_mrt_adjoint":
            what = ("binary fluid with f by MRT %s, lattice %s (nx, ny, nz): dL/df, dL/dg after one adjoint "
                    "step of the state %d step(s) from the seeded initial state (seed %d)"
                    % (MRT_TAUS, shape, steps, seed))
        header = ("%s: %s, oracle FP64; array shape %s, C order, written by tests/golden/make_golden.py"
                  % (name, what, a.shape))
        np.savetxt(path(name), a.reshape(-1), fmt="%.17e", header=header)
        print(path(name))
        if model == "binary_mrt_adjoint":
            gr = adjoint_grads(shape, steps, seed)
            np.savetxt(grads_path(name), gr, fmt="%.17e",
                       header="%s: the adjoint step's parameter sums %s, oracle FP64, written by "
                              "tests/golden/make_golden.py" % (name, ", ".join(MRT_GRAD_NAMES)))
            print(grads_path(name))


if __name__ == "__main__":
    main()
