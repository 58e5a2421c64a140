"""Writes adjoint128_cs.json: the oracle's complex-step directional
derivatives of the B_z misfit loss for the 128 x 128 x 64 adjoint box with
the full stratified-box physics (radiation and Spitzer conduction on).

Loss: L = 1/2 sum_xy (B_z(x, y, 10 Mm) - target)^2 after 20 RK3 steps, the
target being the potential-field B_z at 10 Mm of a second seeded bipole set;
the derivative is taken with respect to the photospheric driver target u*
(2 x 128 x 128) along seeded standard-normal directions.  The complex step
(an imaginary perturbation of size 1e-30 carried through every operation of
the step) has no subtractive cancellation, so the stored numbers are exact to
round-off.  Only the oracle and the seeded input generators are called.

Run from the repository root:  python tests/golden/make_adjoint128_cs.py
(about 20 minutes per direction on one core; the directions run in parallel).
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import mhd as O                                     # noqa: E402
from paper_1908_08557_amd import workloads as W                 # noqa: E402

NSTEPS = 20
ZQ = 10.0
SEEDS = (101, 202)


def _setup():
    w = W.adjoint128()
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    dt = O.cfl_dt(F, w.grid, w.params)
    drv = dict(uh=w.uh_target, ah=w.ah_target)
    return w, F, dt, drv


def _directional(seed):
    w, F, dt, drv = _setup()
    v = np.random.default_rng(seed).standard_normal(w.uh_target.shape)
    Fn, tang = O.run_complex_step(F, np.zeros_like(F), v, 0.0, dt, NSTEPS, w.grid, w.params,
                                  w.lnrho0_z, drv)
    target = w.extra["bz_target_z10"]
    bz = O.bz_at_height(Fn, w.grid, w.params, ZQ)
    dbz = O.bz_at_height(tang, w.grid, w.params, ZQ) - w.params["Bext"][2]
    return dict(seed=seed, dL_dv=float(np.sum((bz - target) * dbz)),
                loss=float(O.bz_misfit_loss(Fn, w.grid, w.params, ZQ, target)))


def main():
    _, _, dt, _ = _setup()
    with ProcessPoolExecutor(len(SEEDS)) as ex:
        res = list(ex.map(_directional, SEEDS))
    out = dict(workload="adjoint128 (128x128x64, 50 Mm box, radiation and conduction on)",
               nsteps=NSTEPS, zq=ZQ, dt=dt, loss=res[0]["loss"],
               directions=[dict(seed=r["seed"], dL_dv=r["dL_dv"]) for r in res],
               direction_recipe="numpy default_rng(seed).standard_normal((2, 128, 128))",
               script="tests/golden/make_adjoint128_cs.py")
    with open(os.path.join(HERE, "adjoint128_cs.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
