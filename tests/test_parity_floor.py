"""The oracle's own spread under a one-ulp perturbation of its input (the
floor the parity tests allow a float64 component to when it exceeds the
stated tolerance): small for a well-conditioned periodic box, well above
1e-16 for the velocity of a stratified box one step from hydrostatic rest,
whose value is the residual of pressure gradient and gravity."""
import numpy as np

from paper_1908_08557_amd import workloads as W
from parity_util import oracle_dt, oracle_floor, oracle_run, perturbed


def test_perturbation_is_one_ulp():
    w = W.small_stratified(16, 16, 8, Lxy=8.0, z1=6.0, nbip=1)
    wp = perturbed(w)
    nz = w.state != 0
    rel = np.abs(wp.state[nz] / w.state[nz] - 1.0)
    assert np.all(rel <= 2.0 ** -51)   # one or two units in the last place
    assert np.mean(wp.state[nz] != w.state[nz]) > 0.99
    assert wp.grid is w.grid and w.state is not wp.state


def test_floor_of_a_periodic_box_is_tiny():
    w = W.periodic_box(16)
    dt = oracle_dt(w)
    ref = oracle_run(w, 1, dt)
    fl = oracle_floor(w, 1, dt, ref)
    assert max(fl.values()) < 1e-13, fl


def test_floor_of_the_velocity_after_one_step_from_rest():
    w = W.small_stratified(32, 32, 24)
    assert np.all(w.state[3:6, 3:-3] == 0.0)           # the box starts at rest
    dt = oracle_dt(w)
    ref = oracle_run(w, 1, dt)
    fl = oracle_floor(w, 1, dt, ref)
    for k in ("Ax", "Ay", "lnrho", "lnT"):
        assert fl[k] < 1e-14, (k, fl[k])
    assert fl["ux"] > 1e-13 and fl["uy"] > 1e-13, fl
