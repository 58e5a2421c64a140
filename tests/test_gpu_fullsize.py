"""GPU parity at the benchmark's full size, in the launch configuration that
bench.py times (512 x 512 x 256, two z chunks of 128 planes, XCD-ordered tiles), and
on the largest box (1024 x 1024 x 256), on sampled outputs: one step of the whole box on the GPU, and for each sampled
zone the oracle run on a 25^3 patch around it.  After one RK3 step a zone
depends on the state within 9 zones (three substages of the 3-zone stencils),
so a patch that reaches 12 zones out, with periodic wrap at its edges, gives
the oracle's value of its centre exactly (up to rounding); samples stay 12
zones away from the photosphere and below the swamp layer, where the solar
boundary rules would enter (the boundary work at these plane sizes is checked
whole in test_gpu_boundary_fullsize.py)."""
import numpy as np
import pytest

from oracle import mhd as O
from paper_1908_08557_amd import workloads as W
from parity_util import (FLOOR_FACTOR, GROUPS, NAMES, NG, RESIDUES, oracle_patch_centre,
                         perturbed)

pytestmark = pytest.mark.gpu

H = 12          # patch half-width
NSAMPLE = 16


def _gpu_one_step(w, precision):
    import torch
    from paper_1908_08557_amd import cmhd
    s = cmhd.solver_for(w, precision)
    st = s.new_state(w.state)
    dt = s.cfl_dt(st)
    t, _ = s.rk3_step(st, 0.0, dt)
    torch.cuda.synchronize()
    out = st.cpu().numpy()
    s.close()
    del st
    torch.cuda.empty_cache()
    return out, dt


def _samples(w, seed):
    g, p = w.grid, w.params
    z = O.zk(g)[NG:NG + g["nz"]]
    kmax = int(np.searchsorted(z, p["z_s"])) - 1 - H
    rng = np.random.default_rng(seed)
    ks = rng.integers(H, kmax + 1, NSAMPLE)
    ks[0], ks[1] = H, kmax                      # both ends of the allowed range
    js = rng.integers(0, g["ny"], NSAMPLE)
    is_ = rng.integers(0, g["nx"], NSAMPLE)
    is_[2], js[2] = g["nx"] - 1, 0              # a patch that wraps in x and y
    return list(zip(ks, js, is_))


def _check(w, got, dt, tol, label, precision):
    """Sampled zones against the oracle, each component relative to its own
    max norm over the box, the cancellation residues (and, in the split
    form, the velocity one step from hydrostatic rest) relative to their
    field.  In float64 a component is held to FLOOR_FACTOR times the
    oracle's own spread where that exceeds tol: the patch is run again from
    a state moved by one unit in the last place.  All figures printed."""
    own = np.array([np.max(np.abs(got[f, NG:-NG])) for f in range(8)])
    grp = np.array([max(own[q] for q in GROUPS[f]) for f in range(8)])
    by_field = [NAMES[f] in RESIDUES or (precision != "fp64" and NAMES[f] in ("ux", "uy", "uz"))
                for f in range(8)]
    scales = np.array([grp[f] if by_field[f] else own[f] for f in range(8)])
    wp = perturbed(w) if precision == "fp64" else None
    worst = np.zeros(8)
    spread = np.zeros(8)
    for (k, j, i) in _samples(w, 11):
        ref = oracle_patch_centre(w, int(k), int(j), int(i), dt, H)
        val = got[:, NG + k, j, i]
        worst = np.maximum(worst, np.abs(val - ref))
        if wp is not None:
            refp = oracle_patch_centre(wp, int(k), int(j), int(i), dt, H)
            spread = np.maximum(spread, np.abs(refp - ref))
    print(f"[parity] {label} sampled own: "
          + " ".join(f"{NAMES[f]}={worst[f] / own[f]:.2e}" for f in range(8)), flush=True)
    print(f"[parity] {label} sampled field: "
          + " ".join(f"{NAMES[f]}={worst[f] / grp[f]:.2e}" for f in range(8)), flush=True)
    lim = np.full(8, tol)
    if wp is not None:
        print(f"[parity] {label} oracle floor: "
              + " ".join(f"{NAMES[f]}={spread[f] / own[f]:.2e}" for f in range(8)), flush=True)
        for f in range(8):
            if not by_field[f]:
                lim[f] = max(tol, FLOOR_FACTOR * spread[f] / own[f])
    rel = worst / scales
    assert np.all(rel <= lim), (label, dict(zip(NAMES, zip(rel, lim))))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_split", 2e-6)])
def test_strat512_one_step_sampled(precision, tol):
    w = W.strat512()
    print(f"[case] strat512 one step {precision}, {NSAMPLE} sampled zones", flush=True)
    got, dt = _gpu_one_step(w, precision)
    _check(w, got, dt, tol, f"strat512 {precision}", precision)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_split", 2e-6)])
def test_strat512_stretched_one_step_sampled(precision, tol):
    w = W.strat512_stretched()
    print(f"[case] strat512_stretched one step {precision}, {NSAMPLE} sampled zones", flush=True)
    got, dt = _gpu_one_step(w, precision)
    _check(w, got, dt, tol, f"strat512_stretched {precision}", precision)


@pytest.mark.timeout(1200)
def test_ar1024_one_step_sampled():
    # the largest box: 1024^2 x 256 over 64 Mm with 32 bipoles (the 2-D
    # transforms at their maximum length), FP32-split as in its workload
    w = W.ar1024()
    print(f"[case] ar1024 one step fp32_split, {NSAMPLE} sampled zones", flush=True)
    got, dt = _gpu_one_step(w, "fp32_split")
    _check(w, got, dt, 2e-6, "ar1024 fp32_split", "fp32_split")
