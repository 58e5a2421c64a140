"""GPU parity: the library's step against the CPU oracle, element by element,
on the same seeded inputs (float64: 1e-12 relative per field after one step,
1e-10 after 100 steps)."""
import math

import numpy as np
import pytest

from oracle import mhd as O
from paper_1908_08557_amd import workloads as W
from parity_util import NG, assert_parity, oracle_dt, oracle_floor, oracle_run

# the velocity of a stratified box one or two steps from hydrostatic rest is
# the residual of the pressure gradient, gravity and the Lorentz force of a
# potential field (J = 0 up to rounding); in the split form its error is the
# float32 rounding of those terms, so it is measured against |u|
SPLIT_SHORT_BY_FIELD = ("ux", "uy", "uz")

pytestmark = pytest.mark.gpu


def _solver(w, precision="fp64"):
    from paper_1908_08557_amd import cmhd
    return cmhd.solver_for(w, precision)


def gpu_run(w, nsteps, dt, t0=0.0, precision="fp64"):
    import torch
    s = _solver(w, precision)
    st = s.new_state(w.state)
    t = t0
    for _ in range(nsteps):
        t, _ = s.rk3_step(st, t, dt)
    torch.cuda.synchronize()
    out = st.cpu().numpy()
    s.close()
    return out


def _norad(w):
    w.params.update(rad_lnT=np.zeros(0), rad_lnL=np.zeros(0), kappa0=0.0)
    return w


CASES = {
    "periodic16": lambda: W.periodic_box(16),
    "strat32x32x24": lambda: W.small_stratified(32, 32, 24),
    "strat32x32x24_norad": lambda: _norad(W.small_stratified(32, 32, 24)),
    "strat16x32x8": lambda: W.small_stratified(16, 32, 8, Lxy=8.0, z1=6.0, nbip=1),
    "strat64x16x12": lambda: W.small_stratified(64, 16, 12, Lxy=16.0, z1=10.0, nbip=2),
    # the extreme plane shapes: 64 x 1 and 1 x 64 tiles (XCD patches one tile
    # high or wide), transforms of length 1024 beside 16, one plane per z
    # chunk; the z spacing of the 512^2 x 256 box, so that the inverted
    # potential field below stays well conditioned at dx = 62.5 km
    "strat1024x16x12": lambda: W.small_stratified(1024, 16, 12, Lxy=64.0, z1=11 * 50.0 / 255,
                                                  nbip=2),
    "strat16x1024x12": lambda: W.small_stratified(16, 1024, 12, Lxy=64.0, z1=11 * 50.0 / 255,
                                                  nbip=2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_one_step(case):
    w = CASES[case]()
    print(f"[case] one step {case}", flush=True)
    dt = oracle_dt(w)
    ref = oracle_run(w, 1, dt)
    got = gpu_run(w, 1, dt)
    assert_parity(got, ref, w.grid["zbc"] == "solar", 1e-12, f"{case} 1 step",
                  floor=oracle_floor(w, 1, dt, ref))


@pytest.mark.parametrize("case", ["periodic16", "strat32x32x24", "strat32x32x24_norad"])
def test_ten_steps(case):
    w = CASES[case]()
    print(f"[case] ten steps {case}", flush=True)
    dt = oracle_dt(w)
    ref = oracle_run(w, 10, dt)
    got = gpu_run(w, 10, dt)
    assert_parity(got, ref, w.grid["zbc"] == "solar", 1e-11, f"{case} 10 steps",
                  floor=oracle_floor(w, 10, dt, ref))


@pytest.mark.parametrize("t0", [0.03, 1.0])
def test_driver_ramp_times(t0):
    # mid-ramp and after the ramp: the nudging target enters with s(t)
    w = _norad(W.small_stratified(32, 32, 16))
    print(f"[case] ramp t0={t0}", flush=True)
    dt = oracle_dt(w)
    ref = oracle_run(w, 3, dt, t0=t0)
    got = gpu_run(w, 3, dt, t0=t0)
    assert_parity(got, ref, True, 1e-12, f"ramp t0={t0}", floor=oracle_floor(w, 3, dt, ref, t0))


def test_strat64_one_step():
    w = W.strat64()
    print("[case] strat64 one step", flush=True)
    dt = oracle_dt(w)
    ref = oracle_run(w, 1, dt)
    assert_parity(gpu_run(w, 1, dt), ref, True, 1e-12, "strat64 1 step",
                  floor=oracle_floor(w, 1, dt, ref))


def newton_case(nx=32, ny=32, nz=24, norad=False):
    """Stratified box with the chromospheric Newtonian cooling on and smooth
    seeded perturbations of ln T and ln rho in the planes k = 1..8, so that
    T != T* and rho != rho0(z) where the cooling acts (both cutoffs reached:
    the density falls through the transition region above 2 Mm)."""
    w = W.enable_newton_cooling(W.small_stratified(nx, ny, nz, Lxy=20.0, z1=20.0))
    if norad:
        # radiation and conduction off: dt is no longer limited by them, so
        # the cooling (tau_t dt up to ~1) changes ln T strongly in one step
        w.params.update(rad_lnT=np.zeros(0), rad_lnL=np.zeros(0), kappa0=0.0)
    rng = np.random.default_rng(11)
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    for f, amp in ((6, 0.3), (7, 0.08)):
        pert = np.zeros((ny, nx))
        for _ in range(4):
            kx, ky = rng.integers(1, 3, size=2)
            ph = rng.uniform(0, 2 * np.pi)
            pert += np.cos(2 * np.pi * (kx * x[None, :] + ky * y[:, None]) + ph)
        for k in range(1, 9):
            w.state[f, NG + k] += amp * pert * (1.0 - k / 9.0)
    return w


@pytest.mark.parametrize("norad", [False, True])
def test_newton_cooling_one_step(norad):
    w = newton_case(norad=norad)
    dt = oracle_dt(w)
    print(f"[case] Newtonian cooling one step (norad={norad}, dt={dt:.3e})", flush=True)
    ref = oracle_run(w, 1, dt)
    assert_parity(gpu_run(w, 1, dt), ref, True, 1e-12, f"newton 1 step norad={norad}",
                  floor=oracle_floor(w, 1, dt, ref))


def test_newton_cooling_ten_steps_and_split():
    import torch
    from paper_1908_08557_amd import cmhd
    w = newton_case()
    print("[case] Newtonian cooling ten steps (FP64) and two steps (FP32-split)", flush=True)
    dt = oracle_dt(w)
    ref = oracle_run(w, 10, dt)
    assert_parity(gpu_run(w, 10, dt), ref, True, 1e-11, "newton 10 steps",
                  floor=oracle_floor(w, 10, dt, ref))
    s = cmhd.solver_for(w, "fp32_split")
    st = s.new_state(w.state)
    t = 0.0
    for _ in range(2):
        t, _ = s.rk3_step(st, t, dt)
    assert_parity(st.cpu().numpy(), oracle_run(w, 2, dt), True, 2e-6, "newton 2 steps split",
                  field_norm=SPLIT_SHORT_BY_FIELD)


def test_newton_cooling_dt_limit():
    # tau_t enters the nudging limit of the time step like tau_u and tau_A
    import torch
    from paper_1908_08557_amd import cmhd
    w = newton_case()
    w.params.update(nc_tau=5e4)
    print("[case] Newtonian cooling dt limit", flush=True)
    s = cmhd.solver_for(w)
    dt = s.cfl_dt(s.new_state(w.state))
    assert dt == pytest.approx(oracle_dt(w), rel=1e-12)
    assert dt <= w.params["c_nudge"] / 5e4 * (1 + 1e-12)


_ZCHUNKED = {}   # oracle result shared by the two precisions


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_z_chunked_substage(precision):
    # 256 x 256 x 32 (256 tiles, 8 z chunks of 4 planes: each block's z
    # window starts and ends inside the box).  FP64 against the oracle after
    # two steps; the FP32-split form against the same oracle at its own
    # tolerance.
    import torch
    from paper_1908_08557_amd import cmhd
    w = W.small_stratified(256, 256, 32, Lxy=80.0, z1=20.0, nbip=4)
    print(f"[case] z-chunked substage 256x256x32 {precision}", flush=True)
    if "ref" not in _ZCHUNKED:
        _ZCHUNKED["dt"] = oracle_dt(w)
        _ZCHUNKED["ref"] = oracle_run(w, 2, _ZCHUNKED["dt"])
        _ZCHUNKED["floor"] = oracle_floor(w, 2, _ZCHUNKED["dt"], _ZCHUNKED["ref"])
    dt = _ZCHUNKED["dt"]
    s = cmhd.solver_for(w, precision)
    st = s.new_state(w.state)
    t = 0.0
    for _ in range(2):
        t, _ = s.rk3_step(st, t, dt)
    got = st.cpu().numpy()
    ref = _ZCHUNKED["ref"]
    if precision == "fp64":
        assert_parity(got, ref, True, 1e-12, "z-chunked 256x256x32 fp64",
                      floor=_ZCHUNKED["floor"])
    else:
        assert_parity(got, ref, True, 2e-6, "z-chunked 256x256x32 fp32_split",
                      field_norm=SPLIT_SHORT_BY_FIELD)


@pytest.mark.timeout(900)
def test_strat64_hundred_steps():
    w = W.strat64()
    print("[case] strat64 100 steps", flush=True)
    dt = oracle_dt(w)
    got = gpu_run(w, 100, dt)
    ref = oracle_run(w, 100, dt)
    assert_parity(got, ref, True, 1e-10, "strat64 100 steps")


@pytest.mark.timeout(600)
def test_strat_norad_hundred_steps():
    # radiation and conduction off: dt is advective (~1.4e-3, about 1.7e5
    # times the step that radiation and conduction allow), so the 100 steps
    # move the stratified box far more than the full-physics case does
    w = CASES["strat32x32x24_norad"]()
    print("[case] strat32x32x24_norad 100 steps", flush=True)
    dt = oracle_dt(w)
    ref = oracle_run(w, 100, dt)
    assert_parity(gpu_run(w, 100, dt), ref, True, 1e-10, "strat32x32x24_norad 100 steps",
                  floor=oracle_floor(w, 100, dt, ref))


def test_periodic16_hundred_steps():
    w = W.periodic_box(16)
    print("[case] periodic16 100 steps", flush=True)
    dt = oracle_dt(w)
    assert_parity(gpu_run(w, 100, dt), oracle_run(w, 100, dt), False, 1e-10,
                  "periodic16 100 steps")


def test_cfl_dt_matches_oracle():
    for case in ("periodic16", "strat32x32x24", "strat32x32x24_norad"):
        w = CASES[case]()
        print(f"[case] cfl {case}", flush=True)
        s = _solver(w)
        st = s.new_state(w.state)
        dt = s.cfl_dt(st)
        ref = oracle_dt(w)
        assert abs(dt - ref) <= 1e-12 * ref, (case, dt, ref)
        s.close()


def test_step_with_cfl_dt_selected_on_device():
    w = W.periodic_box(16)
    s = _solver(w)
    st = s.new_state(w.state)
    t, used = s.rk3_step(st, 0.0, 0.0)
    assert abs(used - oracle_dt(w)) <= 1e-12 * used and t == used


def test_set_driver_from_bz():
    # A_h* computed on the device from B_z (eq. 7), then one step that nudges
    # A_h toward it, against the oracle's A_h* and step
    w = W.small_stratified(64, 32, 12, Lxy=20.0)
    print("[case] A_h* from B_z", flush=True)
    g = w.grid
    bz = W.bipole_field(g["nx"], g["ny"], g["Lx"], g["Ly"], 3, 7, 100.0, 1.5, 4.0)
    w.ah_target = O.ah_from_bz(bz, g["Lx"], g["Ly"])
    dt = oracle_dt(w)
    w.params["tau_A"] = 1.0 / dt   # make the nudging visible in one step
    got = gpu_run_with_bz(w, bz, dt)
    ref = oracle_run(w, 1, dt)
    assert_parity(got, ref, True, 1e-12, "nudging toward A_h* from B_z",
                  floor=oracle_floor(w, 1, dt, ref))


def gpu_run_with_bz(w, bz, dt):
    import torch
    from paper_1908_08557_amd import cmhd
    s = cmhd.Solver(w.grid, w.params, w.lnrho0_z)
    s.set_driver(w.uh_target, bz=bz)
    st = s.new_state(w.state)
    s.rk3_step(st, 0.0, dt)
    torch.cuda.synchronize()
    return st.cpu().numpy()


def test_bz_plane_matches_oracle():
    import torch
    w = W.small_stratified(32, 32, 16)
    print("[case] bz plane", flush=True)
    s = _solver(w)
    st = s.new_state(w.state)
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    for zq in (0.0, 3.3, w.grid["z1"]):
        got = s.bz_plane(st, zq).cpu().numpy()
        ref = O.bz_at_height(F, w.grid, w.params, zq)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), zq


def test_bitwise_determinism_and_resume():
    import torch
    w = W.small_stratified(32, 32, 16)
    print("[case] determinism/resume", flush=True)
    dt = oracle_dt(w)
    a = gpu_run(w, 10, dt)
    b = gpu_run(w, 10, dt)
    assert np.array_equal(a, b)
    half = gpu_run(w, 5, dt)
    w2 = W.small_stratified(32, 32, 16)
    w2.state = half
    t0 = 0.0
    for _ in range(5):
        t0 += dt
    c = gpu_run(w2, 5, dt, t0=t0)
    assert np.array_equal(a[:, NG:-NG], c[:, NG:-NG])
    assert np.array_equal(a[3:5, :NG], c[3:5, :NG])


def test_translation_equivariance_periodic():
    w = W.periodic_box(16)
    dt = oracle_dt(w)
    a = gpu_run(w, 2, dt)
    shift = (2, -3, 5)
    w.state[:, NG:-NG] = np.roll(w.state[:, NG:-NG], shift, axis=(1, 2, 3))
    b = gpu_run(w, 2, dt)
    assert np.array_equal(b[:, NG:-NG], np.roll(a[:, NG:-NG], shift, axis=(1, 2, 3)))


def test_get_fields_layouts():
    w = W.small_stratified(32, 16, 12)
    s = _solver(w)
    st = s.new_state(w.state)
    inner = s.get_fields(st, mask=0b10100001)
    assert inner.shape == (3, 12, 16, 32)
    assert np.array_equal(inner[0], w.state[0, NG:-NG])
    assert np.array_equal(inner[1], w.state[5, NG:-NG])
    assert np.array_equal(inner[2], w.state[7, NG:-NG])
    full = s.get_fields(st, mask=0xFF, with_ghosts=True)
    assert np.array_equal(full, w.state)


def test_invalid_arguments_raise():
    from paper_1908_08557_amd import cmhd
    w = W.small_stratified(32, 32, 12)
    g = dict(w.grid)
    g["nx"] = 24
    with pytest.raises(cmhd.CmhdError):
        cmhd.Solver(g, w.params, w.lnrho0_z)
    s = cmhd.Solver(w.grid, w.params, w.lnrho0_z)
    bad = np.ones((32, 32))          # net flux: rejected (Sect. 2.1 flux balance)
    with pytest.raises(cmhd.CmhdError) as e:
        s.set_driver(w.uh_target, bz=bad)
    assert e.value.code == cmhd.CMHD_EINVAL


def test_nonfinite_state_detected():
    from paper_1908_08557_amd import cmhd
    w = W.small_stratified(32, 32, 12)
    w.state[7, NG + 4, 3, 5] = np.nan
    s = cmhd.solver_for(w)
    st = s.new_state(w.state)
    assert s.check_finite(st) is False
    with pytest.raises(cmhd.CmhdError) as e:
        s.cfl_dt(st)
    assert e.value.code == cmhd.CMHD_ENONFINITE


@pytest.mark.parametrize("physics", ["norad", "full"])
def test_fp32_split_close_to_fp64(physics):
    # 100 steps of the split form against FP64 from the same state and dt:
    # within 1e-5 of every physical field (with radiation and Spitzer
    # conduction on, dt is limited by the optically thin loss near the
    # photosphere)
    w = W.small_stratified(32, 32, 24)
    if physics == "norad":
        w = _norad(w)
    print(f"[case] fp32 split vs fp64, 100 steps ({physics})", flush=True)
    dt = oracle_dt(w)
    a = gpu_run(w, 100, dt, precision="fp64")
    b = gpu_run(w, 100, dt, precision="fp32_split")
    assert_parity(b, a, True, 1e-5, f"fp32_split vs fp64 100 steps ({physics})")


def test_collapsed_time_step_reported():
    # a finite state whose fast-mode speed and conduction overflow: the CFL
    # limits give dt = 0 (forced from the host; every kernel exits normally)
    from paper_1908_08557_amd import cmhd
    w = W.small_stratified(32, 32, 12)
    w.state[7, NG + 4, 3, 5] = 709.0          # T ~ 8e307
    s = cmhd.solver_for(w)
    st = s.new_state(w.state)
    assert s.check_finite(st) is True
    with pytest.raises(cmhd.CmhdError) as e:
        s.cfl_dt(st)
    assert e.value.code == cmhd.CMHD_EDT


@pytest.mark.timeout(600)
@pytest.mark.parametrize("nx,nz", [(128, 37), (256, 37)])
def test_ragged_z_chunks(nx, nz):
    # the last z chunk of the fused kernel is short: 128^2 x 37 marches
    # chunks of 2 planes (19 chunks, the last of 1); 256^2 x 37 chunks of 5
    # planes (8 chunks, the last of 2)
    w = W.small_stratified(nx, nx, nz, Lxy=nx * 0.3, z1=20.0, nbip=2)
    dt = oracle_dt(w)
    print(f"[case] ragged z chunks {nx}x{nx}x{nz}", flush=True)
    ref = oracle_run(w, 1, dt)
    assert_parity(gpu_run(w, 1, dt), ref, True, 1e-12, f"ragged {nx}x{nx}x{nz}",
                  floor=oracle_floor(w, 1, dt, ref))


def _rhs_case(name):
    if name == "newton":
        return newton_case()
    if name == "stretched":
        return W.small_stretched(32, 32, 24)
    return CASES[name]()


@pytest.mark.parametrize("case,precision,t", [
    ("periodic16", "fp64", 0.0), ("strat32x32x24", "fp64", 0.0), ("strat32x32x24", "fp64", 0.03),
    ("strat32x32x24_norad", "fp64", 0.0), ("newton", "fp64", 0.0), ("stretched", "fp64", 0.0),
    ("strat32x32x24", "fp32_split", 0.0)])
def test_eval_rhs_matches_oracle(case, precision, t):
    # cmhd_eval_rhs: dF/dt at every interior zone and at the u_x, u_y ghost
    # rows (nudging alone there), against the oracle's right-hand side; t
    # inside the switch-on ramp scales the nudging target
    import torch
    from paper_1908_08557_amd import cmhd
    w = _rhs_case(case)
    solar = w.grid["zbc"] == "solar"
    if solar and t > 0.0:
        w.params.update(t_ramp=0.06)
    print(f"[case] eval_rhs {case} {precision} t={t}", flush=True)
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    drv = dict(uh=w.uh_target, ah=w.ah_target) if solar else None
    R, Rgh = O.rhs(F, t, w.grid, w.params, drv)
    ref = np.zeros_like(w.state)
    ref[:, NG:-NG] = R
    if solar:
        ref[3:5, :NG] = Rgh
    s = cmhd.solver_for(w, precision)
    got = s.eval_rhs(s.new_state(w.state), t)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    s.close()
    tol = 1e-11 if precision == "fp64" else 1e-5
    assert_parity(got, ref, solar, tol, f"eval_rhs {case} {precision} t={t}")
