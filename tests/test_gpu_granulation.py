"""GPU parity of the granulation driver (Sect. 2.3, eqs. 1-4) and of the
snapshot-interpolated nudging target, against the CPU oracle on the same
seeded random pools: the granule population (births, deaths, advection) is
integer and placement work, compared exactly; the velocity snapshot is float64,
compared to 1e-12 of its maximum; the MHD step with a snapshot pair as driver
to 1e-12 per field after one step and 1e-11 after ten."""
import math

import numpy as np
import pytest

from oracle import granulation as G
from oracle import mhd as O
from paper_1908_08557_amd import workloads as W
from parity_util import assert_parity, oracle_dt

pytestmark = pytest.mark.gpu


def _lib_driver(p):
    from paper_1908_08557_amd import cmhd
    return cmhd.Granulation(p)


def _vext(p, seed):
    # a smooth periodic flow of ~1 km/s (an external, LCT-like field)
    X, Y = G.pixel_coords(p)
    XX, YY = np.meshgrid(X, Y)
    rng = np.random.default_rng(seed)
    a, b, c = rng.uniform(0.5, 1.5, 3)
    kx, ky = 2 * np.pi / p["Lx"], 2 * np.pi / p["Ly"]
    return np.stack([a * np.sin(ky * YY + c) + 0.3, b * np.cos(kx * XX - c) - 0.2])


def _compare_population(lib, ref, label):
    got = lib.granules()
    exp = ref.gr.array()
    print(f"[gran] {label}: {len(exp)} granules", flush=True)
    assert got.shape == exp.shape
    # placement, birth time and advection: identical arithmetic, bit-exact
    assert np.array_equal(got[:, :3], exp[:, :3]), label
    # T, v_max, t_max go through the same libm log/sqrt
    assert np.allclose(got[:, 3:], exp[:, 3:], rtol=1e-15, atol=0), label


def _compare_velocity(lib, ref, t, label, tol=1e-12):
    import torch
    got = lib.velocity(t)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    exp = ref.velocity(t)
    err = np.max(np.abs(got - exp)) / np.max(np.abs(exp))
    print(f"[gran] {label}: velocity max rel err {err:.2e} (max |v| {np.max(np.abs(exp)):.3f})",
          flush=True)
    assert err <= tol, label


@pytest.mark.parametrize("nx,ny,Lx,Ly", [(64, 64, 6.4, 6.4), (128, 64, 12.8, 7.0)])
def test_population_and_velocity_over_updates(nx, ny, Lx, Ly):
    p = G.params(nx, ny, Lx, Ly)
    u, xi = W.granulation_randoms(20000, 21)
    lib = _lib_driver(p)
    ref = G.Driver(p)
    cur = 0
    vext = _vext(p, 5)
    # first fill, a quiet update, advection, then deaths and rebirths
    for k, (t, ve) in enumerate([(0.0, None), (0.01, None), (0.05, vext), (0.35, vext),
                                 (0.52, None), (0.9, vext)]):
        print(f"[case] granulation {nx}x{ny} update {k} t={t}", flush=True)
        b_ref = ref.update(t, u, xi, vext=ve)
        b_lib = lib.update(t, u[cur:], xi[2 * cur:], vext=ve)
        cur += b_lib
        assert b_lib == b_ref and cur == ref.cursor
        _compare_population(lib, ref, f"{nx}x{ny} t={t}")
        _compare_velocity(lib, ref, t + 0.003, f"{nx}x{ny} t={t}")
    lib.close()


def test_population_at_the_benchmark_plane():
    # 512^2 pixels over 50 Mm (the photosphere of the 512x512x256 box):
    # ~4000 granules, placement exact
    p = G.params(512, 512, 50.0, 50.0)
    u, xi = W.granulation_randoms(12000, 8)
    print("[case] granulation 512x512 population", flush=True)
    lib = _lib_driver(p)
    ref = G.Driver(p)
    assert lib.update(0.0, u, xi) == ref.update(0.0, u, xi)
    _compare_population(lib, ref, "512x512 t=0")
    lib.close()


def test_velocity_256_plane():
    p = G.params(256, 256, 25.0, 25.0)
    u, xi = W.granulation_randoms(6000, 9)
    print("[case] granulation 256x256 velocity", flush=True)
    lib = _lib_driver(p)
    ref = G.Driver(p)
    lib.update(0.0, u, xi)
    ref.update(0.0, u, xi)
    _compare_velocity(lib, ref, 0.12, "256x256 t=0.12")
    lib.close()


def test_empty_population_and_pool_exhaustion():
    import torch
    from paper_1908_08557_amd import cmhd
    p = G.params(64, 64, 6.4, 6.4)
    lib = _lib_driver(p)
    v = lib.velocity(0.0)
    torch.cuda.synchronize()
    assert np.max(np.abs(v.cpu().numpy())) == 0.0
    u, xi = W.granulation_randoms(10, 3)
    with pytest.raises(cmhd.CmhdError):
        lib.update(0.0, u, xi)
    ref = G.Granules()
    with pytest.raises(G.PoolExhausted):
        G.fill(ref, 0.0, p, u, xi, 0)
    # the granules born before the pool ran out are kept, as in the oracle
    got = lib.granules()
    assert np.array_equal(got[:, :3], ref.array()[:, :3])
    lib.close()


# ---------------------------------------------------------------------------
# the MHD step with a snapshot pair as driver
# ---------------------------------------------------------------------------

def _snapshot_case():
    w = W.small_stratified(32, 32, 24)
    g = w.grid
    u1 = W.solenoidal_uh(g["nx"], g["ny"], g["Lx"], g["Ly"], seed=17, rms=1.0, ell=1.0)
    return w, w.uh_target, u1


def _runs(w, u0, u1, t0, t1, nsteps, dt):
    import torch
    from paper_1908_08557_amd import cmhd
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    drv = dict(uh0=u0, uh1=u1, t0=t0, t1=t1, ah=w.ah_target)
    F, _ = O.run(F, 0.0, dt, nsteps, w.grid, w.params, w.lnrho0_z, drv)
    ref = O.to_compact(F)
    s = cmhd.solver_for(w)
    s.set_driver_snapshots(u0, t0, u1, t1)
    st = s.new_state(w.state)
    t = 0.0
    for _ in range(nsteps):
        t, _ = s.rk3_step(st, t, dt)
    torch.cuda.synchronize()
    got = st.cpu().numpy()
    s.close()
    return got, ref


def test_snapshot_driver_one_and_ten_steps():
    w, u0, u1 = _snapshot_case()
    dt = oracle_dt(w)
    w.params.update(t_ramp=0.0)
    # the substage times cross the snapshot interval: clipped, interpolated
    t0, t1 = 2.5 * dt, 7.5 * dt
    print(f"[case] snapshot driver strat32x32x24 dt={dt:.3e}", flush=True)
    got, ref = _runs(w, u0, u1, t0, t1, 1, dt)
    assert_parity(got, ref, True, 1e-12, "snapshots 1 step")
    got, ref = _runs(w, u0, u1, t0, t1, 10, dt)
    assert_parity(got, ref, True, 1e-11, "snapshots 10 steps")


def test_snapshot_driver_rejects_bad_times_and_driver_cotangents():
    import torch
    from paper_1908_08557_amd import cmhd
    w, u0, u1 = _snapshot_case()
    s = cmhd.solver_for(w)
    with pytest.raises(cmhd.CmhdError):
        s.set_driver_snapshots(u0, 1.0, u1, 1.0)
    s.set_driver_snapshots(u0, 0.0, u1, 1.0)
    s.bind_adjoint()
    x = s.new_state(w.state)
    with pytest.raises(cmhd.CmhdError):
        s.rk3_step_vjp(x, 0.0, 1e-9, torch.zeros_like(x),
                       uhbar=torch.zeros((2, 32, 32), dtype=torch.float64, device=x.device))
    s.close()
