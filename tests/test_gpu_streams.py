"""The context follows the caller's stream: steps issued on a side stream
(every kernel of the step is launched on the context's stream) equal the
steps on the default stream bitwise; and the kernel-timing
API (cmhd_profile_enable / cmhd_profile_read) counts the substages, resets on
read and rejects an unknown selector."""
import ctypes

import pytest

from paper_1908_08557_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(32, 32, 24), (256, 256, 32)])
def test_steps_on_a_side_stream_equal_default_stream(shape):
    import torch
    from paper_1908_08557_amd import cmhd
    nx, ny, nz = shape
    w = (W.small_stratified(nx, ny, nz) if nx == 32
         else W.small_stratified(nx, ny, nz, Lxy=80.0, nbip=4))
    print(f"[case] side stream {nx}x{ny}x{nz}", flush=True)
    s = cmhd.solver_for(w)
    x0 = s.new_state(w.state)
    dt = s.cfl_dt(x0)
    ref = x0.clone()
    t = 0.0
    for _ in range(2):
        t, _ = s.rk3_step(ref, t, dt)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        x = x0.clone()
        t = 0.0
        for _ in range(2):
            t, _ = s.rk3_step(x, t, dt)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert torch.equal(x, ref)
    s.close()


def test_profile_counts_and_resets():
    import torch
    from paper_1908_08557_amd import cmhd
    w = W.small_stratified(32, 32, 24)
    print("[case] kernel timing API", flush=True)
    s = cmhd.solver_for(w)
    x = s.new_state(w.state)
    dt = s.cfl_dt(x)
    s.profile(True)
    s.profile_read("substage")
    s.profile_read("ghosts")
    t = 0.0
    for _ in range(2):
        t, _ = s.rk3_step(x, t, dt)
    ms, n = s.profile_read("substage")
    gms, gn = s.profile_read("ghosts")
    assert n == 6 and ms > 0.0          # three substages per step
    assert gn == 6 and gms > 0.0        # the boundary work of every substage
    assert s.profile_read("substage") == (0.0, 0)
    s.profile(False)
    s.rk3_step(x, t, dt)
    assert s.profile_read("substage")[1] == 0
    ms_, n_ = ctypes.c_double(0.0), ctypes.c_int(0)
    rc = s.lib.cmhd_profile_read(s.ctx, 7, ctypes.byref(ms_), ctypes.byref(n_))
    assert rc == cmhd.CMHD_EINVAL
    torch.cuda.synchronize()
    s.close()
