"""cmhd_cfl_dt_noalloc, the entry point that allocates nothing, against
cmhd_cfl_dt through the C ABI: the same time step bit for bit (the same
reduction kernel; the maxima are exact in any order), from a context with no
workspace bound, on two calls in a row (the second on a smaller box)."""
import ctypes

import pytest

from paper_1908_08557_amd import workloads as W

pytestmark = pytest.mark.gpu


def _raw_context(s):
    """A second context on the solver's grid with no workspace bound."""
    dptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ctx = ctypes.c_void_p()
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    rc = s.lib.cmhd_init_grid_z(ctypes.byref(s._g), ctypes.byref(s._p), dptr(s._z), dptr(s._lr),
                                dptr(s._lt), ctypes.c_void_p(stream), ctypes.byref(ctx))
    assert rc == 0
    return ctx


def _dts(w):
    import torch
    from paper_1908_08557_amd import cmhd
    s = cmhd.solver_for(w)
    x = s.new_state(w.state)
    ref = s.cfl_dt(x)                  # fills the ghosts of x; reduction in the workspace
    ctx = _raw_context(s)
    dt = ctypes.c_double(0.0)
    rc = s.lib.cmhd_cfl_dt_noalloc(ctx, ctypes.c_void_p(x.data_ptr()), ctypes.byref(dt))
    assert rc == 0, s.lib.cmhd_last_error(ctx).decode()
    again = s.cfl_dt_noalloc(x)        # the same entry point from the bound context
    s.lib.cmhd_destroy(ctx)
    torch.cuda.synchronize()
    s.close()
    return ref, dt.value, again


def test_noalloc_cfl_matches_workspace_cfl_on_two_calls():
    for w in (W.strat64(), W.small_stratified(32, 32, 16)):   # the second is smaller
        print(f"[case] cfl_dt_noalloc {w.name}", flush=True)
        ref, got, again = _dts(w)
        assert got == ref and again == ref, (w.name, ref, got, again)


def test_noalloc_cfl_periodic_box():
    print("[case] cfl_dt_noalloc periodic16", flush=True)
    ref, got, again = _dts(W.periodic_box(16))
    assert got == ref and again == ref


def test_noalloc_cfl_rejects_stretched_grid_without_workspace():
    from paper_1908_08557_amd import cmhd
    w = W.small_stretched(32, 32, 24, Lxy=20.0, nbip=2)
    print("[case] cfl_dt_noalloc stretched grid, no workspace", flush=True)
    s = cmhd.solver_for(w)
    x = s.new_state(w.state)
    ctx = _raw_context(s)
    dt = ctypes.c_double(0.0)
    rc = s.lib.cmhd_cfl_dt_noalloc(ctx, ctypes.c_void_p(x.data_ptr()), ctypes.byref(dt))
    assert rc == cmhd.CMHD_ESTATE
    assert "workspace" in s.lib.cmhd_last_error(ctx).decode()
    s.lib.cmhd_destroy(ctx)
    s.cfl_dt(x)                        # fills the ghosts
    assert s.cfl_dt_noalloc(x) == s.cfl_dt(x)
    s.close()
