"""Checkpoint and resume on the GPU: cmhd_set_fields is the inverse of
cmhd_get_fields, and a run restarted from a snapshot continues bitwise."""
import numpy as np
import pytest

from paper_1908_08557_amd import workloads as W
from parity_util import NG, oracle_dt

pytestmark = pytest.mark.gpu


def test_set_fields_inverts_get_fields():
    import torch
    from paper_1908_08557_amd import cmhd
    w = W.small_stratified(32, 32, 12)
    s = cmhd.solver_for(w)
    st = s.new_state()
    rng = np.random.default_rng(4)
    for mask, ghosts in ((0xFF, True), (0b10100100, False), (0x01, True), (0x80, False)):
        nsel = bin(mask).count("1")
        nzc = w.grid["nz"] + (2 * NG if ghosts else 0)
        src = rng.standard_normal((nsel, nzc, 32, 32))
        before = st.cpu().numpy()
        s.set_fields(st, src, mask, with_ghosts=ghosts)
        assert np.array_equal(s.get_fields(st, mask, with_ghosts=ghosts), src)
        after = st.cpu().numpy()
        # unselected fields and, without ghosts, the ghost planes are untouched
        for f in range(8):
            if not (mask >> f) & 1:
                assert np.array_equal(after[f], before[f])
            elif not ghosts:
                assert np.array_equal(after[f, :NG], before[f, :NG])
                assert np.array_equal(after[f, -NG:], before[f, -NG:])
    with pytest.raises(cmhd.CmhdError):
        s.set_fields(st, np.zeros((0, 12, 32, 32)), 0)
    s.close()


def test_restart_from_snapshot_is_bitwise(tmp_path):
    import torch
    from paper_1908_08557_amd import cmhd, snapshot
    w = W.small_stratified(32, 32, 24, t_ramp=0.06)
    dt = oracle_dt(w)
    print("[case] snapshot restart strat32x32x24", flush=True)
    a = cmhd.solver_for(w)
    x = a.new_state(w.state)
    t = 0.0
    for _ in range(4):
        t, _ = a.rk3_step(x, t, dt)
    ref = x.cpu().numpy()
    b = cmhd.solver_for(w)
    y = b.new_state(w.state)
    t2 = 0.0
    for _ in range(2):
        t2, _ = b.rk3_step(y, t2, dt)
    path = tmp_path / "snap.npz"
    snapshot.save(path, b, y, t2)
    b.close()
    c = cmhd.solver_for(w)
    z, t3 = snapshot.load(path, c)
    assert t3 == t2
    for _ in range(2):
        t3, _ = c.rk3_step(z, t3, dt)
    torch.cuda.synchronize()
    assert t3 == t
    assert np.array_equal(z.cpu().numpy(), ref)
    with np.load(path) as d:
        assert d["lnTT"].shape == (24 + 2 * NG, 32, 32) and float(d["time"]) == t2
    a.close()
    c.close()
