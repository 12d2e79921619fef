"""The C-ABI library: it loads, exports every symbol include/npx.h declares, and
rejects bad arguments on the host before touching a device. No compute calls."""
import ctypes as C
import os
import subprocess

import pytest

from paper_2411_05799_amd import native as N

pytestmark = pytest.mark.skipif(not os.path.exists(N.LIB_PATH),
                                reason="libnpx.so not built (run __graft_entry__.build())")


def test_every_declared_symbol_is_exported():
    names = N.exported_symbols()
    assert "npx_create_world" in names and "npx_step_n" in names
    assert "npx_read_state" in names and "npx_set_controller" in names
    lib = C.CDLL(N.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True,
                         text=True).stdout
    for n in names:
        assert f" T {n}" in out, n


def test_host_side_argument_checks():
    L = N.lib()
    h = C.c_void_p()
    assert L.npx_create_world(None, C.byref(h)) == -1
    assert b"null" in L.npx_last_error()
    assert L.npx_step_n(None, 10, None) == -1
    assert L.npx_read_state(None, 0, None, 0, 0) == -1
    assert L.npx_set_controller(None, 0, None, 0, 0) == -1
    L.npx_destroy_world(None)  # NULL-safe
    assert L.npx_version() == 1


def test_bad_tables_rejected_before_device_use():
    from paper_2411_05799_amd import workloads as W
    import numpy as np
    w = W.config1()
    m = w.morphs[0]
    bad = W.Morph(points=m.points, pt_link=m.pt_link, parent=m.parent.copy(), joint=m.joint)
    bad.parent[3] = 7   # parent must precede the link
    w2 = W.Workload(params=w.params, hf=w.hf, morphs=[bad], inst_morph=w.inst_morph,
                    ctrl=w.ctrl, pose=w.pose)
    with pytest.raises(N.NpxError, match="parent"):
        N.World(w2)
    w3 = W.Workload(params=W.Params(K=0), hf=w.hf, morphs=w.morphs, inst_morph=w.inst_morph,
                    ctrl=w.ctrl, pose=w.pose)
    with pytest.raises(N.NpxError, match="K"):
        N.World(w3)
    w4 = W.Workload(params=w.params, hf=w.hf, morphs=w.morphs,
                    inst_morph=np.array([5], np.int32), ctrl=w.ctrl, pose=w.pose)
    with pytest.raises(N.NpxError, match="instance_morph"):
        N.World(w4)
    w5 = W.Workload(params=W.Params(friction_weighting=2), hf=w.hf, morphs=w.morphs,
                    inst_morph=w.inst_morph, ctrl=w.ctrl, pose=w.pose)
    with pytest.raises(N.NpxError, match="friction_weighting"):
        N.World(w5)
    w6 = W.Workload(params=W.Params(hf_bilinear=3), hf=w.hf, morphs=w.morphs,
                    inst_morph=w.inst_morph, ctrl=w.ctrl, pose=w.pose)
    with pytest.raises(N.NpxError, match="hf_bilinear"):
        N.World(w6)
    w6b = W.Workload(params=W.Params(friction_6dof=2), hf=w.hf, morphs=w.morphs,
                     inst_morph=w.inst_morph, ctrl=w.ctrl, pose=w.pose)
    with pytest.raises(N.NpxError, match="friction_6dof"):
        N.World(w6b)
    w6c = W.Workload(params=W.Params(friction_6dof=True, friction_weighting=True), hf=w.hf,
                     morphs=w.morphs, inst_morph=w.inst_morph, ctrl=w.ctrl, pose=w.pose)
    with pytest.raises(N.NpxError, match="friction_6dof with friction_weighting"):
        N.World(w6c)
    for rate in (-1.0, float("nan")):
        w7 = W.Workload(params=W.Params(max_joint_rate=rate), hf=w.hf, morphs=w.morphs,
                        inst_morph=w.inst_morph, ctrl=w.ctrl, pose=w.pose)
        with pytest.raises(N.NpxError, match="max_joint_rate"):
            N.World(w7)


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(N, "_lib", None)
    monkeypatch.setattr(N, "LIB_PATH", N.LIB_PATH + ".absent")
    with pytest.raises(N.NpxError, match="missing"):
        N.lib()
