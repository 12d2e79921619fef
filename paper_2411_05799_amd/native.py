"""Thin ctypes binding of libnpx.so (include/npx.h): argument marshalling only.

Every step of the path runs in the HIP library; this module only packs numpy
arrays and torch device pointers into the C ABI. Loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

from . import workloads as W

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnpx.so")

NPX_OK = 0
F_COG, F_QUAT, F_VEL, F_OMEGA, F_JOINT, F_JOINT_PREV, F_STEP, F_FLAGS, F_TELE, F_BODY = range(10)
CTRL_SINUSOID = 0
CTRL_TARGETS = 1
TELE_N = 4


class NpxError(RuntimeError):
    pass


class _MorphTables(C.Structure):
    _fields_ = [("n_points", C.c_int32), ("n_links", C.c_int32),
                ("points", C.POINTER(C.c_float)), ("pt_link", C.POINTER(C.c_int32)),
                ("parent", C.POINTER(C.c_int32)), ("joint", C.POINTER(C.c_float))]


class _WorldDesc(C.Structure):
    _fields_ = [("dt", C.c_double), ("joint_interval", C.c_int32), ("g", C.c_double * 3),
                ("mu", C.c_double), ("k_n", C.c_double), ("zeta", C.c_double),
                ("eps_lsq", C.c_double), ("hf_nx", C.c_int32), ("hf_ny", C.c_int32),
                ("hf_s", C.c_double), ("hf_x0", C.c_double), ("hf_y0", C.c_double),
                ("hf_heights", C.POINTER(C.c_float)), ("n_instances", C.c_int64),
                ("n_morphs", C.c_int32), ("morphs", C.POINTER(_MorphTables)),
                ("instance_morph", C.POINTER(C.c_int32)), ("init_pose", C.POINTER(C.c_float)),
                ("ctrl", C.POINTER(C.c_float)), ("friction_weighting", C.c_int32),
                ("hf_bilinear", C.c_int32), ("max_joint_rate", C.c_double),
                ("friction_6dof", C.c_int32), ("ext_device_buffers", C.c_void_p * 4)]


class Launch(C.Structure):
    _fields_ = [("lanes_per_instance", C.c_int32), ("persistent", C.c_int32),
                ("chunk_steps", C.c_int32), ("use_graph", C.c_int32),
                ("waves_per_cu", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


class SurDesc(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("n_hidden_layers", C.c_int32),
                ("n_out", C.c_int32), ("max_batch", C.c_int32), ("precision", C.c_int32),
                ("training", C.c_int32), ("seed", C.c_uint64)]


SUR_BF16, SUR_FP32 = 0, 1


def lib():
    """The HIP library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NpxError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2411_05799_amd.build`")
        # torch's bundled HIP runtime is asked for as libamdhip64.so, which
        # does not match an already loaded /opt/rocm libamdhip64.so.7; loading
        # torch first makes its runtime the process's only one, which this
        # library then binds to (same soname).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.npx_last_error.restype = C.c_char_p
        L.npx_version.restype = C.c_int
        L.npx_create_world.argtypes = [C.POINTER(_WorldDesc), C.POINTER(vp)]
        L.npx_destroy_world.argtypes = [vp]
        L.npx_destroy_world.restype = None
        L.npx_world_dims.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]
        L.npx_set_controller.argtypes = [vp, C.c_int, vp, C.c_size_t, C.c_int]
        L.npx_step_n.argtypes = [vp, C.c_int64, vp]
        L.npx_step_n_noalloc.argtypes = [vp, C.c_int64, vp]
        L.npx_read_state.argtypes = [vp, C.c_int, vp, C.c_size_t, C.c_int]
        L.npx_write_state.argtypes = [vp, C.c_int, vp, C.c_size_t, C.c_int]
        L.npx_read_points.argtypes = [vp, vp, C.c_size_t, C.c_int]
        L.npx_get_launch.argtypes = [vp, C.POINTER(Launch)]
        L.npx_set_launch.argtypes = [vp, C.POINTER(Launch)]
        L.npx_autotune.argtypes = [vp, C.c_int32, vp, C.POINTER(Launch), C.POINTER(Launch),
                                   C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]
        L.npx_flops_per_step.argtypes = [vp, C.c_int64, C.POINTER(C.c_double)]
        d = C.c_double
        L.npx_morph_last_error.restype = C.c_char_p
        L.npx_morph_new.argtypes = [C.POINTER(vp)]
        L.npx_morph_free.argtypes = [vp]
        L.npx_morph_free.restype = None
        L.npx_simplify_mode.argtypes = [vp, C.c_int]
        L.npx_create_point.argtypes = [vp, d, d, d, d]
        L.npx_create_box.argtypes = [vp, d, d, d, d, d, d, d]
        L.npx_create_box_grid.argtypes = [vp, d, d, d, d, d, d, d, C.c_int, C.c_int]
        L.npx_create_cylinder.argtypes = [vp, d, d, d, d, d, d, d, d, C.c_int]
        L.npx_create_sphere.argtypes = [vp, d, d, d, d, d]
        L.npx_create_ray.argtypes = [vp, d, d, d, d, d, d]
        L.npx_connect_bodies.argtypes = [vp, C.c_int, C.c_int]
        L.npx_create_joint.argtypes = [vp, C.c_int, C.c_int, d, d, d, d, d, d]
        L.npx_set_joint_limits.argtypes = [vp, C.c_int, d, d]
        L.npx_move_body.argtypes = [vp, C.c_int, d, d, d]
        L.npx_rotate_body.argtypes = [vp, C.c_int, d, d, d]
        L.npx_get_max_body_id.argtypes = [vp]
        L.npx_finalize_construction.argtypes = [vp]
        L.npx_morph_get_tables.argtypes = [vp, C.POINTER(_MorphTables)]
        L.npx_morph_joint_index.argtypes = [vp, C.c_int]
        L.npx_morph_get_rays.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.POINTER(C.c_float)),
                                         C.POINTER(C.POINTER(C.c_int32))]
        L.npx_morph_get_rays.restype = C.c_int
        L.npx_world_set_rays.argtypes = [vp, C.c_int32, C.c_int32, vp, vp]
        L.npx_world_set_rays.restype = C.c_int
        L.npx_world_ray_ranges.argtypes = [vp, vp, C.c_int64, vp]
        L.npx_world_ray_ranges.restype = C.c_int
        L.npx_world_set_sensors.argtypes = [vp, C.c_int32, C.c_int32, vp]
        L.npx_world_set_sensors.restype = C.c_int
        L.npx_gp_run.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_float, vp]
        L.npx_gp_run.restype = C.c_int
        for name in ("npx_morph_new", "npx_simplify_mode", "npx_create_point", "npx_create_box",
                     "npx_create_box_grid", "npx_create_cylinder", "npx_create_sphere", "npx_create_ray",
                     "npx_connect_bodies", "npx_create_joint", "npx_set_joint_limits",
                     "npx_move_body", "npx_rotate_body", "npx_get_max_body_id",
                     "npx_finalize_construction", "npx_morph_get_tables", "npx_morph_joint_index"):
            getattr(L, name).restype = C.c_int
        i64, pi64 = C.c_int64, C.POINTER(C.c_int64)
        L.npx_sur_create.argtypes = [C.POINTER(SurDesc), C.POINTER(vp)]
        L.npx_sur_destroy.argtypes = [vp]
        L.npx_sur_destroy.restype = None
        L.npx_sur_param_count.argtypes = [vp, pi64]
        L.npx_sur_get_params.argtypes = [vp, vp, i64, C.c_int]
        L.npx_sur_set_params.argtypes = [vp, vp, i64, C.c_int]
        L.npx_sur_set_norm.argtypes = [vp, vp, vp, vp, vp]
        L.npx_sur_set_adam.argtypes = [vp, d, d, d]
        L.npx_sur_forward.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp]
        L.npx_sur_grad.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp, vp, vp]
        L.npx_sur_train_step.argtypes = [vp, vp, i64, vp, i64, vp, i64, d, vp, vp]
        L.npx_sur_norm_stats.argtypes = [vp, i64, i64, C.c_int32, vp, vp, vp]
        L.npx_sur_set_noise.argtypes = [vp, vp, i64, C.c_int32, C.c_int32]
        L.npx_sur_set_noise.restype = C.c_int
        L.npx_sur_widths.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.npx_world_rows.argtypes = [vp, vp, i64, vp]
        L.npx_world_set_rows.argtypes = [vp, vp, i64, vp]
        L.npx_world_set_rows.restype = C.c_int
        L.npx_sur_features.argtypes = [vp, vp, i64, i64, vp, i64, vp]
        L.npx_sur_delta.argtypes = [vp, vp, i64, vp, i64, vp]
        L.npx_sur_advance.argtypes = [vp, vp, i64, vp, i64, i64, vp]
        L.npx_sur_torque.argtypes = [vp, vp, i64, vp, C.c_int, vp]
        L.npx_sur_rollout.argtypes = [vp, vp, vp, i64, i64, C.c_int32, vp, i64, vp, i64, vp, vp]
        L.npx_sur_screen_select.argtypes = [vp, vp, i64, vp, vp, C.c_int32, C.c_float, vp, i64,
                                            C.c_int32, vp, vp, vp]
        L.npx_sur_screen_select.restype = C.c_int
        for name in ("npx_sur_widths", "npx_world_rows", "npx_sur_features", "npx_sur_delta",
                     "npx_sur_advance", "npx_sur_torque", "npx_sur_rollout"):
            getattr(L, name).restype = C.c_int
        for name in ("npx_sur_create", "npx_sur_param_count", "npx_sur_get_params",
                     "npx_sur_set_params", "npx_sur_set_norm", "npx_sur_set_adam",
                     "npx_sur_forward", "npx_sur_grad", "npx_sur_train_step",
                     "npx_sur_norm_stats"):
            getattr(L, name).restype = C.c_int
        for name in ("npx_create_world", "npx_world_dims", "npx_set_controller", "npx_step_n",
                     "npx_read_state", "npx_write_state", "npx_read_points", "npx_get_launch",
                     "npx_set_launch", "npx_autotune", "npx_flops_per_step"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(rc):
    if rc != NPX_OK:
        raise NpxError(f"npx error {rc}: {lib().npx_last_error().decode()}")


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def j_max_of(morphs):
    return max(1, max(m.n_links for m in morphs) - 1)


def pack_ctrl(ctrl_list, j_max):
    """Per-instance [J_i, 3] controllers -> [I][J_max][3] float32."""
    out = np.zeros((len(ctrl_list), j_max, 3), dtype=np.float32)
    for i, c in enumerate(ctrl_list):
        out[i, : c.shape[0]] = c
    return out


class World:
    """A world on the current HIP device (npx_create_world ... npx_destroy_world)."""

    def __init__(self, w: W.Workload, ext=None):
        """ext: optional [state, step, flags, tele] torch device tensors (None
        entries allowed) that hold the world's state in place of its own
        buffers (npx_world_desc.ext_device_buffers): float32 with
        (13 + 2 J_max) x I elements, int32 with I, int32 with I and float64
        with 4 x I, contiguous; kept referenced for the world's life."""
        self.workload = w
        self._keep = []
        self._ext = None
        morphs = (_MorphTables * len(w.morphs))()
        for i, m in enumerate(w.morphs):
            arrs = (_f32(m.points), _i32(m.pt_link), _i32(m.parent), _f32(m.joint))
            self._keep.append(arrs)
            morphs[i] = _MorphTables(m.n_points, m.n_links,
                                     arrs[0].ctypes.data_as(C.POINTER(C.c_float)),
                                     arrs[1].ctypes.data_as(C.POINTER(C.c_int32)),
                                     arrs[2].ctypes.data_as(C.POINTER(C.c_int32)),
                                     arrs[3].ctypes.data_as(C.POINTER(C.c_float)))
        self.j_max_expected = j_max_of(w.morphs)
        H = _f32(w.hf.H)
        im = _i32(w.inst_morph)
        pose = _f32(w.pose)
        ctrl = pack_ctrl(w.ctrl, self.j_max_expected)
        self._keep += [morphs, H, im, pose, ctrl]
        p = w.params
        desc = _WorldDesc(float(p.dt), int(p.K), (C.c_double * 3)(*map(float, p.g)), float(p.mu),
                          float(p.k_n), float(p.zeta), float(p.eps), int(w.hf.nx), int(w.hf.ny),
                          float(w.hf.s), float(w.hf.x0), float(w.hf.y0),
                          H.ctypes.data_as(C.POINTER(C.c_float)), int(w.n_instances),
                          len(w.morphs), morphs, im.ctypes.data_as(C.POINTER(C.c_int32)),
                          pose.ctypes.data_as(C.POINTER(C.c_float)),
                          ctrl.ctypes.data_as(C.POINTER(C.c_float)),
                          int(getattr(p, "friction_weighting", 0)),
                          int(getattr(p, "hf_bilinear", 0)),
                          float(getattr(p, "max_joint_rate", 0.0)),
                          int(getattr(p, "friction_6dof", 0)))
        if ext is not None:
            I = int(w.n_instances)
            want = [("float32", (13 + 2 * self.j_max_expected) * I), ("int32", I),
                    ("int32", I), ("float64", 4 * I)]
            ext = list(ext) + [None] * (4 - len(ext))
            for k, (t, (dt, n)) in enumerate(zip(ext[:4], want)):
                if t is None:
                    continue
                if (str(t.dtype) != "torch." + dt or t.numel() != n or not t.is_contiguous()
                        or t.device.type != "cuda"):
                    raise ValueError(f"ext[{k}]: need a contiguous {dt} device tensor of {n} "
                                     f"elements")
                desc.ext_device_buffers[k] = t.data_ptr()
            self._ext = ext[:4]
        h = C.c_void_p()
        check(lib().npx_create_world(C.byref(desc), C.byref(h)))
        self.h = h
        self._keep = None
        n, j, nm = C.c_int64(), C.c_int32(), C.c_int32()
        check(lib().npx_world_dims(self.h, C.byref(n), C.byref(j), C.byref(nm)))
        self.n_instances, self.j_max, self.n_max = int(n.value), int(j.value), int(nm.value)
        assert self.j_max == self.j_max_expected

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            lib().npx_destroy_world(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls ------------------------------------------------------------------
    def set_controller(self, ctrl):
        """ctrl: list of per-instance [J_i, 3] arrays, an [I, J_max, 3] array or a
        torch device tensor of that shape."""
        if hasattr(ctrl, "data_ptr"):
            check(lib().npx_set_controller(self.h, CTRL_SINUSOID, C.c_void_p(ctrl.data_ptr()),
                                           ctrl.numel(), 1))
            return
        arr = pack_ctrl(ctrl, self.j_max) if isinstance(ctrl, list) else _f32(ctrl)
        check(lib().npx_set_controller(self.h, CTRL_SINUSOID, arr.ctypes.data_as(C.c_void_p),
                                       arr.size, 0))

    def set_targets(self, targets):
        """Joint target angles [I, J_max] (numpy or a torch device tensor),
        commanded from the next joint update on."""
        if hasattr(targets, "data_ptr"):
            if not targets.is_contiguous():
                raise ValueError("targets must be contiguous")
            check(lib().npx_set_controller(self.h, CTRL_TARGETS, C.c_void_p(targets.data_ptr()),
                                           targets.numel(), 1))
            return
        arr = _f32(targets)
        check(lib().npx_set_controller(self.h, CTRL_TARGETS, arr.ctypes.data_as(C.c_void_p),
                                       arr.size, 0))

    def step_n(self, n, stream=None):
        """Advance n frames asynchronously on `stream` (a torch.cuda.Stream or raw handle)."""
        s = _stream_handle(stream)
        check(lib().npx_step_n(self.h, int(n), C.c_void_p(s)))

    def step_n_noalloc(self, n, stream=None):
        """npx_step_n without any allocation (direct launches, static counters)."""
        s = _stream_handle(stream)
        check(lib().npx_step_n_noalloc(self.h, int(n), C.c_void_p(s)))

    def _field_shape(self, field):
        I = self.n_instances
        return {F_COG: ((3, I), np.float32), F_QUAT: ((4, I), np.float32),
                F_VEL: ((3, I), np.float32), F_OMEGA: ((3, I), np.float32),
                F_JOINT: ((self.j_max, I), np.float32), F_JOINT_PREV: ((self.j_max, I), np.float32),
                F_STEP: ((I,), np.int32), F_FLAGS: ((I,), np.int32),
                F_TELE: ((TELE_N, I), np.float64), F_BODY: ((13, I), np.float32)}[field]

    def read_state(self, field, out=None):
        """Field as a numpy array (or into a torch device tensor `out`)."""
        shape, dt = self._field_shape(field)
        if out is not None and hasattr(out, "data_ptr"):
            check(lib().npx_read_state(self.h, field, C.c_void_p(out.data_ptr()),
                                       out.numel() * out.element_size(), 1))
            return out
        a = np.empty(shape, dtype=dt)
        check(lib().npx_read_state(self.h, field, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))
        return a

    def write_state(self, field, value):
        shape, dt = self._field_shape(field)
        if hasattr(value, "data_ptr"):
            check(lib().npx_write_state(self.h, field, C.c_void_p(value.data_ptr()),
                                        value.numel() * value.element_size(), 1))
            return
        a = np.ascontiguousarray(value, dtype=dt).reshape(shape)
        check(lib().npx_write_state(self.h, field, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))

    def read_points(self):
        a = np.empty((self.n_instances, self.n_max, 3), dtype=np.float32)
        check(lib().npx_read_points(self.h, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))
        return a

    def get_launch(self) -> Launch:
        l = Launch()
        check(lib().npx_get_launch(self.h, C.byref(l)))
        return l

    def set_launch(self, **kw):
        l = self.get_launch()
        for k, v in kw.items():
            setattr(l, k, int(v))
        check(lib().npx_set_launch(self.h, C.byref(l)))
        return l

    def autotune(self, steps=50, stream=None, cache=None, key=None):
        """Pick the fastest launch shape; with `cache` (a JSON path) and `key`,
        reuse an earlier choice for the same workload key."""
        if cache and key and os.path.exists(cache):
            try:
                with open(cache) as f:
                    known = json.load(f)
                if key in known:
                    self.set_launch(**known[key]["best"])
                    return known[key]
            except (OSError, ValueError):
                pass
        best = Launch()
        tried = (Launch * 32)()
        times = (C.c_float * 32)()
        n = C.c_int32()
        check(lib().npx_autotune(self.h, int(steps), C.c_void_p(_stream_handle(stream)),
                                 C.byref(best), tried, times, 32, C.byref(n)))
        rec = {"best": best.as_dict(),
               "tried": [dict(tried[i].as_dict(), ms=float(times[i])) for i in range(n.value)]}
        if cache and key:
            known = {}
            if os.path.exists(cache):
                try:
                    with open(cache) as f:
                        known = json.load(f)
                except (OSError, ValueError):
                    known = {}
            known[key] = rec
            with open(cache, "w") as f:
                json.dump(known, f, indent=1, sort_keys=True)
        return rec

    # -- the simulator side of the surrogate (device tensors) --------------------
    def sur_widths(self):
        a, b = C.c_int32(), C.c_int32()
        check(lib().npx_sur_widths(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_rays(self, morph, rays, ray_link):
        """Range-sensor rays of morphology `morph`: rays [n, 6] (start, end in its
        construction frame), ray_link [n] (the link each rides on)."""
        r = np.ascontiguousarray(rays, dtype=np.float32).reshape(-1, 6)
        k = np.ascontiguousarray(ray_link, dtype=np.int32).reshape(-1)
        if r.shape[0] != k.shape[0]:
            raise ValueError("rays and ray_link differ in length")
        check(lib().npx_world_set_rays(self.h, int(morph), int(k.shape[0]),
                                       r.ctypes.data_as(C.c_void_p), k.ctypes.data_as(C.c_void_p)))
        self._ray_max = max(getattr(self, "_ray_max", 0), int(k.shape[0]))

    def ray_ranges(self, out, stream=None):
        """Range of every ray at the current state into a device float32 tensor
        [I, >= the largest ray count] (asynchronous on `stream`)."""
        check(lib().npx_world_ray_ranges(self.h, _ptr(out), out.stride(0),
                                         C.c_void_p(_stream_handle(stream))))
        return out

    def set_sensors(self, morph, links):
        """Foot contact sensors of morphology `morph`: the link of each."""
        k = np.ascontiguousarray(links, dtype=np.int32).reshape(-1)
        check(lib().npx_world_set_sensors(self.h, int(morph), int(k.shape[0]),
                                          k.ctypes.data_as(C.c_void_p)))

    def gp_run(self, programs, vm, targets, n_updates, n_instr, motor_step, stream=None):
        """Machine-code programs (device uint8 [I, 32]) driving the robots for
        n_updates joint updates; vm (int32 [I, 2]) and targets (float32 [I, >= J_max])
        are device tensors carried between calls."""
        check(lib().npx_gp_run(self.h, _ptr(programs), _ptr(vm), _ptr(targets), targets.stride(0),
                               int(n_updates), int(n_instr), float(motor_step),
                               C.c_void_p(_stream_handle(stream))))

    def rows(self, out, stream=None):
        """State rows [I, >= 13 + 2 J] of every instance into a device tensor."""
        check(lib().npx_world_rows(self.h, _ptr(out), out.stride(0),
                                   C.c_void_p(_stream_handle(stream))))
        return out

    def set_rows(self, s, stream=None):
        """Every instance's state from the rows of a device tensor."""
        check(lib().npx_world_set_rows(self.h, _ptr(s), s.stride(0),
                                       C.c_void_p(_stream_handle(stream))))

    def sur_features(self, x, s=None, frame=-1, stream=None):
        """Network inputs into x [I, >= width]: from rows s at `frame`, or from
        the world's own state (s None)."""
        check(lib().npx_sur_features(self.h, _ptr(s), 0 if s is None else s.stride(0), int(frame),
                                     _ptr(x), x.stride(0), C.c_void_p(_stream_handle(stream))))
        return x

    def sur_delta(self, s0, y, stream=None):
        check(lib().npx_sur_delta(self.h, _ptr(s0), s0.stride(0), _ptr(y), y.stride(0),
                                  C.c_void_p(_stream_handle(stream))))
        return y

    def sur_advance(self, s, dy, frame, stream=None):
        check(lib().npx_sur_advance(self.h, _ptr(s), s.stride(0), _ptr(dy), dy.stride(0),
                                    int(frame), C.c_void_p(_stream_handle(stream))))
        return s

    def sur_torque(self, acc, s=None, accumulate=False, stream=None):
        check(lib().npx_sur_torque(self.h, _ptr(s), 0 if s is None else s.stride(0), _ptr(acc),
                                   1 if accumulate else 0, C.c_void_p(_stream_handle(stream))))
        return acc

    def sur_rollout(self, net, s, frame0, n_calls, x_work, y_work, tau_acc=None, stream=None):
        check(lib().npx_sur_rollout(net.h, self.h, _ptr(s), s.stride(0), int(frame0),
                                    int(n_calls), _ptr(x_work), x_work.stride(0), _ptr(y_work),
                                    y_work.stride(0), _ptr(tau_acc),
                                    C.c_void_p(_stream_handle(stream))))
        return s

    def flops_per_step(self, i=None):
        """Algorithmic FP32 operations of one frame (instance i, or summed over all)."""
        idx = range(self.n_instances) if i is None else [i]
        tot = 0.0
        d = C.c_double()
        for k in idx:
            check(lib().npx_flops_per_step(self.h, int(k), C.byref(d)))
            tot += d.value
        return tot


class MorphBuilder:
    """The paper's construction API (npx_morph_*): bodies of mass points, glued
    into links, joined by hinges, finalised into morphology tables."""

    def __init__(self):
        h = C.c_void_p()
        self._call(lib().npx_morph_new(C.byref(h)))
        self.h = h

    @staticmethod
    def _call(rc):
        if rc < 0:
            raise NpxError(f"npx error {rc}: {lib().npx_morph_last_error().decode()}")
        return rc

    def simplify_mode(self, mode):
        return self._call(lib().npx_simplify_mode(self.h, int(mode)))

    def create_point(self, x, y, z, m):
        return self._call(lib().npx_create_point(self.h, x, y, z, m))

    def create_box(self, w, h, d, x, y, z, m, grid_nx=0, grid_ny=0):
        if grid_nx or grid_ny:
            return self._call(lib().npx_create_box_grid(self.h, w, h, d, x, y, z, m,
                                                        int(grid_nx), int(grid_ny)))
        return self._call(lib().npx_create_box(self.h, w, h, d, x, y, z, m))

    def create_cylinder(self, x1, y1, z1, x2, y2, z2, rr, m, ring_pts=8):
        return self._call(lib().npx_create_cylinder(self.h, x1, y1, z1, x2, y2, z2, rr, m,
                                                    int(ring_pts)))

    def create_sphere(self, x, y, z, rr, m):
        return self._call(lib().npx_create_sphere(self.h, x, y, z, rr, m))

    def create_ray(self, x1, y1, z1, x2, y2, z2):
        return self._call(lib().npx_create_ray(self.h, x1, y1, z1, x2, y2, z2))

    def connect_bodies(self, id1, id2):
        return self._call(lib().npx_connect_bodies(self.h, int(id1), int(id2)))

    def create_joint(self, id1, id2, anchor, axis):
        return self._call(lib().npx_create_joint(self.h, int(id1), int(id2), *map(float, anchor),
                                                 *map(float, axis)))

    def set_joint_limits(self, joint, lo, hi):
        return self._call(lib().npx_set_joint_limits(self.h, int(joint), lo, hi))

    def move_body(self, id_, tx, ty, tz):
        return self._call(lib().npx_move_body(self.h, int(id_), tx, ty, tz))

    def rotate_body(self, id_, alpha, beta, gamma):
        return self._call(lib().npx_rotate_body(self.h, int(id_), alpha, beta, gamma))

    def get_max_body_id(self):
        return self._call(lib().npx_get_max_body_id(self.h))

    def finalize_construction(self):
        return self._call(lib().npx_finalize_construction(self.h))

    def joint_index(self, joint_id):
        return self._call(lib().npx_morph_joint_index(self.h, int(joint_id)))

    def tables(self, name="built"):
        """The finalised robot as a workloads.Morph (copies of the tables)."""
        t = _MorphTables()
        self._call(lib().npx_morph_get_tables(self.h, C.byref(t)))
        n, l = t.n_points, t.n_links
        pts = np.ctypeslib.as_array(t.points, shape=(n * 4,)).reshape(n, 4).copy()
        return W.Morph(points=pts, pt_link=np.ctypeslib.as_array(t.pt_link, shape=(n,)).copy(),
                       parent=np.ctypeslib.as_array(t.parent, shape=(l,)).copy(),
                       joint=np.ctypeslib.as_array(t.joint, shape=(l * 8,)).reshape(l, 8).copy(),
                       name=name)

    def rays(self):
        """The finalised robot's range-sensor rays: ([n, 6] start and end in the
        construction frame, [n] link of each)."""
        n = C.c_int32()
        r = C.POINTER(C.c_float)()
        k = C.POINTER(C.c_int32)()
        self._call(lib().npx_morph_get_rays(self.h, C.byref(n), C.byref(r), C.byref(k)))
        if n.value == 0:
            return np.zeros((0, 6), np.float32), np.zeros(0, np.int32)
        return (np.ctypeslib.as_array(r, shape=(n.value * 6,)).reshape(-1, 6).copy(),
                np.ctypeslib.as_array(k, shape=(n.value,)).copy())

    def close(self):
        if getattr(self, "h", None):
            lib().npx_morph_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return C.c_void_p(0 if t is None else t.data_ptr())


class Surrogate:
    """The surrogate network (npx_sur_create ... npx_sur_destroy).  Device
    buffers are torch tensors on the current HIP device: x [rows, >= n_in]
    float32, y [rows, >= n_out] float32, rows int32."""

    def __init__(self, n_in, n_hidden, n_hidden_layers, n_out, max_batch, precision=SUR_BF16,
                 training=True, seed=0):
        d = SurDesc(n_in, n_hidden, n_hidden_layers, n_out, max_batch, precision,
                    1 if training else 0, seed)
        h = C.c_void_p()
        check(lib().npx_sur_create(C.byref(d), C.byref(h)))
        self.h = h
        self.n_in, self.n_out, self.max_batch = n_in, n_out, max_batch
        self.shapes = [(n_hidden, n_in)] + [(n_hidden, n_hidden)] * (n_hidden_layers - 1) + \
                      [(n_out, n_hidden)]

    def close(self):
        if getattr(self, "h", None):
            lib().npx_sur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def param_count(self):
        n = C.c_int64()
        check(lib().npx_sur_param_count(self.h, C.byref(n)))
        return n.value

    def get_params(self):
        a = np.empty(self.param_count(), dtype=np.float32)
        check(lib().npx_sur_get_params(self.h, a.ctypes.data_as(C.c_void_p), a.size, 0))
        return a

    def set_params(self, p):
        if hasattr(p, "data_ptr"):
            check(lib().npx_sur_set_params(self.h, _ptr(p), p.numel(), 1))
            return
        a = _f32(p)
        check(lib().npx_sur_set_params(self.h, a.ctypes.data_as(C.c_void_p), a.size, 0))

    def set_norm(self, x_mean, x_std, y_mean, y_std):
        a = [_f32(v) for v in (x_mean, x_std, y_mean, y_std)]
        check(lib().npx_sur_set_norm(self.h, *[v.ctypes.data_as(C.c_void_p) for v in a]))

    def set_adam(self, beta1=0.9, beta2=0.999, eps=1e-8):
        check(lib().npx_sur_set_adam(self.h, beta1, beta2, eps))

    def set_noise(self, noise=None, col0=0):
        """Training noise [batch, ncols] added to inputs col0.. and taken off the
        same target columns (None: off). Keep the tensor alive while set."""
        self._noise = noise
        if noise is None:
            check(lib().npx_sur_set_noise(self.h, None, 0, 0, 0))
        else:
            check(lib().npx_sur_set_noise(self.h, _ptr(noise), noise.stride(0), col0, noise.shape[1]))

    def forward(self, x, out, rows=None, batch=None, stream=None):
        b = x.shape[0] if rows is None else rows.shape[0]
        b = b if batch is None else batch
        check(lib().npx_sur_forward(self.h, _ptr(x), x.stride(0), _ptr(rows), b, _ptr(out),
                                    out.stride(0), C.c_void_p(_stream_handle(stream))))
        return out

    def grad(self, x, y, loss=None, grad=None, rows=None, batch=None, stream=None):
        b = x.shape[0] if rows is None else rows.shape[0]
        b = b if batch is None else batch
        check(lib().npx_sur_grad(self.h, _ptr(x), x.stride(0), _ptr(y), y.stride(0), _ptr(rows),
                                 b, _ptr(loss), _ptr(grad), C.c_void_p(_stream_handle(stream))))

    def train_step(self, x, y, lr, loss=None, rows=None, batch=None, stream=None):
        b = x.shape[0] if rows is None else rows.shape[0]
        b = b if batch is None else batch
        check(lib().npx_sur_train_step(self.h, _ptr(x), x.stride(0), _ptr(y), y.stride(0),
                                       _ptr(rows), b, float(lr), _ptr(loss),
                                       C.c_void_p(_stream_handle(stream))))


def screen_select(s0, s1, heading, tau, n_calls, torque_weight, flags=None, n_top=0,
                  stream=None):
    """Fitness of every candidate and the indices of the n_top best
    (npx_sur_screen_select): s0, s1 [n, >= 2] state rows (CoG x, y first),
    heading [n, 2], tau [n] summed torque proxy, flags [n] int32 or None; all
    device tensors. Returns (fitness [n] float32, top [n_top] int32) tensors."""
    import torch
    n = s0.shape[0]
    if s1.stride(0) != s0.stride(0) or s0.stride(1) != 1 or s1.stride(1) != 1:
        raise ValueError("s0 and s1 need the same row stride and contiguous rows")
    fit = torch.empty(n, dtype=torch.float32, device=s0.device)
    top = torch.empty(max(1, n_top), dtype=torch.int32, device=s0.device)
    heading = heading.contiguous()
    tau = tau.contiguous()
    check(lib().npx_sur_screen_select(_ptr(s0), _ptr(s1), s0.stride(0), _ptr(heading), _ptr(tau),
                                      int(n_calls), float(torque_weight), _ptr(flags), n,
                                      int(n_top), _ptr(fit), _ptr(top),
                                      C.c_void_p(_stream_handle(stream))))
    return fit, top[:n_top]


def norm_stats(x, cols=None, stream=None):
    """Column means and standard deviations of a device matrix (torch tensors out)."""
    import torch
    cols = x.shape[1] if cols is None else cols
    mean = torch.empty(cols, dtype=torch.float32, device=x.device)
    std = torch.empty(cols, dtype=torch.float32, device=x.device)
    check(lib().npx_sur_norm_stats(_ptr(x), x.stride(0), x.shape[0], cols, _ptr(mean), _ptr(std),
                                   C.c_void_p(_stream_handle(stream))))
    return mean, std


def exported_symbols():
    """Names of every function declared in include/npx.h."""
    import re
    hdr = os.path.join(os.path.dirname(PKG), "include", "npx.h")
    txt = re.sub(r"/\*.*?\*/", "", open(hdr).read(), flags=re.S)
    txt = re.sub(r"//[^\n]*", "", txt)
    return sorted(set(re.findall(r"\b(npx_[a-z_0-9]+)\s*\(", txt)))
