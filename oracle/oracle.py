"""ctypes binding of the FP64 oracle (npx_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from types import SimpleNamespace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnpx_oracle.so")
SRC = os.path.join(HERE, "npx_oracle.c")

# state-vector offsets (mirror of the enum in npx_oracle.h)
C_, Q_, V_, W_, STEP, FLAGS, TELE, HDR = 0, 3, 7, 10, 13, 14, 15, 19
D_FN, D_TAU, D_NC, D_NS, D_A, D_LAMBDA, D_FF, D_A6, D_LEN = 0, 1, 4, 5, 6, 9, 10, 11, 17
# fragile decisions (mirror of the enums in npx_oracle.h)
FR_S1, FR_S5, FR_FIT, FR_S9 = 0, 1, 2, 3
FK_EDGE_X, FK_EDGE_Y, FK_CONTACT, FK_SPREAD, FK_CAP = 0, 1, 2, 3, 4
STAGE_NAMES = {FR_S1: "S1 detection at P^n", FR_S5: "S5 detection at P*", FR_FIT: "fit",
               FR_S9: "S9 torso look-up"}
KIND_NAMES = {FK_EDGE_X: "cell edge x", FK_EDGE_Y: "cell edge y", FK_CONTACT: "contact sign",
              FK_SPREAD: "spread test", FK_CAP: "static-friction cap"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, -O2, no fast-math, contraction off, OpenMP."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
                           SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Morph(C.Structure):
    _fields_ = [("n_points", C.c_int), ("n_links", C.c_int),
                ("points", C.POINTER(C.c_float)), ("pt_link", C.POINTER(C.c_int)),
                ("parent", C.POINTER(C.c_int)), ("joint", C.POINTER(C.c_float))]


class _Fragile(C.Structure):
    _fields_ = [("stage", C.c_int), ("point", C.c_int), ("kind", C.c_int), ("dist", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("K", C.c_int), ("g", C.c_double * 3), ("mu", C.c_double),
                ("k_n", C.c_double), ("zeta", C.c_double), ("eps", C.c_double),
                ("weighted", C.c_int), ("hf_bilinear", C.c_int), ("hf_nx", C.c_int), ("hf_ny", C.c_int), ("hf_s", C.c_double),
                ("hf_x0", C.c_double), ("hf_y0", C.c_double), ("hf", C.POINTER(C.c_float)),
                ("max_rate", C.c_double), ("six_dof", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        fp = C.POINTER(C.c_float)
        L.orc_fk.argtypes = [C.POINTER(_Morph), dp, dp, dp, dp, dp]
        L.orc_cell.argtypes = [C.POINTER(_Params), C.c_double, C.c_double,
                               C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_height.argtypes = [C.POINTER(_Params), C.c_double, C.c_double]
        L.orc_height.restype = C.c_double
        L.orc_ray_range.argtypes = [C.POINTER(_Params), dp, dp]
        L.orc_ray_range.restype = C.c_double
        L.orc_lsq.argtypes = [C.c_int, dp, dp, C.c_double, dp]
        L.orc_lsq_w.argtypes = [C.c_int, dp, dp, dp, C.c_double, dp]
        L.orc_lsq6_w.argtypes = [C.c_int, dp, dp, dp, C.c_double, dp]
        L.orc_sym3_min_eig.argtypes = [dp]
        L.orc_sym3_min_eig.restype = C.c_double
        L.orc_init_state.argtypes = [C.POINTER(_Morph), C.POINTER(_Params), fp, fp, dp]
        L.orc_points.argtypes = [C.POINTER(_Morph), dp, dp]
        L.orc_step.argtypes = [C.POINTER(_Morph), C.POINTER(_Params), fp, dp, dp]
        L.orc_step_ex.argtypes = [C.POINTER(_Morph), C.POINTER(_Params), fp, dp, dp, dp,
                                  C.POINTER(_Fragile), C.c_int, C.POINTER(C.c_int),
                                  C.POINTER(_Fragile), C.c_int]
        L.orc_run.argtypes = [C.POINTER(_Morph), C.POINTER(_Params), fp, dp, C.c_long]
        L.orc_run_batch.argtypes = [C.c_int, C.POINTER(_Morph), C.POINTER(C.c_int),
                                    C.POINTER(_Params), C.POINTER(fp), C.POINTER(dp),
                                    C.c_long, C.c_int]
        _lib = L
    return _lib


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


class OracleMorph:
    def __init__(self, m):
        self.points = np.ascontiguousarray(m.points, dtype=np.float32)
        self.pt_link = np.ascontiguousarray(m.pt_link, dtype=np.int32)
        self.parent = np.ascontiguousarray(m.parent, dtype=np.int32)
        self.joint = np.ascontiguousarray(m.joint, dtype=np.float32)
        self.n_points = int(self.points.shape[0])
        self.n_links = int(self.parent.shape[0])
        self.n_joints = self.n_links - 1
        self.c = _Morph(self.n_points, self.n_links, _fptr(self.points), _iptr(self.pt_link),
                        _iptr(self.parent), _fptr(self.joint))

    def fk(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        y = np.zeros((self.n_points, 3))
        g = np.zeros(3)
        I = np.zeros((3, 3))
        M = np.zeros(1)
        lib().orc_fk(C.byref(self.c), _dptr(q), _dptr(y), _dptr(g), _dptr(I), _dptr(M))
        return y, g, I, float(M[0])


class OracleParams:
    def __init__(self, params, hf):
        self.H = np.ascontiguousarray(hf.H, dtype=np.float32)
        g = (C.c_double * 3)(*[float(x) for x in params.g])
        self.c = _Params(float(params.dt), int(params.K), g, float(params.mu), float(params.k_n),
                         float(params.zeta), float(params.eps),
                         int(getattr(params, "friction_weighting", False)),
                         int(getattr(params, "hf_bilinear", False)), int(hf.nx), int(hf.ny),
                         float(hf.s), float(hf.x0), float(hf.y0), _fptr(self.H),
                         float(getattr(params, "max_joint_rate", 0.0)),
                         int(getattr(params, "friction_6dof", False)))

    def cell(self, x, y):
        i, j = C.c_int(), C.c_int()
        lib().orc_cell(C.byref(self.c), float(x), float(y), C.byref(i), C.byref(j))
        return i.value, j.value

    def height(self, x, y):
        return lib().orc_height(C.byref(self.c), float(x), float(y))

    def ray_range(self, A, B):
        """Distance from A to the first ground point of the segment A -> B
        (look-up-table ground), or |B - A|."""
        a = (C.c_double * 3)(*[float(v) for v in A])
        b = (C.c_double * 3)(*[float(v) for v in B])
        return lib().orc_ray_range(C.byref(self.c), a, b)


def lsq(src, dst, eps=1e-4, weights=None):
    """Friction fit (eqs. 4-6) of the pairs src -> dst; weights: the
    per-pair weights of the force-weighted variant (None: unweighted)."""
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 2)
    dst = np.ascontiguousarray(dst, dtype=np.float64).reshape(-1, 2)
    a = np.zeros(3)
    if weights is None:
        k = lib().orc_lsq(int(src.shape[0]), _dptr(src), _dptr(dst), float(eps), _dptr(a))
    else:
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
        assert w.shape[0] == src.shape[0]
        k = lib().orc_lsq_w(int(src.shape[0]), _dptr(src), _dptr(dst), _dptr(w), float(eps),
                            _dptr(a))
    return a, k


def lsq6(src, dst, eps=1e-4, weights=None):
    """Six-degree-of-freedom friction fit of the 3-D pairs src -> dst (about
    the coordinates' origin): (displacement (3), rotation vector (3)) and the
    branch taken (6 full, 3 yaw only, 2 displacement only, 0 none)."""
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    dst = np.ascontiguousarray(dst, dtype=np.float64).reshape(-1, 3)
    a = np.zeros(6)
    w = None
    if weights is not None:
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
        assert w.shape[0] == src.shape[0]
    k = lib().orc_lsq6_w(int(src.shape[0]), _dptr(src), _dptr(dst),
                         _dptr(w) if w is not None else None, float(eps), _dptr(a))
    assert k >= 0
    return a, k


def sym3_min_eig(A):
    """Smallest eigenvalue of a symmetric 3x3 matrix (the oracle's closed form)."""
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
    return lib().orc_sym3_min_eig(_dptr(A))


class OracleWorld:
    """A workload on the oracle: one float64 state vector per instance."""

    def __init__(self, w):
        self.w = w
        self.morphs = [OracleMorph(m) for m in w.morphs]
        self.params = OracleParams(w.params, w.hf)
        self.ctrl = [np.ascontiguousarray(c, dtype=np.float32) for c in w.ctrl]
        self.inst_morph = np.ascontiguousarray(w.inst_morph, dtype=np.int32)
        self._cmorphs = (_Morph * len(self.morphs))(*[m.c for m in self.morphs])

    def morph_of(self, i):
        return self.morphs[int(self.inst_morph[i])]

    def init_state(self, i):
        m = self.morph_of(i)
        st = np.zeros(HDR + 2 * m.n_joints)
        pose = np.ascontiguousarray(self.w.pose[i], dtype=np.float32)
        rc = lib().orc_init_state(C.byref(m.c), C.byref(self.params.c), _fptr(self.ctrl[i]),
                                  _fptr(pose), _dptr(st))
        assert rc == 0, "invalid morphology"
        return st

    def init_states(self):
        return [self.init_state(i) for i in range(self.w.n_instances)]

    def step(self, i, st, diag=False):
        m = self.morph_of(i)
        d = np.zeros(D_LEN) if diag else None
        rc = lib().orc_step(C.byref(m.c), C.byref(self.params.c), _fptr(self.ctrl[i]), _dptr(st),
                            _dptr(d) if diag else None)
        assert rc == 0
        return d

    def step_ex(self, i, st, margin_m=0.0, margin_rel=0.0, flips=(), diag=False, log_cap=256,
                margin_cap=None):
        """One step of instance i that logs its fragile decisions (look-ups
        within margin_m of a cell edge that could change a contact, contact
        tests with |depth| < margin_m, the fit's spread test within margin_rel
        and its static-friction comparison within margin_cap (default
        margin_rel) of their thresholds) and takes the decisions in `flips` the
        other way. Returns the log as (stage, point, kind, distance) tuples
        (and the diagnostics if diag)."""
        m = self.morph_of(i)
        d = np.zeros(D_LEN) if diag else None
        log = (_Fragile * log_cap)()
        n_log = C.c_int(0)
        fl = (_Fragile * max(1, len(flips)))()
        for k, f in enumerate(flips):
            fl[k] = _Fragile(int(f[0]), int(f[1]), int(f[2]), 0.0)
        margins = np.array([margin_m, margin_rel,
                            margin_rel if margin_cap is None else margin_cap], np.float64)
        rc = lib().orc_step_ex(C.byref(m.c), C.byref(self.params.c), _fptr(self.ctrl[i]),
                               _dptr(st), _dptr(d) if diag else None, _dptr(margins), log,
                               int(log_cap), C.byref(n_log), fl, len(flips))
        assert rc == 0
        out = [(log[k].stage, log[k].point, log[k].kind, log[k].dist)
               for k in range(min(n_log.value, log_cap))]
        return (out, d) if diag else out

    def run(self, i, st, n_steps):
        m = self.morph_of(i)
        rc = lib().orc_run(C.byref(m.c), C.byref(self.params.c), _fptr(self.ctrl[i]), _dptr(st),
                           int(n_steps))
        assert rc == 0

    def run_batch(self, states, n_steps, idx=None, threads=0):
        """Advance states[k] (instance idx[k]) by n_steps on `threads` host threads."""
        idx = np.arange(len(states)) if idx is None else np.asarray(idx)
        n = len(states)
        im = np.ascontiguousarray(self.inst_morph[idx], dtype=np.int32)
        fp = C.POINTER(C.c_float)
        dp = C.POINTER(C.c_double)
        cptr = (fp * n)(*[_fptr(self.ctrl[int(i)]) for i in idx])
        sptr = (dp * n)(*[_dptr(s) for s in states])
        used = lib().orc_run_batch(n, self._cmorphs, _iptr(im), C.byref(self.params.c), cptr,
                                   sptr, int(n_steps), int(threads))
        assert used > 0, "parameters the step does not take"
        return used

    def ray_ends(self, i, st, rays, ray_link):
        """World start and end [n, 3] of rays riding on instance i's links at
        state st: each end is a massless point of its link, moved like the mass
        points (the robot's CoG and inertia are unchanged)."""
        m = self.morph_of(i)
        r = np.asarray(rays, dtype=np.float32).reshape(-1, 6)
        k = np.asarray(ray_link, dtype=np.int32).reshape(-1)
        n = r.shape[0]
        z = np.zeros((n, 1), np.float32)
        aug = SimpleNamespace(points=np.concatenate([m.points, np.hstack([r[:, :3], z]),
                                                     np.hstack([r[:, 3:], z])]),
                              pt_link=np.concatenate([m.pt_link, k, k]),
                              parent=m.parent, joint=m.joint)
        am = OracleMorph(aug)
        P = np.zeros((am.n_points, 3))
        lib().orc_points(C.byref(am.c), _dptr(np.ascontiguousarray(st)), _dptr(P))
        return P[m.n_points:m.n_points + n], P[m.n_points + n:]

    def points(self, i, st):
        m = self.morph_of(i)
        P = np.zeros((m.n_points, 3))
        lib().orc_points(C.byref(m.c), _dptr(np.ascontiguousarray(st)), _dptr(P))
        return P
