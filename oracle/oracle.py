"""ctypes front end of the FP64 CPU oracle (oracle/vmas_oracle.cpp).

TEST INFRASTRUCTURE: imported only by tests/, the smoke check and the CPU
baseline leg of bench.py; the product path never loads it.

Inputs are the seeded arrays of paper_2207_03530_amd.workloads (FP32
values), widened to FP64 here; every computation happens in the C++ oracle
(plus the joint rest length, computed below from the initial state by the
same joint definition).
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# VMAS_ORACLE_LIB selects another build of the same source (the sanitizer
# build of oracle/build.py --sanitize)
LIB_PATH = os.environ.get("VMAS_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f64p = ctypes.POINTER(ctypes.c_double)


class _World(ctypes.Structure):
    _fields_ = [
        ("n_envs", ctypes.c_int32),
        ("env_offset", _i32p),
        ("n_agents", _i32p),
        ("shape", _u8p),
        ("dims", _f64p),
        ("mass", _f64p),
        ("inertia", _f64p),
        ("max_speed", _f64p),
        ("flags", _u8p),
        ("n_joints", ctypes.c_int32),
        ("joint_a", _i32p),
        ("joint_b", _i32p),
        ("anchor_a", _f64p),
        ("anchor_b", _f64p),
        ("rest", _f64p),
        ("joint_collide", _u8p),
        ("dt", ctypes.c_double),
        ("drag", ctypes.c_double),
        ("gx", ctypes.c_double),
        ("gy", ctypes.c_double),
        ("c", ctypes.c_double),
        ("k", ctypes.c_double),
        ("min_dist", ctypes.c_double),
        ("joint_k", ctypes.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            import importlib.util
            spec = importlib.util.spec_from_file_location("_oracle_build",
                                                          os.path.join(HERE, "build.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            mod.build()
        L = ctypes.CDLL(LIB_PATH)
        wp = ctypes.POINTER(_World)
        L.oracle_step.argtypes = [wp, _f64p, _f64p, _u8p, _f64p]
        L.oracle_rollout.argtypes = [wp, _f64p, _f64p, ctypes.c_int, _f64p, _u8p]
        L.oracle_rollout_range.argtypes = [wp, ctypes.c_int, ctypes.c_int, _f64p, _f64p,
                                           ctypes.c_int, _f64p, _u8p]
        L.oracle_rollout_jvp.argtypes = [wp, _f64p, _f64p, _f64p, _f64p, ctypes.c_int]
        _f32p = ctypes.POINTER(ctypes.c_float)
        L.oracle_rollout_fp32.argtypes = [wp, _f32p, _f32p, ctypes.c_int, _f32p]
        L.oracle_joint_lengths_fp32.argtypes = [wp, _f32p, _f64p]
        L.oracle_pair.argtypes = [ctypes.c_int, _f64p, _f64p, ctypes.c_int, _f64p, _f64p, _f64p]
        L.oracle_pair_distances.argtypes = [wp, _f64p, _f64p, _f64p]
        L.oracle_default_inertia.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double]
        L.oracle_default_inertia.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray], t):
    if a is None:
        return ctypes.cast(None, t)
    return a.ctypes.data_as(t)


class OracleWorld:
    """FP64 copy of a workloads.World, ready for the C oracle."""

    def __init__(self, w, c: Optional[float] = None, k: Optional[float] = None):
        self.w = w
        self.N = w.n_entities
        self.A = w.n_agents_total
        self.env_offset = np.ascontiguousarray(w.env_offset, np.int32)
        self.n_agents = np.ascontiguousarray(w.n_agents, np.int32)
        self.shape = np.ascontiguousarray(w.shape, np.uint8)
        self.dims = np.ascontiguousarray(w.dims, np.float64)
        self.mass = np.ascontiguousarray(w.mass, np.float64)
        self.inertia = None if w.inertia is None else np.ascontiguousarray(w.inertia, np.float64)
        self.max_speed = None if w.max_speed is None else np.ascontiguousarray(w.max_speed,
                                                                                np.float64)
        self.flags = np.ascontiguousarray(w.flags, np.uint8)
        J = w.n_joints
        if J:
            self.joint_a = np.ascontiguousarray(w.joint_a, np.int32)
            self.joint_b = np.ascontiguousarray(w.joint_b, np.int32)
            self.anchor_a = np.ascontiguousarray(w.anchor_a, np.float64)
            self.anchor_b = np.ascontiguousarray(w.anchor_b, np.float64)
            self.rest = np.ascontiguousarray(w.joint_rest, np.float64).copy()
            self.joint_collide = (None if w.joint_collide is None
                                  else np.ascontiguousarray(w.joint_collide, np.uint8))
            self._fill_rest(w.state0.astype(np.float64))
        else:
            self.joint_a = self.joint_b = None
            self.anchor_a = self.anchor_b = self.rest = None
            self.joint_collide = None
        s = _World()
        s.n_envs = w.n_envs
        s.env_offset = _p(self.env_offset, _i32p)
        s.n_agents = _p(self.n_agents, _i32p)
        s.shape = _p(self.shape, _u8p)
        s.dims = _p(self.dims, _f64p)
        s.mass = _p(self.mass, _f64p)
        s.inertia = _p(self.inertia, _f64p)
        s.max_speed = _p(self.max_speed, _f64p)
        s.flags = _p(self.flags, _u8p)
        s.n_joints = J
        s.joint_a = _p(self.joint_a, _i32p)
        s.joint_b = _p(self.joint_b, _i32p)
        s.anchor_a = _p(self.anchor_a, _f64p)
        s.anchor_b = _p(self.anchor_b, _f64p)
        s.rest = _p(self.rest, _f64p)
        s.joint_collide = _p(self.joint_collide, _u8p)
        s.dt = w.dt
        s.drag = w.drag
        s.gx, s.gy = float(w.gravity[0]), float(w.gravity[1])
        s.c = w.contact_force if c is None else c
        s.k = w.contact_margin if k is None else k
        s.min_dist = w.min_dist
        s.joint_k = w.joint_stiffness
        self.s = s

    def _fill_rest(self, st: np.ndarray) -> None:
        """Rest length < 0 means: the anchor distance in the initial state."""
        for q in range(self.joint_a.shape[0]):
            if self.rest[q] >= 0:
                continue
            P = []
            for e, anc in ((self.joint_a[q], self.anchor_a[q]), (self.joint_b[q], self.anchor_b[q])):
                th = st[4, e]
                c, s = np.cos(th), np.sin(th)
                P.append((st[0, e] + c * anc[0] - s * anc[1], st[1, e] + s * anc[0] + c * anc[1]))
            self.rest[q] = float(np.hypot(P[0][0] - P[1][0], P[0][1] - P[1][1]))

    # -- calls --------------------------------------------------------------
    def step(self, state: np.ndarray, actions: np.ndarray, want_mask=True, want_forces=False):
        st = np.ascontiguousarray(state, np.float64).copy()
        act = np.ascontiguousarray(actions, np.float64)
        mask = np.zeros(self.w.pair_slots(), np.uint8) if want_mask else None
        forces = np.zeros((3, self.N), np.float64) if want_forces else None
        lib().oracle_step(ctypes.byref(self.s), _p(st, _f64p), _p(act, _f64p), _p(mask, _u8p),
                          _p(forces, _f64p))
        return st, mask, forces

    def rollout(self, state: np.ndarray, actions: np.ndarray, traj: bool = False,
                want_mask: bool = True, env_range=None):
        T = actions.shape[0]
        st = np.ascontiguousarray(state, np.float64).copy()
        act = np.ascontiguousarray(actions, np.float64)
        tr = np.zeros((T + 1, 6, self.N), np.float64) if traj else None
        mask = np.zeros(self.w.pair_slots(), np.uint8) if want_mask else None
        e0, e1 = (0, self.w.n_envs) if env_range is None else env_range
        lib().oracle_rollout_range(ctypes.byref(self.s), e0, e1, _p(st, _f64p), _p(act, _f64p),
                                   T, _p(tr, _f64p), _p(mask, _u8p))
        return st, mask, tr

    def _world_fp32(self):
        """The world as the FP32 evaluation sees it: a rest length taken from
        the initial state is that state's anchor distance evaluated in FP32
        (each side computes it in its own arithmetic, as the joints reading
        of Sec. 3 in this project has it), so such a spring starts exactly at
        rest there too."""
        if getattr(self, "_s32", None) is None:
            self._s32 = self.s
            if self.rest is not None and np.any(np.asarray(self.w.joint_rest) < 0):
                f32 = ctypes.POINTER(ctypes.c_float)
                st0 = np.ascontiguousarray(self.w.state0, np.float32)
                lens = np.zeros(self.rest.shape[0], np.float64)
                lib().oracle_joint_lengths_fp32(ctypes.byref(self.s), st0.ctypes.data_as(f32),
                                                _p(lens, _f64p))
                self._rest32 = np.where(np.asarray(self.w.joint_rest) < 0, lens, self.rest)
                self._s32 = _World.from_buffer_copy(self.s)
                self._s32.rest = _p(self._rest32, _f64p)
        return self._s32

    def rollout_fp32(self, state: np.ndarray, actions: np.ndarray, traj: bool = False):
        """The same definition evaluated in FP32 (not a reference: it sizes the
        FP32 rounding allowance of the parity tests). Returns (final state,
        trajectory [T+1, 6, N] or None), float32."""
        f32 = ctypes.POINTER(ctypes.c_float)
        T = actions.shape[0]
        st = np.ascontiguousarray(state, np.float32).copy()
        act = np.ascontiguousarray(actions, np.float32)
        tr = np.zeros((T + 1, 6, self.N), np.float32) if traj else None
        lib().oracle_rollout_fp32(ctypes.byref(self._world_fp32()), st.ctypes.data_as(f32),
                                  act.ctypes.data_as(f32), T,
                                  None if tr is None else tr.ctypes.data_as(f32))
        return st, tr

    def rollout_jvp(self, state, dstate, actions, dactions):
        T = actions.shape[0]
        st = np.ascontiguousarray(state, np.float64).copy()
        dst = np.ascontiguousarray(dstate, np.float64).copy()
        act = np.ascontiguousarray(actions, np.float64)
        dact = None if dactions is None else np.ascontiguousarray(dactions, np.float64)
        lib().oracle_rollout_jvp(ctypes.byref(self.s), _p(st, _f64p), _p(dst, _f64p),
                                 _p(act, _f64p), _p(dact, _f64p), T)
        return st, dst


def pair_distances(ow: "OracleWorld", state: np.ndarray):
    """(d, d_min) per pair slot from the FP64 narrow phase (NaN: not eligible)."""
    st = np.ascontiguousarray(state, np.float64)
    P = ow.w.pair_slots()
    d = np.zeros(P, np.float64)
    dm = np.zeros(P, np.float64)
    lib().oracle_pair_distances(ctypes.byref(ow.s), _p(st, _f64p), _p(d, _f64p), _p(dm, _f64p))
    return d, dm


def rollout_threaded(ow: OracleWorld, state: np.ndarray, actions: np.ndarray, threads: int):
    """Run the unchanged single-threaded oracle on disjoint environment ranges
    from several Python threads (ctypes releases the GIL). Returns the final
    state."""
    st = np.ascontiguousarray(state, np.float64).copy()
    act = np.ascontiguousarray(actions, np.float64)
    T = actions.shape[0]
    E = ow.w.n_envs
    bounds = np.linspace(0, E, threads + 1).astype(int)
    L = lib()

    def run(e0, e1):
        L.oracle_rollout_range(ctypes.byref(ow.s), int(e0), int(e1), _p(st, _f64p),
                               _p(act, _f64p), T, None, None)

    ths = [threading.Thread(target=run, args=(bounds[q], bounds[q + 1])) for q in range(threads)
           if bounds[q + 1] > bounds[q]]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    return st


def pair(si, di, pose_i, sj, dj, pose_j):
    """Narrow phase of one ordered pair: (d, n[2], p_i[2], p_j[2])."""
    out = np.zeros(7, np.float64)
    di = np.asarray(di, np.float64)
    dj = np.asarray(dj, np.float64)
    pi = np.asarray(pose_i, np.float64)
    pj = np.asarray(pose_j, np.float64)
    lib().oracle_pair(int(si), _p(di, _f64p), _p(pi, _f64p), int(sj), _p(dj, _f64p),
                      _p(pj, _f64p), _p(out, _f64p))
    return out[0], out[1:3].copy(), out[3:5].copy(), out[5:7].copy()


def default_inertia(shape: int, m: float, d0: float, d1: float = 0.0) -> float:
    return lib().oracle_default_inertia(int(shape), float(m), float(d0), float(d1))
