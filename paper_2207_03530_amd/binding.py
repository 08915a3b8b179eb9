"""Thin ctypes binding of the C boundary (include/vmas.h).

Argument marshalling only: every step of the physics runs in the HIP
kernels of libvmas.so. PyTorch supplies device memory (tensors) and the
stream (torch's current stream). If the library is missing this module
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# VMAS_LIB selects another build of the same sources (the host-sanitizer
# build of `python -m paper_2207_03530_amd.build --sanitize`)
LIB_PATH = os.environ.get("VMAS_LIB") or os.path.join(HERE, "libvmas.so")

VMAS_OK = 0
STATUS = {0: "VMAS_OK", 1: "VMAS_ERR_INVALID_ARGUMENT", 2: "VMAS_ERR_OUT_OF_MEMORY",
          3: "VMAS_ERR_DEVICE", 4: "VMAS_ERR_UNSUPPORTED", 5: "VMAS_ERR_NONFINITE"}

# Every symbol include/vmas.h declares.
EXPORTS = ("vmas_create_batch", "vmas_destroy_batch", "vmas_batch_get_info", "vmas_step",
           "vmas_rollout", "vmas_step_backward", "vmas_rollout_backward", "vmas_set_schedule",
           "vmas_autotune", "vmas_schedule_name", "vmas_rollout_graph", "vmas_last_error",
           "vmas_mlp_num_params", "vmas_mlp_create", "vmas_mlp_destroy", "vmas_mlp_get_params",
           "vmas_mlp_forward", "vmas_mlp_backward", "vmas_mlp_train_step", "vmas_pair_features",
           "vmas_step_surrogate", "vmas_nonfinite_envs", "vmas_rollout_backward_noalloc")

VMAS_DEBUG_NONFINITE = 1


class VmasError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_f32p = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class WorldParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("drag", ctypes.c_float),
                ("gravity", ctypes.c_float * 2), ("contact_force", ctypes.c_float),
                ("contact_margin", ctypes.c_float), ("min_dist", ctypes.c_float),
                ("joint_stiffness", ctypes.c_float), ("flags", ctypes.c_uint32)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("env_offset", _i32p), ("n_per_env", ctypes.c_int32),
                ("n_agents", _i32p), ("shape", _u8p), ("dims", _f32p), ("mass", _f32p),
                ("inertia", _f32p), ("max_speed", _f32p), ("flags", _u8p),
                ("n_joints", ctypes.c_int32), ("joint_a", _i32p), ("joint_b", _i32p),
                ("joint_anchor_a", _f32p), ("joint_anchor_b", _f32p), ("joint_rest", _f32p),
                ("joint_collide", _u8p), ("init_state", _f32p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("n_entities", ctypes.c_int32),
                ("n_agents", ctypes.c_int32), ("n_joints", ctypes.c_int32),
                ("n_pair_slots", ctypes.c_int64), ("schedule", ctypes.c_int32),
                ("n_schedules", ctypes.c_int32), ("max_env_size", ctypes.c_int32),
                ("tune_cached", ctypes.c_int32)]


_lib = None


def lib():
    """Load libvmas.so (built by paper_2207_03530_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2207_03530_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.vmas_create_batch.argtypes = [ctypes.POINTER(WorldParams), ctypes.POINTER(BatchDesc),
                                    ctypes.c_int, ctypes.POINTER(vp)]
    L.vmas_destroy_batch.argtypes = [vp]
    L.vmas_batch_get_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    L.vmas_step.argtypes = [vp, vp, vp, vp, vp, vp]
    L.vmas_rollout.argtypes = [vp, vp, vp, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, vp,
                               vp, vp]
    L.vmas_rollout_graph.argtypes = L.vmas_rollout.argtypes
    L.vmas_step_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.vmas_rollout_backward.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                                        vp]
    L.vmas_rollout_backward_noalloc.argtypes = L.vmas_rollout_backward.argtypes
    L.vmas_set_schedule.argtypes = [vp, ctypes.c_int32]
    L.vmas_autotune.argtypes = [vp, vp, vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int32)]
    L.vmas_schedule_name.argtypes = [vp, ctypes.c_int32]
    L.vmas_schedule_name.restype = ctypes.c_char_p
    L.vmas_last_error.restype = ctypes.c_char_p
    L.vmas_mlp_num_params.argtypes = []
    L.vmas_mlp_create.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(vp)]
    L.vmas_mlp_destroy.argtypes = [vp]
    L.vmas_mlp_get_params.argtypes = [vp, vp, vp]
    L.vmas_mlp_forward.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    L.vmas_mlp_backward.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp, vp]
    L.vmas_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_float, vp, vp]
    L.vmas_pair_features.argtypes = [vp, vp, ctypes.c_float, vp, ctypes.c_int64, vp, vp, vp, vp]
    L.vmas_step_surrogate.argtypes = [vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, vp, vp, vp]
    L.vmas_nonfinite_envs.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
    for name in EXPORTS:
        if name not in ("vmas_schedule_name", "vmas_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int) -> None:
    if status != VMAS_OK:
        raise VmasError(status, lib().vmas_last_error().decode())


def _np_ptr(a: Optional[np.ndarray], t):
    return ctypes.cast(None, t) if a is None else a.ctypes.data_as(t)


def _dptr(t, numel: Optional[int] = None, dtype=None, name: str = "tensor"):
    """Device pointer of a contiguous CUDA/HIP tensor (or None)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_params(w, flags: int = 0) -> WorldParams:
    p = WorldParams()
    p.dt = w.dt
    p.drag = w.drag
    p.gravity[0], p.gravity[1] = float(w.gravity[0]), float(w.gravity[1])
    p.contact_force = w.contact_force
    p.contact_margin = w.contact_margin
    p.min_dist = w.min_dist
    p.joint_stiffness = w.joint_stiffness
    p.flags = flags
    return p


class Batch:
    """A batch of environments on one device (handle of vmas_create_batch).
    debug_nonfinite sets VMAS_DEBUG_NONFINITE in the world flags."""

    def __init__(self, world, device: int = 0, debug_nonfinite: bool = False):
        import torch
        self.world = world
        self.device = torch.device("cuda", device)
        self._keep = []
        d = BatchDesc()
        arr = lambda a, dt: None if a is None else np.ascontiguousarray(a, dt)  # noqa: E731
        env_offset = arr(world.env_offset, np.int32)
        n_agents = arr(world.n_agents, np.int32)
        shape = arr(world.shape, np.uint8)
        dims = arr(world.dims, np.float32)
        mass = arr(world.mass, np.float32)
        inertia = arr(world.inertia, np.float32)
        vmax = arr(world.max_speed, np.float32)
        flags = arr(world.flags, np.uint8)
        self._keep += [env_offset, n_agents, shape, dims, mass, inertia, vmax, flags]
        d.n_envs = world.n_envs
        d.env_offset = _np_ptr(env_offset, _i32p)
        d.n_per_env = 0
        d.n_agents = _np_ptr(n_agents, _i32p)
        d.shape = _np_ptr(shape, _u8p)
        d.dims = _np_ptr(dims, _f32p)
        d.mass = _np_ptr(mass, _f32p)
        d.inertia = _np_ptr(inertia, _f32p)
        d.max_speed = _np_ptr(vmax, _f32p)
        d.flags = _np_ptr(flags, _u8p)
        d.n_joints = world.n_joints
        if world.n_joints:
            ja, jb = arr(world.joint_a, np.int32), arr(world.joint_b, np.int32)
            aa, ab = arr(world.anchor_a, np.float32), arr(world.anchor_b, np.float32)
            rest = arr(world.joint_rest, np.float32)
            jc = arr(world.joint_collide, np.uint8)
            self._keep += [ja, jb, aa, ab, rest, jc]
            d.joint_a, d.joint_b = _np_ptr(ja, _i32p), _np_ptr(jb, _i32p)
            d.joint_anchor_a, d.joint_anchor_b = _np_ptr(aa, _f32p), _np_ptr(ab, _f32p)
            d.joint_rest = _np_ptr(rest, _f32p)
            d.joint_collide = _np_ptr(jc, _u8p)
        st0 = arr(world.state0, np.float32)
        self._keep.append(st0)
        d.init_state = _np_ptr(st0, _f32p)
        self.params = make_params(world, VMAS_DEBUG_NONFINITE if debug_nonfinite else 0)
        h = ctypes.c_void_p()
        _check(lib().vmas_create_batch(ctypes.byref(self.params), ctypes.byref(d), device,
                                       ctypes.byref(h)))
        self.handle = h
        self._keep = []
        info = BatchInfo()
        _check(lib().vmas_batch_get_info(self.handle, ctypes.byref(info)))
        self.N, self.A = info.n_entities, info.n_agents
        self.P, self.J = info.n_pair_slots, info.n_joints
        self.n_schedules = info.n_schedules

    # ---------------------------------------------------------------- info --
    def info(self) -> BatchInfo:
        info = BatchInfo()
        _check(lib().vmas_batch_get_info(self.handle, ctypes.byref(info)))
        return info

    def schedule_name(self, q: int) -> str:
        return lib().vmas_schedule_name(self.handle, q).decode()

    def set_schedule(self, q: int) -> None:
        _check(lib().vmas_set_schedule(self.handle, q))

    def autotune(self, state, T: int = 10, actions=None) -> int:
        """Times every plan on a T-step rollout (actions [T][A][2] on the
        device, or drawn in the kernel) and makes the fastest current."""
        import torch
        out = ctypes.c_int32(-1)
        _check(lib().vmas_autotune(self.handle, _dptr(state, 6 * self.N, torch.float32, "state"),
                                   _dptr(actions, T * 2 * self.A, torch.float32, "actions"), T,
                                   _stream(self.device), ctypes.byref(out)))
        return out.value

    # ---------------------------------------------------------------- calls --
    def state_tensor(self, state: Optional[np.ndarray] = None):
        import torch
        s = self.world.state0 if state is None else state
        return torch.as_tensor(np.ascontiguousarray(s, np.float32)).to(self.device)

    def step(self, state, actions, mask=None, forces=None) -> None:
        import torch
        _check(lib().vmas_step(self.handle, _dptr(state, 6 * self.N, torch.float32, "state"),
                               _dptr(actions, 2 * self.A, torch.float32, "actions"),
                               _dptr(mask, self.P, torch.uint8, "mask"),
                               _dptr(forces, 3 * self.N, torch.float32, "forces"),
                               _stream(self.device)))

    def rollout(self, state, actions=None, T: Optional[int] = None, seed: int = 0, t0: int = 0,
                traj=None, final_mask=None, graph: bool = False) -> None:
        import torch
        if actions is not None:
            T = actions.shape[0] if T is None else T
            _dptr(actions, T * 2 * self.A, torch.float32, "actions")
        if T is None:
            raise ValueError("T is required when actions are drawn in the kernel")
        fn = lib().vmas_rollout_graph if graph else lib().vmas_rollout
        _check(fn(self.handle, _dptr(state, 6 * self.N, torch.float32, "state"),
                  _dptr(actions, None, torch.float32, "actions"), ctypes.c_uint64(seed), t0, T,
                  _dptr(traj, (T + 1) * 6 * self.N, torch.float32, "traj"),
                  _dptr(final_mask, self.P, torch.uint8, "final_mask"), _stream(self.device)))

    def step_backward(self, state_t, actions_t, grad_next, grad_state, grad_actions=None) -> None:
        import torch
        f = torch.float32
        _check(lib().vmas_step_backward(
            self.handle, _dptr(state_t, 6 * self.N, f, "state_t"),
            _dptr(actions_t, 2 * self.A, f, "actions_t"),
            _dptr(grad_next, 6 * self.N, f, "grad_state_next"),
            _dptr(grad_state, 6 * self.N, f, "grad_state_t"),
            _dptr(grad_actions, 2 * self.A, f, "grad_actions_t"), _stream(self.device)))

    def prepare_rollout(self, state, actions=None, T: Optional[int] = None, seed: int = 0,
                        t0: int = 0, graph: bool = False):
        """A zero-argument callable that runs vmas_rollout (or
        vmas_rollout_graph) on the given tensors and the current stream.
        The arguments are checked and marshalled here, once; each call is one
        C call, for tight loops where per-call Python work would leave the
        GPU waiting. The tensors must stay alive while the callable is used."""
        import torch
        if actions is not None:
            T = actions.shape[0] if T is None else T
            _dptr(actions, T * 2 * self.A, torch.float32, "actions")
        if T is None:
            raise ValueError("T is required when actions are drawn in the kernel")
        fn = lib().vmas_rollout_graph if graph else lib().vmas_rollout
        args = (self.handle, _dptr(state, 6 * self.N, torch.float32, "state"),
                _dptr(actions, None, torch.float32, "actions"), ctypes.c_uint64(seed),
                ctypes.c_int32(t0), ctypes.c_int32(T), None, None, _stream(self.device))
        keep = (state, actions, self)  # the callable keeps its tensors and handle alive

        def run():
            st = fn(*args)
            if st != VMAS_OK:
                _check(st)
        run.keep = keep
        return run

    def rollout_backward(self, state0, actions, grad_final, ckpt_every: int = 10,
                         grad_state0=None, grad_actions=None, noalloc: bool = False) -> None:
        """vmas_rollout_backward, or vmas_rollout_backward_noalloc (workspace
        in the library's fixed device scratch) when noalloc is set."""
        import torch
        f = torch.float32
        T = actions.shape[0]
        fn = lib().vmas_rollout_backward_noalloc if noalloc else lib().vmas_rollout_backward
        _check(fn(
            self.handle, _dptr(state0, 6 * self.N, f, "state0"),
            _dptr(actions, T * 2 * self.A, f, "actions"), T, ckpt_every,
            _dptr(grad_final, 6 * self.N, f, "grad_state_T"),
            _dptr(grad_state0, 6 * self.N, f, "grad_state0"),
            _dptr(grad_actions, T * 2 * self.A, f, "grad_actions"), _stream(self.device)))

    def pair_features(self, state, features, flags, targets=None, slots=None, band: float = 0.05):
        import torch
        m = self.P if slots is None else slots.shape[0]
        _check(lib().vmas_pair_features(
            self.handle, _dptr(state, 6 * self.N, torch.float32, "state"), ctypes.c_float(band),
            _dptr(slots, m, torch.int64, "slots"), m,
            _dptr(features, 12 * m, torch.float32, "features"),
            _dptr(targets, 2 * m, torch.float32, "targets"),
            _dptr(flags, m, torch.uint8, "flags"), _stream(self.device)))

    def step_surrogate(self, mlp: "Mlp", state, actions, band: float = 0.05,
                       fallback_frac: float = 0.5, forces=None, n_fallback=None) -> None:
        import torch
        _check(lib().vmas_step_surrogate(
            self.handle, mlp.handle, _dptr(state, 6 * self.N, torch.float32, "state"),
            _dptr(actions, 2 * self.A, torch.float32, "actions"), ctypes.c_float(band),
            ctypes.c_float(fallback_frac), _dptr(forces, 3 * self.N, torch.float32, "forces"),
            _dptr(n_fallback, 1, torch.int32, "n_fallback"), _stream(self.device)))

    def nonfinite_envs(self, clear: bool = False):
        """(marks uint8 [n_envs], count) of the environments that have held a
        non-finite state (VMAS_DEBUG_NONFINITE batches)."""
        marks = np.zeros(self.world.n_envs, np.uint8)
        cnt = ctypes.c_int32(0)
        _check(lib().vmas_nonfinite_envs(self.handle, marks.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(cnt), int(clear), _stream(self.device)))
        return marks, cnt.value

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().vmas_destroy_batch(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The contact-surrogate network (handle of vmas_mlp_create)."""

    def __init__(self, params: Optional[np.ndarray] = None, seed: int = 0, device: int = 0):
        import torch
        self.device = torch.device("cuda", device)
        self.n_params = lib().vmas_mlp_num_params()
        p = None
        if params is not None:
            p = np.ascontiguousarray(params, np.float32)
            if p.size != self.n_params:
                raise ValueError(f"params must have {self.n_params} values")
        h = ctypes.c_void_p()
        _check(lib().vmas_mlp_create(None if p is None else p.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.c_uint64(seed), device, ctypes.byref(h)))
        self.handle = h

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        _check(lib().vmas_mlp_get_params(self.handle, out.ctypes.data_as(ctypes.c_void_p),
                                         _stream(self.device)))
        return out

    def forward(self, X, Y) -> None:
        import torch
        n = X.shape[0]
        _check(lib().vmas_mlp_forward(self.handle, _dptr(X, 12 * n, torch.float32, "X"), n,
                                      _dptr(Y, 2 * n, torch.float32, "Y"), _stream(self.device)))

    def backward(self, X, dY, grad=None, dX=None) -> None:
        import torch
        n = X.shape[0]
        _check(lib().vmas_mlp_backward(self.handle, _dptr(X, 12 * n, torch.float32, "X"), n,
                                       _dptr(dY, 2 * n, torch.float32, "dY"),
                                       _dptr(grad, self.n_params, torch.float32, "grad"),
                                       _dptr(dX, 12 * n, torch.float32, "dX"), _stream(self.device)))

    def train_step(self, X, target, lr: float, loss=None) -> None:
        import torch
        n = X.shape[0]
        _check(lib().vmas_mlp_train_step(self.handle, _dptr(X, 12 * n, torch.float32, "X"),
                                         _dptr(target, 2 * n, torch.float32, "target"), n,
                                         ctypes.c_float(lr), _dptr(loss, 1, torch.float32, "loss"),
                                         _stream(self.device)))

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().vmas_mlp_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- the C entry points under their own names (same arguments, Python objects) --

def vmas_create_batch(world, device: int = 0) -> Batch:
    return Batch(world, device)


def vmas_destroy_batch(batch: Batch) -> None:
    batch.close()


def vmas_step(batch: Batch, state, actions, mask=None, forces=None) -> None:
    batch.step(state, actions, mask, forces)


def vmas_rollout(batch: Batch, state, actions=None, seed: int = 0, t0: int = 0, T=None,
                 traj=None, final_mask=None) -> None:
    batch.rollout(state, actions, T=T, seed=seed, t0=t0, traj=traj, final_mask=final_mask)


def vmas_rollout_graph(batch: Batch, state, actions=None, seed: int = 0, t0: int = 0, T=None) -> None:
    batch.rollout(state, actions, T=T, seed=seed, t0=t0, graph=True)


def vmas_step_backward(batch: Batch, state_t, actions_t, grad_state_next, grad_state_t,
                       grad_actions_t=None) -> None:
    batch.step_backward(state_t, actions_t, grad_state_next, grad_state_t, grad_actions_t)


def vmas_rollout_backward(batch: Batch, state0, actions, grad_state_T, ckpt_every: int = 10,
                          grad_state0=None, grad_actions=None) -> None:
    batch.rollout_backward(state0, actions, grad_state_T, ckpt_every, grad_state0, grad_actions)


def vmas_rollout_backward_noalloc(batch: Batch, state0, actions, grad_state_T,
                                  ckpt_every: int = 10, grad_state0=None,
                                  grad_actions=None) -> None:
    batch.rollout_backward(state0, actions, grad_state_T, ckpt_every, grad_state0, grad_actions,
                           noalloc=True)


def vmas_autotune(batch: Batch, state, T: int = 10, actions=None) -> int:
    return batch.autotune(state, T, actions)


def vmas_set_schedule(batch: Batch, schedule: int) -> None:
    batch.set_schedule(schedule)


def vmas_nonfinite_envs(batch: Batch, clear: bool = False):
    return batch.nonfinite_envs(clear)
