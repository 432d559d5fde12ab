"""Python binding of the braxmi C ABI (argument marshalling only).

Device memory and streams come from PyTorch (ROCm); every step of the
physics runs in the HIP library ``libbraxmi.so`` built next to this file.
There is no fallback: if the library is missing or no GPU is present, the
calls raise.

State tensors follow the library layout (environment index fastest):
``pos [3][Bmax][E]``, ``rot [4][Bmax][E]`` (w, x, y, z), ``vel [3][Bmax][E]``,
``ang [3][Bmax][E]``; actions ``[Amax][E]``, action sequences ``[T][Amax][E]``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbraxmi.so")

BRAX_PLAIN, BRAX_FUSED, BRAX_GRAPH, BRAX_NONFINITE_FLAGS = 1, 2, 4, 8
MAX_TYPES = 8

ERRORS = {-1: "BRAX_E_ARG", -2: "BRAX_E_PARSE", -3: "BRAX_E_MODEL", -4: "BRAX_E_DEVICE", -5: "BRAX_E_NOMEM",
          -6: "BRAX_E_UNSUPPORTED"}


class BraxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _State(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("rot", C.c_void_p), ("vel", C.c_void_p), ("ang", C.c_void_p)]


class _EnvParams(C.Structure):
    _fields_ = [("root", C.c_int32), ("forward_weight", C.c_float), ("healthy_reward", C.c_float),
                ("ctrl_cost", C.c_float), ("z_min", C.c_float), ("z_max", C.c_float)]


class _Layout(C.Structure):
    _fields_ = [("n_envs", C.c_int32), ("n_types", C.c_int32), ("b_max", C.c_int32), ("a_max", C.c_int32),
                ("d_max", C.c_int32),
                ("type_envs", C.c_int32 * MAX_TYPES), ("n_bodies", C.c_int32 * MAX_TYPES),
                ("n_joints", C.c_int32 * MAX_TYPES), ("n_actions", C.c_int32 * MAX_TYPES),
                ("n_dof", C.c_int32 * MAX_TYPES), ("n_contacts", C.c_int32 * MAX_TYPES),
                ("substeps", C.c_int32 * MAX_TYPES), ("dt", C.c_float * MAX_TYPES),
                ("device", C.c_int32), ("nonfinite", C.c_void_p), ("tape_step_floats", C.c_int64),
                ("n_params", C.c_int32 * MAX_TYPES), ("p_max", C.c_int32),
                ("n_pairs", C.c_int32 * MAX_TYPES),
                ("vjp_lds_bytes", C.c_int64), ("vjp_params_lds_bytes", C.c_int64), ("lds_limit", C.c_int64),
                ("lanes_per_env", C.c_int32 * MAX_TYPES)]


EXPORTS = ("brax_sys_create", "brax_sys_destroy", "brax_sys_query", "brax_default_angles", "brax_default_qp",
           "brax_step", "brax_step_vjp", "brax_step_vjp_params", "brax_rollout", "brax_rollout_tape",
           "brax_step_vjp_tape", "brax_rollout_vjp_tape",
           "brax_env_configure", "brax_env_step", "brax_autotune", "brax_autotune_on", "brax_schedule",
           "brax_set_schedule",
           "brax_nonfinite", "brax_last_error", "brax_step_vjp_noalloc")

_lib = None


def lib():
    """Load libbraxmi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2106_13281_amd.build)")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.brax_sys_create.argtypes = [P(C.c_char_p), C.c_int32, P(C.c_int32), C.c_int32, C.c_int32,
                                      P(C.c_void_p)]
        L.brax_sys_destroy.argtypes = [C.c_void_p]
        L.brax_sys_destroy.restype = None
        L.brax_sys_query.argtypes = [C.c_void_p, P(_Layout)]
        L.brax_default_angles.argtypes = [C.c_void_p, C.c_int32, P(C.c_float)]
        L.brax_default_qp.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, P(_State), C.c_void_p]
        L.brax_step.argtypes = [C.c_void_p, P(_State), C.c_void_p, P(_State), C.c_int32, C.c_void_p]
        L.brax_step_vjp.argtypes = [C.c_void_p, P(_State), C.c_void_p, P(_State), P(_State), C.c_void_p, C.c_int32,
                                    C.c_void_p]
        L.brax_step_vjp_noalloc.argtypes = [C.c_void_p, P(_State), C.c_void_p, P(_State), P(_State), C.c_void_p,
                                            C.c_int32, C.c_void_p]
        L.brax_rollout.argtypes = [C.c_void_p, P(_State), C.c_void_p, C.c_int32, C.c_int32, P(_State), P(_State),
                                   C.c_int32, C.c_void_p]
        L.brax_step_vjp_params.argtypes = [C.c_void_p, P(_State), C.c_void_p, P(_State), P(_State), C.c_void_p,
                                           C.c_void_p, C.c_int32, C.c_void_p]
        L.brax_rollout_tape.argtypes = [C.c_void_p, P(_State), C.c_void_p, C.c_int32, C.c_void_p, P(_State),
                                        C.c_int32, C.c_void_p]
        L.brax_step_vjp_tape.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, P(_State), P(_State), C.c_void_p,
                                         C.c_int32, C.c_void_p]
        L.brax_rollout_vjp_tape.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, P(_State), P(_State),
                                            C.c_void_p, C.c_int32, C.c_void_p]
        L.brax_env_configure.argtypes = [C.c_void_p, P(_EnvParams)]
        L.brax_env_step.argtypes = [C.c_void_p, P(_State), C.c_void_p, P(_State), P(_State), C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_int32, C.c_void_p]
        L.brax_autotune.argtypes = [C.c_void_p, C.c_void_p]
        L.brax_autotune_on.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
        L.brax_schedule.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32)]
        L.brax_set_schedule.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.brax_nonfinite.argtypes = [C.c_void_p, P(C.c_uint8)]
        L.brax_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("brax_sys_destroy", "brax_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise BraxError(rc, lib().brax_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


@dataclass
class State:
    """Structure-of-arrays state: four FP32 CUDA tensors."""
    pos: torch.Tensor
    rot: torch.Tensor
    vel: torch.Tensor
    ang: torch.Tensor

    @classmethod
    def empty(cls, b_max, n_envs, device="cuda", lead=()):
        f = dict(dtype=torch.float32, device=device)
        return cls(torch.empty(*lead, 3, b_max, n_envs, **f), torch.empty(*lead, 4, b_max, n_envs, **f),
                   torch.empty(*lead, 3, b_max, n_envs, **f), torch.empty(*lead, 3, b_max, n_envs, **f))

    @classmethod
    def zeros_like(cls, s):
        return cls(torch.zeros_like(s.pos), torch.zeros_like(s.rot), torch.zeros_like(s.vel),
                   torch.zeros_like(s.ang))

    def fields(self):
        return (self.pos, self.rot, self.vel, self.ang)

    def clone(self):
        return State(*(t.clone() for t in self.fields()))

    def struct(self):
        for t in self.fields():
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("state tensors must be contiguous float32 CUDA tensors")
        return _State(*(t.data_ptr() for t in self.fields()))

    def __getitem__(self, k):
        """Snapshot k of a trajectory state (leading save index)."""
        return State(*(t[k] for t in self.fields()))


class System:
    """A batch of environments of one or several system types on one GPU."""

    def __init__(self, descs, n_envs, env_desc=None, device=0):
        if isinstance(descs, str):
            descs = [descs]
        arr = (C.c_char_p * len(descs))(*[d.encode() for d in descs])
        ed = None
        if env_desc is not None:
            env_desc = list(int(x) for x in env_desc)
            if len(env_desc) != n_envs:
                raise ValueError("env_desc must have n_envs entries")
            ed = (C.c_int32 * n_envs)(*env_desc)
        h = C.c_void_p()
        _check(lib().brax_sys_create(arr, len(descs), ed, n_envs, device, C.byref(h)))
        self._h = h
        self._L = lib()
        self.device_index = device
        lay = _Layout()
        _check(lib().brax_sys_query(h, C.byref(lay)))
        self.n_envs, self.n_types = lay.n_envs, lay.n_types
        self.b_max, self.a_max, self.d_max = lay.b_max, lay.a_max, lay.d_max
        nt = lay.n_types
        self.type_envs = list(lay.type_envs[:nt])
        self.n_bodies = list(lay.n_bodies[:nt])
        self.n_joints = list(lay.n_joints[:nt])
        self.n_actions = list(lay.n_actions[:nt])
        self.n_dof = list(lay.n_dof[:nt])
        self.n_contacts = list(lay.n_contacts[:nt])
        self.substeps = list(lay.substeps[:nt])
        self.tape_step_floats = lay.tape_step_floats               # floats per step of a forward tape
        self.n_params = list(lay.n_params[:nt])
        self.p_max = lay.p_max
        self.n_pairs = list(lay.n_pairs[:nt])                      # body-body contact candidates
        self.vjp_lds_bytes = lay.vjp_lds_bytes                     # on-chip tape of the fused adjoint
        self.vjp_params_lds_bytes = lay.vjp_params_lds_bytes
        self.lds_limit = lay.lds_limit
        self.lanes_per_env = list(lay.lanes_per_env[:nt])          # fused forward: bodies + contact lanes
        self.dt = list(lay.dt[:nt])
        self.device = torch.device("cuda", device) if device >= 0 else None
        self._side = None  # second stream of the checkpointed backward (created on first use)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.brax_sys_destroy(h)
            self._h = None

    # ------------------------------------------------------------ helpers
    def new_state(self, lead=()):
        return State.empty(self.b_max, self.n_envs, self.device, lead)

    def default_angles(self, t=0):
        out = (C.c_float * max(self.n_dof[t], 1))()
        _check(lib().brax_default_angles(self._h, t, out))
        return torch.tensor(list(out)[: self.n_dof[t]], dtype=torch.float32)

    def _act(self, a, shape):
        if a is None:
            if self.a_max == 0:
                return None
            raise ValueError("actions required")
        if a.dtype != torch.float32 or not a.is_contiguous() or not a.is_cuda or tuple(a.shape) != shape:
            raise ValueError(f"actions must be a contiguous float32 CUDA tensor of shape {shape}")
        return a

    # ------------------------------------------------------------ calls
    def default_qp(self, angles=None, root_offset=None, out=None, stream=None):
        out = self.new_state() if out is None else out
        if angles is not None:
            angles = self._act(angles, (self.d_max, self.n_envs)) if self.d_max else None
        if root_offset is not None:
            root_offset = self._act(root_offset, (3, self.n_envs))
        st = out.struct()
        _check(lib().brax_default_qp(self._h, _ptr(angles), _ptr(root_offset), C.byref(st), _stream(stream)))
        return out

    def step(self, state, act, out=None, flags=0, stream=None):
        out = self.new_state() if out is None else out
        act = self._act(act, (self.a_max, self.n_envs))
        si, so = state.struct(), out.struct()
        _check(lib().brax_step(self._h, C.byref(si), _ptr(act), C.byref(so), flags, _stream(stream)))
        return out

    def step_vjp(self, state, act, g_out, g_in=None, g_act=None, flags=0, stream=None):
        g_in = self.new_state() if g_in is None else g_in
        act = self._act(act, (self.a_max, self.n_envs))
        if g_act is None:
            g_act = torch.empty(self.a_max, self.n_envs, dtype=torch.float32, device=self.device)
        si, sg, sgi = state.struct(), g_out.struct(), g_in.struct()
        _check(lib().brax_step_vjp(self._h, C.byref(si), _ptr(act), C.byref(sg), C.byref(sgi), _ptr(g_act), flags,
                                   _stream(stream)))
        return g_in, g_act

    def step_vjp_noalloc(self, state, act, g_out, g_in, g_act, flags=0, stream=None):
        """step_vjp through brax_step_vjp_noalloc: the library allocates nothing
        (the caller passes every output; the per-phase adjoint's workspace is the
        library's fixed per-GPU array)."""
        act = self._act(act, (self.a_max, self.n_envs))
        si, sg, sgi = state.struct(), g_out.struct(), g_in.struct()
        _check(lib().brax_step_vjp_noalloc(self._h, C.byref(si), _ptr(act), C.byref(sg), C.byref(sgi), _ptr(g_act),
                                           flags, _stream(stream)))
        return g_in, g_act

    def step_vjp_params(self, state, act, g_out, g_in=None, g_act=None, g_params=None, flags=0, stream=None):
        """step_vjp plus the per-environment cotangents of the system parameters [p_max][E]."""
        g_in = self.new_state() if g_in is None else g_in
        act = self._act(act, (self.a_max, self.n_envs))
        if g_act is None:
            g_act = torch.empty(self.a_max, self.n_envs, dtype=torch.float32, device=self.device)
        if g_params is None:
            g_params = torch.empty(self.p_max, self.n_envs, dtype=torch.float32, device=self.device)
        si, sg, sgi = state.struct(), g_out.struct(), g_in.struct()
        _check(lib().brax_step_vjp_params(self._h, C.byref(si), _ptr(act), C.byref(sg), C.byref(sgi), _ptr(g_act),
                                          _ptr(g_params), flags, _stream(stream)))
        return g_in, g_act, g_params

    def rollout(self, state, acts, save_every=0, out=None, traj=None, flags=0, stream=None):
        T = acts.shape[0] if acts is not None else 0
        out = self.new_state() if out is None else out
        if T:
            acts = self._act(acts, (T, self.a_max, self.n_envs))
        n_save = T // save_every if save_every > 0 else 0
        if n_save and traj is None:
            traj = self.new_state(lead=(n_save,))
        si, so = state.struct(), out.struct()
        tr = traj.struct() if n_save else None
        _check(lib().brax_rollout(self._h, C.byref(si), _ptr(acts) if T else None, T, save_every,
                                  C.byref(tr) if tr is not None else None, C.byref(so), flags, _stream(stream)))
        return out, (traj if n_save else None)

    def rollout_tape(self, state, acts, tape=None, out=None, flags=0, stream=None):
        """rollout that also writes the forward tape [T][tape_step_floats] for step_vjp_tape."""
        T = acts.shape[0] if acts is not None else 0
        out = self.new_state() if out is None else out
        if T:
            acts = self._act(acts, (T, self.a_max, self.n_envs))
        shape = (T, self.tape_step_floats)
        if tape is None:
            tape = torch.empty(shape, dtype=torch.float32, device=self.device)
        if tuple(tape.shape) != shape or tape.dtype != torch.float32 or not tape.is_contiguous():
            raise ValueError(f"tape must be a contiguous float32 tensor of shape {shape}")
        si, so = state.struct(), out.struct()
        _check(lib().brax_rollout_tape(self._h, C.byref(si), _ptr(acts) if T else None, T, _ptr(tape) if T else None,
                                       C.byref(so), flags, _stream(stream)))
        return out, tape

    def step_vjp_tape(self, tape, act, g_out, g_in=None, g_act=None, flags=0, stream=None):
        """step_vjp from one step's tape slice [tape_step_floats] instead of recomputing the step."""
        shape = (self.tape_step_floats,)
        if tuple(tape.shape) != shape or tape.dtype != torch.float32 or not tape.is_contiguous():
            raise ValueError(f"tape must be a contiguous float32 tensor of shape {shape}")
        g_in = self.new_state() if g_in is None else g_in
        act = self._act(act, (self.a_max, self.n_envs))
        if g_act is None:
            g_act = torch.empty(self.a_max, self.n_envs, dtype=torch.float32, device=self.device)
        sg, sgi = g_out.struct(), g_in.struct()
        _check(lib().brax_step_vjp_tape(self._h, _ptr(tape), _ptr(act), C.byref(sg), C.byref(sgi), _ptr(g_act),
                                        flags, _stream(stream)))
        return g_in, g_act

    def rollout_vjp_tape(self, tape, acts, g_out, g_in=None, g_acts=None, flags=0, stream=None):
        """Adjoint of T steps from their tape [T][tape_step_floats] (rollout_tape over
        the same acts [T][Amax][E]) in one launch: (g_in, g_acts [T][Amax][E])."""
        T = int(acts.shape[0])
        shape = (T, self.tape_step_floats)
        if tuple(tape.shape) != shape or tape.dtype != torch.float32 or not tape.is_contiguous():
            raise ValueError(f"tape must be a contiguous float32 tensor of shape {shape}")
        acts = self._act(acts, (T, self.a_max, self.n_envs))
        g_in = self.new_state() if g_in is None else g_in
        if g_acts is None:
            g_acts = torch.empty(T, self.a_max, self.n_envs, dtype=torch.float32, device=self.device)
        elif tuple(g_acts.shape) != (T, self.a_max, self.n_envs) or g_acts.dtype != torch.float32 \
                or not g_acts.is_contiguous():
            raise ValueError(f"g_acts must be a contiguous float32 tensor of shape {(T, self.a_max, self.n_envs)}")
        sg, sgi = g_out.struct(), g_in.struct()
        _check(lib().brax_rollout_vjp_tape(self._h, _ptr(tape), _ptr(acts), T, C.byref(sg), C.byref(sgi),
                                           _ptr(g_acts), flags, _stream(stream)))
        return g_in, g_acts

    def env_configure(self, params):
        """Environment-layer parameters, one dict per system type with keys root,
        forward_weight, healthy_reward, ctrl_cost, z_min, z_max."""
        if len(params) != self.n_types:
            raise ValueError(f"{self.n_types} parameter sets expected")
        arr = (_EnvParams * self.n_types)()
        for i, p in enumerate(params):
            arr[i] = _EnvParams(int(p.get("root", 0)), float(p.get("forward_weight", 1.0)),
                                float(p.get("healthy_reward", 1.0)), float(p.get("ctrl_cost", 0.5)),
                                float(p.get("z_min", -math.inf)), float(p.get("z_max", math.inf)))
        _check(lib().brax_env_configure(self._h, arr))

    @property
    def obs_dim(self):
        return 11 + 2 * self.d_max

    def env_step(self, state, act, reset, out=None, obs=None, reward=None, done=None, flags=0, stream=None):
        """(out, obs [Omax][E], reward [E], done [E] uint8) of one environment step."""
        out = self.new_state() if out is None else out
        act = self._act(act, (self.a_max, self.n_envs))
        dev = self.device
        obs = torch.empty(self.obs_dim, self.n_envs, dtype=torch.float32, device=dev) if obs is None else obs
        reward = torch.empty(self.n_envs, dtype=torch.float32, device=dev) if reward is None else reward
        done = torch.empty(self.n_envs, dtype=torch.uint8, device=dev) if done is None else done
        si, sr, so = state.struct(), reset.struct(), out.struct()
        _check(lib().brax_env_step(self._h, C.byref(si), _ptr(act), C.byref(sr), C.byref(so), _ptr(obs),
                                   _ptr(reward), _ptr(done), flags, _stream(stream)))
        return out, obs, reward, done

    def autotune(self, stream=None):
        _check(lib().brax_autotune(self._h, _stream(stream)))
        return self.schedule()

    def autotune_on(self, state, acts, stream=None):
        """autotune with trials on the caller's workload: T-step rollouts from
        `state` with `acts` [T][A_max][E] (T = acts.shape[0])."""
        T = acts.shape[0]
        acts = self._act(acts, (T, self.a_max, self.n_envs))
        si = state.struct()
        _check(lib().brax_autotune_on(self._h, C.byref(si), _ptr(acts), T, _stream(stream)))
        return self.schedule()

    def schedule(self):
        a, b = C.c_int32(), C.c_int32()
        _check(lib().brax_schedule(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_schedule(self, envs_per_wave, waves_per_block):
        _check(lib().brax_set_schedule(self._h, envs_per_wave, waves_per_block))
        return self.schedule()

    def nonfinite(self):
        """Per-environment non-finite flags of the last call made with BRAX_NONFINITE_FLAGS (host copy)."""
        buf = (C.c_uint8 * max(self.n_envs, 1))()
        _check(lib().brax_nonfinite(self._h, buf))
        return torch.tensor(list(buf)[: self.n_envs], dtype=torch.uint8)


class RolloutFn(torch.autograd.Function):
    """Differentiable T-step rollout (final state) with checkpoints every k steps.

    Forward keeps the state every k steps, computed segment by segment with
    brax_rollout_tape into a scratch segment tape (the taped kernel, so that
    the checkpoints and the backward's recomputed segments come from the same
    compiled code and the gradient does not depend on k); the last segment's
    tape is kept for the backward. Backward recomputes each other segment
    from its checkpoint and runs the step adjoint backwards
    through it: with tape=True the recompute writes every substep's tape
    (brax_rollout_tape, one segment at a time) and the adjoint reads it
    (brax_rollout_vjp_tape, one launch per segment; each recompute runs on a
    second stream during the adjoint of the segment after it); with tape=False the recompute keeps the step states
    (brax_rollout) and brax_step_vjp recomputes each step's substeps itself. Inputs: the four
    initial-state tensors and the action sequence [T][Amax][E]; outputs: the
    four final-state tensors.
    """

    @staticmethod
    def forward(ctx, system, k, tape, pos, rot, vel, ang, acts):
        T = acts.shape[0]
        k = max(1, min(int(k), max(T, 1)))
        s0 = State(pos.detach().contiguous(), rot.detach().contiguous(), vel.detach().contiguous(),
                   ang.detach().contiguous())
        acts_d = acts.detach().contiguous()
        ckpts = [s0]
        cur = s0
        t = 0
        scratch = torch.empty((min(k, max(T, 1)), system.tape_step_floats), dtype=torch.float32,
                              device=acts_d.device) if T else None
        while t < T:
            n = min(k, T - t)
            nxt, _ = system.rollout_tape(cur, acts_d[t:t + n], tape=scratch[:n])
            ckpts.append(nxt)
            cur = nxt
            t += n
        ctx.system, ctx.k, ctx.T, ctx.tape = system, k, T, bool(tape)
        # the last segment's tape is the one the backward starts with: kept
        # (with the tape adjoint), so that segment is not recomputed
        ctx.last_tape = scratch if tape else None
        ctx.save_for_backward(acts_d, *[x for c in ckpts[:-1] for x in c.fields()])
        return cur.pos, cur.rot, cur.vel, cur.ang

    @staticmethod
    def backward(ctx, gp, gr, gv, gw):
        system, k, T, use_tape = ctx.system, ctx.k, ctx.T, ctx.tape
        saved = ctx.saved_tensors
        acts = saved[0]
        ck = [State(*saved[1 + 4 * i: 5 + 4 * i]) for i in range((len(saved) - 1) // 4)]

        def z(g, ref):
            return torch.zeros_like(ref) if g is None else g.contiguous()

        g = State(z(gp, ck[0].pos), z(gr, ck[0].rot), z(gv, ck[0].vel), z(gw, ck[0].ang))
        g_acts = torch.zeros_like(acts)
        seg_starts = list(range(0, T, k))
        last, ctx.last_tape = ctx.last_tape, None
        if use_tape:
            g = _segments_backward(system, ck, acts, seg_starts, k, T, g, g_acts, last)
            return None, None, None, g.pos, g.rot, g.vel, g.ang, g_acts
        for si in reversed(range(len(seg_starts))):
            t0 = seg_starts[si]
            n = min(k, T - t0)
            # states s_{t0}, ..., s_{t0+n-1}
            states = [ck[si]]
            if n > 1:
                _, traj = system.rollout(ck[si], acts[t0:t0 + n - 1], save_every=1)
                states += [traj[i] for i in range(n - 1)]
            for i in reversed(range(n)):
                g_in, g_a = system.step_vjp(_contig(states[i]), acts[t0 + i], g)
                g_acts[t0 + i] = g_a
                g = g_in
        return None, None, None, g.pos, g.rot, g.vel, g.ang, g_acts


def _segments_backward(system, ck, acts, seg_starts, k, T, g, g_acts, last):
    """Tape adjoint of the segments, last first. Segment si's tape is
    recomputed from its checkpoint (brax_rollout_tape) on a second stream
    while segment si+1's adjoint (brax_rollout_vjp_tape) runs on the current
    one: both are small launches on disjoint SIMDs, so the recompute hides
    behind the adjoint. Two tape buffers alternate; a buffer is rewritten only
    after the adjoint that read it has finished (events), and every adjoint
    waits for its tape. `last`: the forward's tape of the last segment, or
    None (then it is recomputed too)."""
    nseg = len(seg_starts)
    if nseg == 0:
        return g
    main = torch.cuda.current_stream(acts.device)
    if system._side is None:
        system._side = torch.cuda.Stream(device=acts.device)  # default priority
    side = system._side
    rows = min(k, T)
    use_last = last is not None and tuple(last.shape) == (rows, system.tape_step_floats)
    bufs = [torch.empty((rows, system.tape_step_floats), dtype=torch.float32, device=acts.device),
            last if use_last else None]
    if bufs[1] is None:
        bufs[1] = torch.empty_like(bufs[0])
    for b in bufs:
        b.record_stream(side)
    freed = [None, None]     # event after the adjoint that last read each buffer
    tapes = {}
    side.wait_stream(main)   # checkpoints, actions and buffers are ready
    nxt = [0]

    def recompute(si):
        j = nxt[0]
        nxt[0] ^= 1
        t0 = seg_starts[si]
        n = min(k, T - t0)
        with torch.cuda.stream(side):
            if freed[j] is not None:
                side.wait_event(freed[j])
            system.rollout_tape(ck[si], acts[t0:t0 + n], tape=bufs[j][:n], stream=side)
            ev = torch.cuda.Event()
            ev.record(side)
        tapes[si] = (j, ev)

    if use_last:
        tapes[nseg - 1] = (1, None)   # the forward's tape is in buffer 1
    else:
        recompute(nseg - 1)
    for si in reversed(range(nseg)):
        if si > 0:
            recompute(si - 1)         # overlaps the adjoint below
        j, ev = tapes.pop(si)
        if ev is not None:
            main.wait_event(ev)
        t0 = seg_starts[si]
        n = min(k, T - t0)
        g, _ = system.rollout_vjp_tape(bufs[j][:n], acts[t0:t0 + n], g, g_acts=g_acts[t0:t0 + n], stream=main)
        freed[j] = torch.cuda.Event()
        freed[j].record(main)
    return g


def _contig(s):
    return State(*(t.contiguous() for t in s.fields()))


# device memory a rollout's whole forward tape may take before rollout_grad
# falls back to checkpoints (k=None)
TAPE_BUDGET_BYTES = 8 << 30
CHECKPOINT_EVERY = 10


def checkpoint_interval(system, T, tape=True, budget=TAPE_BUDGET_BYTES):
    """The checkpoint interval rollout_grad takes for k=None: the whole
    rollout (T steps, so one taped forward launch, the tape kept and one
    adjoint launch, with no recompute) when its tape fits `budget` bytes,
    else CHECKPOINT_EVERY steps. The gradient is the same either way."""
    T = int(T)
    if tape and T * system.tape_step_floats * 4 <= budget:
        return max(T, 1)
    return CHECKPOINT_EVERY


def rollout_grad(system, state, acts, k=None, tape=True):
    """Apply RolloutFn: returns the final State, differentiable w.r.t. state and acts.
    k: checkpoint interval in steps; None chooses it by checkpoint_interval."""
    if k is None:
        k = checkpoint_interval(system, acts.shape[0], tape)
    p, r, v, w = RolloutFn.apply(system, k, tape, state.pos, state.rot, state.vel, state.ang, acts)
    return State(p, r, v, w)
