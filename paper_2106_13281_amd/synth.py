"""Seeded synthetic workloads: random draws and layout moves only.

This module holds none of the physics. It draws the random numbers a
workload needs (reset perturbations and action sequences) and moves state
between the per-environment layout ``[E][B][13]`` and the library's
structure-of-arrays layout. Both the HIP path and its checker read the same
FP32 arrays it produces.

Random streams: ``numpy.random.default_rng(SeedSequence([seed, stream]))``,
stream 0 = reset perturbation, stream 1 = actions. Draws are FP32.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

SYSTEM_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "systems")


def system_path(name):
    return os.path.join(SYSTEM_DIR, f"{name}.txt")


def system_text(name):
    with open(system_path(name)) as f:
        return f.read()


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: system, batch, horizon and draw ranges."""
    system: str
    envs: int
    steps: int
    act_range: float        # actions ~ U(-act_range, act_range)
    angle_noise: float      # per-DOF reset angle perturbation ~ U(-x, x) rad
    root_noise: float       # root x, y ~ U(-x, x); drop height ~ U(0, x) m


# The workload shapes (small chain, quadruped, biped, differentiation,
# manipulator, planar runner, grasp; the mixed batch below). Sizes:
# environments x steps.
WORKLOADS = {
    "chain": Workload("chain", 64, 200, 1.0, 0.2, 0.0),
    "quadruped": Workload("quadruped", 4096, 1000, 1.0, 0.1, 0.1),
    "biped": Workload("biped", 2048, 1000, 0.4, 0.1, 0.0),
    "quadruped_diff": Workload("quadruped", 1024, 100, 1.0, 0.1, 0.1),
    "manipulator": Workload("manipulator", 819, 1000, 1.0, 0.1, 0.0),
    # planar runner with target-angle actuators: actions are joint angles (rad)
    "cheetah": Workload("cheetah", 2048, 1000, 0.6, 0.1, 0.1),
    # the manipulator with finger-box body-body contacts
    "grasp": Workload("grasp", 4096, 1000, 1.0, 0.1, 0.0),
}

# Mixed batch: 8192 environments, 25% chains, 40% quadrupeds, 25% bipeds,
# 10% manipulators (counts rounded half up: 2048 / 3277 / 2048 / 819).
MIXED_TYPES = ("chain", "quadruped", "biped", "manipulator")
MIXED_COUNTS = (2048, 3277, 2048, 819)


def _rng(seed, stream):
    return np.random.default_rng(np.random.SeedSequence([seed, stream]))


def reset_noise(seed, n_env, n_dof, angle_noise, root_noise):
    """(angle perturbation [E][D], root offset [E][3]) as FP32."""
    g = _rng(seed, 0)
    ang = g.uniform(-angle_noise, angle_noise, size=(n_env, n_dof)).astype(np.float32)
    root = np.zeros((n_env, 3), dtype=np.float32)
    if root_noise > 0:
        root[:, 0:2] = g.uniform(-root_noise, root_noise, size=(n_env, 2)).astype(np.float32)
        root[:, 2] = g.uniform(0.0, root_noise, size=n_env).astype(np.float32)
    return ang, root


def actions(seed, n_steps, n_env, n_act, act_range):
    """Action sequence [T][E][A] FP32, drawn in that order."""
    g = _rng(seed, 1)
    return g.uniform(-act_range, act_range, size=(n_steps, n_env, n_act)).astype(np.float32)


def state_noise(seed, n_env, n_body, vel_scale, ang_scale, stream=2):
    """Random velocities [E][B][3] and angular velocities [E][B][3] (FP32)."""
    g = _rng(seed, stream)
    v = g.uniform(-vel_scale, vel_scale, size=(n_env, n_body, 3)).astype(np.float32)
    w = g.uniform(-ang_scale, ang_scale, size=(n_env, n_body, 3)).astype(np.float32)
    return v, w


def mixed_assignment(seed=0):
    """Per-environment system type (index into MIXED_TYPES) for the mixed batch.

    A seeded permutation of the type counts, so types are interleaved and the
    library has to group environments itself.
    """
    types = np.concatenate([np.full(n, k, dtype=np.int32) for k, n in enumerate(MIXED_COUNTS)])
    g = _rng(seed, 3)
    return types[g.permutation(types.size)]


# ---------------------------------------------------------------- layouts
def to_soa(X, b_max=None):
    """[E][B][13] -> (pos [3][Bmax][E], rot [4][Bmax][E], vel [3][Bmax][E], ang [3][Bmax][E]) FP32.

    Padded body slots (B..Bmax) are zero.
    """
    X = np.asarray(X)
    E, B, _ = X.shape
    bm = B if b_max is None else b_max
    out = []
    for lo, n in ((0, 3), (3, 4), (7, 3), (10, 3)):
        a = np.zeros((n, bm, E), dtype=np.float32)
        a[:, :B, :] = np.transpose(X[:, :, lo:lo + n], (2, 1, 0))
        out.append(np.ascontiguousarray(a))
    return tuple(out)


def from_soa(pos, rot, vel, ang, n_body=None):
    """Inverse of to_soa: -> [E][B][13] (float64)."""
    pos, rot, vel, ang = (np.asarray(a, dtype=np.float64) for a in (pos, rot, vel, ang))
    B = pos.shape[1] if n_body is None else n_body
    E = pos.shape[2]
    X = np.zeros((E, B, 13))
    for lo, a in ((0, pos), (3, rot), (7, vel), (10, ang)):
        X[:, :, lo:lo + a.shape[0]] = np.transpose(a[:, :B, :], (2, 1, 0))
    return X


def acts_to_device_layout(acts, a_max=None):
    """[T][E][A] -> [T][Amax][E] FP32 (padded actions are zero)."""
    acts = np.asarray(acts, dtype=np.float32)
    T, E, A = acts.shape
    am = A if a_max is None else a_max
    out = np.zeros((T, am, E), dtype=np.float32)
    out[:, :A, :] = np.transpose(acts, (0, 2, 1))
    return out
