"""FP64 reference of the environment layer after the step (test infrastructure).

The paper (Section 4.2, Table 1, App. E) describes gym-like environments on top
of the physics step: observation, reward, termination and reset bookkeeping,
with locomotion rewards close to the MuJoCo gym ones (forward progress, a
reward for staying healthy, a control cost, no contact cost) and termination
on the torso height leaving a range (humanoid: 0.6 to 2.1). It gives no
formulas; this module writes out the reading the library implements:

  obs    = [z_root, q_root (4), v_root (3), w_root (3),
            theta_k for every joint DOF (D), (w_child - w_parent) . e_k (D)]
           (theta_k and e_k are the joint's Euler angles and axes, as in the
           joint law), zero-padded to 11 + 2 * D_max in a mixed batch;
  reward = forward_weight * (x_root' - x_root) / dt
           + healthy_reward * [healthy'] - ctrl_cost * sum_k a_k^2;
  done   = not healthy', healthy' = z_min <= z_root' <= z_max;
  out    = the reset state where done, else the stepped state; obs is taken
           of out.

Used only by tests; calls the oracle's stepper and joint-angle routine.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class EnvParams:
    root: int = 0
    forward_weight: float = 1.0
    healthy_reward: float = 1.0
    ctrl_cost: float = 0.5
    z_min: float = -np.inf
    z_max: float = np.inf


def obs_dim(ndof):
    return 11 + 2 * ndof


def observe(o, X, p: EnvParams, ndof_max=None):
    """Observations [E][11 + 2 D] of states X [E][B][13] (oracle `o`)."""
    X = np.asarray(X, dtype=np.float64)
    s = o.system
    D = s.ndof
    O = obs_dim(D if ndof_max is None else ndof_max)
    out = np.zeros((X.shape[0], O))
    for e in range(X.shape[0]):
        r = X[e, p.root]
        out[e, 0] = r[2]
        out[e, 1:5] = r[3:7]
        out[e, 5:8] = r[7:10]
        out[e, 8:11] = r[10:13]
        th, ax = o.joint_angles(X[e])
        k = 0
        for j, jt in enumerate(s.joints):
            wrel = X[e, jt["child"], 10:13] - X[e, jt["parent"], 10:13]
            for d in range(jt["dof"]):
                out[e, 11 + k] = th[j, d]
                out[e, 11 + D + k] = float(np.dot(wrel, ax[j, d]))
                k += 1
    return out


def env_step(o, X, act, reset, p: EnvParams, ndof_max=None):
    """(out, obs, reward, done) of one environment step from X with actions act."""
    X = np.asarray(X, dtype=np.float64)
    act = np.asarray(act, dtype=np.float64)
    Xn = o.step(X, act)
    dt = o.system.dt
    fwd = (Xn[:, p.root, 0] - X[:, p.root, 0]) / dt
    z = Xn[:, p.root, 2]
    healthy = (z >= p.z_min) & (z <= p.z_max)
    reward = p.forward_weight * fwd + p.healthy_reward * healthy - p.ctrl_cost * (act ** 2).sum(axis=1)
    done = ~healthy
    out = np.where(done[:, None, None], np.asarray(reset, dtype=np.float64), Xn)
    return out, observe(o, out, p, ndof_max), reward, done
