"""Pins of the oracle's joint axes (CPU).

The joint angles are the intrinsic X-Y-Z Euler angles of the child's joint
frame relative to the parent's (App. A: one angle per repeated
`angle_limit`); the axes about which actuators and limit springs act are the
Euler axes ê1 = parent x, ê2 = the intermediate y, ê3 = child z. What fixes
them independently of how the oracle writes them is the kinematics of Euler
angles: a rotation of the child by a small angle δ about world axis u
changes the angles by dθ with u = Σ_k dθ_k ê_k. So rotating the child about
ê_k moves θ_k by δ and the other two angles only at O(δ²) — checked here by
central differences at random poses of the biped's 1-, 2- and 3-axis joints
away from gimbal lock (a slipped sign or swapped column in any ê_k fails).
Then an actuator's torque (Sec. 3: actions are torques) is the gear times the
action along that same ê_k, and a limit spring's torque is -k_lim times the
angle's excess along it.
"""
import numpy as np
from scipy.spatial.transform import Rotation

import oracle
from paper_2106_13281_amd import synth


def _random_states(o, n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, o.nb, 13))
    X[:, :, 0:3] = rng.normal(0, 0.3, (n, o.nb, 3))
    X[:, :, 3:7] = Rotation.random(n * o.nb, random_state=seed).as_quat()[:, [3, 0, 1, 2]].reshape(n, o.nb, 4)
    X[:, :, 7:13] = rng.normal(0, 1.0, (n, o.nb, 6))
    return X


def _rotate_child(X, child, axis, delta):
    """Rotate body `child` of state X [nb][13] by `delta` about the world `axis`."""
    Y = X.copy()
    q = Y[child, 3:7]
    r = Rotation.from_rotvec(delta * np.asarray(axis)) * Rotation.from_quat([q[1], q[2], q[3], q[0]])
    x, y, z, w = r.as_quat()
    Y[child, 3:7] = [w, x, y, z]
    return Y


def test_euler_axes_are_the_rates_of_the_joint_angles():
    o = oracle.Oracle(synth.system_text("biped"))
    s = o._s
    delta = 1e-5
    checked = np.zeros(4, int)          # per DOF count of the joint
    for X in _random_states(o, 60, seed=5):
        th, ax = o.joint_angles(X)
        for j in range(o.nj):
            # away from gimbal lock and from the +-pi wrap of theta1, theta3
            if abs(np.sin(th[j, 1])) > 0.9 or np.abs(th[j, [0, 2]]).max() > 3.0:
                continue
            for k in range(3):
                thp, _ = o.joint_angles(_rotate_child(X, s.j_child[j], ax[j, k], +delta))
                thm, _ = o.joint_angles(_rotate_child(X, s.j_child[j], ax[j, k], -delta))
                rate = (thp[j] - thm[j]) / (2 * delta)
                want = np.eye(3)[k]
                assert np.abs(rate - want).max() < 1e-7, (j, k, th[j], rate)
                assert abs(np.linalg.norm(ax[j, k]) - 1.0) < 1e-12
            checked[s.j_dof[j]] += 1
    assert checked[1] >= 50 and checked[2] >= 50 and checked[3] >= 30, checked


def test_euler_axis_two_matches_the_intermediate_frame():
    """ê2 is the parent's y axis turned by θ1 about the parent's x axis (the
    frame between the first and second elementary rotations)."""
    o = oracle.Oracle(synth.system_text("biped"))
    s = o._s
    for X in _random_states(o, 10, seed=6):
        th, ax = o.joint_angles(X)
        for j in range(o.nj):
            P = s.j_parent[j]
            qP = X[P, 3:7]
            RP = Rotation.from_quat([qP[1], qP[2], qP[3], qP[0]]).as_matrix()
            FP = np.array(s.j_frame_p[j][:]).reshape(3, 3)
            Aw = RP @ FP
            inter = Aw @ Rotation.from_euler("x", th[j, 0]).as_matrix()
            assert np.abs(ax[j, 0] - Aw[:, 0]).max() < 1e-12
            assert np.abs(ax[j, 1] - inter[:, 1]).max() < 1e-12


def test_actuator_torque_is_gear_times_action_along_the_euler_axis():
    o = oracle.Oracle(synth.system_text("biped"))
    s = o._s
    for X in _random_states(o, 8, seed=7):
        _, ax = o.joint_angles(X)
        f0, t0 = o.joint_forces(X, np.zeros(o.na))
        for k in range(o.na):
            a = np.zeros(o.na)
            a[k] = 0.7
            f1, t1 = o.joint_forces(X, a)
            j, axis, gear = s.a_joint[k], s.a_axis[k], s.a_gear[k]
            want = 0.7 * gear * ax[j, axis]
            dt = t1 - t0
            assert np.abs(f1 - f0).max() == 0.0
            assert np.abs(dt[s.j_child[j]] - want).max() < 1e-9 * gear
            assert np.abs(dt[s.j_parent[j]] + want).max() < 1e-9 * gear
            others = [b for b in range(o.nb) if b not in (s.j_child[j], s.j_parent[j])]
            assert np.abs(dt[others]).max() == 0.0


def test_limit_torque_is_minus_stiffness_times_excess_along_the_euler_axes():
    o = oracle.Oracle(synth.system_text("biped"))
    s = o._s
    hits = 0
    for X in _random_states(o, 12, seed=8):
        th, ax = o.joint_angles(X)
        for j in range(o.nj):
            k_lim = s.j_k_lim[j]
            try:
                o._param("j_k_lim", (j,), 0.0)
                _, t0 = o.joint_forces(X)
                o._param("j_k_lim", (j,), 2.0 * k_lim)
                _, t2 = o.joint_forces(X)
            finally:
                o._param("j_k_lim", (j,), k_lim)
            want = np.zeros(3)
            for k in range(s.j_dof[j]):
                excess = th[j, k] - np.clip(th[j, k], s.j_lo[j][k], s.j_hi[j][k])
                want += -2.0 * k_lim * excess * ax[j, k]
                hits += excess != 0
            dt = t2 - t0
            assert np.abs(dt[s.j_child[j]] - want).max() < 1e-9 * (1 + np.abs(want).max())
            assert np.abs(dt[s.j_parent[j]] + want).max() < 1e-9 * (1 + np.abs(want).max())
    assert hits >= 40
