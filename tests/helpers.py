"""Shared test helpers: workload construction and the parity metric.

The parity metric (per environment and per field): max |gpu - oracle| over
the field's components and bodies, divided by max(max |oracle|, floor) with
floors 1 m, 1 (quaternion), 1 m/s, 1 rad/s; quaternions are sign-aligned
first. Environments whose run passes within a small distance of a jump of
the step (contact activation, impulse on/off, angle wrap) are classified as
branch-ambiguous and reported separately: there FP32 and FP64 may take
different but equally correct branches.
"""
import numpy as np

import oracle
from paper_2106_13281_amd import synth

FIELDS = (("pos", 0, 3), ("rot", 3, 7), ("vel", 7, 10), ("ang", 10, 13))


def rel_err(Xg, Xo):
    """[E][4] relative error per field (see module docstring)."""
    out = []
    for _, lo, hi in FIELDS:
        g, o = np.array(Xg[:, :, lo:hi], dtype=np.float64), Xo[:, :, lo:hi]
        if lo == 3:
            sgn = np.sign((g * o).sum(-1, keepdims=True))
            sgn[sgn == 0] = 1
            g = g * sgn
        num = np.abs(g - o).reshape(len(g), -1).max(1)
        den = np.maximum(np.abs(o).reshape(len(o), -1).max(1), 1.0)
        out.append(num / den)
    return np.stack(out, 1)


def ambiguous(margins, thresh):
    """Environments whose run came within `thresh` of a jump of the step."""
    return margins[:, list(oracle.JUMP_MARGINS)].min(1) < thresh


def fp32_sensitivity(o, X0, acts, Xo, seeds=(1, 2, 3), rel=6e-8):
    """How far the oracle's own FP64 rollout from X0 under acts [T][E][A]
    moves when its state is perturbed at FP32 rounding level (relative `rel`,
    random signs) before every step: the largest rel_err against its
    unperturbed result Xo over the seeds, per environment. An FP32 run of the
    same rollout cannot be expected to agree with the oracle more closely
    than this."""
    acts = np.asarray(acts, dtype=np.float64)
    spread = np.zeros(len(X0))
    for seed in seeds:
        jit = np.random.default_rng(seed)
        X = np.array(X0, dtype=np.float64)
        for t in range(len(acts)):
            X = o.step(X * (1 + rel * jit.choice([-1.0, 1.0], size=X.shape)), acts[t])
        spread = np.maximum(spread, rel_err(X, Xo).max(1))
    return spread


def check_rollout(r, sens, tol):
    """Rollout parity: every environment meets `tol` unless the oracle itself
    is ill-conditioned there, i.e. its result moves by at least tol / 10
    under FP32-level perturbations (`sens`, see fp32_sensitivity). Over many
    steps with contacts a few environments are (chaotic contact sequences);
    they are excused one by one, never by a quota."""
    bad = r.max(1) >= tol
    sensitive = sens >= 0.1 * tol
    print(f"  over tolerance: {int(bad.sum())} of {len(bad)}, all FP32-sensitive in the oracle "
          f"({int(sensitive.sum())} sensitive); errors {r.max(1)[bad]}, sensitivities {sens[bad]}", flush=True)
    assert not (bad & ~sensitive).any(), (r.max(1)[bad & ~sensitive], sens[bad & ~sensitive])


def make_states(name, E, seed=0, warm=30, vel_noise=0.0):
    """Oracle reset pose with the workload's perturbation, advanced `warm`
    steps by the oracle (so contacts are active), rounded to FP32.

    Returns (oracle, X [E][B][13] float64 holding FP32 values, acts [T][E][A] FP32).
    """
    wl = synth.WORKLOADS[name]
    o = oracle.Oracle(synth.system_text(wl.system))
    s = o.system
    ang, root = synth.reset_noise(seed, E, s.ndof, wl.angle_noise, wl.root_noise)
    X = np.stack([o.default_qp(s.default_angles() + ang[e].astype(np.float64), root[e]) for e in range(E)])
    acts = synth.actions(seed, warm + 40, E, s.na, wl.act_range)
    if warm:
        X, _, _ = o.rollout(X, acts[:warm])
    if vel_noise:
        v, w = synth.state_noise(seed, E, s.nb, vel_noise, 2 * vel_noise)
        X[:, :, 7:10] += v
        X[:, :, 10:13] += w
    X = X.astype(np.float32).astype(np.float64)
    # renormalise the rounded quaternion exactly as both sides will see it
    return o, X, acts[warm:]
