"""Write algorithmic_flops.json: floating-point operations per environment step.

Counted by the oracle's counting scalar (add, sub, mul, div, sqrt, atan2,
asin, sin, cos each count one; a fused multiply-add is two) on states sampled
along seeded rollouts of each workload, so inactive contact candidates cost
only their detection, as in the method. `vjp_mean` is the oracle's count of
one reverse (adjoint) sweep through the step on the same states (the adjoint
rule of each operation the output depends on; see orc_count_vjp_flops), so
forward + VJP of one environment step is `mean + vjp_mean`. Calls only the
oracle.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2106_13281_amd import synth  # noqa: E402


def count(name, E=32, warm=20, steps=100, every=5):
    wl = synth.WORKLOADS[name]
    o = oracle.Oracle(synth.system_text(wl.system))
    s = o.system
    ang, root = synth.reset_noise(0, E, s.ndof, wl.angle_noise, wl.root_noise)
    X = np.stack([o.default_qp(s.default_angles() + ang[e].astype(np.float64), root[e]) for e in range(E)])
    acts = synth.actions(0, warm + steps, E, s.na, wl.act_range).astype(np.float64)
    X, tr, _ = o.rollout(X, acts, traj=True)
    vals, rev = [], []
    for t in range(warm, warm + steps - 1, every):
        for e in range(E):
            vals.append(o.count_flops(tr[t, e], acts[t + 1, e]))
            rev.append(o.count_vjp_flops(tr[t, e], acts[t + 1, e]))
    return float(np.mean(vals)), int(np.min(vals)), int(np.max(vals)), float(np.mean(rev))


def main():
    out = {"unit": "FLOP per environment step (all substeps)", "workloads": {}}
    for name in ("chain", "quadruped", "biped", "manipulator", "cheetah", "grasp"):
        mean, lo, hi, rev = count(name)
        out["workloads"][name] = {"mean": mean, "min": lo, "max": hi, "vjp_mean": rev}
        print(name, mean, lo, hi, rev)
    with open(os.path.join(HERE, "algorithmic_flops.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
