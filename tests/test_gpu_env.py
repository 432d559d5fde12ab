"""GPU parity of the environment layer (brax_env_step) against the FP64
reference in oracle/env.py: stepped-or-reset state, observation, reward and
termination, on a homogeneous and a mixed batch, in place and graph-replayed."""
import numpy as np
import pytest
import torch

import oracle
from oracle.env import EnvParams, env_step
from paper_2106_13281_amd import braxmi, synth
from tests.helpers import ambiguous, make_states, rel_err

pytestmark = pytest.mark.gpu


def to_dev(X, b_max=None):
    return braxmi.State(*(torch.from_numpy(a).cuda() for a in synth.to_soa(X, b_max)))


def from_dev(st, nb):
    torch.cuda.synchronize()
    return synth.from_soa(*(t.cpu().numpy() for t in st.fields()), n_body=nb)


def acts_dev(a, a_max=None):
    return torch.from_numpy(synth.acts_to_device_layout(a[None], a_max)).cuda()[0].contiguous()


def params_for(o, X, a, seed):
    """Healthy range set so that about half of the environments terminate."""
    z = o.step(X, a.astype(np.float64))[:, 0, 2]
    zmid = float(np.median(z))
    return EnvParams(root=0, forward_weight=1.0, healthy_reward=0.5, ctrl_cost=0.25, z_min=-1.0, z_max=zmid), zmid


def check_env(o, X, a, R, p, out, obs, rew, done, mg, nb, D, Dm):
    ref_out, ref_obs, ref_r, ref_d = env_step(o, X, a.astype(np.float64), R, p, ndof_max=Dm)
    zref = o.step(X, a.astype(np.float64))[:, 0, 2]
    near = np.abs(zref - p.z_max) < 1e-5                       # termination decided within rounding
    amb = ambiguous(mg, 1e-6) | near
    scale_r = 1 + np.abs(ref_r).max()
    lo, hi = np.abs(ref_obs[:, :11 + D]).max(), np.abs(ref_obs[:, 11 + D:]).max()
    bad = ((done.astype(bool) != ref_d)
           | (rel_err(out[:, :nb], ref_out).max(1) >= 1e-4)
           | (np.abs(rew - ref_r) >= 2e-3 * scale_r)          # forward term: a position difference over dt
           | (np.abs(obs[:, :11 + D] - ref_obs[:, :11 + D]).max(1) >= 1e-4 * (1 + lo))
           | (np.abs(obs[:, 11 + D:] - ref_obs[:, 11 + D:]).max(1) >= 1e-3 * (1 + hi)))
    print(f"  excused (ambiguous, over tolerance): {int(bad.sum())} of {len(bad)}", flush=True)
    assert not (bad & ~amb).any(), np.flatnonzero(bad & ~amb)
    assert bad.sum() <= 0.01 * len(bad)
    return ref_d


def test_env_step_matches_reference_quadruped():
    E = 64
    o, X, acts = make_states("quadruped", E, seed=41, warm=12)
    _, R, _ = make_states("quadruped", E, seed=42, warm=0)
    a = acts[0]
    p, _ = params_for(o, X, a, 41)
    _, mg = o.step(X, a.astype(np.float64), margins=True)
    sysg = braxmi.System(synth.system_text("quadruped"), E)
    sysg.env_configure([dict(root=p.root, forward_weight=p.forward_weight, healthy_reward=p.healthy_reward,
                             ctrl_cost=p.ctrl_cost, z_min=p.z_min, z_max=p.z_max)])
    out, obs, rew, done = sysg.env_step(to_dev(X), acts_dev(a), to_dev(R))
    ref_d = check_env(o, X, a, R, p, from_dev(out, o.nb), obs.cpu().numpy().T, rew.cpu().numpy(),
                      done.cpu().numpy(), mg, o.nb, o.system.ndof, o.system.ndof)
    assert 0.2 < ref_d.mean() < 0.8
    # in place (out aliases in) and graph-replayed give the same bits
    st = to_dev(X)
    out2, obs2, rew2, done2 = sysg.env_step(st, acts_dev(a), to_dev(R), out=st)
    for x, y in zip(out.fields(), out2.fields()):
        assert torch.equal(x, y)
    assert torch.equal(obs, obs2) and torch.equal(rew, rew2) and torch.equal(done, done2)
    ob, rw, dn = torch.empty_like(obs), torch.empty_like(rew), torch.empty_like(done)
    gout = sysg.new_state()
    s_in, a_in, r_in = to_dev(X), acts_dev(a), to_dev(R)
    for rep in range(3):
        sysg.env_step(s_in, a_in, r_in, out=gout, obs=ob, reward=rw, done=dn, flags=braxmi.BRAX_GRAPH)
        torch.cuda.synchronize()
        assert torch.equal(ob, obs) and torch.equal(rw, rew) and torch.equal(dn, done), rep
        for x, y in zip(out.fields(), gout.fields()):
            assert torch.equal(x, y)
        _ = torch.randn(1000, device="cuda").sum()


def test_env_step_matches_reference_mixed_batch():
    types = list(synth.MIXED_TYPES)
    per_type = 12
    env = [k % len(types) for k in range(per_type * len(types))]
    descs = [synth.system_text(n) for n in types]
    mixed = braxmi.System(descs, len(env), env_desc=env)
    bm, am, Dm = mixed.b_max, mixed.a_max, mixed.d_max
    Xm = np.zeros((len(env), bm, 13))
    Xm[:, :, 3] = 1.0
    Rm = np.zeros_like(Xm)
    Rm[:, :, 3] = 1.0
    Am = np.zeros((len(env), am), np.float32)
    data, prm = {}, []
    for t, n in enumerate(types):
        o, X, acts = make_states(n, per_type, seed=50 + t, warm=8)
        _, R, _ = make_states(n, per_type, seed=60 + t, warm=0)
        p, _ = params_for(o, X, acts[0], t)
        idx = [i for i in range(len(env)) if env[i] == t]
        Xm[idx, :o.nb], Rm[idx, :o.nb], Am[idx, :o.na] = X, R, acts[0]
        data[n] = (o, X, R, acts[0], p, idx)
        prm.append(dict(root=0, forward_weight=p.forward_weight, healthy_reward=p.healthy_reward,
                        ctrl_cost=p.ctrl_cost, z_min=p.z_min, z_max=p.z_max))
    mixed.env_configure(prm)
    out, obs, rew, done = mixed.env_step(to_dev(Xm, bm), acts_dev(Am, am), to_dev(Rm, bm))
    Xo, O, Rw, Dn = from_dev(out, bm), obs.cpu().numpy().T, rew.cpu().numpy(), done.cpu().numpy()
    for n in types:
        o, X, R, a, p, idx = data[n]
        _, mg = o.step(X, a.astype(np.float64), margins=True)
        check_env(o, X, a, R, p, Xo[idx], O[idx], Rw[idx], Dn[idx], mg, o.nb, o.system.ndof, Dm)
        assert np.abs(O[idx, 11 + 2 * o.system.ndof:]).max(initial=0) == 0


def test_env_configure_rejects_bad_parameters():
    sysg = braxmi.System(synth.system_text("quadruped"), 4)
    with pytest.raises(braxmi.BraxError):
        sysg.env_configure([dict(root=9)])
    with pytest.raises(braxmi.BraxError):
        sysg.env_configure([dict(root=0, z_min=1.0, z_max=0.5)])
    st = sysg.default_qp()
    with pytest.raises(braxmi.BraxError):                      # not configured yet
        sysg.env_step(st, torch.zeros(sysg.a_max, 4, device="cuda"), st, out=sysg.new_state())
