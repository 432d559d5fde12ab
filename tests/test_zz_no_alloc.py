"""brax_step_vjp_noalloc: the adjoint of one step without any allocation in
the call, its per-phase workspace being the library's fixed per-GPU array.

It must give what brax_step_vjp gives for the same arguments (the same
kernels, so bit for bit), on consecutive calls that share the array, the
second on a smaller batch of another system, and the first again after it.
"""
import numpy as np
import pytest
import torch

from paper_2106_13281_amd import braxmi, synth
from tests.helpers import make_states

pytestmark = pytest.mark.gpu


def to_dev(X, b_max=None):
    return braxmi.State(*(torch.from_numpy(a).cuda() for a in synth.to_soa(X, b_max)))


def case(name, E, seed):
    o, X, acts = make_states(name, E, seed=seed, warm=15)
    sysg = braxmi.System(synth.system_text(synth.WORKLOADS[name].system), E)
    a = torch.from_numpy(synth.acts_to_device_layout(acts[:1], sysg.a_max)).cuda()[0].contiguous()
    g = np.random.default_rng(seed + 1).normal(size=X.shape).astype(np.float32).astype(np.float64)
    return sysg, to_dev(X), a, to_dev(g)


def outputs(sysg):
    g_in = sysg.new_state()
    g_act = torch.empty(sysg.a_max, sysg.n_envs, dtype=torch.float32, device="cuda")
    return g_in, g_act


def same(x, y):
    gx, ax = x
    gy, ay = y
    torch.cuda.synchronize()
    return all(torch.equal(u, v) for u, v in zip(gx.fields(), gy.fields())) and torch.equal(ax, ay)


@pytest.mark.parametrize("flags", [braxmi.BRAX_PLAIN, braxmi.BRAX_FUSED])
def test_noalloc_vjp_equals_step_vjp_on_consecutive_calls(flags):
    big = case("quadruped", 157, 41)       # several wavefronts and a ragged tail
    small = case("chain", 40, 43)          # a smaller batch of another system
    ref_big = big[0].step_vjp(big[1], big[2], big[3], flags=flags)
    ref_small = small[0].step_vjp(small[1], small[2], small[3], flags=flags)
    first = big[0].step_vjp_noalloc(big[1], big[2], big[3], *outputs(big[0]), flags=flags)
    assert same(first, ref_big)
    second = small[0].step_vjp_noalloc(small[1], small[2], small[3], *outputs(small[0]), flags=flags)
    assert same(second, ref_small)
    # the array now holds the small batch's leftovers; the big one again
    third = big[0].step_vjp_noalloc(big[1], big[2], big[3], *outputs(big[0]), flags=flags)
    assert same(third, ref_big)
    for g_in, g_act in (first, second, third):
        assert all(torch.isfinite(f).all() for f in g_in.fields()) and torch.isfinite(g_act).all()


def test_noalloc_vjp_rejects_graph_and_oversized_batches():
    sysg, s, a, g = case("chain", 40, 45)
    g_in, g_act = outputs(sysg)
    with pytest.raises(braxmi.BraxError) as ei:
        sysg.step_vjp_noalloc(s, a, g, g_in, g_act, flags=braxmi.BRAX_GRAPH)
    assert ei.value.code == -1  # BRAX_E_ARG
    # 32768 quadrupeds: the per-phase workspace (about 245 MB) exceeds the fixed 64 MiB
    E = 32768
    big = braxmi.System(synth.system_text("quadruped"), E)
    st = big.default_qp()
    acts = torch.zeros(big.a_max, E, dtype=torch.float32, device="cuda")
    gi, ga = outputs(big)
    with pytest.raises(braxmi.BraxError) as ei:
        big.step_vjp_noalloc(st, acts, st, gi, ga, flags=braxmi.BRAX_PLAIN)
    assert ei.value.code == -6  # BRAX_E_UNSUPPORTED
    # the fused adjoint of the same batch needs no workspace
    ref = big.step_vjp(st, acts, st, flags=braxmi.BRAX_FUSED)
    got = big.step_vjp_noalloc(st, acts, st, gi, ga, flags=braxmi.BRAX_FUSED)
    assert same(got, ref)
