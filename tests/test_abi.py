"""The C-ABI library: exports, host-side validation and parser agreement.

No GPU needed: a handle created with device -1 parses and validates only.
"""
import ctypes as C
import os
import re

import pytest

import oracle
from paper_2106_13281_amd import braxmi, synth
from tests.pair_scenes import KIND_PAIRS, cluster, two_body

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "braxmi.h")
SYSTEMS = ("chain", "quadruped", "biped", "manipulator", "cheetah", "grasp")
MIXED = synth.MIXED_TYPES      # the four types of the mixed batch


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(brax_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = braxmi.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(braxmi.EXPORTS)


def host(descs, n=4, env_desc=None):
    return braxmi.System(descs, n, env_desc=env_desc, device=-1)


@pytest.mark.parametrize("name", SYSTEMS)
def test_library_and_oracle_parsers_agree(name):
    """Two independent parsers (C++ library, Python oracle) read the same sizes."""
    text = synth.system_text(name)
    s = host(text)
    o = oracle.Oracle(text).system
    assert s.n_bodies == [o.nb]
    assert s.n_joints == [o.nj]
    assert s.n_actions == [o.na]
    assert s.n_dof == [o.ndof]
    assert s.n_contacts == [o.nc]
    assert s.substeps == [o.substeps]
    assert abs(s.dt[0] - o.dt) < 1e-7
    ang = s.default_angles(0).numpy()
    assert abs(ang - o.default_angles()).max() < 1e-6


def test_mixed_batch_layout():
    descs = [synth.system_text(n) for n in MIXED]
    env = synth.mixed_assignment(0)
    s = host(descs, len(env), env_desc=env)
    assert s.type_envs == list(synth.MIXED_COUNTS)
    assert s.b_max == 11 and s.a_max == 17 and s.d_max == 17


def expect(code, descs, n=1, env_desc=None, match=None):
    with pytest.raises(braxmi.BraxError) as ei:
        host(descs, n, env_desc)
    assert ei.value.code == code, str(ei.value)
    if match:
        assert re.search(match, str(ei.value)), str(ei.value)


BODY = 'bodies {{ name: "{n}" mass: 1 inertia {{ x: 1 y: 1 z: 1 }} }}\n'


def joint(p, c, lims=1, extra=""):
    return (f'joints {{ name: "{p}{c}" parent: "{p}" child: "{c}" stiffness: 100 {extra}'
            + "angle_limit { min: -10 max: 10 } " * lims + "}\n")


def test_parse_errors_carry_line_and_column():
    expect(-2, "bodies { name: \"a\" mass: 1\n  foo: 3 }", match=r"2:3: unknown field 'foo'")
    expect(-2, "bodies { name: \"a\" mass: 1 ", match=r"missing '}'")
    expect(-2, "substeps: }", match=r"1:11")
    expect(-2, 'bodies { name: "a" mass: 1 inertia { x: 1 w: 2 } }', match=r"unknown field 'w'")
    expect(-2, "dt: 0.01 $", match=r"unexpected character")


def test_model_errors():
    two = BODY.format(n="a") + BODY.format(n="b")
    expect(-3, 'bodies { name: "a" mass: 0 inertia { x: 1 y: 1 z: 1 } }', match="mass")
    expect(-3, 'bodies { name: "a" mass: 1 inertia { x: 1 y: 0 z: 1 } }', match="inertia")
    expect(-3, 'bodies { name: "a" mass: 1 }', match="no inertia")
    expect(-3, 'bodies { name: "a" mass: 1 colliders { capsule { radius: 0.2 length: 0.3 } } }', match="2 radius")
    expect(-3, two + joint("a", "c"), match="unknown child")
    expect(-3, two + joint("a", "b") + joint("b", "a"), match="two parents|cycle")
    three = two + BODY.format(n="c")
    expect(-3, three + joint("a", "c") + joint("b", "c"), match="two parents")
    expect(-3, three + joint("a", "b") + joint("b", "c") + joint("c", "a"), match="two parents|cycle")
    expect(-3, two + joint("a", "b", lims=4), match="1 to 3")
    expect(-3, two + 'joints { name: "j" parent: "a" child: "b" angle_limit { min: 10 max: -10 } }', match="min > max")
    expect(-3, BODY.format(n="a") + BODY.format(n="a"), match="twice")
    expect(-3, two + joint("a", "b") + 'actuators { name: "x" joint: "nope" strength: 1 }', match="unknown joint")
    expect(-3, "", match="no bodies")
    expect(-3, "substeps: 0\n" + BODY.format(n="a"), match="substeps")


def test_argument_errors():
    L = braxmi.lib()
    h = C.c_void_p()
    assert L.brax_sys_create(None, 1, None, 1, -1, C.byref(h)) == -1
    arr = (C.c_char_p * 1)(BODY.format(n="a").encode())
    assert L.brax_sys_create(arr, 0, None, 1, -1, C.byref(h)) == -1
    assert L.brax_sys_create(arr, 1, None, -1, -1, C.byref(h)) == -1
    assert L.brax_sys_create(arr, 1, None, 1, -1, None) == -1
    bad = (C.c_int32 * 2)(0, 1)
    assert L.brax_sys_create(arr, 1, bad, 2, -1, C.byref(h)) == -1
    assert b"out of range" in L.brax_last_error()
    assert not h.value
    # a host-only handle refuses device work with BRAX_E_ARG
    s = host(BODY.format(n="a"), 3)
    st = braxmi._State()
    assert L.brax_step(s._h, C.byref(st), None, C.byref(st), 0, None) == -1
    assert L.brax_rollout(s._h, C.byref(st), None, -1, 0, None, C.byref(st), 0, None) == -1
    assert L.brax_rollout_vjp_tape(s._h, None, None, 1, C.byref(st), C.byref(st), None, 0, None) == -1
    assert b"host-only" in L.brax_last_error()
    assert L.brax_autotune_on(s._h, C.byref(st), None, 8, None) == -1
    assert b"host-only" in L.brax_last_error()
    assert L.brax_autotune_on(None, C.byref(st), None, 8, None) == -1
    assert L.brax_sys_query(None, None) == -1
    L.brax_sys_destroy(None)  # no-op


def test_last_error_is_thread_local():
    import threading
    L = braxmi.lib()
    L.brax_sys_query(None, None)
    seen = []

    def worker():
        seen.append(L.brax_last_error())

    th = threading.Thread(target=worker)
    th.start()
    th.join()
    assert seen == [b""]
    assert L.brax_last_error() != b""


@pytest.mark.parametrize("text", [two_body(ka, kb) for ka, kb in KIND_PAIRS] + [cluster(False), cluster(True)])
def test_body_contact_candidates_agree_with_the_oracle(text):
    """Both parsers expand the declared body pairs into the same number of
    candidates (a capsule against a box gives two)."""
    assert host(text).n_pairs == [oracle.Oracle(text).system.np]


def test_body_contact_errors():
    box = 'bodies {{ name: "{n}" mass: 1 colliders {{ box {{ halfsize {{ x: 0.1 y: 0.1 z: 0.1 }} }} }} }}\n'
    ball = 'bodies {{ name: "{n}" mass: 1 colliders {{ sphere {{ radius: 0.1 }} }} }}\n'
    expect(-3, box.format(n="a") + box.format(n="b") + 'body_contacts { first: "a" second: "b" }', match="box")
    expect(-3, ball.format(n="a") + 'body_contacts { first: "a" second: "z" }', match="bad pair")
    expect(-3, ball.format(n="a") + 'body_contacts { first: "a" second: "a" }', match="bad pair")
    expect(-2, ball.format(n="a") + ball.format(n="b") + 'body_contacts { first: "a" second: "b" third: "c" }',
           match="unknown field")
    # spheres around one: fifteen fit (the hub collects eight shares in one
    # evaluation slot and seven in the next); with two spheres on the hub,
    # nine satellites give it eighteen candidates, beyond the per-body limit
    def star(n, hub=ball):
        text = hub.format(n="hub") + "".join(ball.format(n=f"s{i}") for i in range(n))
        return text + "".join(f'body_contacts {{ first: "s{i}" second: "hub" }}\n' for i in range(n))
    assert host(star(15)).n_pairs == [15]
    two = 'bodies {{ name: "{n}" mass: 1 colliders {{ sphere {{ radius: 0.1 }} }} colliders {{ sphere {{ radius: 0.1 }} }} }}\n'
    expect(-3, star(9, two), match="more than 16 body-body")


def test_flag_values_and_combinations():
    """BRAX_PLAIN = 1, BRAX_FUSED = 2 (the default when neither is set),
    BRAX_GRAPH = 4, BRAX_NONFINITE_FLAGS = 8; PLAIN with FUSED and unknown
    bits are BRAX_E_ARG, checked before anything else of the call (here on a
    batch of zero environments, which launches nothing)."""
    text = open(HEADER).read()
    for name, value in (("BRAX_PLAIN", 1), ("BRAX_FUSED", 2), ("BRAX_GRAPH", 4), ("BRAX_NONFINITE_FLAGS", 8)):
        assert re.search(rf"\b{name}\s*=\s*{value}\b", text), name
        assert getattr(braxmi, name) == value
    L = braxmi.lib()
    s = host(BODY.format(n="a"), 3)
    st = braxmi._State()
    for flags, msg in ((3, b"both set"), (16, b"unknown flag"), (2, b"host-only"), (0, b"host-only")):
        assert L.brax_rollout(s._h, C.byref(st), None, 0, 0, None, C.byref(st), flags, None) == -1
        assert msg in L.brax_last_error(), (flags, L.brax_last_error())
        assert L.brax_step_vjp(s._h, C.byref(st), None, C.byref(st), C.byref(st), None, flags, None) == -1
        assert msg in L.brax_last_error(), (flags, L.brax_last_error())


def test_contact_lanes_per_environment():
    """A body with more than two ground-contact candidates takes contact lanes
    in the fused forward (one per two further candidates): the manipulator's
    box (8 corners) adds 3 lanes to its 7 bodies; capsules and spheres (at
    most two candidates) add none."""
    for name, nl in (("manipulator", 10), ("grasp", 10), ("quadruped", 9), ("biped", None), ("chain", None)):
        s = host(synth.system_text(name))
        want = nl if nl is not None else s.n_bodies[0]
        assert s.lanes_per_env == [want], name
    box = ('bodies { name: "a" mass: 1 inertia { x: 1 y: 1 z: 1 } '
           'colliders { box { halfsize { x: 0.1 y: 0.1 z: 0.1 } } } '
           'colliders { capsule { radius: 0.05 length: 0.4 } } }\n')
    s = host(box)
    assert s.n_contacts == [10] and s.lanes_per_env == [5]  # 10 candidates: the body lane and 4 contact lanes


def test_adjoint_tape_size_is_reported_against_the_lds_limit():
    """The fused adjoint keeps each substep's tape on chip: 17 floats per lane
    (20 with parameter cotangents) x 64 lanes per substep, beside the
    wavefront's exchange rows (20 floats per lane); the query reports it
    beside the per-workgroup limit (160 KiB for a host-only handle), so a
    system with many substeps is seen to exceed it (such batches take the
    per-phase adjoint; the parameter adjoint refuses them)."""
    few = "substeps: 10\n" + BODY.format(n="a")
    many = "substeps: 200\n" + BODY.format(n="a")
    s10, s200 = host(few), host(many)
    xch = 20 * 64 * 4
    assert s10.vjp_lds_bytes == 10 * 17 * 64 * 4 + xch
    assert s10.vjp_params_lds_bytes == 10 * 20 * 64 * 4 + xch
    assert s10.lds_limit == 160 * 1024
    assert s10.vjp_lds_bytes <= s10.lds_limit
    assert s200.vjp_lds_bytes == 200 * 17 * 64 * 4 + xch > s200.lds_limit
    # the bench and test systems all fit
    for name in SYSTEMS:
        s = host(synth.system_text(name))
        assert s.vjp_params_lds_bytes <= s.lds_limit, name


def test_checkpoint_interval_keeps_the_whole_tape_within_the_budget():
    """rollout_grad's default checkpoint interval: the whole rollout where its
    forward tape (T x tape_step_floats x 4 bytes) fits the budget, else the
    fixed interval; with tape=False always the fixed interval. The tape of
    1024 quadrupeds takes 64 lanes x 17 floats x 10 substeps per wavefront
    and step."""
    s = host(synth.system_text("quadruped"), n=1024)
    per_step = s.tape_step_floats * 4
    assert s.tape_step_floats % (64 * 17 * 10) == 0
    assert braxmi.checkpoint_interval(s, 100) == 100
    assert braxmi.checkpoint_interval(s, 100, budget=100 * per_step) == 100
    assert braxmi.checkpoint_interval(s, 100, budget=100 * per_step - 1) == braxmi.CHECKPOINT_EVERY
    assert braxmi.checkpoint_interval(s, 100, tape=False) == braxmi.CHECKPOINT_EVERY
    assert braxmi.checkpoint_interval(s, 0) == 1
    assert 100 * per_step <= braxmi.TAPE_BUDGET_BYTES
