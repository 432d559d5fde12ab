"""Pins of the oracle's body-body contacts (CPU).

Geometry: the oracle reports |r_a + r_b - distance| of every candidate as a
branch margin; with two bodies far from the ground and at rest its minimum
is the smallest |gap| between the candidates' surfaces, which is checked
against a convex minimisation of the distance between the core features
(scipy; a capsule against a box is its two end spheres plus its axis
segment where the segment's point nearest the box lies between the ends).
A capsule lying across a box edge takes the impulse of its nearest point
in closed form, and a capsule axis reaching into a box its deepest point's
depth (scipy's bounded minimisation of the signed distance). Dynamics: equal and
opposite impulses conserve total linear and angular momentum exactly
(isotropic bodies, no gravity); a head-on elastic frictionless collision of
equal spheres exchanges their velocities exactly.
"""
import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial.transform import Rotation

import oracle

from tests.pair_scenes import two_body


def features(o, X):
    """World core features of the two bodies' (single) colliders."""
    out = []
    for i, b in enumerate(o.system.bodies):
        col = b["colliders"][0]
        R = Rotation.from_quat([X[i, 4], X[i, 5], X[i, 6], X[i, 3]]).as_matrix()
        p = X[i, 0:3]
        c = p + R @ col["pos"]
        Rc = R @ col["R"]
        if col["kind"] == "sphere":
            out.append(("point", c, col["radius"]))
        elif col["kind"] == "capsule":
            hh = col["length"] / 2 - col["radius"]
            out.append(("segment", (c + Rc @ [0, 0, hh], c - Rc @ [0, 0, hh]), col["radius"]))
        else:
            out.append(("box", (c, Rc, np.asarray(col["half"])), 0.0))
    return out


def param_point(kind, g, u):
    if kind == "point":
        return g
    if kind == "segment":
        return g[0] + u[0] * (g[1] - g[0])
    c, R, h = g
    return c + R @ (h * u)


def surface_gap(fa, fb):
    """min distance between the core features minus the radii (convex)."""
    (ka, ga, ra), (kb, gb, rb) = fa, fb
    na = {"point": 0, "segment": 1, "box": 3}[ka]
    nb = {"point": 0, "segment": 1, "box": 3}[kb]
    lo = lambda k: [0.0] if k == "segment" else [-1.0] * 3
    bounds = [(l, 1.0) for l in (lo(ka) if na else [])] + [(l, 1.0) for l in (lo(kb) if nb else [])]

    def f(x):
        pa = param_point(ka, ga, x[:na])
        pb = param_point(kb, gb, x[na:])
        return float(np.sum((pa - pb) ** 2))
    best = np.inf
    for seed in range(6):
        x0 = np.random.default_rng(seed).uniform(0.05, 0.95, na + nb)
        if na + nb == 0:
            best = f(np.zeros(0))
            break
        r = minimize(f, x0, bounds=bounds, method="L-BFGS-B", options=dict(ftol=1e-18, gtol=1e-14, maxiter=2000))
        best = min(best, r.fun)
    return np.sqrt(best) - ra - rb


@pytest.mark.parametrize("ka,kb", [("sphere", "sphere"), ("sphere", "capsule"), ("capsule", "sphere"),
                                   ("capsule", "capsule"), ("sphere", "box"), ("capsule", "box"),
                                   ("box", "capsule"), ("sphere", "boxr"), ("boxr", "capsule")])
def test_pair_depth_matches_convex_distance(ka, kb):
    o = oracle.Oracle(two_body(ka, kb))
    rng = np.random.default_rng(3)
    checked = 0
    for trial in range(60):
        X = np.zeros((1, 2, 13))
        X[0, :, 3:7] = Rotation.random(2, random_state=trial).as_quat()[:, [3, 0, 1, 2]]
        X[0, 0, 0:3] = [0.0, 0.0, 5.0]
        X[0, 1, 0:3] = [0.0, 0.0, 5.0] + rng.uniform(-0.4, 0.4, 3)
        fa, fb = features(o, X[0])
        # a capsule against a box: its two end spheres, and its axis segment
        # where the segment's point nearest the box lies between the ends
        # (then the segment's gap is the smallest; where it lies at an end it
        # is that end's gap, so it can be listed in either case)
        split = lambda f: [("point", g, f[2]) for g in f[1]] if f[0] == "segment" else [f]
        has_box = ka.startswith("box") or kb.startswith("box")
        if has_box:
            fas, fbs = split(fa), split(fb)
        else:
            fas, fbs = [fa], [fb]
        gaps = [surface_gap(x, y) for x in fas for y in fbs]
        axis_clear = True
        if has_box and "segment" in (fa[0], fb[0]):
            full = surface_gap(fa, fb)
            gaps.append(full)
            axis_clear = full > -min(fa[2], fb[2]) + 1e-6   # the axis itself stays outside the box
        if not has_box or (min(gaps) > -0.02 and axis_clear):  # deep box penetrations: the nearest-face rule
            _, mg = o.step(X, np.zeros((1, 0)), margins=True)
            assert abs(mg[0, 0] - min(abs(g) for g in gaps)) < 1e-7, (trial, mg[0, 0], gaps)
            checked += 1
    assert checked >= 20


@pytest.mark.parametrize("ka,kb", [("sphere", "capsule"), ("capsule", "capsule"), ("capsule", "box"),
                                   ("sphere", "box")])
def test_pair_collisions_conserve_momentum(ka, kb):
    o = oracle.Oracle(two_body(ka, kb, e=0.3, mu=0.8, substeps=4, dt=0.004))
    m = np.array([2.0, 3.0])
    I = np.array([0.05, 0.07])
    rng = np.random.default_rng(11)
    hits = 0
    for trial in range(12):
        X = np.zeros((1, 2, 13))
        X[0, :, 3:7] = Rotation.random(2, random_state=100 + trial).as_quat()[:, [3, 0, 1, 2]]
        X[0, 0, 0:3] = [-0.35, 0.0, 5.0]
        X[0, 1, 0:3] = [0.35, 0.0, 5.0] + rng.uniform(-0.05, 0.05, 3)
        X[0, 0, 7:10] = [2.0, 0.0, 0.0] + rng.normal(0, 0.3, 3)
        X[0, 1, 7:10] = [-2.0, 0.0, 0.0] + rng.normal(0, 0.3, 3)
        X[0, :, 10:13] = rng.normal(0, 3.0, (2, 3))
        _, tr, mg = o.rollout(X, np.zeros((60, 1, 0)), traj=True, margins=True)
        P0 = (m[:, None] * X[0, :, 7:10]).sum(0)
        L0 = (np.cross(X[0, :, 0:3], m[:, None] * X[0, :, 7:10]) + I[:, None] * X[0, :, 10:13]).sum(0)
        P1 = (m[:, None] * tr[:, 0, :, 7:10]).sum(1)
        L1 = (np.cross(tr[:, 0, :, 0:3], m[:, None] * tr[:, 0, :, 7:10]) + I[:, None] * tr[:, 0, :, 10:13]).sum(1)
        assert np.abs(P1 - P0).max() < 1e-11 * (1 + np.abs(P0).max())
        assert np.abs(L1 - L0).max() < 1e-11 * (1 + np.abs(L0).max())
        v_rel_before = np.linalg.norm(X[0, 0, 7:10] - X[0, 1, 7:10])
        moved = np.abs(tr[-1, 0, :, 7:10] - X[0, :, 7:10]).max()
        hits += moved > 0.1 * v_rel_before
    assert hits >= 6             # most trials do collide


def test_head_on_elastic_equal_spheres_exchange_velocities():
    text = two_body("sphere", "sphere", e=1.0, mu=0.0, beta=0.0).replace('mass: 3 inertia { x: 0.07 y: 0.07 z: 0.07 }',
                                                                         'mass: 2 inertia { x: 0.05 y: 0.05 z: 0.05 }')
    o = oracle.Oracle(text)
    X = np.zeros((1, 2, 13))
    X[0, :, 3] = 1.0
    X[0, 0, 0:3] = [-0.1, 0.0, 5.0]
    X[0, 1, 0:3] = [0.1, 0.0, 5.0]                  # overlapping by 0.02 m, approaching
    X[0, 0, 7] = 1.5
    X[0, 1, 7] = -0.5
    Xn = o.step(X, np.zeros((1, 0)))
    assert abs(Xn[0, 0, 7] - (-0.5)) < 1e-14 and abs(Xn[0, 1, 7] - 1.5) < 1e-14
    assert np.abs(Xn[0, :, 8:10]).max() == 0 and np.abs(Xn[0, :, 10:13]).max() == 0


def test_point_inside_box_uses_the_nearest_face():
    """A sphere centre 0.03 m inside the box's top face (the nearest face):
    depth = r + 0.03 along that face's normal."""
    o = oracle.Oracle(two_body("sphere", "box"))
    X = np.zeros((1, 2, 13))
    X[0, :, 3] = 1.0
    X[0, 1, 0:3] = [0.0, 0.0, 5.0]
    X[0, 0, 0:3] = [0.05, -0.02, 5.0 + 0.1 - 0.03]      # box half height 0.1
    _, mg = o.step(X, np.zeros((1, 0)), margins=True)
    assert abs(mg[0, 0] - (0.1 + 0.03)) < 1e-12
    # the impulse pushes the sphere up (+z) and the box down
    Xn = o.step(X, np.zeros((1, 0)))
    assert Xn[0, 0, 9] > 0 and Xn[0, 1, 9] < 0 and abs(Xn[0, 0, 7]) < 1e-12


def _two_spheres(mu, seed):
    """Two free spheres (r 0.1 and 0.12, masses 2 and 3, isotropic inertia),
    no gravity, overlapping by about 1 cm, approaching along the line of
    centres and slipping across it, both spinning."""
    o = oracle.Oracle(two_body("sphere", "sphere", e=0.0, mu=mu, beta=0.2, substeps=1, dt=0.002))
    rng = np.random.default_rng(seed)
    X = np.zeros((1, 2, 13))
    X[0, :, 3:7] = Rotation.random(2, random_state=seed).as_quat()[:, [3, 0, 1, 2]]
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    X[0, 0, 0:3] = [0.0, 0.0, 5.0]
    X[0, 1, 0:3] = X[0, 0, 0:3] - 0.21 * n              # n points from b to a
    t = np.cross(n, rng.normal(size=3))
    t /= np.linalg.norm(t)
    X[0, 0, 7:10] = -0.8 * n + 1.5 * t
    X[0, 1, 7:10] = 0.4 * n - 0.5 * t
    X[0, :, 10:13] = rng.normal(0, 4.0, (2, 3))
    return o, X


def _contact_frame(Xn):
    """Normal (from b to a), depth and the middle of the overlap, from the
    post-kinematic positions (a step moves positions only in its kinematic
    update, so the stepped state holds them)."""
    pa, pb = Xn[0, 0, 0:3], Xn[0, 1, 0:3]
    d = pa - pb
    dist = np.linalg.norm(d)
    n = d / dist
    depth = 0.1 + 0.12 - dist
    x = pb + (0.12 - depth / 2) * n
    return n, depth, x


def test_pair_sticking_friction_stops_the_slip_at_the_contact_point():
    """Coulomb cone wide enough (mu = 10) that the tangential impulse is the
    one that stops the slip: after the step the two spheres' velocities at
    the contact point agree in the tangent plane. This holds only with the
    tangential effective mass of both bodies, translations and rotations
    (1/m_a + 1/m_b + (r_a x t).Ia^-1(r_a x t) + (r_b x t).Ib^-1(r_b x t)),
    taken at the point where the impulse is applied (Sec. 7.2; the impulse
    law of the ground contact, between two bodies)."""
    for seed in range(6):
        o, X = _two_spheres(10.0, seed)
        Xn = o.step(X, np.zeros((1, 0)))
        n, depth, x = _contact_frame(Xn)
        assert depth > 0
        ua = Xn[0, 0, 7:10] + np.cross(Xn[0, 0, 10:13], x - Xn[0, 0, 0:3])
        ub = Xn[0, 1, 7:10] + np.cross(Xn[0, 1, 10:13], x - Xn[0, 1, 0:3])
        u = ua - ub
        ut = u - np.dot(u, n) * n
        u0 = (X[0, 0, 7:10] + np.cross(X[0, 0, 10:13], x - Xn[0, 0, 0:3])
              - X[0, 1, 7:10] - np.cross(X[0, 1, 10:13], x - Xn[0, 1, 0:3]))
        assert np.linalg.norm(u0 - np.dot(u0, n) * n) > 0.5      # it was slipping
        assert np.linalg.norm(ut) < 1e-13, (seed, ut)
        assert np.dot(u, n) > -1e-12                             # no longer approaching


def test_pair_sliding_friction_is_mu_times_the_normal_impulse_at_the_overlap_middle():
    """Narrow cone (mu = 0.05): the impulse J on the first sphere has
    tangential part exactly mu times its normal part, opposite to the slip;
    both spheres' angular momenta change by r x (+-J) with the lever arms
    ending at the middle of the overlap, |r_a| = r_a - depth/2 and
    |r_b| = r_b - depth/2 (a contact point anywhere else along the normal
    gives other angular changes)."""
    m = np.array([2.0, 3.0])
    I = np.array([0.05, 0.07])
    for seed in range(6):
        o, X = _two_spheres(0.05, seed)
        Xn = o.step(X, np.zeros((1, 0)))
        n, depth, x = _contact_frame(Xn)
        J = m[0] * (Xn[0, 0, 7:10] - X[0, 0, 7:10])
        assert np.abs(J + m[1] * (Xn[0, 1, 7:10] - X[0, 1, 7:10])).max() < 1e-13
        jn = np.dot(J, n)
        jt = J - jn * n
        assert jn > 0
        assert abs(np.linalg.norm(jt) - 0.05 * jn) < 1e-13 * jn, (seed, np.linalg.norm(jt) / jn)
        u0 = (X[0, 0, 7:10] + np.cross(X[0, 0, 10:13], x - Xn[0, 0, 0:3])
              - X[0, 1, 7:10] - np.cross(X[0, 1, 10:13], x - Xn[0, 1, 0:3]))
        slip = u0 - np.dot(u0, n) * n
        assert np.dot(jt, slip) < -0.999 * np.linalg.norm(jt) * np.linalg.norm(slip)
        ra = -(0.1 - depth / 2) * n
        rb = (0.12 - depth / 2) * n
        assert np.abs(I[0] * (Xn[0, 0, 10:13] - X[0, 0, 10:13]) - np.cross(ra, J)).max() < 1e-13
        assert np.abs(I[1] * (Xn[0, 1, 10:13] - X[0, 1, 10:13]) - np.cross(rb, -J)).max() < 1e-13


SPHERE_ON_BOX = """substeps: 10
dt: 0.05
gravity {{ z: -9.81 }}
friction: {mu}
elasticity: 0
baumgarte: 0.2
bodies {{ name: "ball" mass: 1 inertia {{ x: 0.004 y: 0.004 z: 0.004 }}
  colliders {{ sphere {{ radius: 0.1 }} }} }}
bodies {{ name: "table" mass: 50 inertia {{ x: 1 y: 1 z: 1 }}
  frozen {{ position {{ x: 1 y: 1 z: 1 }} rotation {{ x: 1 y: 1 z: 1 }} }}
  colliders {{ box {{ halfsize {{ x: 1 y: 1 z: 0.1 }} }} }} }}
body_contacts {{ first: "ball" second: "table" }}
"""


def test_sphere_sliding_on_a_frozen_box_rolls_at_the_lever_arm_speed():
    """A solid ball (m 1 kg, r 0.1 m, I = 2/5 m r^2) resting on a frozen box
    at the contact fixed point depth* = g h^2 / beta (h = 5 ms: the Baumgarte
    impulse then cancels the substep's gravity exactly, as on the ground),
    launched at v0 = 1 m/s without spin. While it slips its speed drops by
    exactly mu g h per substep; then it rolls, and since the friction
    impulse's angular momentum about the contact level is conserved, at
    v = v0 m l^2 / (m l^2 + I) with the lever arm l = r - depth*/2 from the
    centre to the middle of the overlap (l = r would give 5/7 v0: 0.714286;
    here 0.711766), with w = v / l."""
    g, h, beta, r, m, I, mu, v0 = 9.81, 0.005, 0.2, 0.1, 1.0, 0.004, 0.5, 1.0
    o = oracle.Oracle(SPHERE_ON_BOX.format(mu=mu))
    depth = g * h * h / beta
    X = np.zeros((1, 2, 13))
    X[0, :, 3] = 1.0
    X[0, 1, 0:3] = [0.0, 0.0, 1.0]                      # top face at z = 1.1
    X[0, 0, 0:3] = [-0.3, 0.0, 1.1 + r - depth]
    X[0, 0, 7] = v0
    Xs, tr, _ = o.rollout(X, np.zeros((6, 1, 0)), traj=True)
    # first step (10 substeps): still slipping, exact Coulomb deceleration
    assert abs(tr[0, 0, 0, 7] - (v0 - 10 * mu * g * h)) < 1e-12
    ell = r - depth / 2
    assert abs(tr[0, 0, 0, 11] - 10 * mu * m * g * h * ell / I) < 1e-10
    # then rolling at the conserved angular momentum's speed
    v_roll = v0 * m * ell ** 2 / (m * ell ** 2 + I)
    for t in (3, 5):
        assert abs(tr[t, 0, 0, 7] - v_roll) < 1e-12, (tr[t, 0, 0, 7], v_roll)
        assert abs(tr[t, 0, 0, 11] - v_roll / ell) < 1e-10
    assert abs(v_roll - 5.0 / 7.0) > 1e-3                 # the pin tells the contact points apart
    # the normal direction stays at the fixed point; the table never moves
    assert abs(Xs[0, 0, 2] - X[0, 0, 2]) < 1e-12 and abs(Xs[0, 0, 9]) < 1e-12
    assert np.array_equal(Xs[0, 1], X[0, 1])


CAPSULE_ON_FROZEN_BOX = """substeps: 1
dt: 0.002
friction: 0.7
elasticity: 0.0
baumgarte: 0.2
bodies {{ name: "cap" mass: 2 inertia {{ x: 0.05 y: 0.04 z: 0.03 }}
  colliders {{ capsule {{ radius: {r} length: {L} }} }} }}
bodies {{ name: "box" mass: 3 inertia {{ x: 0.07 y: 0.07 z: 0.07 }}
  frozen {{ position {{ x: 1 y: 1 z: 1 }} rotation {{ x: 1 y: 1 z: 1 }} }}
  colliders {{ box {{ halfsize {{ x: 0.2 y: 0.15 z: 0.1 }} }} }} }}
body_contacts {{ first: "cap" second: "box" }}
"""


LIFT = np.array([0.0, 0.0, 5.0])   # far above the ground plane (no gravity in these scenes)


def _capsule_state(centre, axis_rot):
    """[1][2][13]: the capsule at `centre` (relative to the box) with rotation
    `axis_rot` (its local z is the axis), at rest; the box, unrotated and at
    rest, 5 m above the ground."""
    X = np.zeros((1, 2, 13))
    X[0, 0, 0:3] = LIFT + centre
    X[0, 0, 3:7] = axis_rot.as_quat()[[3, 0, 1, 2]]
    X[0, 1, 0:3] = LIFT
    X[0, 1, 3] = 1.0
    return X


@pytest.mark.parametrize("d", [0.01, 0.03])
def test_capsule_across_a_box_edge_takes_the_impulse_of_its_nearest_point(d):
    """A capsule lying across the box's edge y = 0.15, z = 0.1 at distance d
    (< r) from it, its axis perpendicular to the edge and to the edge's
    bisector n = (0, 1, 1)/sqrt 2: the nearest point is the capsule's middle,
    the ends are clear of the box. One substep at rest, no gravity, box
    frozen: the only impulse acts along n at a lever arm parallel to n, so
    v' = beta (r - d) / h n exactly and w' = 0. (A capsule taken as its two
    end spheres would pass through the edge.)"""
    r, L, h, beta = 0.05, 0.6, 0.002, 0.2
    o = oracle.Oracle(CAPSULE_ON_FROZEN_BOX.format(r=r, L=L))
    n = np.array([0.0, 1.0, 1.0]) / np.sqrt(2.0)
    edge = np.array([0.05, 0.15, 0.1])
    rot = Rotation.from_euler("x", -135.0, degrees=True)      # local z -> (0, 1, -1)/sqrt 2
    assert np.allclose(rot.apply([0, 0, 1]), [0.0, 1 / np.sqrt(2), -1 / np.sqrt(2)])
    X = _capsule_state(edge + d * n, rot)
    Xn, mg = o.step(X, np.zeros((1, 0)), margins=True)
    assert np.abs(Xn[0, 0, 7:10] - beta * (r - d) / h * n).max() < 1e-12
    assert np.abs(Xn[0, 0, 10:13]).max() < 1e-12
    assert abs(mg[0, 0] - (r - d)) < 1e-12           # the smallest |depth| is the middle's
    assert np.abs(Xn[0, 1, 7:13]).max() == 0.0         # the frozen box does not move


def _signed_box_distance(p, half):
    q = np.abs(p) - half
    return np.linalg.norm(np.maximum(q, 0.0)) + min(q.max(), 0.0)


@pytest.mark.parametrize("trial", range(6))
def test_capsule_axis_reaching_into_a_box_takes_its_deepest_point(trial):
    """A long thin capsule whose axis passes through the box while both ends
    stay clear of it: the only candidate in contact is the axis segment, and
    its depth is r minus the smallest signed distance of an axis point from
    the box (a convex function of the axis parameter), found here by
    scipy's bounded scalar minimisation."""
    from scipy.optimize import minimize_scalar
    r, L = 0.02, 1.4
    o = oracle.Oracle(CAPSULE_ON_FROZEN_BOX.format(r=r, L=L))
    half = np.array([0.2, 0.15, 0.1])
    rng = np.random.default_rng(50 + trial)
    while True:
        rot = Rotation.random(random_state=1000 * trial + int(rng.integers(1 << 30)))
        centre = rng.uniform(-0.5, 0.5) * half
        axis = rot.apply([0, 0, 1])
        hh = L / 2 - r
        ends = [centre + hh * axis, centre - hh * axis]
        sd = lambda s: _signed_box_distance(ends[0] + s * (ends[1] - ends[0]), half)
        if min(sd(0.0), sd(1.0)) > r + 0.05:
            break
    best = minimize_scalar(sd, bounds=(0.0, 1.0), method="bounded", options=dict(xatol=1e-12))
    assert best.fun < 0.0                                # the axis reaches into the box
    _, mg = o.step(_capsule_state(centre, rot), np.zeros((1, 0)), margins=True)
    assert abs(mg[0, 0] - (r - best.fun)) < 1e-7, (mg[0, 0], r - best.fun)
