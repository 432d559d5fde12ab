"""Seeded scenes for the body-body contact tests (system texts and initial
states only; no physics here).

two_body(ka, kb): bodies "a" and "b", one collider each (sphere, capsule or
box), declared as a contact pair, no gravity.
cluster(frozen_hub): a box "hub" with two spheres and two capsules around it
and seven declared pairs (box-sphere, box-capsule, capsule-capsule,
sphere-sphere, sphere-capsule), so that bodies take part in several
candidates, both as the lane that evaluates them and as the one that
collects the other's share.
approach(...): bodies placed around a centre about 0.9 m above the ground,
moving towards it, random orientations and spins.
"""
import numpy as np
from scipy.spatial.transform import Rotation

BODY = {
    "sphere": 'colliders {{ sphere {{ radius: {r} }} }}',
    "capsule": 'colliders {{ capsule {{ radius: {r} length: {L} }} }}',
    "box": 'colliders {{ box {{ halfsize {{ x: {hx} y: {hy} z: {hz} }} }} }}',
    # a box collider off its body's centre and rotated in it
    "boxr": ('colliders {{ position {{ x: 0.04 y: -0.03 }} rotation {{ x: 30 y: 20 z: 10 }} '
             'box {{ halfsize {{ x: {hx} y: {hy} z: {hz} }} }} }}'),
}
KIND_PAIRS = [("sphere", "sphere"), ("sphere", "capsule"), ("capsule", "sphere"), ("capsule", "capsule"),
              ("sphere", "box"), ("box", "sphere"), ("capsule", "box"), ("box", "capsule"),
              ("sphere", "boxr"), ("boxr", "capsule")]


def two_body(ka, kb, e=0.0, mu=0.5, beta=0.2, substeps=1, dt=0.002):
    geo = dict(r=0.1, L=0.6, hx=0.2, hy=0.15, hz=0.1)
    ga = BODY[ka].format(**geo)
    gb = BODY[kb].format(**dict(geo, r=0.12, L=0.5))
    return f"""substeps: {substeps}
dt: {dt}
friction: {mu}
elasticity: {e}
baumgarte: {beta}
bodies {{ name: "a" mass: 2 inertia {{ x: 0.05 y: 0.05 z: 0.05 }} {ga} }}
bodies {{ name: "b" mass: 3 inertia {{ x: 0.07 y: 0.07 z: 0.07 }} {gb} }}
body_contacts {{ first: "a" second: "b" }}
"""


CLUSTER_BODIES = ("hub", "s1", "s2", "c1", "c2")


def cluster(frozen_hub=False):
    frozen = 'frozen { position { x: 1 y: 1 z: 1 } rotation { x: 1 y: 1 z: 1 } }' if frozen_hub else ""
    return f"""substeps: 4
dt: 0.004
friction: 0.8
elasticity: 0.3
baumgarte: 0.2
bodies {{ name: "hub" mass: 4 inertia {{ x: 0.06 y: 0.06 z: 0.06 }} {frozen}
  colliders {{ box {{ halfsize {{ x: 0.15 y: 0.15 z: 0.15 }} }} }} }}
bodies {{ name: "s1" mass: 1 inertia {{ x: 0.004 y: 0.004 z: 0.004 }} colliders {{ sphere {{ radius: 0.1 }} }} }}
bodies {{ name: "s2" mass: 1.5 inertia {{ x: 0.006 y: 0.006 z: 0.006 }} colliders {{ sphere {{ radius: 0.11 }} }} }}
bodies {{ name: "c1" mass: 1 inertia {{ x: 0.02 y: 0.02 z: 0.02 }}
  colliders {{ capsule {{ radius: 0.08 length: 0.5 }} }} }}
bodies {{ name: "c2" mass: 1.2 inertia {{ x: 0.025 y: 0.025 z: 0.025 }}
  colliders {{ rotation {{ x: 90 }} capsule {{ radius: 0.07 length: 0.45 }} }} }}
body_contacts {{ first: "hub" second: "s1" }}
body_contacts {{ first: "hub" second: "s2" }}
body_contacts {{ first: "hub" second: "c1" }}
body_contacts {{ first: "c2" second: "hub" }}
body_contacts {{ first: "c1" second: "c2" }}
body_contacts {{ first: "s1" second: "s2" }}
body_contacts {{ first: "s1" second: "c1" }}
"""


def approach(E, nb, seed, speed=2.0, dist=0.5, z=0.9):
    """[E][nb][13] states: body 0 at the centre (at rest), the others on a
    circle of radius `dist` around it, moving towards it at `speed` (plus
    noise); random orientations and angular velocities. For nb == 2 the two
    bodies start at -0.35 and +0.35 on x and both move."""
    rng = np.random.default_rng(seed)
    X = np.zeros((E, nb, 13))
    X[:, :, 3:7] = Rotation.random(E * nb, random_state=seed).as_quat()[:, [3, 0, 1, 2]].reshape(E, nb, 4)
    c = np.array([0.0, 0.0, z])
    if nb == 2:
        X[:, 0, 0:3] = c + [-0.35, 0.0, 0.0]
        X[:, 1, 0:3] = c + [0.35, 0.0, 0.0] + rng.uniform(-0.05, 0.05, (E, 3))
        X[:, 0, 7:10] = np.array([speed, 0.0, 0.0]) + rng.normal(0, 0.3, (E, 3))
        X[:, 1, 7:10] = np.array([-speed, 0.0, 0.0]) + rng.normal(0, 0.3, (E, 3))
    else:
        X[:, 0, 0:3] = c
        for i in range(1, nb):
            ang = 2 * np.pi * (i - 1) / (nb - 1) + rng.normal(0, 0.1, E)
            d = np.stack([np.cos(ang), np.sin(ang), rng.normal(0, 0.05, E)], 1)
            X[:, i, 0:3] = c + dist * d
            X[:, i, 7:10] = -speed * d + rng.normal(0, 0.3, (E, 3))
    X[:, :, 10:13] = rng.normal(0, 3.0, (E, nb, 3))
    return X.astype(np.float32).astype(np.float64)


def edge_box(frozen_box, box_first=False, r=0.05, L=0.6):
    """A capsule "cap" and a box "box" (half extents 0.2, 0.15, 0.1), declared
    as a contact pair (capsule first, or box first), no gravity."""
    frozen = 'frozen { position { x: 1 y: 1 z: 1 } rotation { x: 1 y: 1 z: 1 } }' if frozen_box else ""
    first, second = ("box", "cap") if box_first else ("cap", "box")
    return f"""substeps: 4
dt: 0.004
friction: 0.6
elasticity: 0.2
baumgarte: 0.2
bodies {{ name: "cap" mass: 2 inertia {{ x: 0.05 y: 0.04 z: 0.03 }}
  colliders {{ capsule {{ radius: {r} length: {L} }} }} }}
bodies {{ name: "box" mass: 3 inertia {{ x: 0.07 y: 0.06 z: 0.05 }} {frozen}
  colliders {{ box {{ halfsize {{ x: 0.2 y: 0.15 z: 0.1 }} }} }} }}
body_contacts {{ first: "{first}" second: "{second}" }}
"""


def edge_states(E, seed, frozen_box, r=0.05):
    """[E][2][13]: the capsule lying across the box's edge y = 0.15, z = 0.1
    (its axis about perpendicular to the edge and to the edge's bisector
    n = (0, 1, 1)/sqrt 2, tilted by a few degrees), its axis within r of the
    edge (in contact there, its ends clear of the box), moving towards the
    box; the box unrotated; its centre 1 m above the ground (its ends and
    the capsule clear of it)."""
    rng = np.random.default_rng(seed)
    lift = np.array([0.0, 0.0, 1.0])
    n = np.array([0.0, 1.0, 1.0]) / np.sqrt(2.0)
    base = Rotation.from_euler("x", -135.0, degrees=True)
    X = np.zeros((E, 2, 13))
    for e in range(E):
        edge = np.array([rng.uniform(-0.15, 0.15), 0.15, 0.1])
        rot = Rotation.from_rotvec(rng.normal(0.0, 0.1, 3)) * base
        X[e, 0, 0:3] = lift + edge + rng.uniform(0.2, 0.8) * r * n
        X[e, 0, 3:7] = rot.as_quat()[[3, 0, 1, 2]]
        X[e, 0, 7:10] = -0.2 * n + rng.normal(0.0, 0.1, 3)
        X[e, 0, 10:13] = rng.normal(0.0, 1.0, 3)
        X[e, 1, 0:3] = lift
        X[e, 1, 3] = 1.0
        if not frozen_box:
            X[e, 1, 7:10] = rng.normal(0.0, 0.05, 3)
            X[e, 1, 10:13] = rng.normal(0.0, 0.3, 3)
    return X.astype(np.float32).astype(np.float64)
