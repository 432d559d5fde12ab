"""System description for the oracle: text parser, derived quantities, reset pose.

TEST INFRASTRUCTURE ONLY (part of the oracle): used by the tests, the smoke
check and the CPU-baseline leg of the benchmark, never by the product path.
Written independently of the library's own C++ parser.

The text format follows the ProtoBuf text form of the paper's Appendix A
(``substeps``, ``dt``, ``gravity``, ``bodies`` with ``mass``, ``inertia`` and
``frozen``, ``joints`` with ``parent``, ``child``, ``stiffness``,
``child_offset``/``parent_offset`` and repeated ``angle_limit``), plus the
fields the paper leaves to the engine (colliders, actuators, joint frames,
damping, contact constants). Angles in the file are degrees.

Readings of the paper encoded here (all FP64):
* inertia — principal moments in the body frame; when a body gives none it is
  that of uniform solid colliders (sphere 2/5 m r^2; box m(b^2+c^2)/3 on
  half-extents; capsule = cylinder plus two hemispheres, mass split by volume).
* joint DOF = number of ``angle_limit`` entries (Appendix A); the free axes
  are the joint frame's x, y, z, the relative rotation of the child's joint
  frame to the parent's is intrinsic X-Y-Z.
* ``default_qp`` (Section 4.1) places each tree in a valid joint
  configuration: child rotation R_C = R_P J_P Rx Ry Rz(theta) J_C^T and the
  child's anchor on the parent's anchor; roots without a given position are
  lifted so the lowest contact point sits ``clearance`` above the ground.
"""
from __future__ import annotations

import math
import re

import numpy as np

MAXB, MAXJ, MAXC, MAXA, MAXP = 16, 16, 96, 48, 32

# body-body contact candidate kinds: the core feature of the first body
# (point, segment or box) against that of the second
PP, PS, SP, SS, PB, BP, SB, BS = range(8)


# ----------------------------------------------------------------- parsing
_TOKEN = re.compile(r'\s*(?:(#[^\n]*)|([A-Za-z_][A-Za-z0-9_]*)|("(?:[^"\\]|\\.)*")|'
                    r'([-+]?(?:\d+\.?\d*|\.\d+)(?:[eE][-+]?\d+)?)|([{}:]))')


def _tokens(text):
    pos = 0
    out = []
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            if text[pos:].strip() == "":
                break
            raise ValueError(f"cannot tokenize near {text[pos:pos + 20]!r}")
        pos = m.end()
        if m.group(1):
            continue
        if m.group(2):
            out.append(("id", m.group(2)))
        elif m.group(3):
            out.append(("str", m.group(3)[1:-1]))
        elif m.group(4):
            out.append(("num", float(m.group(4))))
        elif m.group(5):
            out.append(("sym", m.group(5)))
    return out


def parse(text):
    """Parse the text into nested dicts: field name -> list of values/dicts."""
    toks = _tokens(text)
    i = 0

    def message(end_brace):
        nonlocal i
        msg = {}
        while i < len(toks):
            kind, v = toks[i]
            if kind == "sym" and v == "}":
                if not end_brace:
                    raise ValueError("unbalanced '}'")
                i += 1
                return msg
            if kind != "id":
                raise ValueError(f"expected a field name, got {v!r}")
            name = v
            i += 1
            if i < len(toks) and toks[i] == ("sym", ":"):
                i += 1
                if i >= len(toks):
                    raise ValueError("missing value")
                kind2, v2 = toks[i]
                i += 1
                if kind2 == "sym" and v2 == "{":
                    msg.setdefault(name, []).append(message(True))
                elif kind2 in ("num", "str", "id"):
                    msg.setdefault(name, []).append(v2)
                else:
                    raise ValueError(f"bad value for {name}")
            elif i < len(toks) and toks[i] == ("sym", "{"):
                i += 1
                msg.setdefault(name, []).append(message(True))
            else:
                raise ValueError(f"expected ':' or '{{' after {name}")
        if end_brace:
            raise ValueError("missing '}'")
        return msg

    return message(False)


def _one(msg, name, default=None):
    v = msg.get(name)
    if not v:
        return default
    return v[-1]


def _vec(msg, name, default=(0.0, 0.0, 0.0)):
    m = _one(msg, name)
    if m is None:
        return np.array(default, dtype=np.float64)
    return np.array([float(_one(m, k, 0.0)) for k in "xyz"], dtype=np.float64)


# ----------------------------------------------------------------- rotations
def rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)


def rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=np.float64)


def rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)


def euler_xyz(angles):
    """Intrinsic X-Y-Z rotation Rx(a) Ry(b) Rz(c), angles in radians."""
    return rot_x(angles[0]) @ rot_y(angles[1]) @ rot_z(angles[2])


def mat_to_quat(R):
    """Unit quaternion (w, x, y, z), w >= 0, of a rotation matrix (Shepperd's method)."""
    tr = R[0, 0] + R[1, 1] + R[2, 2]
    cands = [tr, R[0, 0], R[1, 1], R[2, 2]]
    k = int(np.argmax(cands))
    if k == 0:
        w = math.sqrt(1.0 + tr) / 2
        q = [w, (R[2, 1] - R[1, 2]) / (4 * w), (R[0, 2] - R[2, 0]) / (4 * w), (R[1, 0] - R[0, 1]) / (4 * w)]
    elif k == 1:
        x = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) / 2
        q = [(R[2, 1] - R[1, 2]) / (4 * x), x, (R[0, 1] + R[1, 0]) / (4 * x), (R[0, 2] + R[2, 0]) / (4 * x)]
    elif k == 2:
        y = math.sqrt(1.0 - R[0, 0] + R[1, 1] - R[2, 2]) / 2
        q = [(R[0, 2] - R[2, 0]) / (4 * y), (R[0, 1] + R[1, 0]) / (4 * y), y, (R[1, 2] + R[2, 1]) / (4 * y)]
    else:
        z = math.sqrt(1.0 - R[0, 0] - R[1, 1] + R[2, 2]) / 2
        q = [(R[1, 0] - R[0, 1]) / (4 * z), (R[0, 2] + R[2, 0]) / (4 * z), (R[1, 2] + R[2, 1]) / (4 * z), z]
    q = np.array(q, dtype=np.float64)
    q /= np.linalg.norm(q)
    if q[0] < 0:
        q = -q
    return q


# ----------------------------------------------------------------- colliders
def collider_inertia(col, mass):
    """Inertia tensor (3x3, about the collider centre, collider frame) of a uniform solid."""
    kind = col["kind"]
    if kind == "sphere":
        r = col["radius"]
        return np.eye(3) * (0.4 * mass * r * r)
    if kind == "box":
        a, b, c = col["half"]
        return np.diag([mass * (b * b + c * c) / 3, mass * (a * a + c * c) / 3, mass * (a * a + b * b) / 3])
    r, L = col["radius"], col["length"]
    H = L - 2 * r
    vc = math.pi * r * r * H
    vs = 4.0 / 3.0 * math.pi * r ** 3
    mc = mass * vc / (vc + vs)
    ms = mass - mc
    i_ax = mc * r * r / 2 + ms * 2 * r * r / 5
    i_perp = mc * (H * H / 12 + r * r / 4) + ms * (2 * r * r / 5 + H * H / 4 + 3 * H * r / 8)
    return np.diag([i_perp, i_perp, i_ax])


def collider_volume(col):
    kind = col["kind"]
    if kind == "sphere":
        return 4.0 / 3.0 * math.pi * col["radius"] ** 3
    if kind == "box":
        a, b, c = col["half"]
        return 8 * a * b * c
    r, L = col["radius"], col["length"]
    return math.pi * r * r * (L - 2 * r) + 4.0 / 3.0 * math.pi * r ** 3


def collider_points(col):
    """Contact candidates (body-frame centre, radius) of a collider against the plane."""
    R, c = col["R"], col["pos"]
    if col["kind"] == "sphere":
        return [(c.copy(), col["radius"])]
    if col["kind"] == "capsule":
        hh = col["length"] / 2 - col["radius"]
        return [(c + R @ np.array([0, 0, s * hh]), col["radius"]) for s in (1.0, -1.0)]
    a, b, cc = col["half"]
    pts = []
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                pts.append((c + R @ np.array([sx * a, sy * b, sz * cc]), 0.0))
    return pts


def _feature(col):
    """Core feature of a collider in its body's frame: ('point', centre, r),
    ('segment', (end0, end1), r) or ('box', (centre, R, half), 0)."""
    R, c = col["R"], col["pos"]
    if col["kind"] == "sphere":
        return "point", c.copy(), col["radius"]
    if col["kind"] == "capsule":
        hh = col["length"] / 2 - col["radius"]
        return "segment", (c + R @ np.array([0, 0, hh]), c + R @ np.array([0, 0, -hh])), col["radius"]
    return "box", (c.copy(), R.copy(), np.asarray(col["half"], dtype=np.float64)), 0.0


def pair_candidates(a, ca, b, cb):
    """Contact candidates between collider ca of body a and cb of body b:
    sphere-sphere, sphere-capsule, capsule-capsule, sphere-box; a capsule
    against a box contributes its two end spheres and its axis segment, the
    latter only where the segment's point nearest the box lies strictly
    between its ends; box-box is not modelled."""
    ka, ga, ra = _feature(ca)
    kb, gb, rb = _feature(cb)
    z3, eye = np.zeros(3), np.eye(3)

    def rec(kind, a0, a1, rA, b0, b1, rB, ah=z3, aR=eye, bh=z3, bR=eye):
        return dict(a=a, b=b, kind=kind, a0=a0, a1=a1, ra=rA, b0=b0, b1=b1, rb=rB, ah=ah, aR=aR, bh=bh, bR=bR)
    if ka == "box" and kb == "box":
        raise ValueError("box-box body contacts are not modelled")
    if ka == "point" and kb == "point":
        return [rec(PP, ga, ga, ra, gb, gb, rb)]
    if ka == "point" and kb == "segment":
        return [rec(PS, ga, ga, ra, gb[0], gb[1], rb)]
    if ka == "segment" and kb == "point":
        return [rec(SP, ga[0], ga[1], ra, gb, gb, rb)]
    if ka == "segment" and kb == "segment":
        return [rec(SS, ga[0], ga[1], ra, gb[0], gb[1], rb)]
    if kb == "box":
        pts = [ga] if ka == "point" else list(ga)
        out = [rec(PB, p, p, ra, gb[0], gb[0], 0.0, bh=gb[2], bR=gb[1]) for p in pts]
        if ka == "segment":
            out.append(rec(SB, ga[0], ga[1], ra, gb[0], gb[0], 0.0, bh=gb[2], bR=gb[1]))
        return out
    pts = [gb] if kb == "point" else list(gb)
    out = [rec(BP, ga[0], ga[0], 0.0, p, p, rb, ah=ga[2], aR=ga[1]) for p in pts]
    if kb == "segment":
        out.append(rec(BS, ga[0], ga[0], 0.0, gb[0], gb[1], rb, ah=ga[2], aR=ga[1]))
    return out


# ----------------------------------------------------------------- the system
class System:
    """FP64 system description plus the flat arrays the C++ oracle reads."""

    def __init__(self, text):
        cfg = parse(text)
        self.substeps = int(_one(cfg, "substeps", 1))
        self.dt = float(_one(cfg, "dt", 0.01))
        self.gravity = _vec(cfg, "gravity")
        self.beta = float(_one(cfg, "baumgarte", 0.2))
        self.elasticity = float(_one(cfg, "elasticity", 0.0))
        self.friction = float(_one(cfg, "friction", 1.0))
        self.clearance = float(_one(cfg, "clearance", 0.01))
        if self.substeps < 1 or not self.dt > 0:
            raise ValueError("substeps must be >= 1 and dt > 0")

        self.bodies = []
        names = {}
        for bm in cfg.get("bodies", []):
            name = _one(bm, "name")
            if name is None or name in names:
                raise ValueError(f"body name missing or repeated: {name}")
            mass = float(_one(bm, "mass", 0.0))
            if not mass > 0:
                raise ValueError(f"body {name}: mass must be > 0")
            cols = []
            for cm in bm.get("colliders", []):
                col = {"pos": _vec(cm, "position"),
                       "R": euler_xyz(np.radians(_vec(cm, "rotation")))}
                if "sphere" in cm:
                    col.update(kind="sphere", radius=float(_one(_one(cm, "sphere"), "radius", 0.0)))
                elif "capsule" in cm:
                    cp = _one(cm, "capsule")
                    col.update(kind="capsule", radius=float(_one(cp, "radius", 0.0)),
                               length=float(_one(cp, "length", 0.0)))
                    if col["length"] < 2 * col["radius"]:
                        raise ValueError(f"body {name}: capsule length < 2 radius")
                elif "box" in cm:
                    col.update(kind="box", half=_vec(_one(cm, "box"), "halfsize"))
                else:
                    raise ValueError(f"body {name}: collider without shape")
                cols.append(col)
            frozen = _one(bm, "frozen", {})
            fp = _vec(frozen, "position")
            fr = _vec(frozen, "rotation")
            if "inertia" in bm:
                inertia = _vec(bm, "inertia")
            else:
                if not cols:
                    raise ValueError(f"body {name}: no inertia and no colliders")
                vols = np.array([collider_volume(c) for c in cols])
                I = np.zeros((3, 3))
                for c, vol in zip(cols, vols):
                    mc = mass * vol / vols.sum()
                    Ic = c["R"] @ collider_inertia(c, mc) @ c["R"].T
                    d = c["pos"]
                    I += Ic + mc * (d @ d * np.eye(3) - np.outer(d, d))
                off = I - np.diag(np.diag(I))
                if np.abs(off).max() > 1e-9 * np.abs(np.diag(I)).max():
                    raise ValueError(f"body {name}: derived inertia is not diagonal in the body frame")
                inertia = np.diag(I).copy()
            if not (inertia > 0).all():
                raise ValueError(f"body {name}: inertia must be > 0")
            pos = _one(bm, "position")
            names[name] = len(self.bodies)
            self.bodies.append(dict(name=name, mass=mass, inertia=inertia, colliders=cols,
                                    free_pos=1.0 - (fp != 0), free_rot=1.0 - (fr != 0),
                                    position=None if pos is None else _vec(bm, "position")))
        self.nb = len(self.bodies)
        if self.nb == 0 or self.nb > MAXB:
            raise ValueError("need 1..16 bodies")

        self.joints = []
        jnames = {}
        children = set()
        for jm in cfg.get("joints", []):
            name = _one(jm, "name")
            p, c = _one(jm, "parent"), _one(jm, "child")
            if p not in names or c not in names:
                raise ValueError(f"joint {name}: unknown body")
            if names[c] in children:
                raise ValueError(f"joint {name}: body {c} has two parents")
            children.add(names[c])
            k = float(_one(jm, "stiffness", 0.0))
            lims = jm.get("angle_limit", [])
            if not 1 <= len(lims) <= 3:
                raise ValueError(f"joint {name}: 1..3 angle_limit entries required")
            lo = np.zeros(3)
            hi = np.zeros(3)
            for a, lm in enumerate(lims):
                lo[a] = math.radians(float(_one(lm, "min", 0.0)))
                hi[a] = math.radians(float(_one(lm, "max", 0.0)))
                if lo[a] > hi[a]:
                    raise ValueError(f"joint {name}: angle_limit min > max")
            rot = np.radians(_vec(jm, "rotation"))
            crot = np.radians(_vec(jm, "child_rotation")) if "child_rotation" in jm else rot
            jnames[name] = len(self.joints)
            self.joints.append(dict(
                name=name, parent=names[p], child=names[c], dof=len(lims),
                anchor_p=_vec(jm, "parent_offset"), anchor_c=_vec(jm, "child_offset"),
                frame_p=euler_xyz(rot), frame_c=euler_xyz(crot),
                k_lin=k, c_lin=float(_one(jm, "damping", 0.0)),
                k_ang=float(_one(jm, "angular_stiffness", k)),
                c_ang=float(_one(jm, "angular_damping", 0.0)),
                k_lim=float(_one(jm, "limit_stiffness", k)),
                lo=lo, hi=hi))
        self.nj = len(self.joints)
        if self.nj > MAXJ:
            raise ValueError("too many joints")
        # tree check: following parents from any body must end at a root
        parent_of = {j["child"]: j["parent"] for j in self.joints}
        for b in range(self.nb):
            seen = set()
            x = b
            while x in parent_of:
                if x in seen:
                    raise ValueError("joint graph has a cycle")
                seen.add(x)
                x = parent_of[x]
        self.parent_of = parent_of

        # (joint, axis, gear, mode): mode 0 = torque gear * clip(a, -1, 1);
        # mode 1 = target angle: gear * (clamp(a, lo, hi) - theta), a in radians
        self.actions = []
        for am in cfg.get("actuators", []):
            jn = _one(am, "joint")
            if jn not in jnames:
                raise ValueError(f"actuator on unknown joint {jn}")
            j = jnames[jn]
            gear = float(_one(am, "strength", 0.0))
            kinds = [k for k in ("torque", "angle") if k in am]
            if len(kinds) > 1:
                raise ValueError(f"actuator {jn}: both torque and angle")
            mode = 1 if kinds == ["angle"] else 0
            for ax in range(self.joints[j]["dof"]):
                self.actions.append((j, ax, gear, mode))
        self.na = len(self.actions)
        if self.na > MAXA:
            raise ValueError("too many actions")

        self.contacts = []  # (body, local centre, radius)
        for bi, b in enumerate(self.bodies):
            for col in b["colliders"]:
                for c, r in collider_points(col):
                    self.contacts.append((bi, c, r))
        self.nc = len(self.contacts)
        if self.nc > MAXC:
            raise ValueError("too many contact candidates")
        # body-body contact candidates of the declared pairs (every collider of
        # the first body against every collider of the second)
        bnames = {b["name"]: i for i, b in enumerate(self.bodies)}
        self.pairs = []
        for pm in cfg.get("body_contacts", []):
            fa, fb = _one(pm, "first"), _one(pm, "second")
            if fa not in bnames or fb not in bnames or fa == fb:
                raise ValueError(f"body_contacts: bad pair {fa} / {fb}")
            a, b = bnames[fa], bnames[fb]
            for ca in self.bodies[a]["colliders"]:
                for cb in self.bodies[b]["colliders"]:
                    self.pairs += pair_candidates(a, ca, b, cb)
        self.np = len(self.pairs)
        if self.np > MAXP:
            raise ValueError("too many body-body contact candidates")
        self.ndof = sum(j["dof"] for j in self.joints)

    # ------------------------------------------------------------- reset pose
    def default_angles(self):
        """Per-DOF default angle: 0 inside the limits, else the mid-range."""
        out = []
        for j in self.joints:
            for a in range(j["dof"]):
                lo, hi = j["lo"][a], j["hi"][a]
                out.append(0.0 if lo <= 0.0 <= hi else 0.5 * (lo + hi))
        return np.array(out, dtype=np.float64)

    def default_qp(self, angles=None, root_offset=None):
        """Reset state [nb][13] (p, q, v, w) for per-DOF angles (radians).

        ``root_offset`` (3,) is added to the first body's position when that
        body is a free root (the reset perturbation).
        """
        if angles is None:
            angles = self.default_angles()
        angles = np.asarray(angles, dtype=np.float64)
        R = [None] * self.nb
        p = [None] * self.nb
        dof0 = []
        acc = 0
        for j in self.joints:
            dof0.append(acc)
            acc += j["dof"]
        by_child = {j["child"]: (ji, j) for ji, j in enumerate(self.joints)}

        def place(b):
            if R[b] is not None:
                return
            if b not in by_child:
                R[b] = np.eye(3)
                pos = self.bodies[b]["position"]
                p[b] = np.zeros(3) if pos is None else pos.copy()
                return
            ji, j = by_child[b]
            place(j["parent"])
            th = np.zeros(3)
            th[:j["dof"]] = angles[dof0[ji]:dof0[ji] + j["dof"]]
            Rp = R[j["parent"]]
            R[b] = Rp @ j["frame_p"] @ euler_xyz(th) @ j["frame_c"].T
            p[b] = p[j["parent"]] + Rp @ j["anchor_p"] - R[b] @ j["anchor_c"]

        for b in range(self.nb):
            place(b)
        # lift every root tree without a given position to the clearance height
        def root_of(b):
            while b in self.parent_of:
                b = self.parent_of[b]
            return b
        roots = sorted({root_of(b) for b in range(self.nb)})
        for r in roots:
            if self.bodies[r]["position"] is not None:
                continue
            members = [b for b in range(self.nb) if root_of(b) == r]
            low = math.inf
            for (bi, c, rad) in self.contacts:
                if bi in members:
                    low = min(low, (p[bi] + R[bi] @ c)[2] - rad)
            if math.isfinite(low):
                for b in members:
                    p[b] = p[b] + np.array([0.0, 0.0, self.clearance - low])
        if root_offset is not None and 0 not in self.parent_of and self.bodies[0]["free_pos"].any():
            off = np.asarray(root_offset, dtype=np.float64)
            members = [b for b in range(self.nb) if root_of(b) == 0]
            for b in members:
                p[b] = p[b] + off
        X = np.zeros((self.nb, 13))
        for b in range(self.nb):
            X[b, 0:3] = p[b]
            X[b, 3:7] = mat_to_quat(R[b])
        return X

    # ------------------------------------------------------------- flat arrays
    def flat(self):
        """Field dict matching the C++ OrcSys struct."""
        f = {}
        f["nb"], f["nj"], f["nc"], f["na"], f["substeps"] = self.nb, self.nj, self.nc, self.na, self.substeps
        f["dt"], f["beta"], f["elasticity"], f["friction"] = self.dt, self.beta, self.elasticity, self.friction
        f["gravity"] = self.gravity
        f["mass"] = [b["mass"] for b in self.bodies]
        f["inertia"] = [b["inertia"] for b in self.bodies]
        f["free_pos"] = [b["free_pos"] for b in self.bodies]
        f["free_rot"] = [b["free_rot"] for b in self.bodies]
        f["c_body"] = [c[0] for c in self.contacts]
        f["c_local"] = [c[1] for c in self.contacts]
        f["c_radius"] = [c[2] for c in self.contacts]
        f["j_parent"] = [j["parent"] for j in self.joints]
        f["j_child"] = [j["child"] for j in self.joints]
        f["j_dof"] = [j["dof"] for j in self.joints]
        f["j_anchor_p"] = [j["anchor_p"] for j in self.joints]
        f["j_anchor_c"] = [j["anchor_c"] for j in self.joints]
        f["j_frame_p"] = [j["frame_p"].reshape(9) for j in self.joints]
        f["j_frame_c"] = [j["frame_c"].reshape(9) for j in self.joints]
        for k in ("k_lin", "c_lin", "k_ang", "c_ang", "k_lim"):
            f["j_" + k] = [j[k] for j in self.joints]
        f["j_lo"] = [j["lo"] for j in self.joints]
        f["j_hi"] = [j["hi"] for j in self.joints]
        f["a_joint"] = [a[0] for a in self.actions]
        f["a_axis"] = [a[1] for a in self.actions]
        f["a_gear"] = [a[2] for a in self.actions]
        f["a_mode"] = [a[3] for a in self.actions]
        f["np"] = self.np
        for k in ("a", "b", "kind", "ra", "rb"):
            f["p_" + k] = [p[k] for p in self.pairs]
        for k in ("a0", "a1", "b0", "b1", "ah", "bh"):
            f["p_" + k] = [p[k] for p in self.pairs]
        f["p_aR"] = [p["aR"].reshape(9) for p in self.pairs]
        f["p_bR"] = [p["bR"].reshape(9) for p in self.pairs]
        return f
