// Body-body contacts in FP32 (device code; also compiles for the host).
//
// The paper's collisions between colliders (Section 7.2) with the impulse of
// its ground contact: each candidate pairs a core feature of the first body
// (a point, a segment, or a box; plus a radius) with one of the second body.
// The closest points of the two features give the normal n (from the second
// body towards the first) and the depth ra + rb - distance; where the depth is
// positive, the velocity-level normal impulse with restitution and Baumgarte
// term acts on the relative velocity at the middle of the overlap, with a
// Coulomb friction impulse from the same state. The first body takes +J, the
// second -J. A body whose translations (rotations) are all frozen has no
// inverse mass (inertia) here.
#pragma once
#include "bx_phys.h"

namespace bx {

// One side of a candidate: a body's post-kinematic state and frame.
struct PairSide {
  v3 p, v, w;
  m3 R;
  s3 Iwinv;
};

// Lane-varying choices between two values are made field by field on
// copies, never by choosing between the addresses of two locals (which would
// move them to scratch memory).
BXF v3 sel(bool c, v3 a, v3 b) { return V(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z); }
BXF m3 sel(bool c, const m3& a, const m3& b) {
  m3 r;
  for (int i = 0; i < 9; ++i) r.m[i] = c ? a.m[i] : b.m[i];
  return r;
}
BXF s3 sel(bool c, const s3& a, const s3& b) {
  return s3{c ? a.xx : b.xx, c ? a.yy : b.yy, c ? a.zz : b.zz, c ? a.xy : b.xy, c ? a.xz : b.xz, c ? a.yz : b.yz};
}
BXF PairSide sel(bool c, const PairSide& a, const PairSide& b) {
  return PairSide{sel(c, a.p, b.p), sel(c, a.v, b.v), sel(c, a.w, b.w), sel(c, a.R, b.R), sel(c, a.Iwinv, b.Iwinv)};
}

// Closest features of a candidate and what their adjoint needs.
struct PairGeo {
  v3 ca, cb, n;        // closest point on the first body, on the second, unit normal (second -> first)
  float dist;          // their distance along n (signed for a point against a box)
  // point / segment kinds: the first side a0 + s da, the second b0 + t db (world)
  v3 a0, da, b0, db;
  float s, t;          // closest-point parameters
  float sraw, traw;    // before clamping
  float a, b, c, e, f, den;  // segment-segment quadratic
  int kase;            // segment-segment case (see seg_seg)
  // point-box kinds
  v3 p, bc, q, cl, nbx;  // point, box centre, box coordinates of p, closest box point in them, box normal
  m3 Rb;                 // box rotation (box to world)
  int face;              // -1: p outside the box, else the nearest face's axis
  float sg;              // that face's side (+1 / -1)
  // segment-box kinds: the segment a0 + s da in box coordinates q0s + s dqs,
  // the parameter of its point nearest the box and how it was found
  v3 q0s, dqs;
  float sst;             // that parameter
  int sbin;              // 0: the segment stays outside the box, 1: it reaches it
  int act;               // outside: coordinates beyond their face at the minimiser (bit k)
  v3 sig;                // their sides (+1 / -1)
  float sD;              // outside: sum of dqs_k^2 over those coordinates
  int li, lj;            // inside: the two lines +-q_k - h_k crossing at the parameter (-1: an end)
};

// Parameter in [0, 1] of the point of segment a + u d closest to p; 0 for a
// zero-length segment. raw: the value before clamping.
BXF float seg_param(v3 p, v3 a, v3 d, float& raw) {
  const float dd = dot(d, d);
  raw = dd > 0.f ? dot(p - a, d) / dd : 0.f;
  return dd > 0.f ? clampf(raw, 0.f, 1.f) : 0.f;
}

// Parameters (s, t) of the closest points of segments p0 + s d1 and q0 + t d2
// on [0, 1]^2: the unconstrained minimiser's s clamped, t from that s, and
// where t had to be clamped, s again from the clamped t. Cases: 0 first
// segment of zero length, 1 second of zero length, 2 t inside [0, 1], 3 t
// clamped to 0, 4 t clamped to 1.
BXF void seg_seg(v3 p0, v3 d1, v3 q0, v3 d2, PairGeo& g) {
  const v3 r = p0 - q0;
  g.a = dot(d1, d1);
  g.e = dot(d2, d2);
  g.f = dot(d2, r);
  g.c = dot(d1, r);
  g.b = dot(d1, d2);
  g.den = 0.f;
  if (!(g.a > 0.f)) {
    g.kase = 0;
    g.s = g.sraw = 0.f;
    g.traw = g.e > 0.f ? g.f / g.e : 0.f;
    g.t = g.e > 0.f ? clampf(g.traw, 0.f, 1.f) : 0.f;
    return;
  }
  if (!(g.e > 0.f)) {
    g.kase = 1;
    g.t = g.traw = 0.f;
    g.sraw = -g.c / g.a;
    g.s = clampf(g.sraw, 0.f, 1.f);
    return;
  }
  g.den = g.a * g.e - g.b * g.b;
  g.sraw = g.den > 0.f ? (g.b * g.f - g.c * g.e) / g.den : 0.f;
  g.s = clampf(g.sraw, 0.f, 1.f);
  g.traw = (g.b * g.s + g.f) / g.e;
  g.kase = 2;
  g.t = g.traw;
  if (g.traw < 0.f) {
    g.kase = 3;
    g.t = 0.f;
    g.sraw = -g.c / g.a;
    g.s = clampf(g.sraw, 0.f, 1.f);
  } else if (g.traw > 1.f) {
    g.kase = 4;
    g.t = 1.f;
    g.sraw = (g.b - g.c) / g.a;
    g.s = clampf(g.sraw, 0.f, 1.f);
  }
}

// Point p against the box with centre c, rotation Rb (box to world) and half
// extents h: the box point cb closest to p and the unit normal n from the box
// towards p; for p inside, the nearest face's point and outward normal.
// Returns the signed distance of p from the surface along n (negative inside).
BXF float point_box(v3 p, v3 c, const m3& Rb, const float* h, PairGeo& g) {
  const v3 q = mul_t(Rb, p - c);
  g.q = q;
  const bool inside = fabsf(q.x) <= h[0] && fabsf(q.y) <= h[1] && fabsf(q.z) <= h[2];
  if (!inside) {
    g.face = -1;
    g.cl = V(clampf(q.x, -h[0], h[0]), clampf(q.y, -h[1], h[1]), clampf(q.z, -h[2], h[2]));
    const v3 cb = c + mul(Rb, g.cl);
    const v3 d = p - cb;
    const float dist = sqrtf(dot(d, d));
    g.nbx = (1.f / dist) * d;
    g.cb = cb;
    return dist;
  }
  const float g0 = h[0] - fabsf(q.x), g1 = h[1] - fabsf(q.y), g2 = h[2] - fabsf(q.z);
  int k = 0;
  float gk = g0;
  if (g1 < gk) { k = 1; gk = g1; }
  if (g2 < gk) { k = 2; gk = g2; }
  g.face = k;
  const float qk = k == 0 ? q.x : (k == 1 ? q.y : q.z);
  g.sg = qk >= 0.f ? 1.f : -1.f;
  v3 cl = q;
  if (k == 0) cl.x = g.sg * h[0];
  else if (k == 1) cl.y = g.sg * h[1];
  else cl.z = g.sg * h[2];
  g.cl = cl;
  g.cb = c + mul(Rb, cl);
  // column k of Rb, chosen by value (k varies across lanes)
  const v3 ck = sel(k == 0, col(Rb, 0), sel(k == 1, col(Rb, 1), col(Rb, 2)));
  g.nbx = g.sg * ck;
  return -gk;
}

// The parameter s in [0, 1] of the point of segment a0 + s da nearest the
// box (centre c, rotation Rb box to world, half extents h); in box
// coordinates the segment is q(s) = q0 + s dq. Outside the box the squared
// distance sum_k max(|q_k| - h_k, 0)^2 is convex: its smallest minimiser is
// the smallest candidate (the ends and the parameters where some |q_k| =
// h_k) where half its slope, sum_k (q_k - clamp q_k) dq_k, is >= 0, or the
// zero of that slope on the piece before it, where the coordinates beyond
// their faces are fixed and the slope is linear: s = -N / D with
// N = sum (q0_k - sg_k h_k) dq_k, D = sum dq_k^2 over them. Where the
// segment passes through the box (the parameters with every |q_k| < h_k
// form an interval of positive length) the deepest point is taken instead:
// the smallest of max_k (|q_k| - h_k) over the ends and the crossings of two
// of the six lines +-q_k(s) - h_k (the smallest s on ties).
BXF float seg_box_param(v3 a0, v3 da, v3 c, const m3& Rb, const float* h, PairGeo& g) {
  const v3 q0 = mul_t(Rb, a0 - c), dq = mul_t(Rb, da);
  g.q0s = q0;
  g.dqs = dq;
  const float qa[3] = {q0.x, q0.y, q0.z}, qd[3] = {dq.x, dq.y, dq.z};
  // straight-line code (selects, no branches) up to the through-box test:
  // the lanes of a wavefront take it together
  float sL = -1.f, sR = 2.f;
  auto consider = [&](float s) {
    float f = 0.f;
    for (int k = 0; k < 3; ++k) {
      const float q = qa[k] + s * qd[k];
      f += (q - clampf(q, -h[k], h[k])) * qd[k];
    }
    const bool up = f >= 0.f;
    sR = up ? fminf(sR, s) : sR;
    sL = (!up && s > sL) ? s : sL;
  };
  consider(0.f);
  consider(1.f);
  // the face crossings t1, t2 of each coordinate; one that does not move
  // (dq_k = 0) gives infinite or undefined crossings, which clamp to an end
  // already considered or fail every comparison (no change), and leave the
  // through-box interval below unbounded (|q_k| < h_k) or empty
  float t1[3], t2[3];
  float te = 0.f, tx = 1.f;
  for (int k = 0; k < 3; ++k) {
    t1[k] = (-h[k] - qa[k]) / qd[k];
    t2[k] = (h[k] - qa[k]) / qd[k];
    te = fmaxf(te, fminf(t1[k], t2[k]));
    tx = fminf(tx, fmaxf(t1[k], t2[k]));
  }
  g.sbin = 0;
  g.li = g.lj = -1;
  g.act = 0;
  g.sig = V(0.f, 0.f, 0.f);
  g.sD = 0.f;
  // the slope's signs at the ends decide an end as the minimiser (it is
  // >= 0 at 0, or < 0 at 1), unless the segment passes through the box;
  // the other candidates then change neither sL nor sR
  if (!(te < tx) && (sL < 0.f || sR > 1.f)) return sR > 1.f ? 1.f : sR;
  for (int k = 0; k < 3; ++k) {
    consider(clampf(t2[k], 0.f, 1.f));
    consider(clampf(t1[k], 0.f, 1.f));
  }
  // outside: the minimiser on the bracket [sL, sR], from the coordinates
  // beyond their faces at its middle
  const float mid = 0.5f * (sL + sR);
  float N = 0.f, D = 0.f, sg[3];
  int act = 0;
  for (int k = 0; k < 3; ++k) {
    const float q = qa[k] + mid * qd[k];
    const bool out = fabsf(q) > h[k];
    const float sk = q >= 0.f ? 1.f : -1.f;
    sg[k] = out ? sk : 0.f;
    N += out ? (qa[k] - sk * h[k]) * qd[k] : 0.f;
    D += out ? qd[k] * qd[k] : 0.f;
    act |= out ? 1 << k : 0;
  }
  const bool bracket = !(sR > 1.f) && !(sL < 0.f);
  const float s = sR > 1.f ? 1.f : (sL < 0.f ? sR : (D > 0.f ? clampf(-N / D, sL, sR) : sR));
  g.act = bracket ? act : 0;
  g.sig = bracket ? V(sg[0], sg[1], sg[2]) : V(0.f, 0.f, 0.f);
  g.sD = bracket ? D : 0.f;
  // does the segment pass through the box? (the parameters with every
  // |q_k(s)| < h_k form an interval of positive length)
  if (!(te < tx)) return s;
  // it does: its deepest point
  g.sbin = 1;
  g.act = 0;
  auto depth_at = [&](float t) {
    float m = fabsf(qa[0] + t * qd[0]) - h[0];
    m = fmaxf(m, fabsf(qa[1] + t * qd[1]) - h[1]);
    return fmaxf(m, fabsf(qa[2] + t * qd[2]) - h[2]);
  };
  float bs = 0.f, bv = depth_at(0.f);
  {
    const float v1 = depth_at(1.f);
    if (v1 < bv) {
      bs = 1.f;
      bv = v1;
    }
  }
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j) {
      const float si = (i & 1) ? -1.f : 1.f, sj = (j & 1) ? -1.f : 1.f;
      const float bi = si * qd[i >> 1], bj = sj * qd[j >> 1];
      if (bi == bj) continue;
      const float ai = si * qa[i >> 1] - h[i >> 1], aj = sj * qa[j >> 1] - h[j >> 1];
      const float t = (aj - ai) / (bi - bj);
      if (!(t > 0.f && t < 1.f)) continue;
      const float v = depth_at(t);
      if (v < bv || (v == bv && t < bs)) {
        bs = t;
        bv = v;
        g.li = i;
        g.lj = j;
      }
    }
  if (bs == 0.f || bs == 1.f) g.li = g.lj = -1;
  return bs;
}

// Closest points of a candidate's features: ca on the first body, cb on the
// second, unit normal n from cb towards ca, and their distance along n
// (signed for a point against a box). Returns false where the normal is
// undefined (coincident core points).
BXF bool pair_geometry(const PairT& c, const PairSide& A, const PairSide& B, PairGeo& g) {
  if (c.kind >= PK_PB) {
    // a point (PB, BP) or a capsule's axis segment (SB, BS) against a box,
    // whose body is the second for PB and SB: the segment is a candidate
    // only where its point nearest the box lies strictly between its ends
    // (the ends are the capsule's end-sphere candidates), and that point is
    // then taken as a point candidate; both kinds share the point-box part
    const bool seg = c.kind >= PK_SB;
    const bool box_b = c.kind == PK_PB || c.kind == PK_SB;
    const m3 SR = sel(box_b, A.R, B.R), XR = sel(box_b, B.R, A.R);
    const v3 o0 = ld3(box_b ? c.a0 : c.b0);
    g.a0 = sel(box_b, A.p, B.p) + mul(SR, o0);
    g.bc = sel(box_b, B.p, A.p) + mul(XR, ld3(box_b ? c.b0 : c.a0));
    if (c.box_rot)
      g.Rb = mul(XR, box_b ? c.bR : c.aR);
    else
      g.Rb = XR;
    const float* h = box_b ? c.bh : c.ah;
    g.p = g.a0;
    if (seg) {
      g.da = mul(SR, ld3(box_b ? c.a1 : c.b1) - o0);
      g.sst = seg_box_param(g.a0, g.da, g.bc, g.Rb, h, g);
      if (!(g.sst > 0.f && g.sst < 1.f)) return false;
      g.p = g.a0 + g.sst * g.da;
    }
    g.dist = point_box(g.p, g.bc, g.Rb, h, g);
    const v3 cbox = g.cb;
    g.ca = sel(box_b, g.p, cbox);
    g.cb = sel(box_b, cbox, g.p);
    g.n = sel(box_b, g.nbx, -g.nbx);
    return true;
  }
  g.a0 = A.p + mul(A.R, ld3(c.a0));
  g.b0 = B.p + mul(B.R, ld3(c.b0));
  g.s = g.t = g.sraw = g.traw = 0.f;
  g.da = g.db = V(0.f, 0.f, 0.f);
  if (c.kind == PK_SP || c.kind == PK_SS) g.da = mul(A.R, ld3(c.a1) - ld3(c.a0));
  if (c.kind == PK_PS || c.kind == PK_SS) g.db = mul(B.R, ld3(c.b1) - ld3(c.b0));
  if (c.kind == PK_PS) g.t = seg_param(g.a0, g.b0, g.db, g.traw);
  else if (c.kind == PK_SP) g.s = seg_param(g.b0, g.a0, g.da, g.sraw);
  else if (c.kind == PK_SS) seg_seg(g.a0, g.da, g.b0, g.db, g);
  g.ca = g.a0 + g.s * g.da;
  g.cb = g.b0 + g.t * g.db;
  const v3 d = g.ca - g.cb;
  g.dist = sqrtf(dot(d, d));
  if (!(g.dist > 0.f)) return false;
  g.n = (1.f / g.dist) * d;
  return true;
}

// Effective inverse mass of the candidate along unit direction u at lever
// arms rA, rB: imA + imB + (rA x u) . IwA^-1 (rA x u) + (rB x u) . IwB^-1 (rB x u).
BXF float pair_k(const PairT& c, const PairSide& A, const PairSide& B, v3 rA, v3 rB, v3 u) {
  const v3 za = cross(rA, u), zb = cross(rB, u);
  float k = c.im_a + c.im_b;
  if (c.rot_a) k += dot(za, mul(A.Iwinv, za));
  if (c.rot_b) k += dot(zb, mul(B.Iwinv, zb));
  return k;
}

// The impulse of a candidate and what its adjoint needs.
struct PairImp {
  float depth, vn, num, kn, jn, sp, kt, stop, jt;
  v3 x, rA, rB, u, t, J;  // contact point, lever arms, relative velocity, slip direction, impulse on the first body
  bool use_cap;           // the Coulomb cap is the applied friction impulse
};

// Returns whether an impulse applies: depth > 0 and a positive normal
// impulse. Needs pair_geometry's result.
BXF bool pair_impulse(const PairT& c, const TypeT& ty, const PairSide& A, const PairSide& B, const PairGeo& g,
                      PairImp& m) {
  m.depth = (c.ra + c.rb) - g.dist;
  if (!(m.depth > 0.f)) return false;
  m.x = g.cb + (c.rb - 0.5f * m.depth) * g.n;  // the middle of the overlap
  m.rA = m.x - A.p;
  m.rB = m.x - B.p;
  m.u = (A.v + cross(A.w, m.rA)) - (B.v + cross(B.w, m.rB));
  m.vn = dot(m.u, g.n);
  m.num = ty.beta_h * m.depth - ty.one_plus_e * m.vn;
  if (!(m.num > 0.f)) return false;
  m.kn = pair_k(c, A, B, m.rA, m.rB, g.n);
  m.jn = m.num / m.kn;
  m.J = m.jn * g.n;
  const v3 ut = m.u - m.vn * g.n;
  m.sp = sqrtf(dot(ut, ut));
  m.t = V(0.f, 0.f, 0.f);
  m.kt = m.stop = m.jt = 0.f;
  m.use_cap = false;
  if (m.sp > 0.f) {
    m.t = (1.f / m.sp) * ut;
    m.kt = pair_k(c, A, B, m.rA, m.rB, m.t);
    m.stop = m.sp / m.kt;
    const float cap = ty.mu * m.jn;
    m.use_cap = cap <= m.stop;
    m.jt = m.use_cap ? cap : m.stop;
    m.J = m.J - m.jt * m.t;
  }
  return true;
}

// The velocity changes of an applied candidate: the first body's (dvA, dwA)
// and the second's (dvB, dwB).
BXF void pair_shares(const PairT& c, const PairSide& A, const PairSide& B, const PairImp& m, v3& dvA, v3& dwA,
                     v3& dvB, v3& dwB) {
  const v3 z3 = V(0.f, 0.f, 0.f);
  dvA = c.im_a * m.J;
  dvB = -(c.im_b * m.J);
  dwA = c.rot_a ? mul(A.Iwinv, cross(m.rA, m.J)) : z3;
  dwB = c.rot_b ? -mul(B.Iwinv, cross(m.rB, m.J)) : z3;
}

// One candidate: whether an impulse applies and, if so, the shares.
BXF bool pair_eval(const PairT& c, const TypeT& ty, const PairSide& A, const PairSide& B, v3& dvA, v3& dwA, v3& dvB,
                   v3& dwB) {
  PairGeo g;
  PairImp m;
  if (!pair_geometry(c, A, B, g) || !pair_impulse(c, ty, A, B, g, m)) return false;
  pair_shares(c, A, B, m, dvA, dwA, dvB, dwB);
  return true;
}

}  // namespace bx
