// Body-body contacts in FP32 (device code; also compiles for the host).
//
// The paper's collisions between colliders (Section 6.2) with the impulse of
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

// Parameter in [0, 1] of the point of segment a + u d closest to p; 0 for a
// zero-length segment.
BXF float seg_param(v3 p, v3 a, v3 d) {
  const float dd = dot(d, d);
  return dd > 0.f ? clampf(dot(p - a, d) / dd, 0.f, 1.f) : 0.f;
}

// Parameters (s, t) of the closest points of segments p0 + s d1 and q0 + t d2
// on [0, 1]^2: the unconstrained minimiser's s clamped, t from that s, and
// where t had to be clamped, s again from the clamped t.
BXF void seg_seg(v3 p0, v3 d1, v3 q0, v3 d2, float& s, float& t) {
  const v3 r = p0 - q0;
  const float a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
  if (!(a > 0.f)) {
    s = 0.f;
    t = e > 0.f ? clampf(f / e, 0.f, 1.f) : 0.f;
    return;
  }
  const float c = dot(d1, r);
  if (!(e > 0.f)) {
    t = 0.f;
    s = clampf(-c / a, 0.f, 1.f);
    return;
  }
  const float b = dot(d1, d2);
  const float den = a * e - b * b;
  s = den > 0.f ? clampf((b * f - c * e) / den, 0.f, 1.f) : 0.f;
  t = (b * s + f) / e;
  if (t < 0.f) {
    t = 0.f;
    s = clampf(-c / a, 0.f, 1.f);
  } else if (t > 1.f) {
    t = 1.f;
    s = clampf((b - c) / a, 0.f, 1.f);
  }
}

// Point p against the box with centre c, rotation Rb (box to world) and half
// extents h: the box point cb closest to p and the unit normal n from the box
// towards p; for p inside, the nearest face's point and outward normal.
// Returns the signed distance of p from the surface along n (negative inside).
// `face` returns -1 outside, else the nearest face's axis.
BXF float point_box(v3 p, v3 c, const m3& Rb, const float* h, v3& cb, v3& n, int& face) {
  const v3 q = mul_t(Rb, p - c);
  const bool inside = fabsf(q.x) <= h[0] && fabsf(q.y) <= h[1] && fabsf(q.z) <= h[2];
  if (!inside) {
    face = -1;
    cb = c + mul(Rb, V(clampf(q.x, -h[0], h[0]), clampf(q.y, -h[1], h[1]), clampf(q.z, -h[2], h[2])));
    const v3 d = p - cb;
    const float dist = sqrtf(dot(d, d));
    n = (1.f / dist) * d;
    return dist;
  }
  const float g0 = h[0] - fabsf(q.x), g1 = h[1] - fabsf(q.y), g2 = h[2] - fabsf(q.z);
  int k = 0;
  float g = g0;
  if (g1 < g) { k = 1; g = g1; }
  if (g2 < g) { k = 2; g = g2; }
  face = k;
  const float qk = k == 0 ? q.x : (k == 1 ? q.y : q.z);
  const float sg = qk >= 0.f ? 1.f : -1.f;
  v3 cl = q;
  if (k == 0) cl.x = sg * h[0];
  else if (k == 1) cl.y = sg * h[1];
  else cl.z = sg * h[2];
  cb = c + mul(Rb, cl);
  n = sg * col(Rb, k);
  return -g;
}

// Closest points of a candidate's features: ca on the first body, cb on the
// second, unit normal n from cb towards ca, and their distance along n
// (signed for a point against a box). Returns false where the normal is
// undefined (coincident core points).
BXF bool pair_geometry(const PairT& c, const PairSide& A, const PairSide& B, v3& ca, v3& cb, v3& n, float& dist) {
  if (c.kind >= PK_PB) {
    const bool box_b = c.kind == PK_PB;
    const PairSide& P = box_b ? A : B;  // the point's body
    const PairSide& X = box_b ? B : A;  // the box's body
    const v3 p = P.p + mul(P.R, ld3(box_b ? c.a0 : c.b0));
    const v3 bc = X.p + mul(X.R, ld3(box_b ? c.b0 : c.a0));
    const m3 Rb = mul(X.R, box_b ? c.bR : c.aR);
    v3 cbox, nb;
    int face;
    dist = point_box(p, bc, Rb, box_b ? c.bh : c.ah, cbox, nb, face);
    ca = box_b ? p : cbox;
    cb = box_b ? cbox : p;
    n = box_b ? nb : -nb;
    return true;
  }
  const v3 a0 = A.p + mul(A.R, ld3(c.a0)), b0 = B.p + mul(B.R, ld3(c.b0));
  float s = 0.f, t = 0.f;
  v3 da = V(0.f, 0.f, 0.f), db = V(0.f, 0.f, 0.f);
  if (c.kind == PK_SP || c.kind == PK_SS) da = mul(A.R, ld3(c.a1) - ld3(c.a0));
  if (c.kind == PK_PS || c.kind == PK_SS) db = mul(B.R, ld3(c.b1) - ld3(c.b0));
  if (c.kind == PK_PS) t = seg_param(a0, b0, db);
  else if (c.kind == PK_SP) s = seg_param(b0, a0, da);
  else if (c.kind == PK_SS) seg_seg(a0, da, b0, db, s, t);
  ca = a0 + s * da;
  cb = b0 + t * db;
  const v3 d = ca - cb;
  dist = sqrtf(dot(d, d));
  if (!(dist > 0.f)) return false;
  n = (1.f / dist) * d;
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

// One candidate. Returns whether an impulse applies; J is the impulse on the
// first body at the contact point x (the second body takes -J).
BXF bool pair_eval(const PairT& c, const TypeT& ty, const PairSide& A, const PairSide& B, v3& J, v3& x) {
  v3 ca, cb, n;
  float dist;
  if (!pair_geometry(c, A, B, ca, cb, n, dist)) return false;
  const float depth = (c.ra + c.rb) - dist;
  if (!(depth > 0.f)) return false;
  x = cb + (c.rb - 0.5f * depth) * n;  // the middle of the overlap
  const v3 rA = x - A.p, rB = x - B.p;
  const v3 u = (A.v + cross(A.w, rA)) - (B.v + cross(B.w, rB));
  const float vn = dot(u, n);
  const float num = ty.beta_h * depth - ty.one_plus_e * vn;
  if (!(num > 0.f)) return false;
  const float jn = num / pair_k(c, A, B, rA, rB, n);
  J = jn * n;
  const v3 ut = u - vn * n;
  const float sp = sqrtf(dot(ut, ut));
  if (sp > 0.f) {
    const v3 tt = (1.f / sp) * ut;
    const float stop = sp / pair_k(c, A, B, rA, rB, tt);
    const float cap = ty.mu * jn;
    const float jt = cap <= stop ? cap : stop;
    J = J - jt * tt;
  }
  return true;
}

// The velocity changes of an applied candidate: the first body's (dvA, dwA)
// and the second's (dvB, dwB).
BXF void pair_shares(const PairT& c, const PairSide& A, const PairSide& B, v3 J, v3 x, v3& dvA, v3& dwA, v3& dvB,
                     v3& dwB) {
  const v3 z3 = V(0.f, 0.f, 0.f);
  dvA = c.im_a * J;
  dvB = -(c.im_b * J);
  dwA = c.rot_a ? mul(A.Iwinv, cross(x - A.p, J)) : z3;
  dwB = c.rot_b ? -mul(B.Iwinv, cross(x - B.p, J)) : z3;
}

}  // namespace bx
