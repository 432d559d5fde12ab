// Per-item physics of one substep in FP32 (device code; also compiles for the
// host). Each function is one item of Algorithm 1 (Section 3): a body's
// kinematic update, a joint's spring update with its actuators, one
// ground-contact candidate, a body's potential and collision updates.
//
// Frames: world z up, ground plane z = 0. Quaternions (w, x, y, z), Hamilton
// product, body to world. Velocities and angular velocities in the world frame.
#pragma once
#include <math.h>

#include "bx_tables.h"

#define BXF __host__ __device__ __forceinline__

namespace bx {

struct v3 {
  float x, y, z;
};
struct q4 {
  float w, x, y, z;
};
struct m3 {
  float m[9];  // row-major
};
// symmetric 3x3: xx, yy, zz, xy, xz, yz
struct s3 {
  float xx, yy, zz, xy, xz, yz;
};

BXF v3 V(float x, float y, float z) { return v3{x, y, z}; }
BXF v3 operator+(v3 a, v3 b) { return v3{a.x + b.x, a.y + b.y, a.z + b.z}; }
BXF v3 operator-(v3 a, v3 b) { return v3{a.x - b.x, a.y - b.y, a.z - b.z}; }
BXF v3 operator-(v3 a) { return v3{-a.x, -a.y, -a.z}; }
BXF v3 operator*(float s, v3 a) { return v3{s * a.x, s * a.y, s * a.z}; }
BXF v3& operator+=(v3& a, v3 b) { a = a + b; return a; }
BXF v3& operator-=(v3& a, v3 b) { a = a - b; return a; }
BXF float dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
BXF v3 cross(v3 a, v3 b) { return v3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
BXF v3 ld3(const float* p) { return v3{p[0], p[1], p[2]}; }

BXF v3 mul(const m3& A, v3 v) {
  return v3{A.m[0] * v.x + A.m[1] * v.y + A.m[2] * v.z, A.m[3] * v.x + A.m[4] * v.y + A.m[5] * v.z,
            A.m[6] * v.x + A.m[7] * v.y + A.m[8] * v.z};
}
BXF v3 mul_t(const m3& A, v3 y) {  // A^T y
  return v3{A.m[0] * y.x + A.m[3] * y.y + A.m[6] * y.z, A.m[1] * y.x + A.m[4] * y.y + A.m[7] * y.z,
            A.m[2] * y.x + A.m[5] * y.y + A.m[8] * y.z};
}
BXF v3 mul(const s3& S, v3 v) {
  return v3{S.xx * v.x + S.xy * v.y + S.xz * v.z, S.xy * v.x + S.yy * v.y + S.yz * v.z,
            S.xz * v.x + S.yz * v.y + S.zz * v.z};
}
BXF m3 mul(const m3& A, const float* B) {  // A * B, B row-major constant
  m3 C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.m[3 * i + j] = A.m[3 * i] * B[j] + A.m[3 * i + 1] * B[3 + j] + A.m[3 * i + 2] * B[6 + j];
  return C;
}
BXF v3 col(const m3& A, int j) { return v3{A.m[j], A.m[3 + j], A.m[6 + j]}; }

BXF q4 qmul(q4 a, q4 b) {
  return q4{a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
            a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

// Rotation matrix of a unit quaternion (body to world).
BXF m3 quat_to_mat(q4 q) {
  // products with the doubled components (exact doubling)
  const float x2 = q.x + q.x, y2 = q.y + q.y, z2 = q.z + q.z;
  const float xx = q.x * x2, yy = q.y * y2, zz = q.z * z2;
  const float xy = q.x * y2, xz = q.x * z2, yz = q.y * z2;
  const float wx = q.w * x2, wy = q.w * y2, wz = q.w * z2;
  m3 R;
  R.m[0] = 1.f - (yy + zz); R.m[1] = xy - wz;         R.m[2] = xz + wy;
  R.m[3] = xy + wz;         R.m[4] = 1.f - (xx + zz); R.m[5] = yz - wx;
  R.m[6] = xz - wy;         R.m[7] = yz + wx;         R.m[8] = 1.f - (xx + yy);
  return R;
}

// R diag(d) R^T
BXF s3 rot_diag(const m3& R, const float* d) {
  float a0 = R.m[0] * d[0], a1 = R.m[1] * d[1], a2 = R.m[2] * d[2];
  float b0 = R.m[3] * d[0], b1 = R.m[4] * d[1], b2 = R.m[5] * d[2];
  float c0 = R.m[6] * d[0], c1 = R.m[7] * d[1], c2 = R.m[8] * d[2];
  s3 S;
  S.xx = a0 * R.m[0] + a1 * R.m[1] + a2 * R.m[2];
  S.yy = b0 * R.m[3] + b1 * R.m[4] + b2 * R.m[5];
  S.zz = c0 * R.m[6] + c1 * R.m[7] + c2 * R.m[8];
  S.xy = a0 * R.m[3] + a1 * R.m[4] + a2 * R.m[5];
  S.xz = a0 * R.m[6] + a1 * R.m[7] + a2 * R.m[8];
  S.yz = b0 * R.m[6] + b1 * R.m[7] + b2 * R.m[8];
  return S;
}

// Frozen axes: select (not multiply), so NaN/Inf in a frozen component do
// not leak and a frozen component is exactly zero.
BXF v3 keep(v3 a, const float* f) {
  return v3{f[0] != 0.f ? a.x : 0.f, f[1] != 0.f ? a.y : 0.f, f[2] != 0.f ? a.z : 0.f};
}
// v + keep(h x) with one rounding: the frozen components keep v exactly.
BXF v3 keep_fma(v3 v, float h, v3 x, const float* f) {
  return v3{f[0] != 0.f ? fmaf(h, x.x, v.x) : v.x, f[1] != 0.f ? fmaf(h, x.y, v.y) : v.y,
            f[2] != 0.f ? fmaf(h, x.z, v.z) : v.z};
}
BXF float clampf(float x, float lo, float hi) { return x < lo ? lo : (x > hi ? hi : x); }

// atan2 for the joint angles. The octant reduction t = min(|x|,|y|) /
// max(|x|,|y|) in [0, 1] is followed by atan t = t P(t^2), P of degree 7 fitted
// (minimax, in absolute error) to atan on [0, 1], then by the reflections
// pi/2 - r, pi - r and the sign of y. Absolute error about 1.2e-7 rad in FP32;
// atan2(+-0, -0) = +-pi and atan2(+-0, +0) = +-0 as in C.
BXF float atan2_poly(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
  const float t = mx > 0.f ? mn * (1.f / mx) : 0.f;
  const float u = t * t;
  float p = -4.054381535e-3f;
  p = p * u + 2.186222805e-2f;
  p = p * u - 5.591116410e-2f;
  p = p * u + 9.642101199e-2f;
  p = p * u - 1.390858575e-1f;
  p = p * u + 1.994655492e-1f;
  p = p * u - 3.332985952e-1f;
  p = p * u + 9.999993351e-1f;
  float r = p * t;
  r = ay > ax ? 1.57079637f - r : r;
  r = signbit(x) ? 3.14159274f - r : r;
  return copysignf(r, y);
}

struct Body {
  v3 p;
  q4 q;
  v3 v, w;
};

// Derived per-body quantities of one substep.
struct Frame {
  m3 R;       // orientation
  s3 Iw;      // world inertia R diag(I) R^T
  s3 Iwinv;   // its inverse R diag(1/I) R^T
};

// Kinematic integrator (Algorithm 1, first line): frozen axes hold zero
// velocity; p += h v; q <- normalize(q + h/2 (0, w) (x) q).
// The kinematic update for a state whose frozen velocity components are
// already zero (the integrators below keep them zero).
BXF void kinematic_unmasked(Body& s, float h) {
  s.p = s.p + h * s.v;
  // (0, w) (x) q written out: the product with a pure quaternion has no
  // terms in its zero real part
  const float hh = 0.5f * h;
  const v3 w = V(hh * s.w.x, hh * s.w.y, hh * s.w.z);
  const q4 a = s.q;
  const q4 q{a.w - (w.x * a.x + w.y * a.y + w.z * a.z), a.x + (w.x * a.w + w.y * a.z - w.z * a.y),
             a.y + (w.y * a.w - w.x * a.z + w.z * a.x), a.z + (w.z * a.w + w.x * a.y - w.y * a.x)};
  float inv = 1.f / sqrtf(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
  s.q = q4{q.w * inv, q.x * inv, q.y * inv, q.z * inv};
}
BXF void kinematic(const BodyT& B, Body& s, float h) {
  s.v = keep(s.v, B.free_p);
  s.w = keep(s.w, B.free_r);
  kinematic_unmasked(s, h);
}

BXF Frame derive(const BodyT& B, const Body& s) {
  Frame f;
  f.R = quat_to_mat(s.q);
  f.Iw = rot_diag(f.R, B.I);
  f.Iwinv = rot_diag(f.R, B.Iinv);
  return f;
}
// The frame from a given rotation without the world inertia, which the
// forward step does not use (Iw is left zero).
BXF Frame derive_inv(const BodyT& B, const m3& R) {
  Frame f;
  f.R = R;
  f.Iw = s3{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  f.Iwinv = rot_diag(R, B.Iinv);
  return f;
}

// Joint geometry shared by a joint's spring update and its actuators: the
// anchors relative to each centre of mass, the joint-frame axes in world
// coordinates, and the intrinsic X-Y-Z Euler angles of the child's joint frame
// relative to the parent's (M = AwP^T AwC = Rx Ry Rz) with their axes
// (parent x, intermediate y, child z).
struct JointGeo {
  v3 rP, rC;
  v3 e1P, e2P, e3P, e1C, e2C, e3C;
  float m12, m22, m01, m00, m02;
  float c1, s1;
  float th[3];
  v3 ax[3];
};

// The child's side of the geometry, which needs no parent data: its anchor
// offset, its joint-frame axes and its anchor velocity.
struct JointChild {
  v3 rC, uC, e1C, e2C, e3C;
};

template <int MAXDOF>
BXF JointChild joint_child(const JointT& J, const Body& C, const m3& RC) {
  JointChild c;
  c.rC = mul(RC, ld3(J.ac));
  m3 AwC = mul(RC, J.FC);
  c.e1C = col(AwC, 0);
  c.e2C = MAXDOF > 1 ? col(AwC, 1) : V(0.f, 0.f, 0.f);
  c.e3C = col(AwC, 2);
  c.uC = C.v + cross(C.w, c.rC);
  return c;
}

template <int MAXDOF>
BXF JointGeo joint_geo(const JointT& J, const m3& RP, const JointChild& c) {
  JointGeo g;
  g.rP = mul(RP, ld3(J.ap));
  g.rC = c.rC;
  m3 AwP = mul(RP, J.FP);
  g.e1P = col(AwP, 0);
  g.e2P = col(AwP, 1);
  g.e3P = col(AwP, 2);
  g.e1C = c.e1C;
  g.e3C = c.e3C;
  g.m12 = dot(g.e2P, g.e3C);
  g.m22 = dot(g.e3P, g.e3C);
  g.th[0] = atan2_poly(-g.m12, g.m22);
  float r = sqrtf(g.m12 * g.m12 + g.m22 * g.m22);
  g.c1 = 1.f;
  g.s1 = 0.f;
  if (r > 0.f) {
    g.c1 = g.m22 / r;
    g.s1 = -g.m12 / r;
  }
  g.ax[0] = g.e1P;
  g.ax[1] = g.c1 * g.e2P + g.s1 * g.e3P;
  g.ax[2] = g.e3C;
  if (MAXDOF > 1) {
    g.e2C = c.e2C;
    g.m01 = dot(g.e1P, g.e2C);
    g.m00 = dot(g.e1P, g.e1C);
    g.m02 = dot(g.e1P, g.e3C);
    g.th[1] = asinf(clampf(g.m02, -1.f, 1.f));
    g.th[2] = atan2_poly(-g.m01, g.m00);
  }
  return g;
}

// The geometry the step itself needs (joint_eval). For one-axis joints only
// e1P, the angle th1 and its axis are used: m12 = e2P.e3C and m22 = e3P.e3C
// are taken as the parent joint frame's y and z columns against RP^T e3C,
// without forming e2P and e3P. The fields the step does not read are left
// unset on that path (the adjoint takes joint_geo).
template <int MAXDOF>
BXF JointGeo joint_geo_step(const JointT& J, const m3& RP, const JointChild& c) {
  if (MAXDOF > 1) return joint_geo<MAXDOF>(J, RP, c);
  JointGeo g;
  g.rP = mul(RP, ld3(J.ap));
  g.rC = c.rC;
  g.e1P = mul(RP, V(J.FP[0], J.FP[3], J.FP[6]));
  g.e1C = c.e1C;
  g.e3C = c.e3C;
  const v3 v = mul_t(RP, c.e3C);
  g.m12 = J.FP[1] * v.x + J.FP[4] * v.y + J.FP[7] * v.z;
  g.m22 = J.FP[2] * v.x + J.FP[5] * v.y + J.FP[8] * v.z;
  g.th[0] = atan2_poly(-g.m12, g.m22);
  g.ax[0] = g.e1P;
  return g;
}

template <int MAXDOF>
BXF JointGeo joint_geo(const JointT& J, const m3& RP, const m3& RC) {
  Body none;
  none.v = none.w = V(0.f, 0.f, 0.f);
  return joint_geo<MAXDOF>(J, RP, joint_child<MAXDOF>(J, none, RC));
}

// Spring joint (Section 7.1) from the parent's and the child's
// post-kinematic state. Force/torque on the child (fc, tc) and on the parent
// (fp, tp):
//   anchor spring-damper  F = k_lin (xP - xC) + c_lin (uP - uC), at each anchor;
//   alignment spring      1 DOF: k_ang e1C x e1P; 2 DOF: -k_ang (e1P.e2C) e2C x e1P;
//   angular damper        c_ang (wP - wC);
//   limit springs         -k_lim (th_k - clamp(th_k)) about Euler axis k < dof.
struct JointOut {
  v3 fc, tc, fp, tp;
  v3 tpn;  // -tp: a gather that subtracts it needs no negation
};

template <int MAXDOF>
BXF v3 joint_spring(const JointT& J, const Body& P, const Body& C, const JointGeo& g, v3 uC, v3& F) {
  v3 d = (P.p - C.p) + (g.rP - g.rC);
  v3 uP = P.v + cross(P.w, g.rP);
  F = J.k_lin * d + J.c_lin * (uP - uC);
  v3 tau;
  if (MAXDOF == 1 || J.dof == 1)
    tau = J.k_ang * cross(g.e1C, g.e1P);
  else if (J.dof == 2)
    tau = (-J.k_ang * g.m01) * cross(g.e2C, g.e1P);
  else
    tau = V(0.f, 0.f, 0.f);
  tau += J.c_ang * (P.w - C.w);
  for (int k = 0; k < MAXDOF; ++k)
    if (MAXDOF == 1 || k < J.dof) tau += (-J.k_lim * (g.th[k] - clampf(g.th[k], J.lo[k], J.hi[k]))) * g.ax[k];
  return tau;
}
template <int MAXDOF>
BXF v3 joint_spring(const JointT& J, const Body& P, const Body& C, const JointGeo& g, v3& F) {
  return joint_spring<MAXDOF>(J, P, C, g, C.v + cross(C.w, g.rC), F);
}

// Actuators of a joint (Algorithm 1, actuator loop): about Euler axis k, on
// the child (and its opposite on the parent), a torque gear_k a_k, or for a
// target-angle actuator gear_k (a_k - theta_k); act_pd selects the second.
template <int MAXDOF>
BXF v3 joint_actuator(const JointT& J, const JointGeo& g, const float* a) {
  v3 tau = (J.gear[0] * (a[0] - J.act_pd[0] * g.th[0])) * g.ax[0];
  for (int k = 1; k < MAXDOF; ++k)
    if (k < J.dof) tau += (J.gear[k] * (a[k] - J.act_pd[k] * g.th[k])) * g.ax[k];
  return tau;
}

// Spring and actuators together (the fused path), from the child's side
// computed beforehand.
template <int MAXDOF>
BXF JointOut joint_eval(const JointT& J, const Body& P, const m3& RP, const Body& C, const JointChild& c,
                        const float* a /* clipped actions per axis, 0 if none */) {
  JointGeo g = joint_geo_step<MAXDOF>(J, RP, c);
  v3 F;
  v3 tau = joint_spring<MAXDOF>(J, P, C, g, c.uC, F) + joint_actuator<MAXDOF>(J, g, a);
  JointOut o;
  o.fc = F;
  o.tc = cross(g.rC, F) + tau;
  o.fp = -F;
  o.tpn = cross(g.rP, F) + tau;
  o.tp = -o.tpn;
  return o;
}
template <int MAXDOF>
BXF JointOut joint_eval(const JointT& J, const Body& P, const m3& RP, const Body& C, const m3& RC, const float* a) {
  return joint_eval<MAXDOF>(J, P, RP, C, joint_child<MAXDOF>(J, C, RC), a);
}

// One ground-contact candidate (Section 7.2): velocity-level normal impulse
// with restitution and Baumgarte term, jn = max(0, -(1+e) vn + beta depth / h)
// / kn, and a Coulomb friction impulse from the same pre-impulse state,
// jt = min(mu jn, s / kt). Adds the velocity changes to dv, dw and returns
// whether an impulse was applied. contact_apply takes the candidate's radius
// rho, its centre rotated to the world rl = R l and its depth, as
// contact_eval forms them.
BXF bool contact_apply(float rho, const TypeT& ty, const BodyT& B, const Body& s, const Frame& f, v3 rl, float depth,
                       v3& dv, v3& dw) {
  if (!(depth > 0.f)) return false;
  v3 r = V(rl.x, rl.y, rl.z - rho);  // lowest point relative to the centre of mass
  v3 u = s.v + cross(s.w, r);
  v3 a = mul(f.Iwinv, V(r.y, -r.x, 0.f));       // Iwinv (r x z)
  float kn = B.inv_m + (a.x * r.y - a.y * r.x);  // z . ((Iwinv (r x z)) x r)
  float num = ty.beta_h * depth - ty.one_plus_e * u.z;
  if (!(num > 0.f)) return false;
  float jn = num / kn;
  // J = jn z - jt t, so Iwinv (r x J) = jn Iwinv (r x z) - jt Iwinv (r x t):
  // both products are already formed for kn and kt
  v3 J = V(0.f, 0.f, jn);
  v3 dwc = jn * a;
  const float sp2 = u.x * u.x + u.y * u.y;
  if (sp2 > 0.f) {
    const float isp = 1.f / sqrtf(sp2);
    const float sp = sp2 * isp;
    v3 t = V(u.x * isp, u.y * isp, 0.f);
    v3 z = cross(r, t);
    v3 bz = mul(f.Iwinv, z);
    float kt = B.inv_m + dot(z, bz);  // t.((Iwinv (r x t)) x r) = (r x t).Iwinv (r x t)
    float stop = sp / kt;
    float cap = ty.mu * jn;
    float jt = cap <= stop ? cap : stop;
    J.x = -jt * t.x;
    J.y = -jt * t.y;
    dwc = dwc - jt * bz;
  }
  dv += B.inv_m * J;
  dw += dwc;
  return true;
}
BXF bool contact_eval(const ContactT& c, const TypeT& ty, const BodyT& B, const Body& s, const Frame& f, v3& dv,
                      v3& dw) {
  const v3 rl = mul(f.R, ld3(c.l));
  return contact_apply(c.rho, ty, B, s, f, rl, c.rho - (s.p.z + rl.z), dv, dw);
}

// Potential integrator: v += h (g + f/m); w += h Iwinv (t - w x (Iw w)).
// Iw w is formed in the body frame, R (I o (R^T w)), which needs no world
// inertia matrix.
// MASKED = false: for a system type without frozen axes (the same result,
// without the per-axis selects).
template <bool MASKED = true>
BXF void potential(const BodyT& B, const TypeT& ty, Body& s, const Frame& f, v3 force, v3 torque) {
  v3 acc = ld3(ty.g) + B.inv_m * force;
  v3 wb = mul_t(f.R, s.w);
  v3 gyro = cross(s.w, mul(f.R, V(B.I[0] * wb.x, B.I[1] * wb.y, B.I[2] * wb.z)));
  v3 alpha = mul(f.Iwinv, torque - gyro);
  if (MASKED) {
    s.v = keep_fma(s.v, ty.h, acc, B.free_p);
    s.w = keep_fma(s.w, ty.h, alpha, B.free_r);
  } else {
    s.v = V(fmaf(ty.h, acc.x, s.v.x), fmaf(ty.h, acc.y, s.v.y), fmaf(ty.h, acc.z, s.v.z));
    s.w = V(fmaf(ty.h, alpha.x, s.w.x), fmaf(ty.h, alpha.y, s.w.y), fmaf(ty.h, alpha.z, s.w.z));
  }
}

// Collision integrator: the body's contact impulses averaged over the n
// candidates that applied one.
template <bool MASKED = true>
BXF void collision(const BodyT& B, Body& s, v3 dv, v3 dw, int n) {
  if (n > 0) {
    float inv = 1.f / (float)n;
    if (MASKED) {
      s.v = keep_fma(s.v, inv, dv, B.free_p);
      s.w = keep_fma(s.w, inv, dw, B.free_r);
    } else {
      s.v = V(fmaf(inv, dv.x, s.v.x), fmaf(inv, dv.y, s.v.y), fmaf(inv, dv.z, s.v.z));
      s.w = V(fmaf(inv, dw.x, s.w.x), fmaf(inv, dw.y, s.w.y), fmaf(inv, dw.z, s.w.z));
    }
  }
}

BXF bool finite_body(const Body& s) {
  float acc = s.p.x + s.p.y + s.p.z + s.q.w + s.q.x + s.q.y + s.q.z + s.v.x + s.v.y + s.v.z + s.w.x + s.w.y + s.w.z;
  return isfinite(acc) && !isnan(acc);
}

}  // namespace bx
