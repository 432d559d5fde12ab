// FP64 reference stepper for the batched maximal-coordinate rigid-body step.
//
// TEST INFRASTRUCTURE ONLY — the oracle. It is called by the tests, by the
// smoke check and by the CPU-baseline leg of the benchmark, never by the
// product path, and it shares no code with the HIP library.
//
// What it follows (Brax, arXiv 2106.13281):
//   * Section 3, Algorithm 1 — one physics step: kinematic integration, then
//     joint, actuator and collider updates all computed from the same
//     (post-kinematic) qp, then the potential integrator applies the joint and
//     actuator updates and the collision integrator applies the collider
//     updates. The step is repeated `substeps` times per dt (Appendix A).
//   * Section 3 — maximal coordinates: the only dynamic data per body are
//     position, orientation, velocity and angular velocity (the QP); the
//     update is symplectic (semi-implicit) Euler.
//   * Section 7.1 "Spring Joints" — joints are stiff springs (with damping).
//   * Section 7.2 "Collisions" — velocity-level contact impulses with
//     Baumgarte stabilisation against the ground.
//   * Appendix A — the system fields (mass, inertia, frozen axes, joint
//     stiffness, offsets, angle limits, dt, substeps, gravity).
// The paper gives no formula for the joint force law, the contact impulse or
// the friction model; the readings implemented here are the ones listed in
// the design notes (anchor spring + alignment spring + limit springs + angular
// damping; normal impulse with restitution and Baumgarte term; Coulomb
// friction from the same pre-impulse state; contacts on one body averaged).
//
// Layout: state per environment is [nb][13] doubles:
//   p(3) q(4: w,x,y,z, body->world, Hamilton) v(3) w(3), all world frame.
// Actions per environment: [na] doubles.
//
// Every function is templated on the scalar type (double, Dual<N>, Counted);
// see orc_scalar.h.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include <omp.h>

#include "orc_scalar.h"

namespace orc {

thread_local int64_t g_flops = 0;
thread_local std::vector<TraceNode>* g_trace = nullptr;

enum { MAXB = 16, MAXJ = 16, MAXC = 96, MAXA = 48, MAXP = 32 };
enum { PP, PS, SP, SS, PB, BP, SB, BS };  // body-body candidate: first body's feature vs the second's

// Flat system description filled by the Python side of the oracle
// (oracle/__init__.py mirrors this struct field by field).
struct OrcSys {
  int32_t nb, nj, nc, na, substeps, pad0;
  double dt, beta, elasticity, friction;
  double gravity[3];
  double mass[MAXB];
  double inertia[MAXB][3];      // principal moments, body frame
  double free_pos[MAXB][3];     // 1 = axis integrates, 0 = frozen (world axes)
  double free_rot[MAXB][3];
  int32_t c_body[MAXC];
  int32_t pad1;
  double c_local[MAXC][3];      // contact centre in the body frame
  double c_radius[MAXC];        // sphere/capsule radius; 0 for box corners
  int32_t j_parent[MAXJ], j_child[MAXJ], j_dof[MAXJ];
  int32_t pad2;
  double j_anchor_p[MAXJ][3], j_anchor_c[MAXJ][3];   // anchor in parent / child body frame
  double j_frame_p[MAXJ][9], j_frame_c[MAXJ][9];     // joint frame rotation in body frame, row-major
  double j_k_lin[MAXJ], j_c_lin[MAXJ], j_k_ang[MAXJ], j_c_ang[MAXJ], j_k_lim[MAXJ];
  double j_lo[MAXJ][3], j_hi[MAXJ][3];               // radians
  int32_t a_joint[MAXA], a_axis[MAXA];               // action k drives joint a_joint[k], axis a_axis[k]
  double a_gear[MAXA];
  int32_t a_mode[MAXA];                              // 0 torque, 1 target angle
  // body-body contact candidates: bodies, kind, the first body's feature
  // (point a0, segment a0-a1 or box centre a0 / rotation aR / half extents ah)
  // and radius, the same for the second body; all in body frames
  int32_t np, pad3;
  int32_t p_a[MAXP], p_b[MAXP], p_kind[MAXP];
  double p_a0[MAXP][3], p_a1[MAXP][3], p_ra[MAXP], p_b0[MAXP][3], p_b1[MAXP][3], p_rb[MAXP];
  double p_ah[MAXP][3], p_bh[MAXP][3], p_aR[MAXP][9], p_bR[MAXP][9];
};

// ------------------------------------------------------------ small vectors
template <class T> struct V3 { T x, y, z; };
template <class T> struct Qt { T w, x, y, z; };
template <class T> struct M3 { T m[3][3]; };

template <class T> V3<T> vec(T x, T y, T z) { return V3<T>{x, y, z}; }
template <class T> V3<T> add(const V3<T>& a, const V3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> V3<T> sub(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> V3<T> scale(const T& s, const V3<T>& a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> V3<T> neg(const V3<T>& a) { return {-a.x, -a.y, -a.z}; }
template <class T> T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> V3<T> hadamard(const double m[3], const V3<T>& a) {
  // frozen-axis mask: multiply by 0/1 constants (no arithmetic counted)
  return {m[0] != 0 ? a.x : T(0.0), m[1] != 0 ? a.y : T(0.0), m[2] != 0 ? a.z : T(0.0)};
}
template <class T> V3<T> matvec(const M3<T>& A, const V3<T>& v) {
  return {A.m[0][0] * v.x + A.m[0][1] * v.y + A.m[0][2] * v.z,
          A.m[1][0] * v.x + A.m[1][1] * v.y + A.m[1][2] * v.z,
          A.m[2][0] * v.x + A.m[2][1] * v.y + A.m[2][2] * v.z};
}
template <class T> M3<T> matmul(const M3<T>& A, const M3<T>& B) {
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.m[i][j] = A.m[i][0] * B.m[0][j] + A.m[i][1] * B.m[1][j] + A.m[i][2] * B.m[2][j];
  return C;
}
template <class T> M3<T> transpose(const M3<T>& A) {
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.m[i][j] = A.m[j][i];
  return C;
}
template <class T> M3<T> const_mat(const double* rowmajor) {
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.m[i][j] = T(rowmajor[3 * i + j]);
  return C;
}
template <class T> V3<T> column(const M3<T>& A, int j) { return {A.m[0][j], A.m[1][j], A.m[2][j]}; }
template <class T> V3<T> const_vec(const double* v) { return {T(v[0]), T(v[1]), T(v[2])}; }

// Hamilton product (w, x, y, z).
template <class T> Qt<T> qmul(const Qt<T>& a, const Qt<T>& b) {
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
// Rotation matrix (body -> world) of a unit quaternion.
template <class T> M3<T> quat_to_mat(const Qt<T>& q) {
  M3<T> R;
  R.m[0][0] = 1.0 - 2.0 * (q.y * q.y + q.z * q.z);
  R.m[0][1] = 2.0 * (q.x * q.y - q.w * q.z);
  R.m[0][2] = 2.0 * (q.x * q.z + q.w * q.y);
  R.m[1][0] = 2.0 * (q.x * q.y + q.w * q.z);
  R.m[1][1] = 1.0 - 2.0 * (q.x * q.x + q.z * q.z);
  R.m[1][2] = 2.0 * (q.y * q.z - q.w * q.x);
  R.m[2][0] = 2.0 * (q.x * q.z - q.w * q.y);
  R.m[2][1] = 2.0 * (q.y * q.z + q.w * q.x);
  R.m[2][2] = 1.0 - 2.0 * (q.x * q.x + q.y * q.y);
  return R;
}
// R diag(d) R^T
template <class T> M3<T> rotate_diag(const M3<T>& R, const V3<T>& d) {
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C.m[i][j] = R.m[i][0] * d.x * R.m[j][0] + R.m[i][1] * d.y * R.m[j][1] + R.m[i][2] * d.z * R.m[j][2];
  return C;
}

template <class T> T clampv(const T& x, double lo, double hi) {
  if (val(x) < lo) return T(lo);
  if (val(x) > hi) return T(hi);
  return x;
}

// Per-body quantities the phases share.
template <class T> struct Body {
  V3<T> p, v, w;
  Qt<T> q;
};
template <class T> struct Derived {
  M3<T> R, Iw, Iwinv;
};

template <class T> Body<T> load_body(const T* X) {
  Body<T> b;
  b.p = {X[0], X[1], X[2]};
  b.q = {X[3], X[4], X[5], X[6]};
  b.v = {X[7], X[8], X[9]};
  b.w = {X[10], X[11], X[12]};
  return b;
}
template <class T> void store_body(const Body<T>& b, T* X) {
  X[0] = b.p.x; X[1] = b.p.y; X[2] = b.p.z;
  X[3] = b.q.w; X[4] = b.q.x; X[5] = b.q.y; X[6] = b.q.z;
  X[7] = b.v.x; X[8] = b.v.y; X[9] = b.v.z;
  X[10] = b.w.x; X[11] = b.w.y; X[12] = b.w.z;
}

// Margins of the step's discontinuities, kept so parity checks can tell a
// genuine mismatch from an environment sitting on a branch boundary.
// The first three are jumps of the result itself; the last four are kinks
// (the result is continuous, its derivative jumps), which matter only when
// derivatives are compared.
enum { NMARGIN = 8 };
struct Margins {
  double contact_depth = 1e30;    // |penetration| of every candidate (m)
  double contact_speed = 1e30;    // |normal-impulse numerator| of candidates in contact (m/s)
  double angle_wrap = 1e30;       // pi - |theta| for limited free angles (rad)
  double slip_speed = 1e30;       // tangential contact speed of impulsive contacts (m/s)
  double cone_gap = 1e30;         // |mu jn - s/kt| / (mu jn): Coulomb cone vs sticking
  double limit_gap = 1e30;        // distance of a free angle to its limits (rad)
  double clip_gap = 1e30;         // 1 - |a| of every action
  double feature_gap = 1e30;      // distance of a closest-feature parameter to a clamp / face switch (m)
  void store(double* out) const {
    out[0] = contact_depth; out[1] = contact_speed; out[2] = angle_wrap; out[3] = slip_speed;
    out[4] = cone_gap; out[5] = limit_gap; out[6] = clip_gap; out[7] = feature_gap;
  }
};

// ------------------------------------------------------------ the phases
// Kinematic integrator (Algorithm 1, first line): advance positions and
// orientations with the current velocities. Frozen axes hold zero velocity.
template <class T> void kinematic(const OrcSys& s, int i, Body<T>& b, double h) {
  b.v = hadamard(s.free_pos[i], b.v);
  b.w = hadamard(s.free_rot[i], b.w);
  b.p = add(b.p, scale(T(h), b.v));
  Qt<T> wq = {T(0.0), b.w.x, b.w.y, b.w.z};
  Qt<T> dq = qmul(wq, b.q);
  T hh = T(0.5 * h);
  Qt<T> q = {b.q.w + hh * dq.w, b.q.x + hh * dq.x, b.q.y + hh * dq.y, b.q.z + hh * dq.z};
  T n = osqrt(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
  b.q = {q.w / n, q.x / n, q.y / n, q.z / n};
}

template <class T> Derived<T> derive(const OrcSys& s, int i, const Body<T>& b) {
  Derived<T> d;
  d.R = quat_to_mat(b.q);
  V3<T> I = const_vec<T>(s.inertia[i]);
  V3<T> Iinv = {T(1.0 / s.inertia[i][0]), T(1.0 / s.inertia[i][1]), T(1.0 / s.inertia[i][2])};
  d.Iw = rotate_diag(d.R, I);
  d.Iwinv = rotate_diag(d.R, Iinv);
  return d;
}

// Joint frames in world coordinates and the intrinsic X-Y-Z Euler angles of
// the child's joint frame relative to the parent's: M = AwP^T AwC = Rx(t1) Ry(t2) Rz(t3).
template <class T> struct JointFrame {
  M3<T> AwP, AwC;
  T th[3];
  V3<T> axis[3];  // Euler axes: parent x, intermediate y, child z
};
template <class T> JointFrame<T> joint_frame(const OrcSys& s, int j, const Derived<T>& dP, const Derived<T>& dC) {
  JointFrame<T> f;
  f.AwP = matmul(dP.R, const_mat<T>(s.j_frame_p[j]));
  f.AwC = matmul(dC.R, const_mat<T>(s.j_frame_c[j]));
  M3<T> M = matmul(transpose(f.AwP), f.AwC);
  f.th[0] = oatan2(-M.m[1][2], M.m[2][2]);
  f.th[1] = oasin(clampv(M.m[0][2], -1.0, 1.0));
  f.th[2] = oatan2(-M.m[0][1], M.m[0][0]);
  V3<T> e1P = column(f.AwP, 0), e2P = column(f.AwP, 1), e3P = column(f.AwP, 2);
  T c1 = ocos(f.th[0]), s1 = osin(f.th[0]);
  f.axis[0] = e1P;
  f.axis[1] = add(scale(c1, e2P), scale(s1, e3P));
  f.axis[2] = column(f.AwC, 2);
  return f;
}

// Joint update (Algorithm 1, joint loop; Section 7.1 spring joints).
template <class T>
void joint_apply(const OrcSys& s, int j, const Body<T>* B, const Derived<T>* D, const JointFrame<T>& fr, V3<T>* f,
                 V3<T>* t, Margins* mg) {
  const int P = s.j_parent[j], C = s.j_child[j], n = s.j_dof[j];
  V3<T> rP = matvec(D[P].R, const_vec<T>(s.j_anchor_p[j]));
  V3<T> rC = matvec(D[C].R, const_vec<T>(s.j_anchor_c[j]));
  V3<T> xP = add(B[P].p, rP), xC = add(B[C].p, rC);
  V3<T> d = sub(xP, xC);
  V3<T> uP = add(B[P].v, cross(B[P].w, rP));
  V3<T> uC = add(B[C].v, cross(B[C].w, rC));
  // anchor spring and damper: force on the child at its anchor, minus that on the parent
  V3<T> F = add(scale(T(s.j_k_lin[j]), d), scale(T(s.j_c_lin[j]), sub(uP, uC)));

  V3<T> e1P = column(fr.AwP, 0), e1C = column(fr.AwC, 0), e2C = column(fr.AwC, 1);
  V3<T> tau = {T(0.0), T(0.0), T(0.0)};
  // alignment spring on the constrained rotational axes
  if (n == 1) {
    tau = scale(T(s.j_k_ang[j]), cross(e1C, e1P));       // V = k (1 - e1P.e1C)
  } else if (n == 2) {
    T c = dot(e1P, e2C);                                 // V = k/2 (e1P.e2C)^2
    tau = scale(T(-s.j_k_ang[j]) * c, cross(e2C, e1P));
  }
  // angular damping on the relative angular velocity
  tau = add(tau, scale(T(s.j_c_ang[j]), sub(B[P].w, B[C].w)));
  // limit springs on each free angle
  for (int k = 0; k < n; ++k) {
    T th = fr.th[k];
    T excess = th - clampv(th, s.j_lo[j][k], s.j_hi[j][k]);
    tau = add(tau, scale(T(-s.j_k_lim[j]) * excess, fr.axis[k]));
    if (mg && k != 1 && (s.j_lo[j][k] > -M_PI || s.j_hi[j][k] < M_PI))
      mg->angle_wrap = std::min(mg->angle_wrap, M_PI - std::fabs(val(th)));
    if (mg)
      mg->limit_gap = std::min(mg->limit_gap, std::min(std::fabs(val(th) - s.j_lo[j][k]),
                                                       std::fabs(val(th) - s.j_hi[j][k])));
  }
  f[C] = add(f[C], F);
  t[C] = add(t[C], add(cross(rC, F), tau));
  f[P] = sub(f[P], F);
  t[P] = sub(t[P], add(cross(rP, F), tau));
}

// Actuator update (Algorithm 1, actuator loop; Section 3: actions are
// torques or target angles), about the joint's Euler axis, on the child and
// opposite on the parent: a torque actuator applies gear * a; a target-angle
// actuator drives the angle towards a (radians, clamped to the joint's
// range) with gear * (a - theta).
template <class T>
void actuator_apply(const OrcSys& s, int k, const T& a, const JointFrame<T>* frames, V3<T>* t) {
  const int j = s.a_joint[k];
  const int P = s.j_parent[j], C = s.j_child[j];
  const JointFrame<T>& fr = frames[j];
  const T drive = s.a_mode[k] == 1 ? a - fr.th[s.a_axis[k]] : a;
  V3<T> tau = scale(T(s.a_gear[k]) * drive, fr.axis[s.a_axis[k]]);
  t[C] = add(t[C], tau);
  t[P] = sub(t[P], tau);
}

// Collider update (Algorithm 1, collider loop; Section 7.2): one contact
// candidate against the ground plane z = 0 with normal +z.
template <class T>
void collider_apply(const OrcSys& s, int c, const Body<T>* B, const Derived<T>* D, double h, V3<T>* dv,
                    V3<T>* dw, int* cnt, Margins* mg) {
  const int i = s.c_body[c];
  const double rho = s.c_radius[c];
  V3<T> y = add(B[i].p, matvec(D[i].R, const_vec<T>(s.c_local[c])));
  T depth = T(rho) - y.z;
  if (mg) mg->contact_depth = std::min(mg->contact_depth, std::fabs(val(depth)));
  if (!(val(depth) > 0)) return;
  V3<T> zhat = {T(0.0), T(0.0), T(1.0)};
  V3<T> r = sub(sub(y, scale(T(rho), zhat)), B[i].p);     // lowest point relative to the centre of mass
  V3<T> u = add(B[i].v, cross(B[i].w, r));
  T vn = u.z;
  T invm = T(1.0 / s.mass[i]);
  T kn = invm + dot(zhat, cross(matvec(D[i].Iwinv, cross(r, zhat)), r));
  T num = T(-(1.0 + s.elasticity)) * vn + T(s.beta / h) * depth;
  if (mg) mg->contact_speed = std::min(mg->contact_speed, std::fabs(val(num)));
  if (!(val(num) > 0)) return;                            // jn = max(0, num)/kn == 0: no impulse
  T jn = num / kn;
  V3<T> ut = {u.x, u.y, T(0.0)};
  T sp = osqrt(ut.x * ut.x + ut.y * ut.y);
  V3<T> J = scale(jn, zhat);
  if (mg) mg->slip_speed = std::min(mg->slip_speed, val(sp));
  if (val(sp) > 0) {
    V3<T> tdir = scale(T(1.0) / sp, ut);
    T kt = invm + dot(tdir, cross(matvec(D[i].Iwinv, cross(r, tdir)), r));
    T stop = sp / kt;                                     // impulse that stops the sliding
    T cap = T(s.friction) * jn;                           // Coulomb cone
    T jt = (val(cap) <= val(stop)) ? cap : stop;
    if (mg && val(cap) > 0) mg->cone_gap = std::min(mg->cone_gap, std::fabs(val(cap) - val(stop)) / val(cap));
    J = sub(J, scale(jt, tdir));
  }
  dv[i] = add(dv[i], scale(invm, J));
  dw[i] = add(dw[i], matvec(D[i].Iwinv, cross(r, J)));
  cnt[i] += 1;
}

// ------------------------------------------------------------ body-body contacts
// Closest point of segment a-b to p (parameter clamped to [0, 1]).
template <class T> V3<T> closest_on_segment(const V3<T>& p, const V3<T>& a, const V3<T>& b, Margins* mg) {
  V3<T> d = sub(b, a);
  T dd = dot(d, d);
  if (!(val(dd) > 0)) return a;
  T t = dot(sub(p, a), d) / dd;
  if (mg) mg->feature_gap = std::min(mg->feature_gap, std::min(std::fabs(val(t)), std::fabs(val(t) - 1.0)) * std::sqrt(val(dd)));
  t = clampv(t, 0.0, 1.0);
  return add(a, scale(t, d));
}
// Closest points of segments p0-p1 and q0-q1: minimise |P(s) - Q(t)|^2 over
// [0, 1]^2 (the unconstrained minimiser clamped in s, then t from s, then s
// again from the clamped t).
template <class T> void closest_segments(const V3<T>& p0, const V3<T>& p1, const V3<T>& q0, const V3<T>& q1, V3<T>& cp,
                                         V3<T>& cq, Margins* mg) {
  V3<T> d1 = sub(p1, p0), d2 = sub(q1, q0), r = sub(p0, q0);
  T a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
  if (!(val(a) > 0)) {
    cp = p0;
    cq = closest_on_segment(p0, q0, q1, mg);
    return;
  }
  if (!(val(e) > 0)) {
    cq = q0;
    cp = closest_on_segment(q0, p0, p1, mg);
    return;
  }
  T c = dot(d1, r), b = dot(d1, d2);
  T den = a * e - b * b;
  T s = T(0.0);
  auto gap = [&](const T& x, double len) {
    if (mg) mg->feature_gap = std::min(mg->feature_gap, std::min(std::fabs(val(x)), std::fabs(val(x) - 1.0)) * len);
  };
  if (val(den) > 0) {
    s = (b * f - c * e) / den;
    gap(s, std::sqrt(val(a)));
    s = clampv(s, 0.0, 1.0);
  }
  T t = (b * s + f) / e;
  gap(t, std::sqrt(val(e)));
  if (val(t) < 0) {
    t = T(0.0);
    s = -c / a;
    gap(s, std::sqrt(val(a)));
    s = clampv(s, 0.0, 1.0);
  } else if (val(t) > 1) {
    t = T(1.0);
    s = (b - c) / a;
    gap(s, std::sqrt(val(a)));
    s = clampv(s, 0.0, 1.0);
  }
  cp = add(p0, scale(s, d1));
  cq = add(q0, scale(t, d2));
}
// Point p against a box (centre c, rotation R box to world, half extents h):
// the box point closest to p and the outward normal; inside the box, the
// nearest face point and that face's normal. Returns the signed distance of
// p from the box surface along the normal (negative inside).
template <class T> T point_box(const V3<T>& p, const V3<T>& c, const M3<T>& R, const double* h, V3<T>& cb, V3<T>& n,
                               Margins* mg) {
  V3<T> q = matvec(transpose(R), sub(p, c));
  T qa[3] = {q.x, q.y, q.z};
  bool inside = true;
  for (int k = 0; k < 3; ++k) {
    if (mg) mg->feature_gap = std::min(mg->feature_gap, std::fabs(std::fabs(val(qa[k])) - h[k]));
    if (std::fabs(val(qa[k])) > h[k]) inside = false;
  }
  if (!inside) {
    T cl[3];
    for (int k = 0; k < 3; ++k) cl[k] = clampv(qa[k], -h[k], h[k]);
    cb = add(c, matvec(R, V3<T>{cl[0], cl[1], cl[2]}));
    V3<T> d = sub(p, cb);
    T dist = osqrt(dot(d, d));
    n = scale(T(1.0) / dist, d);
    return dist;
  }
  int k = 0;
  double best = 1e300;
  for (int i = 0; i < 3; ++i) {
    double g = h[i] - std::fabs(val(qa[i]));
    if (g < best) {
      best = g;
      k = i;
    }
  }
  if (mg) {  // a switch of the nearest face
    for (int i = 0; i < 3; ++i)
      if (i != k) mg->feature_gap = std::min(mg->feature_gap, std::fabs((h[i] - std::fabs(val(qa[i]))) - best));
  }
  const double sg = val(qa[k]) >= 0 ? 1.0 : -1.0;
  T cl[3] = {qa[0], qa[1], qa[2]};
  cl[k] = T(sg * h[k]);
  cb = add(c, matvec(R, V3<T>{cl[0], cl[1], cl[2]}));
  V3<T> ek = {T(k == 0 ? sg : 0.0), T(k == 1 ? sg : 0.0), T(k == 2 ? sg : 0.0)};
  n = matvec(R, ek);
  return T(-1.0) * (T(h[k]) - (sg > 0 ? qa[k] : T(-1.0) * qa[k]));
}
// Segment a0-a1 against a box (centre c, rotation R box to world, half
// extents h): the parameter s* in [0, 1] of the segment point nearest the
// box, or of the deepest one where the segment passes through the box. In
// box coordinates the segment is q(s) = q0 + s dq. It passes through the box
// where the parameters with every |q_k(s)| < h_k form an interval of
// positive length. Outside, the squared distance sum_k max(|q_k| - h_k, 0)^2
// is convex and quadratic between the parameters where some |q_k(s)| = h_k:
// the candidates are the two ends, those parameters and each piece's
// stationary point inside its piece. Through the box, the deepest point
// minimises the signed distance max_k (|q_k| - h_k), linear between the
// parameters where two of the six lines +-q_k(s) - h_k cross: the candidates
// are the two ends and those crossings. The smallest value wins (the
// smallest s among equal ones).
// act: how far (in m) the point is from switching between an end and the
// interior (the distance of an interior point from the nearer end, or of
// the first or last piece's stationary point beyond an end).
template <class T> T segment_box(const V3<T>& a0, const V3<T>& a1, const V3<T>& c, const M3<T>& R, const double* h,
                                 double& act, Margins* mg) {
  const M3<T> Rt = transpose(R);
  const V3<T> q0v = matvec(Rt, sub(a0, c)), dqv = matvec(Rt, sub(a1, a0));
  const T q0[3] = {q0v.x, q0v.y, q0v.z}, dq[3] = {dqv.x, dqv.y, dqv.z};
  const double L = std::sqrt(val(dot(dqv, dqv)));
  auto qat = [&](const T& s, int k) { return q0[k] + s * dq[k]; };
  auto best_of = [&](const std::vector<T>& cs, auto fn, double& second) {
    size_t bi = 0;
    double bv = 1e300;
    second = 1e300;
    for (size_t i = 0; i < cs.size(); ++i) {
      const double v = val(fn(cs[i]));
      if (v < bv || (v == bv && val(cs[i]) < val(cs[bi]))) {
        if (i) second = std::min(second, bv);
        bv = v;
        bi = i;
      } else {
        second = std::min(second, v);
      }
    }
    return bi;
  };
  // the interval of parameters strictly inside every slab |q_k| < h_k
  double te = 0.0, tx = 1.0;
  for (int k = 0; k < 3; ++k) {
    if (val(dq[k]) != 0) {
      const double t1 = (-h[k] - val(q0[k])) / val(dq[k]), t2 = (h[k] - val(q0[k])) / val(dq[k]);
      te = std::max(te, std::min(t1, t2));
      tx = std::min(tx, std::max(t1, t2));
    } else if (!(std::fabs(val(q0[k])) < h[k])) {
      te = 1.0;
      tx = 0.0;
    }
  }
  if (mg) mg->feature_gap = std::min(mg->feature_gap, std::fabs(tx - te) * L);
  double second = 0;
  T s;
  if (te < tx) {
    // through the box: the deepest point
    auto inside_sd = [&](const T& t) {
      T g = T(-1e300);
      for (int k = 0; k < 3; ++k) {
        const T qk = qat(t, k);
        const T ex = val(qk) >= 0 ? qk - T(h[k]) : T(-1.0) * qk - T(h[k]);
        if (val(ex) > val(g)) g = ex;
      }
      return g;
    };
    std::vector<T> ic = {T(0.0), T(1.0)};
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        const double si = (i & 1) ? -1.0 : 1.0, sj = (j & 1) ? -1.0 : 1.0;
        const int ki = i / 2, kj = j / 2;
        const T bi_ = T(si) * dq[ki], bj_ = T(sj) * dq[kj];
        if (val(bi_) == val(bj_)) continue;
        const T ai = T(si) * q0[ki] - T(h[ki]), aj = T(sj) * q0[kj] - T(h[kj]);
        const T sc = (aj - ai) / (bi_ - bj_);
        if (val(sc) > 0 && val(sc) < 1) ic.push_back(sc);
      }
    const size_t bi = best_of(ic, inside_sd, second);
    s = ic[bi];
    if (mg) mg->feature_gap = std::min(mg->feature_gap, std::fabs(second - val(inside_sd(s))));
  } else {
    auto outside_sq = [&](const T& t) {
      T f = T(0.0);
      for (int k = 0; k < 3; ++k) {
        const T qk = qat(t, k);
        const T ex = val(qk) >= 0 ? qk - T(h[k]) : T(-1.0) * qk - T(h[k]);
        if (val(ex) > 0) f = f + ex * ex;
      }
      return f;
    };
    // the parameters where |q_k(s)| = h_k, inside (0, 1), sorted
    std::vector<T> cuts;
    for (int k = 0; k < 3; ++k)
      for (double sg : {-1.0, 1.0})
        if (val(dq[k]) != 0) {
          const T sc = (T(sg * h[k]) - q0[k]) / dq[k];
          if (val(sc) > 0 && val(sc) < 1) cuts.push_back(sc);
        }
    std::sort(cuts.begin(), cuts.end(), [](const T& x, const T& y) { return val(x) < val(y); });
    std::vector<T> cand = {T(0.0), T(1.0)};
    for (const T& x : cuts) cand.push_back(x);
    // each piece's stationary point: active coordinates and their sides fixed
    std::vector<double> ends = {0.0};
    for (const T& x : cuts) ends.push_back(val(x));
    ends.push_back(1.0);
    for (size_t i = 0; i + 1 < ends.size(); ++i) {
      const double mid = 0.5 * (ends[i] + ends[i + 1]);
      T num = T(0.0), den = T(0.0);
      for (int k = 0; k < 3; ++k) {
        const double qm = val(q0[k]) + mid * val(dq[k]);
        if (std::fabs(qm) > h[k]) {
          const double sg = qm >= 0 ? 1.0 : -1.0;
          num = num + (q0[k] - T(sg * h[k])) * dq[k];
          den = den + dq[k] * dq[k];
        }
      }
      if (val(den) > 0) {
        const T st = T(-1.0) * num / den;
        if (val(st) > ends[i] && val(st) < ends[i + 1]) cand.push_back(st);
      }
    }
    const size_t bi = best_of(cand, outside_sq, second);
    s = cand[bi];
    if (mg)
      for (int k = 0; k < 3; ++k)  // a coordinate reaching its face: the piece switches
        mg->feature_gap = std::min(mg->feature_gap, std::fabs(std::fabs(val(qat(s, k))) - h[k]));
    if (val(s) == 0.0 || val(s) == 1.0) {
      // the stationary point of the end's piece, beyond that end
      const double mid = val(s) == 0.0 ? 0.5 * ends[1] : 0.5 * (ends[ends.size() - 2] + 1.0);
      double num = 0, den = 0;
      for (int k = 0; k < 3; ++k) {
        const double qm = val(q0[k]) + mid * val(dq[k]);
        if (std::fabs(qm) > h[k]) {
          num += (val(q0[k]) - (qm >= 0 ? 1.0 : -1.0) * h[k]) * val(dq[k]);
          den += val(dq[k]) * val(dq[k]);
        }
      }
      act = den > 0 ? std::fabs(-num / den - val(s)) * L : 0.0;
      return s;
    }
  }
  act = std::min(val(s), 1.0 - val(s)) * L;
  return s;
}
// One body-body contact candidate (the paper's collisions between colliders,
// Section 7.2, with the impulse of the ground contact): closest features,
// normal n from the second body to the first, depth; the velocity-level
// normal impulse with restitution and Baumgarte term on the relative
// velocity at the middle of the overlap, Coulomb friction from the same
// state; +J on the first body, -J on the second. A body whose translations
// (rotations) are all frozen contributes no inverse mass (inertia).
template <class T>
void pair_apply(const OrcSys& s, int c, const Body<T>* B, const Derived<T>* D, double h, V3<T>* dv, V3<T>* dw,
                int* cnt, Margins* mg) {
  const int ia = s.p_a[c], ib = s.p_b[c], kind = s.p_kind[c];
  const Body<T>& A = B[ia];
  const Body<T>& Bb = B[ib];
  auto wpt = [&](const Body<T>& bd, const Derived<T>& d, const double* l) { return add(bd.p, matvec(d.R, const_vec<T>(l))); };
  V3<T> ca, cb, n;
  T dist;
  const double ra = s.p_ra[c], rb = s.p_rb[c];
  if (kind == SB || kind == BS) {
    // a capsule's axis against a box: a candidate only where the segment's
    // nearest point lies strictly between its ends (the two ends are the
    // capsule's end-sphere candidates)
    const bool box_b = kind == SB;
    const Body<T>& sb = box_b ? A : Bb;            // the segment's body
    const Body<T>& xb = box_b ? Bb : A;            // the box's body
    const Derived<T>& sdr = box_b ? D[ia] : D[ib];
    const Derived<T>& xd = box_b ? D[ib] : D[ia];
    const V3<T> a0 = wpt(sb, sdr, box_b ? s.p_a0[c] : s.p_b0[c]), a1 = wpt(sb, sdr, box_b ? s.p_a1[c] : s.p_b1[c]);
    const V3<T> bc = wpt(xb, xd, box_b ? s.p_b0[c] : s.p_a0[c]);
    const M3<T> R = matmul(xd.R, const_mat<T>(box_b ? s.p_bR[c] : s.p_aR[c]));
    // the branch margins of the closest features count only where the
    // candidate is (or, at an end, would be) in contact
    Margins loc;
    double act = 0;
    const T sst = segment_box(a0, a1, bc, R, box_b ? s.p_bh[c] : s.p_ah[c], act, mg ? &loc : nullptr);
    const bool interior = val(sst) > 0 && val(sst) < 1;
    if (!interior && !mg) return;
    // that segment point against the box
    const V3<T> ps = add(a0, scale(sst, sub(a1, a0)));
    V3<T> cbox, nb;
    const T sd = point_box(ps, bc, R, box_b ? s.p_bh[c] : s.p_ah[c], cbox, nb, mg ? &loc : nullptr);
    if (mg && val(sd) < ra + rb) mg->feature_gap = std::min(mg->feature_gap, std::min(loc.feature_gap, act));
    if (!interior) return;
    if (box_b) {
      ca = ps; cb = cbox; n = nb; dist = sd;
    } else {
      ca = cbox; cb = ps; n = scale(T(-1.0), nb); dist = sd;
    }
  } else if (kind == PB || kind == BP) {
    const bool box_b = kind == PB;
    const Body<T>& pb = box_b ? A : Bb;            // the point's body
    const Body<T>& xb = box_b ? Bb : A;            // the box's body
    const Derived<T>& pd = box_b ? D[ia] : D[ib];
    const Derived<T>& xd = box_b ? D[ib] : D[ia];
    V3<T> p = wpt(pb, pd, box_b ? s.p_a0[c] : s.p_b0[c]);
    V3<T> bc = wpt(xb, xd, box_b ? s.p_b0[c] : s.p_a0[c]);
    M3<T> R = matmul(xd.R, const_mat<T>(box_b ? s.p_bR[c] : s.p_aR[c]));
    V3<T> cbox, nb;
    T sd = point_box(p, bc, R, box_b ? s.p_bh[c] : s.p_ah[c], cbox, nb, mg);
    if (box_b) {
      ca = p; cb = cbox; n = nb; dist = sd;
    } else {
      ca = cbox; cb = p; n = scale(T(-1.0), nb); dist = sd;
    }
  } else {
    V3<T> a0 = wpt(A, D[ia], s.p_a0[c]), a1 = wpt(A, D[ia], s.p_a1[c]);
    V3<T> b0 = wpt(Bb, D[ib], s.p_b0[c]), b1 = wpt(Bb, D[ib], s.p_b1[c]);
    if (kind == PP) { ca = a0; cb = b0; }
    else if (kind == PS) { ca = a0; cb = closest_on_segment(a0, b0, b1, mg); }
    else if (kind == SP) { cb = b0; ca = closest_on_segment(b0, a0, a1, mg); }
    else closest_segments(a0, a1, b0, b1, ca, cb, mg);
    V3<T> d = sub(ca, cb);
    dist = osqrt(dot(d, d));
    if (!(val(dist) > 0)) return;
    n = scale(T(1.0) / dist, d);
  }
  T depth = T(ra + rb) - dist;
  if (mg) mg->contact_depth = std::min(mg->contact_depth, std::fabs(val(depth)));
  if (!(val(depth) > 0)) return;
  // the middle of the overlap: between the two surface points along n
  V3<T> x = add(cb, scale(T(rb) - T(0.5) * depth, n));
  V3<T> rA = sub(x, A.p), rB = sub(x, Bb.p);
  auto frozen3 = [](const double* f) { return f[0] == 0 && f[1] == 0 && f[2] == 0; };
  const double imA = frozen3(s.free_pos[ia]) ? 0.0 : 1.0 / s.mass[ia];
  const double imB = frozen3(s.free_pos[ib]) ? 0.0 : 1.0 / s.mass[ib];
  const bool rotA = !frozen3(s.free_rot[ia]), rotB = !frozen3(s.free_rot[ib]);
  auto kfun = [&](const V3<T>& dir) {
    T k = T(imA + imB);
    if (rotA) k = k + dot(dir, cross(matvec(D[ia].Iwinv, cross(rA, dir)), rA));
    if (rotB) k = k + dot(dir, cross(matvec(D[ib].Iwinv, cross(rB, dir)), rB));
    return k;
  };
  V3<T> u = sub(add(A.v, cross(A.w, rA)), add(Bb.v, cross(Bb.w, rB)));
  T vn = dot(u, n);
  T num = T(-(1.0 + s.elasticity)) * vn + T(s.beta / h) * depth;
  if (mg) mg->contact_speed = std::min(mg->contact_speed, std::fabs(val(num)));
  if (!(val(num) > 0)) return;
  T kn = kfun(n);
  T jn = num / kn;
  V3<T> J = scale(jn, n);
  V3<T> ut = sub(u, scale(vn, n));
  T sp = osqrt(dot(ut, ut));
  if (mg) mg->slip_speed = std::min(mg->slip_speed, val(sp));
  if (val(sp) > 0) {
    V3<T> t = scale(T(1.0) / sp, ut);
    T kt = kfun(t);
    T stop = sp / kt;
    T cap = T(s.friction) * jn;
    T jt = (val(cap) <= val(stop)) ? cap : stop;
    if (mg && val(cap) > 0) mg->cone_gap = std::min(mg->cone_gap, std::fabs(val(cap) - val(stop)) / val(cap));
    J = sub(J, scale(jt, t));
  }
  dv[ia] = add(dv[ia], scale(T(imA), J));
  if (rotA) dw[ia] = add(dw[ia], matvec(D[ia].Iwinv, cross(rA, J)));
  dv[ib] = sub(dv[ib], scale(T(imB), J));
  if (rotB) dw[ib] = sub(dw[ib], matvec(D[ib].Iwinv, cross(rB, J)));
  cnt[ia] += 1;
  cnt[ib] += 1;
}

// One environment step = `substeps` repetitions of Algorithm 1.
template <class T>
void step_env(const OrcSys& s, T* X, const T* act_in, Margins* mg) {
  const int nb = s.nb;
  const double h = s.dt / s.substeps;
  T a[MAXA];
  for (int k = 0; k < s.na; ++k) {
    // torque actions are clipped to [-1, 1], target angles to the joint's range
    double lo = -1.0, hi = 1.0;
    if (s.a_mode[k] == 1) {
      lo = s.j_lo[s.a_joint[k]][s.a_axis[k]];
      hi = s.j_hi[s.a_joint[k]][s.a_axis[k]];
    }
    a[k] = clampv(act_in[k], lo, hi);
    if (mg) mg->clip_gap = std::min(mg->clip_gap, std::min(std::fabs(val(act_in[k]) - lo), std::fabs(val(act_in[k]) - hi)));
  }
  Body<T> B[MAXB];
  Derived<T> D[MAXB];
  for (int i = 0; i < nb; ++i) B[i] = load_body(X + 13 * i);
  for (int it = 0; it < s.substeps; ++it) {
    // qp = kinematic_integrator.apply(qp, dt)
    for (int i = 0; i < nb; ++i) kinematic(s, i, B[i], h);
    for (int i = 0; i < nb; ++i) D[i] = derive(s, i, B[i]);
    // joint frames and Euler angles, shared by the joint and actuator updates
    JointFrame<T> fr[MAXJ];
    for (int j = 0; j < s.nj; ++j) fr[j] = joint_frame(s, j, D[s.j_parent[j]], D[s.j_child[j]]);
    V3<T> fj[MAXB], tj[MAXB], ta[MAXB], dv[MAXB], dw[MAXB];
    int cnt[MAXB];
    for (int i = 0; i < nb; ++i) {
      fj[i] = tj[i] = ta[i] = dv[i] = dw[i] = V3<T>{T(0.0), T(0.0), T(0.0)};
      cnt[i] = 0;
    }
    // dp_j += jo.apply(qp)
    for (int j = 0; j < s.nj; ++j) joint_apply(s, j, B, D, fr[j], fj, tj, mg);
    // dp_a += ac.apply(qp, action)
    for (int k = 0; k < s.na; ++k) actuator_apply(s, k, a[k], fr, ta);
    // dp_c += co.apply(qp)
    for (int c = 0; c < s.nc; ++c) collider_apply(s, c, B, D, h, dv, dw, cnt, mg);
    for (int c = 0; c < s.np; ++c) pair_apply(s, c, B, D, h, dv, dw, cnt, mg);
    // qp = potential_integrator.apply(qp, dp_j + dp_a, dt)
    for (int i = 0; i < nb; ++i) {
      V3<T> g = const_vec<T>(s.gravity);
      V3<T> acc = add(g, scale(T(1.0 / s.mass[i]), fj[i]));
      B[i].v = add(B[i].v, hadamard(s.free_pos[i], scale(T(h), acc)));
      V3<T> tq = add(tj[i], ta[i]);
      V3<T> gyro = cross(B[i].w, matvec(D[i].Iw, B[i].w));
      V3<T> alpha = matvec(D[i].Iwinv, sub(tq, gyro));
      B[i].w = add(B[i].w, hadamard(s.free_rot[i], scale(T(h), alpha)));
    }
    // qp = collision_integrator.apply(qp, dp_c): contacts on one body are averaged
    for (int i = 0; i < nb; ++i) {
      if (cnt[i] == 0) continue;
      T inv = T(1.0 / cnt[i]);
      B[i].v = add(B[i].v, hadamard(s.free_pos[i], scale(inv, dv[i])));
      B[i].w = add(B[i].w, hadamard(s.free_rot[i], scale(inv, dw[i])));
    }
  }
  for (int i = 0; i < nb; ++i) store_body(B[i], X + 13 * i);
}

}  // namespace orc

using namespace orc;

extern "C" {

int orc_sizeof_sys(void) { return (int)sizeof(OrcSys); }
int orc_num_margins(void) { return NMARGIN; }

// Advance n_env environments by n_steps steps. X: [n_env][nb*13] in/out.
// act: [n_steps][n_env][na]. traj (nullable): [n_steps][n_env][nb*13], the
// state after every step. margins (nullable): [n_env][3], minimum over the
// whole run of the NMARGIN branch margins (see Margins).
int orc_rollout(const OrcSys* s, double* X, const double* act, int n_env, int n_steps, double* traj,
                double* margins, int n_threads) {
  if (!s || !X || (n_steps > 0 && !act) || n_env < 0 || n_steps < 0) return -1;
  const int ns = s->nb * 13;
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
  for (int e = 0; e < n_env; ++e) {
    Margins mg;
    for (int t = 0; t < n_steps; ++t) {
      step_env<double>(*s, X + (size_t)e * ns, act + ((size_t)t * n_env + e) * s->na, margins ? &mg : nullptr);
      if (traj) std::memcpy(traj + ((size_t)t * n_env + e) * ns, X + (size_t)e * ns, sizeof(double) * ns);
    }
    if (margins) mg.store(margins + (size_t)NMARGIN * e);
  }
  return 0;
}

// Threads the OpenMP runtime will use for orc_rollout with n_threads <= 0.
int orc_max_threads(void) { return omp_get_max_threads(); }

// Jacobian of one step for each environment: jac [n_env][nb*13][nb*13 + na],
// d(state_out)/d(state_in, action), by forward-mode dual numbers through the
// same code as orc_rollout.
int orc_step_jacobian(const OrcSys* s, const double* X, const double* act, int n_env, double* jac,
                      int n_threads) {
  if (!s || !X || !act || !jac || n_env < 0) return -1;
  constexpr int ND = 8;
  const int ns = s->nb * 13, nin = ns + s->na;
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic)
  for (int e = 0; e < n_env; ++e) {
    std::vector<Dual<ND>> Xd(ns), Ad(s->na > 0 ? s->na : 1);
    for (int c0 = 0; c0 < nin; c0 += ND) {
      for (int i = 0; i < ns; ++i) {
        Xd[i] = Dual<ND>(X[(size_t)e * ns + i]);
        for (int k = 0; k < ND; ++k) Xd[i].d[k] = (c0 + k == i) ? 1.0 : 0.0;
      }
      for (int i = 0; i < s->na; ++i) {
        Ad[i] = Dual<ND>(act[(size_t)e * s->na + i]);
        for (int k = 0; k < ND; ++k) Ad[i].d[k] = (c0 + k == ns + i) ? 1.0 : 0.0;
      }
      step_env<Dual<ND>>(*s, Xd.data(), Ad.data(), nullptr);
      for (int o = 0; o < ns; ++o)
        for (int k = 0; k < ND && c0 + k < nin; ++k) jac[((size_t)e * ns + o) * nin + c0 + k] = Xd[o].d[k];
    }
  }
  return 0;
}

// Floating-point operations of one environment step from the given state,
// counted by running the same code on the Counted scalar.
int64_t orc_count_flops(const OrcSys* s, const double* X, const double* act) {
  std::vector<Counted> Xc(s->nb * 13), Ac(s->na > 0 ? s->na : 1);
  for (int i = 0; i < s->nb * 13; ++i) Xc[i] = Counted(X[i]);
  for (int i = 0; i < s->na; ++i) Ac[i] = Counted(act[i]);
  g_flops = 0;
  step_env<Counted>(*s, Xc.data(), Ac.data(), nullptr);
  return g_flops;
}

// Floating-point operations of one reverse (adjoint) sweep through one
// environment step from the given state: the step is traced on the Traced
// scalar, the operations the outputs depend on are found by walking the
// trace backwards from the output state, and each contributes the cost of
// its adjoint rule (a fused multiply-add counts two):
//   z = x +- y   1 per operand that depends on the inputs (accumulate z')
//   z = x * y    2 per such operand (x' += z' y)
//   z = x / y    1 for t = z'/y, then 1 if x depends on the inputs (x' += t),
//                2 if y does (y' -= t z)
//   sqrt 3 (x' += z' * 0.5/z), asin 6 (1/sqrt(1 - x^2), then x' += z' *
//   that), sin and cos 3, atan2 4 (den = x^2 + y^2, t = z'/den) + 2 per
//   operand that depends on the inputs; a sign flip is free.
// This is the arithmetic of a reverse sweep over a stored forward pass; the
// forward pass itself is counted by orc_count_flops.
int64_t orc_count_vjp_flops(const OrcSys* s, const double* X, const double* act) {
  std::vector<TraceNode> trace;
  trace.reserve(1 << 16);
  g_trace = &trace;
  const int ns = s->nb * 13;
  std::vector<Traced> Xt(ns), At(s->na > 0 ? s->na : 1);
  for (int i = 0; i < ns; ++i) Xt[i] = trace_leaf(X[i]);
  for (int i = 0; i < s->na; ++i) At[i] = trace_leaf(act[i]);
  step_env<Traced>(*s, Xt.data(), At.data(), nullptr);
  g_trace = nullptr;
  std::vector<char> need(trace.size(), 0);
  for (int i = 0; i < ns; ++i)
    if (Xt[i].id >= 0) need[Xt[i].id] = 1;
  int64_t n = 0;
  for (int64_t k = (int64_t)trace.size() - 1; k >= 0; --k) {
    if (!need[k]) continue;
    const TraceNode& t = trace[k];
    const int na = t.a >= 0, nb = t.b >= 0;
    if (na) need[t.a] = 1;
    if (nb) need[t.b] = 1;
    switch (t.op) {
      case T_ADD: case T_SUB: n += na + nb; break;
      case T_MUL: n += 2 * (na + nb); break;
      case T_DIV: n += 1 + na + 2 * nb; break;
      case T_SQRT: case T_SIN: case T_COS: n += 3; break;
      case T_ASIN: n += 6; break;
      case T_ATAN2: n += 4 + 2 * (na + nb); break;
      default: break;
    }
  }
  return n;
}

// ---- single-phase entry points used by the pin tests ---------------------
// Rotation matrix of a quaternion (row-major 3x3).
void orc_quat_to_mat(const double* q, double* R) {
  Qt<double> qq = {q[0], q[1], q[2], q[3]};
  M3<double> M = quat_to_mat(qq);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[3 * i + j] = M.m[i][j];
}

// Euler angles (radians) and world Euler axes of every joint for one
// environment state X [nb*13]: theta [nj][3], axes [nj][3][3].
void orc_joint_angles(const OrcSys* s, const double* X, double* theta, double* axes) {
  Body<double> B[MAXB];
  Derived<double> D[MAXB];
  for (int i = 0; i < s->nb; ++i) {
    B[i] = load_body(X + 13 * i);
    D[i] = derive(*s, i, B[i]);
  }
  for (int j = 0; j < s->nj; ++j) {
    JointFrame<double> f = joint_frame(*s, j, D[s->j_parent[j]], D[s->j_child[j]]);
    for (int k = 0; k < 3; ++k) {
      theta[3 * j + k] = f.th[k];
      axes[9 * j + 3 * k + 0] = f.axis[k].x;
      axes[9 * j + 3 * k + 1] = f.axis[k].y;
      axes[9 * j + 3 * k + 2] = f.axis[k].z;
    }
  }
}

// Joint plus actuator force and torque on every body at a given (already
// kinematically integrated) state, without integrating: f [nb][3], t [nb][3].
void orc_joint_forces(const OrcSys* s, const double* X, const double* act, double* f, double* t) {
  Body<double> B[MAXB];
  Derived<double> D[MAXB];
  V3<double> fj[MAXB], tj[MAXB];
  for (int i = 0; i < s->nb; ++i) {
    B[i] = load_body(X + 13 * i);
    D[i] = derive(*s, i, B[i]);
    fj[i] = tj[i] = V3<double>{0, 0, 0};
  }
  JointFrame<double> fr[MAXJ];
  for (int j = 0; j < s->nj; ++j) fr[j] = joint_frame(*s, j, D[s->j_parent[j]], D[s->j_child[j]]);
  for (int j = 0; j < s->nj; ++j) joint_apply(*s, j, B, D, fr[j], fj, tj, (Margins*)nullptr);
  for (int k = 0; k < s->na; ++k) actuator_apply(*s, k, clampv(act[k], -1.0, 1.0), fr, tj);
  for (int i = 0; i < s->nb; ++i) {
    f[3 * i + 0] = fj[i].x; f[3 * i + 1] = fj[i].y; f[3 * i + 2] = fj[i].z;
    t[3 * i + 0] = tj[i].x; t[3 * i + 1] = tj[i].y; t[3 * i + 2] = tj[i].z;
  }
}

}  // extern "C"
