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
//   * Section 6.1 "Spring Joints" — joints are stiff springs (with damping).
//   * Section 6.2 "Collisions" — velocity-level contact impulses with
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

enum { MAXB = 16, MAXJ = 16, MAXC = 96, MAXA = 48 };

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
enum { NMARGIN = 7 };
struct Margins {
  double contact_depth = 1e30;    // |penetration| of every candidate (m)
  double contact_speed = 1e30;    // |normal-impulse numerator| of candidates in contact (m/s)
  double angle_wrap = 1e30;       // pi - |theta| for limited free angles (rad)
  double slip_speed = 1e30;       // tangential contact speed of impulsive contacts (m/s)
  double cone_gap = 1e30;         // |mu jn - s/kt| / (mu jn): Coulomb cone vs sticking
  double limit_gap = 1e30;        // distance of a free angle to its limits (rad)
  double clip_gap = 1e30;         // 1 - |a| of every action
  void store(double* out) const {
    out[0] = contact_depth; out[1] = contact_speed; out[2] = angle_wrap; out[3] = slip_speed;
    out[4] = cone_gap; out[5] = limit_gap; out[6] = clip_gap;
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

// Joint update (Algorithm 1, joint loop; Section 6.1 spring joints).
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

// Collider update (Algorithm 1, collider loop; Section 6.2): one contact
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
