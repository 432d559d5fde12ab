// Hand-written adjoints (vector-Jacobian products) of the per-item physics in
// bx_phys.h, in FP32. Each adjoint recomputes what it needs of its forward
// item from the forward inputs, then accumulates input cotangents ("bar"
// values) from output cotangents. Conventions at kinks follow the branch the
// forward takes: max(0,x) passes the gradient only when the impulse is applied;
// the Coulomb cap is used when cap <= stop; clamp and clip pass the gradient on
// the closed interval; contact activation and the contact count carry none;
// asin at |x| >= 1 has derivative zero.
#pragma once
#include "bx_phys.h"

namespace bx {

// ------------------------------------------------------------ primitive adjoints
struct Bar {  // cotangent of one body's state
  v3 p;
  q4 q;
  v3 v, w;
};
BXF Bar bar_zero() {
  Bar b;
  b.p = b.v = b.w = V(0.f, 0.f, 0.f);
  b.q = q4{0.f, 0.f, 0.f, 0.f};
  return b;
}
BXF void bar_add(Bar& a, const Bar& b) {
  a.p += b.p;
  a.q = q4{a.q.w + b.q.w, a.q.x + b.q.x, a.q.y + b.q.y, a.q.z + b.q.z};
  a.v += b.v;
  a.w += b.w;
}
BXF m3 m3_zero() { return m3{{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}}; }
BXF s3 s3_zero() { return s3{0.f, 0.f, 0.f, 0.f, 0.f, 0.f}; }

// y = A v  ->  A_bar += y_bar v^T
BXF void outer_add(m3& A, v3 yb, v3 v) {
  A.m[0] += yb.x * v.x; A.m[1] += yb.x * v.y; A.m[2] += yb.x * v.z;
  A.m[3] += yb.y * v.x; A.m[4] += yb.y * v.y; A.m[5] += yb.y * v.z;
  A.m[6] += yb.z * v.x; A.m[7] += yb.z * v.y; A.m[8] += yb.z * v.z;
}
// y = S v for a symmetric S stored once per off-diagonal pair
BXF void sym_outer_add(s3& S, v3 yb, v3 v) {
  S.xx += yb.x * v.x;
  S.yy += yb.y * v.y;
  S.zz += yb.z * v.z;
  S.xy += yb.x * v.y + yb.y * v.x;
  S.xz += yb.x * v.z + yb.z * v.x;
  S.yz += yb.y * v.z + yb.z * v.y;
}
// S = R diag(d) R^T  ->  R_bar
BXF void rot_diag_adj(const m3& R, const float* d, const s3& Sb, m3& Rb) {
  // S_ij = sum_k R_ik d_k R_jk; off-diagonals stored once
  const float* r = R.m;
  for (int k = 0; k < 3; ++k) {
    float r0 = r[k], r1 = r[3 + k], r2 = r[6 + k];
    Rb.m[k] += d[k] * (2.f * Sb.xx * r0 + Sb.xy * r1 + Sb.xz * r2);
    Rb.m[3 + k] += d[k] * (2.f * Sb.yy * r1 + Sb.xy * r0 + Sb.yz * r2);
    Rb.m[6 + k] += d[k] * (2.f * Sb.zz * r2 + Sb.xz * r0 + Sb.yz * r1);
  }
}
// R = quat_to_mat(q)  ->  q_bar (derivative of the polynomial form)
BXF void quat_to_mat_adj(q4 q, const m3& Rb, q4& qb) {
  const float* b = Rb.m;
  qb.w += 2.f * (-q.z * b[1] + q.y * b[2] + q.z * b[3] - q.x * b[5] - q.y * b[6] + q.x * b[7]);
  qb.x += 2.f * (q.y * b[1] + q.z * b[2] + q.y * b[3] - 2.f * q.x * b[4] - q.w * b[5] + q.z * b[6] + q.w * b[7] -
                 2.f * q.x * b[8]);
  qb.y += 2.f * (-2.f * q.y * b[0] + q.x * b[1] + q.w * b[2] + q.x * b[3] + q.z * b[5] - q.w * b[6] + q.z * b[7] -
                 2.f * q.y * b[8]);
  qb.z += 2.f * (-2.f * q.z * b[0] - q.w * b[1] + q.x * b[2] + q.w * b[3] - 2.f * q.z * b[4] + q.y * b[5] +
                 q.x * b[6] + q.y * b[7]);
}
// Frame (R, Iw, Iwinv) cotangents -> q_bar
BXF void frame_adj(const BodyT& B, const Body& s, const Frame& f, const m3& Rb_in, const s3& Iwinvb, q4& qb) {
  m3 Rb = Rb_in;
  rot_diag_adj(f.R, B.Iinv, Iwinvb, Rb);
  quat_to_mat_adj(s.q, Rb, qb);
}
// Cotangents of a body's frame (R, Iwinv), summed over the items of a
// substep that read it; frame_adj is linear in them, so one conversion to
// q_bar per body and substep serves every item. Ib: the cotangent of the
// principal moments from the gyroscopic term (for parameter gradients).
struct FrameBar {
  m3 Rb;
  s3 Iwinvb;
  v3 Ib;
};
BXF FrameBar framebar_zero() { return FrameBar{m3_zero(), s3_zero(), V(0.f, 0.f, 0.f)}; }
BXF void frame_adj(const BodyT& B, const Body& s, const Frame& f, const FrameBar& fr, q4& qb) {
  frame_adj(B, s, f, fr.Rb, fr.Iwinvb, qb);
}
// c = a x b  ->  a_bar += b x c_bar, b_bar += c_bar x a
BXF void cross_adj(v3 a, v3 b, v3 cb, v3& ab, v3& bb) {
  ab += cross(b, cb);
  bb += cross(cb, a);
}
BXF q4 qscale(float s, q4 a) { return q4{s * a.w, s * a.x, s * a.y, s * a.z}; }
BXF q4 qadd(q4 a, q4 b) { return q4{a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z}; }

// ------------------------------------------------------------ kinematic
// Forward: v' = keep(v), w' = keep(w), p1 = p + h v', q1 = normalize(q + h/2 (0,w') (x) q).
// Given the cotangent of (p1, q1, v', w'), return that of (p, q, v, w).
BXF Bar kinematic_adj(const BodyT& B, const Body& pre, float h, const Bar& ob) {
  v3 w = keep(pre.w, B.free_r);
  float hh = 0.5f * h;
  q4 dq = qmul(q4{0.f, w.x, w.y, w.z}, pre.q);
  q4 qu{pre.q.w + hh * dq.w, pre.q.x + hh * dq.x, pre.q.y + hh * dq.y, pre.q.z + hh * dq.z};
  float inv = 1.f / sqrtf(qu.w * qu.w + qu.x * qu.x + qu.y * qu.y + qu.z * qu.z);
  q4 q1{qu.w * inv, qu.x * inv, qu.y * inv, qu.z * inv};
  float pr = q1.w * ob.q.w + q1.x * ob.q.x + q1.y * ob.q.y + q1.z * ob.q.z;
  q4 qub{(ob.q.w - q1.w * pr) * inv, (ob.q.x - q1.x * pr) * inv, (ob.q.y - q1.y * pr) * inv,
         (ob.q.z - q1.z * pr) * inv};
  Bar r;
  // dq = L(wq) q: q_bar += L(wq)^T dq_bar; wq_bar = R(q)^T dq_bar, dq_bar = hh qu_bar
  q4 db = qscale(hh, qub);
  const q4 a{0.f, w.x, w.y, w.z};
  q4 qb{a.w * db.w + a.x * db.x + a.y * db.y + a.z * db.z, -a.x * db.w + a.w * db.x + a.z * db.y - a.y * db.z,
        -a.y * db.w - a.z * db.x + a.w * db.y + a.x * db.z, -a.z * db.w + a.y * db.x - a.x * db.y + a.w * db.z};
  const q4& b = pre.q;
  // R(b)^T db, keeping the vector part (the scalar part of (0, w) is constant)
  v3 wb = V(-b.x * db.w + b.w * db.x - b.z * db.y + b.y * db.z, -b.y * db.w + b.z * db.x + b.w * db.y - b.x * db.z,
            -b.z * db.w - b.y * db.x + b.x * db.y + b.w * db.z);
  r.q = qadd(qub, qb);
  r.p = ob.p;
  r.v = keep(ob.v + h * ob.p, B.free_p);
  r.w = keep(ob.w + wb, B.free_r);
  return r;
}

// ------------------------------------------------------------ potential + collision
// Forward (per body, after the kinematic update, with frame f):
//   v2 = v' + keep(h (g + f_tot/m)), w2 = w' + keep(h Iwinv (t_tot - w' x (Iw w')))
//   v3 = v2 + keep(dv_sum/n), w3 = w2 + keep(dw_sum/n)            (n > 0)
// Given the cotangent of (p1, q1, v3, w3) (ob), returns the partial cotangent
// of the post-kinematic state and the cotangents of f_tot, t_tot and of the
// contact sums (dvb, dwb; zero when n == 0).
// invm_bar accumulates the cotangent of 1/m given the total force f_tot.
BXF Bar integrate_adj(const BodyT& B, const TypeT& ty, const Body& post, const Frame& f, v3 t_tot, int n,
                      const Bar& ob, v3& fb, v3& tb, v3& dvb, v3& dwb, FrameBar& fr, v3 f_tot, float& invm_bar) {
  const float h = ty.h;
  Bar r;
  r.p = ob.p;
  r.q = ob.q;
  r.v = ob.v;
  r.w = ob.w;
  if (n > 0) {
    float inv = 1.f / (float)n;
    dvb = inv * keep(ob.v, B.free_p);
    dwb = inv * keep(ob.w, B.free_r);
  } else {
    dvb = dwb = V(0.f, 0.f, 0.f);
  }
  fb = (h * B.inv_m) * keep(ob.v, B.free_p);
  invm_bar += h * dot(keep(ob.v, B.free_p), f_tot);
  v3 ab = h * keep(ob.w, B.free_r);           // cotangent of alpha = Iwinv x
  // the gyroscopic term in the body frame, as the forward forms it:
  // wb = R^T w', y = I wb, u = R y (the world inertia times w'), gyro = w' x u
  const v3 wb = mul_t(f.R, post.w);
  const v3 y = V(B.I[0] * wb.x, B.I[1] * wb.y, B.I[2] * wb.z);
  v3 u = mul(f.R, y);
  v3 x = t_tot - cross(post.w, u);
  sym_outer_add(fr.Iwinvb, ab, x);
  v3 xb = mul(f.Iwinv, ab);
  tb = xb;
  v3 gb = -xb;                               // gyro = w' x u
  v3 ub = V(0.f, 0.f, 0.f);
  cross_adj(post.w, u, gb, r.w, ub);
  // u = R y: R_bar += ub y^T, y_bar = R^T ub; y = I wb: wb_bar = I y_bar,
  // I_bar += y_bar wb; wb = R^T w': w'_bar += R wb_bar, R_bar += w' wb_bar^T
  const v3 yb = mul_t(f.R, ub);
  const v3 wbb = V(B.I[0] * yb.x, B.I[1] * yb.y, B.I[2] * yb.z);
  r.w += mul(f.R, wbb);
  outer_add(fr.Rb, ub, y);
  outer_add(fr.Rb, post.w, wbb);
  fr.Ib += V(yb.x * wb.x, yb.y * wb.y, yb.z * wb.z);
  return r;
}
BXF Bar integrate_adj(const BodyT& B, const TypeT& ty, const Body& post, const Frame& f, v3 t_tot, int n,
                      const Bar& ob, v3& fb, v3& tb, v3& dvb, v3& dwb) {
  FrameBar fr = framebar_zero();
  float unused = 0.f;
  Bar r = integrate_adj(B, ty, post, f, t_tot, n, ob, fb, tb, dvb, dwb, fr, V(0.f, 0.f, 0.f), unused);
  frame_adj(B, post, f, fr, r.q);
  return r;
}

// ------------------------------------------------------------ contact
// Cotangent of the body's post-kinematic state from one applied contact,
// given the cotangents of the body's contact sums (dvb, dwb).
// invm_bar / mu_bar accumulate the cotangents of 1/m and of the friction
// coefficient.
BXF Bar contact_adj(const ContactT& c, const TypeT& ty, const BodyT& B, const Body& s, const Frame& f, v3 dvb, v3 dwb,
                    bool& applied, FrameBar& fr, float& invm_bar, float& mu_bar) {
  Bar r = bar_zero();
  applied = false;
  v3 l = ld3(c.l);
  v3 rl = mul(f.R, l);
  float depth = c.rho - (s.p.z + rl.z);
  if (!(depth > 0.f)) return r;
  v3 rr = V(rl.x, rl.y, rl.z - c.rho);
  v3 u = s.v + cross(s.w, rr);
  v3 zz = V(rr.y, -rr.x, 0.f);
  v3 a = mul(f.Iwinv, zz);
  float kn = B.inv_m + (a.x * rr.y - a.y * rr.x);
  float num = ty.beta_h * depth - ty.one_plus_e * u.z;
  if (!(num > 0.f)) return r;
  applied = true;
  float jn = num / kn;
  v3 J = V(0.f, 0.f, jn);
  // the forward's friction branch and normalisation (contact_eval)
  const float sp2 = u.x * u.x + u.y * u.y;
  const bool slip = sp2 > 0.f;
  v3 t = V(0.f, 0.f, 0.f), zt = V(0.f, 0.f, 0.f), b = V(0.f, 0.f, 0.f);
  float kt = 0.f, stop = 0.f, cap = 0.f, jt = 0.f, isp = 0.f, sp = 0.f;
  bool use_cap = false;
  if (slip) {
    isp = 1.f / sqrtf(sp2);
    sp = sp2 * isp;
    t = V(u.x * isp, u.y * isp, 0.f);
    zt = cross(rr, t);
    b = mul(f.Iwinv, zt);
    kt = B.inv_m + dot(zt, b);
    stop = sp / kt;
    cap = ty.mu * jn;
    use_cap = cap <= stop;
    jt = use_cap ? cap : stop;
    J.x = -jt * t.x;
    J.y = -jt * t.y;
  }
  // outputs: dv = inv_m J; dw = Iwinv (r x J)
  v3 y = cross(rr, J);
  sym_outer_add(fr.Iwinvb, dwb, y);
  v3 yb = mul(f.Iwinv, dwb);
  v3 rb = V(0.f, 0.f, 0.f), Jb = B.inv_m * dvb;
  invm_bar += dot(dvb, J);                   // dv = inv_m J
  cross_adj(rr, J, yb, rb, Jb);
  float jnb = Jb.z;
  v3 ub = V(0.f, 0.f, 0.f);
  if (slip) {
    float jtb = -(Jb.x * t.x + Jb.y * t.y);
    v3 tb = V(-jt * Jb.x, -jt * Jb.y, 0.f);
    float capb = use_cap ? jtb : 0.f, stopb = use_cap ? 0.f : jtb;
    jnb += ty.mu * capb;
    mu_bar += capb * jn;                     // cap = mu jn
    float spb = stopb / kt;
    float ktb = -stopb * sp / (kt * kt);
    invm_bar += ktb;
    // kt = inv_m + zt . Iwinv zt, zt = r x t (Iwinv symmetric)
    sym_outer_add(fr.Iwinvb, ktb * zt, zt);
    v3 ztb = (2.f * ktb) * b;
    cross_adj(rr, t, ztb, rb, tb);
    // t = u_xy / sp, sp = |u_xy|
    float tdot = tb.x * t.x + tb.y * t.y;
    ub.x += (tb.x - t.x * tdot) * isp + spb * t.x;
    ub.y += (tb.y - t.y * tdot) * isp + spb * t.y;
  }
  // jn = num / kn
  float numb = jnb / kn;
  float knb = -jnb * jn / kn;
  invm_bar += knb;                           // kn = inv_m + ...
  float depthb = ty.beta_h * numb;
  ub.z += -ty.one_plus_e * numb;
  // kn = inv_m + a.x r.y - a.y r.x, a = Iwinv zz, zz = (r.y, -r.x, 0)
  v3 abar = V(knb * rr.y, -knb * rr.x, 0.f);
  rb.y += knb * a.x;
  rb.x += -knb * a.y;
  sym_outer_add(fr.Iwinvb, abar, zz);
  v3 zzb = mul(f.Iwinv, abar);
  rb.y += zzb.x;
  rb.x += -zzb.y;
  // u = v + w x r
  r.v += ub;
  cross_adj(s.w, rr, ub, r.w, rb);
  // r = R l - rho z; depth = rho - p.z - (R l).z
  v3 rlb = rb;
  r.p.z -= depthb;
  rlb.z -= depthb;
  outer_add(fr.Rb, rlb, l);
  return r;
}
BXF Bar contact_adj(const ContactT& c, const TypeT& ty, const BodyT& B, const Body& s, const Frame& f, v3 dvb, v3 dwb,
                    bool& applied) {
  FrameBar fr = framebar_zero();
  float u0 = 0.f, u1 = 0.f;
  Bar r = contact_adj(c, ty, B, s, f, dvb, dwb, applied, fr, u0, u1);
  if (applied) frame_adj(B, s, f, fr, r.q);
  return r;
}

// ------------------------------------------------------------ joint geometry
struct GeoBar {
  v3 rP, rC;
  v3 e1P, e2P, e3P, e1C, e2C, e3C;
  float th[3];
  v3 ax[3];
};
BXF GeoBar geobar_zero() {
  GeoBar g;
  g.rP = g.rC = g.e1P = g.e2P = g.e3P = g.e1C = g.e2C = g.e3C = V(0.f, 0.f, 0.f);
  g.th[0] = g.th[1] = g.th[2] = 0.f;
  g.ax[0] = g.ax[1] = g.ax[2] = V(0.f, 0.f, 0.f);
  return g;
}

// Geometry cotangents -> q_bar of parent and child.
// The child's rotation cotangent is added to RbC (its frame_adj follows
// later); the parent's is turned into q_bar here.
template <int MAXDOF>
BXF void joint_geo_adj(const JointT& J, const Body& P, const JointGeo& g, GeoBar gb, q4& qbP, m3& RbC_acc) {
  float m12b = 0.f, m22b = 0.f, m01b = 0.f, m00b = 0.f, m02b = 0.f;
  // axes: ax0 = e1P, ax1 = c1 e2P + s1 e3P, ax2 = e3C
  gb.e1P += gb.ax[0];
  gb.e3C += gb.ax[2];
  float c1b = dot(gb.ax[1], g.e2P), s1b = dot(gb.ax[1], g.e3P);
  gb.e2P += g.c1 * gb.ax[1];
  gb.e3P += g.s1 * gb.ax[1];
  // (c1, s1) = (x, y) / r with x = m22, y = -m12
  float x = g.m22, yy = -g.m12;
  float r2 = x * x + yy * yy;
  if (r2 > 0.f) {
    float r = sqrtf(r2), r3 = r2 * r;
    float xb = (yy * yy * c1b - x * yy * s1b) / r3;
    float ybb = (x * x * s1b - x * yy * c1b) / r3;
    // th1 = atan2(y, x)
    xb += -gb.th[0] * yy / r2;
    ybb += gb.th[0] * x / r2;
    m22b += xb;
    m12b -= ybb;
  }
  if (MAXDOF > 1) {
    if (g.m02 > -1.f && g.m02 < 1.f) m02b += gb.th[1] / sqrtf(1.f - g.m02 * g.m02);
    float d3 = g.m00 * g.m00 + g.m01 * g.m01;
    if (d3 > 0.f) {
      // th3 = atan2(-m01, m00)
      m01b += -gb.th[2] * g.m00 / d3;
      m00b += gb.th[2] * g.m01 / d3;
    }
    gb.e1P += m01b * g.e2C + m00b * g.e1C + m02b * g.e3C;
    gb.e2C += m01b * g.e1P;
    gb.e1C += m00b * g.e1P;
    gb.e3C += m02b * g.e1P;
  }
  gb.e2P += m12b * g.e3C;
  gb.e3C += m12b * g.e2P + m22b * g.e3P;
  gb.e3P += m22b * g.e3C;
  // columns of AwP = RP FP, AwC = RC FC: R_bar += Aw_bar FP^T
  m3 AbP, AbC;
  v3 cP[3] = {gb.e1P, gb.e2P, gb.e3P}, cC[3] = {gb.e1C, gb.e2C, gb.e3C};
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      AbP.m[3 * i + k] = i == 0 ? cP[k].x : (i == 1 ? cP[k].y : cP[k].z);
      AbC.m[3 * i + k] = i == 0 ? cC[k].x : (i == 1 ? cC[k].y : cC[k].z);
    }
  m3 RbP = m3_zero();
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      float sp = 0.f, sc = 0.f;
      for (int k = 0; k < 3; ++k) {
        sp += AbP.m[3 * i + k] * J.FP[3 * j + k];
        sc += AbC.m[3 * i + k] * J.FC[3 * j + k];
      }
      RbP.m[3 * i + j] = sp;
      RbC_acc.m[3 * i + j] += sc;
    }
  outer_add(RbP, gb.rP, ld3(J.ap));
  outer_add(RbC_acc, gb.rC, ld3(J.ac));
  quat_to_mat_adj(P.q, RbP, qbP);
}
template <int MAXDOF>
BXF void joint_geo_adj(const JointT& J, const Body& P, const Body& C, const JointGeo& g, const GeoBar& gb, q4& qbP,
                       q4& qbC) {
  m3 RbC = m3_zero();
  joint_geo_adj<MAXDOF>(J, P, g, gb, qbP, RbC);
  quat_to_mat_adj(C.q, RbC, qbC);
}

// Spring part of a joint's adjoint on given geometry: accumulates into the
// state cotangents (bP, bC) and the geometry cotangents (gb).
template <int MAXDOF>
// jbar (nullable) accumulates the cotangents of k_lin, c_lin, k_ang, c_ang, k_lim.
BXF void spring_adj_core(const JointT& J, const Body& P, const Body& C, const JointGeo& g, v3 fcb, v3 tcb, v3 fpb,
                         v3 tpb, Bar& bP, Bar& bC, GeoBar& gb, float* jbar = nullptr) {
  v3 F;
  (void)joint_spring<MAXDOF>(J, P, C, g, F);
  // fc = F, tc = rC x F + tau, fp = -F, tp = -(rP x F) - tau
  v3 Fb = fcb - fpb;
  v3 taub = tcb - tpb;
  cross_adj(g.rC, F, tcb, gb.rC, Fb);
  cross_adj(g.rP, F, -tpb, gb.rP, Fb);
  // limits: tau += -k_lim ex_k ax_k, ex = th - clamp(th)
  for (int k = 0; k < MAXDOF; ++k) {
    if (MAXDOF == 1 || k < J.dof) {
      float ex = g.th[k] - clampf(g.th[k], J.lo[k], J.hi[k]);
      gb.ax[k] += (-J.k_lim * ex) * taub;
      float exb = -J.k_lim * dot(g.ax[k], taub);
      if (jbar) jbar[4] += -ex * dot(g.ax[k], taub);
      bool inside = g.th[k] >= J.lo[k] && g.th[k] <= J.hi[k];
      gb.th[k] += inside ? 0.f : exb;
    }
  }
  // damper
  bP.w += J.c_ang * taub;
  bC.w += -J.c_ang * taub;
  if (jbar) jbar[3] += dot(P.w - C.w, taub);
  // alignment
  if (MAXDOF == 1 || J.dof == 1) {
    v3 a = J.k_ang * taub;  // tau = k (e1C x e1P)
    cross_adj(g.e1C, g.e1P, a, gb.e1C, gb.e1P);
    if (jbar) jbar[2] += dot(cross(g.e1C, g.e1P), taub);
  } else if (J.dof == 2) {
    v3 wv = cross(g.e2C, g.e1P);  // tau = (-k m01) wv
    float m01b = -J.k_ang * dot(wv, taub);
    v3 wb = (-J.k_ang * g.m01) * taub;
    if (jbar) jbar[2] += -g.m01 * dot(wv, taub);
    cross_adj(g.e2C, g.e1P, wb, gb.e2C, gb.e1P);
    gb.e1P += m01b * g.e2C;
    gb.e2C += m01b * g.e1P;
  }
  // anchor spring-damper: F = k d + c (uP - uC)
  v3 db = J.k_lin * Fb;
  v3 uPb = J.c_lin * Fb, uCb = -J.c_lin * Fb;
  if (jbar) {
    const v3 d = (P.p - C.p) + (g.rP - g.rC);
    const v3 du = (P.v + cross(P.w, g.rP)) - (C.v + cross(C.w, g.rC));
    jbar[0] += dot(d, Fb);
    jbar[1] += dot(du, Fb);
  }
  bP.v += uPb;
  cross_adj(P.w, g.rP, uPb, bP.w, gb.rP);
  bC.v += uCb;
  cross_adj(C.w, g.rC, uCb, bC.w, gb.rC);
  bP.p += db;
  bC.p += -db;
  gb.rP += db;
  gb.rC += -db;
}

// Actuator part on given geometry: child torque cotangent tcb, parent tpb.
template <int MAXDOF>
// gbar (nullable) accumulates the cotangents of the actuator strengths per axis.
BXF void actuator_adj_core(const JointT& J, const JointGeo& g, const float* a, v3 tcb, v3 tpb, GeoBar& gb,
                           float* ab, float* gbar = nullptr) {
  v3 taub = tcb - tpb;
  for (int k = 0; k < 3; ++k) ab[k] = 0.f;
  for (int k = 0; k < MAXDOF; ++k) {
    if (MAXDOF == 1 || k < J.dof) {
      // tau += gear (a - pd theta) ax
      gb.ax[k] += (J.gear[k] * (a[k] - J.act_pd[k] * g.th[k])) * taub;
      ab[k] = J.gear[k] * dot(g.ax[k], taub);
      gb.th[k] -= J.act_pd[k] * ab[k];
      if (gbar) gbar[k] += (a[k] - J.act_pd[k] * g.th[k]) * dot(g.ax[k], taub);
    }
  }
}

// Spring joint adjoint: given the cotangents of (fc, tc, fp, tp), accumulate
// into the parent's and child's post-kinematic state cotangents.
template <int MAXDOF>
BXF void joint_spring_adj(const JointT& J, const Body& P, const m3& RP, const Body& C, const m3& RC, v3 fcb, v3 tcb,
                          v3 fpb, v3 tpb, Bar& bP, Bar& bC) {
  JointGeo g = joint_geo<MAXDOF>(J, RP, RC);
  GeoBar gb = geobar_zero();
  spring_adj_core<MAXDOF>(J, P, C, g, fcb, tcb, fpb, tpb, bP, bC, gb);
  joint_geo_adj<MAXDOF>(J, P, C, g, gb, bP.q, bC.q);
}

// Actuator adjoint: given the cotangent of the child's torque (the parent
// gets the opposite torque), accumulate into both rotations and return the
// cotangents of the clipped actions.
template <int MAXDOF>
BXF void joint_actuator_adj(const JointT& J, const Body& P, const m3& RP, const Body& C, const m3& RC, const float* a,
                            v3 tcb, v3 tpb, Bar& bP, Bar& bC, float* ab) {
  JointGeo g = joint_geo<MAXDOF>(J, RP, RC);
  GeoBar gb = geobar_zero();
  actuator_adj_core<MAXDOF>(J, g, a, tcb, tpb, gb, ab);
  joint_geo_adj<MAXDOF>(J, P, C, g, gb, bP.q, bC.q);
}

// Geometry adjoint of a one-axis joint on joint_geo_step's geometry: the
// cotangents of rP, rC, e1P, e1C, th0 and ax0 (= e1P) into the parent's
// quaternion (qbP) and the child's rotation (RbC_acc). There th0 =
// atan2(-m12, m22) with m12, m22 the parent frame's y and z columns
// against v = RP^T e3C.
BXF void joint_geo1_adj(const JointT& J, const Body& P, const m3& RP, const JointGeo& g, GeoBar gb, q4& qbP,
                        m3& RbC_acc) {
  gb.e1P += gb.ax[0];
  float m12b = 0.f, m22b = 0.f;
  const float x = g.m22, yy = -g.m12, r2 = x * x + yy * yy;
  if (r2 > 0.f) {
    m22b = -gb.th[0] * yy / r2;
    m12b = -(gb.th[0] * x / r2);
  }
  const v3 vb = m12b * V(J.FP[1], J.FP[4], J.FP[7]) + m22b * V(J.FP[2], J.FP[5], J.FP[8]);
  m3 RbP = m3_zero();
  outer_add(RbP, g.e3C, vb);  // v = RP^T e3C
  const v3 e3Cb = mul(RP, vb);
  outer_add(RbP, gb.e1P, V(J.FP[0], J.FP[3], J.FP[6]));  // e1P = RP fp1
  outer_add(RbP, gb.rP, ld3(J.ap));                       // rP = RP ap
  outer_add(RbC_acc, gb.e1C, V(J.FC[0], J.FC[3], J.FC[6]));
  outer_add(RbC_acc, e3Cb, V(J.FC[2], J.FC[5], J.FC[8]));
  outer_add(RbC_acc, gb.rC, ld3(J.ac));
  quat_to_mat_adj(P.q, RbP, qbP);
}

// Spring and actuators together (the fused path): geometry computed once;
// the child's rotation cotangent is added to its frame cotangents fr. A
// one-axis joint takes the step's own geometry (joint_geo_step) and its
// adjoint, without the Euler frame of the multi-axis joints.
template <int MAXDOF>
BXF void joint_eval_adj(const JointT& J, const Body& P, const m3& RP, const Body& C, const m3& RC, const float* a,
                        v3 fcb, v3 tcb, v3 fpb, v3 tpb, Bar& bP, Bar& bC, float* ab, FrameBar& fr,
                        float* jbar = nullptr, float* gbar = nullptr) {
  if (MAXDOF == 1) {
    const JointGeo g = joint_geo_step<1>(J, RP, joint_child<1>(J, C, RC));
    GeoBar gb = geobar_zero();
    spring_adj_core<1>(J, P, C, g, fcb, tcb, fpb, tpb, bP, bC, gb, jbar);
    actuator_adj_core<1>(J, g, a, tcb, tpb, gb, ab, gbar);
    joint_geo1_adj(J, P, RP, g, gb, bP.q, fr.Rb);
    return;
  }
  JointGeo g = joint_geo<MAXDOF>(J, RP, RC);
  GeoBar gb = geobar_zero();
  spring_adj_core<MAXDOF>(J, P, C, g, fcb, tcb, fpb, tpb, bP, bC, gb, jbar);
  actuator_adj_core<MAXDOF>(J, g, a, tcb, tpb, gb, ab, gbar);
  joint_geo_adj<MAXDOF>(J, P, g, gb, bP.q, fr.Rb);
}

}  // namespace bx
