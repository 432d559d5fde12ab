// Adjoint of a body-body contact candidate (bx_pair.h) in FP32, with the
// conventions of bx_adj.h: the adjoint follows the branch the forward takes
// (the impulse passes only when applied, the Coulomb cap when cap <= stop,
// clamped closest-point parameters pass on the closed interval, the nearest
// face of a box is held), activation and counts carry no derivative.
#pragma once
#include "bx_adj.h"
#include "bx_pair.h"

namespace bx {

// Cotangents of one side of a candidate: its body's post-kinematic state and
// frame, and its inverse mass as the candidate reads it.
struct PairSideBar {
  v3 p, v, w;
  m3 R;
  s3 Iwinv;
  float im;
};
BXF PairSideBar pairbar_zero() {
  PairSideBar r;
  r.p = r.v = r.w = V(0.f, 0.f, 0.f);
  r.R = m3_zero();
  r.Iwinv = s3_zero();
  r.im = 0.f;
  return r;
}

// k(u) = imA + imB + [rot a] za . SA za + [rot b] zb . SB zb, za = rA x u
BXF void pair_k_adj(const PairT& c, const PairSide& A, const PairSide& B, v3 rA, v3 rB, v3 u, float kb,
                    PairSideBar& Ab, PairSideBar& Bb, v3& rAb, v3& rBb, v3& ub) {
  Ab.im += kb;
  Bb.im += kb;
  if (c.rot_a) {
    const v3 za = cross(rA, u);
    sym_outer_add(Ab.Iwinv, kb * za, za);
    cross_adj(rA, u, (2.f * kb) * mul(A.Iwinv, za), rAb, ub);
  }
  if (c.rot_b) {
    const v3 zb = cross(rB, u);
    sym_outer_add(Bb.Iwinv, kb * zb, zb);
    cross_adj(rB, u, (2.f * kb) * mul(B.Iwinv, zb), rBb, ub);
  }
}

BXF bool pass01(float raw) { return raw >= 0.f && raw <= 1.f; }

BXF PairSideBar sel(bool c, const PairSideBar& a, const PairSideBar& b) {
  PairSideBar r;
  r.p = sel(c, a.p, b.p);
  r.v = sel(c, a.v, b.v);
  r.w = sel(c, a.w, b.w);
  r.R = sel(c, a.R, b.R);
  r.Iwinv = sel(c, a.Iwinv, b.Iwinv);
  r.im = c ? a.im : b.im;
  return r;
}
BXF void add_to(m3& A, const m3& B) {
  for (int i = 0; i < 9; ++i) A.m[i] += B.m[i];
}

// Segment-segment parameters (seg_seg, case g.kase) -> cotangents of the
// directions d1, d2 and of r = p0 - q0.
BXF void seg_seg_adj(const PairGeo& g, v3 d1, v3 d2, v3 r, float sb, float tb, v3& d1b, v3& d2b, v3& rb) {
  float ab = 0.f, bb = 0.f, cb = 0.f, eb = 0.f, fb = 0.f;
  if (g.kase == 0) {  // t = clamp(f / e)
    if (g.e > 0.f && pass01(g.traw)) {
      fb += tb / g.e;
      eb -= tb * g.traw / g.e;
    }
  } else if (g.kase == 1 || g.kase == 3) {  // s = clamp(-c / a)
    if (pass01(g.sraw)) {
      cb -= sb / g.a;
      ab -= sb * g.sraw / g.a;
    }
  } else if (g.kase == 4) {  // s = clamp((b - c) / a)
    if (pass01(g.sraw)) {
      bb += sb / g.a;
      cb -= sb / g.a;
      ab -= sb * g.sraw / g.a;
    }
  } else {  // t = (b s + f) / e, s = clamp((b f - c e) / den), den = a e - b^2
    bb += tb * g.s / g.e;
    const float s0b = sb + tb * g.b / g.e;
    fb += tb / g.e;
    eb -= tb * g.traw / g.e;
    if (g.den > 0.f && pass01(g.sraw)) {
      const float numb = s0b / g.den, denb = -s0b * g.sraw / g.den;
      bb += numb * g.f - 2.f * denb * g.b;
      fb += numb * g.b;
      cb -= numb * g.e;
      eb += denb * g.a - numb * g.c;
      ab += denb * g.e;
    }
  }
  // a = d1.d1, e = d2.d2, f = d2.r, c = d1.r, b = d1.d2
  d1b += (2.f * ab) * d1 + cb * r + bb * d2;
  d2b += (2.f * eb) * d2 + fb * r + bb * d1;
  rb += fb * d2 + cb * d1;
}

// point_box -> cotangents of the point p, the box centre c and its rotation Rb,
// given those of the box point cbox, the box normal nbx and the signed distance.
BXF void point_box_adj(const PairGeo& g, const float* h, v3 cboxb, v3 nbxb, float sdb, v3& pb, v3& cb, m3& Rbb) {
  v3 qb;
  if (g.face < 0) {
    // d = p - cbox, sd = |d|, nbx = d / sd
    const v3 n = g.nbx;
    const v3 db = sdb * n + (1.f / g.dist) * (nbxb - dot(n, nbxb) * n);
    pb += db;
    const v3 cbt = cboxb - db;  // cbox = c + Rb cl, d = p - cbox
    cb += cbt;
    outer_add(Rbb, cbt, g.cl);
    const v3 clb = mul_t(g.Rb, cbt);
    qb = V(fabsf(g.q.x) <= h[0] ? clb.x : 0.f, fabsf(g.q.y) <= h[1] ? clb.y : 0.f, fabsf(g.q.z) <= h[2] ? clb.z : 0.f);
  } else {
    const int k = g.face;
    cb += cboxb;
    outer_add(Rbb, cboxb, g.cl);
    v3 clb = mul_t(g.Rb, cboxb);
    // the face coordinate of cl is the constant sg h_k; sd = |q_k| - h_k
    if (k == 0) clb.x = g.sg * sdb;
    else if (k == 1) clb.y = g.sg * sdb;
    else clb.z = g.sg * sdb;
    qb = clb;
    // nbx = sg (column k of Rb); k varies across lanes, so no indexing by it
    for (int j = 0; j < 3; ++j) {
      const float on = j == k ? g.sg : 0.f;
      Rbb.m[j] += on * nbxb.x;
      Rbb.m[3 + j] += on * nbxb.y;
      Rbb.m[6 + j] += on * nbxb.z;
    }
  }
  // q = Rb^T (p - c)
  const v3 w = g.p - g.bc;
  outer_add(Rbb, w, qb);
  const v3 wb = mul(g.Rb, qb);
  pb += wb;
  cb -= wb;
}

// seg_box_param -> cotangents of the segment's box coordinates q0s, dqs from
// that of the parameter: outside, s = -N / D over the coordinates beyond
// their faces; inside, the crossing s = (a_j - a_i) / (b_i - b_j) of lines
// a_m + b_m s = sg_m q_{k_m}(s) - h_{k_m}. An end (s = 0 or 1) passes nothing.
BXF void seg_box_param_adj(const PairGeo& g, const float* h, float sb, v3& q0b, v3& dqb) {
  const float qa[3] = {g.q0s.x, g.q0s.y, g.q0s.z}, qd[3] = {g.dqs.x, g.dqs.y, g.dqs.z};
  const float sg[3] = {g.sig.x, g.sig.y, g.sig.z};
  float a[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 0.f};
  if (g.sbin == 0) {
    if (g.sD > 0.f)
      for (int k = 0; k < 3; ++k)
        if (g.act & (1 << k)) {
          a[k] -= sb * qd[k] / g.sD;
          d[k] -= sb * (qa[k] - sg[k] * h[k] + 2.f * g.sst * qd[k]) / g.sD;
        }
  } else if (g.li >= 0) {
    const int ki = g.li >> 1, kj = g.lj >> 1;
    const float si = (g.li & 1) ? -1.f : 1.f, sj = (g.lj & 1) ? -1.f : 1.f;
    const float den = si * qd[ki] - sj * qd[kj];
    const float w = sb / den;
    for (int k = 0; k < 3; ++k) {
      a[k] += (k == kj ? sj * w : 0.f) - (k == ki ? si * w : 0.f);
      d[k] += (k == kj ? sj * g.sst * w : 0.f) - (k == ki ? si * g.sst * w : 0.f);
    }
  }
  q0b += V(a[0], a[1], a[2]);
  dqb += V(d[0], d[1], d[2]);
}

// Closest features -> side cotangents, given those of cb (through the
// contact point), n and dist.
BXF void pair_geometry_adj(const PairT& c, const PairGeo& g, v3 cbb, v3 nb, float distb, PairSideBar& Ab,
                           PairSideBar& Bb) {
  if (c.kind >= PK_SB) {
    const bool box_b = c.kind == PK_SB;
    const float* h = box_b ? c.bh : c.ah;
    // SB: cb = cbox, n = nbx; BS: cb = p, n = -nbx; p = a0 + s da
    const v3 z3 = V(0.f, 0.f, 0.f);
    v3 pb = sel(box_b, z3, cbb), ccb = z3;
    m3 Rbb = m3_zero();
    point_box_adj(g, h, sel(box_b, cbb, z3), sel(box_b, nb, -nb), distb, pb, ccb, Rbb);
    v3 a0b = pb, dab = g.sst * pb;
    const float sb = dot(pb, g.da);
    v3 q0b = z3, dqb = z3;
    seg_box_param_adj(g, h, sb, q0b, dqb);
    // q0s = Rb^T (a0 - c), dqs = Rb^T da
    outer_add(Rbb, g.a0 - g.bc, q0b);
    const v3 wb = mul(g.Rb, q0b);
    a0b += wb;
    ccb -= wb;
    outer_add(Rbb, g.da, dqb);
    dab += mul(g.Rb, dqb);
    // a0 = S.p + S.R l0, da = S.R (l1 - l0) (the segment's body); bc = X.p + X.R lc, Rb = X.R bR (the box's)
    m3 SRb = m3_zero(), XRb = m3_zero();
    const v3 l0 = ld3(box_b ? c.a0 : c.b0), l1 = ld3(box_b ? c.a1 : c.b1);
    outer_add(SRb, a0b, l0);
    outer_add(SRb, dab, l1 - l0);
    outer_add(XRb, ccb, ld3(box_b ? c.b0 : c.a0));
    if (c.box_rot) {
      const float* bR = box_b ? c.bR : c.aR;
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
          XRb.m[3 * i + k] +=
              Rbb.m[3 * i] * bR[3 * k] + Rbb.m[3 * i + 1] * bR[3 * k + 1] + Rbb.m[3 * i + 2] * bR[3 * k + 2];
    } else {
      add_to(XRb, Rbb);
    }
    Ab.p += sel(box_b, a0b, ccb);
    Bb.p += sel(box_b, ccb, a0b);
    add_to(Ab.R, sel(box_b, SRb, XRb));
    add_to(Bb.R, sel(box_b, XRb, SRb));
    return;
  }
  if (c.kind >= PK_PB) {
    const bool box_b = c.kind == PK_PB;
    // PB: cb = cbox, n = nbx; BP: cb = p, n = -nbx
    const v3 z3 = V(0.f, 0.f, 0.f);
    v3 pb = sel(box_b, z3, cbb), ccb = z3;
    m3 Rbb = m3_zero();
    point_box_adj(g, box_b ? c.bh : c.ah, sel(box_b, cbb, z3), sel(box_b, nb, -nb), distb, pb, ccb, Rbb);
    // p = P.p + P.R lp (the point's body), bc = X.p + X.R lc, Rb = X.R bR (the box's body)
    m3 PRb = m3_zero(), XRb = m3_zero();
    outer_add(PRb, pb, ld3(box_b ? c.a0 : c.b0));
    outer_add(XRb, ccb, ld3(box_b ? c.b0 : c.a0));
    if (c.box_rot) {
      const float* bR = box_b ? c.bR : c.aR;
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
          XRb.m[3 * i + k] +=
              Rbb.m[3 * i] * bR[3 * k] + Rbb.m[3 * i + 1] * bR[3 * k + 1] + Rbb.m[3 * i + 2] * bR[3 * k + 2];
    } else {
      add_to(XRb, Rbb);
    }
    Ab.p += sel(box_b, pb, ccb);
    Bb.p += sel(box_b, ccb, pb);
    add_to(Ab.R, sel(box_b, PRb, XRb));
    add_to(Bb.R, sel(box_b, XRb, PRb));
    return;
  }
  // d = ca - cb, dist = |d|, n = d / dist
  const v3 db = distb * g.n + (1.f / g.dist) * (nb - dot(g.n, nb) * g.n);
  const v3 cab = db, cbt = cbb - db;
  // ca = a0 + s da, cb = b0 + t db
  v3 a0b = cab, b0b = cbt;
  v3 dab = g.s * cab, dbb = g.t * cbt;
  const float sb = dot(cab, g.da), tb = dot(cbt, g.db);
  if (c.kind == PK_PS) {  // t = clamp((a0 - b0).db / db.db)
    if (dot(g.db, g.db) > 0.f && pass01(g.traw)) {
      const float dd = dot(g.db, g.db);
      const float gb = tb / dd, ddb = -tb * g.traw / dd;
      a0b += gb * g.db;
      b0b -= gb * g.db;
      dbb += gb * (g.a0 - g.b0) + (2.f * ddb) * g.db;
    }
  } else if (c.kind == PK_SP) {  // s = clamp((b0 - a0).da / da.da)
    if (dot(g.da, g.da) > 0.f && pass01(g.sraw)) {
      const float dd = dot(g.da, g.da);
      const float gb = sb / dd, ddb = -sb * g.sraw / dd;
      b0b += gb * g.da;
      a0b -= gb * g.da;
      dab += gb * (g.b0 - g.a0) + (2.f * ddb) * g.da;
    }
  } else if (c.kind == PK_SS) {
    v3 rb = V(0.f, 0.f, 0.f);
    seg_seg_adj(g, g.da, g.db, g.a0 - g.b0, sb, tb, dab, dbb, rb);
    a0b += rb;
    b0b -= rb;
  }
  // a0 = A.p + A.R la0, da = A.R (la1 - la0); the same for b
  Ab.p += a0b;
  outer_add(Ab.R, a0b, ld3(c.a0));
  if (c.kind == PK_SP || c.kind == PK_SS) outer_add(Ab.R, dab, ld3(c.a1) - ld3(c.a0));
  Bb.p += b0b;
  outer_add(Bb.R, b0b, ld3(c.b0));
  if (c.kind == PK_PS || c.kind == PK_SS) outer_add(Bb.R, dbb, ld3(c.b1) - ld3(c.b0));
}

// Adjoint of one candidate: given the cotangents of the two bodies' velocity
// change sums (dvA_b, dwA_b, dvB_b, dwB_b), accumulate the cotangents of both
// sides into Ab, Bb and of the friction coefficient into mu_b. Returns
// whether the forward applied an impulse (otherwise nothing is added).
BXF bool pair_adj(const PairT& c, const TypeT& ty, const PairSide& A, const PairSide& B, v3 dvAb, v3 dwAb, v3 dvBb,
                  v3 dwBb, PairSideBar& Ab, PairSideBar& Bb, float& mub) {
  PairGeo g;
  PairImp m;
  if (!pair_geometry(c, A, B, g) || !pair_impulse(c, ty, A, B, g, m)) return false;
  const v3 z3 = V(0.f, 0.f, 0.f);
  // shares: dvA = imA J, dwA = [rot a] SA (rA x J), dvB = -imB J, dwB = -[rot b] SB (rB x J)
  v3 Jb = c.im_a * dvAb - c.im_b * dvBb;
  Ab.im += dot(dvAb, m.J);
  Bb.im -= dot(dvBb, m.J);
  v3 rAb = z3, rBb = z3;
  if (c.rot_a) {
    sym_outer_add(Ab.Iwinv, dwAb, cross(m.rA, m.J));
    cross_adj(m.rA, m.J, mul(A.Iwinv, dwAb), rAb, Jb);
  }
  if (c.rot_b) {
    const v3 nb2 = -dwBb;
    sym_outer_add(Bb.Iwinv, nb2, cross(m.rB, m.J));
    cross_adj(m.rB, m.J, mul(B.Iwinv, nb2), rBb, Jb);
  }
  // J = jn n - jt t
  float jnb = dot(Jb, g.n), vnb = 0.f, depthb = 0.f;
  v3 nb = m.jn * Jb, ub = z3;
  if (m.sp > 0.f) {
    const float jtb = -dot(Jb, m.t);
    v3 tb = (-m.jt) * Jb;
    const float capb = m.use_cap ? jtb : 0.f, stopb = m.use_cap ? 0.f : jtb;
    jnb += ty.mu * capb;  // cap = mu jn
    mub += capb * m.jn;
    // stop = sp / kt
    const float spb = stopb / m.kt;
    const float ktb = -stopb * m.stop / m.kt;
    pair_k_adj(c, A, B, m.rA, m.rB, m.t, ktb, Ab, Bb, rAb, rBb, tb);
    // t = ut / sp, sp = |ut|, ut = u - vn n
    const v3 utb = (1.f / m.sp) * (tb - dot(tb, m.t) * m.t) + spb * m.t;
    ub += utb;
    vnb -= dot(utb, g.n);
    nb -= m.vn * utb;
  }
  // jn = num / kn
  const float numb = jnb / m.kn, knb = -jnb * m.jn / m.kn;
  pair_k_adj(c, A, B, m.rA, m.rB, g.n, knb, Ab, Bb, rAb, rBb, nb);
  // num = beta_h depth - (1 + e) vn; vn = u . n
  depthb += ty.beta_h * numb;
  vnb -= ty.one_plus_e * numb;
  ub += vnb * g.n;
  nb += vnb * m.u;
  // u = vA + wA x rA - vB - wB x rB
  Ab.v += ub;
  cross_adj(A.w, m.rA, ub, Ab.w, rAb);
  Bb.v -= ub;
  cross_adj(B.w, m.rB, -ub, Bb.w, rBb);
  // rA = x - pA, rB = x - pB; x = cb + (rb - depth / 2) n
  const v3 xb = rAb + rBb;
  Ab.p -= rAb;
  Bb.p -= rBb;
  nb += (c.rb - 0.5f * m.depth) * xb;
  depthb -= 0.5f * dot(xb, g.n);
  // depth = ra + rb - dist
  pair_geometry_adj(c, g, xb, nb, -depthb, Ab, Bb);
  return true;
}

}  // namespace bx
