// Body-body contacts in the one-lane-per-body kernels (device code).
//
// Each candidate is evaluated on the lane of one of its two bodies (its
// handler, chosen when the tables are packed); the other body's state and
// frame come by cross-lane reads. The handler keeps its own body's share and
// leaves the other's, which that body's lane collects in the same evaluation
// slot from the handler lanes listed in its table row. The loops run to the
// type's maxima so that every cross-lane read executes on the whole
// wavefront; a lane without work in a slot reads its own values and
// discards them.
#pragma once
#include "bx_access.h"
#include "bx_pair_adj.h"

namespace bx {

__device__ __forceinline__ v3 shfl_v3(v3 a, int src) { return V(shfl(a.x, src), shfl(a.y, src), shfl(a.z, src)); }

// The state and frame of the body on lane src.
__device__ __forceinline__ PairSide shfl_side(const PairSide& s, int src) {
  PairSide o;
  o.p = shfl_v3(s.p, src);
  o.v = shfl_v3(s.v, src);
  o.w = shfl_v3(s.w, src);
#pragma unroll
  for (int k = 0; k < 9; ++k) o.R.m[k] = shfl(s.R.m[k], src);
  o.Iwinv = s3{shfl(s.Iwinv.xx, src), shfl(s.Iwinv.yy, src), shfl(s.Iwinv.zz, src),
               shfl(s.Iwinv.xy, src), shfl(s.Iwinv.xz, src), shfl(s.Iwinv.yz, src)};
  return o;
}

// Forward: adds this body's body-body velocity changes to dv, dw and the
// applied candidates to cnt (post-kinematic state s, frame f).
__device__ __forceinline__ void pair_phase(const Tables* __restrict__ tab, int t, int b, int base, const Body& s,
                                           const Frame& f, v3& dv, v3& dw, int& cnt) {
  const TypeT& ty = tab->type[t];
  const BodyT& Bg = tab->body[t][b];
  const int nh = Bg.nh;
  const PairSide me{s.p, s.v, s.w, f.R, f.Iwinv};
  for (int i = 0; i < ty.max_handled; ++i) {
    const bool mine = i < nh;
    const PairT& P = tab->pair[t][Bg.hp[i]];  // hp[i] = 0 past nh: a valid candidate, unused
    const bool first = P.a == b;
    const PairSide o = shfl_side(me, base + (mine ? (first ? P.b : P.a) : b));
    v3 odv = V(0.f, 0.f, 0.f), odw = odv;
    float on = 0.f;
    if (mine) {
      const PairSide A = sel(first, me, o), B = sel(first, o, me);
      v3 dvA, dwA, dvB, dwB;
      if (pair_eval(P, ty, A, B, dvA, dwA, dvB, dwB)) {
        dv += sel(first, dvA, dvB);
        dw += sel(first, dwA, dwB);
        odv = sel(first, dvB, dvA);
        odw = sel(first, dwB, dwA);
        on = 1.f;
        ++cnt;
      }
    }
    const int nr = Bg.nrecv[i];
    const uint32_t rv = Bg.recv[i];
    for (int k = 0; k < ty.recv_n[i]; ++k) {
      const int hsrc = base + (k < nr ? (int)((rv >> (4 * k)) & 15u) : b);
      const v3 a = shfl_v3(odv, hsrc), w = shfl_v3(odw, hsrc);
      const float got = shfl(on, hsrc);
      if (k < nr && got != 0.f) {
        dv += a;
        dw += w;
        ++cnt;
      }
    }
  }
}

// Adjoint: given this body's cotangents of its velocity-change sums (dvb,
// dwb), adds the cotangents of its post-kinematic state to tot, of its frame
// to fr, of its inverse mass to invm_bar (unless it has none here) and of the
// friction coefficient (on handler lanes) to mu_bar.
__device__ __forceinline__ void pair_phase_adj(const Tables* __restrict__ tab, int t, int b, int base,
                                               const Body& post, const Frame& f, v3 dvb, v3 dwb, Bar& tot,
                                               FrameBar& fr, float& invm_bar, float& mu_bar) {
  const TypeT& ty = tab->type[t];
  const BodyT& Bg = tab->body[t][b];
  const int nh = Bg.nh;
  const PairSide me{post.p, post.v, post.w, f.R, f.Iwinv};
  auto add = [&](const PairSideBar& x) {
    tot.p += x.p;
    tot.v += x.v;
    tot.w += x.w;
#pragma unroll
    for (int k = 0; k < 9; ++k) fr.Rb.m[k] += x.R.m[k];
    fr.Iwinvb.xx += x.Iwinv.xx;
    fr.Iwinvb.yy += x.Iwinv.yy;
    fr.Iwinvb.zz += x.Iwinv.zz;
    fr.Iwinvb.xy += x.Iwinv.xy;
    fr.Iwinvb.xz += x.Iwinv.xz;
    fr.Iwinvb.yz += x.Iwinv.yz;
    invm_bar += x.im;
  };
  for (int i = 0; i < ty.max_handled; ++i) {
    const bool mine = i < nh;
    const PairT& P = tab->pair[t][Bg.hp[i]];
    const bool first = P.a == b;
    const int src = base + (mine ? (first ? P.b : P.a) : b);
    const PairSide o = shfl_side(me, src);
    const v3 odvb = shfl_v3(dvb, src), odwb = shfl_v3(dwb, src);
    PairSideBar ob = pairbar_zero();  // the other body's cotangents, left for its lane
    if (mine) {
      const PairSide A = sel(first, me, o), B = sel(first, o, me);
      PairSideBar Ab = pairbar_zero(), Bb = pairbar_zero();
      if (pair_adj(P, ty, A, B, sel(first, dvb, odvb), sel(first, dwb, odwb), sel(first, odvb, dvb),
                   sel(first, odwb, dwb), Ab, Bb, mu_bar)) {
        // a body without inverse mass here (all translations frozen) has no mass cotangent from it
        if (P.im_a == 0.f) Ab.im = 0.f;
        if (P.im_b == 0.f) Bb.im = 0.f;
        add(sel(first, Ab, Bb));
        ob = sel(first, Bb, Ab);
      }
    }
    const int nr = Bg.nrecv[i];
    const uint32_t rv = Bg.recv[i];
    for (int k = 0; k < ty.recv_n[i]; ++k) {
      const int hsrc = base + (k < nr ? (int)((rv >> (4 * k)) & 15u) : b);
      PairSideBar x;
      x.p = shfl_v3(ob.p, hsrc);
      x.v = shfl_v3(ob.v, hsrc);
      x.w = shfl_v3(ob.w, hsrc);
#pragma unroll
      for (int q = 0; q < 9; ++q) x.R.m[q] = shfl(ob.R.m[q], hsrc);
      x.Iwinv = s3{shfl(ob.Iwinv.xx, hsrc), shfl(ob.Iwinv.yy, hsrc), shfl(ob.Iwinv.zz, hsrc),
                   shfl(ob.Iwinv.xy, hsrc), shfl(ob.Iwinv.xz, hsrc), shfl(ob.Iwinv.yz, hsrc)};
      x.im = shfl(ob.im, hsrc);
      if (k < nr) add(x);
    }
  }
}

}  // namespace bx
