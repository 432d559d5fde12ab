// Body-body contacts in the one-lane-per-body kernels (device code).
//
// Each candidate is evaluated on the lane of one body of the environment
// (its handler, chosen when the tables are packed so that the candidates
// spread over all of the environment's lanes); the two bodies' states and
// frames come from the side rows every lane writes to LDS once per substep.
// The handler writes both shares to its exchange row; in the same evaluation
// slot each body's lane collects its shares from the handler lanes listed in
// its table row, first-body shares and second-body shares in two passes. An
// evaluation slot in which no lane of the wavefront has a candidate that
// passes its bound test (one feature's distance from a ball around the
// other's: no contact is possible where it fails) is skipped as a whole. The loops run to the type's maxima, so that the
// wavefront takes every read together; a lane without work in a slot reads
// its own values and discards them.
#pragma once
#include "bx_access.h"
#include "bx_pair_adj.h"

namespace bx {

__device__ __forceinline__ v3 shfl_v3(v3 a, int src) { return V(shfl(a.x, src), shfl(a.y, src), shfl(a.z, src)); }

// One wavefront's copy, in LDS, of its system type's body-body tables: the
// lanes read them at lane-varying indices every substep, which from LDS
// costs a fraction of the latency of the device-memory tables.
struct PairLanes {
  // each lane's post-kinematic state and frame for the handlers, rewritten
  // every substep: p.xyz v.x | v.yz w.xy | w.z R0-2 | R3-6 | R7-8 Iwinv.xx yy |
  // Iwinv.zz xy xz yz (rows of 28 floats: 16-byte reads of eight consecutive
  // lanes fall on distinct banks)
  float4 side[64][7];
  PairT pair[MAXP];
  int32_t nh[MAXB];
  int32_t hp[MAXB][MAXH];
  int32_t nra[MAXB][MAXH];
  uint32_t recva[MAXB][MAXH];
  int32_t nrb[MAXB][MAXH];
  uint32_t recvb[MAXB][MAXH];
};

// All lanes of the wavefront copy type t's tables into L; the wavefront's
// own later LDS reads see the writes (LDS operations of a wavefront are
// performed in order).
// nl: lanes per environment (bodies, then contact lanes).
__device__ __forceinline__ void pair_lanes_load(const Tables* __restrict__ tab, int t, PairLanes* L, int lane,
                                                int nl) {
  const TypeT& ty = tab->type[t];
  const int n_words = ty.np * (int)(sizeof(PairT) / 4);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&tab->pair[t][0]);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&L->pair[0]);
  for (int x = lane; x < n_words; x += 64) dst[x] = src[x];
  for (int x = lane; x < nl * MAXH; x += 64) {
    const int b = x / MAXH, i = x - b * MAXH;
    const BodyT& B = tab->body[t][b];
    if (i == 0) L->nh[b] = B.nh;
    L->hp[b][i] = B.hp[i];
    L->nra[b][i] = B.nra[i];
    L->recva[b][i] = B.recva[i];
    L->nrb[b][i] = B.nrb[i];
    L->recvb[b][i] = B.recvb[i];
  }
  __builtin_amdgcn_wave_barrier();
}

// The state and frame of the body on lane src, whose position p was read already.
__device__ __forceinline__ PairSide shfl_side(const PairSide& s, int src, v3 p) {
  PairSide o;
  o.p = p;
  o.v = shfl_v3(s.v, src);
  o.w = shfl_v3(s.w, src);
#pragma unroll
  for (int k = 0; k < 9; ++k) o.R.m[k] = shfl(s.R.m[k], src);
  o.Iwinv = s3{shfl(s.Iwinv.xx, src), shfl(s.Iwinv.yy, src), shfl(s.Iwinv.zz, src),
               shfl(s.Iwinv.xy, src), shfl(s.Iwinv.xz, src), shfl(s.Iwinv.yz, src)};
  return o;
}

__device__ __forceinline__ void side_put(PairLanes& L, int lane, const Body& s, const Frame& f) {
  float4* r = L.side[lane];
  const m3& R = f.R;
  const s3& I = f.Iwinv;
  r[0] = make_float4(s.p.x, s.p.y, s.p.z, s.v.x);
  r[1] = make_float4(s.v.y, s.v.z, s.w.x, s.w.y);
  r[2] = make_float4(s.w.z, R.m[0], R.m[1], R.m[2]);
  r[3] = make_float4(R.m[3], R.m[4], R.m[5], R.m[6]);
  r[4] = make_float4(R.m[7], R.m[8], I.xx, I.yy);
  r[5] = make_float4(I.zz, I.xy, I.xz, I.yz);
}

// The side of the body on lane src, whose first row r0 was read already.
__device__ __forceinline__ PairSide side_get(const PairLanes& L, int src, float4 r0) {
  const float4* r = L.side[src];
  const float4 r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4], r5 = r[5];
  PairSide o;
  o.p = V(r0.x, r0.y, r0.z);
  o.v = V(r0.w, r1.x, r1.y);
  o.w = V(r1.z, r1.w, r2.x);
  o.R.m[0] = r2.y; o.R.m[1] = r2.z; o.R.m[2] = r2.w;
  o.R.m[3] = r3.x; o.R.m[4] = r3.y; o.R.m[5] = r3.z; o.R.m[6] = r3.w;
  o.R.m[7] = r4.x; o.R.m[8] = r4.y;
  o.Iwinv = s3{r4.z, r4.w, r5.x, r5.y, r5.z, r5.w};
  return o;
}

// The bound test of candidate P (see PairT::lo): the line feature of the
// body at pL, RL against the ball around the feature of the body at pK, RK.
__device__ __forceinline__ bool pair_bound(const PairT& P, v3 pL, const m3& RL, v3 pK, const m3& RK) {
  const float4 lo = *reinterpret_cast<const float4*>(P.lo);
  const float4 ld = *reinterpret_cast<const float4*>(P.ld);
  const float4 kc = *reinterpret_cast<const float4*>(P.kc);
  const v3 a = pL + mul(RL, V(lo.x, lo.y, lo.z));
  const v3 d = mul(RL, V(ld.x, ld.y, ld.z));
  const v3 r = (pK + mul(RK, V(kc.x, kc.y, kc.z))) - a;
  const float dd = dot(d, d);
  const float u = dd > 0.f ? clampf(dot(r, d) / dd, 0.f, 1.f) : 0.f;
  const v3 q = r - u * d;
  return dot(q, q) <= lo.w;
}
// The line body's and the other body's lanes of candidate P.
__device__ __forceinline__ int pair_line_lane(const PairT& P, int base) { return base + (P.kc[3] != 0.f ? P.b : P.a); }
__device__ __forceinline__ int pair_ball_lane(const PairT& P, int base) { return base + (P.kc[3] != 0.f ? P.a : P.b); }

// Position and rotation of the body on lane src from the exchange rows
// (while they hold every lane's post-kinematic state and rotation).
__device__ __forceinline__ void xch_get_pR(const XchRows* X, int src, v3& p, m3& R) {
  const float4 a0 = X->r[src][0], r0 = X->r[src][2], r1 = X->r[src][3];
  const float2 a2 = *reinterpret_cast<const float2*>(&X->r[src][4]);
  p = V(a0.x, a0.y, a0.z);
  R.m[0] = r0.x; R.m[1] = r0.y; R.m[2] = r0.z; R.m[3] = r0.w;
  R.m[4] = r1.x; R.m[5] = r1.y; R.m[6] = r1.z; R.m[7] = r1.w;
  R.m[8] = a2.y;
}
// The same from the side rows.
__device__ __forceinline__ void side_get_pR(const PairLanes& L, int src, v3& p, m3& R) {
  const float4 r0 = L.side[src][0], r2 = L.side[src][2], r3 = L.side[src][3], r4 = L.side[src][4];
  p = V(r0.x, r0.y, r0.z);
  R.m[0] = r2.y; R.m[1] = r2.z; R.m[2] = r2.w;
  R.m[3] = r3.x; R.m[4] = r3.y; R.m[5] = r3.z; R.m[6] = r3.w;
  R.m[7] = r4.x; R.m[8] = r4.y;
}

// Slot 0 of a lane's candidates, read once per launch: its index (-1
// without one) and the lanes of its line and ball bodies, for the early
// bound test on the exchange rows.
struct PairSlot0 {
  int pi, sl, sk;
};
__device__ __forceinline__ PairSlot0 pair_slot0(const PairLanes& L, int b, int base) {
  PairSlot0 q{-1, base + b, base + b};
  if (L.nh[b] > 0) {
    const int pi = L.hp[b][0];
    q = PairSlot0{pi, pair_line_lane(L.pair[pi], base), pair_ball_lane(L.pair[pi], base)};
  }
  return q;
}
// The early bound test of slot 0 (1 passed, 0 not), while every lane's
// exchange row holds its post-kinematic position and its rotation.
__device__ __forceinline__ int pair_near0(const XchRows* X, const PairLanes& L, const PairSlot0& q) {
  v3 pL, pK;
  m3 RL, RK;
  xch_get_pR(X, q.sl, pL, RL);
  xch_get_pR(X, q.sk, pK, RK);
  const bool near = pair_bound(L.pair[q.pi < 0 ? 0 : q.pi], pL, RL, pK, RK);
  return (q.pi >= 0 && near) ? 1 : 0;
}

// The adjoint's test: whether the candidate's body origins are within its
// reach (no contact beyond it; looser than the bound test).
__device__ __forceinline__ bool pair_near(const PairT& P, bool mine, v3 pA, v3 pB) {
  const v3 d = pA - pB;
  return mine && dot(d, d) <= P.reach * P.reach;
}

// Forward: adds this body's body-body velocity changes to dv, dw and the
// applied candidates to cnt (post-kinematic state s, frame f). The shares
// travel through the wavefront's exchange rows X, free at this point of the
// substep: dvA on | dwA on | dvB on | dwB on. near0: slot 0's early reach
// test (pair_near0), or -1 to test it here; the side rows are written only
// once some slot is to be evaluated or tested from them.
__device__ __forceinline__ void pair_phase(const Tables* __restrict__ tab, int t, PairLanes& L, XchRows* X, int lane,
                                           int b, int base, const Body& s, const Frame& f, v3& dv, v3& dw, int& cnt,
                                           int near0 = -1) {
  const TypeT& ty = tab->type[t];
  const int nh = L.nh[b];
  bool sides = false;  // wave-uniform
  for (int i = 0; i < ty.max_handled; ++i) {
    const bool mine = i < nh;
    const PairT& P = L.pair[L.hp[b][i]];  // hp = 0 past nh: a valid candidate, unused
    const int sa = base + (mine ? P.a : b), sb = base + (mine ? P.b : b);
    bool near;
    if (i == 0 && near0 >= 0) {
      near = near0 != 0;
    } else {
      if (!sides) side_put(L, lane, s, f);
      sides = true;
      v3 pL, pK;
      m3 RL, RK;
      side_get_pR(L, mine ? pair_line_lane(P, base) : base + b, pL, RL);
      side_get_pR(L, mine ? pair_ball_lane(P, base) : base + b, pK, RK);
      near = mine && pair_bound(P, pL, RL, pK, RK);
    }
    if (__ballot(near) == 0ull) continue;  // wave-uniform
    if (!sides) side_put(L, lane, s, f);
    sides = true;
    const PairSide A = side_get(L, sa, L.side[sa][0]), B = side_get(L, sb, L.side[sb][0]);
    v3 dvA = V(0.f, 0.f, 0.f), dwA = dvA, dvB = dvA, dwB = dvA;
    float on = 0.f;
    if (near && pair_eval(P, ty, A, B, dvA, dwA, dvB, dwB)) on = 1.f;
    X->r[lane][0] = make_float4(dvA.x, dvA.y, dvA.z, on);
    X->r[lane][1] = make_float4(dwA.x, dwA.y, dwA.z, on);
    X->r[lane][2] = make_float4(dvB.x, dvB.y, dvB.z, on);
    X->r[lane][3] = make_float4(dwB.x, dwB.y, dwB.z, on);
    // collect: first-body shares, then second-body shares
    for (int side = 0; side < 2; ++side) {
      const int nr = side == 0 ? L.nra[b][i] : L.nrb[b][i];
      const uint32_t rv = side == 0 ? L.recva[b][i] : L.recvb[b][i];
      const int kmax = side == 0 ? ty.recv_na[i] : ty.recv_nb[i];
      // four rows read together, then added in order (at most MAXR = 8 shares)
      for (int k0 = 0; k0 < kmax; k0 += 4) {
        float4 a[4], w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = k0 + j;
          const int hsrc = base + (k < nr ? (int)((rv >> (4 * (k & 7))) & 15u) : b);
          a[j] = X->r[hsrc][2 * side];
          w[j] = X->r[hsrc][2 * side + 1];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (k0 + j < nr && a[j].w != 0.f) {
            dv += V(a[j].x, a[j].y, a[j].z);
            dw += V(w[j].x, w[j].y, w[j].z);
            ++cnt;
          }
        }
      }
    }
  }
}

// Adjoint: given this body's cotangents of its velocity-change sums (dvb,
// dwb), adds the cotangents of its post-kinematic state to tot, of its frame
// to fr, of its inverse mass to invm_bar (unless it has none here) and of the
// friction coefficient (on handler lanes) to mu_bar.
__device__ __forceinline__ void pair_phase_adj(const Tables* __restrict__ tab, int t, const PairLanes& L, int b,
                                               int base, const Body& post, const Frame& f, v3 dvb, v3 dwb, Bar& tot,
                                               FrameBar& fr, float& invm_bar, float& mu_bar) {
  const TypeT& ty = tab->type[t];
  const int nh = L.nh[b];
  const PairSide me{post.p, post.v, post.w, f.R, f.Iwinv};
  for (int i = 0; i < ty.max_handled; ++i) {
    const bool mine = i < nh;
    const PairT& P = L.pair[L.hp[b][i]];
    const int sa = base + (mine ? P.a : b), sb = base + (mine ? P.b : b);
    const v3 pA = shfl_v3(post.p, sa), pB = shfl_v3(post.p, sb);
    const bool near = pair_near(P, mine, pA, pB);
    if (__ballot(near) == 0ull) continue;  // wave-uniform
    const PairSide A = shfl_side(me, sa, pA), B = shfl_side(me, sb, pB);
    const v3 dvbA = shfl_v3(dvb, sa), dwbA = shfl_v3(dwb, sa), dvbB = shfl_v3(dvb, sb), dwbB = shfl_v3(dwb, sb);
    PairSideBar Ab = pairbar_zero(), Bb = pairbar_zero();
    if (near && pair_adj(P, ty, A, B, dvbA, dwbA, dvbB, dwbB, Ab, Bb, mu_bar)) {
      // a body without inverse mass here (all translations frozen) has no mass cotangent from it
      if (P.im_a == 0.f) Ab.im = 0.f;
      if (P.im_b == 0.f) Bb.im = 0.f;
    }
    for (int side = 0; side < 2; ++side) {
      const int nr = side == 0 ? L.nra[b][i] : L.nrb[b][i];
      const uint32_t rv = side == 0 ? L.recva[b][i] : L.recvb[b][i];
      const int kmax = side == 0 ? ty.recv_na[i] : ty.recv_nb[i];
      const PairSideBar ob = sel(side == 0, Ab, Bb);
      for (int k = 0; k < kmax; ++k) {
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
        if (k < nr) {
          tot.p += x.p;
          tot.v += x.v;
          tot.w += x.w;
#pragma unroll
          for (int q = 0; q < 9; ++q) fr.Rb.m[q] += x.R.m[q];
          fr.Iwinvb.xx += x.Iwinv.xx;
          fr.Iwinvb.yy += x.Iwinv.yy;
          fr.Iwinvb.zz += x.Iwinv.zz;
          fr.Iwinvb.xy += x.Iwinv.xy;
          fr.Iwinvb.xz += x.Iwinv.xz;
          fr.Iwinvb.yz += x.Iwinv.yz;
          invm_bar += x.im;
        }
      }
    }
  }
}

}  // namespace bx
