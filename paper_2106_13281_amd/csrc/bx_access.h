// Device-side state access shared by the forward and adjoint kernels.
//
// State layout: structure of arrays, environment index fastest,
//   field[(c * Bmax + b) * E + e]   (pos/vel/ang c < 3, rot c < 4).
#pragma once
#include <hip/hip_runtime.h>

#include "bx_internal.h"
#include "bx_phys.h"

namespace bx {

__device__ __forceinline__ Body load_body(const Fields& f, int b, int e, int Bm, int E) {
  Body s;
  s.p = V(f.pos[(0 * Bm + b) * E + e], f.pos[(1 * Bm + b) * E + e], f.pos[(2 * Bm + b) * E + e]);
  s.q = q4{f.rot[(0 * Bm + b) * E + e], f.rot[(1 * Bm + b) * E + e], f.rot[(2 * Bm + b) * E + e],
           f.rot[(3 * Bm + b) * E + e]};
  s.v = V(f.vel[(0 * Bm + b) * E + e], f.vel[(1 * Bm + b) * E + e], f.vel[(2 * Bm + b) * E + e]);
  s.w = V(f.ang[(0 * Bm + b) * E + e], f.ang[(1 * Bm + b) * E + e], f.ang[(2 * Bm + b) * E + e]);
  return s;
}

__device__ __forceinline__ void store_body(const Fields& f, size_t base, const Body& s, int b, int e, int Bm,
                                           int E) {
  f.pos[base + (0 * Bm + b) * E + e] = s.p.x;
  f.pos[base + (1 * Bm + b) * E + e] = s.p.y;
  f.pos[base + (2 * Bm + b) * E + e] = s.p.z;
  f.rot[base + (0 * Bm + b) * E + e] = s.q.w;
  f.rot[base + (1 * Bm + b) * E + e] = s.q.x;
  f.rot[base + (2 * Bm + b) * E + e] = s.q.y;
  f.rot[base + (3 * Bm + b) * E + e] = s.q.z;
  f.vel[base + (0 * Bm + b) * E + e] = s.v.x;
  f.vel[base + (1 * Bm + b) * E + e] = s.v.y;
  f.vel[base + (2 * Bm + b) * E + e] = s.v.z;
  f.ang[base + (0 * Bm + b) * E + e] = s.w.x;
  f.ang[base + (1 * Bm + b) * E + e] = s.w.y;
  f.ang[base + (2 * Bm + b) * E + e] = s.w.z;
}

// Trajectory snapshots are laid out like the state with a leading save index;
// `base` is the element offset of snapshot k of a 3-component field, scaled
// per field by the component count.
__device__ __forceinline__ void store_snapshot(const Fields& f, size_t k, const Body& s, int b, int e, int Bm,
                                               int E) {
  size_t n3 = (size_t)3 * Bm * E, n4 = (size_t)4 * Bm * E;
  Fields g{f.pos + k * n3, f.rot + k * n4, f.vel + k * n3, f.ang + k * n3};
  store_body(g, 0, s, b, e, Bm, E);
}

__device__ __forceinline__ void zero_body(const Fields& f, int b, int e, int Bm, int E) {
  Body z;
  z.p = z.v = z.w = V(0.f, 0.f, 0.f);
  z.q = q4{0.f, 0.f, 0.f, 0.f};
  store_body(f, 0, z, b, e, Bm, E);
}

// Tape of the fused path, wavefront-major: per substep and work item, TAPE_N
// rows of 64 floats (one per lane; rows 0-12 the state before the kinematic
// update, 13-15 the total torque, 16 the applied-contact count), so that
// every store and load of a row is 256 contiguous bytes.
__device__ __forceinline__ void wtape_state(float* tp, const Body& s, int lane) {
  const float v[13] = {s.p.x, s.p.y, s.p.z, s.q.w, s.q.x, s.q.y, s.q.z, s.v.x, s.v.y, s.v.z, s.w.x, s.w.y, s.w.z};
#pragma unroll
  for (int k = 0; k < 13; ++k) tp[k * 64 + lane] = v[k];
}
__device__ __forceinline__ void wtape_rest(float* tp, v3 torque, int cnt, int lane) {
  tp[13 * 64 + lane] = torque.x;
  tp[14 * 64 + lane] = torque.y;
  tp[15 * 64 + lane] = torque.z;
  tp[16 * 64 + lane] = (float)cnt;
}
// one record's rows into registers (issued ahead of use by the adjoint, so
// that the load's latency overlaps the substep before it)
__device__ __forceinline__ void wtape_fetch(const float* tp, int lane, float (&v)[17]) {
#pragma unroll
  for (int k = 0; k < 17; ++k) v[k] = tp[k * 64 + lane];
}
__device__ __forceinline__ void wtape_unpack(const float (&v)[17], Body& s, v3& torque, int& cnt) {
  s.p = V(v[0], v[1], v[2]);
  s.q = q4{v[3], v[4], v[5], v[6]};
  s.v = V(v[7], v[8], v[9]);
  s.w = V(v[10], v[11], v[12]);
  torque = V(v[13], v[14], v[15]);
  cnt = (int)v[16];
}

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2):
// block b runs on XCD b % 8. Neighbouring work items (environments) share the
// 128-byte lines of the environment-fastest arrays (actions, state), so the
// block index is permuted in groups of 64 blocks: within a group, XCD x takes
// the 8 consecutive items 8x..8x+7. Dispatch order (heaviest work first in a
// mixed batch) is kept at the granularity of a group; a last partial group
// gives each XCD one contiguous range. A bijection on [0, n) whatever the
// dispatch order is.
__device__ __forceinline__ int xcd_block(int b, int n) {
  constexpr int NXCD = 8, RUN = 8, G = NXCD * RUN;
  const int g0 = (b / G) * G, i = b - g0, m = n - g0 < G ? n - g0 : G;
  if (m == G) return g0 + (i % NXCD) * RUN + i / NXCD;
  const int q = m / NXCD, r = m % NXCD, x = i % NXCD;
  return g0 + x * q + (x < r ? x : r) + i / NXCD;
}

// Index of this wavefront's work item in a launch of blocks of whole
// wavefronts. It is the same on every lane of the wavefront; readfirstlane
// makes that visible to the compiler, so the work item, its system type and
// the type's constants are held in scalar registers and tests on them are
// scalar branches rather than per-lane masks.
__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// Action of joint axis x, clipped to its range ([-1, 1] for a torque,
// the joint's range for a target angle); 0 for an axis without actuator.
__device__ __forceinline__ float act_of(const float* act, const JointT& J, int x, int e, int E) {
  return J.act[x] >= 0 ? clampf(act[(size_t)J.act[x] * E + e], J.act_lo[x], J.act_hi[x]) : 0.f;
}
// The same action unclipped (0 for an axis without actuator), for loads
// issued ahead of their use.
__device__ __forceinline__ float act_raw(const float* act, const JointT& J, int x, int e, int E) {
  return J.act[x] >= 0 ? act[(size_t)J.act[x] * E + e] : 0.f;
}

// Forward tape of one substep, [TAPE_N][Bmax][E]: the body's state before the
// kinematic update (13), the total torque it received (3), its count of
// applied contacts (1).
__device__ __forceinline__ void tape_state(float* tp, const Body& s, int b, int e, int Bm, int E) {
  const size_t st = (size_t)Bm * E;
  float* q = tp + (size_t)b * E + e;
  q[0] = s.p.x;
  q[st] = s.p.y;
  q[2 * st] = s.p.z;
  q[3 * st] = s.q.w;
  q[4 * st] = s.q.x;
  q[5 * st] = s.q.y;
  q[6 * st] = s.q.z;
  q[7 * st] = s.v.x;
  q[8 * st] = s.v.y;
  q[9 * st] = s.v.z;
  q[10 * st] = s.w.x;
  q[11 * st] = s.w.y;
  q[12 * st] = s.w.z;
}
__device__ __forceinline__ void tape_torque(float* tp, v3 t, int b, int e, int Bm, int E) {
  tp[((size_t)13 * Bm + b) * E + e] = t.x;
  tp[((size_t)14 * Bm + b) * E + e] = t.y;
  tp[((size_t)15 * Bm + b) * E + e] = t.z;
}
__device__ __forceinline__ void tape_count(float* tp, int n, int b, int e, int Bm, int E) {
  tp[((size_t)16 * Bm + b) * E + e] = (float)n;
}
__device__ __forceinline__ Body tape_load_state(const float* tp, int b, int e, int Bm, int E) {
  const size_t st = (size_t)Bm * E;
  const float* q = tp + (size_t)b * E + e;
  Body s;
  s.p = V(q[0], q[st], q[2 * st]);
  s.q = q4{q[3 * st], q[4 * st], q[5 * st], q[6 * st]};
  s.v = V(q[7 * st], q[8 * st], q[9 * st]);
  s.w = V(q[10 * st], q[11 * st], q[12 * st]);
  return s;
}
__device__ __forceinline__ v3 tape_load_torque(const float* tp, int b, int e, int Bm, int E) {
  return V(tp[((size_t)13 * Bm + b) * E + e], tp[((size_t)14 * Bm + b) * E + e], tp[((size_t)15 * Bm + b) * E + e]);
}
__device__ __forceinline__ int tape_load_count(const float* tp, int b, int e, int Bm, int E) {
  return (int)tp[((size_t)16 * Bm + b) * E + e];
}

// Cross-lane read within the wavefront (ds_bpermute).
__device__ __forceinline__ float shfl(float v, int src) { return __shfl(v, src, 64); }

// Keeps a value in a VGPR: the empty asm makes it opaque, so the compiler
// cannot re-load it from the constant tables inside the hot loop.
__device__ __forceinline__ void pin(float& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(int& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin3(float* x) {
  pin(x[0]);
  pin(x[1]);
  pin(x[2]);
}

// Per-lane constants copied once into registers.
template <int MAXDOF>
__device__ __forceinline__ void pin_consts(BodyT& B, JointT& J, bool has_joint, ContactT* C, int nc) {
  pin(B.inv_m);
  pin3(B.I);
  pin3(B.Iinv);
  pin3(B.free_p);
  pin3(B.free_r);
  if (has_joint) {
    pin3(J.ap);
    pin3(J.ac);
    for (int k = 0; k < 9; ++k) {
      pin(J.FP[k]);
      pin(J.FC[k]);
    }
    pin(J.k_lin);
    pin(J.c_lin);
    pin(J.k_ang);
    pin(J.c_ang);
    pin(J.k_lim);
    for (int k = 0; k < MAXDOF; ++k) {
      pin(J.lo[k]);
      pin(J.hi[k]);
      pin(J.gear[k]);
    }
  }
  for (int c = 0; c < nc; ++c) {
    pin3(C[c].l);
    pin(C[c].rho);
  }
}

// A wavefront's exchange rows in LDS, one per lane, through which lanes read
// one another's values (a parent's state and rotation, a child's reaction or
// cotangent) in a few 16-byte accesses, where cross-lane permutes take one
// instruction per value. A wavefront's LDS operations complete in program
// order: a read that follows a write sees it, and a write that follows a
// read leaves that read intact, so a row is rewritten as soon as its last
// reader has been issued and no barrier is needed. Rows of 20 floats keep
// the 16-byte accesses of eight consecutive lanes on distinct banks.
struct XchRows {
  float4 r[64][5];
};

// Position and velocities (columns 0-7), then the rotation matrix (8-15)
// with the last angular velocity component beside its last entry (16, 17):
// written in two parts so that the first is on its way while R is formed.
__device__ __forceinline__ void xch_put_pvw(XchRows* X, int lane, const Body& s) {
  X->r[lane][0] = make_float4(s.p.x, s.p.y, s.p.z, s.v.x);
  X->r[lane][1] = make_float4(s.v.y, s.v.z, s.w.x, s.w.y);
}
__device__ __forceinline__ void xch_put_rot(XchRows* X, int lane, float wz, const m3& R) {
  X->r[lane][2] = make_float4(R.m[0], R.m[1], R.m[2], R.m[3]);
  X->r[lane][3] = make_float4(R.m[4], R.m[5], R.m[6], R.m[7]);
  *reinterpret_cast<float2*>(&X->r[lane][4]) = make_float2(wz, R.m[8]);
}
// Position, velocities and rotation of the body on lane src (P.q is not set).
__device__ __forceinline__ void xch_get_pvw_rot(const XchRows* X, int src, Body& P, m3& RP) {
  const float4 a0 = X->r[src][0], a1 = X->r[src][1], r0 = X->r[src][2], r1 = X->r[src][3];
  const float2 a2 = *reinterpret_cast<const float2*>(&X->r[src][4]);
  P.p = V(a0.x, a0.y, a0.z);
  P.v = V(a0.w, a1.x, a1.y);
  P.w = V(a1.z, a1.w, a2.x);
  RP.m[0] = r0.x; RP.m[1] = r0.y; RP.m[2] = r0.z; RP.m[3] = r0.w;
  RP.m[4] = r1.x; RP.m[5] = r1.y; RP.m[6] = r1.z; RP.m[7] = r1.w;
  RP.m[8] = a2.y;
}
// Two 3-vectors (columns 0-5).
__device__ __forceinline__ void xch_put2(XchRows* X, int lane, v3 a, v3 b) {
  X->r[lane][0] = make_float4(a.x, a.y, a.z, b.x);
  *reinterpret_cast<float2*>(&X->r[lane][1]) = make_float2(b.y, b.z);
}
__device__ __forceinline__ void xch_get2(const XchRows* X, int src, v3& a, v3& b) {
  const float4 x0 = X->r[src][0];
  const float2 x1 = *reinterpret_cast<const float2*>(&X->r[src][1]);
  a = V(x0.x, x0.y, x0.z);
  b = V(x0.w, x1.x, x1.y);
}
// A full body state or its cotangent (p, q, v, w: columns 0-12).
template <class S>
__device__ __forceinline__ void xch_put_body(XchRows* X, int lane, const S& s) {
  X->r[lane][0] = make_float4(s.p.x, s.p.y, s.p.z, s.q.w);
  X->r[lane][1] = make_float4(s.q.x, s.q.y, s.q.z, s.v.x);
  X->r[lane][2] = make_float4(s.v.y, s.v.z, s.w.x, s.w.y);
  X->r[lane][3].x = s.w.z;
}
template <class S>
__device__ __forceinline__ S xch_get_body(const XchRows* X, int src) {
  const float4 a0 = X->r[src][0], a1 = X->r[src][1], a2 = X->r[src][2];
  const float a3 = X->r[src][3].x;
  S s;
  s.p = V(a0.x, a0.y, a0.z);
  s.q = q4{a0.w, a1.x, a1.y, a1.z};
  s.v = V(a1.w, a2.x, a2.y);
  s.w = V(a2.z, a2.w, a3);
  return s;
}

// Contact candidates of a body kept in registers (more are read from the table).
constexpr int REG_CONTACTS = 2;
// Children whose reactions are gathered with all cross-lane reads in flight at once.
constexpr int GATHER = 4;

}  // namespace bx
