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

__device__ __forceinline__ float act_of(const float* act, int a, int e, int E) {
  return a >= 0 ? clampf(act[(size_t)a * E + e], -1.f, 1.f) : 0.f;
}

// Forward tape of one substep, [TAPE_N][Bmax][E]: the body's state before the
// kinematic update (13), the total torque it received (3), its count of
// applied contacts (1).
__device__ __forceinline__ void tape_state(float* tp, const Body& s, int b, int e, int Bm, int E) {
  const float v[13] = {s.p.x, s.p.y, s.p.z, s.q.w, s.q.x, s.q.y, s.q.z, s.v.x, s.v.y, s.v.z, s.w.x, s.w.y, s.w.z};
  for (int c = 0; c < 13; ++c) tp[((size_t)c * Bm + b) * E + e] = v[c];
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
  float v[13];
  for (int c = 0; c < 13; ++c) v[c] = tp[((size_t)c * Bm + b) * E + e];
  Body s;
  s.p = V(v[0], v[1], v[2]);
  s.q = q4{v[3], v[4], v[5], v[6]};
  s.v = V(v[7], v[8], v[9]);
  s.w = V(v[10], v[11], v[12]);
  return s;
}
__device__ __forceinline__ v3 tape_load_torque(const float* tp, int b, int e, int Bm, int E) {
  return V(tp[((size_t)13 * Bm + b) * E + e], tp[((size_t)14 * Bm + b) * E + e], tp[((size_t)15 * Bm + b) * E + e]);
}
__device__ __forceinline__ int tape_load_count(const float* tp, int b, int e, int Bm, int E) {
  return (int)tp[((size_t)16 * Bm + b) * E + e];
}

}  // namespace bx
