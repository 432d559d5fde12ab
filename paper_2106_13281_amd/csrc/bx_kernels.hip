// HIP kernels for gfx950: reset pose, plain per-phase step, fused persistent
// step/rollout.
//
// State layout: structure of arrays, environment index fastest,
//   field[(c * Bmax + b) * E + e]   (pos/vel/ang c < 3, rot c < 4).
// Environments of a batch are grouped by system type through `env_list`
// (the global environment ids of type t are env_list[off_t .. off_t + n_t)).
#include <hip/hip_runtime.h>

#include "bx_access.h"
#include "bx_internal.h"
#include "bx_pair_lanes.h"
#include "bx_phys.h"

namespace bx {

// ------------------------------------------------------------------ reset pose
// One thread per environment. Forward kinematics down each tree (parent
// before child): R_C = R_P J_P Rx Ry Rz(theta) J_C^T, child anchor on the
// parent anchor; roots without a given position lifted to the clearance;
// optional offset of the first body's tree.
__device__ m3 euler_xyz(float a, float b, float c) {
  float ca = cosf(a), sa = sinf(a), cb = cosf(b), sb = sinf(b), cc = cosf(c), sc = sinf(c);
  // Rx(a) Ry(b) Rz(c)
  m3 M;
  M.m[0] = cb * cc;                  M.m[1] = -cb * sc;                 M.m[2] = sb;
  M.m[3] = sa * sb * cc + ca * sc;   M.m[4] = -sa * sb * sc + ca * cc;  M.m[5] = -sa * cb;
  M.m[6] = -ca * sb * cc + sa * sc;  M.m[7] = ca * sb * sc + sa * cc;   M.m[8] = ca * cb;
  return M;
}

__device__ m3 mm(const m3& A, const m3& B) {
  m3 C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C.m[3 * i + j] = A.m[3 * i] * B.m[j] + A.m[3 * i + 1] * B.m[3 + j] + A.m[3 * i + 2] * B.m[6 + j];
  return C;
}
__device__ m3 mmT(const m3& A, const float* B) {  // A * B^T
  m3 C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C.m[3 * i + j] = A.m[3 * i] * B[3 * j] + A.m[3 * i + 1] * B[3 * j + 1] + A.m[3 * i + 2] * B[3 * j + 2];
  return C;
}

// Unit quaternion (w >= 0) of a rotation matrix, largest-pivot method.
__device__ q4 mat_to_quat(const m3& R) {
  float tr = R.m[0] + R.m[4] + R.m[8];
  q4 q;
  if (tr >= R.m[0] && tr >= R.m[4] && tr >= R.m[8]) {
    float w = 0.5f * sqrtf(1.f + tr);
    float k = 0.25f / w;
    q = q4{w, (R.m[7] - R.m[5]) * k, (R.m[2] - R.m[6]) * k, (R.m[3] - R.m[1]) * k};
  } else if (R.m[0] >= R.m[4] && R.m[0] >= R.m[8]) {
    float x = 0.5f * sqrtf(1.f + R.m[0] - R.m[4] - R.m[8]);
    float k = 0.25f / x;
    q = q4{(R.m[7] - R.m[5]) * k, x, (R.m[1] + R.m[3]) * k, (R.m[2] + R.m[6]) * k};
  } else if (R.m[4] >= R.m[8]) {
    float y = 0.5f * sqrtf(1.f - R.m[0] + R.m[4] - R.m[8]);
    float k = 0.25f / y;
    q = q4{(R.m[2] - R.m[6]) * k, (R.m[1] + R.m[3]) * k, y, (R.m[5] + R.m[7]) * k};
  } else {
    float z = 0.5f * sqrtf(1.f - R.m[0] - R.m[4] + R.m[8]);
    float k = 0.25f / z;
    q = q4{(R.m[3] - R.m[1]) * k, (R.m[2] + R.m[6]) * k, (R.m[5] + R.m[7]) * k, z};
  }
  float n = 1.f / sqrtf(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
  if (q.w < 0.f) n = -n;
  return q4{q.w * n, q.x * n, q.y * n, q.z * n};
}

__global__ void k_default_qp(const Tables* __restrict__ tab, const int32_t* __restrict__ env_type, int E, int Bm,
                             const float* __restrict__ angles, const float* __restrict__ root_off, Fields out) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int t = env_type[e];
  const TypeT& ty = tab->type[t];
  m3 R[MAXB];
  v3 p[MAXB];
  for (int i = 0; i < ty.nb; ++i) {
    const int b = tab->topo[t][i];
    const BodyT& B = tab->body[t][b];
    if (B.joint < 0) {
      R[b] = m3{{1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}};
      p[b] = B.has_pos ? ld3(B.pos0) : V(0.f, 0.f, 0.f);
    } else {
      const JointT& J = tab->joint[t][B.joint];
      float th[3] = {0.f, 0.f, 0.f};
      for (int k = 0; k < J.dof; ++k) th[k] = angles ? angles[(size_t)(J.dof0 + k) * E + e] : J.def_angle[k];
      m3 RPJ = mul(R[J.parent], J.FP);
      R[b] = mmT(mm(RPJ, euler_xyz(th[0], th[1], th[2])), J.FC);
      p[b] = p[J.parent] + mul(R[J.parent], ld3(J.ap)) - mul(R[b], ld3(J.ac));
    }
  }
  // lift every root tree without a given position to the clearance height
  for (int r = 0; r < ty.nb; ++r) {
    const BodyT& Br = tab->body[t][r];
    if (Br.joint >= 0 || Br.has_pos) continue;
    float low = INFINITY;
    for (int c = 0; c < ty.nc; ++c) {
      const ContactT& C = tab->contact[t][c];
      if (tab->body[t][C.body].root != r) continue;
      low = fminf(low, (p[C.body] + mul(R[C.body], ld3(C.l))).z - C.rho);
    }
    if (low < INFINITY) {
      for (int b = 0; b < ty.nb; ++b)
        if (tab->body[t][b].root == r) p[b].z += ty.clearance - low;
    }
  }
  if (root_off) {
    const BodyT& B0 = tab->body[t][0];
    if (B0.joint < 0 && (B0.free_p[0] != 0.f || B0.free_p[1] != 0.f || B0.free_p[2] != 0.f)) {
      v3 off = V(root_off[e], root_off[(size_t)E + e], root_off[(size_t)2 * E + e]);
      for (int b = 0; b < ty.nb; ++b)
        if (tab->body[t][b].root == 0) p[b] = p[b] + off;
    }
  }
  for (int b = 0; b < Bm; ++b) {
    if (b < ty.nb) {
      Body s;
      s.p = p[b];
      s.q = mat_to_quat(R[b]);
      s.v = s.w = V(0.f, 0.f, 0.f);
      store_body(out, 0, s, b, e, Bm, E);
    } else {
      zero_body(out, b, e, Bm, E);
    }
  }
}

// ------------------------------------------------------------------ plain path
// One launch per phase per substep, one thread per (item, environment of
// the type); environment index fastest. Per-joint and per-contact results
// go to fixed slots and are gathered by the integrators in a fixed order.

// Kinematic phase; on the first substep it reads `in` (and zeroes the padded
// body slots of `out`), afterwards it updates `out` in place.
__global__ void k_plain_kinematic(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n,
                                  int E, int Bm, Fields in, Fields out, int zero_pad, float* __restrict__ tape) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = idx / n, k = idx - b * n;
  if (b >= Bm) return;
  const int e = envs[k];
  const TypeT& ty = tab->type[t];
  if (b >= ty.nb) {
    if (zero_pad) zero_body(out, b, e, Bm, E);
    return;
  }
  Body s = load_body(in, b, e, Bm, E);
  if (tape) tape_state(tape, s, b, e, Bm, E);
  kinematic(tab->body[t][b], s, ty.h);
  store_body(out, 0, s, b, e, Bm, E);
}

// Joint and actuator phase: slot j holds (fc, tc, fp, tp) = 12 floats.
template <int MAXDOF>
__global__ void k_plain_joint(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n,
                              int E, int Bm, Fields st, const float* __restrict__ act, float* __restrict__ jslot) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = idx / n, k = idx - j * n;
  const TypeT& ty = tab->type[t];
  if (j >= ty.nj) return;
  const int e = envs[k];
  const JointT& J = tab->joint[t][j];
  Body P = load_body(st, J.parent, e, Bm, E);
  Body C = load_body(st, J.child, e, Bm, E);
  m3 RP = quat_to_mat(P.q), RC = quat_to_mat(C.q);
  float a[3];
  for (int x = 0; x < 3; ++x) a[x] = act_of(act, J, x, e, E);
  JointOut o = joint_eval<MAXDOF>(J, P, RP, C, RC, a);
  const int NJ = ty.nj;
  float vals[12] = {o.fc.x, o.fc.y, o.fc.z, o.tc.x, o.tc.y, o.tc.z, o.fp.x, o.fp.y, o.fp.z, o.tp.x, o.tp.y, o.tp.z};
  for (int x = 0; x < 12; ++x) jslot[((size_t)x * NJ + j) * n + k] = vals[x];
}

// Collider phase: slot c holds (dv, dw, applied) = 7 floats.
__global__ void k_plain_contact(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n,
                                int E, int Bm, Fields st, float* __restrict__ cslot) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = idx / n, k = idx - c * n;
  const TypeT& ty = tab->type[t];
  if (c >= ty.nc) return;
  const int e = envs[k];
  const ContactT& C = tab->contact[t][c];
  const BodyT& B = tab->body[t][C.body];
  Body s = load_body(st, C.body, e, Bm, E);
  Frame f = derive(B, s);
  v3 dv = V(0.f, 0.f, 0.f), dw = V(0.f, 0.f, 0.f);
  bool on = contact_eval(C, ty, B, s, f, dv, dw);
  const int NC = ty.nc;
  float vals[7] = {dv.x, dv.y, dv.z, dw.x, dw.y, dw.z, on ? 1.f : 0.f};
  for (int x = 0; x < 7; ++x) cslot[((size_t)x * NC + c) * n + k] = vals[x];
}

// Body-body phase: slot c (after the ground-contact slots) holds (dv, dw)
// of the first body, (dv, dw) of the second and applied = 13 floats.
__global__ void k_plain_pair(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n, int E,
                             int Bm, Fields st, float* __restrict__ cslot) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = idx / n, k = idx - c * n;
  const TypeT& ty = tab->type[t];
  if (c >= ty.np) return;
  const int e = envs[k];
  const PairT& P = tab->pair[t][c];
  PairSide side[2];
  for (int i = 0; i < 2; ++i) {
    const int b = i == 0 ? P.a : P.b;
    const Body s = load_body(st, b, e, Bm, E);
    const Frame f = derive(tab->body[t][b], s);
    side[i] = PairSide{s.p, s.v, s.w, f.R, f.Iwinv};
  }
  v3 dvA = V(0.f, 0.f, 0.f), dwA = dvA, dvB = dvA, dwB = dvA;
  const bool on = pair_eval(P, ty, side[0], side[1], dvA, dwA, dvB, dwB);
  float vals[13] = {dvA.x, dvA.y, dvA.z, dwA.x, dwA.y, dwA.z, dvB.x, dvB.y, dvB.z, dwB.x, dwB.y, dwB.z, on ? 1.f : 0.f};
  float* ps = cslot + (size_t)7 * ty.nc * n;
  for (int x2 = 0; x2 < 13; ++x2) ps[((size_t)x2 * ty.np + c) * n + k] = vals[x2];
}

// Potential integrator: gathers the body's own joint (as child) then its
// children's joints (as parent), in that order.
__global__ void k_plain_potential(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n,
                                  int E, int Bm, Fields st, const float* __restrict__ jslot, float* __restrict__ tape) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = idx / n, k = idx - b * n;
  const TypeT& ty = tab->type[t];
  if (b >= ty.nb) return;
  const int e = envs[k];
  const BodyT& B = tab->body[t][b];
  const int NJ = ty.nj;
  auto slot = [&](int x, int j) { return jslot[((size_t)x * NJ + j) * n + k]; };
  v3 f = V(0.f, 0.f, 0.f), tq = V(0.f, 0.f, 0.f);
  if (B.joint >= 0) {
    f = V(slot(0, B.joint), slot(1, B.joint), slot(2, B.joint));
    tq = V(slot(3, B.joint), slot(4, B.joint), slot(5, B.joint));
  }
  for (int i = 0; i < B.nch; ++i) {
    const int j = tab->body[t][B.ch[i]].joint;
    f += V(slot(6, j), slot(7, j), slot(8, j));
    tq += V(slot(9, j), slot(10, j), slot(11, j));
  }
  Body s = load_body(st, b, e, Bm, E);
  Frame fr = derive(B, s);
  if (tape) tape_torque(tape, tq, b, e, Bm, E);
  potential(B, ty, s, fr, f, tq);
  store_body(st, 0, s, b, e, Bm, E);
}

// Collision integrator: averages the body's applied contact impulses.
__global__ void k_plain_collision(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n,
                                  int E, int Bm, Fields st, const float* __restrict__ cslot, uint8_t* nonfinite,
                                  int last, float* __restrict__ tape) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = idx / n, k = idx - b * n;
  const TypeT& ty = tab->type[t];
  if (b >= ty.nb) return;
  const int e = envs[k];
  const BodyT& B = tab->body[t][b];
  const int NC = ty.nc;
  auto slot = [&](int x, int c) { return cslot[((size_t)x * NC + c) * n + k]; };
  v3 dv = V(0.f, 0.f, 0.f), dw = V(0.f, 0.f, 0.f);
  int cnt = 0;
  for (int c = B.c0; c < B.c1; ++c) {
    if (slot(6, c) != 0.f) {
      dv += V(slot(0, c), slot(1, c), slot(2, c));
      dw += V(slot(3, c), slot(4, c), slot(5, c));
      ++cnt;
    }
  }
  // then the body-body candidates it takes part in, in candidate order
  const float* ps = cslot + (size_t)7 * NC * n;
  const int NP = ty.np;
  for (int i = 0; i < B.npair; ++i) {
    const int c = B.pairs[i];
    auto pv = [&](int x) { return ps[((size_t)x * NP + c) * n + k]; };
    if (pv(12) != 0.f) {
      const int o = tab->pair[t][c].a == b ? 0 : 6;
      dv += V(pv(o), pv(o + 1), pv(o + 2));
      dw += V(pv(o + 3), pv(o + 4), pv(o + 5));
      ++cnt;
    }
  }
  Body s = load_body(st, b, e, Bm, E);
  if (tape) tape_count(tape, cnt, b, e, Bm, E);
  collision(B, s, dv, dw, cnt);
  store_body(st, 0, s, b, e, Bm, E);
  if (last && nonfinite && !finite_body(s)) nonfinite[e] = 1;
}

// ------------------------------------------------------------------ fused path
// One lane per body, floor(64 / nb) environments per wavefront; the lane of
// body b also evaluates the joint whose child is b (with its actuators) and
// b's own contact candidates. Neighbour data moves through the wavefront's
// exchange rows in LDS: the child lane reads its parent's state; the parent
// lane reads each child's reaction (fp, tp) in child order. State stays in
// registers across all substeps and steps; only actions are read per step.

// What the environment epilogue reads and writes (see brax_env_step).
struct EnvArgs {
  const EnvT* env;   // per type
  Fields reset;      // reset state of every environment
  float* obs;        // [Omax][E]
  float* reward;     // [E]
  uint8_t* done;     // [E]
  int Omax;
};

// LDS bytes of one wavefront of the fused kernels: its exchange rows and,
// for batches with body-body candidates, its copy of their tables (placed
// after the exchange rows of all wavefronts of the block).
static inline size_t fused_lds_per_wave(bool pairs) {
  return sizeof(XchRows) + (pairs ? sizeof(PairLanes) : 0);
}

__device__ __forceinline__ XchRows* xch_lanes(float4* lds) {
  return reinterpret_cast<XchRows*>(lds) + (threadIdx.x >> 6);
}
__device__ __forceinline__ PairLanes* pair_lanes(float4* lds) {
  return reinterpret_cast<PairLanes*>(reinterpret_cast<XchRows*>(lds) + (blockDim.x >> 6)) + (threadIdx.x >> 6);
}

// TAPE: also write each substep's tape record (state before the kinematic
// update, total torque, count of applied contacts) to the wavefront-major
// tape[step][sub][work item w of n_work][TAPE_N][64], for the adjoint that
// reads it instead of recomputing the step.
// REGC: contact candidates of a body kept in registers (the rest are read
// from the table inside the loop).
// ENV: after the step(s), the environment layer on the state in registers
// (reward, termination, reset of finished environments, observation of the
// final state), so that an environment step is one launch.
// CL: the batch has contact lanes (see TypeT::nl); kernels for batches
// without keep one lane per body and none of the lane-group code.
template <int MAXDOF, bool TAPE, bool PAIRS, int REGC = REG_CONTACTS, bool ENV = false, bool CL = false>
__device__ __forceinline__ void fused_run(const Tables* __restrict__ tab, const WaveWork& wk,
                                          const int32_t* __restrict__ env_list, const int32_t* __restrict__ type_off,
                                          int E, int Bm, const Fields& in, const Fields& out,
                                          const float* __restrict__ acts, int Am, int T, int save_every,
                                          const Fields& traj, uint8_t* nonfinite, float* __restrict__ tape,
                                          int smax, int w, int n_work, XchRows* X, PairLanes* pl = nullptr,
                                          const EnvArgs* ea = nullptr) {
  const int t = wk.type;
  const TypeT ty = tab->type[t];
  const int nb = ty.nb;
  // without a tape, a body with many contact candidates has contact lanes
  // (lanes nb .. nl-1 of the environment) that hold copies of its state;
  // the tape kernels keep one lane per body (their tape is read lane by lane)
  constexpr bool LANES = CL && !TAPE;
  const int nl = LANES ? ty.nl : nb;
  const int lane = threadIdx.x & 63;
  // lanes past the wavefront's last environment slot shadow the first
  // slot's lanes: every row they read lies within the wavefront's 64, and
  // they store nothing
  const int per_wave = 64 / nl;
  const bool spare = lane >= per_wave * nl;
  const int slot = spare ? 0 : lane / nl;
  const int b = spare ? lane - per_wave * nl : lane - slot * nl;
  const int base = slot * nl;
  const bool live = !spare && slot < wk.count;
  const int e = env_list[type_off[t] + wk.k0 + (live ? slot : 0)];
  BodyT B = tab->body[t][b];
  const int bs = LANES ? B.body_of : b;  // the body whose state this lane holds
  const bool has_joint = B.joint >= 0;
  JointT J = tab->joint[t][has_joint ? B.joint : 0];
  const int src_parent = base + (has_joint ? J.parent : b);
  const int cfirst = LANES ? B.l0 : B.c0;
  const int n_con = LANES ? B.l1 - B.l0 : B.c1 - B.c0;
  const int max_con = LANES ? ty.max_lc : ty.max_contacts;
  ContactT Creg[REGC];
#pragma unroll
  for (int k = 0; k < REGC; ++k) Creg[k] = tab->contact[t][cfirst + (n_con > k ? k : 0)];
  pin_consts<MAXDOF>(B, J, has_joint, Creg, REGC);
  const float h = ty.h;

  if (PAIRS && ty.np > 0) pair_lanes_load(tab, t, pl, lane, nl);
  const PairSlot0 ps0 = (PAIRS && ty.np > 0) ? pair_slot0(*pl, b, base) : PairSlot0{-1, lane, lane};
  Body s = load_body(in, bs, e, Bm, E);
  const float x_before = s.p.x;  // the environment layer's root progress
  // frozen velocity components zeroed once; every update below keeps them zero
  s.v = keep(s.v, B.free_p);
  s.w = keep(s.w, B.free_r);
  int n_save = 0;
  // actions acts[step][Am][E], held over the substeps of a step; each step's
  // are loaded one step ahead so that the loads' latency is hidden
  float raw_next[3] = {0.f, 0.f, 0.f};
  if (has_joint && T > 0)
    for (int x = 0; x < MAXDOF; ++x) raw_next[x] = act_raw(acts, J, x, e, E);
  for (int step = 0; step < T; ++step) {
    float a[3] = {0.f, 0.f, 0.f};
    for (int x = 0; x < MAXDOF; ++x) a[x] = clampf(raw_next[x], J.act_lo[x], J.act_hi[x]);
    if (has_joint && step + 1 < T)
      for (int x = 0; x < MAXDOF; ++x) raw_next[x] = act_raw(acts + (size_t)(step + 1) * Am * E, J, x, e, E);
    for (int sub = 0; sub < ty.substeps; ++sub) {
      float* tp = TAPE ? tape + (((size_t)step * smax + sub) * n_work + w) * TAPE_N * 64 : nullptr;
      if (TAPE) wtape_state(tp, s, lane);
      kinematic_unmasked(s, h);
      // parent's post-kinematic state through the exchange rows: this body's
      // state is written first and its rotation formed while that is in
      // flight; the parent's rotation matrix is read from the parent lane's
      xch_put_pvw(X, lane, s);
      const m3 R = quat_to_mat(s.q);
      xch_put_rot(X, lane, s.w.z, R);
      Body P;
      m3 RP;
      xch_get_pvw_rot(X, src_parent, P, RP);
      // body-body slot 0: its bound test on the positions and rotations in
      // the rows now
      const int near0 = (PAIRS && ty.np > 0) ? pair_near0(X, *pl, ps0) : 0;
      P.q = s.q;  // unused: the joint reads the parent's orientation as RP
      Frame f = derive_inv(B, R);
      JointChild jc = joint_child<MAXDOF>(J, s, R);
      // the contact candidates while the parent's state is in flight (they
      // need none of it): the first REGC from registers (no dynamic indexing;
      // a slot no body of the type has is skipped by the whole wave), the
      // rest from the table
      v3 dv = V(0.f, 0.f, 0.f), dw = V(0.f, 0.f, 0.f);
      int cnt = 0;
      if (REGC == 2 && !TAPE && (!CL || PAIRS)) {
        // the penetrating candidates first, in candidate order (the same
        // sums), so that the second evaluation's impulse runs only where a
        // lane has two penetrating candidates, not wherever one has its
        // second (measured per kernel: biped 14.0 -> 13.0 ms, planar runner
        // 10.3 -> 10.0, grasp 24.7 -> 24.2; the contact-lane kernels without
        // body-body contacts lost 2-3% and keep the plain order)
        const v3 rl0 = mul(f.R, ld3(Creg[0].l)), rl1 = mul(f.R, ld3(Creg[REGC - 1].l));
        const float d0 = Creg[0].rho - (s.p.z + rl0.z), d1 = Creg[REGC - 1].rho - (s.p.z + rl1.z);
        const bool p0 = 0 < max_con && n_con > 0 && d0 > 0.f;
        const bool p1 = 1 < max_con && n_con > 1 && d1 > 0.f;
        if (p0 || p1)
          cnt += contact_apply(p0 ? Creg[0].rho : Creg[REGC - 1].rho, ty, B, s, f, sel(p0, rl0, rl1), p0 ? d0 : d1,
                               dv, dw)
                     ? 1
                     : 0;
        if (p0 && p1) cnt += contact_apply(Creg[REGC - 1].rho, ty, B, s, f, rl1, d1, dv, dw) ? 1 : 0;
      } else {
#pragma unroll
        for (int k = 0; k < REGC; ++k)
          if (k < max_con && n_con > k) cnt += contact_eval(Creg[k], ty, B, s, f, dv, dw) ? 1 : 0;
      }
      for (int c = REGC; c < n_con; ++c) cnt += contact_eval(tab->contact[t][cfirst + c], ty, B, s, f, dv, dw) ? 1 : 0;
      // joint evaluated on every lane (a root uses its own state as the
      // parent and its result is discarded)
      JointOut jo = joint_eval<MAXDOF>(J, P, RP, s, jc, a);
      // children's reactions (child order); a child's reaction on its parent
      // is the opposite of its (F, rP x F + tau), read as is and subtracted
      v3 cf[GATHER], ct[GATHER];
      xch_put2(X, lane, jo.fc, jo.tpn);
#pragma unroll
      for (int i = 0; i < GATHER; ++i) {
        if (i < ty.max_children) {
          const int src = base + (i < B.nch ? (int)((B.ch_packed >> (4 * i)) & 15u) : b);
          xch_get2(X, src, cf[i], ct[i]);
        }
      }
      const v3 z3 = V(0.f, 0.f, 0.f);
      v3 force = has_joint ? jo.fc : z3, torque = has_joint ? jo.tc : z3;
#pragma unroll
      for (int i = 0; i < GATHER; ++i) {
        if (i < B.nch) {
          force -= cf[i];
          torque -= ct[i];
        }
      }
      for (int i = GATHER; i < ty.max_children; ++i) {
        const int src = base + (i < B.nch ? (int)((B.ch_packed >> (4 * i)) & 15u) : b);
        v3 fc, tq;
        xch_get2(X, src, fc, tq);
        if (i < B.nch) {
          force -= fc;
          torque -= tq;
        }
      }
      // a body's contact candidates spread over its lane group: every lane of
      // the group adds the group's sums in group order (the same total on
      // each, so the copies of the state stay equal); the exchange rows are
      // free once the children's reactions have been read
      if (LANES && nl > nb) {
        X->r[lane][0] = make_float4(dv.x, dv.y, dv.z, (float)cnt);
        X->r[lane][1] = make_float4(dw.x, dw.y, dw.z, 0.f);
        v3 sv = V(0.f, 0.f, 0.f), sw = sv;
        int sc = 0;
        // four rows read together, then added in order (a group has at most 8 lanes)
        for (int i0 = 0; i0 < ty.max_ng; i0 += 4) {
          float4 gv[4], gw[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int i = i0 + j;
            const int src = base + (i < B.ng ? (int)((B.grp_packed >> (4 * (i & 7))) & 15u) : b);
            gv[j] = X->r[src][0];
            gw[j] = X->r[src][1];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (i0 + j < B.ng) {
              sv += V(gv[j].x, gv[j].y, gv[j].z);
              sw += V(gw[j].x, gw[j].y, gw[j].z);
              sc += (int)gv[j].w;
            }
          }
        }
        dv = sv;
        dw = sw;
        cnt = sc;
      }
      // body-body contacts after the joint sums, where fewer values are live
      if (PAIRS && ty.np > 0) pair_phase(tab, t, *pl, X, lane, b, base, s, f, dv, dw, cnt, near0);
      if (TAPE) wtape_rest(tp, torque, cnt, lane);
      // without frozen axes in the type (wave-uniform) the integrators skip the masks
      if (ty.frozen) {
        potential(B, ty, s, f, force, torque);
        collision(B, s, dv, dw, cnt);
      } else {
        potential<false>(B, ty, s, f, force, torque);
        collision<false>(B, s, dv, dw, cnt);
      }
    }
    if (save_every > 0 && (step + 1) % save_every == 0) {
      if (live && b < nb) store_snapshot(traj, (size_t)n_save, s, b, e, Bm, E);
      ++n_save;
    }
  }
  if (nonfinite) {
    const unsigned long long bad = __ballot(live && !finite_body(s));
    const unsigned long long group = (nb >= 64) ? ~0ull : ((1ull << nb) - 1ull);
    if (live && b == 0) nonfinite[e] = ((bad >> base) & group) ? 1 : 0;
  }
  bool finished = false;
  if (ENV) {
    // reward and termination from the stepped state (the root's lane holds it)
    const EnvT P = ea->env[t];
    const int rl = base + P.root;
    const float x0 = shfl(x_before, rl), x1 = shfl(s.p.x, rl), z1 = shfl(s.p.z, rl);
    const bool healthy = z1 >= P.z_min && z1 <= P.z_max;
    finished = !healthy;
    // control cost: the squared actions as passed, summed over the
    // environment's lanes in body order
    float sq = 0.f;
    for (int x = 0; x < MAXDOF; ++x) sq += raw_next[x] * raw_next[x];
    float ctrl = 0.f;
    for (int i = 0; i < nb; ++i) ctrl += shfl(sq, base + i);
    if (live && b == P.root) {
      ea->reward[e] = P.forward_weight * (x1 - x0) / ty.dt + (healthy ? P.healthy_reward : 0.f) - P.ctrl_cost * ctrl;
      ea->done[e] = healthy ? 0 : 1;
    }
    // a finished environment continues from its reset state
    if (finished && live) s = load_body(ea->reset, bs, e, Bm, E);
    // observation of the final state: joint angles and relative angular
    // velocity about each Euler axis on the child's lane (the parent's
    // rotation and angular velocity read across lanes), the root's entries
    // and the padding on the root's lane
    const m3 Rf = quat_to_mat(s.q);
    m3 RPf;
#pragma unroll
    for (int i = 0; i < 9; ++i) RPf.m[i] = shfl(Rf.m[i], src_parent);
    const v3 wP = V(shfl(s.w.x, src_parent), shfl(s.w.y, src_parent), shfl(s.w.z, src_parent));
    const JointGeo g = joint_geo<MAXDOF>(J, RPf, joint_child<MAXDOF>(J, s, Rf));
    const v3 wrel = s.w - wP;
    const int D = ty.ndof;
    if (live && has_joint && b < nb) {
      for (int k = 0; k < MAXDOF; ++k) {
        if (k < J.dof) {
          ea->obs[(size_t)(11 + J.dof0 + k) * E + e] = g.th[k];
          ea->obs[(size_t)(11 + D + J.dof0 + k) * E + e] = dot(wrel, g.ax[k]);
        }
      }
    }
    if (live && b == P.root) {
      const float head[11] = {s.p.z, s.q.w, s.q.x, s.q.y, s.q.z, s.v.x, s.v.y, s.v.z, s.w.x, s.w.y, s.w.z};
#pragma unroll
      for (int k = 0; k < 11; ++k) ea->obs[(size_t)k * E + e] = head[k];
      for (int k = 11 + 2 * D; k < ea->Omax; ++k) ea->obs[(size_t)k * E + e] = 0.f;
    }
  }
  if (live && b < nb) {
    store_body(out, 0, s, b, e, Bm, E);
    // padded body slots of a smaller system are written as zeros (a finished
    // environment's as its reset state's)
    for (int pb = nb + b; pb < Bm; pb += nb) {
      if (ENV && finished)
        store_body(out, 0, load_body(ea->reset, pb, e, Bm, E), pb, e, Bm, E);
      else
        zero_body(out, pb, e, Bm, E);
    }
  }
}

// ONE_AXIS: every type of the batch has joints of at most one axis, so only
// that path is compiled in (fewer registers). REGC: contact candidates per
// body held in registers (8 for batches with a body of more than two, such
// as a box's eight corners; 2 otherwise, where more registers only cost).
template <bool ONE_AXIS, int REGC, bool CL>
__global__ __launch_bounds__(256) void k_fused(const Tables* __restrict__ tab, const WaveWork* __restrict__ work,
                                               int n_work, const int32_t* __restrict__ env_list,
                                               const int32_t* __restrict__ type_off, int E, int Bm, Fields in,
                                               Fields out, const float* __restrict__ acts, int Am, int T,
                                               int save_every, Fields traj, uint8_t* nonfinite, float* tape,
                                               int smax) {
  extern __shared__ float4 fused_lds[];  // exchange rows, one set per wavefront of the block
  const int w = wave_index();
  if (w >= n_work) return;
  const WaveWork wk = work[w];
  XchRows* X = xch_lanes(fused_lds);
  // wave-uniform: joints of at most one axis take the shorter path
  if (ONE_AXIS || tab->type[wk.type].max_dof <= 1)
    fused_run<1, false, false, REGC, false, CL>(tab, wk, env_list, type_off, E, Bm, in, out, acts, Am, T,
                                                save_every, traj, nonfinite, nullptr, 0, w, n_work, X);
  else
    fused_run<3, false, false, REGC, false, CL>(tab, wk, env_list, type_off, E, Bm, in, out, acts, Am, T,
                                                save_every, traj, nonfinite, nullptr, 0, w, n_work, X);
}

// The same with the forward tape: a kernel of its own, so that the tape
// code does not add to the registers of the kernel above. Its states may
// differ from k_fused's at the rounding level (the compiler may fuse
// multiply-adds differently in the two), so a checkpointed gradient takes
// both its checkpoints and its recomputed segments from this kernel.
template <int REGC>
__global__ __launch_bounds__(256) void k_fused_tape(const Tables* __restrict__ tab,
                                                    const WaveWork* __restrict__ work, int n_work,
                                                    const int32_t* __restrict__ env_list,
                                                    const int32_t* __restrict__ type_off, int E, int Bm, Fields in,
                                                    Fields out, const float* __restrict__ acts, int Am, int T,
                                                    int save_every, Fields traj, uint8_t* nonfinite, float* tape,
                                                    int smax) {
  extern __shared__ float4 fused_lds[];
  const int w = wave_index();
  if (w >= n_work) return;
  const WaveWork wk = work[w];
  XchRows* X = xch_lanes(fused_lds);
  if (tab->type[wk.type].max_dof <= 1)
    fused_run<1, true, false, REGC>(tab, wk, env_list, type_off, E, Bm, in, out, acts, Am, T, save_every, traj,
                                    nonfinite, tape, smax, w, n_work, X);
  else
    fused_run<3, true, false, REGC>(tab, wk, env_list, type_off, E, Bm, in, out, acts, Am, T, save_every, traj,
                                    nonfinite, tape, smax, w, n_work, X);
}

// The same for batches with body-body contacts: kernels of their own (with
// and without the tape), so that the registers the body-body phase needs do
// not lower the occupancy of the kernel above. REGC as for k_fused (8 for a
// batch with a box, whose corners are otherwise read from the table in the
// substep loop).
template <bool TAPE, bool ONE_AXIS, int REGC, bool CL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_fused_pairs(const Tables* __restrict__ tab,
                                                     const WaveWork* __restrict__ work, int n_work,
                                                     const int32_t* __restrict__ env_list,
                                                     const int32_t* __restrict__ type_off, int E, int Bm, Fields in,
                                                     Fields out, const float* __restrict__ acts, int Am, int T,
                                                     int save_every, Fields traj, uint8_t* nonfinite, float* tape,
                                                     int smax) {
  extern __shared__ float4 fused_lds[];  // exchange rows, then body-body tables, one set per wavefront
  const int w = wave_index();
  if (w >= n_work) return;
  const WaveWork wk = work[w];
  XchRows* X = xch_lanes(fused_lds);
  PairLanes* pl = pair_lanes(fused_lds);
  if (ONE_AXIS || tab->type[wk.type].max_dof <= 1)
    fused_run<1, TAPE, true, REGC, false, CL>(tab, wk, env_list, type_off, E, Bm, in, out, acts, Am, T, save_every,
                                              traj, nonfinite, tape, smax, w, n_work, X, pl);
  else
    fused_run<3, TAPE, true, REGC, false, CL>(tab, wk, env_list, type_off, E, Bm, in, out, acts, Am, T, save_every,
                                              traj, nonfinite, tape, smax, w, n_work, X, pl);
}

// One environment step with the environment layer fused after it (T = 1):
// kernels of their own so that the epilogue's registers do not weigh on the
// rollout kernels. PAIRS: batches with body-body candidates.
template <bool PAIRS, int REGC, bool CL>
__global__ __launch_bounds__(256) void k_fused_env(const Tables* __restrict__ tab, const WaveWork* __restrict__ work,
                                                   int n_work, const int32_t* __restrict__ env_list,
                                                   const int32_t* __restrict__ type_off, int E, int Bm, Fields in,
                                                   Fields out, const float* __restrict__ acts, int Am,
                                                   uint8_t* nonfinite, EnvArgs ea) {
  extern __shared__ float4 fused_lds[];  // exchange rows, then body-body tables (PAIRS), per wavefront
  const int w = wave_index();
  if (w >= n_work) return;
  const WaveWork wk = work[w];
  XchRows* X = xch_lanes(fused_lds);
  PairLanes* pl = PAIRS ? pair_lanes(fused_lds) : nullptr;
  const Fields none{nullptr, nullptr, nullptr, nullptr};
  if (tab->type[wk.type].max_dof <= 1)
    fused_run<1, false, PAIRS, REGC, true, CL>(tab, wk, env_list, type_off, E, Bm, in, out, acts, Am, 1, 0, none,
                                               nonfinite, nullptr, 0, w, n_work, X, pl, &ea);
  else
    fused_run<3, false, PAIRS, REGC, true, CL>(tab, wk, env_list, type_off, E, Bm, in, out, acts, Am, 1, 0, none,
                                               nonfinite, nullptr, 0, w, n_work, X, pl, &ea);
}

// ------------------------------------------------------------------ small helpers
__global__ void k_copy_state(int n3, int n4, Fields in, Fields out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) {
    out.pos[i] = in.pos[i];
    out.vel[i] = in.vel[i];
    out.ang[i] = in.ang[i];
  }
  if (i < n4) out.rot[i] = in.rot[i];
}

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------ environment layer
hipError_t launch_env_step(const LaunchCtx& c, const WaveWork* work, int n_work, int waves_per_block,
                           const EnvT* env, int Omax, Fields in, Fields out, const float* act, Fields reset, float* obs,
                           float* reward, uint8_t* done, bool flags, hipStream_t s) {
  if (n_work == 0) return hipSuccess;
  bool pairs = false, many_contacts = false, cl = false;
  for (int t = 0; t < c.n_types; ++t) {
    pairs = pairs || c.host_tab->type[t].np > 0;
    many_contacts = many_contacts || c.host_tab->type[t].max_lc > REG_CONTACTS;  // per lane, contact lanes included
    cl = cl || c.host_tab->type[t].nl > c.host_tab->type[t].nb;
  }
  const dim3 grid(cdiv(n_work, waves_per_block)), block(64 * waves_per_block);
  uint8_t* nf = flags ? c.nonfinite : nullptr;
  const EnvArgs ea{env, reset, obs, reward, done, Omax};
  const size_t lds = fused_lds_per_wave(pairs) * waves_per_block;
#define BX_ENV(P, R, L)                                                                                            \
  hipLaunchKernelGGL((k_fused_env<P, R, L>), grid, block, lds, s, c.tab, work, n_work, c.env_list, c.type_off, c.E, \
                     c.Bm, in, out, act, c.Am, nf, ea)
  // with contact lanes, candidates past a lane's first two are read from the table
  if (pairs && cl)
    BX_ENV(true, REG_CONTACTS, true);
  else if (pairs)
    BX_ENV(true, REG_CONTACTS, false);
  else if (cl)
    BX_ENV(false, REG_CONTACTS, true);
  else if (many_contacts)
    BX_ENV(false, 8, false);
  else
    BX_ENV(false, REG_CONTACTS, false);
#undef BX_ENV
  return hipGetLastError();
}

__global__ void k_fill_u8(uint8_t* p, int n, uint8_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_default_qp(const LaunchCtx& c, const float* angles, const float* root_off, Fields out,
                             hipStream_t s) {
  if (c.E == 0) return hipSuccess;
  hipLaunchKernelGGL(k_default_qp, dim3(cdiv(c.E, 64)), dim3(64), 0, s, c.tab, c.env_type, c.E, c.Bm, angles,
                     root_off, out);
  return hipGetLastError();
}

hipError_t launch_fused(const LaunchCtx& c, const WaveWork* work, int n_work, int waves_per_block, Fields in,
                        Fields out, const float* acts, int T, int save_every, Fields traj, bool flags,
                        hipStream_t s, float* tape, int smax) {
  if (n_work == 0) return hipSuccess;
  bool pairs = false, one_axis = true, many_contacts = false, many_lane_contacts = false, cl = false;
  for (int t = 0; t < c.n_types; ++t) {
    pairs = pairs || c.host_tab->type[t].np > 0;
    one_axis = one_axis && c.host_tab->type[t].max_dof <= 1;
    // per lane: the tape kernels hold a body's candidates on its lane, the
    // others spread them over contact lanes
    many_contacts = many_contacts || c.host_tab->type[t].max_contacts > REG_CONTACTS;
    many_lane_contacts = many_lane_contacts || c.host_tab->type[t].max_lc > REG_CONTACTS;
    cl = cl || c.host_tab->type[t].nl > c.host_tab->type[t].nb;
  }
  // kernels with contact lanes hold two candidates per lane in registers
  // (further ones, of a type whose lanes did not fit, are read from the table)
  if (cl) many_lane_contacts = false;
  const size_t lds = fused_lds_per_wave(pairs) * waves_per_block;
  if (pairs) {
    const dim3 grid(cdiv(n_work, waves_per_block)), block(64 * waves_per_block);
    uint8_t* nf = flags ? c.nonfinite : nullptr;
    // the tape kernel keeps two register candidates (the tape rows take the registers)
    if (tape)
      hipLaunchKernelGGL((k_fused_pairs<true, false, REG_CONTACTS>), grid, block, lds, s, c.tab, work, n_work,
                         c.env_list, c.type_off, c.E, c.Bm, in, out, acts, c.Am, T, save_every, traj, nf, tape, smax);
    else if (one_axis && many_lane_contacts)
      hipLaunchKernelGGL((k_fused_pairs<false, true, 8>), grid, block, lds, s, c.tab, work, n_work, c.env_list,
                         c.type_off, c.E, c.Bm, in, out, acts, c.Am, T, save_every, traj, nf, nullptr, 0);
    else if (one_axis && cl)
      hipLaunchKernelGGL((k_fused_pairs<false, true, REG_CONTACTS, true>), grid, block, lds, s, c.tab, work, n_work,
                         c.env_list, c.type_off, c.E, c.Bm, in, out, acts, c.Am, T, save_every, traj, nf, nullptr, 0);
    else if (one_axis)
      hipLaunchKernelGGL((k_fused_pairs<false, true, REG_CONTACTS>), grid, block, lds, s, c.tab, work, n_work,
                         c.env_list, c.type_off, c.E, c.Bm, in, out, acts, c.Am, T, save_every, traj, nf, nullptr, 0);
    else if (cl)
      hipLaunchKernelGGL((k_fused_pairs<false, false, REG_CONTACTS, true>), grid, block, lds, s, c.tab, work, n_work,
                         c.env_list, c.type_off, c.E, c.Bm, in, out, acts, c.Am, T, save_every, traj, nf, nullptr, 0);
    else
      hipLaunchKernelGGL((k_fused_pairs<false, false, REG_CONTACTS>), grid, block, lds, s, c.tab, work, n_work,
                         c.env_list, c.type_off, c.E, c.Bm, in, out, acts, c.Am, T, save_every, traj, nf, nullptr, 0);
    return hipGetLastError();
  }
  if (tape && many_contacts)
    hipLaunchKernelGGL((k_fused_tape<8>), dim3(cdiv(n_work, waves_per_block)), dim3(64 * waves_per_block), lds, s,
                       c.tab, work, n_work, c.env_list, c.type_off, c.E, c.Bm, in, out, acts, c.Am, T, save_every,
                       traj, flags ? c.nonfinite : nullptr, tape, smax);
  else if (tape)
    hipLaunchKernelGGL((k_fused_tape<REG_CONTACTS>), dim3(cdiv(n_work, waves_per_block)), dim3(64 * waves_per_block),
                       lds, s, c.tab, work, n_work, c.env_list, c.type_off, c.E, c.Bm, in, out, acts, c.Am, T,
                       save_every, traj, flags ? c.nonfinite : nullptr, tape, smax);
  else {
    const dim3 grid(cdiv(n_work, waves_per_block)), block(64 * waves_per_block);
    uint8_t* nf = flags ? c.nonfinite : nullptr;
#define BX_FUSED(A, R, L)                                                                                         \
  hipLaunchKernelGGL((k_fused<A, R, L>), grid, block, lds, s, c.tab, work, n_work, c.env_list, c.type_off, c.E, c.Bm, \
                     in, out, acts, c.Am, T, save_every, traj, nf, nullptr, 0)
    if (one_axis && cl)
      BX_FUSED(true, REG_CONTACTS, true);
    else if (cl)
      BX_FUSED(false, REG_CONTACTS, true);
    else if (one_axis && many_lane_contacts)
      BX_FUSED(true, 8, false);
    else if (one_axis)
      BX_FUSED(true, REG_CONTACTS, false);
    else if (many_lane_contacts)
      BX_FUSED(false, 8, false);
    else
      BX_FUSED(false, REG_CONTACTS, false);
#undef BX_FUSED
  }
  return hipGetLastError();
}

hipError_t launch_copy_state(const LaunchCtx& c, Fields in, Fields out, hipStream_t s) {
  const int n3 = 3 * c.Bm * c.E, n4 = 4 * c.Bm * c.E;
  if (n4 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_state, dim3(cdiv(n4, 256)), dim3(256), 0, s, n3, n4, in, out);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, int n, uint8_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(cdiv(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// One plain step: for every type, `substeps` x (kinematic, joint+actuator,
// contact, potential, collision) launches. `in` is read by the first
// kinematic launch only; everything after works in place on `out`.
hipError_t launch_plain_step(const LaunchCtx& c, Fields in, Fields out, const float* act, float* const* jslot,
                             float* const* cslot, bool flags, hipStream_t s, float* tape) {
  const int TB = 256;
  for (int t = 0; t < c.n_types; ++t) {
    const int n = c.type_cnt_h[t];
    if (n == 0) continue;
    const TypeT& ty = c.host_tab->type[t];
    const int32_t* envs = c.env_list + c.type_off_h[t];
    for (int sub = 0; sub < ty.substeps; ++sub) {
      const bool first = sub == 0;
      float* tp = tape ? tape + (size_t)sub * TAPE_N * c.Bm * c.E : nullptr;
      hipLaunchKernelGGL(k_plain_kinematic, dim3(cdiv((long)c.Bm * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, c.E,
                         c.Bm, first ? in : out, out, first ? 1 : 0, tp);
      if (ty.nj > 0) {
        if (ty.max_dof <= 1)
          hipLaunchKernelGGL(k_plain_joint<1>, dim3(cdiv((long)ty.nj * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n,
                             c.E, c.Bm, out, act, jslot[t]);
        else
          hipLaunchKernelGGL(k_plain_joint<3>, dim3(cdiv((long)ty.nj * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n,
                             c.E, c.Bm, out, act, jslot[t]);
      }
      if (ty.nc > 0)
        hipLaunchKernelGGL(k_plain_contact, dim3(cdiv((long)ty.nc * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, c.E,
                           c.Bm, out, cslot[t]);
      if (ty.np > 0)
        hipLaunchKernelGGL(k_plain_pair, dim3(cdiv((long)ty.np * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, c.E,
                           c.Bm, out, cslot[t]);
      hipLaunchKernelGGL(k_plain_potential, dim3(cdiv((long)ty.nb * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, c.E,
                         c.Bm, out, jslot[t], tp);
      hipLaunchKernelGGL(k_plain_collision, dim3(cdiv((long)ty.nb * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, c.E,
                         c.Bm, out, cslot[t], flags ? c.nonfinite : nullptr, sub == ty.substeps - 1 ? 1 : 0, tp);
      hipError_t err = hipGetLastError();
      if (err != hipSuccess) return err;
    }
  }
  return hipSuccess;
}

}  // namespace bx
