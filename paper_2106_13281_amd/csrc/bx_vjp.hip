// Adjoint of one step on the GPU (vector-Jacobian product of brax_step).
//
// 1. Forward recompute of the step's substeps, writing a tape per substep:
//    each body's state before the kinematic update, the total torque it
//    received and its count of applied contacts.
// 2. Reverse over the substeps, one launch per phase (Algorithm 1 reversed):
//      integrate  collision + potential integrators -> cotangents of the
//                 body's post-kinematic state, of its force/torque sums and
//                 of its contact sums
//      joint      spring joints           -> parent/child state cotangents
//      actuator   torque actuators        -> rotation cotangents, action cotangents
//      contact    ground contacts         -> body state cotangents
//      kinematic  gathers all of the above in a fixed order, then the
//                 kinematic integrator's adjoint -> cotangent of the
//                 substep's input state
//    Per-joint/contact results go to fixed slots; the gather order is fixed,
//    so the result is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "bx_access.h"
#include "bx_adj.h"
#include "bx_pair_lanes.h"
#include "bx_vjp.h"

namespace bx {

namespace {

constexpr int TB = 256;
inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ Bar load_bar(const Fields& f, int b, int e, int Bm, int E) {
  Body s = load_body(f, b, e, Bm, E);
  Bar r;
  r.p = s.p;
  r.q = s.q;
  r.v = s.v;
  r.w = s.w;
  return r;
}
__device__ __forceinline__ void store_bar(const Fields& f, const Bar& r, int b, int e, int Bm, int E) {
  Body s;
  s.p = r.p;
  s.q = r.q;
  s.v = r.v;
  s.w = r.w;
  store_body(f, 0, s, b, e, Bm, E);
}
// 13-float bar in a [13 * N][n] slot array at item i, environment slot k
__device__ __forceinline__ void slot_store_bar(float* sl, int x0, int N, int i, int n, int k, const Bar& r) {
  const float v[13] = {r.p.x, r.p.y, r.p.z, r.q.w, r.q.x, r.q.y, r.q.z, r.v.x, r.v.y, r.v.z, r.w.x, r.w.y, r.w.z};
  for (int x = 0; x < 13; ++x) sl[((size_t)(x0 + x) * N + i) * n + k] = v[x];
}
__device__ __forceinline__ void slot_add_bar(const float* sl, int x0, int N, int i, int n, int k, Bar& r) {
  float v[13];
  for (int x = 0; x < 13; ++x) v[x] = sl[((size_t)(x0 + x) * N + i) * n + k];
  Bar a;
  a.p = V(v[0], v[1], v[2]);
  a.q = q4{v[3], v[4], v[5], v[6]};
  a.v = V(v[7], v[8], v[9]);
  a.w = V(v[10], v[11], v[12]);
  bar_add(r, a);
}
// per-body vectors [6][Bm][E]
__device__ __forceinline__ void store2(float* p, v3 a, v3 b, int bb, int e, int Bm, int E) {
  const float v[6] = {a.x, a.y, a.z, b.x, b.y, b.z};
  for (int x = 0; x < 6; ++x) p[((size_t)x * Bm + bb) * E + e] = v[x];
}
__device__ __forceinline__ void load2(const float* p, v3& a, v3& b, int bb, int e, int Bm, int E) {
  float v[6];
  for (int x = 0; x < 6; ++x) v[x] = p[((size_t)x * Bm + bb) * E + e];
  a = V(v[0], v[1], v[2]);
  b = V(v[3], v[4], v[5]);
}
__device__ __forceinline__ Body post_kin(const Tables* tab, int t, const float* tape_s, int b, int e, int Bm, int E) {
  Body s = tape_load_state(tape_s, b, e, Bm, E);
  kinematic(tab->body[t][b], s, tab->type[t].h);
  return s;
}

// g_in <- g_out on real bodies, 0 on padded body slots.
__global__ void k_adj_init(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n, int E,
                           int Bm, Fields g_out, Fields g_in) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = idx / n, k = idx - b * n;
  if (b >= Bm) return;
  const int e = envs[k];
  if (b < tab->type[t].nb) {
    store_body(g_in, 0, load_body(g_out, b, e, Bm, E), b, e, Bm, E);
  } else {
    Body z;
    z.p = z.v = z.w = V(0.f, 0.f, 0.f);
    z.q = q4{0.f, 0.f, 0.f, 0.f};
    store_body(g_in, 0, z, b, e, Bm, E);
  }
}

__global__ void k_fill_f32(float* p, size_t n, float v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Integrate phase adjoint (collision then potential integrator).
__global__ void k_adj_integrate(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n,
                                int E, int Bm, const float* __restrict__ tape_s, Fields G, float* __restrict__ bpart,
                                float* __restrict__ ftb, float* __restrict__ dvw) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = idx / n, k = idx - b * n;
  const TypeT& ty = tab->type[t];
  if (b >= ty.nb) return;
  const int e = envs[k];
  const BodyT& B = tab->body[t][b];
  Body post = post_kin(tab, t, tape_s, b, e, Bm, E);
  Frame f = derive(B, post);
  Bar ob = load_bar(G, b, e, Bm, E);
  v3 fb, tb, dvb, dwb;
  Bar part = integrate_adj(B, ty, post, f, tape_load_torque(tape_s, b, e, Bm, E), tape_load_count(tape_s, b, e, Bm, E),
                           ob, fb, tb, dvb, dwb);
  store_bar(Fields{bpart, bpart + 3 * Bm * E, bpart + 7 * Bm * E, bpart + 10 * Bm * E}, part, b, e, Bm, E);
  store2(ftb, fb, tb, b, e, Bm, E);
  store2(dvw, dvb, dwb, b, e, Bm, E);
}

// Joint (spring) phase adjoint: slot j holds (parent bar, child bar).
template <int MAXDOF>
__global__ void k_adj_joint(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n, int E,
                            int Bm, const float* __restrict__ tape_s, const float* __restrict__ ftb,
                            float* __restrict__ jbar) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = idx / n, k = idx - j * n;
  const TypeT& ty = tab->type[t];
  if (j >= ty.nj) return;
  const int e = envs[k];
  const JointT& J = tab->joint[t][j];
  Body P = post_kin(tab, t, tape_s, J.parent, e, Bm, E);
  Body C = post_kin(tab, t, tape_s, J.child, e, Bm, E);
  m3 RP = quat_to_mat(P.q), RC = quat_to_mat(C.q);
  v3 fcb, tcb, fpb, tpb;
  load2(ftb, fcb, tcb, J.child, e, Bm, E);
  load2(ftb, fpb, tpb, J.parent, e, Bm, E);
  Bar bP = bar_zero(), bC = bar_zero();
  joint_spring_adj<MAXDOF>(J, P, RP, C, RC, fcb, tcb, fpb, tpb, bP, bC);
  slot_store_bar(jbar, 0, ty.nj, j, n, k, bP);
  slot_store_bar(jbar, 13, ty.nj, j, n, k, bC);
}

// Actuator phase adjoint: slot j holds (parent bar, child bar); the action
// cotangents are accumulated into g_act (one writer per action and
// environment per substep; substeps run in order).
template <int MAXDOF>
__global__ void k_adj_actuator(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n, int E,
                               int Bm, const float* __restrict__ tape_s, const float* __restrict__ ftb,
                               const float* __restrict__ act, float* __restrict__ abar, float* __restrict__ g_act) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = idx / n, k = idx - j * n;
  const TypeT& ty = tab->type[t];
  if (j >= ty.nj) return;
  const int e = envs[k];
  const JointT& J = tab->joint[t][j];
  Body P = post_kin(tab, t, tape_s, J.parent, e, Bm, E);
  Body C = post_kin(tab, t, tape_s, J.child, e, Bm, E);
  m3 RP = quat_to_mat(P.q), RC = quat_to_mat(C.q);
  v3 fcb, tcb, fpb, tpb;
  load2(ftb, fcb, tcb, J.child, e, Bm, E);
  load2(ftb, fpb, tpb, J.parent, e, Bm, E);
  float a[3], raw[3], ab[3];
  for (int x = 0; x < 3; ++x) {
    raw[x] = J.act[x] >= 0 ? act[(size_t)J.act[x] * E + e] : 0.f;
    a[x] = clampf(raw[x], J.act_lo[x], J.act_hi[x]);
  }
  Bar bP = bar_zero(), bC = bar_zero();
  joint_actuator_adj<MAXDOF>(J, P, RP, C, RC, a, tcb, tpb, bP, bC, ab);
  slot_store_bar(abar, 0, ty.nj, j, n, k, bP);
  slot_store_bar(abar, 13, ty.nj, j, n, k, bC);
  for (int x = 0; x < MAXDOF; ++x)
    if (x < J.dof && J.act[x] >= 0 && raw[x] >= J.act_lo[x] && raw[x] <= J.act_hi[x]) g_act[(size_t)J.act[x] * E + e] += ab[x];
}

// Contact phase adjoint: slot c holds the body bar (zero when no impulse).
__global__ void k_adj_contact(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n, int E,
                              int Bm, const float* __restrict__ tape_s, const float* __restrict__ dvw,
                              float* __restrict__ cbar) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = idx / n, k = idx - c * n;
  const TypeT& ty = tab->type[t];
  if (c >= ty.nc) return;
  const int e = envs[k];
  const ContactT& Cc = tab->contact[t][c];
  const BodyT& B = tab->body[t][Cc.body];
  Body s = post_kin(tab, t, tape_s, Cc.body, e, Bm, E);
  Frame f = derive(B, s);
  v3 dvb, dwb;
  load2(dvw, dvb, dwb, Cc.body, e, Bm, E);
  bool applied;
  Bar r = contact_adj(Cc, ty, B, s, f, dvb, dwb, applied);
  if (!applied) r = bar_zero();
  slot_store_bar(cbar, 0, ty.nc, c, n, k, r);
}

// Body-body phase adjoint: slot c holds the first body's bar, then the
// second's (zero when no impulse).
__global__ void k_adj_pair(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n, int E,
                           int Bm, const float* __restrict__ tape_s, const float* __restrict__ dvw,
                           float* __restrict__ pbar) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = idx / n, k = idx - c * n;
  const TypeT& ty = tab->type[t];
  if (c >= ty.np) return;
  const int e = envs[k];
  const PairT& P = tab->pair[t][c];
  const int ids[2] = {P.a, P.b};
  Body post[2];
  Frame f[2];
  PairSide side[2];
  v3 dvb[2], dwb[2];
  for (int i = 0; i < 2; ++i) {
    post[i] = post_kin(tab, t, tape_s, ids[i], e, Bm, E);
    f[i] = derive(tab->body[t][ids[i]], post[i]);
    side[i] = PairSide{post[i].p, post[i].v, post[i].w, f[i].R, f[i].Iwinv};
    load2(dvw, dvb[i], dwb[i], ids[i], e, Bm, E);
  }
  PairSideBar sb[2] = {pairbar_zero(), pairbar_zero()};
  float mu_b = 0.f;
  const bool on = pair_adj(P, ty, side[0], side[1], dvb[0], dwb[0], dvb[1], dwb[1], sb[0], sb[1], mu_b);
  for (int i = 0; i < 2; ++i) {
    Bar r = bar_zero();
    if (on) {
      r.p = sb[i].p;
      r.v = sb[i].v;
      r.w = sb[i].w;
      frame_adj(tab->body[t][ids[i]], post[i], f[i], FrameBar{sb[i].R, sb[i].Iwinv, V(0.f, 0.f, 0.f)}, r.q);
    }
    slot_store_bar(pbar, 13 * i, ty.np, c, n, k, r);
  }
}

// Gather and kinematic adjoint: G <- cotangent of the substep's input state.
__global__ void k_adj_kinematic(const Tables* __restrict__ tab, int t, const int32_t* __restrict__ envs, int n,
                                int E, int Bm, const float* __restrict__ tape_s, const float* __restrict__ bpart,
                                const float* __restrict__ jbar, const float* __restrict__ abar,
                                const float* __restrict__ cbar, const float* __restrict__ pbar, Fields G) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = idx / n, k = idx - b * n;
  const TypeT& ty = tab->type[t];
  if (b >= ty.nb) return;
  const int e = envs[k];
  const BodyT& B = tab->body[t][b];
  Bar tot = load_bar(Fields{const_cast<float*>(bpart), const_cast<float*>(bpart) + 3 * Bm * E,
                            const_cast<float*>(bpart) + 7 * Bm * E, const_cast<float*>(bpart) + 10 * Bm * E},
                     b, e, Bm, E);
  if (B.joint >= 0) {
    slot_add_bar(jbar, 13, ty.nj, B.joint, n, k, tot);
    slot_add_bar(abar, 13, ty.nj, B.joint, n, k, tot);
  }
  for (int i = 0; i < B.nch; ++i) {
    const int j = tab->body[t][B.ch[i]].joint;
    slot_add_bar(jbar, 0, ty.nj, j, n, k, tot);
    slot_add_bar(abar, 0, ty.nj, j, n, k, tot);
  }
  for (int c = B.c0; c < B.c1; ++c) slot_add_bar(cbar, 0, ty.nc, c, n, k, tot);
  for (int i = 0; i < B.npair; ++i) {
    const int c = B.pairs[i];
    slot_add_bar(pbar, tab->pair[t][c].a == b ? 0 : 13, ty.np, c, n, k, tot);
  }
  Body pre = tape_load_state(tape_s, b, e, Bm, E);
  store_bar(G, kinematic_adj(B, pre, ty.h, tot), b, e, Bm, E);
}

// ------------------------------------------------------------ fused adjoint
// One lane per body as in the fused forward kernel. The forward substeps run
// first with their tape in LDS ([substep][TAPE_N][64 lanes] per wavefront,
// lane fastest); then the substeps run backwards, each lane computing its
// body's integrate, joint (+ actuator) and contact adjoints. The parent's
// post-kinematic state and force/torque cotangents come through the
// wavefront's exchange rows; each child's cotangent for its parent is read
// by the parent lane in child order.

// FROM_TAPE: the forward substeps are not recomputed; their tape records are
// read from the wavefront-major hbm_tape[step][sub][work item w of n_work][TAPE_N][64]
// (written by the fused forward with a tape, same work list; tstride floats
// per step) instead of the LDS tape, and T consecutive steps are
// differentiated in reverse in one pass (act and g_act [T][Am][E]), the
// state cotangent staying in registers between them. Without a tape T is 1.
// PARAMS: also the cotangents of the system parameters, per environment,
// into g_params[P_max][E] (order: mass per body, inertia per body x, y, z,
// per joint k_lin, c_lin, k_ang, c_ang, k_lim, strength per action,
// friction); the LDS tape then also keeps each body's total force.
template <int MAXDOF, bool FROM_TAPE, bool PARAMS, bool PAIRS, int REGC>
__device__ __forceinline__ void fused_vjp_run(const Tables* __restrict__ tab, const WaveWork& wk,
                                              const int32_t* __restrict__ env_list,
                                              const int32_t* __restrict__ type_off, int E, int Bm, int Am,
                                              const Fields& in, const float* __restrict__ act, const Fields& g_out,
                                              const Fields& g_in, float* __restrict__ g_act, float* lds,
                                              XchRows* X, const float* __restrict__ hbm_tape, int w, int n_work,
                                              float* __restrict__ g_params = nullptr, int p_max = 0,
                                              PairLanes* pl = nullptr, int T = 1, size_t tstride = 0) {
  constexpr int TN = PARAMS ? TAPE_N + 3 : TAPE_N;  // LDS tape rows per substep
  const int t = wk.type;
  const TypeT ty = tab->type[t];
  const int nb = ty.nb;
  const int lane = threadIdx.x & 63;
  // lanes past the last environment slot shadow the first slot's lanes (as
  // in the forward kernels: their reads stay within the wavefront's rows)
  const int per_wave = 64 / nb;
  const bool spare = lane >= per_wave * nb;
  const int slot = spare ? 0 : lane / nb;
  const int b = spare ? lane - per_wave * nb : lane - slot * nb;
  const int base = slot * nb;
  const bool live = !spare && slot < wk.count;
  const int e = env_list[type_off[t] + wk.k0 + (live ? slot : 0)];
  BodyT B = tab->body[t][b];
  const bool has_joint = B.joint >= 0;
  JointT J = tab->joint[t][has_joint ? B.joint : 0];
  const int src_parent = base + (has_joint ? J.parent : b);
  const int n_con = B.c1 - B.c0;
  ContactT Creg[REGC];  // the first REGC contact candidates in registers
#pragma unroll
  for (int k = 0; k < REGC; ++k) Creg[k] = tab->contact[t][B.c0 + (n_con > k ? k : 0)];
  pin_consts<MAXDOF>(B, J, has_joint, Creg, REGC);
  const float h = ty.h;
  if (PAIRS && ty.np > 0) pair_lanes_load(tab, t, pl, lane, nb);
  const size_t AE = (size_t)Am * E;
  // actions of the step being differentiated, the last one first
  float a[3] = {0.f, 0.f, 0.f}, raw[3] = {0.f, 0.f, 0.f};
  if (has_joint)
    for (int x = 0; x < MAXDOF; ++x) {
      raw[x] = J.act[x] >= 0 ? act[(T - 1) * AE + (size_t)J.act[x] * E + e] : 0.f;
      a[x] = clampf(raw[x], J.act_lo[x], J.act_hi[x]);
    }

  // forward substeps with their tape in LDS
  Body s = FROM_TAPE ? Body{} : load_body(in, b, e, Bm, E);
  for (int sub = 0; sub < (FROM_TAPE ? 0 : ty.substeps); ++sub) {
    float* tp = lds + sub * TN * 64 + lane;
    tp[0] = s.p.x; tp[64] = s.p.y; tp[128] = s.p.z;
    tp[192] = s.q.w; tp[256] = s.q.x; tp[320] = s.q.y; tp[384] = s.q.z;
    tp[448] = s.v.x; tp[512] = s.v.y; tp[576] = s.v.z;
    tp[640] = s.w.x; tp[704] = s.w.y; tp[768] = s.w.z;
    kinematic(B, s, h);
    // as in the forward kernel: this body's state written first, the
    // parent's rotation matrix read from the parent lane's row
    xch_put_pvw(X, lane, s);
    const m3 R = quat_to_mat(s.q);
    xch_put_rot(X, lane, s.w.z, R);
    Body P;
    m3 RP;
    xch_get_pvw_rot(X, src_parent, P, RP);
    P.q = s.q;  // unused: the joint reads the parent's orientation as RP
    Frame f = derive_inv(B, R);
    JointChild jc = joint_child<MAXDOF>(J, s, R);
    const v3 z3 = V(0.f, 0.f, 0.f);
    JointOut jo = joint_eval<MAXDOF>(J, P, RP, s, jc, a);
    if (!has_joint) jo.fc = jo.tc = jo.fp = jo.tp = jo.tpn = z3;
    // children's reactions read un-negated and subtracted (as in the forward)
    v3 cf[GATHER], ct[GATHER];
    xch_put2(X, lane, jo.fc, jo.tpn);
#pragma unroll
    for (int i = 0; i < GATHER; ++i) {
      if (i < ty.max_children) {
        const int src = base + (i < B.nch ? (int)((B.ch_packed >> (4 * i)) & 15u) : b);
        xch_get2(X, src, cf[i], ct[i]);
      }
    }
    v3 dv = z3, dw = z3;
    int cnt = 0;
    // the first REGC candidates from registers (no dynamic indexing), the rest from the table;
    // a candidate is skipped by the whole wave when it touches the ground on no lane
#pragma unroll
    for (int k = 0; k < REGC; ++k)
      if (k < ty.max_contacts && n_con > k) cnt += contact_eval(Creg[k], ty, B, s, f, dv, dw) ? 1 : 0;
    for (int c = REGC; c < n_con; ++c) cnt += contact_eval(tab->contact[t][B.c0 + c], ty, B, s, f, dv, dw) ? 1 : 0;
    v3 force = jo.fc, torque = jo.tc;
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
    if (PAIRS && ty.np > 0) pair_phase(tab, t, *pl, X, lane, b, base, s, f, dv, dw, cnt);
    tp[832] = torque.x; tp[896] = torque.y; tp[960] = torque.z;
    tp[1024] = (float)cnt;
    if (PARAMS) {
      tp[1088] = force.x;
      tp[1152] = force.y;
      tp[1216] = force.z;
    }
    potential(B, ty, s, f, force, torque);
    collision(B, s, dv, dw, cnt);
  }

  // reverse substeps
  Bar G = live ? load_bar(g_out, b, e, Bm, E) : bar_zero();
  float ga[3] = {0.f, 0.f, 0.f};
  // parameter cotangents of this lane: its body's 1/m, inertia and
  // inverse inertia, its joint's five constants and strengths, friction
  float invm_bar = 0.f, mu_bar = 0.f, Ib[3] = {0.f, 0.f, 0.f}, Iinvb[3] = {0.f, 0.f, 0.f};
  float jbar[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, gbar[3] = {0.f, 0.f, 0.f};
  // tape records from HBM one substep ahead of their use
  auto rec_at = [&](int step, int sub) {
    return hbm_tape + step * tstride + ((size_t)sub * n_work + w) * TAPE_N * 64;
  };
  float rec[17];
  if (FROM_TAPE) wtape_fetch(rec_at(T - 1, ty.substeps - 1), lane, rec);
  for (int step = T - 1; step >= 0; --step) {
    // the previous step's actions, loaded while this one is differentiated
    float raw_prev[3] = {0.f, 0.f, 0.f};
    if (has_joint && step > 0)
      for (int x = 0; x < MAXDOF; ++x)
        raw_prev[x] = J.act[x] >= 0 ? act[(step - 1) * AE + (size_t)J.act[x] * E + e] : 0.f;
    for (int sub = ty.substeps - 1; sub >= 0; --sub) {
      Body pre;
      v3 ttot, ftot = V(0.f, 0.f, 0.f);
      int n;
      if (FROM_TAPE) {
        wtape_unpack(rec, pre, ttot, n);
        if (sub > 0)
          wtape_fetch(rec_at(step, sub - 1), lane, rec);
        else if (step > 0)
          wtape_fetch(rec_at(step - 1, ty.substeps - 1), lane, rec);
      } else {
        const float* tp = lds + sub * TN * 64 + lane;
        if (PARAMS) ftot = V(tp[1088], tp[1152], tp[1216]);
        pre.p = V(tp[0], tp[64], tp[128]);
        pre.q = q4{tp[192], tp[256], tp[320], tp[384]};
        pre.v = V(tp[448], tp[512], tp[576]);
        pre.w = V(tp[640], tp[704], tp[768]);
        ttot = V(tp[832], tp[896], tp[960]);
        n = (int)tp[1024];
      }
      Body post = pre;
      kinematic(B, post, h);
      xch_put_body(X, lane, post);
      Body P = xch_get_body<Body>(X, src_parent);
      Frame f = derive_inv(B, quat_to_mat(post.q));  // the adjoint needs no world inertia
      v3 fb, tb, dvb, dwb;
      // this body's frame cotangents from every item of the substep, turned
      // into its quaternion cotangent once at the end
      FrameBar fr = framebar_zero();
      Bar tot = integrate_adj(B, ty, post, f, ttot, n, G, fb, tb, dvb, dwb, fr, ftot, invm_bar);
      xch_put2(X, lane, fb, tb);
      v3 fbP, tbP;
      xch_get2(X, src_parent, fbP, tbP);
      Bar bP = bar_zero(), bC = bar_zero();
      {
        // evaluated on every lane so that it interleaves with the contacts; a
        // root's joint gets zero cotangents, and the adjoint being linear in
        // them, every output is then exactly zero
        const v3 z3 = V(0.f, 0.f, 0.f);
        float ab[3];
        joint_eval_adj<MAXDOF>(J, P, quat_to_mat(P.q), post, f.R, a, has_joint ? fb : z3, has_joint ? tb : z3,
                               has_joint ? fbP : z3, has_joint ? tbP : z3, bP, bC, ab, fr, PARAMS ? jbar : nullptr,
                               PARAMS ? gbar : nullptr);
        for (int x = 0; x < MAXDOF; ++x) ga[x] += ab[x];
      }
      // children's cotangents for this body: reads in flight during the contact adjoints
      Bar cb[GATHER];
      xch_put_body(X, lane, bP);
#pragma unroll
      for (int i = 0; i < GATHER; ++i) {
        if (i < ty.max_children) {
          const int src = base + (i < B.nch ? (int)((B.ch_packed >> (4 * i)) & 15u) : b);
          cb[i] = xch_get_body<Bar>(X, src);
        }
      }
      auto contact_back = [&](const ContactT& C) {
        bool applied;
        Bar bc = contact_adj(C, ty, B, post, f, dvb, dwb, applied, fr, invm_bar, mu_bar);
        if (applied) bar_add(tot, bc);
      };
#pragma unroll
      for (int k = 0; k < REGC; ++k)
        if (k < ty.max_contacts && n_con > k) contact_back(Creg[k]);
      for (int c = REGC; c < n_con; ++c) contact_back(tab->contact[t][B.c0 + c]);
      if (PAIRS && ty.np > 0) pair_phase_adj(tab, t, *pl, b, base, post, f, dvb, dwb, tot, fr, invm_bar, mu_bar);
      bar_add(tot, bC);
      if (PARAMS) {
        // the principal moments' cotangent from the gyroscopic term (body
        // frame, integrate_adj), and Iwinv = R diag(1/I) R^T: d/d(1/I_k) =
        // r_k^T S_bar r_k (r_k column k of R; an off-diagonal cotangent
        // already holds both of its entries)
        Ib[0] += fr.Ib.x;
        Ib[1] += fr.Ib.y;
        Ib[2] += fr.Ib.z;
        for (int k = 0; k < 3; ++k) {
          const v3 r = col(f.R, k);
          auto quad = [&](const s3& S) {
            return S.xx * r.x * r.x + S.yy * r.y * r.y + S.zz * r.z * r.z + S.xy * r.x * r.y + S.xz * r.x * r.z +
                   S.yz * r.y * r.z;
          };
          Iinvb[k] += quad(fr.Iwinvb);
        }
      }
      frame_adj(B, post, f, fr, tot.q);
#pragma unroll
      for (int i = 0; i < GATHER; ++i)
        if (i < B.nch) bar_add(tot, cb[i]);
      for (int i = GATHER; i < ty.max_children; ++i) {
        const int src = base + (i < B.nch ? (int)((B.ch_packed >> (4 * i)) & 15u) : b);
        Bar x = xch_get_body<Bar>(X, src);
        if (i < B.nch) bar_add(tot, x);
      }
      G = kinematic_adj(B, pre, h, tot);
    }
    // this step's action cotangents (zero where the action was clamped)
    if (live) {
      float* ga_t = g_act + step * AE;
      if (has_joint)
        for (int x = 0; x < MAXDOF; ++x)
          if (x < J.dof && J.act[x] >= 0)
            ga_t[(size_t)J.act[x] * E + e] = (raw[x] >= J.act_lo[x] && raw[x] <= J.act_hi[x]) ? ga[x] : 0.f;
      if (b == 0)
        for (int x = ty.na; x < Am; ++x) ga_t[(size_t)x * E + e] = 0.f;
    }
    if (has_joint)
      for (int x = 0; x < MAXDOF; ++x) {
        raw[x] = raw_prev[x];
        a[x] = clampf(raw[x], J.act_lo[x], J.act_hi[x]);
        ga[x] = 0.f;
      }
  }
  if (live) {
    store_bar(g_in, G, b, e, Bm, E);
    for (int pb = nb + b; pb < Bm; pb += nb) zero_body(g_in, pb, e, Bm, E);
  }
  if (PARAMS) {
    // friction: summed over the environment's lanes (all lanes take part in the permutes)
    float mu_env = 0.f;
    for (int i = 0; i < nb; ++i) mu_env += shfl(mu_bar, base + i);
    if (live) {
      const int nj = ty.nj, np = 4 * nb + 5 * nj + ty.na + 1;
      g_params[(size_t)b * E + e] = -invm_bar * B.inv_m * B.inv_m;  // m = 1 / inv_m
      for (int k = 0; k < 3; ++k)
        g_params[(size_t)(nb + 3 * b + k) * E + e] = Ib[k] - Iinvb[k] * B.Iinv[k] * B.Iinv[k];
      if (has_joint) {
        for (int q = 0; q < 5; ++q) g_params[(size_t)(4 * nb + q * nj + B.joint) * E + e] = jbar[q];
        for (int x = 0; x < MAXDOF; ++x)
          if (x < J.dof && J.act[x] >= 0) g_params[(size_t)(4 * nb + 5 * nj + J.act[x]) * E + e] = gbar[x];
      }
      if (b == 0) {
        g_params[(size_t)(np - 1) * E + e] = mu_env;
        for (int q = np; q < p_max; ++q) g_params[(size_t)q * E + e] = 0.f;
      }
    }
  }
}

template <bool PAIRS, bool ONE_AXIS, int REGC>
__global__ __launch_bounds__(64) void k_fused_vjp(const Tables* __restrict__ tab, const WaveWork* __restrict__ work,
                                                  int n_work, const int32_t* __restrict__ env_list,
                                                  const int32_t* __restrict__ type_off, int E, int Bm, int Am,
                                                  int smax, Fields in, const float* __restrict__ act, Fields g_out,
                                                  Fields g_in, float* __restrict__ g_act) {
  extern __shared__ float4 lds_tape[];  // [exchange rows] [body-body tables (PAIRS)] [substep tape]
  const int w = xcd_block(blockIdx.x, gridDim.x);
  if (w >= n_work) return;
  const WaveWork wk = work[w];
  XchRows* X = reinterpret_cast<XchRows*>(lds_tape);
  PairLanes* pl = PAIRS ? reinterpret_cast<PairLanes*>(X + 1) : nullptr;
  float* lds = reinterpret_cast<float*>(X + 1) + (PAIRS ? sizeof(PairLanes) / 4 : 0);
  (void)smax;
  if (ONE_AXIS || tab->type[wk.type].max_dof <= 1)
    fused_vjp_run<1, false, false, PAIRS, REGC>(tab, wk, env_list, type_off, E, Bm, Am, in, act, g_out, g_in, g_act, lds,
        X, nullptr, w, n_work, nullptr, 0, pl);
  else
    fused_vjp_run<3, false, false, PAIRS, REGC>(tab, wk, env_list, type_off, E, Bm, Am, in, act, g_out, g_in, g_act, lds,
        X, nullptr, w, n_work, nullptr, 0, pl);
}

// The adjoint of one step with the cotangents of the system parameters.
template <bool PAIRS, bool ONE_AXIS, int REGC>
__global__ __launch_bounds__(64) void k_fused_vjp_params(const Tables* __restrict__ tab,
                                                         const WaveWork* __restrict__ work, int n_work,
                                                         const int32_t* __restrict__ env_list,
                                                         const int32_t* __restrict__ type_off, int E, int Bm, int Am,
                                                         Fields in, const float* __restrict__ act, Fields g_out,
                                                         Fields g_in, float* __restrict__ g_act,
                                                         float* __restrict__ g_params, int p_max) {
  extern __shared__ float4 lds_tape[];  // [exchange rows] [body-body tables (PAIRS)] [substep tape]
  const int w = xcd_block(blockIdx.x, gridDim.x);
  if (w >= n_work) return;
  const WaveWork wk = work[w];
  XchRows* X = reinterpret_cast<XchRows*>(lds_tape);
  PairLanes* pl = PAIRS ? reinterpret_cast<PairLanes*>(X + 1) : nullptr;
  float* lds = reinterpret_cast<float*>(X + 1) + (PAIRS ? sizeof(PairLanes) / 4 : 0);
  if (ONE_AXIS || tab->type[wk.type].max_dof <= 1)
    fused_vjp_run<1, false, true, PAIRS, REGC>(tab, wk, env_list, type_off, E, Bm, Am, in, act, g_out, g_in, g_act, lds,
                                         X, nullptr, w, n_work, g_params, p_max, pl);
  else
    fused_vjp_run<3, false, true, PAIRS, REGC>(tab, wk, env_list, type_off, E, Bm, Am, in, act, g_out, g_in, g_act, lds,
                                         X, nullptr, w, n_work, g_params, p_max, pl);
}

// The adjoint of T consecutive steps from their forward tape in HBM (no
// recompute; LDS holds only the exchange rows and body-body tables), the
// last step first.
template <bool PAIRS, bool ONE_AXIS, int REGC>
__global__ __launch_bounds__(64) void k_fused_vjp_tape(const Tables* __restrict__ tab,
                                                       const WaveWork* __restrict__ work, int n_work,
                                                       const int32_t* __restrict__ env_list,
                                                       const int32_t* __restrict__ type_off, int E, int Bm, int Am,
                                                       const float* __restrict__ tape, size_t tstride, int T,
                                                       const float* __restrict__ act, Fields g_out, Fields g_in,
                                                       float* __restrict__ g_act) {
  extern __shared__ float4 lds_xch[];  // [exchange rows] [body-body tables (PAIRS)]
  const int w = xcd_block(blockIdx.x, gridDim.x);
  if (w >= n_work) return;
  const WaveWork wk = work[w];
  const Fields none{nullptr, nullptr, nullptr, nullptr};
  XchRows* X = reinterpret_cast<XchRows*>(lds_xch);
  PairLanes* pl = PAIRS ? reinterpret_cast<PairLanes*>(X + 1) : nullptr;
  if (ONE_AXIS || tab->type[wk.type].max_dof <= 1)
    fused_vjp_run<1, true, false, PAIRS, REGC>(tab, wk, env_list, type_off, E, Bm, Am, none, act, g_out, g_in, g_act,
        nullptr, X, tape, w, n_work, nullptr, 0, pl, T, tstride);
  else
    fused_vjp_run<3, true, false, PAIRS, REGC>(tab, wk, env_list, type_off, E, Bm, Am, none, act, g_out, g_in, g_act,
        nullptr, X, tape, w, n_work, nullptr, 0, pl, T, tstride);
}

// Whether a type of the batch has body-body contact candidates: the kernels
// with the body-body phases are launched for such batches only.
bool any_pairs(const LaunchCtx& c) {
  for (int t = 0; t < c.n_types; ++t)
    if (c.host_tab->type[t].np > 0) return true;
  return false;
}

// Whether every type of the batch has joints of at most one axis: such
// batches take the kernels compiled for that path alone (fewer registers).
bool all_one_axis(const LaunchCtx& c) {
  for (int t = 0; t < c.n_types; ++t)
    if (c.host_tab->type[t].max_dof > 1) return false;
  return true;
}

// Whether a type of the batch has a body with more contact candidates than
// the default held in registers: one-axis such batches take the kernels
// holding 8.
bool many_contacts(const LaunchCtx& c) {
  for (int t = 0; t < c.n_types; ++t)
    if (c.host_tab->type[t].max_contacts > REG_CONTACTS) return true;
  return false;
}

}  // namespace

// Launches kernel template K<PAIRS, ONE_AXIS, REGC> with ONE_AXIS and REGC from
// the batch (`c` in scope); the remaining arguments are hipLaunchKernelGGL's.
// Eight contact candidates are held in registers only for one-axis batches:
// with three-axis joints the adjoint already fills the registers and the six
// more candidates spill (a mixed batch's segment adjoint measured 774 us with
// eight, 626 us with two), while a one-axis manipulator gains (388 -> 346 us).
#define LAUNCH_AXES(K, PAIRS, ...)                                     \
  do {                                                                 \
    const bool one_ = all_one_axis(c);                                 \
    if (one_ && many_contacts(c))                                      \
      hipLaunchKernelGGL((K<PAIRS, true, 8>), __VA_ARGS__);            \
    else if (one_)                                                     \
      hipLaunchKernelGGL((K<PAIRS, true, REG_CONTACTS>), __VA_ARGS__); \
    else                                                               \
      hipLaunchKernelGGL((K<PAIRS, false, REG_CONTACTS>), __VA_ARGS__); \
  } while (0)

size_t vjp_workspace_bytes(const Tables& tab, int n_types, const int* type_cnt, int E, int Bm) {
  size_t smax = 1;
  size_t per_type = 0;
  for (int t = 0; t < n_types; ++t) {
    smax = std::max(smax, (size_t)tab.type[t].substeps);
    size_t nt = std::max(type_cnt[t], 1);
    per_type += nt * (26 * (size_t)std::max(tab.type[t].nj, 1) * 2 + 13 * (size_t)std::max(tab.type[t].nc, 1) +
                      26 * (size_t)tab.type[t].np);
  }
  const size_t nbe = (size_t)Bm * std::max(E, 1);
  return ((smax * TAPE_N + 13 + 13 + 6 + 6) * nbe + per_type + 64) * sizeof(float);
}

int vjp_reserve(VjpWork& w, const Tables& tab, int n_types, const int* type_cnt, int E, int Bm) {
  const size_t need = vjp_workspace_bytes(tab, n_types, type_cnt, E, Bm) / sizeof(float);
  if (w.buf && w.bytes >= need * sizeof(float)) return 0;
  vjp_free(w);
  if (hipMalloc(&w.buf, need * sizeof(float)) != hipSuccess) {
    w.buf = nullptr;
    w.bytes = 0;
    return -5;
  }
  w.bytes = need * sizeof(float);
  return 0;
}

// Workspace of the adjoint for callers that cannot allocate
// (brax_step_vjp_noalloc): a device array of fixed size in the library's code
// object, one copy per GPU, held until the process ends. Host code never
// passes `scratch` itself to a kernel (on the host the name stands for a
// host-side shadow, not a device address): noalloc_init looks up the
// device's own address once per device and every use goes through it.
static __device__ __align__(256) float scratch[NOALLOC_WORKSPACE_BYTES / sizeof(float)];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {nullptr};
}  // namespace

int noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return -1;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return 0;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) return -1;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
  g_scratch_ptr[device] = static_cast<float*>(p);
  return 0;
}

float* noalloc_workspace(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

void vjp_free(VjpWork& w) {
  if (w.buf) (void)hipFree(w.buf);
  w.buf = nullptr;
  w.bytes = 0;
}

size_t vjp_lds_bytes(const Tables& tab, int n_types, bool params) {
  size_t smax = 1;
  bool pairs = false;
  for (int t = 0; t < n_types; ++t) {
    smax = std::max(smax, (size_t)tab.type[t].substeps);
    pairs = pairs || tab.type[t].np > 0;
  }
  return sizeof(XchRows) + smax * (TAPE_N + (params ? 3 : 0)) * 64 * sizeof(float) + (pairs ? sizeof(PairLanes) : 0);
}

hipError_t launch_vjp_params(const LaunchCtx& c, const VjpSched& sched, Fields in, const float* act, Fields g_out,
                             Fields g_in, float* g_act, float* g_params, int p_max, hipStream_t s) {
  if (sched.n_work == 0) return hipSuccess;
  size_t smax = 1;
  for (int t = 0; t < c.n_types; ++t) smax = std::max(smax, (size_t)c.host_tab->type[t].substeps);
  const size_t lds = sizeof(XchRows) + smax * (TAPE_N + 3) * 64 * sizeof(float);
  if (any_pairs(c))
    LAUNCH_AXES(k_fused_vjp_params, true, dim3(sched.n_work), dim3(64), lds + sizeof(PairLanes), s, c.tab, sched.work,
                sched.n_work, c.env_list, c.type_off, c.E, c.Bm, c.Am, in, act, g_out, g_in, g_act, g_params, p_max);
  else
    LAUNCH_AXES(k_fused_vjp_params, false, dim3(sched.n_work), dim3(64), lds, s, c.tab, sched.work, sched.n_work,
                c.env_list, c.type_off, c.E, c.Bm, c.Am, in, act, g_out, g_in, g_act, g_params, p_max);
  return hipGetLastError();
}

hipError_t launch_vjp_tape(const LaunchCtx& c, const VjpSched& sched, const float* tape, size_t tstride, int T,
                           const float* act, Fields g_out, Fields g_in, float* g_act, hipStream_t s) {
  if (sched.n_work == 0 || T <= 0) return hipSuccess;
  if (any_pairs(c))
    LAUNCH_AXES(k_fused_vjp_tape, true, dim3(sched.n_work), dim3(64), sizeof(XchRows) + sizeof(PairLanes), s, c.tab, sched.work,
                sched.n_work, c.env_list, c.type_off, c.E, c.Bm, c.Am, tape, tstride, T, act, g_out, g_in, g_act);
  else
    LAUNCH_AXES(k_fused_vjp_tape, false, dim3(sched.n_work), dim3(64), sizeof(XchRows), s, c.tab, sched.work, sched.n_work,
                c.env_list, c.type_off, c.E, c.Bm, c.Am, tape, tstride, T, act, g_out, g_in, g_act);
  return hipGetLastError();
}

hipError_t launch_vjp(const LaunchCtx& c, VjpWork& w, const VjpSched& sched, Fields in, const float* act,
                      Fields g_out, Fields g_in, float* g_act, bool plain, hipStream_t s) {
  const int E = c.E, Bm = c.Bm;
  const size_t nbe = (size_t)Bm * E;
  size_t smax = 1;
  for (int t = 0; t < c.n_types; ++t) smax = std::max(smax, (size_t)c.host_tab->type[t].substeps);
  float* tape = w.buf;
  float* p = tape + smax * TAPE_N * nbe;
  Fields fout{p, p + 3 * nbe, p + 7 * nbe, p + 10 * nbe};
  p += 13 * nbe;
  float* bpart = p;
  p += 13 * nbe;
  float* ftb = p;
  p += 6 * nbe;
  float* dvw = p;
  p += 6 * nbe;
  if (!plain) {
    // one wavefront per block; its tape lives in LDS
    const size_t lds = sizeof(XchRows) + smax * TAPE_N * 64 * sizeof(float);
    if (sched.n_work == 0) return hipSuccess;
    if (any_pairs(c))
      LAUNCH_AXES(k_fused_vjp, true, dim3(sched.n_work), dim3(64), lds + sizeof(PairLanes), s, c.tab, sched.work,
                  sched.n_work, c.env_list, c.type_off, E, Bm, c.Am, (int)smax, in, act, g_out, g_in, g_act);
    else
      LAUNCH_AXES(k_fused_vjp, false, dim3(sched.n_work), dim3(64), lds, s, c.tab, sched.work, sched.n_work,
                  c.env_list, c.type_off, E, Bm, c.Am, (int)smax, in, act, g_out, g_in, g_act);
    return hipGetLastError();
  }
  if (c.Am > 0) {
    const size_t na = (size_t)c.Am * E;
    hipLaunchKernelGGL(k_fill_f32, dim3(cdiv((long)na, TB)), dim3(TB), 0, s, g_act, na, 0.f);
  }
  // 1. forward with tape (plain per-phase kernels)
  hipError_t err = launch_plain_step(c, in, fout, act, sched.jslot, sched.cslot, false, s, tape);
  if (err != hipSuccess) return err;
  // 2. reverse, type by type
  for (int t = 0; t < c.n_types; ++t) {
    const int n = c.type_cnt_h[t];
    if (n == 0) continue;
    const TypeT& ty = c.host_tab->type[t];
    const int32_t* envs = c.env_list + c.type_off_h[t];
    const size_t nj = std::max(ty.nj, 1), nc = std::max(ty.nc, 1);
    float* jbar = p;
    float* abar = jbar + 26 * nj * n;
    float* cbar = abar + 26 * nj * n;
    float* pbar = cbar + 13 * nc * n;
    p = pbar + 26 * (size_t)ty.np * n;
    hipLaunchKernelGGL(k_adj_init, dim3(cdiv((long)Bm * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, E, Bm, g_out,
                       g_in);
    for (int sub = ty.substeps - 1; sub >= 0; --sub) {
      const float* tape_s = tape + (size_t)sub * TAPE_N * nbe;
      hipLaunchKernelGGL(k_adj_integrate, dim3(cdiv((long)ty.nb * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, E, Bm,
                         tape_s, g_in, bpart, ftb, dvw);
      if (ty.nj > 0) {
        if (ty.max_dof <= 1) {
          hipLaunchKernelGGL(k_adj_joint<1>, dim3(cdiv((long)ty.nj * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, E,
                             Bm, tape_s, ftb, jbar);
          hipLaunchKernelGGL(k_adj_actuator<1>, dim3(cdiv((long)ty.nj * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n,
                             E, Bm, tape_s, ftb, act, abar, g_act);
        } else {
          hipLaunchKernelGGL(k_adj_joint<3>, dim3(cdiv((long)ty.nj * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, E,
                             Bm, tape_s, ftb, jbar);
          hipLaunchKernelGGL(k_adj_actuator<3>, dim3(cdiv((long)ty.nj * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n,
                             E, Bm, tape_s, ftb, act, abar, g_act);
        }
      }
      if (ty.nc > 0)
        hipLaunchKernelGGL(k_adj_contact, dim3(cdiv((long)ty.nc * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, E, Bm,
                           tape_s, dvw, cbar);
      if (ty.np > 0)
        hipLaunchKernelGGL(k_adj_pair, dim3(cdiv((long)ty.np * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, E, Bm,
                           tape_s, dvw, pbar);
      hipLaunchKernelGGL(k_adj_kinematic, dim3(cdiv((long)ty.nb * n, TB)), dim3(TB), 0, s, c.tab, t, envs, n, E, Bm,
                         tape_s, bpart, jbar, abar, cbar, pbar, g_in);
      if ((err = hipGetLastError()) != hipSuccess) return err;
    }
  }
  return hipGetLastError();
}

}  // namespace bx
