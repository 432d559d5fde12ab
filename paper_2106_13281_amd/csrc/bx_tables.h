// Per-system constant tables, packed on the host and read by the kernels.
//
// One table set per system type of a batch; a type is one system
// description (bodies, joints, actuators, colliders of Appendix A plus the
// engine constants). Everything here is immutable during stepping.
#pragma once
#include <cstddef>
#include <cstdint>

namespace bx {

constexpr int MAXT = 8;    // system types per batch
constexpr int MAXB = 16;   // bodies per system
constexpr int MAXJ = 16;   // joints per system
constexpr int MAXC = 96;   // ground-contact candidates per system
constexpr int MAXA = 48;   // actions per system
constexpr int MAXCH = 8;   // children per body
constexpr int MAXP = 32;   // body-body contact candidates per system
constexpr int MAXPI = 16;  // body-body candidates one body takes part in
constexpr int MAXH = 8;    // body-body candidates one lane evaluates (fused kernels)
constexpr int MAXR = 8;    // shares of one side one body collects per evaluation slot
// body-body candidate kinds: the first body's core feature against the second's
enum PairKind : int32_t { PK_PP = 0, PK_PS = 1, PK_SP = 2, PK_SS = 3, PK_PB = 4, PK_BP = 5, PK_SB = 6, PK_BS = 7 };

struct TypeT {
  int32_t nb, nj, nc, na, ndof, substeps;
  int32_t max_dof;         // largest joint DOF (1..3; 0 without joints)
  int32_t max_children;    // largest child count of a body
  int32_t max_contacts;    // largest contact-candidate count of a body
  int32_t np;              // body-body contact candidates
  int32_t max_handled;     // largest count of candidates one lane evaluates
  int32_t recv_na[MAXH];   // per evaluation slot: largest count of first-body shares one body collects
  int32_t recv_nb[MAXH];   // the same for second-body shares
  float dt, h;             // step and substep length (s)
  float beta_h;            // Baumgarte factor over h (1/s)
  float one_plus_e;        // 1 + restitution
  float mu;                // Coulomb friction
  float clearance;         // reset height of the lowest contact point (m)
  float g[3];              // gravity (m/s^2)
  int32_t frozen;          // 1 if some body of the type has a frozen axis
  // the fused forward without a tape spreads the contact candidates of a
  // body with more than two over extra lanes that hold copies of its state
  // (contact lanes): lanes per environment there, the largest count of
  // candidates one such lane evaluates, and the largest lane group of a body
  int32_t nl, max_lc, max_ng;
};

struct BodyT {
  float m, inv_m;
  float I[3], Iinv[3];     // principal moments, body frame
  float free_p[3], free_r[3];  // 1 = world axis integrates, 0 = frozen
  int32_t joint;           // joint whose child this body is; -1 for a root
  int32_t parent;          // parent body; -1 for a root
  int32_t c0, c1;          // contact candidates [c0, c1) belong to this body
  int32_t nch;             // number of child bodies
  int32_t ch[MAXCH];       // child bodies (ascending joint order)
  uint32_t ch_packed;      // the same, 4 bits per child (child i in bits 4i..4i+3)
  int32_t root;            // root body of this body's tree
  int32_t has_pos;         // root with a given reset position
  float pos0[3];           // that position
  int32_t npair;           // body-body candidates this body takes part in (as first or second)
  int32_t pairs[MAXPI];    // their indices, ascending
  // fused kernels: each candidate is evaluated on the lane of some body of
  // the system (its handler), which leaves both bodies' shares in registers
  // for their lanes to collect in the same evaluation slot
  int32_t nh;              // candidates this body's lane evaluates
  int32_t hp[MAXH];        // their indices (evaluation slots 0 .. nh-1)
  int32_t nra[MAXH];       // per slot: shares this body collects as a candidate's first body
  uint32_t recva[MAXH];    // per slot: the handler bodies of those shares, 4 bits each
  int32_t nrb[MAXH];       // the same as a candidate's second body
  uint32_t recvb[MAXH];
  // lanes of the fused forward without a tape: entries nb .. nl-1 are contact
  // lanes, copies of their body's entry that evaluate candidates [l0, l1)
  // (a body lane evaluates its first ones); body_of: the body whose state the
  // lane holds; its group: the lanes holding that body (body lane first),
  // 4 bits each, whose contact sums every lane of the group adds in order
  int32_t l0, l1;
  int32_t body_of;
  int32_t ng;
  uint32_t grp_packed;
};

struct JointT {
  int32_t parent, child, dof, dof0;  // dof0: first DOF index of this joint
  float ap[3], ac[3];      // anchor in parent / child body frame
  float FP[9], FC[9];      // joint frame (row-major rotation) in parent / child body frame
  float k_lin, c_lin, k_ang, c_ang, k_lim;
  float lo[3], hi[3];      // angle limits (rad)
  float gear[3];           // actuator strength per axis (0 = not actuated)
  int32_t act[3];          // action index per axis (-1 = not actuated)
  float act_lo[3], act_hi[3];  // action clip range: [-1, 1] (torque) or the joint's range (target angle)
  float act_pd[3];         // 1 for a target-angle actuator (torque gear (a - theta)), 0 for torque (gear a)
  float def_angle[3];      // reset angle per axis
};

struct ContactT {
  int32_t body;
  float l[3];              // centre in the body frame
  float rho;               // radius (0 for box corners)
};

// One body-body contact candidate: the first body's core feature (a point
// a0, a segment a0-a1, or a box with centre a0, rotation aR box to body and
// half extents ah) with radius ra, the same for the second body; inverse
// mass im (0 when all translations are frozen) and whether rotations
// respond (0 when all are frozen) of each body.
struct PairT {
  int32_t a, b, kind, rot_a, rot_b;
  int32_t box_rot;         // the box collider is rotated in its body (aR / bR not the identity)
  int32_t pad;
  float reach;             // no contact while the two body origins are farther apart than this
  // the bound test of the fused forward: the line feature lo + u ld (u in
  // [0, 1]; a segment, or a point with ld = 0) in the frame of the body
  // named by kc[3] (1: b, 0: a) against the ball around kc in the other
  // body's frame; no contact while the line's distance from kc exceeds
  // sqrt(lo[3]) (the radii, the other feature's extent from kc, a margin).
  // 16-byte aligned within the struct (offset 32; the size is a multiple of 16)
  float lo[4], ld[4], kc[4];
  float a0[3], a1[3], ra;
  float b0[3], b1[3], rb;
  float ah[3], bh[3];
  float aR[9], bR[9];
  float im_a, im_b;
};

// the fused kernels read lo, ld and kc as 16-byte vectors from their LDS copy
static_assert(offsetof(PairT, lo) % 16 == 0 && offsetof(PairT, ld) % 16 == 0 && offsetof(PairT, kc) % 16 == 0 &&
                  sizeof(PairT) % 16 == 0,
              "PairT layout");

struct Tables {
  TypeT type[MAXT];
  BodyT body[MAXT][MAXB];
  JointT joint[MAXT][MAXJ];
  ContactT contact[MAXT][MAXC];
  PairT pair[MAXT][MAXP];
  int32_t topo[MAXT][MAXB];  // bodies, every parent before its children
};

// Environment-layer parameters of one system type (reward, termination).
struct EnvT {
  int32_t root;            // body whose x progress is rewarded and whose height decides termination
  float forward_weight;    // reward per m/s of root x velocity over the step
  float healthy_reward;    // reward while the root height is within [z_min, z_max]
  float ctrl_cost;         // cost per unit of sum_k a_k^2 (actions as given)
  float z_min, z_max;      // healthy root heights (m)
};

// One wavefront's share of the fused launch: `count` environments of one
// type, taken from that type's environment list starting at `k0`.
struct WaveWork {
  int32_t type, k0, count, pad;
};

}  // namespace bx
