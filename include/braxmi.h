/* braxmi — batched maximal-coordinate rigid-body step on one MI355X (gfx950).
 *
 * The method is the physics step of Brax (arXiv 2106.13281): a scene is a set
 * of bodies in maximal coordinates whose only changing data are position,
 * orientation, velocity and angular velocity (Section 3, the QP); one step
 * `qp' = step(qp, actions)` (Section 3) runs `substeps` repetitions of
 * Algorithm 1 — kinematic integration, then joint, actuator and collider
 * updates computed from the same qp, then the potential integrator (joint and
 * actuator updates, gravity) and the collision integrator (collider updates).
 * Joints are springs (Section 7.1), contacts are velocity-level impulses with
 * Baumgarte stabilisation against the ground plane and between the colliders
 * of declared body pairs (Section 7.2), systems are
 * described in the ProtoBuf-like text of Appendix A, and the step is
 * differentiable (Sections 2 and 5.1.4).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every call returns BRAX_OK (0) or a negative BRAX_E_* code; the
 *   message of the calling thread's last failure is brax_last_error(). No
 *   C++ exception crosses this boundary. Arguments are checked on the host
 *   before anything is launched; a failed check launches nothing.
 * - Ownership: the caller owns every state, action and gradient buffer (all
 *   DEVICE pointers, FP32). The brax_sys owns its constant tables, workspace
 *   and cached HIP graphs and frees them in brax_sys_destroy.
 * - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *   Step/rollout/VJP calls are asynchronous on it. A brax_sys is used by one
 *   stream at a time: its workspace is shared by its calls. Exception:
 *   brax_rollout_tape and brax_rollout_vjp_tape with neither BRAX_GRAPH nor
 *   BRAX_NONFINITE_FLAGS use none of the handle's workspace and may run on
 *   several streams at once, on disjoint output buffers (a checkpointed
 *   backward recomputes one segment's tape while the previous one's adjoint
 *   runs).
 * - State layout (structure of arrays, environment index fastest):
 *     element (c, b, e) of a field = ptr[(c * Bmax + b) * E + e]
 *   pos, vel, ang: c in [0,3) (x, y, z; world frame, m, m/s, rad/s)
 *   rot:           c in [0,4) (w, x, y, z; unit quaternion, body to world)
 *   E = number of environments, Bmax = the largest body count over the
 *   system types of the batch. Body slots b >= B of a smaller system are
 *   ignored on input and written as zeros.
 * - Actions: act[a * E + e], a in [0, Amax); rollouts take acts[t][a][e].
 *   Each action drives one joint axis: a torque actuator clips it to
 *   [-1, 1] and applies the torque gear * action; a target-angle actuator
 *   clips it to the axis' angle range and applies gear * (action - angle).
 *   Action slots beyond a system's own count are ignored.
 * - Non-finite state is not an error: NaN/Inf propagate. With
 *   BRAX_NONFINITE_FLAGS a per-environment byte (1 = some output non-finite)
 *   is written to the buffer brax_sys_query reports.
 */
#ifndef BRAXMI_H
#define BRAXMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct brax_sys brax_sys; /* opaque; owned by the library */

typedef struct {
  float* pos; /* [3][Bmax][E] */
  float* rot; /* [4][Bmax][E] */
  float* vel; /* [3][Bmax][E] */
  float* ang; /* [3][Bmax][E] */
} brax_state;

enum {
  BRAX_OK = 0,
  BRAX_E_ARG = -1,         /* null pointer, bad size, bad flag, bad index */
  BRAX_E_PARSE = -2,       /* system text does not parse; message has line:col */
  BRAX_E_MODEL = -3,       /* parses but is not a valid system (see brax_sys_create) */
  BRAX_E_DEVICE = -4,      /* a HIP call failed */
  BRAX_E_NOMEM = -5,       /* device or host allocation failed */
  BRAX_E_UNSUPPORTED = -6  /* valid request the library does not handle */
};

/* Kernel choice: BRAX_FUSED (or neither bit: the default) runs one
 * persistent fused kernel, BRAX_PLAIN one launch per phase per substep;
 * both bits together are BRAX_E_ARG. */
enum {
  BRAX_PLAIN = 1,          /* one launch per phase per substep (baseline) */
  BRAX_FUSED = 2,          /* one persistent fused kernel (the default) */
  BRAX_GRAPH = 4,          /* capture the launch(es) in a HIP graph and replay it; the graph is
                              cached per call kind and set of buffer addresses. A call that is a
                              single kernel launch (the fused paths) is launched directly, since
                              replaying a one-node graph costs more than the launch itself */
  BRAX_NONFINITE_FLAGS = 8 /* also write per-environment non-finite flags */
};

#define BRAX_MAX_TYPES 8
#define BRAX_MAX_BODIES 16
#define BRAX_MAX_JOINTS 16
#define BRAX_MAX_CONTACTS 96
#define BRAX_MAX_ACTIONS 48

typedef struct {
  int32_t n_envs, n_types, b_max, a_max, d_max;
  int32_t type_envs[BRAX_MAX_TYPES];   /* environments of each type */
  int32_t n_bodies[BRAX_MAX_TYPES];
  int32_t n_joints[BRAX_MAX_TYPES];
  int32_t n_actions[BRAX_MAX_TYPES];
  int32_t n_dof[BRAX_MAX_TYPES];
  int32_t n_contacts[BRAX_MAX_TYPES];
  int32_t substeps[BRAX_MAX_TYPES];
  float dt[BRAX_MAX_TYPES];
  int32_t device;                      /* -1 for a host-only (validate) handle */
  uint8_t* nonfinite;                  /* device [E] flags (BRAX_NONFINITE_FLAGS) */
  int64_t tape_step_floats;            /* floats per step of a brax_rollout_tape tape */
  int32_t n_params[BRAX_MAX_TYPES];    /* system parameters per type (brax_step_vjp_params) */
  int32_t p_max;                       /* the largest of n_params */
  int32_t n_pairs[BRAX_MAX_TYPES];     /* body-body contact candidates per type */
  int64_t vjp_lds_bytes;               /* on-chip memory per wavefront of the fused brax_step_vjp */
  int64_t vjp_params_lds_bytes;        /* the same for brax_step_vjp_params */
  int64_t lds_limit;                   /* the device's per-workgroup limit (160 KiB for a host-only handle) */
  int32_t lanes_per_env[BRAX_MAX_TYPES]; /* lanes per environment of the fused forward without a tape: one
                                            per body, plus one per two further ground-contact candidates of
                                            a body with more than two (copies of its state that each
                                            evaluate two of its candidates) */
} brax_layout;

/* Build a batch of n_envs environments from n_descs system descriptions.
 * descs: host array of NUL-terminated texts in the Appendix A format
 *   (substeps, dt, gravity, bodies{name mass inertia frozen colliders position},
 *   joints{name parent child stiffness damping angular_stiffness
 *   angular_damping limit_stiffness parent_offset child_offset rotation
 *   child_rotation angle_limit{min max}...}, actuators{name joint strength
 *   torque{} | angle{}}, body_contacts{first second}, baumgarte, elasticity,
 *   friction, clearance). body_contacts declares a body pair whose colliders
 *   collide with each other: each collider is reduced to a core feature (a
 *   sphere's centre, a capsule's axis segment, a box) plus a radius, every
 *   collider of the first body is paired with every one of the second, and
 *   a capsule against a box contributes its two end spheres and its axis
 *   segment, the segment a candidate only where its point nearest the box
 *   (the deepest one where the axis passes through the box) lies strictly
 *   between its ends.
 * env_desc: host [n_envs] index of each environment's description, or NULL
 *   (all use descs[0]). Environments of one type need not be contiguous.
 * device: HIP device ordinal, or -1 to parse and validate only (no device
 *   work; the handle then only answers brax_sys_query).
 * Errors: BRAX_E_ARG (null/size), BRAX_E_PARSE (with line:col),
 *   BRAX_E_MODEL (unknown or repeated body, a body with two parents, a cycle,
 *   mass <= 0, inertia <= 0, capsule length < 2 radius, angle_limit min > max,
 *   DOF outside 1..3, a body without inertia or colliders, a body_contacts
 *   pair naming an unknown body, the same body twice or two boxes, table
 *   limits),
 *   BRAX_E_DEVICE, BRAX_E_NOMEM. On error *out is NULL. */
int brax_sys_create(const char* const* descs, int32_t n_descs, const int32_t* env_desc, int32_t n_envs,
                    int32_t device, brax_sys** out);

/* Free a batch (synchronises its device first). NULL is a no-op. */
void brax_sys_destroy(brax_sys* sys);

/* Sizes of the batch. */
int brax_sys_query(const brax_sys* sys, brax_layout* out);

/* Default angle of each DOF of one system type (radians; 0 when inside the
 * limits, else the mid-range), host out[n_dof[type]]. */
int brax_default_angles(const brax_sys* sys, int32_t type, float* out);

/* Reset pose (Section 4.1, default_qp): each tree placed in a valid joint
 * configuration. joint_angles: device [Dmax][E] per-DOF angles in radians, or
 * NULL for the defaults. root_offset: device [3][E] added to the first body's
 * position when it is a free root, or NULL. Roots without a given position are
 * first lifted so their lowest contact point is `clearance` above the ground.
 * Velocities are zero. */
int brax_default_qp(const brax_sys* sys, const float* joint_angles, const float* root_offset, brax_state* out,
                    void* stream);

/* One environment step, qp' = step(qp, act) (Section 3): `substeps`
 * repetitions of Algorithm 1 with the action held. `out` may alias `in`. */
int brax_step(const brax_sys* sys, const brax_state* in, const float* act, brax_state* out, int32_t flags,
              void* stream);

/* Adjoint of brax_step (Sections 2 and 5.1.4: gradients through the step):
 * given g_out = dL/d(out), writes g_in = dL/d(in) and g_act = dL/d(act)
 * (overwritten, not accumulated) for the same function brax_step computes.
 * The forward substeps are recomputed inside. The fused adjoint keeps their
 * tape on chip (brax_layout.vjp_lds_bytes per wavefront); a batch whose
 * tape exceeds lds_limit (many substeps) runs the per-phase adjoint of
 * BRAX_PLAIN instead, whose tape lives in the handle's device workspace. At kinks the one-sided
 * conventions are: max(0,x)' = [x > 0]; the Coulomb cap is taken when
 * cap <= stop; clamp' = 1 and clip' = 1 on the closed interval;
 * contact activation and counts have zero derivative. g_in may not alias
 * in or g_out. Body-body contacts follow the same conventions; their closest
 * features pass the gradient with the feature pair and face held (a
 * clamped closest-point parameter passes on the closed interval). */
int brax_step_vjp(const brax_sys* sys, const brax_state* in, const float* act, const brax_state* g_out,
                  brax_state* g_in, float* g_act, int32_t flags, void* stream);

/* brax_step_vjp for callers that cannot allocate device memory (code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, results and kernel choice, but the call
 * allocates nothing. Where brax_step_vjp takes the per-phase adjoint
 * (BRAX_PLAIN, or an on-chip tape beyond lds_limit), its workspace is a
 * fixed 64 MiB device array of the library, one per GPU, held until the
 * process ends, instead of the handle's workspace grown on demand; the fused
 * adjoint needs none. Every call on one GPU shares that GPU's array (which
 * keeps the last call's contents; nothing in it needs to start at zero), so
 * calls that overlap on one GPU, from any handles or streams, race: run
 * them one at a time. Errors: as brax_step_vjp; BRAX_E_UNSUPPORTED when the
 * per-phase workspace the batch needs exceeds the 64 MiB; BRAX_E_ARG for
 * BRAX_GRAPH (capture the call yourself instead). */
int brax_step_vjp_noalloc(const brax_sys* sys, const brax_state* in, const float* act, const brax_state* g_out,
                          brax_state* g_in, float* g_act, int32_t flags, void* stream);

/* T consecutive steps with acts [T][Amax][E]. With save_every > 0, the state
 * after steps save_every, 2*save_every, ... is written to traj (each field
 * [T/save_every][C][Bmax][E]); traj may be NULL when save_every == 0. The
 * final state goes to `out` (may alias `in`). T == 0 copies in to out. */
int brax_rollout(const brax_sys* sys, const brax_state* in, const float* acts, int32_t T, int32_t save_every,
                 brax_state* traj, brax_state* out, int32_t flags, void* stream);

/* brax_rollout (save_every 0) that also records what the adjoint needs of
 * every substep (Sections 3 and 5.1.4: the backward pass through the steps
 * of Algorithm 1): per body and substep, the state before the kinematic
 * update (13 floats), the total joint and actuator torque (3) and the number
 * of contacts that applied an impulse (1). tape: device, caller-owned,
 * T * brax_layout.tape_step_floats floats, step t at offset
 * t * tape_step_floats; its layout inside a step is the library's own
 * (wavefront-major, for coalesced access) and is read only by
 * brax_step_vjp_tape and brax_rollout_vjp_tape of the same sys. Fused path
 * only: BRAX_PLAIN gives BRAX_E_UNSUPPORTED. The states agree with
 * brax_rollout's up to rounding (a separately compiled kernel, whose
 * multiply-add fusions may differ); repeated calls give the same bits. */
int brax_rollout_tape(const brax_sys* sys, const brax_state* in, const float* acts, int32_t T, float* tape,
                      brax_state* out, int32_t flags, void* stream);

/* brax_step_vjp that also writes the cotangents of the system parameters
 * (Section 2: gradients through the simulation; here with respect to the
 * constants of the system description), per environment: g_params
 * [p_max][E] (device, caller-owned, overwritten), for each system type in
 * this order: mass of every body (nb), principal inertia of every body (x,
 * y, z; 3 nb), then per joint (nj each) the anchor stiffness, anchor
 * damping, angular stiffness, angular damping and limit stiffness, then the
 * strength of every action (na), then the friction coefficient (1): n_params
 * = 4 nb + 5 nj + na + 1 entries; rows beyond them are zero. The gradient of
 * a loss summed over environments sharing the parameters is the sum over
 * E. Fused path only; BRAX_E_UNSUPPORTED when brax_layout.vjp_params_lds_bytes
 * exceeds lds_limit. */
int brax_step_vjp_params(const brax_sys* sys, const brax_state* in, const float* act, const brax_state* g_out,
                         brax_state* g_in, float* g_act, float* g_params, int32_t flags, void* stream);

/* Adjoint of one step from its tape (the tape_step_floats written by
 * brax_rollout_tape of the same sys for that step, with the same actions)
 * instead of recomputing the forward substeps: the outputs and kink
 * conventions of brax_step_vjp (equal up to rounding, the forward values
 * coming from the taped kernel). g_in may not alias g_out. Fused path only. */
int brax_step_vjp_tape(const brax_sys* sys, const float* tape, const float* act, const brax_state* g_out,
                       brax_state* g_in, float* g_act, int32_t flags, void* stream);

/* Adjoint of T consecutive steps from their tape (Section 3: the backward
 * pass through a trajectory of steps), in one launch: the same results as T
 * calls of brax_step_vjp_tape from the last step to the first, each call's
 * g_in the next one's g_out, with the state cotangent held on chip between
 * steps. tape: T * tape_step_floats floats as written by brax_rollout_tape
 * of the same sys over the same acts [T][Amax][E]; g_out: cotangent of the
 * state after step T; g_in (overwritten): cotangent of the state before step
 * 0, may not alias g_out; g_acts [T][Amax][E] (device, caller-owned,
 * overwritten): the action cotangents of every step, zero where an action
 * was clamped and in rows beyond a type's actions. T == 0 copies g_out to
 * g_in. Fused path only: BRAX_PLAIN gives BRAX_E_UNSUPPORTED. */
int brax_rollout_vjp_tape(const brax_sys* sys, const float* tape, const float* acts, int32_t T,
                          const brax_state* g_out, brax_state* g_in, float* g_acts, int32_t flags, void* stream);

/* Environment layer (Section 4.2: gym-like environments; App. E: rewards
 * close to the MuJoCo gym ones without a contact cost, termination on the
 * torso height leaving a range). Per system type: */
typedef struct {
  int32_t root;          /* body whose x progress is rewarded and whose height decides termination */
  float forward_weight;  /* reward per m/s of root x velocity over the step */
  float healthy_reward;  /* reward while z_min <= root z <= z_max after the step */
  float ctrl_cost;       /* cost per unit of sum_k a_k^2 (the actions as passed) */
  float z_min, z_max;    /* healthy root heights, metres (use +-inf for none) */
} brax_env_params;

/* Set the environment-layer parameters, one entry per system type (host
 * array of n_types). Synchronous; BRAX_E_ARG for a root out of range or
 * z_min > z_max. */
int brax_env_configure(brax_sys* sys, const brax_env_params* params);

/* One environment step of every environment, on `stream`: brax_step from
 * `in` to `out`, then
 *   reward[e] = forward_weight (x_root' - x_root) / dt
 *               + healthy_reward [healthy] - ctrl_cost sum_k a_k^2,
 *   done[e]   = !healthy, healthy = z_min <= z_root' <= z_max (after the step),
 * then every finished environment's `out` state is replaced by its `reset`
 * state (all Bmax bodies), and obs [Omax][E] (Omax = 11 + 2 * d_max) is the
 * observation of `out`: z_root, q_root (4), v_root (3), w_root (3), the joint
 * angles (D, joint order, as in the joint law) and the relative angular
 * velocity (w_child - w_parent) projected on each Euler axis (D), zero-padded.
 * `out` may alias `in`; `reset` may not alias `out`. Device pointers, caller
 * owned; done is uint8. Fused path only. */
int brax_env_step(const brax_sys* sys, const brax_state* in, const float* act, const brax_state* reset,
                  brax_state* out, float* obs, float* reward, uint8_t* done, int32_t flags, void* stream);

/* Time the fused kernel's launch shapes on `stream` and keep the fastest
 * for later calls (the result does not depend on the shape). Per system
 * type, environments per wavefront from full wavefronts down, and the
 * value that gives the type about one wavefront per SIMD (tried first in a
 * batch of one type, last otherwise); wavefronts per block from one up. A
 * later shape replaces the best so far only if it is more than 1% faster,
 * so that repeated tunings of one batch settle on the same shape. */
int brax_autotune(brax_sys* sys, void* stream);

/* brax_autotune with trials on the caller's workload: each trial is a
 * T-step rollout from `in` with actions `act` ([T][A_max][E], as
 * brax_rollout), so that the shapes are compared on the states and actions
 * of use (trials from the reset pose miss how contacts and body-body
 * candidates come and go). Device pointers, caller owned, read only; the
 * trials' output goes to the library's own scratch state. BRAX_E_ARG for
 * T < 1 or a NULL field. */
int brax_autotune_on(brax_sys* sys, const brax_state* in, const float* act, int32_t T, void* stream);

/* Launch shape in use: environments per wavefront (of the first system type)
 * and wavefronts per block. */
int brax_schedule(const brax_sys* sys, int32_t* envs_per_wave, int32_t* waves_per_block);

/* Set the launch shape: envs_per_wave environments per wavefront for every
 * type (clamped to each type's maximum floor(64 / bodies); <= 0 keeps the
 * maximum) and waves_per_block in {1, 2, 4}. Results do not depend on it.
 * BRAX_E_ARG for other block shapes. */
int brax_set_schedule(brax_sys* sys, int32_t envs_per_wave, int32_t waves_per_block);

/* Copy the per-environment non-finite flags written by the last call made
 * with BRAX_NONFINITE_FLAGS to host out[n_envs] (synchronises the device). */
int brax_nonfinite(const brax_sys* sys, uint8_t* out);

/* Message of the calling thread's last failure ("" if none). Never NULL. */
const char* brax_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BRAXMI_H */
