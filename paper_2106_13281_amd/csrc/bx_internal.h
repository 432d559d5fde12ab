// Internal declarations shared by the host API and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "bx_tables.h"

namespace bx {

constexpr int TAPE_N = 17;  // floats per body per substep in the forward tape

struct Fields {
  float* pos;
  float* rot;
  float* vel;
  float* ang;
};

// ------------------------------------------------------------ host model
struct ColliderD {
  int kind;  // 0 sphere, 1 capsule, 2 box
  double pos[3];
  double R[9];
  double radius, length, half[3];
};
struct BodyD {
  std::string name;
  double mass;
  double I[3];
  double free_p[3], free_r[3];
  bool has_pos;
  double pos[3];
  std::vector<ColliderD> cols;
};
struct JointD {
  std::string name;
  int parent, child, dof;
  double ap[3], ac[3], FP[9], FC[9];
  double k_lin, c_lin, k_ang, c_ang, k_lim;
  double lo[3], hi[3];
};
struct ActD {
  int joint, axis;
  double gear;
  int mode;  // 0 torque, 1 target angle
};
struct ContactD {
  int body;
  double l[3];
  double rho;
};
// Body-body contact candidate between two declared bodies: each side is a
// core feature in its body's frame (point a0, segment a0-a1, or box with
// centre a0, rotation aR and half extents ah) with a radius.
struct PairD {
  int a, b, kind;  // PairKind
  int handler;     // the body whose lane evaluates it in the fused kernels (any body of the system)
  double a0[3], a1[3], ra, ah[3], aR[9];
  double b0[3], b1[3], rb, bh[3], bR[9];
};
struct SystemDesc {
  int substeps;
  double dt, g[3], beta, elasticity, mu, clearance;
  std::vector<BodyD> bodies;
  std::vector<JointD> joints;
  std::vector<ActD> actions;
  std::vector<ContactD> contacts;
  std::vector<PairD> pairs;
  int ndof;
};

// Parse and validate one description. Returns 0 or a BRAX_E_* code with a
// message in `err` (parse errors carry line:col).
int build_system(const char* text, SystemDesc& out, std::string& err);

// Fill the tables of type `t` from a description.
void pack_type(const SystemDesc& d, Tables& tab, int t);

// ------------------------------------------------------------ launchers
// All launch on `stream` and return the hipError_t of the launch.
struct LaunchCtx {
  const Tables* tab;            // device tables
  const Tables* host_tab;       // host copy (sizes, counts)
  int E, Bm, Am;
  int n_types;
  const int32_t* env_type;      // device [E]
  const int32_t* env_list;      // device, grouped by type
  const int32_t* type_off;      // device [n_types]
  int type_off_h[MAXT], type_cnt_h[MAXT];
  uint8_t* nonfinite;           // device [E]
};

hipError_t launch_default_qp(const LaunchCtx& c, const float* angles, const float* root_off, Fields out,
                             hipStream_t s);
// tape (nullable): also write the wavefront-major tape
// [T][smax][n_work][TAPE_N][64] (see bx_access.h).
hipError_t launch_fused(const LaunchCtx& c, const WaveWork* work, int n_work, int waves_per_block, Fields in,
                        Fields out, const float* acts, int T, int save_every, Fields traj, bool flags, hipStream_t s,
                        float* tape = nullptr, int smax = 0);
// Plain path: one step (all substeps) of every type; acts points at this
// step's [Am][E] actions. jslot/cslot: per-type scratch. tape (nullable):
// per substep [TAPE_N][Bm][E] records for the adjoint, see bx_access.h.
hipError_t launch_plain_step(const LaunchCtx& c, Fields in, Fields out, const float* act, float* const* jslot,
                             float* const* cslot, bool flags, hipStream_t s, float* tape = nullptr);
hipError_t launch_copy_state(const LaunchCtx& c, Fields in, Fields out, hipStream_t s);
// One environment step with the environment layer fused after it, in one
// launch: the fused step, then reward, done, the reset of finished
// environments and the observations [Omax][E] of the final state.
hipError_t launch_env_step(const LaunchCtx& c, const WaveWork* work, int n_work, int waves_per_block,
                           const EnvT* env, int Omax, Fields in, Fields out, const float* act, Fields reset, float* obs,
                           float* reward, uint8_t* done, bool flags, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int n, uint8_t v, hipStream_t s);

}  // namespace bx
