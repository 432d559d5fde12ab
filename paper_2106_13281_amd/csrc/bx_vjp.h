// Adjoint (vector-Jacobian product) of one step: workspace and launcher.
#pragma once
#include "bx_internal.h"

namespace bx {

// Device workspace of the adjoint: forward tape, per-body partial
// cotangents and per-joint/contact slots. Grown on demand, owned by the sys.
struct VjpWork {
  size_t bytes = 0;
  float* buf = nullptr;
};

// What the forward recompute needs from the sys: the fused schedule and the
// plain path's per-type slots.
struct VjpSched {
  const WaveWork* work;
  int n_work;
  int waves_per_block;
  float* const* jslot;
  float* const* cslot;
};

// On-chip memory (LDS) per wavefront of the recomputing fused adjoint: its
// forward tape of every substep (TAPE_N floats per lane, 3 more with the
// parameter cotangents) plus the body-body candidate lists of batches that
// have them.
size_t vjp_lds_bytes(const Tables& tab, int n_types, bool params);
// The largest LDS allocation of one workgroup on gfx950 (160 KiB), the limit
// a host-only handle reports.
constexpr size_t LDS_LIMIT_GFX950 = 160 * 1024;

// Bytes of device workspace the per-phase adjoint of a batch needs.
size_t vjp_workspace_bytes(const Tables& tab, int n_types, const int* type_cnt, int E, int Bm);
// 0 or BRAX_E_NOMEM.
int vjp_reserve(VjpWork& w, const Tables& tab, int n_types, const int* type_cnt, int E, int Bm);
void vjp_free(VjpWork& w);
// The fixed device workspace of brax_step_vjp_noalloc (64 MiB per GPU).
constexpr size_t NOALLOC_WORKSPACE_BYTES = size_t(64) << 20;
// With `device` current: look up (once per device) the device address of the
// fixed workspace. 0, or -1 when the lookup fails.
int noalloc_init(int device);
// That address (nullptr before noalloc_init succeeded on the device).
float* noalloc_workspace(int device);
// g_in <- d(step)/d(in)^T g_out, g_act <- d(step)/d(act)^T g_out (both overwritten).
hipError_t launch_vjp(const LaunchCtx& c, VjpWork& w, const VjpSched& sched, Fields in, const float* act,
                      Fields g_out, Fields g_in, float* g_act, bool plain, hipStream_t s);
// The adjoint with the cotangents of the system parameters, per environment,
// g_params[p_max][E] (see brax_step_vjp_params for the order).
hipError_t launch_vjp_params(const LaunchCtx& c, const VjpSched& sched, Fields in, const float* act, Fields g_out,
                             Fields g_in, float* g_act, float* g_params, int p_max, hipStream_t s);
// The same adjoint, over T consecutive steps (the last first), from their
// wavefront-major forward tape [T][Smax][n_work][TAPE_N][64] (tstride floats
// per step; written by the fused forward with the same work list), without
// recomputing the steps: act and g_act [T][Am][E].
hipError_t launch_vjp_tape(const LaunchCtx& c, const VjpSched& sched, const float* tape, size_t tstride, int T,
                           const float* act, Fields g_out, Fields g_in, float* g_act, hipStream_t s);

}  // namespace bx
