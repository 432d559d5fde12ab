// C ABI of the library: argument checks, system tables, schedules, graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/braxmi.h"
#include "bx_internal.h"
#include "bx_vjp.h"

using namespace bx;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) return fail(BRAX_E_DEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// Keeps the caller's current device and restores it on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

// A captured graph holds the addresses of every buffer its launches use, so
// the key lists every device pointer of the call (all four fields of each
// state, the actions, tapes and outputs, the workspace); a call that differs
// in any of them captures a graph of its own.
struct GraphKey {
  int kind = 0;  // 0 step, 1 rollout, 2 adjoint, 3 rollout with tape, 4 adjoint from a tape, 5 environment
                 // step, 6 adjoint with parameters, 7 adjoint of T steps from a tape
  int flags = 0, T = 0, save_every = 0;
  std::vector<const void*> p;
  GraphKey(int kind_, int flags_, int T_, int save_every_ = 0)
      : kind(kind_), flags(flags_), T(T_), save_every(save_every_) {}
  GraphKey& add(const void* x) {
    p.push_back(x);
    return *this;
  }
  GraphKey& add(const brax_state* st) {
    for (const void* x : {(const void*)(st ? st->pos : nullptr), (const void*)(st ? st->rot : nullptr),
                          (const void*)(st ? st->vel : nullptr), (const void*)(st ? st->ang : nullptr)})
      p.push_back(x);
    return *this;
  }
  bool operator<(const GraphKey& o) const {
    return std::tie(kind, flags, T, save_every, p) < std::tie(o.kind, o.flags, o.T, o.save_every, o.p);
  }
};

struct brax_sys {
  int device = -1;
  int E = 0, n_types = 0, Bm = 0, Am = 0, Dm = 0;
  std::vector<SystemDesc> descs;
  Tables host_tab{};
  Tables* d_tab = nullptr;
  std::vector<int32_t> env_type, env_list;
  int type_off[MAXT] = {0}, type_cnt[MAXT] = {0};
  int32_t* d_env_type = nullptr;
  int32_t* d_env_list = nullptr;
  int32_t* d_type_off = nullptr;
  size_t lds_limit = LDS_LIMIT_GFX950;  // per-workgroup LDS of the device
  // fused schedule
  int envs_per_wave[MAXT] = {0};
  int waves_per_block = 1;
  std::vector<WaveWork> work;
  WaveWork* d_work = nullptr;
  // adjoint schedule: full wavefronts (its launch holds a tape in LDS, so
  // fewer wavefronts mean fewer rounds), fixed at creation
  std::vector<WaveWork> vjp_work;
  WaveWork* d_vjp_work = nullptr;
  int smax = 1;  // largest substep count of the batch's types (tape stride)
  // environment layer (brax_env_configure)
  bool env_ready = false;
  EnvT* d_env = nullptr;
  // plain scratch per type
  float* d_jslot[MAXT] = {nullptr};
  float* d_cslot[MAXT] = {nullptr};
  // adjoint workspace
  VjpWork vjp{};
  uint8_t* d_nonfinite = nullptr;
  std::map<GraphKey, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  std::set<GraphKey> direct_keys;  // BRAX_GRAPH calls whose capture held one node: launched directly

  LaunchCtx ctx() const {
    LaunchCtx c{};
    c.tab = d_tab;
    c.host_tab = &host_tab;
    c.E = E;
    c.Bm = Bm;
    c.Am = Am;
    c.n_types = n_types;
    c.env_type = d_env_type;
    c.env_list = d_env_list;
    c.type_off = d_type_off;
    for (int t = 0; t < MAXT; ++t) {
      c.type_off_h[t] = type_off[t];
      c.type_cnt_h[t] = type_cnt[t];
    }
    c.nonfinite = d_nonfinite;
    return c;
  }
};

namespace {

void free_all(brax_sys* s) {
  if (s->device >= 0) {
    DeviceGuard g(s->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : s->graphs) {
      (void)hipGraphExecDestroy(kv.second.second);
      (void)hipGraphDestroy(kv.second.first);
    }
    (void)hipFree(s->d_tab);
    (void)hipFree(s->d_env_type);
    (void)hipFree(s->d_env_list);
    (void)hipFree(s->d_type_off);
    (void)hipFree(s->d_work);
    (void)hipFree(s->d_vjp_work);
    (void)hipFree(s->d_env);
    (void)hipFree(s->d_nonfinite);
    for (int t = 0; t < MAXT; ++t) {
      (void)hipFree(s->d_jslot[t]);
      (void)hipFree(s->d_cslot[t]);
    }
    vjp_free(s->vjp);
  }
  delete s;
}

// Split every type's environments into wavefronts of envs_per_wave[t] and
// order the wavefronts heaviest first (substeps x per-lane work estimate).
std::vector<WaveWork> make_work(const brax_sys* s, const int* envs_per_wave) {
  struct Item {
    double cost;
    WaveWork w;
  };
  std::vector<Item> items;
  for (int t = 0; t < s->n_types; ++t) {
    const TypeT& ty = s->host_tab.type[t];
    int epw = envs_per_wave[t];
    double cost = ty.substeps * (150.0 + (ty.nj > 0 ? 250.0 * ty.max_dof : 0.0) + 130.0 * ty.max_contacts);
    for (int k0 = 0; k0 < s->type_cnt[t]; k0 += epw)
      items.push_back(Item{cost, WaveWork{t, k0, std::min(epw, s->type_cnt[t] - k0), 0}});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
  std::vector<WaveWork> out;
  for (auto& it : items) out.push_back(it.w);
  return out;
}

void build_work(brax_sys* s) { s->work = make_work(s, s->envs_per_wave); }

int upload_work(brax_sys* s) {
  (void)hipFree(s->d_work);
  s->d_work = nullptr;
  if (s->work.empty()) return BRAX_OK;
  HIP_TRY(hipMalloc(&s->d_work, sizeof(WaveWork) * s->work.size()));
  HIP_TRY(hipMemcpy(s->d_work, s->work.data(), sizeof(WaveWork) * s->work.size(), hipMemcpyHostToDevice));
  return BRAX_OK;
}

Fields F(const brax_state* st) { return Fields{st->pos, st->rot, st->vel, st->ang}; }

bool state_ok(const brax_state* st) { return st && st->pos && st->rot && st->vel && st->ang; }

// Run `body(stream)` directly, or capture it once per key into a HIP graph
// and replay that graph. A capture that holds a single node (one fused
// kernel) is not kept as a graph: replaying a one-node graph costs more than
// launching its kernel, so such keys are remembered and run directly.
template <class Fn>
int run_maybe_graph(brax_sys* s, bool use_graph, const GraphKey& key, hipStream_t stream, Fn body) {
  if (!use_graph) return body(stream);
  if (s->direct_keys.count(key)) return body(stream);
  auto it = s->graphs.find(key);
  if (it == s->graphs.end()) {
    hipStream_t cap = stream;
    bool own = false;
    if (cap == nullptr) {  // the legacy default stream cannot be captured
      HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      own = true;
    }
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    int rc = body(cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &g);
    if (own) (void)hipStreamDestroy(cap);
    if (rc != BRAX_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(BRAX_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    size_t n_nodes = 0;
    e = hipGraphGetNodes(g, nullptr, &n_nodes);
    if (e == hipSuccess && n_nodes <= 1) {
      (void)hipGraphDestroy(g);
      if (s->direct_keys.size() >= 64) s->direct_keys.clear();  // bounded
      s->direct_keys.insert(key);
      return body(stream);
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(BRAX_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    if (s->graphs.size() >= 16) {  // bounded cache
      auto old = s->graphs.begin();
      (void)hipGraphExecDestroy(old->second.second);
      (void)hipGraphDestroy(old->second.first);
      s->graphs.erase(old);
    }
    it = s->graphs.emplace(key, std::make_pair(g, x)).first;
  }
  HIP_TRY(hipGraphLaunch(it->second.second, stream));
  return BRAX_OK;
}

int check_flags(int32_t flags) {
  if (flags & ~(BRAX_PLAIN | BRAX_FUSED | BRAX_GRAPH | BRAX_NONFINITE_FLAGS))
    return fail(BRAX_E_ARG, "unknown flag bits 0x%x", flags);
  if ((flags & BRAX_PLAIN) && (flags & BRAX_FUSED)) return fail(BRAX_E_ARG, "BRAX_PLAIN and BRAX_FUSED both set");
  return BRAX_OK;
}

}  // namespace

extern "C" {

const char* brax_last_error(void) { return g_err.c_str(); }

int brax_sys_create(const char* const* descs, int32_t n_descs, const int32_t* env_desc, int32_t n_envs,
                    int32_t device, brax_sys** out) {
  g_err.clear();
  if (!out) return fail(BRAX_E_ARG, "out is NULL");
  *out = nullptr;
  if (!descs) return fail(BRAX_E_ARG, "descs is NULL");
  if (n_descs < 1 || n_descs > MAXT) return fail(BRAX_E_ARG, "n_descs must be in 1..%d", MAXT);
  if (n_envs < 0) return fail(BRAX_E_ARG, "n_envs must be >= 0");
  if (n_envs > (1 << 24)) return fail(BRAX_E_ARG, "n_envs too large");
  if (device < -1) return fail(BRAX_E_ARG, "device must be >= -1");
  std::unique_ptr<brax_sys, void (*)(brax_sys*)> s(new brax_sys(), free_all);
  s->device = -1;
  s->n_types = n_descs;
  s->E = n_envs;
  s->descs.resize(n_descs);
  for (int t = 0; t < n_descs; ++t) {
    if (!descs[t]) return fail(BRAX_E_ARG, "descs[%d] is NULL", t);
    std::string err;
    int rc = build_system(descs[t], s->descs[t], err);
    if (rc != BRAX_OK) return fail(rc, "system %d: %s", t, err.c_str());
    pack_type(s->descs[t], s->host_tab, t);
    s->Bm = std::max(s->Bm, s->host_tab.type[t].nb);
    s->Am = std::max(s->Am, s->host_tab.type[t].na);
    s->Dm = std::max(s->Dm, s->host_tab.type[t].ndof);
  }
  s->env_type.resize(n_envs);
  for (int e = 0; e < n_envs; ++e) {
    int t = env_desc ? env_desc[e] : 0;
    if (t < 0 || t >= n_descs) return fail(BRAX_E_ARG, "env_desc[%d] = %d out of range", e, t);
    s->env_type[e] = t;
    s->type_cnt[t]++;
  }
  int off = 0;
  for (int t = 0; t < n_descs; ++t) {
    s->type_off[t] = off;
    off += s->type_cnt[t];
  }
  s->env_list.resize(n_envs);
  {
    int fill[MAXT];
    for (int t = 0; t < n_descs; ++t) fill[t] = s->type_off[t];
    for (int e = 0; e < n_envs; ++e) s->env_list[fill[s->env_type[e]]++] = e;
  }
  // forward work list: lanes per environment include contact lanes
  for (int t = 0; t < n_descs; ++t) s->envs_per_wave[t] = std::max(1, 64 / s->host_tab.type[t].nl);
  for (int t = 0; t < n_descs; ++t) s->smax = std::max(s->smax, s->host_tab.type[t].substeps);
  s->waves_per_block = 1;
  build_work(s.get());
  if (device < 0) {
    *out = s.release();
    return BRAX_OK;
  }
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device >= ndev) return fail(BRAX_E_ARG, "device %d not present (%d devices)", device, ndev);
  s->device = device;
  DeviceGuard g(device);
  if (!g.ok) return fail(BRAX_E_DEVICE, "cannot select device %d", device);
  {
    int lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    if (lds > 0) s->lds_limit = (size_t)lds;
  }
  auto dmalloc = [&](void** p, size_t n) -> int {
    if (n == 0) n = 4;
    hipError_t e = hipMalloc(p, n);
    if (e == hipErrorOutOfMemory) return fail(BRAX_E_NOMEM, "device allocation of %zu bytes failed", n);
    if (e != hipSuccess) return fail(BRAX_E_DEVICE, "hipMalloc: %s", hipGetErrorString(e));
    return BRAX_OK;
  };
  int rc;
  if ((rc = dmalloc((void**)&s->d_tab, sizeof(Tables)))) return rc;
  HIP_TRY(hipMemcpy(s->d_tab, &s->host_tab, sizeof(Tables), hipMemcpyHostToDevice));
  if ((rc = dmalloc((void**)&s->d_env_type, sizeof(int32_t) * n_envs))) return rc;
  if ((rc = dmalloc((void**)&s->d_env_list, sizeof(int32_t) * n_envs))) return rc;
  if ((rc = dmalloc((void**)&s->d_type_off, sizeof(int32_t) * MAXT))) return rc;
  if ((rc = dmalloc((void**)&s->d_nonfinite, (size_t)n_envs))) return rc;
  if (n_envs) {
    HIP_TRY(hipMemcpy(s->d_env_type, s->env_type.data(), sizeof(int32_t) * n_envs, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->d_env_list, s->env_list.data(), sizeof(int32_t) * n_envs, hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(s->d_type_off, s->type_off, sizeof(int32_t) * MAXT, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(s->d_nonfinite, 0, (size_t)std::max(n_envs, 1)));
  for (int t = 0; t < n_descs; ++t) {
    const TypeT& ty = s->host_tab.type[t];
    size_t n = (size_t)s->type_cnt[t];
    if ((rc = dmalloc((void**)&s->d_jslot[t], sizeof(float) * 12 * std::max(ty.nj, 1) * std::max(n, (size_t)1))))
      return rc;
    // ground-contact slots (7 floats each), then body-body slots (13 floats each)
    if ((rc = dmalloc((void**)&s->d_cslot[t],
                      sizeof(float) * (7 * std::max(ty.nc, 1) + 13 * ty.np) * std::max(n, (size_t)1))))
      return rc;
  }
  if ((rc = upload_work(s.get()))) return rc;
  // the fixed workspace of brax_step_vjp_noalloc: its device address, once per device
  if (noalloc_init(device) != 0) return fail(BRAX_E_DEVICE, "no device address for the fixed adjoint workspace");
  {
    int full[MAXT];
    for (int t = 0; t < n_descs; ++t) full[t] = std::max(1, 64 / s->host_tab.type[t].nb);
    s->vjp_work = make_work(s.get(), full);
    if (!s->vjp_work.empty()) {
      if ((rc = dmalloc((void**)&s->d_vjp_work, sizeof(WaveWork) * s->vjp_work.size()))) return rc;
      HIP_TRY(hipMemcpy(s->d_vjp_work, s->vjp_work.data(), sizeof(WaveWork) * s->vjp_work.size(),
                        hipMemcpyHostToDevice));
    }
  }
  *out = s.release();
  return BRAX_OK;
}

void brax_sys_destroy(brax_sys* sys) {
  if (sys) free_all(sys);
}

int brax_sys_query(const brax_sys* s, brax_layout* out) {
  if (!s || !out) return fail(BRAX_E_ARG, "NULL argument");
  std::memset(out, 0, sizeof *out);
  out->n_envs = s->E;
  out->n_types = s->n_types;
  out->b_max = s->Bm;
  out->a_max = s->Am;
  out->d_max = s->Dm;
  out->tape_step_floats = (int64_t)s->smax * (int64_t)s->vjp_work.size() * TAPE_N * 64;
  out->p_max = 0;
  for (int t = 0; t < s->n_types; ++t) {
    const TypeT& ty = s->host_tab.type[t];
    out->n_params[t] = 4 * ty.nb + 5 * ty.nj + ty.na + 1;
    out->n_pairs[t] = ty.np;
    out->lanes_per_env[t] = ty.nl;
    out->p_max = std::max(out->p_max, out->n_params[t]);
  }
  for (int t = 0; t < s->n_types; ++t) {
    const TypeT& ty = s->host_tab.type[t];
    out->type_envs[t] = s->type_cnt[t];
    out->n_bodies[t] = ty.nb;
    out->n_joints[t] = ty.nj;
    out->n_actions[t] = ty.na;
    out->n_dof[t] = ty.ndof;
    out->n_contacts[t] = ty.nc;
    out->substeps[t] = ty.substeps;
    out->dt[t] = ty.dt;
  }
  out->device = s->device;
  out->nonfinite = s->d_nonfinite;
  out->vjp_lds_bytes = (int64_t)vjp_lds_bytes(s->host_tab, s->n_types, false);
  out->vjp_params_lds_bytes = (int64_t)vjp_lds_bytes(s->host_tab, s->n_types, true);
  out->lds_limit = (int64_t)s->lds_limit;
  return BRAX_OK;
}

int brax_default_angles(const brax_sys* s, int32_t type, float* out) {
  if (!s || !out) return fail(BRAX_E_ARG, "NULL argument");
  if (type < 0 || type >= s->n_types) return fail(BRAX_E_ARG, "type %d out of range", type);
  const TypeT& ty = s->host_tab.type[type];
  for (int j = 0; j < ty.nj; ++j) {
    const JointT& J = s->host_tab.joint[type][j];
    for (int k = 0; k < J.dof; ++k) out[J.dof0 + k] = J.def_angle[k];
  }
  return BRAX_OK;
}

int brax_default_qp(const brax_sys* sys, const float* joint_angles, const float* root_offset, brax_state* out,
                    void* stream) {
  brax_sys* s = const_cast<brax_sys*>(sys);
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (s->E == 0) return BRAX_OK;
  if (!state_ok(out)) return fail(BRAX_E_ARG, "out state has a NULL field");
  DeviceGuard g(s->device);
  HIP_TRY(launch_default_qp(s->ctx(), joint_angles, root_offset, F(out), (hipStream_t)stream));
  return BRAX_OK;
}

int brax_step(const brax_sys* sys, const brax_state* in, const float* act, brax_state* out, int32_t flags,
              void* stream) {
  brax_sys* s = const_cast<brax_sys*>(sys);
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (const int frc = check_flags(flags)) return frc;
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  int rc = check_flags(flags);
  if (rc) return rc;
  if (s->E == 0) return BRAX_OK;
  if (!state_ok(in) || !state_ok(out)) return fail(BRAX_E_ARG, "state has a NULL field");
  if (!act && s->Am > 0) return fail(BRAX_E_ARG, "act is NULL");
  DeviceGuard g(s->device);
  hipStream_t st = (hipStream_t)stream;
  const bool nf = flags & BRAX_NONFINITE_FLAGS;
  GraphKey key(0, flags, 1);
  key.add(in).add(out).add(act);
  return run_maybe_graph(s, flags & BRAX_GRAPH, key, st, [&](hipStream_t cs) -> int {
    LaunchCtx c = s->ctx();
    if (flags & BRAX_PLAIN) {
      if (nf) HIP_TRY(launch_fill_u8(s->d_nonfinite, s->E, 0, cs));
      HIP_TRY(launch_plain_step(c, F(in), F(out), act, s->d_jslot, s->d_cslot, nf, cs));
    } else {
      HIP_TRY(launch_fused(c, s->d_work, (int)s->work.size(), s->waves_per_block, F(in), F(out), act, 1, 0,
                           Fields{nullptr, nullptr, nullptr, nullptr}, nf, cs));
    }
    return BRAX_OK;
  });
}

int brax_rollout(const brax_sys* sys, const brax_state* in, const float* acts, int32_t T, int32_t save_every,
                 brax_state* traj, brax_state* out, int32_t flags, void* stream) {
  brax_sys* s = const_cast<brax_sys*>(sys);
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (const int frc = check_flags(flags)) return frc;
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (T < 0) return fail(BRAX_E_ARG, "T must be >= 0");
  if (save_every < 0) return fail(BRAX_E_ARG, "save_every must be >= 0");
  if (s->E == 0) return check_flags(flags);
  if (!state_ok(in) || !state_ok(out)) return fail(BRAX_E_ARG, "state has a NULL field");
  if (T > 0 && !acts && s->Am > 0) return fail(BRAX_E_ARG, "acts is NULL");
  if (save_every > 0 && T / save_every > 0 && !state_ok(traj)) return fail(BRAX_E_ARG, "traj state has a NULL field");
  int rc = check_flags(flags);
  if (rc) return rc;
  DeviceGuard g(s->device);
  hipStream_t st = (hipStream_t)stream;
  const bool nf = flags & BRAX_NONFINITE_FLAGS;
  Fields tr = (save_every > 0 && traj) ? F(traj) : Fields{nullptr, nullptr, nullptr, nullptr};
  GraphKey key(1, flags, T, save_every);
  key.add(in).add(out).add(acts).add(tr.pos).add(tr.rot).add(tr.vel).add(tr.ang);
  return run_maybe_graph(s, flags & BRAX_GRAPH, key, st, [&](hipStream_t cs) -> int {
    LaunchCtx c = s->ctx();
    if (T == 0) {
      if (in->pos != out->pos) HIP_TRY(launch_copy_state(c, F(in), F(out), cs));
      if (nf) HIP_TRY(launch_fill_u8(s->d_nonfinite, s->E, 0, cs));
      return BRAX_OK;
    }
    if (flags & BRAX_PLAIN) {
      if (nf) HIP_TRY(launch_fill_u8(s->d_nonfinite, s->E, 0, cs));
      const size_t per_step = (size_t)s->Am * s->E;
      int n_save = 0;
      for (int t = 0; t < T; ++t) {
        const bool last = t == T - 1;
        HIP_TRY(launch_plain_step(c, t == 0 ? F(in) : F(out), F(out), acts ? acts + per_step * t : nullptr,
                                  s->d_jslot, s->d_cslot, nf && last, cs));
        if (save_every > 0 && (t + 1) % save_every == 0) {
          size_t n3 = (size_t)3 * s->Bm * s->E, n4 = (size_t)4 * s->Bm * s->E;
          Fields dst{tr.pos + n3 * n_save, tr.rot + n4 * n_save, tr.vel + n3 * n_save, tr.ang + n3 * n_save};
          HIP_TRY(launch_copy_state(c, F(out), dst, cs));
          ++n_save;
        }
      }
    } else {
      HIP_TRY(launch_fused(c, s->d_work, (int)s->work.size(), s->waves_per_block, F(in), F(out), acts, T,
                           save_every, tr, nf, cs));
    }
    return BRAX_OK;
  });
}

int brax_rollout_tape(const brax_sys* sys, const brax_state* in, const float* acts, int32_t T, float* tape,
                      brax_state* out, int32_t flags, void* stream) {
  brax_sys* s = const_cast<brax_sys*>(sys);
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (const int frc = check_flags(flags)) return frc;
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (T < 0) return fail(BRAX_E_ARG, "T must be >= 0");
  if (flags & BRAX_PLAIN) return fail(BRAX_E_UNSUPPORTED, "the tape is written by the fused path only");
  if (s->E == 0) return check_flags(flags);
  if (!state_ok(in) || !state_ok(out)) return fail(BRAX_E_ARG, "state has a NULL field");
  if (T > 0 && !acts && s->Am > 0) return fail(BRAX_E_ARG, "acts is NULL");
  if (T > 0 && !tape) return fail(BRAX_E_ARG, "tape is NULL");
  int rc = check_flags(flags);
  if (rc) return rc;
  DeviceGuard g(s->device);
  hipStream_t st = (hipStream_t)stream;
  const bool nf = flags & BRAX_NONFINITE_FLAGS;
  GraphKey key(3, flags, T);
  key.add(in).add(out).add(acts).add(tape);
  return run_maybe_graph(s, flags & BRAX_GRAPH, key, st, [&](hipStream_t cs) -> int {
    LaunchCtx c = s->ctx();
    if (T == 0) {
      if (in->pos != out->pos) HIP_TRY(launch_copy_state(c, F(in), F(out), cs));
      if (nf) HIP_TRY(launch_fill_u8(s->d_nonfinite, s->E, 0, cs));
      return BRAX_OK;
    }
    // the adjoint's work list, so that both sides index the tape by the same wavefronts
    HIP_TRY(launch_fused(c, s->d_vjp_work, (int)s->vjp_work.size(), 1, F(in), F(out), acts, T, 0,
                         Fields{nullptr, nullptr, nullptr, nullptr}, nf, cs, tape, s->smax));
    return BRAX_OK;
  });
}

int brax_env_configure(brax_sys* s, const brax_env_params* params) {
  if (!s || !params) return fail(BRAX_E_ARG, "NULL argument");
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  EnvT h[MAXT] = {};
  for (int t = 0; t < s->n_types; ++t) {
    const brax_env_params& p = params[t];
    if (p.root < 0 || p.root >= s->host_tab.type[t].nb)
      return fail(BRAX_E_ARG, "type %d: root body %d out of range [0, %d)", t, p.root, s->host_tab.type[t].nb);
    if (!(p.z_min <= p.z_max)) return fail(BRAX_E_ARG, "type %d: z_min > z_max", t);
    h[t] = EnvT{p.root, p.forward_weight, p.healthy_reward, p.ctrl_cost, p.z_min, p.z_max};
  }
  DeviceGuard g(s->device);
  HIP_TRY(hipDeviceSynchronize());  // a running call may read the old parameters
  if (!s->d_env) {
    if (hipMalloc(&s->d_env, sizeof(EnvT) * MAXT) != hipSuccess)
      return fail(BRAX_E_NOMEM, "environment-layer allocation failed");
  }
  HIP_TRY(hipMemcpy(s->d_env, h, sizeof(EnvT) * MAXT, hipMemcpyHostToDevice));
  s->env_ready = true;
  return BRAX_OK;
}

int brax_env_step(const brax_sys* sys, const brax_state* in, const float* act, const brax_state* reset,
                  brax_state* out, float* obs, float* reward, uint8_t* done, int32_t flags, void* stream) {
  brax_sys* s = const_cast<brax_sys*>(sys);
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (const int frc = check_flags(flags)) return frc;
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (!s->env_ready) return fail(BRAX_E_ARG, "brax_env_configure has not been called");
  if (flags & BRAX_PLAIN) return fail(BRAX_E_UNSUPPORTED, "the environment step runs on the fused path only");
  if (s->E == 0) return check_flags(flags);
  if (!state_ok(in) || !state_ok(out) || !state_ok(reset)) return fail(BRAX_E_ARG, "state has a NULL field");
  if (!act && s->Am > 0) return fail(BRAX_E_ARG, "act is NULL");
  if (!obs || !reward || !done) return fail(BRAX_E_ARG, "obs, reward or done is NULL");
  if (reset->pos == out->pos) return fail(BRAX_E_ARG, "reset may not alias out");
  int rc = check_flags(flags);
  if (rc) return rc;
  DeviceGuard g(s->device);
  hipStream_t st = (hipStream_t)stream;
  const int omax = 11 + 2 * s->Dm;
  GraphKey key(5, flags, 1);
  key.add(in).add(act).add(reset).add(out).add(obs).add(reward).add(done).add(s->d_env);
  return run_maybe_graph(s, flags & BRAX_GRAPH, key, st, [&](hipStream_t cs) -> int {
    LaunchCtx c = s->ctx();
    HIP_TRY(launch_env_step(c, s->d_work, (int)s->work.size(), s->waves_per_block, s->d_env, omax, F(in), F(out), act,
                            F(reset), obs, reward, done, (flags & BRAX_NONFINITE_FLAGS) != 0, cs));
    return BRAX_OK;
  });
}

int brax_nonfinite(const brax_sys* s, uint8_t* out) {
  if (!s || !out) return fail(BRAX_E_ARG, "NULL argument");
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (s->E == 0) return BRAX_OK;
  DeviceGuard g(s->device);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, s->d_nonfinite, (size_t)s->E, hipMemcpyDeviceToHost));
  return BRAX_OK;
}

int brax_schedule(const brax_sys* s, int32_t* envs_per_wave, int32_t* waves_per_block) {
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (envs_per_wave) *envs_per_wave = s->envs_per_wave[0];
  if (waves_per_block) *waves_per_block = s->waves_per_block;
  return BRAX_OK;
}

int brax_set_schedule(brax_sys* s, int32_t envs_per_wave, int32_t waves_per_block) {
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
    return fail(BRAX_E_ARG, "waves_per_block must be 1, 2 or 4");
  for (int t = 0; t < s->n_types; ++t) {
    const int full = std::max(1, 64 / s->host_tab.type[t].nl);
    s->envs_per_wave[t] = envs_per_wave <= 0 ? full : std::min(envs_per_wave, full);
  }
  s->waves_per_block = waves_per_block;
  build_work(s);
  if (s->device >= 0) {
    DeviceGuard g(s->device);
    int rc = upload_work(s);
    if (rc) return rc;
  }
  for (auto& kv : s->graphs) {
    (void)hipGraphExecDestroy(kv.second.second);
    (void)hipGraphDestroy(kv.second.first);
  }
  s->graphs.clear();
  return BRAX_OK;
}

// Times the launch shapes from state `in` with T steps of actions `act`
// (both caller-owned, read only), or, with in = NULL, from the reset pose
// after 32 steps of zero actions with 8 steps of zero actions.
static int autotune_impl(brax_sys* s, const brax_state* in, const float* act, int T_in, hipStream_t st) {
  if (s->E == 0) return BRAX_OK;
  DeviceGuard g(s->device);
  const size_t n3 = (size_t)3 * s->Bm * s->E, n4 = (size_t)4 * s->Bm * s->E;
  const bool own = in == nullptr;
  const int T = own ? 8 : T_in;
  // scratch: the trials' output state and, without a caller's state, the
  // reset state and zero actions
  float* buf = nullptr;
  size_t nbuf = (3 * n3 + n4) + (own ? (3 * n3 + n4) + (size_t)std::max(s->Am, 1) * s->E * T : 0);
  HIP_TRY(hipMalloc(&buf, sizeof(float) * nbuf));
  HIP_TRY(hipMemsetAsync(buf, 0, sizeof(float) * nbuf, st));
  Fields b{buf, buf + n3, buf + n3 + n4, buf + 2 * n3 + n4};
  float* a0 = buf + 3 * n3 + n4;
  Fields a = own ? Fields{a0, a0 + n3, a0 + n3 + n4, a0 + 2 * n3 + n4} : F(in);
  const float* acts = own ? buf + 2 * (3 * n3 + n4) : act;
  LaunchCtx c = s->ctx();
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = BRAX_OK;
  // own timing state: the reset pose after 32 steps of zero actions, so that
  // the bodies have dropped onto the ground and contacts are active as in use
  if (own) {
    if (launch_default_qp(c, nullptr, nullptr, b, st) != hipSuccess ||
        launch_fused(c, s->d_work, (int)s->work.size(), s->waves_per_block, b, a, acts, 1, 0, Fields{}, false, st) !=
            hipSuccess)
      rc = fail(BRAX_E_DEVICE, "autotune reset failed");
    for (int k = 1; k < 32 && !rc; ++k)
      if (launch_fused(c, s->d_work, (int)s->work.size(), s->waves_per_block, a, a, acts, 1, 0, Fields{}, false,
                       st) != hipSuccess)
        rc = fail(BRAX_E_DEVICE, "autotune reset failed");
  }
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess || n_cu <= 0)
    n_cu = 256;
  const int n_simd = 4 * n_cu;  // four SIMDs per compute unit
  // candidates: environments per wavefront (per type) and wavefronts per block
  const int wpb_c[] = {1, 2, 4};
  int best_epw[MAXT];
  for (int t = 0; t < s->n_types; ++t) best_epw[t] = s->envs_per_wave[t];
  float best_total = 1e30f;
  int best_wpb = s->waves_per_block;
  std::vector<int> epw_c;
  for (int wpb : wpb_c) {
    if (rc) break;
    for (int t = 0; t < s->n_types; ++t) {
      // from a full wavefront down to half of one, at most 6 values evenly
      // spaced, and the value that gives the type about one wavefront per
      // SIMD. A batch of one type times that one first, so that it stays
      // unless another is clearly faster (fewer environments per wavefront
      // skip more contact and body-body slots that no lane of the wavefront
      // needs, which a short trial may not show); in a batch of several
      // types, whose wavefronts share the SIMDs, it comes last
      const int full = std::max(1, 64 / s->host_tab.type[t].nl);
      const int low = std::max(1, full / 2);
      const int fill = std::min(full, std::max(1, (s->type_cnt[t] + n_simd - 1) / n_simd));
      epw_c.clear();
      if (s->n_types == 1) epw_c.push_back(fill);
      const int span = full - low + 1, nc = std::min(span, 6);
      for (int i = 0; i < nc; ++i) {
        const int epw = full - (nc > 1 ? (i * (span - 1)) / (nc - 1) : 0);
        if (epw != fill) epw_c.push_back(epw);
      }
      if (s->n_types > 1) epw_c.push_back(fill);
      float best_t = 1e30f;
      for (int epw : epw_c) {
        // time this type alone with the others at their current best
        int saved[MAXT];
        for (int u = 0; u < s->n_types; ++u) saved[u] = s->envs_per_wave[u];
        for (int u = 0; u < s->n_types; ++u) s->envs_per_wave[u] = best_epw[u];
        s->envs_per_wave[t] = epw;
        build_work(s);
        if ((rc = upload_work(s))) break;
        float ms = 0, acc = 1e30f;
        for (int rep = 0; rep < 3 && !rc; ++rep) {
          if (hipEventRecord(e0, st) != hipSuccess ||
              launch_fused(c, s->d_work, (int)s->work.size(), wpb, a, b, acts, T, 0, Fields{}, false, st) !=
                  hipSuccess ||
              hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = fail(BRAX_E_DEVICE, "autotune launch failed");
          acc = std::min(acc, ms);
        }
        for (int u = 0; u < s->n_types; ++u) s->envs_per_wave[u] = saved[u];
        // a later (emptier) shape must be faster by more than the timing
        // noise (1%), so that repeated tunings settle on the same shape
        if (acc < 0.99f * best_t) {
          best_t = acc;
          best_epw[t] = epw;
        }
      }
      if (rc) break;
    }
    if (rc) break;
    // whole batch at this block shape
    for (int u = 0; u < s->n_types; ++u) s->envs_per_wave[u] = best_epw[u];
    build_work(s);
    if ((rc = upload_work(s))) break;
    float ms = 0, acc = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess ||
          launch_fused(c, s->d_work, (int)s->work.size(), wpb, a, b, acts, T, 0, Fields{}, false, st) != hipSuccess ||
          hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = fail(BRAX_E_DEVICE, "autotune launch failed");
        break;
      }
      acc = std::min(acc, ms);
    }
    if (!rc && acc < 0.99f * best_total) {
      best_total = acc;
      best_wpb = wpb;
    }
  }
  if (!rc) {
    for (int u = 0; u < s->n_types; ++u) s->envs_per_wave[u] = best_epw[u];
    s->waves_per_block = best_wpb;
    build_work(s);
    rc = upload_work(s);
  }
  (void)hipStreamSynchronize(st);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  // cached graphs hold the old schedule
  for (auto& kv : s->graphs) {
    (void)hipGraphExecDestroy(kv.second.second);
    (void)hipGraphDestroy(kv.second.first);
  }
  s->graphs.clear();
  return rc;
}

int brax_autotune(brax_sys* s, void* stream) {
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  return autotune_impl(s, nullptr, nullptr, 0, (hipStream_t)stream);
}

int brax_autotune_on(brax_sys* s, const brax_state* in, const float* act, int32_t T, void* stream) {
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (T < 1) return fail(BRAX_E_ARG, "T must be >= 1");
  if (s->E == 0) return BRAX_OK;
  if (!state_ok(in)) return fail(BRAX_E_ARG, "state has a NULL field");
  if (!act && s->Am > 0) return fail(BRAX_E_ARG, "act is NULL");
  return autotune_impl(s, in, act, T, (hipStream_t)stream);
}

namespace {

// Argument checks shared by brax_step_vjp and brax_step_vjp_noalloc.
int check_step_vjp(const brax_sys* s, const brax_state* in, const float* act, const brax_state* g_out,
                   const brax_state* g_in, const float* g_act, int32_t flags) {
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (const int frc = check_flags(flags)) return frc;
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (s->E == 0) return BRAX_OK;
  if (!state_ok(in) || !state_ok(g_out) || !state_ok(g_in)) return fail(BRAX_E_ARG, "state has a NULL field");
  if (!act && s->Am > 0) return fail(BRAX_E_ARG, "act is NULL");
  if (!g_act && s->Am > 0) return fail(BRAX_E_ARG, "g_act is NULL");
  if (g_in->pos == in->pos || g_in->pos == g_out->pos) return fail(BRAX_E_ARG, "g_in may not alias in or g_out");
  return BRAX_OK;
}

// The adjoint takes the per-phase kernels (tape in a device workspace) for
// BRAX_PLAIN or when the fused kernel's on-chip tape exceeds the device limit.
bool vjp_takes_plain(const brax_sys* s, int32_t flags) {
  return (flags & BRAX_PLAIN) || vjp_lds_bytes(s->host_tab, s->n_types, false) > s->lds_limit;
}

}  // namespace

int brax_step_vjp(const brax_sys* sys, const brax_state* in, const float* act, const brax_state* g_out,
                  brax_state* g_in, float* g_act, int32_t flags, void* stream) {
  brax_sys* s = const_cast<brax_sys*>(sys);
  int rc = check_step_vjp(s, in, act, g_out, g_in, g_act, flags);
  if (rc || s->E == 0) return rc;
  DeviceGuard g(s->device);
  hipStream_t st = (hipStream_t)stream;
  if ((rc = vjp_reserve(s->vjp, s->host_tab, s->n_types, s->type_cnt, s->E, s->Bm)))
    return fail(BRAX_E_NOMEM, "adjoint workspace allocation failed");
  GraphKey key(2, flags, 1);
  key.add(in).add(act).add(g_out).add(g_in).add(g_act).add(s->vjp.buf);
  return run_maybe_graph(s, flags & BRAX_GRAPH, key, st, [&](hipStream_t cs) -> int {
    LaunchCtx c = s->ctx();
    VjpSched sched{s->d_vjp_work, (int)s->vjp_work.size(), 1, s->d_jslot, s->d_cslot};
    HIP_TRY(launch_vjp(c, s->vjp, sched, F(in), act, F(g_out), F(g_in), g_act, vjp_takes_plain(s, flags), cs));
    return BRAX_OK;
  });
}

int brax_step_vjp_noalloc(const brax_sys* sys, const brax_state* in, const float* act, const brax_state* g_out,
                          brax_state* g_in, float* g_act, int32_t flags, void* stream) {
  const brax_sys* s = sys;
  int rc = check_step_vjp(s, in, act, g_out, g_in, g_act, flags);
  if (rc || s->E == 0) return rc;
  if (flags & BRAX_GRAPH)
    return fail(BRAX_E_ARG, "BRAX_GRAPH is not taken here (capturing allocates); capture the call yourself");
  const bool plain = vjp_takes_plain(s, flags);
  VjpWork w{};
  if (plain) {
    const size_t need = vjp_workspace_bytes(s->host_tab, s->n_types, s->type_cnt, s->E, s->Bm);
    if (need > NOALLOC_WORKSPACE_BYTES)
      return fail(BRAX_E_UNSUPPORTED, "the per-phase adjoint of this batch needs %zu bytes of workspace, more than "
                  "the fixed %zu", need, NOALLOC_WORKSPACE_BYTES);
    w.buf = noalloc_workspace(s->device);
    if (!w.buf) return fail(BRAX_E_DEVICE, "no fixed adjoint workspace on device %d", s->device);
    w.bytes = NOALLOC_WORKSPACE_BYTES;
  }
  DeviceGuard g(s->device);
  LaunchCtx c = s->ctx();
  VjpSched sched{s->d_vjp_work, (int)s->vjp_work.size(), 1, s->d_jslot, s->d_cslot};
  HIP_TRY(launch_vjp(c, w, sched, F(in), act, F(g_out), F(g_in), g_act, plain, (hipStream_t)stream));
  return BRAX_OK;
}

int brax_step_vjp_params(const brax_sys* sys, const brax_state* in, const float* act, const brax_state* g_out,
                         brax_state* g_in, float* g_act, float* g_params, int32_t flags, void* stream) {
  brax_sys* s = const_cast<brax_sys*>(sys);
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (const int frc = check_flags(flags)) return frc;
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (flags & BRAX_PLAIN) return fail(BRAX_E_UNSUPPORTED, "parameter cotangents are computed on the fused path only");
  if (s->E == 0) return check_flags(flags);
  if (!state_ok(in) || !state_ok(g_out) || !state_ok(g_in)) return fail(BRAX_E_ARG, "state has a NULL field");
  if (!act && s->Am > 0) return fail(BRAX_E_ARG, "act is NULL");
  if (!g_act && s->Am > 0) return fail(BRAX_E_ARG, "g_act is NULL");
  if (!g_params) return fail(BRAX_E_ARG, "g_params is NULL");
  if (vjp_lds_bytes(s->host_tab, s->n_types, true) > s->lds_limit)
    return fail(BRAX_E_UNSUPPORTED, "the parameter adjoint's on-chip tape (%zu bytes for %d substeps) exceeds the %zu-byte "
                "workgroup limit", vjp_lds_bytes(s->host_tab, s->n_types, true), s->smax, s->lds_limit);
  if (g_in->pos == in->pos || g_in->pos == g_out->pos) return fail(BRAX_E_ARG, "g_in may not alias in or g_out");
  int rc = check_flags(flags);
  if (rc) return rc;
  int p_max = 0;
  for (int t = 0; t < s->n_types; ++t)
    p_max = std::max(p_max, 4 * s->host_tab.type[t].nb + 5 * s->host_tab.type[t].nj + s->host_tab.type[t].na + 1);
  DeviceGuard g(s->device);
  hipStream_t st = (hipStream_t)stream;
  GraphKey key(6, flags, 1);
  key.add(in).add(act).add(g_out).add(g_in).add(g_act).add(g_params);
  return run_maybe_graph(s, flags & BRAX_GRAPH, key, st, [&](hipStream_t cs) -> int {
    LaunchCtx c = s->ctx();
    VjpSched sched{s->d_vjp_work, (int)s->vjp_work.size(), 1, s->d_jslot, s->d_cslot};
    HIP_TRY(launch_vjp_params(c, sched, F(in), act, F(g_out), F(g_in), g_act, g_params, p_max, cs));
    return BRAX_OK;
  });
}

int brax_step_vjp_tape(const brax_sys* sys, const float* tape, const float* act, const brax_state* g_out,
                       brax_state* g_in, float* g_act, int32_t flags, void* stream) {
  brax_sys* s = const_cast<brax_sys*>(sys);
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (const int frc = check_flags(flags)) return frc;
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (flags & BRAX_PLAIN) return fail(BRAX_E_UNSUPPORTED, "the tape adjoint runs on the fused path only");
  if (s->E == 0) return check_flags(flags);
  if (!tape) return fail(BRAX_E_ARG, "tape is NULL");
  if (!state_ok(g_out) || !state_ok(g_in)) return fail(BRAX_E_ARG, "state has a NULL field");
  if (!act && s->Am > 0) return fail(BRAX_E_ARG, "act is NULL");
  if (!g_act && s->Am > 0) return fail(BRAX_E_ARG, "g_act is NULL");
  if (g_in->pos == g_out->pos) return fail(BRAX_E_ARG, "g_in may not alias g_out");
  int rc = check_flags(flags);
  if (rc) return rc;
  DeviceGuard g(s->device);
  hipStream_t st = (hipStream_t)stream;
  GraphKey key(4, flags, 1);
  key.add(tape).add(act).add(g_out).add(g_in).add(g_act);
  return run_maybe_graph(s, flags & BRAX_GRAPH, key, st, [&](hipStream_t cs) -> int {
    LaunchCtx c = s->ctx();
    VjpSched sched{s->d_vjp_work, (int)s->vjp_work.size(), 1, s->d_jslot, s->d_cslot};
    HIP_TRY(launch_vjp_tape(c, sched, tape, 0, 1, act, F(g_out), F(g_in), g_act, cs));
    return BRAX_OK;
  });
}

int brax_rollout_vjp_tape(const brax_sys* sys, const float* tape, const float* acts, int32_t T,
                          const brax_state* g_out, brax_state* g_in, float* g_acts, int32_t flags, void* stream) {
  brax_sys* s = const_cast<brax_sys*>(sys);
  if (!s) return fail(BRAX_E_ARG, "sys is NULL");
  if (const int frc = check_flags(flags)) return frc;
  if (s->device < 0) return fail(BRAX_E_ARG, "host-only handle (created with device -1)");
  if (flags & BRAX_PLAIN) return fail(BRAX_E_UNSUPPORTED, "the tape adjoint runs on the fused path only");
  if (T < 0) return fail(BRAX_E_ARG, "T < 0");
  if (!state_ok(g_out) || !state_ok(g_in)) return fail(BRAX_E_ARG, "state has a NULL field");
  if (g_in->pos == g_out->pos) return fail(BRAX_E_ARG, "g_in may not alias g_out");
  int rc = check_flags(flags);
  if (rc) return rc;
  if (s->E == 0) return BRAX_OK;
  if (!tape && T > 0) return fail(BRAX_E_ARG, "tape is NULL");
  if (!acts && s->Am > 0 && T > 0) return fail(BRAX_E_ARG, "acts is NULL");
  if (!g_acts && s->Am > 0 && T > 0) return fail(BRAX_E_ARG, "g_acts is NULL");
  DeviceGuard g(s->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t tstride = (size_t)s->smax * s->vjp_work.size() * TAPE_N * 64;
  GraphKey key(7, flags, T);
  key.add(tape).add(acts).add(g_out).add(g_in).add(g_acts);
  return run_maybe_graph(s, flags & BRAX_GRAPH, key, st, [&](hipStream_t cs) -> int {
    LaunchCtx c = s->ctx();
    if (T == 0) {
      // no step: the cotangent passes through unchanged
      HIP_TRY(launch_copy_state(c, F(g_out), F(g_in), cs));
      return BRAX_OK;
    }
    VjpSched sched{s->d_vjp_work, (int)s->vjp_work.size(), 1, s->d_jslot, s->d_cslot};
    HIP_TRY(launch_vjp_tape(c, sched, tape, tstride, T, acts, F(g_out), F(g_in), g_acts, cs));
    return BRAX_OK;
  });
}

}  // extern "C"
