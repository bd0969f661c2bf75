// Host runtime of libsmpc: context, validation, robot upload, workspace and launches.
//
// Every entry point checks its arguments completely before it makes any HIP call,
// so invalid requests fail without touching the device (and can be tested on a
// machine without a GPU).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <algorithm>
#include <utility>
#include <vector>

#include "smpc.h"
#include "smpc_internal.h"

using namespace smpc;

// A context owns its device resources, which are acquired lazily by the first plan
// step: creating a context and setting a robot make no HIP call.
struct smpc_ctx {
  int device = 0;
  DevRobot host_robot{};        // packed robot, uploaded when robot_dirty
  DevRobot* dev_robot = nullptr;
  bool robot_set = false;
  bool robot_dirty = false;
  float qref[kNdof];
  double raw_d_qlo[kNdof], raw_d_qhi[kNdof], raw_d_qdlo[kNdof], raw_d_qdhi[kNdof];
  double raw_d_qddlo[kNdof], raw_d_qddhi[kNdof];
  double slot_radius[kSlots];
  void* workspace = nullptr;
  size_t workspace_bytes = 0;
  std::vector<hipEvent_t> prof_events;  // 3 per recorded step
  int prof_capacity = 0;                // steps that may still be recorded
  int prof_recorded = 0;
  std::string last_error;
};

namespace {

smpc_status fail(smpc_ctx* ctx, smpc_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return st;
}

bool finite_all(const float* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

bool finite_all(const double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

// Sets the context's device current and restores the caller's device on exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

smpc_status validate_robot(smpc_ctx* ctx, const smpc_robot_desc* d) {
  if (d->n_dof != kNdof)
    return fail(ctx, SMPC_E_UNSUPPORTED, "n_dof=%d: only %d-DoF arms are supported", d->n_dof,
                kNdof);
  if (!finite_all(d->a, kNdof) || !finite_all(d->d, kNdof) || !finite_all(d->alpha, kNdof))
    return fail(ctx, SMPC_E_INVALID_ARG, "non-finite DH parameter");
  const double* lo[3] = {d->q_min, d->qd_min, d->qdd_min};
  const double* hi[3] = {d->q_max, d->qd_max, d->qdd_max};
  const char* names[3] = {"q", "qd", "qdd"};
  for (int g = 0; g < 3; ++g) {
    if (!finite_all(lo[g], kNdof) || !finite_all(hi[g], kNdof))
      return fail(ctx, SMPC_E_INVALID_ARG, "non-finite %s limit", names[g]);
    for (int j = 0; j < kNdof; ++j)
      if (!(lo[g][j] < hi[g][j]))
        return fail(ctx, SMPC_E_INVALID_ARG, "%s_min[%d] >= %s_max[%d]", names[g], j, names[g],
                    j);
  }
  if (!finite_all(d->q_ref, kNdof)) return fail(ctx, SMPC_E_INVALID_ARG, "non-finite q_ref");
  if (d->n_spheres < 0 || d->n_spheres > SMPC_MAX_SPHERES)
    return fail(ctx, SMPC_E_INVALID_ARG, "n_spheres=%d outside [0, %d]", d->n_spheres,
                SMPC_MAX_SPHERES);
  int per_link[kNdof + 1] = {0};
  for (int s = 0; s < d->n_spheres; ++s) {
    const int l = d->sphere_link[s];
    if (l < 1 || l > kNdof)
      return fail(ctx, SMPC_E_INVALID_ARG, "sphere_link[%d]=%d outside 1..%d", s, l, kNdof);
    if (++per_link[l] > kSpl)
      return fail(ctx, SMPC_E_UNSUPPORTED, "link %d carries more than %d spheres", l, kSpl);
    if (!finite_all(d->sphere_center[s], 3) || !std::isfinite(d->sphere_radius[s]) ||
        d->sphere_radius[s] < 0.0)
      return fail(ctx, SMPC_E_INVALID_ARG, "sphere %d: non-finite centre or bad radius", s);
  }
  if (d->n_pairs < 0 || d->n_pairs > SMPC_MAX_PAIRS)
    return fail(ctx, SMPC_E_INVALID_ARG, "n_pairs=%d outside [0, %d]", d->n_pairs,
                SMPC_MAX_PAIRS);
  for (int i = 0; i < d->n_pairs; ++i) {
    const int a = d->pairs[i][0], b = d->pairs[i][1];
    if (a < 0 || b < 0 || a >= d->n_spheres || b >= d->n_spheres || a == b)
      return fail(ctx, SMPC_E_INVALID_ARG, "pair %d = (%d, %d) invalid", i, a, b);
  }
  return SMPC_OK;
}

smpc_status validate_args(smpc_ctx* ctx, const smpc_plan_args* a) {
  if (!ctx->robot_set) return fail(ctx, SMPC_E_INVALID_ARG, "no robot set on this context");
  if (a->K < 1) return fail(ctx, SMPC_E_INVALID_ARG, "K=%d must be >= 1", a->K);
  if (a->H < 1 || a->H > kMaxH)
    return fail(ctx, SMPC_E_INVALID_ARG, "H=%d outside [1, %d]", a->H, kMaxH);
  if ((long long)a->K * a->H * kNdof > (1LL << 31) - 1)
    return fail(ctx, SMPC_E_INVALID_ARG, "K*H*7 exceeds 2^31-1 elements");
  if (!std::isfinite(a->dt) || !(a->dt > 0.f))
    return fail(ctx, SMPC_E_INVALID_ARG, "dt must be finite and > 0");
  if (!std::isfinite(a->lambda) || !(a->lambda > 0.f))
    return fail(ctx, SMPC_E_INVALID_ARG, "lambda must be finite and > 0");
  if (!finite_all(a->q0, kNdof) || !finite_all(a->qd0, kNdof))
    return fail(ctx, SMPC_E_INVALID_ARG, "non-finite joint state");
  if (!finite_all(a->T_goal, 16)) return fail(ctx, SMPC_E_INVALID_ARG, "non-finite T_goal");
  const float* T = a->T_goal;
  if (T[12] != 0.f || T[13] != 0.f || T[14] != 0.f || T[15] != 1.f)
    return fail(ctx, SMPC_E_INVALID_ARG, "T_goal last row must be [0 0 0 1]");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double dot = 0.0;
      for (int r = 0; r < 3; ++r) dot += (double)T[r * 4 + i] * (double)T[r * 4 + j];
      if (std::fabs(dot - (i == j ? 1.0 : 0.0)) > 1e-4)
        return fail(ctx, SMPC_E_INVALID_ARG, "T_goal rotation is not orthonormal");
    }
  const smpc_cost_weights& w = a->weights;
  const float wv[] = {w.w_pose_t, w.w_pose_r, w.w_term_t, w.w_term_r, w.w_env, w.d_act,
                      w.w_self, w.w_q, w.w_qd, w.w_qdd, w.limit_margin_frac, w.w_smooth, w.w_ns};
  for (float x : wv)
    if (!std::isfinite(x) || x < 0.f)
      return fail(ctx, SMPC_E_INVALID_ARG, "cost weights must be finite and >= 0");
  if (!(w.limit_margin_frac < 0.5f))
    return fail(ctx, SMPC_E_INVALID_ARG, "limit_margin_frac must be < 0.5");
  const smpc_grid& g = a->esdf;
  if (!g.data) return fail(ctx, SMPC_E_INVALID_ARG, "esdf.data is NULL");
  if (g.nx < 2 || g.ny < 2 || g.nz < 2)
    return fail(ctx, SMPC_E_INVALID_ARG, "grid dimensions must be >= 2");
  if (g.dtype != SMPC_GRID_F32 && g.dtype != SMPC_GRID_F16)
    return fail(ctx, SMPC_E_INVALID_ARG, "unknown grid dtype %d", g.dtype);
  const long long elems = (long long)g.nx * g.ny * g.nz;
  if (elems * (g.dtype == SMPC_GRID_F16 ? 2 : 4) >= (1LL << 31))
    return fail(ctx, SMPC_E_INVALID_ARG, "grid exceeds 2^31 bytes");
  if (!finite_all(g.origin, 3) || !std::isfinite(g.voxel) || !(g.voxel > 0.f))
    return fail(ctx, SMPC_E_INVALID_ARG, "grid origin/voxel must be finite, voxel > 0");
  if (!a->U_in || !a->U_out) return fail(ctx, SMPC_E_INVALID_ARG, "U_in/U_out is NULL");
  if (!a->noise) {
    for (int j = 0; j < kNdof; ++j)
      if (!std::isfinite(a->sigma[j]) || a->sigma[j] < 0.f)
        return fail(ctx, SMPC_E_INVALID_ARG, "sampling: sigma must be finite and >= 0");
  }
  return SMPC_OK;
}

void tighten(const double* lo, const double* hi, double frac, float* out_lo, float* out_hi) {
  for (int j = 0; j < kNdof; ++j) {
    const double e = frac * (hi[j] - lo[j]);
    out_lo[j] = (float)(lo[j] + e);
    out_hi[j] = (float)(hi[j] - e);
  }
}

StepParams make_params(const smpc_ctx* ctx, const smpc_plan_args* a, const LaunchConfig& lc) {
  StepParams p;
  std::memset(&p, 0, sizeof p);
  for (int j = 0; j < kNdof; ++j) {
    p.q0[j] = a->q0[j];
    p.qd0[j] = a->qd0[j];
    p.qref[j] = ctx->qref[j];
  }
  const float* T = a->T_goal;
  // R_g^T (row-major) and R_g^T t_g.
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) p.RgT[r * 3 + c] = T[c * 4 + r];
  for (int r = 0; r < 3; ++r) {
    double acc = 0.0;
    for (int i = 0; i < 3; ++i) acc += (double)T[i * 4 + r] * (double)T[i * 4 + 3];
    p.tgr[r] = (float)acc;
  }
  const double frac = a->weights.limit_margin_frac;
  tighten(ctx->raw_d_qlo, ctx->raw_d_qhi, frac, p.qlo, p.qhi);
  tighten(ctx->raw_d_qdlo, ctx->raw_d_qdhi, frac, p.qdlo, p.qdhi);
  tighten(ctx->raw_d_qddlo, ctx->raw_d_qddhi, frac, p.qddlo, p.qddhi);
  for (int s = 0; s < kSlots; ++s)
    p.env_thr[s] = (float)((double)a->weights.d_act + ctx->slot_radius[s]);
  const smpc_cost_weights& w = a->weights;
  p.w_pose_t = w.w_pose_t;
  p.w_pose_r = w.w_pose_r;
  p.w_term_t = w.w_term_t;
  p.w_term_r = w.w_term_r;
  p.w_env = w.w_env;
  p.w_self = w.w_self;
  p.w_q = w.w_q;
  p.w_qd = w.w_qd;
  p.w_qdd = w.w_qdd;
  p.w_smooth = w.w_smooth;
  p.w_ns = w.w_ns;
  const double inv_voxel = 1.0 / (double)a->esdf.voxel;
  p.inv_voxel = (float)inv_voxel;
  p.gcx = (float)(-(double)a->esdf.origin[0] * inv_voxel - 0.5);
  p.gcy = (float)(-(double)a->esdf.origin[1] * inv_voxel - 0.5);
  p.gcz = (float)(-(double)a->esdf.origin[2] * inv_voxel - 0.5);
  p.nx = a->esdf.nx;
  p.ny = a->esdf.ny;
  p.nz = a->esdf.nz;
  const int elem = a->esdf.dtype == SMPC_GRID_F16 ? 2 : 4;
  p.grid_bytes = (uint32_t)((long long)a->esdf.nx * a->esdf.ny * a->esdf.nz * elem);
  p.seed_lo = (uint32_t)a->seed;
  p.seed_hi = (uint32_t)(a->seed >> 32);
  for (int j = 0; j < kNdof; ++j) p.sigma[j] = a->sigma[j];
  p.K = a->K;
  p.H = a->H;
  p.R = lc.R;
  p.P = lc.P;
  p.dt = a->dt;
  p.inv_lambda = (float)(1.0 / (double)a->lambda);
  return p;
}

}  // namespace

extern "C" {

int32_t smpc_version(void) { return 100; }

const char* smpc_status_string(smpc_status st) {
  switch (st) {
    case SMPC_OK: return "ok";
    case SMPC_E_INVALID_ARG: return "invalid argument";
    case SMPC_E_OOM: return "out of device memory";
    case SMPC_E_DEVICE: return "device error";
    case SMPC_E_NUMERIC: return "no finite rollout cost";
    case SMPC_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* smpc_last_error(const smpc_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : "null context";
}

smpc_status smpc_create(smpc_ctx** out, int32_t hip_device) {
  if (!out) return SMPC_E_INVALID_ARG;
  *out = nullptr;
  if (hip_device < 0) return SMPC_E_INVALID_ARG;
  smpc_ctx* ctx = new (std::nothrow) smpc_ctx();
  if (!ctx) return SMPC_E_OOM;
  ctx->device = hip_device;
  *out = ctx;
  return SMPC_OK;
}

static void destroy_events(smpc_ctx* ctx) {
  for (hipEvent_t e : ctx->prof_events) (void)hipEventDestroy(e);
  ctx->prof_events.clear();
  ctx->prof_capacity = 0;
  ctx->prof_recorded = 0;
}

void smpc_destroy(smpc_ctx* ctx) {
  if (!ctx) return;
  if (ctx->dev_robot || ctx->workspace || !ctx->prof_events.empty()) {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    destroy_events(ctx);
    if (ctx->dev_robot) (void)hipFree(ctx->dev_robot);
    if (ctx->workspace) (void)hipFree(ctx->workspace);
  }
  delete ctx;
}

smpc_status smpc_set_robot(smpc_ctx* ctx, const smpc_robot_desc* d) {
  if (!ctx) return SMPC_E_INVALID_ARG;
  if (!d) return fail(ctx, SMPC_E_INVALID_ARG, "robot description is NULL");
  ctx->last_error.clear();
  const smpc_status st = validate_robot(ctx, d);
  if (st != SMPC_OK) return st;

  DevRobot r;
  std::memset(&r, 0, sizeof r);
  for (int j = 0; j < kNdof; ++j) {
    r.ca[j] = (float)std::cos(d->alpha[j]);
    r.sa[j] = (float)std::sin(d->alpha[j]);
    r.a[j] = (float)d->a[j];
    r.d[j] = (float)d->d[j];
    ctx->raw_d_qlo[j] = (double)(float)d->q_min[j];
    ctx->raw_d_qhi[j] = (double)(float)d->q_max[j];
    ctx->raw_d_qdlo[j] = (double)(float)d->qd_min[j];
    ctx->raw_d_qdhi[j] = (double)(float)d->qd_max[j];
    ctx->raw_d_qddlo[j] = (double)(float)d->qdd_min[j];
    ctx->raw_d_qddhi[j] = (double)(float)d->qdd_max[j];
    ctx->qref[j] = (float)d->q_ref[j];
  }
  // Spheres of link l fill slots (l - 1) * kSpl + j.  Within a link the sphere that
  // gives the smallest bounding radius (max over the link's spheres of
  // |c_i - c_0| + r_i) goes to slot 0: the kernel centres the link's bounding
  // sphere there.
  int slot_of[SMPC_MAX_SPHERES];
  for (int s = 0; s < kSlots; ++s) ctx->slot_radius[s] = 0.0;
  double bound_r[kNdof] = {0};
  for (int l = 1; l <= kNdof; ++l) {
    int members[kSpl], n = 0;
    for (int s = 0; s < d->n_spheres; ++s)
      if (d->sphere_link[s] == l) members[n++] = s;
    if (n == 0) continue;
    int best = 0;
    double best_R = 1e300;
    for (int c = 0; c < n; ++c) {
      double R = 0.0;
      for (int i = 0; i < n; ++i) {
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
          const double diff = (double)(float)d->sphere_center[members[i]][k] -
                              (double)(float)d->sphere_center[members[c]][k];
          d2 += diff * diff;
        }
        R = std::max(R, std::sqrt(d2) + (double)(float)d->sphere_radius[members[i]]);
      }
      if (R < best_R) {
        best_R = R;
        best = c;
      }
    }
    std::swap(members[0], members[best]);
    bound_r[l - 1] = best_R + kBoundMargin;
    r.lbound[l - 1] = (float)bound_r[l - 1];
    for (int j = 0; j < n; ++j) {
      const int s = members[j];
      const int slot = (l - 1) * kSpl + j;
      slot_of[s] = slot;
      const float radius = (float)d->sphere_radius[s];
      r.sc[slot][0] = (float)d->sphere_center[s][0];
      r.sc[slot][1] = (float)d->sphere_center[s][1];
      r.sc[slot][2] = (float)d->sphere_center[s][2];
      r.sc[slot][3] = radius;
      r.slot_active |= 1u << slot;
      ctx->slot_radius[slot] = (double)radius;
    }
  }
  int n_unique = 0;
  uint32_t seen[kSlots] = {0};
  for (int i = 0; i < d->n_pairs; ++i) {
    int a = slot_of[d->pairs[i][0]], b = slot_of[d->pairs[i][1]];
    if (a > b) std::swap(a, b);
    if (seen[a] & (1u << b)) continue;  // duplicate pair: counted once
    seen[a] |= 1u << b;
    const double rs = ctx->slot_radius[a] + ctx->slot_radius[b];
    float4 rec;
    int32_t ia = a, ib = b;
    std::memcpy(&rec.x, &ia, 4);
    std::memcpy(&rec.y, &ib, 4);
    rec.z = (float)(rs * rs);
    rec.w = (float)rs;
    r.pair_rec[n_unique] = rec;
    ++n_unique;
    const int la = a / kSpl, lb = b / kSpl, lp = la * kNdof + lb;
    const int bit = (a % kSpl) * kSpl + (b % kSpl);
    r.lp_mask[lp] |= 1u << bit;
    r.lp_rr2[lp][bit] = (float)(rs * rs);
    r.lp_rs[lp][bit] = (float)rs;
    const double bt = bound_r[la] + bound_r[lb];
    r.lp_bthr[lp] = (float)(bt * bt);
  }
  r.n_pairs = n_unique;
  ctx->host_robot = r;
  ctx->robot_set = true;
  ctx->robot_dirty = true;
  return SMPC_OK;
}

smpc_status smpc_plan_step(smpc_ctx* ctx, const smpc_plan_args* a, void* stream) {
  if (!ctx) return SMPC_E_INVALID_ARG;
  if (!a) return fail(ctx, SMPC_E_INVALID_ARG, "args is NULL");
  ctx->last_error.clear();
  const smpc_status st = validate_args(ctx, a);
  if (st != SMPC_OK) return st;

  const LaunchConfig lc = plan_launch_config(a->K, a->H);
  const StepParams p = make_params(ctx, a, lc);

  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, SMPC_E_DEVICE, "hipSetDevice(%d) failed", ctx->device);
  if (!ctx->dev_robot &&
      hipMalloc(reinterpret_cast<void**>(&ctx->dev_robot), sizeof(DevRobot)) != hipSuccess) {
    ctx->dev_robot = nullptr;
    return fail(ctx, SMPC_E_OOM, "robot buffer allocation failed");
  }
  if (ctx->robot_dirty) {
    // Ordered before this step's kernels on `stream`; synchronous so the host copy
    // may change afterwards.
    if (hipMemcpy(ctx->dev_robot, &ctx->host_robot, sizeof(DevRobot),
                  hipMemcpyHostToDevice) != hipSuccess)
      return fail(ctx, SMPC_E_DEVICE, "robot upload failed");
    ctx->robot_dirty = false;
  }
  const size_t need = workspace_bytes(a->K, a->H, lc.P);
  if (need > ctx->workspace_bytes) {
    // Grow-only arena.  hipFree waits for outstanding work that may use the old one.
    if (ctx->workspace) (void)hipFree(ctx->workspace);
    ctx->workspace = nullptr;
    ctx->workspace_bytes = 0;
    if (hipMalloc(&ctx->workspace, need) != hipSuccess) {
      ctx->workspace = nullptr;
      return fail(ctx, SMPC_E_OOM, "workspace allocation of %zu bytes failed", need);
    }
    ctx->workspace_bytes = need;
  }
  const Workspace ws = carve_workspace(ctx->workspace, a->K, a->H, lc.P);
  hipEvent_t* ev = nullptr;
  if (ctx->prof_recorded < ctx->prof_capacity) ev = &ctx->prof_events[3 * ctx->prof_recorded++];
  const int e = launch_plan_step(ctx->dev_robot, p, lc, ws, *a, stream, ev);
  if (e != 0)
    return fail(ctx, SMPC_E_DEVICE, "kernel launch failed: %s",
                hipGetErrorString(static_cast<hipError_t>(e)));
  return SMPC_OK;
}

smpc_status smpc_sample_noise(uint64_t seed, int32_t K, int32_t H, const float* sigma,
                              float* eps_out, uint32_t* words_out, void* stream) {
  if (K < 1 || H < 1 || H > kMaxH || !sigma || (!eps_out && !words_out))
    return SMPC_E_INVALID_ARG;
  if ((long long)K * H * 8 > (1LL << 31) - 1) return SMPC_E_INVALID_ARG;
  for (int j = 0; j < kNdof; ++j)
    if (!std::isfinite(sigma[j]) || sigma[j] < 0.f) return SMPC_E_INVALID_ARG;
  return launch_sample_noise(seed, K, H, sigma, eps_out, words_out, stream) == 0
             ? SMPC_OK
             : SMPC_E_DEVICE;
}

smpc_status smpc_grid_to_f16(const float* src, void* dst, int64_t n, float clamp, void* stream) {
  if (!src || !dst || n < 0 || !std::isfinite(clamp) || !(clamp > 0.f))
    return SMPC_E_INVALID_ARG;
  if (n == 0) return SMPC_OK;
  return launch_grid_to_f16(src, dst, (long long)n, clamp, stream) == 0 ? SMPC_OK
                                                                        : SMPC_E_DEVICE;
}

smpc_status smpc_profile_enable(smpc_ctx* ctx, int32_t n_steps) {
  if (!ctx) return SMPC_E_INVALID_ARG;
  if (n_steps < 0 || n_steps > (1 << 20))
    return fail(ctx, SMPC_E_INVALID_ARG, "n_steps=%d outside [0, 2^20]", n_steps);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, SMPC_E_DEVICE, "hipSetDevice(%d) failed", ctx->device);
  (void)hipDeviceSynchronize();
  destroy_events(ctx);
  ctx->prof_events.resize((size_t)3 * n_steps);
  for (size_t i = 0; i < ctx->prof_events.size(); ++i) {
    if (hipEventCreate(&ctx->prof_events[i]) != hipSuccess) {
      ctx->prof_events.resize(i);
      destroy_events(ctx);
      return fail(ctx, SMPC_E_DEVICE, "hipEventCreate failed");
    }
  }
  ctx->prof_capacity = n_steps;
  ctx->prof_recorded = 0;
  return SMPC_OK;
}

smpc_status smpc_profile_read(smpc_ctx* ctx, float* rollout_ms, float* merge_ms,
                              int32_t capacity, int32_t* n_steps) {
  if (!ctx) return SMPC_E_INVALID_ARG;
  if (!rollout_ms || !merge_ms || !n_steps || capacity < 0)
    return fail(ctx, SMPC_E_INVALID_ARG, "null output or negative capacity");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, SMPC_E_DEVICE, "hipSetDevice(%d) failed", ctx->device);
  const int n = ctx->prof_recorded < capacity ? ctx->prof_recorded : capacity;
  for (int i = 0; i < n; ++i) {
    hipEvent_t* ev = &ctx->prof_events[3 * i];
    if (hipEventSynchronize(ev[2]) != hipSuccess ||
        hipEventElapsedTime(&rollout_ms[i], ev[0], ev[1]) != hipSuccess ||
        hipEventElapsedTime(&merge_ms[i], ev[1], ev[2]) != hipSuccess)
      return fail(ctx, SMPC_E_DEVICE, "reading profiling events failed");
  }
  *n_steps = n;
  ctx->prof_recorded = 0;
  return SMPC_OK;
}

}  // extern "C"
