// Host runtime of libsmpc: context, validation, robot upload, workspace and launches.
//
// Every entry point checks its arguments completely before it makes any HIP call,
// so invalid requests fail without touching the device (and can be tested on a
// machine without a GPU).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <algorithm>
#include <deque>
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

// Two device byte ranges [a, a + na) and [b, b + nb) share a byte (NULL: never).
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b) return false;
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
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
  if (a->receding != 0 && a->receding != 1)
    return fail(ctx, SMPC_E_INVALID_ARG, "receding must be 0 or 1");
  const size_t ub = (size_t)a->H * kNdof * sizeof(float), sb = 2 * kNdof * sizeof(float);
  if (a->receding && overlaps(a->U_out, ub, a->U_in, ub))
    return fail(ctx, SMPC_E_INVALID_ARG, "receding: U_out overlaps U_in");
  if (overlaps(a->u0_out, kNdof * sizeof(float), a->U_in, ub) ||
      overlaps(a->u0_out, kNdof * sizeof(float), a->state_in, sb) ||
      overlaps(a->state_out, sb, a->U_in, ub) || overlaps(a->state_out, sb, a->state_in, sb))
    return fail(ctx, SMPC_E_INVALID_ARG, "u0_out/state_out overlaps an input");
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
    p.env_thr[s] = (ctx->host_robot.slot_active & (1u << s))
                       ? (float)((double)a->weights.d_act + ctx->slot_radius[s])
                       : -1e30f;  // empty slot: hinge is always 0
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
  // Scaling by 1/8 is exact and commutes with rounding, so fma(x, inv_voxel8, gc8) is
  // fma(x, inv_voxel, gc) / 8 bit for bit.
  p.inv_voxel8 = p.inv_voxel * 0.125f;
  p.gc8[0] = p.gcx * 0.125f;
  p.gc8[1] = p.gcy * 0.125f;
  p.gc8[2] = p.gcz * 0.125f;
  p.nx = a->esdf.nx;
  p.ny = a->esdf.ny;
  p.nz = a->esdf.nz;
  const int elem = a->esdf.dtype == SMPC_GRID_F16 ? 2 : 4;
  p.grid_bytes = (uint32_t)((long long)a->esdf.nx * a->esdf.ny * a->esdf.nz * elem);
  p.ncx = coarse_cells_1d(a->esdf.nx);
  p.ncy = coarse_cells_1d(a->esdf.ny);
  p.ncz = coarse_cells_1d(a->esdf.nz);
  p.coarse_bytes =
      a->esdf.coarse ? (uint32_t)((long long)p.ncx * p.ncy * p.ncz * (long long)sizeof(float)) : 0u;
  p.cmax[0] = (float)(p.ncx - 1);
  p.cmax[1] = (float)(p.ncy - 1);
  p.cmax[2] = (float)(p.ncz - 1);
  p.cstride[0] = (float)p.ncx;
  p.cstride[1] = (float)((long long)p.ncx * p.ncy);
  p.seed_lo = (uint32_t)a->seed;
  p.seed_hi = (uint32_t)(a->seed >> 32);
  for (int j = 0; j < kNdof; ++j) p.sigma[j] = a->sigma[j];
  p.K = a->K;
  p.H = a->H;
  p.R = lc.R;
  p.P = lc.P;
  p.dt = a->dt;
  p.k_lambda = (float)(1.4426950408889634 / (double)a->lambda);
  return p;
}

// The request descriptor of one plan step (by value in the kernel arguments).
Request single_request(const smpc_plan_args* a, const StepParams& p, const Workspace& ws) {
  Request q;
  std::memset(&q, 0, sizeof q);
  q.p = p;
  q.grid = a->esdf.data;
  q.coarse = a->esdf.coarse;
  q.noise = a->noise;
  q.U_in = a->U_in;
  q.U_out = a->U_out;
  q.costs_out = a->costs_out;
  q.weights_out = a->weights_out;
  q.stats_out = a->stats_out;
  q.u0_out = a->u0_out;
  q.state_in = a->state_in;
  q.state_out = a->state_out;
  q.shift_out = a->receding;
  q.ws = ws;
  q.c0_in_ws = (a->costs_out || a->stats_out) ? 1 : 0;
  return q;
}

// Allocates the device robot buffer if needed and uploads a changed robot.  The
// caller has made the context's device current.
smpc_status ensure_device_robot(smpc_ctx* ctx) {
  if (!ctx->dev_robot &&
      hipMalloc(reinterpret_cast<void**>(&ctx->dev_robot), sizeof(DevRobot)) != hipSuccess) {
    ctx->dev_robot = nullptr;
    return fail(ctx, SMPC_E_OOM, "robot buffer allocation failed");
  }
  if (ctx->robot_dirty) {
    // Synchronous, so it is ordered before every later launch and the host copy may
    // change afterwards.
    if (hipMemcpy(ctx->dev_robot, &ctx->host_robot, sizeof(DevRobot),
                  hipMemcpyHostToDevice) != hipSuccess)
      return fail(ctx, SMPC_E_DEVICE, "robot upload failed");
    ctx->robot_dirty = false;
  }
  return SMPC_OK;
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
    r.lp[lp].mask |= 1u << bit;
    r.lp[lp].rr2[bit] = (float)(rs * rs);
    r.lp[lp].rs[bit] = (float)rs;
    const double bt = bound_r[la] + bound_r[lb];
    r.lp[lp].bthr = (float)(bt * bt);
    const double sb = ctx->slot_radius[a] + bound_r[lb];
    r.lp[lp].sthr[a % kSpl] = (float)(sb * sb);
  }
  r.n_pairs = n_unique;
  ctx->host_robot = r;
  ctx->robot_set = true;
  ctx->robot_dirty = true;
  return SMPC_OK;
}

// Bounds of another grid restricted to a ball (smpc_grid_coarse_min_ball's arguments, the
// ball in continuous-index units).
struct BallBounds {
  const smpc_grid* g;
  float c[3];
  float r2;
  float* out;
};

// Checks smpc_grid_coarse_min_ball's arguments and puts the ball in index units: its
// radius widened by one voxel, which covers the float32 rounding of the sphere
// positions and of the cell test.
static smpc_status ball_bounds(const smpc_grid* g, const float* center, float radius,
                               float* coarse_out, BallBounds& b) {
  if (!g || !g->data || !coarse_out || !center || g->nx < 2 || g->ny < 2 || g->nz < 2 ||
      (g->dtype != SMPC_GRID_F32 && g->dtype != SMPC_GRID_F16))
    return SMPC_E_INVALID_ARG;
  const long long elem = g->dtype == SMPC_GRID_F16 ? 2 : 4;
  if ((long long)g->nx * g->ny * g->nz * elem >= (1LL << 31)) return SMPC_E_INVALID_ARG;
  if (!finite_all(center, 3) || !finite_all(g->origin, 3) || !std::isfinite(g->voxel) ||
      !(g->voxel > 0.f) || std::isnan(radius) || radius < 0.f)
    return SMPC_E_INVALID_ARG;
  for (int a = 0; a < 3; ++a)
    b.c[a] = (float)(((double)center[a] - (double)g->origin[a]) / (double)g->voxel - 0.5);
  const double r = std::isinf(radius) ? HUGE_VAL : (double)radius / (double)g->voxel + 1.0;
  b.r2 = std::isinf(r) ? HUGE_VALF : (float)(r * r);
  b.g = g;
  b.out = coarse_out;
  return SMPC_OK;
}

// smpc_plan_step, and with `next` the bounds of another grid built by the merge launch.
static smpc_status plan_step_impl(smpc_ctx* ctx, const smpc_plan_args* a, void* stream,
                                  const BallBounds* next) {
  const smpc_status st = validate_args(ctx, a);
  if (st != SMPC_OK) return st;

  LaunchConfig lc = plan_launch_config(a->K, a->H);
  lc.far_pairs = robot_far_pairs(ctx->host_robot);
  const StepParams p = make_params(ctx, a, lc);

  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, SMPC_E_DEVICE, "hipSetDevice(%d) failed", ctx->device);
  const smpc_status rs = ensure_device_robot(ctx);
  if (rs != SMPC_OK) return rs;
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
  const bool f16 = a->esdf.dtype == SMPC_GRID_F16;
  const int e =
      next ? launch_plan_step_bounds(ctx->dev_robot, single_request(a, p, ws), lc, f16,
                                     next->g->data, next->g->dtype == SMPC_GRID_F16, next->g->nx,
                                     next->g->ny, next->g->nz, next->c, next->r2, next->out,
                                     stream, ev)
           : launch_plan_step(ctx->dev_robot, single_request(a, p, ws), lc, f16, stream, ev);
  if (e != 0)
    return fail(ctx, SMPC_E_DEVICE, "kernel launch failed: %s",
                hipGetErrorString(static_cast<hipError_t>(e)));
  return SMPC_OK;
}

smpc_status smpc_plan_step(smpc_ctx* ctx, const smpc_plan_args* a, void* stream) {
  if (!ctx) return SMPC_E_INVALID_ARG;
  if (!a) return fail(ctx, SMPC_E_INVALID_ARG, "args is NULL");
  ctx->last_error.clear();
  return plan_step_impl(ctx, a, stream, nullptr);
}

smpc_status smpc_plan_step_then_bounds(smpc_ctx* ctx, const smpc_plan_args* a,
                                       const smpc_grid* next_grid, const float* center,
                                       float radius, float* coarse_out, void* stream) {
  if (!ctx) return SMPC_E_INVALID_ARG;
  if (!a) return fail(ctx, SMPC_E_INVALID_ARG, "args is NULL");
  ctx->last_error.clear();
  BallBounds nb;
  if (ball_bounds(next_grid, center, radius, coarse_out, nb) != SMPC_OK)
    return fail(ctx, SMPC_E_INVALID_ARG, "invalid next grid, ball or bounds buffer");
  // The table written is the one the step reads, or lies apart from it: the rollouts
  // read theirs while the bounds blocks of the same launch write another.
  const float* rd = a->esdf.coarse;
  if (rd && coarse_out != rd) {
    const uintptr_t r0 = reinterpret_cast<uintptr_t>(rd);
    const uintptr_t w0 = reinterpret_cast<uintptr_t>(coarse_out);
    const uintptr_t r1 = r0 + (uintptr_t)smpc_grid_coarse_cells(a->esdf.nx, a->esdf.ny,
                                                                  a->esdf.nz) * 4u;
    const uintptr_t w1 = w0 + (uintptr_t)smpc_grid_coarse_cells(next_grid->nx, next_grid->ny,
                                                                  next_grid->nz) * 4u;
    if (w0 < r1 && r0 < w1)
      return fail(ctx, SMPC_E_INVALID_ARG,
                  "coarse_out overlaps the table the step reads without being it");
  }
  return plan_step_impl(ctx, a, stream, &nb);
}

smpc_status smpc_plan_step_noalloc(smpc_ctx* ctx, const smpc_plan_args* a, void* stream) {
  if (!ctx) return SMPC_E_INVALID_ARG;
  if (!a) return fail(ctx, SMPC_E_INVALID_ARG, "args is NULL");
  ctx->last_error.clear();
  const smpc_status st = validate_args(ctx, a);
  if (st != SMPC_OK) return st;
  LaunchConfig lc = plan_launch_config(a->K, a->H);
  lc.far_pairs = robot_far_pairs(ctx->host_robot);
  const size_t need = workspace_bytes(a->K, a->H, lc.P);
  if (need > kScratchBytes)
    return fail(ctx, SMPC_E_INVALID_ARG,
                "K=%d, H=%d needs a %zu-byte workspace; the static scratch holds %zu bytes", a->K,
                a->H, need, kScratchBytes);
  if (!ctx->dev_robot || ctx->robot_dirty)
    return fail(ctx, SMPC_E_INVALID_ARG,
                "robot is not on the device yet: run smpc_plan_step once after smpc_set_robot");
  const StepParams p = make_params(ctx, a, lc);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, SMPC_E_DEVICE, "hipSetDevice(%d) failed", ctx->device);
  void* base = nullptr;
  const int se = scratch_address(ctx->device, &base);
  if (se != 0)
    return fail(ctx, SMPC_E_DEVICE, "static scratch lookup failed: %s",
                hipGetErrorString(static_cast<hipError_t>(se)));
  const Workspace ws = carve_workspace(base, a->K, a->H, lc.P);
  const int e = launch_plan_step(ctx->dev_robot, single_request(a, p, ws), lc,
                                 a->esdf.dtype == SMPC_GRID_F16, stream, nullptr);
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

int64_t smpc_grid_coarse_cells(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 2 || ny < 2 || nz < 2) return 0;
  return (int64_t)coarse_cells_1d(nx) * coarse_cells_1d(ny) * coarse_cells_1d(nz);
}

smpc_status smpc_grid_coarse_min(const smpc_grid* g, float* coarse_out, void* stream) {
  if (!g || !g->data || !coarse_out || g->nx < 2 || g->ny < 2 || g->nz < 2 ||
      (g->dtype != SMPC_GRID_F32 && g->dtype != SMPC_GRID_F16))
    return SMPC_E_INVALID_ARG;
  const long long elem = g->dtype == SMPC_GRID_F16 ? 2 : 4;
  if ((long long)g->nx * g->ny * g->nz * elem >= (1LL << 31)) return SMPC_E_INVALID_ARG;
  return launch_grid_coarse_min(g->data, g->dtype == SMPC_GRID_F16, g->nx, g->ny, g->nz,
                                nullptr, 0.f, coarse_out, stream) == 0
             ? SMPC_OK
             : SMPC_E_DEVICE;
}

smpc_status smpc_grid_coarse_min_ball(const smpc_grid* g, const float* center, float radius,
                                      float* coarse_out, void* stream) {
  BallBounds b;
  const smpc_status st = ball_bounds(g, center, radius, coarse_out, b);
  if (st != SMPC_OK) return st;
  return launch_grid_coarse_min(g->data, g->dtype == SMPC_GRID_F16, g->nx, g->ny, g->nz, b.c,
                                b.r2, coarse_out, stream) == 0
             ? SMPC_OK
             : SMPC_E_DEVICE;
}

smpc_status smpc_robot_reach(const smpc_ctx* ctx, float* center_out, float* radius_out) {
  if (!ctx || !center_out || !radius_out || !ctx->robot_set) return SMPC_E_INVALID_ARG;
  // With modified DH the origin of frame i moves by TransX(a_i) and then by d_i along a
  // direction orthogonal to it, so |O_i - O_{i-1}| = sqrt(a_i^2 + d_i^2) exactly, and a
  // sphere centre lies |c| from its frame's origin.  Computed from the float32 values
  // the device uses, with 1 mm for the device's rounding.
  const DevRobot& r = ctx->host_robot;
  double chain[kNdof + 1] = {0.0};  // chain[l]: bound on |O_l|, the origin of frame l
  for (int i = 0; i < kNdof; ++i) chain[i + 1] = chain[i] + std::hypot((double)r.a[i], (double)r.d[i]);
  double reach = 0.0;
  for (int s = 0; s < kSlots; ++s)
    if (r.slot_active & (1u << s))
      reach = std::max(reach, chain[s / kSpl + 1] + std::sqrt((double)r.sc[s][0] * r.sc[s][0] +
                                                             (double)r.sc[s][1] * r.sc[s][1] +
                                                             (double)r.sc[s][2] * r.sc[s][2]));
  for (int a = 0; a < 3; ++a) center_out[a] = 0.f;  // the base is at the world origin
  *radius_out = (float)(reach + 1e-3);
  return SMPC_OK;
}

smpc_status smpc_grid_to_f16(const float* src, void* dst, int64_t n, float clamp, void* stream) {
  if (!src || !dst || n < 0 || !std::isfinite(clamp) || !(clamp > 0.f))
    return SMPC_E_INVALID_ARG;
  if (n == 0) return SMPC_OK;
  return launch_grid_to_f16(src, dst, (long long)n, clamp, stream) == 0 ? SMPC_OK
                                                                        : SMPC_E_DEVICE;
}

size_t smpc_ogm_workspace_bytes(int32_t width, int32_t height) {
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return 0;
  return ((size_t)width * height + kOgmTableFloats) * sizeof(float);
}

smpc_status smpc_ogm_update(smpc_ctx* ctx, const float* q, const float* depth,
                            const smpc_camera* cam, float* log_odds, uint8_t* occ_out,
                            int32_t nx, int32_t ny, int32_t nz, const float* origin, float voxel,
                            const smpc_ogm_params* prm, void* work, size_t work_bytes,
                            void* stream) {
  if (!ctx) return SMPC_E_INVALID_ARG;
  ctx->last_error.clear();
  if (!depth || !cam || !log_odds || !origin || !prm || !work)
    return fail(ctx, SMPC_E_INVALID_ARG, "null pointer argument");
  if (q && !ctx->robot_set) return fail(ctx, SMPC_E_INVALID_ARG, "robot mask without a robot");
  if (q && !finite_all(q, kNdof)) return fail(ctx, SMPC_E_INVALID_ARG, "non-finite q");
  const float intr[] = {cam->fx, cam->fy, cam->cx, cam->cy};
  if (!finite_all(intr, 4) || !(cam->fx > 0.f) || !(cam->fy > 0.f))
    return fail(ctx, SMPC_E_INVALID_ARG, "intrinsics must be finite, fx and fy > 0");
  if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384)
    return fail(ctx, SMPC_E_INVALID_ARG, "image %dx%d outside [1, 16384]", cam->width,
                cam->height);
  if (!std::isfinite(cam->min_depth) || !std::isfinite(cam->max_depth) ||
      !(cam->min_depth > 0.f) || cam->min_depth > cam->max_depth)
    return fail(ctx, SMPC_E_INVALID_ARG, "depth range must satisfy 0 < min <= max");
  const float* T = cam->T_wc;
  if (!finite_all(T, 16)) return fail(ctx, SMPC_E_INVALID_ARG, "non-finite T_wc");
  if (T[12] != 0.f || T[13] != 0.f || T[14] != 0.f || T[15] != 1.f)
    return fail(ctx, SMPC_E_INVALID_ARG, "T_wc last row must be [0 0 0 1]");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double dot = 0.0;
      for (int r = 0; r < 3; ++r) dot += (double)T[r * 4 + i] * (double)T[r * 4 + j];
      if (std::fabs(dot - (i == j ? 1.0 : 0.0)) > 1e-4)
        return fail(ctx, SMPC_E_INVALID_ARG, "T_wc rotation is not orthonormal");
    }
  if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz >= (1LL << 31))
    return fail(ctx, SMPC_E_INVALID_ARG, "grid %dx%dx%d: sides >= 1, fewer than 2^31 voxels",
                nx, ny, nz);
  const size_t need = smpc_ogm_workspace_bytes(cam->width, cam->height);
  if (work_bytes < need || ((uintptr_t)work & 3u))
    return fail(ctx, SMPC_E_INVALID_ARG, "work needs %zu bytes, 4-byte aligned", need);
  if (!finite_all(origin, 3) || !std::isfinite(voxel) || !(voxel > 0.f))
    return fail(ctx, SMPC_E_INVALID_ARG, "origin/voxel must be finite, voxel > 0");
  const float pv[] = {prm->tol, prm->l_hit, prm->l_miss, prm->l_min,
                      prm->l_max, prm->l_occ, prm->robot_pad};
  if (!finite_all(pv, 7) || prm->tol < 0.f || prm->robot_pad < 0.f || prm->l_min > prm->l_max)
    return fail(ctx, SMPC_E_INVALID_ARG,
                "parameters must be finite, tol >= 0, robot_pad >= 0, l_min <= l_max");
  const size_t nvox = (size_t)nx * ny * nz, npix = (size_t)cam->width * cam->height;
  struct Span {
    uintptr_t lo, hi;
  };
  const Span spans[4] = {{(uintptr_t)depth, (uintptr_t)depth + 4 * npix},
                         {(uintptr_t)work, (uintptr_t)work + need},
                         {(uintptr_t)log_odds, (uintptr_t)log_odds + 4 * nvox},
                         {(uintptr_t)occ_out, occ_out ? (uintptr_t)occ_out + nvox : 0}};
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b)
      if (spans[a].lo < spans[b].hi && spans[b].lo < spans[a].hi)
        return fail(ctx, SMPC_E_INVALID_ARG, "depth, work, log_odds and occ_out overlap");

  OgmArgs oa;
  std::memset(&oa, 0, sizeof oa);
  oa.fx = cam->fx;
  oa.fy = cam->fy;
  oa.cx = cam->cx;
  oa.cy = cam->cy;
  oa.width = cam->width;
  oa.height = cam->height;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) oa.R[r * 3 + c] = T[r * 4 + c];
    oa.t[r] = T[r * 4 + 3];
    oa.origin[r] = origin[r];
  }
  oa.min_depth = cam->min_depth;
  oa.max_depth = cam->max_depth;
  oa.use_mask = q ? 1 : 0;
  if (q)
    for (int j = 0; j < kNdof; ++j) oa.q[j] = q[j];
  oa.robot_pad = prm->robot_pad;
  oa.voxel = voxel;
  oa.nx = nx;
  oa.ny = ny;
  oa.nz = nz;
  oa.tol = prm->tol;
  oa.l_hit = prm->l_hit;
  oa.l_miss = prm->l_miss;
  oa.l_min = prm->l_min;
  oa.l_max = prm->l_max;
  oa.l_occ = prm->l_occ;
  {
    // K R^T applied to origin + (i + 1/2) voxel - t, as one affine map of the index.
    const double Kc[3][3] = {{cam->fx, 0.0, cam->cx}, {0.0, cam->fy, cam->cy}, {0.0, 0.0, 1.0}};
    double KRt[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += Kc[r][k] * (double)T[c * 4 + k];  // (R^T)[k][c] = R[c][k]
        KRt[r][c] = acc;
      }
    double p0[3];
    for (int c = 0; c < 3; ++c)
      p0[c] = (double)origin[c] + 0.5 * (double)voxel - (double)T[c * 4 + 3];
    for (int r = 0; r < 3; ++r) {
      double acc = 0.0;
      for (int c = 0; c < 3; ++c) {
        oa.M[r * 3 + c] = (float)(KRt[r][c] * (double)voxel);
        acc += KRt[r][c] * p0[c];
      }
      oa.m[r] = (float)acc;
    }
  }
  oa.inv_nx = 1.0 / (double)nx;
  {
    // Division by an invariant d >= 2 for numerators below 2^31: with l = ceil(log2 d)
    // and mul = ceil(2^(31 + l) / d) < 2^32, n / d = (n * mul) >> (31 + l).
    auto magic = [](uint64_t d, uint32_t& mul, uint32_t& shift) {
      if (d < 2) {
        mul = 0;
        shift = 0;
        return;
      }
      uint32_t l = 0;
      while ((1ull << l) < d) ++l;
      mul = (uint32_t)(((1ull << (31 + l)) + d - 1) / d);
      shift = l - 1;
    };
    magic((uint64_t)nx, oa.nx_mul, oa.nx_shift);
    magic((uint64_t)nx * (uint64_t)ny, oa.plane_mul, oa.plane_shift);
  }
  oa.inv_plane = 1.0 / ((double)nx * (double)ny);

  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, SMPC_E_DEVICE, "hipSetDevice(%d) failed", ctx->device);
  if (q) {
    const smpc_status rs = ensure_device_robot(ctx);
    if (rs != SMPC_OK) return rs;
  }
  if (launch_ogm(q ? ctx->dev_robot : nullptr, oa, depth, log_odds, occ_out,
                 static_cast<float*>(work), (hipStream_t)stream) != 0)
    return fail(ctx, SMPC_E_DEVICE, "occupancy kernel launch failed");
  return SMPC_OK;
}

size_t smpc_edt_workspace_bytes(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1 || nx > kEdtMaxSide || ny > kEdtMaxSide || nz > kEdtMaxSide)
    return 0;
  return edt_workspace_bytes((long long)nx * ny * nz);
}

smpc_status smpc_edt(const uint8_t* occ, int32_t nx, int32_t ny, int32_t nz, float voxel,
                     float* phi_out, uint32_t* d2_out, void* work, size_t work_bytes,
                     void* stream) {
  const size_t need = smpc_edt_workspace_bytes(nx, ny, nz);
  if (!occ || !work || (!phi_out && !d2_out) || need == 0 || work_bytes < need ||
      ((uintptr_t)work & 3u) || !std::isfinite(voxel) || !(voxel > 0.f))
    return SMPC_E_INVALID_ARG;
  const size_t nvox = (size_t)nx * ny * nz;
  struct Span {
    uintptr_t lo, hi;
  };
  const Span spans[4] = {{(uintptr_t)occ, (uintptr_t)occ + nvox},
                         {(uintptr_t)work, (uintptr_t)work + need},
                         {(uintptr_t)phi_out, phi_out ? (uintptr_t)phi_out + 4 * nvox : 0},
                         {(uintptr_t)d2_out, d2_out ? (uintptr_t)d2_out + 8 * nvox : 0}};
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b)
      if (spans[a].lo < spans[b].hi && spans[b].lo < spans[a].hi) return SMPC_E_INVALID_ARG;
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
          hipSuccess)
    return SMPC_E_DEVICE;
  if (edt_lds_bytes(std::max(ny, nz)) > (size_t)max_lds) return SMPC_E_UNSUPPORTED;
  return launch_edt(occ, nx, ny, nz, voxel, phi_out, d2_out, work, (hipStream_t)stream) == 0
             ? SMPC_OK
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
  // Timing-only events: without the system-scope fence (an L2 write-back and
  // invalidate) that a default event performs when it is recorded, which would add to
  // the measured kernel and slow the one after it.
  for (size_t i = 0; i < ctx->prof_events.size(); ++i) {
    if (hipEventCreateWithFlags(&ctx->prof_events[i], hipEventDisableSystemFence) !=
        hipSuccess) {
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

// ---------------------------------------------------------------------------
// Serving
// ---------------------------------------------------------------------------

namespace {

constexpr int kResultStride = 12;  // floats per request: u0[7], stats[4], pad

struct Controller {
  smpc_controller_desc desc;
  LaunchConfig lc;
  size_t ws_bytes = 0;
  float* ubar[2] = {nullptr, nullptr};  // device [H][7] ping-pong
  int cur = 0;                          // buffer holding the current nominal sequence
  int queued = 0;                       // requests queued or in flight
};

struct BatchSlot {
  int n = 0;                            // requests in the batch (0: slot free)
  std::vector<int64_t> tags;
  std::vector<int32_t> ctls;
  hipEvent_t done = nullptr;
  void* ws = nullptr;                   // half of the budget
  // Upload buffers: the batch's request descriptors, then its block maps
  // (k1 blocks + k2 blocks int32), copied host -> device by one graph node.
  size_t up_cap = 0;
  unsigned char* h_up = nullptr;        // pinned
  unsigned char* d_up = nullptr;
  size_t res_cap = 0;                   // requests the result buffers hold
  float* h_res = nullptr;               // pinned [res_cap * kResultStride]
  float* d_res = nullptr;
  void* graph = nullptr;                // the slot's batch graph (launch_batch_graph)
};

}  // namespace

struct smpc_server {
  smpc_ctx* ctx = nullptr;
  size_t budget = 0;
  int max_batch = 1;
  int elem_dtype = -1;
  std::vector<Controller> ctl;
  std::deque<smpc_request> queue;
  std::deque<smpc_completion> done;
  BatchSlot slot[2];
  int oldest = 0;                       // slot of the oldest batch in flight
  int n_in_flight = 0;                  // batches in flight
  std::string last_error;
};

namespace {

smpc_status sfail(smpc_server* s, smpc_status st, const std::string& msg) {
  s->last_error = msg;
  return st;
}

void free_slot(BatchSlot& b) {
  destroy_batch_graph(b.graph);
  if (b.done) (void)hipEventDestroy(b.done);
  if (b.ws) (void)hipFree(b.ws);
  if (b.d_up) (void)hipFree(b.d_up);
  if (b.d_res) (void)hipFree(b.d_res);
  if (b.h_up) (void)hipHostFree(b.h_up);
  if (b.h_res) (void)hipHostFree(b.h_res);
  b = BatchSlot();
}

// Grow a slot's upload and result buffers (only while the slot is free; the graph
// takes the new addresses at its next launch).
bool reserve_slot(BatchSlot& b, size_t up_bytes, size_t reqs) {
  if (up_bytes > b.up_cap) {
    const size_t cap = std::max(up_bytes, 2 * b.up_cap);
    if (b.h_up) (void)hipHostFree(b.h_up);
    if (b.d_up) (void)hipFree(b.d_up);
    b.h_up = nullptr;
    b.d_up = nullptr;
    b.up_cap = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&b.h_up), cap) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&b.d_up), cap) != hipSuccess)
      return false;
    b.up_cap = cap;
  }
  if (reqs > b.res_cap) {
    if (b.h_res) (void)hipHostFree(b.h_res);
    if (b.d_res) (void)hipFree(b.d_res);
    b.h_res = nullptr;
    b.d_res = nullptr;
    b.res_cap = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&b.h_res), reqs * kResultStride * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&b.d_res), reqs * kResultStride * 4) != hipSuccess)
      return false;
    b.res_cap = reqs;
  }
  return true;
}

// The plan-step arguments of request r for controller c (sampling mode).
smpc_plan_args request_args(const Controller& c, const smpc_request& r) {
  smpc_plan_args a;
  std::memset(&a, 0, sizeof a);
  std::memcpy(a.q0, r.q0, sizeof a.q0);
  std::memcpy(a.qd0, r.qd0, sizeof a.qd0);
  std::memcpy(a.T_goal, r.T_goal, sizeof a.T_goal);
  a.esdf = c.desc.esdf;
  a.noise = nullptr;
  a.seed = r.seed;
  std::memcpy(a.sigma, c.desc.sigma, sizeof a.sigma);
  a.K = c.desc.K;
  a.H = c.desc.H;
  a.dt = c.desc.dt;
  a.lambda = c.desc.lambda;
  a.weights = c.desc.weights;
  a.U_in = c.ubar[c.cur];
  a.U_out = c.ubar[1 - c.cur];
  a.costs_out = c.desc.costs_out;
  return a;
}

// Retire finished batches, oldest first.
smpc_status retire(smpc_server* s) {
  while (s->n_in_flight > 0) {
    BatchSlot& b = s->slot[s->oldest];
    const hipError_t q = hipEventQuery(b.done);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) return sfail(s, SMPC_E_DEVICE, "batch event query failed");
    for (int i = 0; i < b.n; ++i) {
      const float* r = b.h_res + (size_t)i * kResultStride;
      smpc_completion c;
      c.tag = b.tags[i];
      c.controller = b.ctls[i];
      c.status = r[kNdof + 3] == 0.f ? SMPC_OK : SMPC_E_NUMERIC;
      std::memcpy(c.u0, r, sizeof c.u0);
      c.S_min = r[kNdof + 0];
      c.Z = r[kNdof + 1];
      c.ess = r[kNdof + 2];
      s->done.push_back(c);
      --s->ctl[b.ctls[i]].queued;
    }
    b.n = 0;
    s->oldest ^= 1;
    --s->n_in_flight;
  }
  return SMPC_OK;
}

// Form and launch one batch in the free slot; returns the number of requests launched.
smpc_status launch_next(smpc_server* s, void* stream, int* launched) {
  *launched = 0;
  const int si = (s->oldest + s->n_in_flight) & 1;
  BatchSlot& b = s->slot[si];
  const size_t half = s->budget / 2;
  std::vector<int> take;
  std::vector<size_t> ws_off;
  std::vector<char> used(s->ctl.size(), 0);
  size_t ws_total = 0, k1_total = 0, k2_total = 0;
  for (size_t i = 0; i < s->queue.size() && (int)take.size() < s->max_batch; ++i) {
    const smpc_request& r = s->queue[i];
    const Controller& c = s->ctl[r.controller];
    if (used[r.controller]) continue;           // one request per controller per batch
    const size_t need = (c.ws_bytes + 255) & ~size_t(255);
    if (ws_total + need > half) continue;        // waits for memory
    used[r.controller] = 1;
    take.push_back((int)i);
    ws_off.push_back(ws_total);
    ws_total += need;
    k1_total += (size_t)c.lc.P;
    k2_total += (size_t)c.lc.k2_blocks;
  }
  if (take.empty()) return SMPC_OK;
  const size_t req_bytes = take.size() * sizeof(Request);
  const size_t up_bytes = req_bytes + (k1_total + k2_total) * sizeof(int32_t);
  if (!reserve_slot(b, up_bytes, (size_t)s->max_batch))
    return sfail(s, SMPC_E_OOM, "batch buffer allocation failed");
  Request* h_reqs = reinterpret_cast<Request*>(b.h_up);
  int32_t* h_maps = reinterpret_cast<int32_t*>(b.h_up + req_bytes);
  const Request* d_reqs = reinterpret_cast<const Request*>(b.d_up);
  const int32_t* d_maps = reinterpret_cast<const int32_t*>(b.d_up + req_bytes);

  size_t lds = 0;
  int k1 = 0, k2 = 0;
  b.tags.assign(take.size(), 0);
  b.ctls.assign(take.size(), 0);
  for (size_t t = 0; t < take.size(); ++t) {
    const smpc_request& r = s->queue[take[t]];
    Controller& c = s->ctl[r.controller];
    const smpc_plan_args a = request_args(c, r);
    Request& q = h_reqs[t];
    std::memset(&q, 0, sizeof q);
    q.p = make_params(s->ctx, &a, c.lc);
    q.grid = a.esdf.data;
    q.coarse = a.esdf.coarse;
    q.noise = nullptr;
    q.U_in = a.U_in;
    q.U_out = a.U_out;
    q.U_star_out = c.desc.U_star_out;
    q.costs_out = c.desc.costs_out;
    q.u0_out = b.d_res + t * kResultStride;
    q.stats_out = b.d_res + t * kResultStride + kNdof;
    q.ws = carve_workspace(static_cast<unsigned char*>(b.ws) + ws_off[t], c.desc.K, c.desc.H,
                           c.lc.P);
    q.k1_begin = k1;
    q.k2_begin = k2;
    q.shift_out = 1;
    for (int j = 0; j < c.lc.P; ++j) h_maps[k1 + j] = (int32_t)t;
    for (int j = 0; j < c.lc.k2_blocks; ++j) h_maps[k1_total + k2 + j] = (int32_t)t;
    k1 += c.lc.P;
    k2 += c.lc.k2_blocks;
    lds = std::max(lds, c.lc.k1_lds);
    c.cur ^= 1;  // the next request of this controller reads this step's result
    b.tags[t] = r.tag;
    b.ctls[t] = r.controller;
  }
  // One graph launch: descriptors and maps up, both batch kernels, results down.
  const int e = launch_batch_graph(&b.graph, s->ctx->dev_robot, b.d_up, b.h_up, up_bytes, d_reqs,
                                   d_maps, (int)k1_total, d_maps + k1_total, (int)k2_total, lds,
                                   s->elem_dtype == SMPC_GRID_F16,
                                   robot_far_pairs(s->ctx->host_robot), b.h_res, b.d_res,
                                   take.size() * kResultStride * 4, stream);
  if (e != 0) return sfail(s, SMPC_E_DEVICE, std::string("batch launch failed: ") +
                                                 hipGetErrorString(static_cast<hipError_t>(e)));
  if (hipEventRecord(b.done, static_cast<hipStream_t>(stream)) != hipSuccess)
    return sfail(s, SMPC_E_DEVICE, "batch event record failed");
  b.n = (int)take.size();
  for (int t = (int)take.size() - 1; t >= 0; --t) s->queue.erase(s->queue.begin() + take[t]);
  ++s->n_in_flight;
  *launched = (int)take.size();
  return SMPC_OK;
}

}  // namespace

extern "C" {

uint64_t smpc_plan_workspace_bytes(int32_t K, int32_t H) {
  if (K < 1 || H < 1 || H > kMaxH) return 0;
  const LaunchConfig lc = plan_launch_config(K, H);
  return (uint64_t)((workspace_bytes(K, H, lc.P) + 255) & ~size_t(255));
}

smpc_status smpc_server_create(smpc_server** out, smpc_ctx* ctx, uint64_t hbm_budget_bytes,
                               int32_t max_batch) {
  if (!out) return SMPC_E_INVALID_ARG;
  *out = nullptr;
  if (!ctx || max_batch < 1 || hbm_budget_bytes < 4096) return SMPC_E_INVALID_ARG;
  if (!ctx->robot_set) return fail(ctx, SMPC_E_INVALID_ARG, "server: no robot set");
  smpc_server* s = new (std::nothrow) smpc_server();
  if (!s) return SMPC_E_OOM;
  s->ctx = ctx;
  s->budget = (size_t)hbm_budget_bytes & ~size_t(511);
  s->max_batch = max_batch;
  DeviceGuard g(ctx->device);
  if (!g.ok || ensure_device_robot(ctx) != SMPC_OK) {
    delete s;
    return SMPC_E_DEVICE;
  }
  for (BatchSlot& b : s->slot) {
    if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&b.ws, s->budget / 2) != hipSuccess) {
      for (BatchSlot& c : s->slot) free_slot(c);
      delete s;
      return SMPC_E_OOM;
    }
  }
  *out = s;
  return SMPC_OK;
}

void smpc_server_destroy(smpc_server* s) {
  if (!s) return;
  DeviceGuard g(s->ctx->device);
  (void)hipDeviceSynchronize();
  for (BatchSlot& b : s->slot) free_slot(b);
  for (Controller& c : s->ctl)
    for (float* u : c.ubar)
      if (u) (void)hipFree(u);
  delete s;
}

smpc_status smpc_server_add_controller(smpc_server* s, const smpc_controller_desc* d,
                                       int32_t* id_out) {
  if (!s) return SMPC_E_INVALID_ARG;
  s->last_error.clear();
  if (!d || !id_out) return sfail(s, SMPC_E_INVALID_ARG, "null argument");
  if (s->elem_dtype >= 0 && d->esdf.dtype != s->elem_dtype)
    return sfail(s, SMPC_E_UNSUPPORTED, "all controllers of a server share one grid dtype");
  Controller c;
  c.desc = *d;
  // Validate like a plan step of this controller (with placeholder buffers).
  smpc_request probe;
  std::memset(&probe, 0, sizeof probe);
  for (int j = 0; j < kNdof; ++j) probe.q0[j] = 0.f;
  probe.T_goal[0] = probe.T_goal[5] = probe.T_goal[10] = probe.T_goal[15] = 1.f;
  float dummy;
  c.ubar[0] = c.ubar[1] = &dummy;
  const smpc_plan_args a = request_args(c, probe);
  if (validate_args(s->ctx, &a) != SMPC_OK)
    return sfail(s, SMPC_E_INVALID_ARG, std::string("controller: ") + s->ctx->last_error);
  c.lc = plan_launch_config(d->K, d->H);
  c.ws_bytes = workspace_bytes(d->K, d->H, c.lc.P);
  if (((c.ws_bytes + 255) & ~size_t(255)) > s->budget / 2)
    return sfail(s, SMPC_E_OOM, "controller workspace exceeds half the HBM budget");
  DeviceGuard g(s->ctx->device);
  const size_t ub = (size_t)d->H * kNdof * sizeof(float);
  c.ubar[0] = c.ubar[1] = nullptr;
  for (float*& u : c.ubar) {
    if (hipMalloc(reinterpret_cast<void**>(&u), ub) != hipSuccess ||
        hipMemset(u, 0, ub) != hipSuccess)
      return sfail(s, SMPC_E_OOM, "controller buffers");
  }
  s->elem_dtype = d->esdf.dtype;
  s->ctl.push_back(c);
  *id_out = (int32_t)s->ctl.size() - 1;
  return SMPC_OK;
}

smpc_status smpc_server_reset_controller(smpc_server* s, int32_t id) {
  if (!s) return SMPC_E_INVALID_ARG;
  if (id < 0 || id >= (int32_t)s->ctl.size()) return sfail(s, SMPC_E_INVALID_ARG, "bad id");
  Controller& c = s->ctl[id];
  if (c.queued) return sfail(s, SMPC_E_INVALID_ARG, "controller has requests outstanding");
  DeviceGuard g(s->ctx->device);
  const size_t ub = (size_t)c.desc.H * kNdof * sizeof(float);
  if (hipMemset(c.ubar[c.cur], 0, ub) != hipSuccess)
    return sfail(s, SMPC_E_DEVICE, "reset failed");
  return SMPC_OK;
}

smpc_status smpc_server_submit(smpc_server* s, const smpc_request* r) {
  if (!s) return SMPC_E_INVALID_ARG;
  s->last_error.clear();
  if (!r) return sfail(s, SMPC_E_INVALID_ARG, "null request");
  if (r->controller < 0 || r->controller >= (int32_t)s->ctl.size() || r->reserved != 0)
    return sfail(s, SMPC_E_INVALID_ARG, "bad controller id");
  Controller& c = s->ctl[r->controller];
  const smpc_plan_args a = request_args(c, *r);
  if (validate_args(s->ctx, &a) != SMPC_OK)
    return sfail(s, SMPC_E_INVALID_ARG, std::string("request: ") + s->ctx->last_error);
  s->queue.push_back(*r);
  ++c.queued;
  return SMPC_OK;
}

smpc_status smpc_server_pump(smpc_server* s, void* stream, int32_t* n_launched) {
  if (!s) return SMPC_E_INVALID_ARG;
  if (n_launched) *n_launched = 0;
  DeviceGuard g(s->ctx->device);
  if (!g.ok) return sfail(s, SMPC_E_DEVICE, "hipSetDevice failed");
  smpc_status st = retire(s);
  if (st != SMPC_OK) return st;
  int total = 0;
  while (s->n_in_flight < 2 && !s->queue.empty()) {
    int n = 0;
    st = launch_next(s, stream, &n);
    if (st != SMPC_OK) return st;
    if (n == 0) break;
    total += n;
  }
  if (n_launched) *n_launched = total;
  return SMPC_OK;
}

smpc_status smpc_server_poll(smpc_server* s, smpc_completion* out, int32_t capacity,
                             int32_t* n_out) {
  if (!s || !n_out || capacity < 0 || (capacity > 0 && !out)) return SMPC_E_INVALID_ARG;
  int n = 0;
  while (n < capacity && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = n;
  return SMPC_OK;
}

int32_t smpc_server_queued(const smpc_server* s) { return s ? (int32_t)s->queue.size() : 0; }

int32_t smpc_server_in_flight(const smpc_server* s) {
  if (!s) return 0;
  int n = 0;
  for (int i = 0; i < s->n_in_flight; ++i) n += s->slot[(s->oldest + i) & 1].n;
  return n;
}

const char* smpc_server_last_error(const smpc_server* s) {
  return s ? s->last_error.c_str() : "null server";
}

}  // extern "C"
