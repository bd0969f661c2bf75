/*
 * smpc.h -- C interface of libsmpc, a gfx950 (MI355X) implementation of one plan
 * step of the sampling-based MPC planner of ParaMaP (arXiv:2512.22575, Sec. IV).
 *
 * One call of smpc_plan_step() performs one pass of the paper's Algorithm 1 for a
 * 7-DoF arm and a given set of K sampled disturbance sequences of length H:
 *
 *   u_k^(m)  = ubar_k + eps_k^(m)                         (eq. 27)
 *   roll out q_{k+1} = f(q_k, u_k) from (q0, qd0)         (eq. 7)
 *   forward kinematics of all link frames                 (eq. 6)
 *   S^(m) = l_f(T_H) + sum_{k<H} l(q_k, x_k, u_k)          (eq. 28, costs eqs. 16-25)
 *   w^(m) = exp(-(S^(m) - S_min)/lambda) / Z               (eq. 29)
 *   U*    = Ubar + sum_m w^(m) eps^(m)                     (eq. 30)
 *
 * Readings of points the paper leaves open, fixed by this interface:
 *   - dynamics: semi-implicit Euler, qd_{k+1} = qd_k + u_k dt, q_{k+1} = q_k + qd_{k+1} dt;
 *   - kinematics: modified DH, A_i = RotX(alpha_i) TransX(a_i) RotZ(q_i) TransZ(d_i),
 *     base at the world origin, end effector = frame 7;
 *   - running terms on (q_k, qd_k, u_k) for k = 0..H-1, terminal pose term on q_H;
 *   - distance field: trilinear between voxel centres, query clamped to the grid;
 *   - joint-limit tightening margin = limit_margin_frac * (max - min) (eq. 21);
 *   - Q_k = diag(w_pose_t I3, w_pose_r I3), Q_H = diag(w_term_t I3, w_term_r I3);
 *   - non-finite rollout costs get weight 0.
 *
 * Conventions
 *   - All floating-point data are IEEE binary32 unless a field says double.
 *   - "device" pointers are HIP device allocations on the context's device;
 *     "host" data are read during the call and not retained.
 *   - Every entry point validates its arguments on the host before any device
 *     work is enqueued; on error nothing is enqueued and a negative status is
 *     returned (details in smpc_last_error()).  No C++ exception crosses this ABI.
 *   - A context is not thread-safe.  Plan steps issued on one stream run in
 *     order; plan steps of one context must not run concurrently on different
 *     streams (they share the context's workspace).
 */
#ifndef SMPC_H
#define SMPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t smpc_status;

enum {
  SMPC_OK = 0,
  SMPC_E_INVALID_ARG = -1, /* argument out of range, null pointer, non-finite value  */
  SMPC_E_OOM = -2,         /* device workspace allocation failed                      */
  SMPC_E_DEVICE = -3,      /* a HIP runtime call or kernel launch failed              */
  SMPC_E_NUMERIC = -4,     /* every rollout cost is non-finite (reported in stats)    */
  SMPC_E_UNSUPPORTED = -5  /* valid request outside what this library implements      */
};

#define SMPC_NDOF 7
#define SMPC_MAX_H 64              /* horizon limit: one rollout fits one wavefront    */
#define SMPC_SPHERES_PER_LINK 4    /* sphere slots per link                            */
#define SMPC_MAX_SPHERES 28        /* 7 links x 4 slots                                */
#define SMPC_MAX_PAIRS 378         /* 28 * 27 / 2                                      */

enum { SMPC_GRID_F32 = 0, SMPC_GRID_F16 = 1 };

typedef struct smpc_ctx smpc_ctx;

/*
 * Robot description (host memory, copied by smpc_set_robot).
 *   a, d, alpha : modified-DH parameters; joint i (1-based) uses entry i-1 (eq. 6).
 *   *_min/_max  : admissible ranges of q, qd and qdd (eqs. 21-22); min < max.
 *   q_ref       : null-space reference posture (eq. 24).
 *   spheres     : n_spheres collision spheres (Sec. IV-B-2, eq. 17); sphere s is
 *                 rigidly attached to frame sphere_link[s] in 1..7, its centre is
 *                 sphere_center[s] in that frame (metres), radius >= 0.  At most
 *                 SMPC_SPHERES_PER_LINK spheres per link.
 *   pairs       : n_pairs self-collision pairs (eq. 18), sphere indices i != j.
 */
typedef struct {
  int32_t n_dof; /* must be SMPC_NDOF */
  double a[SMPC_NDOF];
  double d[SMPC_NDOF];
  double alpha[SMPC_NDOF];
  double q_min[SMPC_NDOF], q_max[SMPC_NDOF];
  double qd_min[SMPC_NDOF], qd_max[SMPC_NDOF];
  double qdd_min[SMPC_NDOF], qdd_max[SMPC_NDOF];
  double q_ref[SMPC_NDOF];
  int32_t n_spheres;
  int32_t sphere_link[SMPC_MAX_SPHERES];
  double sphere_center[SMPC_MAX_SPHERES][3];
  double sphere_radius[SMPC_MAX_SPHERES];
  int32_t n_pairs;
  int32_t pairs[SMPC_MAX_PAIRS][2];
} smpc_robot_desc;

/* Cost weights (Sec. IV-B).  All finite and >= 0; limit_margin_frac in [0, 0.5). */
typedef struct {
  float w_pose_t, w_pose_r;  /* Q_k blocks, running pose cost (eq. 16)     */
  float w_term_t, w_term_r;  /* Q_H blocks, terminal cost (eq. 25)          */
  float w_env, d_act;        /* environment hinge weight and activation (m) */
  float w_self;              /* self-collision hinge weight (eq. 20)        */
  float w_q, w_qd, w_qdd;    /* joint-limit weights (eq. 22)                */
  float limit_margin_frac;   /* tightening margin as a fraction of range    */
  float w_smooth;            /* acceleration smoothness (eq. 23)            */
  float w_ns;                /* null-space regularisation (eq. 24)          */
} smpc_cost_weights;

/*
 * Signed distance grid phi (Sec. IV-B-2, eq. 17), device memory, metres.
 * Layout: element (ix, iy, iz) at index (iz * ny + iy) * nx + ix (x fastest).
 * origin is the corner of voxel (0,0,0); voxel centres are at
 * origin + (i + 1/2) * voxel.  nx, ny, nz >= 2; total size < 2^31 bytes.
 */
typedef struct {
  const void* data;
  int32_t nx, ny, nz;
  int32_t dtype; /* SMPC_GRID_F32, or SMPC_GRID_F16 (IEEE binary16, widened to float32) */
  float origin[3];
  float voxel;
  /* Optional (NULL: none): device float lower bounds of phi per coarse cell, built by
   * smpc_grid_coarse_min from the same grid contents.  A rollout sphere whose cell
   * bound clears its collision threshold skips the trilinear lookup: its hinge is
   * exactly 0 either way, so costs and U* are bitwise the same with or without it.
   * Bounds that do not belong to the grid's current contents give wrong costs. */
  const float* coarse;
} smpc_grid;

/* Edge of a coarse bound cell, in voxels. */
#define SMPC_COARSE_CELL 8

/*
 * Arguments of one plan step.
 *   q0, qd0   : current joint state (host, by value).
 *   T_goal    : target end-effector pose, row-major 4x4 SE(3) (host, by value);
 *               last row must be [0 0 0 1] and the rotation orthonormal to 1e-4.
 *   esdf      : distance grid (device).
 *   noise     : device float [K][H][7] disturbances eps (Algorithm 1, sampling
 *               step), or NULL to sample them on the device from `seed` and
 *               `sigma` (see smpc_sample_noise for the generator).
 *   seed, sigma: sampling mode only: 64-bit Philox key and per-joint standard
 *               deviations (finite, >= 0).
 *   K, H      : samples and horizon; K >= 1, 1 <= H <= SMPC_MAX_H.
 *   dt        : control period (s), finite and > 0.
 *   lambda    : temperature of eq. 29, finite and > 0.
 *   U_in      : device float [H][7], nominal sequence Ubar.
 *   U_out     : device float [H][7], receives U*; may alias U_in (not when receding).
 *   costs_out : device float [K] receiving S^(m), or NULL.
 *   weights_out: device float [K] receiving w^(m), or NULL.
 *   stats_out : device float [4] receiving {S_min, Z, ESS, status}, or NULL;
 *               status is 0, or SMPC_E_NUMERIC when every cost is non-finite (then
 *               U_out = U_in and the weights are 0).  Z = sum_m exp(-(S-S_min)/lambda),
 *               ESS = 1 / sum_m w^2.
 * Receding-horizon execution (Sec. IV-C, last paragraph: the first control of U* is
 * applied for one period and the rest warm-starts the next period; Algorithm 1
 * starts the nominal sequence from zero, so the control shifted in last is 0):
 *   receding  : 0: U_out receives U*.  1: U_out receives [u*_1 .. u*_{H-1}, 0], the
 *               nominal sequence of the next period; U_out must then not overlap U_in.
 *   u0_out    : device-accessible float [7] receiving u*_0, or NULL: device memory,
 *               or pinned host memory (hipHostMalloc), which the merge kernel then
 *               writes directly, so u*_0 is on the host once the step has completed.
 *   state_in  : device float [14] holding (q0, qd0), or NULL to use q0 and qd0 above.
 *               Lets a loop keep its state on the device with no host round trip.
 *   state_out : device float [14] receiving the state one period dt later when u*_0
 *               is applied with the rollouts' integrator: qd' = qd0 + u*_0 dt,
 *               q' = q0 + qd' dt; or NULL.
 *   No output (u0_out, state_out) may overlap an input (U_in, state_in).  When no
 *   cost is finite u*_0 = ubar_0 is executed.
 * All work is enqueued on `stream` (a hipStream_t; NULL = default stream) and the
 * call returns without waiting for it.
 */
typedef struct {
  float q0[SMPC_NDOF];
  float qd0[SMPC_NDOF];
  float T_goal[16];
  smpc_grid esdf;
  const float* noise;
  uint64_t seed;
  float sigma[SMPC_NDOF];
  int32_t K;
  int32_t H;
  float dt;
  float lambda;
  smpc_cost_weights weights;
  const float* U_in;
  float* U_out;
  float* costs_out;
  float* weights_out;
  float* stats_out;
  int32_t receding;
  float* u0_out;
  const float* state_in;
  float* state_out;
} smpc_plan_args;

/* Create a context on HIP device `hip_device`.  *out receives the handle. */
smpc_status smpc_create(smpc_ctx** out, int32_t hip_device);

/* Destroy a context and free its device memory (waits for the device). NULL is a no-op. */
void smpc_destroy(smpc_ctx* ctx);

/* Validate a robot description and copy it into the context (host memory; no device
 * call).  The next smpc_plan_step uploads it to the device. */
smpc_status smpc_set_robot(smpc_ctx* ctx, const smpc_robot_desc* desc);

/* Validate `args` and enqueue one plan step on `stream` (asynchronous). */
smpc_status smpc_plan_step(smpc_ctx* ctx, const smpc_plan_args* args, void* stream);

/* Bytes of the static device array that smpc_plan_step_noalloc takes its workspace from. */
#define SMPC_NOALLOC_SCRATCH_BYTES (4u << 20)

/*
 * smpc_plan_step for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same validation,
 * kernels and results as smpc_plan_step, but the workspace is a static device array of
 * SMPC_NOALLOC_SCRATCH_BYTES per device (held until the process ends) instead of the
 * context's arena, and no hipMalloc or hipFree is called.
 *   - The robot must already be on the device: smpc_plan_step has run on this context
 *     since its last smpc_set_robot.  Otherwise SMPC_E_INVALID_ARG.
 *   - smpc_plan_workspace_bytes(K, H) <= SMPC_NOALLOC_SCRATCH_BYTES (K up to 21246 at
 *     H = 40, 9116 at H = 64), else SMPC_E_INVALID_ARG; nothing is enqueued on any
 *     error.
 *   - All calls on one device share that device's array and it keeps the last call's
 *     contents (nothing in it needs to start at zero): calls that may overlap on one
 *     device (other streams, other contexts) race and must be ordered by the caller.
 */
smpc_status smpc_plan_step_noalloc(smpc_ctx* ctx, const smpc_plan_args* args, void* stream);

/* Static description of a status code. */
const char* smpc_status_string(smpc_status status);

/* Detail of the last failure on this context ("" if none).  Valid until the next call. */
const char* smpc_last_error(const smpc_ctx* ctx);

/*
 * The disturbances that smpc_plan_step samples when noise == NULL (Algorithm 1's
 * sampling step with D = N(0, diag(sigma^2))): for rollout m and step k the
 * Philox4x32-10 generator (Salmon et al., SC'11) with key = seed (low word first)
 * is evaluated at counters n = 2 (m H + k) and n + 1, each as (n mod 2^32,
 * n >> 32, 0, 0); every 32-bit word w gives u = ((w >> 9) + 1/2) 2^-23; Box-Muller
 * turns (u0, u1) into (sqrt(-2 ln u0) cos 2 pi u1, sqrt(-2 ln u0) sin 2 pi u1); the
 * first counter's words give joints 0..3, the second's joints 4..6.
 *   eps_out   : device float [K][H][7] receiving sigma_j z_j, or NULL;
 *   words_out : device uint32 [K][H][8] receiving the raw words, or NULL.
 * At least one output must be non-NULL; 1 <= H <= SMPC_MAX_H; K*H*8 < 2^31.
 * Runs on the device current to the calling thread, asynchronously on `stream`.
 */
smpc_status smpc_sample_noise(uint64_t seed, int32_t K, int32_t H, const float* sigma,
                              float* eps_out, uint32_t* words_out, void* stream);

/*
 * Convert a float32 grid (device, n elements) into binary16 (device, n elements,
 * stored as uint16 bit patterns): each value is clamped to [-clamp, clamp] and
 * rounded to the nearest float16 (ties to even).  clamp finite and > 0.
 * Runs on the device current to the calling thread, asynchronously on `stream`.
 */
smpc_status smpc_grid_to_f16(const float* src, void* dst, int64_t n, float clamp, void* stream);

/*
 * Number of coarse cells of a grid: cx(n) = ceil((n - 1) / SMPC_COARSE_CELL) per
 * axis, cx(nx) * cx(ny) * cx(nz) in all; 0 when a side is < 2.
 */
int64_t smpc_grid_coarse_cells(int32_t nx, int32_t ny, int32_t nz);

/*
 * Lower bounds of trilinear phi for smpc_grid.coarse.  Cell (cx, cy, cz), stored at
 * (cz * ncy + cy) * ncx + cx, covers the lookups whose lower corner index i0 (R5:
 * min(floor(u), n - 2) per axis) lies in [8 c, 8 c + 7]; its bound is the minimum
 * of phi over voxels [8 c, min(8 c + 8, n - 1)] per axis, minus 1e-5 m + 2^-18 times
 * the largest |phi| there, which covers float32 rounding in the interpolation.
 *   grid      : host struct describing the device grid (data, sizes, dtype; its
 *               `coarse` field is ignored).
 *   coarse_out: device float [smpc_grid_coarse_cells(nx, ny, nz)].
 * Runs on the device current to the calling thread, asynchronously on `stream`.
 */
smpc_status smpc_grid_coarse_min(const smpc_grid* grid, float* coarse_out, void* stream);

/*
 * smpc_grid_coarse_min for the lookups of points within `radius` metres of `center`
 * (world frame, the frame of grid->origin; grid->origin and grid->voxel are used):
 * cells that no such lookup reaches (R5's clamping included) get -inf, which never lets
 * a lookup be skipped, so a plan step stays exact wherever its spheres go; the others
 * get smpc_grid_coarse_min's bound.  Rows of cells outside the ball are not read.
 * radius = +inf gives smpc_grid_coarse_min's table; center finite, radius >= 0.
 * With smpc_robot_reach's ball a table holds a bound for every cell the arm can query.
 * Runs on the device current to the calling thread, asynchronously on `stream`.
 */
smpc_status smpc_grid_coarse_min_ball(const smpc_grid* grid, const float center[3],
                                      float radius, float* coarse_out, void* stream);

/*
 * smpc_plan_step (Alg. 1 for args `a`), and smpc_grid_coarse_min_ball of `next_grid`
 * (the map of the next control period in a receding-horizon loop, Sec. IV-C) into
 * `coarse_out`, built by the step's own launches: the results are those of the two
 * calls made one after the other.
 *   next_grid, center, radius, coarse_out: as smpc_grid_coarse_min_ball.
 *   coarse_out is either the table `a` reads (a->esdf.coarse) or does not overlap it
 *   (else SMPC_E_INVALID_ARG).  Apart from it, the bounds blocks run beside the rollouts
 *   (eqs. 17-28) in their launch; as that table, they run beside the merge of the
 *   rollouts (eqs. 29-30), which starts after the rollouts have read it and never reads
 *   it.  coarse_out must not overlap the step's other outputs.
 * When next_grid's dtype differs from a->esdf's, or its rows are not a multiple of 16
 * bytes in a 16-byte-aligned grid, the bounds are built by a launch of their own after
 * the step.  Argument errors return SMPC_E_INVALID_ARG before anything is enqueued.
 * Runs on the context's device, asynchronously on `stream`.
 */
smpc_status smpc_plan_step_then_bounds(smpc_ctx* ctx, const smpc_plan_args* a,
                                       const smpc_grid* next_grid, const float center[3],
                                       float radius, float* coarse_out, void* stream);

/*
 * A ball holding every sphere centre of the context's robot at any joint values: the
 * base (the world origin, R3) and radius max over spheres s on link l of
 * sum_{i <= l} sqrt(a_i^2 + d_i^2) + |c_s|, plus 1 mm (with modified DH each joint moves
 * the frame origin by exactly sqrt(a_i^2 + d_i^2)).
 * SMPC_E_INVALID_ARG when no robot is set.  Host only.
 */
smpc_status smpc_robot_reach(const smpc_ctx* ctx, float center_out[3], float* radius_out);

/* ---- Occupancy mapping (Sec. III-A) with the robot mask (Remark 2) ----------- */

/* Pinhole depth camera.  Pixel (i, j) covers [i, i + 1) x [j, j + 1) in image
 * coordinates u = fx x / z + cx, v = fy y / z + cy of a camera-frame point (x, y, z);
 * depth is the camera-frame z of the return. */
typedef struct {
  float fx, fy, cx, cy;         /* intrinsics (pixels), fx, fy > 0 */
  int32_t width, height;        /* image size, each in [1, 16384] */
  float T_wc[16];               /* camera-to-world pose, row-major SE(3) */
  float min_depth, max_depth;   /* returns outside [min_depth, max_depth] are no return */
} smpc_camera;

/* Occupancy update parameters (log-odds). */
typedef struct {
  float tol;                    /* |z - d| <= tol: the voxel is on the surface (m), >= 0 */
  float l_hit, l_miss;          /* increments for occupied (> 0) and free (< 0) voxels */
  float l_min, l_max;           /* clamp, l_min <= l_max */
  float l_occ;                  /* a voxel is occupied when its log-odds exceeds l_occ */
  float robot_pad;              /* padding of the robot sphere model (m), >= 0 */
} smpc_ogm_params;

/* Device workspace smpc_ogm_update needs for a width x height image (bytes); 0 when
 * a size is out of range. */
size_t smpc_ogm_workspace_bytes(int32_t width, int32_t height);

/*
 * One occupancy update by voxel projection (Sec. III-A): every voxel centre is
 * projected into the depth image, reads the pixel whose square contains the
 * projection, and is classified against that pixel's depth d by its camera-frame
 * z: |z - d| <= tol occupied (log-odds + l_hit), z < d - tol free (+ l_miss), else
 * unknown (unchanged); voxels behind the camera, outside the image or on a pixel
 * without a return are unknown; log-odds are clamped to [l_min, l_max].
 * Robot mask (Remark 2), when q is given: the robot's collision spheres at joint
 * positions q, each padded by robot_pad, are computed on the device; returns whose
 * back-projected point (pixel centre at depth d) lies in a padded sphere are
 * discarded before the update, and voxels whose centre lies in one are set to l_min.
 *   ctx       : context; its robot must be set when q is given.
 *   q         : host float[7] joint positions, or NULL (no mask).
 *   depth     : device float [height][width] (metres; non-finite or out of range:
 *               no return).
 *   cam, prm  : host structs.
 *   log_odds  : device float [nz][ny][nx] (x fastest), updated in place.
 *   occ_out   : device uint8 [nz][ny][nx] (1 = occupied), or NULL.
 *   origin    : host float[3], corner of voxel (0,0,0); voxel edge in metres.
 *   work      : device scratch of smpc_ogm_workspace_bytes(width, height) bytes,
 *               4-byte aligned; on return its first width * height floats hold the
 *               depth image with the discarded returns set to 0.
 * nx * ny * nz < 2^31.  Runs asynchronously on `stream`.
 */
smpc_status smpc_ogm_update(smpc_ctx* ctx, const float* q, const float* depth,
                            const smpc_camera* cam, float* log_odds, uint8_t* occ_out,
                            int32_t nx, int32_t ny, int32_t nz, const float* origin, float voxel,
                            const smpc_ogm_params* prm, void* work, size_t work_bytes,
                            void* stream);

/* ---- Distance field construction (Sec. III-B) ------------------------------- */

/* Longest grid side smpc_edt accepts, in voxels. */
#define SMPC_EDT_MAX_SIDE 512

/*
 * Device workspace smpc_edt needs for an nx x ny x nz grid: eight bytes per voxel.
 * Returns 0 when a side lies outside [1, SMPC_EDT_MAX_SIDE].
 */
size_t smpc_edt_workspace_bytes(int32_t nx, int32_t ny, int32_t nz);

/*
 * Signed distance field of an occupancy grid, the map the planner reads
 * (Sec. III-B: occupied voxels are zero-distance sources of an exact separable
 * squared Euclidean distance transform built from 1-D Felzenszwalb-Huttenlocher
 * passes).
 *   occ       : device uint8 [nz][ny][nx] (x fastest); nonzero = occupied.
 *   voxel     : voxel edge in metres, finite and > 0.
 *   phi_out   : device float [nz][ny][nx], or NULL:
 *               phi = voxel * (sqrt(D_out) - sqrt(D_in)), evaluated in float64 and
 *               rounded to float32 -- positive in free space, negative inside
 *               obstacles, in the layout smpc_grid expects.
 *   d2_out    : device uint32 [2][nz][ny][nx], or NULL: [0] = D_out, the squared
 *               index distance from each voxel centre to the nearest occupied one,
 *               [1] = D_in, to the nearest free one (each 0 on its own sources;
 *               nx^2 + ny^2 + nz^2 everywhere when the grid holds no such voxel).
 *   work      : device scratch of at least smpc_edt_workspace_bytes(nx, ny, nz)
 *               bytes, 4-byte aligned.
 * At least one of phi_out and d2_out is non-NULL; no two of occ, phi_out, d2_out
 * and work overlap.  Each side must lie in [1, SMPC_EDT_MAX_SIDE];
 * SMPC_E_UNSUPPORTED when the device cannot give one block the LDS the longer of
 * ny and nz needs (about 270 bytes per voxel of that side, 200 when both are at
 * most 255).
 * Runs on the device current to the calling thread, asynchronously on `stream`;
 * the caller owns every buffer.
 */
smpc_status smpc_edt(const uint8_t* occ, int32_t nx, int32_t ny, int32_t nz, float voxel,
                     float* phi_out, uint32_t* d2_out, void* work, size_t work_bytes,
                     void* stream);

/*
 * Per-kernel timing (profiling aid).  smpc_profile_enable(ctx, n) makes the next n
 * plan steps record HIP events on their stream before the rollout-cost kernel,
 * between the two kernels and after the merge kernel; n = 0 disables recording.
 * smpc_profile_read waits for the recorded events and returns, per recorded
 * step, the durations in milliseconds of the rollout-cost kernel (rollout_ms[i])
 * and of the merge kernel (merge_ms[i]) -- for smpc_plan_step_then_bounds, of the
 * launch among the two that also held the next grid's bounds, or of the bounds'
 * own launch after the merge when neither could; *n_steps receives the count written
 * (at most `capacity`).  Reading resets the record.  Events are created by
 * smpc_profile_enable, for timing only: they carry no system-scope memory fence, so
 * waiting for them does not make the step's outputs visible to the host (synchronise
 * the stream for that).  Both calls return SMPC_E_DEVICE on HIP failures.
 */
smpc_status smpc_profile_enable(smpc_ctx* ctx, int32_t n_steps);
smpc_status smpc_profile_read(smpc_ctx* ctx, float* rollout_ms, float* merge_ms,
                              int32_t capacity, int32_t* n_steps);

/* ------------------------------------------------------------------------------
 * Serving: many independent controllers, each with a resident distance grid and a
 * resident warm-started nominal sequence, served by continuous batching.
 *
 * A request is one plan step of one controller from the joint state and target it
 * carries; the disturbances are sampled on the device from the request's seed (see
 * smpc_sample_noise).  The server keeps a FIFO queue; smpc_server_pump() retires
 * finished batches and forms new ones from the queue in arrival order -- at most one
 * request per controller per batch, and only while the batch's workspace fits in
 * half of the HBM budget (a request that can never fit is refused at submit) -- and
 * launches each batch as one rollout-cost launch and one merge launch covering all
 * of its requests.  Up to two batches are in flight, so requests that arrive while
 * one batch runs are admitted into the next, which is queued behind it on the device.
 * After a step, the controller's nominal sequence becomes [u*_1 .. u*_{H-1}, 0]
 * (receding horizon) and u*_0 is returned in the completion.  A request's result is
 * bitwise the same whether it runs alone or in a batch.
 * The server is not thread-safe; all its work runs on the stream given to pump.
 * ------------------------------------------------------------------------------ */
typedef struct smpc_server smpc_server;

/* A controller: its grid (device memory owned by the caller, valid while the
 * controller exists) and the constants of its plan steps.  The grid dtype must be
 * the same for every controller of a server. */
typedef struct {
  smpc_grid esdf;
  int32_t K, H;
  float dt;
  float lambda;
  smpc_cost_weights weights;
  float sigma[SMPC_NDOF];
  /* Optional device outputs (NULL: not written), overwritten by each served request of
   * this controller and valid once its completion has been polled: U* before the
   * receding-horizon shift, [H][7], and the rollout costs, [K]. */
  float* U_star_out;
  float* costs_out;
} smpc_controller_desc;

typedef struct {
  int64_t tag;        /* caller's identifier, returned in the completion */
  int32_t controller; /* id from smpc_server_add_controller */
  int32_t reserved;   /* must be 0 */
  float q0[SMPC_NDOF];
  float qd0[SMPC_NDOF];
  float T_goal[16];
  uint64_t seed;      /* sampling seed of this step */
} smpc_request;

typedef struct {
  int64_t tag;
  int32_t controller;
  int32_t status;     /* SMPC_OK, or SMPC_E_NUMERIC when no rollout cost was finite */
  float u0[SMPC_NDOF];/* u*_0, the control to execute */
  float S_min, Z, ess;
} smpc_completion;

/* Device workspace bytes one plan step of K rollouts and horizon H uses (0 if the
 * sizes are invalid); a server needs twice the largest of its controllers' values. */
uint64_t smpc_plan_workspace_bytes(int32_t K, int32_t H);

/* Create a server on `ctx` (which must hold the robot).  hbm_budget_bytes bounds the
 * device memory of requests in flight; max_batch bounds requests per batch (>= 1). */
smpc_status smpc_server_create(smpc_server** out, smpc_ctx* ctx, uint64_t hbm_budget_bytes,
                               int32_t max_batch);
/* Destroy a server (waits for its work).  NULL is a no-op. */
void smpc_server_destroy(smpc_server* server);
/* Register a controller; its nominal sequence starts at 0.  *id_out receives its id. */
smpc_status smpc_server_add_controller(smpc_server* server, const smpc_controller_desc* desc,
                                       int32_t* id_out);
/* Set a controller's nominal sequence back to 0 (synchronous; no request of it may be
 * queued or in flight). */
smpc_status smpc_server_reset_controller(smpc_server* server, int32_t id);
/* Queue a request (validated on the host; nothing is launched). */
smpc_status smpc_server_submit(smpc_server* server, const smpc_request* request);
/* Retire finished batches and launch new ones on `stream`; never waits for the device.
 * *n_launched (optional) receives the number of requests launched by this call. */
smpc_status smpc_server_pump(smpc_server* server, void* stream, int32_t* n_launched);
/* Move up to `capacity` completions, oldest first, into `out`; *n_out receives the count. */
smpc_status smpc_server_poll(smpc_server* server, smpc_completion* out, int32_t capacity,
                             int32_t* n_out);
/* Requests queued (not yet launched) and in flight (launched, not yet retired). */
int32_t smpc_server_queued(const smpc_server* server);
int32_t smpc_server_in_flight(const smpc_server* server);
/* Detail of the last failure of a server call ("" if none). */
const char* smpc_server_last_error(const smpc_server* server);

/* Library version as major*10000 + minor*100 + patch. */
int32_t smpc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SMPC_H */
