// Internal layouts shared by the host runtime and the gfx950 kernels of libsmpc.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#include "smpc.h"

namespace smpc {

constexpr int kNdof = SMPC_NDOF;
constexpr int kSpl = SMPC_SPHERES_PER_LINK;   // sphere slots per link
constexpr int kSlots = kNdof * kSpl;          // slot s = (link - 1) * kSpl + j
constexpr int kMaxPairs = SMPC_MAX_PAIRS;
constexpr int kMaxH = SMPC_MAX_H;
constexpr int kK1Threads = 256;               // rollout-cost block size (4 waves)
constexpr int kK2Threads = 256;               // reduce/update block size
constexpr int kOutPerBlock = 8;               // U* outputs merged per K2 block
constexpr int kWeightsPerBlock = 1024;        // weights_out elements per K2 block

// Self-collision constants of one link pair (la <= lb): bit i * kSpl + j of mask marks
// the pair (slot la*kSpl+i, slot lb*kSpl+j).  One record, so that a group's constants
// arrive in a few wide scalar loads.
struct alignas(16) LinkPair {
  uint32_t mask;
  float bthr;                  // (R_la + R_lb)^2 of the link bounding spheres
  uint32_t pad_[2];
  float sthr[kSpl];            // (r_i + R_lb)^2: sphere i of la vs lb's bound
  float rr2[kSpl * kSpl];      // (r_i + r_j)^2 per pair (0 if not a pair)
  float rs[kSpl * kSpl];       // r_i + r_j
};

// Robot constants in device memory.  Every field is read at a wave-uniform
// address, so the kernels fetch it with scalar loads.
struct DevRobot {
  float ca[kNdof], sa[kNdof];  // cos/sin of alpha_i (computed in double on the host)
  float a[kNdof], d[kNdof];
  float sc[kSlots][4];         // sphere slot centre (x, y, z) in its link frame, radius
  uint32_t slot_active;        // bit s set when slot s holds a sphere
  uint32_t pad0_[3];
  // Self-collision pairs grouped by link pair, index la * kNdof + lb.
  LinkPair lp[kNdof * kNdof];
  float lbound[kNdof];         // bounding radius of each link's spheres about its slot-0 sphere
  int32_t n_pairs;             // distinct pairs after de-duplication
  int32_t pad_[3];
  // The same pairs as records (slot a, slot b as int bits, (r_a + r_b)^2, r_a + r_b).
  float4 pair_rec[kMaxPairs];
};

// Margin added to each link bounding radius (metres).  Float32 sphere positions
// are accurate to ~1e-6 m, so a pair culled by the bounding test has a hinge of
// exactly 0 in the per-pair test as well.
constexpr double kBoundMargin = 1e-4;

// Per-call constants, passed by value as a kernel argument.
struct StepParams {
  float q0[kNdof], qd0[kNdof];
  float RgT[9];                // R_g^T, row-major
  float tgr[3];                // R_g^T t_g
  float qlo[kNdof], qhi[kNdof];      // tightened limits (eq. 21)
  float qdlo[kNdof], qdhi[kNdof];
  float qddlo[kNdof], qddhi[kNdof];
  float qref[kNdof];
  float env_thr[kSlots];       // d_act + r_s; hinge is max(0, env_thr - phi)
  float w_pose_t, w_pose_r, w_term_t, w_term_r;
  float w_env, w_self, w_q, w_qd, w_qdd, w_smooth, w_ns;
  float inv_voxel;             // 1 / voxel
  float gcx, gcy, gcz;         // -origin / voxel - 1/2 per axis (continuous-index offset)
  float inv_voxel8, gc8[3];    // the same divided by 8 (exactly: coarse-cell coordinates)
  int32_t nx, ny, nz;
  uint32_t grid_bytes;
  int32_t ncx, ncy, ncz;       // coarse bound cells per axis
  uint32_t coarse_bytes;       // 0: no coarse bounds
  float cmax[3];               // ncx - 1, ncy - 1, ncz - 1
  float cstride[2];            // ncx, ncx * ncy (cell index strides)
  int32_t K, H, R, P;          // samples, horizon, rollouts per K1 block, K1 blocks
  float dt;
  float k_lambda;              // log2(e) / lambda (softmax factors by exp2)
  uint32_t seed_lo, seed_hi;   // sampling mode: Philox key
  float sigma[kNdof];          // sampling mode: per-joint standard deviation
};

struct SigmaArg {
  float v[kNdof];
};

// Device workspace carved from one allocation.
struct Workspace {
  double* S;        // [K]   per-rollout cost without the k = 0 state terms
  double* part_m;   // [P]   per-block minimum of S (+inf when the block has none finite)
  float* part_Z;    // [P]   sum_m exp(-(S - part_m)/lambda)
  float* part_Z2;   // [P]   sum_m exp(-2 (S - part_m)/lambda)
  float* part_N;    // [HO8 / 8][P][8] sum_m exp(-(S - part_m)/lambda) eps^(m) per output
                    // chunk of 8 (HO8 = 7H padded to 8), chunk-major
  float* c0;        // [1]   state terms of state 0 (when computed by the rollout launch)
};

// One plan step as the kernels see it (by value for a single step, in a device
// array for a batch).
struct Request {
  StepParams p;
  const void* grid;            // device distance grid
  const float* coarse;         // device coarse lower bounds of the grid, or null
  const float* noise;          // device [K][H][7], or null: sample on the device
  const float* U_in;           // device [H][7]
  float* U_out;                // device [H][7]
  float* costs_out;            // device [K] or null
  float* weights_out;          // device [K] or null
  float* stats_out;            // device [4] or null
  float* u0_out;               // device [7] or null: receives u*_0
  const float* state_in;       // device [14] (q0, qd0), or null: p.q0 and p.qd0
  float* state_out;            // device [14] or null: state after executing u*_0 for dt
  float* U_star_out;           // device [H][7] or null: U* (unshifted) besides U_out
  Workspace ws;
  int32_t k1_begin;            // first rollout-cost block of this request in a batch
  int32_t k2_begin;            // first merge block of this request in a batch
  int32_t shift_out;           // 1: U_out = [u*_1 .. u*_{H-1}, 0] (receding horizon)
  int32_t c0_in_ws;            // 1: an extra rollout-launch block leaves c0 in ws.c0
};

struct LaunchConfig {
  int R;            // rollouts per K1 block
  int k1_threads;   // K1 block size (multiple of 64)
  int P;            // number of K1 blocks
  size_t k1_lds;    // dynamic LDS bytes of K1
  int k2_blocks;    // K2 grid
  bool far_pairs = false;  // every self-collision pair joins links two or more apart
};

// Whether every self-collision pair of the robot joins links two or more apart (the
// link-pair groups of a link with itself and with its neighbour are empty).
inline bool robot_far_pairs(const DevRobot& r) {
  for (int la = 0; la < kNdof; ++la)
    for (int lb = la; lb < kNdof && lb <= la + 1; ++lb)
      if (r.lp[la * kNdof + lb].mask != 0u) return false;
  return true;
}

LaunchConfig plan_launch_config(int K, int H);
size_t workspace_bytes(int K, int H, int P);
Workspace carve_workspace(void* base, int K, int H, int P);

// Static device scratch of smpc_plan_step_noalloc (one per device).
constexpr size_t kScratchBytes = SMPC_NOALLOC_SCRATCH_BYTES;
constexpr int kScratchDevices = 64;
// Device address of the scratch on `device`, which must be current (looked up once per
// device).  Returns a hipError_t value (0 = success).
int scratch_address(int device, void** out);

// Enqueue both kernels of one plan step.  Returns a hipError_t value (0 = success).
// When `events` is non-null, events[0..2] (hipEvent_t) are recorded before the
// rollout-cost kernel, between the kernels and after the merge kernel.
int launch_plan_step(const DevRobot* robot, const Request& q, const LaunchConfig& lc, bool f16,
                     void* stream, void* events);

// launch_plan_step whose launches also build the coarse bounds of another grid,
// restricted to a ball (as launch_grid_coarse_min with ball_c non-null): in the rollout
// launch when `out` is not the table the step reads (the two must not overlap), else in
// the merge launch; when the grid is not fit for either (another element type, rows not
// a multiple of 16 bytes, unaligned) the bounds follow the plan step in a launch of
// their own.
int launch_plan_step_bounds(const DevRobot* robot, const Request& q, const LaunchConfig& lc,
                            bool f16, const void* grid, bool grid_f16, int nx, int ny, int nz,
                            const float* ball_c, float ball_r2, float* out, void* stream,
                            void* events);

// A batch of requests (device array `reqs`; block maps k1_map [k1_blocks] and k2_map
// [k2_blocks] give each block's request index) as one HIP graph (descriptor upload,
// both batch kernels, result download),
// created at the first launch and re-parameterised for every later one.  `*graph` is
// the slot's handle (null before the first launch); the caller relaunches it only after
// the previous launch has completed (a launch for a robot of the other pair kind, `far`,
// rebuilds the graph).  up: host -> device bytes (descriptors and maps);
// res: device -> host result bytes.  Returns a hipError_t value.
int launch_batch_graph(void** graph, const DevRobot* robot, void* d_up, const void* h_up,
                       size_t up_bytes, const Request* reqs, const int32_t* k1_map,
                       int k1_blocks, const int32_t* k2_map, int k2_blocks, size_t k1_lds,
                       bool f16, bool far, void* h_res, const void* d_res, size_t res_bytes,
                       void* stream);
void destroy_batch_graph(void* graph);

// Disturbances of the sampling mode written to memory (eps [K][H][7], words [K][H][8];
// either may be null).  Returns a hipError_t value.
int launch_sample_noise(uint64_t seed, int K, int H, const float* sigma, float* eps,
                        uint32_t* words, void* stream);

// float32 -> float16 grid conversion with clamping.  Returns a hipError_t value.
int launch_grid_to_f16(const float* src, void* dst, long long n, float clamp, void* stream);
constexpr int kCoarseCell = SMPC_COARSE_CELL;
constexpr int kCoarseShift = 3;  // log2(kCoarseCell)
static_assert((1 << kCoarseShift) == kCoarseCell, "coarse cell edge");
inline int coarse_cells_1d(int n) { return (n - 2) / kCoarseCell + 1; }
// Coarse bounds; ball_c (3 floats, continuous-index units) and ball_r2 restrict them to
// the cells the lookups of a ball reach (the others get -inf); ball_c null: every cell.
int launch_grid_coarse_min(const void* grid, bool f16, int nx, int ny, int nz,
                           const float* ball_c, float ball_r2, float* out, void* stream);

// Occupancy update (smpc_ogm_update): everything the two kernels need, by value.
struct OgmArgs {
  float fx, fy, cx, cy;
  int32_t width, height;
  float R[9];                  // camera-to-world rotation, row-major
  float t[3];                  // camera position
  float min_depth, max_depth;
  float q[kNdof];              // joint positions of the robot mask
  int32_t use_mask;
  float robot_pad;
  float origin[3];
  float voxel;
  int32_t nx, ny, nz;
  float tol, l_hit, l_miss, l_min, l_max, l_occ;
  // Voxel (ix, iy, iz) -> (X, Y, Z) = M (ix, iy, iz) + m: Z is the camera-frame depth
  // of the voxel centre and (X / Z, Y / Z) its image coordinates (u, v).
  float M[9], m[3];
  double inv_nx, inv_plane;    // 1 / nx and 1 / (nx ny) for the voxel index split
  // n / d = umulhi(n, mul) >> shift for n < 2^31 (d = nx and nx ny; set when nx >= 2)
  uint32_t nx_mul, nx_shift, plane_mul, plane_shift;
};
// Sphere table after the cleaned image: per slot centre and padded radius^2, the
// bounding box of the padded spheres in metres (6 floats) and in voxel indices
// widened by one voxel (6 int32: x, y, z lower bounds, then upper bounds).
// Workspace: cleaned image (npix floats), then the sphere table (kOgmTableFloats).
constexpr int kOgmTableFloats = 128;
constexpr int kOgmBox = kSlots * 4;
constexpr int kOgmIndexBox = kOgmBox + 6;
constexpr int kOgmSphereFloats = kOgmIndexBox + 6;
static_assert(kOgmSphereFloats <= kOgmTableFloats, "sphere table fits its slot");
int launch_ogm(const DevRobot* robot, const OgmArgs& a, const float* depth, float* log_odds,
               uint8_t* occ, float* work, hipStream_t stream);

constexpr int kEdtMaxSide = SMPC_EDT_MAX_SIDE;
// Signed distance field from occupancy (smpc_edt.hip); sizes already validated.
size_t edt_workspace_bytes(long long nvox);
size_t edt_lds_bytes(int n_line);  // LDS of one block for lines of n_line voxels
int launch_edt(const uint8_t* occ, int nx, int ny, int nz, float voxel, float* phi,
               uint32_t* d2, void* work, hipStream_t stream);

}  // namespace smpc
