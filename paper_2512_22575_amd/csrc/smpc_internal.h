// Internal layouts shared by the host runtime and the gfx950 kernels of libsmpc.
#pragma once

#include <stdint.h>

#include "smpc.h"

namespace smpc {

constexpr int kNdof = SMPC_NDOF;
constexpr int kSpl = SMPC_SPHERES_PER_LINK;   // sphere slots per link
constexpr int kSlots = kNdof * kSpl;          // slot s = (link - 1) * kSpl + j
constexpr int kMaxPairs = SMPC_MAX_PAIRS;
constexpr int kMaxH = SMPC_MAX_H;
constexpr int kK1MaxThreads = 512;            // rollout-cost block size limit
constexpr int kK2Threads = 256;               // reduce/update block size
constexpr int kWeightsPerWave = 1024;         // weights_out elements per wave in K2

// Robot constants in device memory.  Every field is read at a wave-uniform
// address, so the kernels fetch it with scalar loads.
struct DevRobot {
  float ca[kNdof], sa[kNdof];  // cos/sin of alpha_i (computed in double on the host)
  float a[kNdof], d[kNdof];
  float sc[kSlots][4];         // sphere slot centre (x, y, z) in its link frame, radius
  uint32_t slot_active;        // bit s set when slot s holds a sphere
  uint32_t pair_mask[kSlots];  // bit t (t > s) set when slots (s, t) form a pair
  float pair_rsum[kSlots][kSlots];   // r_s + r_t
  float pair_rsum2[kSlots][kSlots];  // (r_s + r_t)^2, rounded from double
  int32_t n_pairs;
  int32_t pad_[3];
  int16_t pair_list[kMaxPairs][2];   // the same pairs as a list of slot indices
};

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
  float gox, goy, goz, inv_voxel;    // grid origin and 1/voxel
  int32_t nx, ny, nz;
  uint32_t grid_bytes;
  int32_t K, H, R, P;          // samples, horizon, rollouts per K1 block, K1 blocks
  float dt;
  float inv_lambda;
};

// Device workspace carved from one allocation.
struct Workspace {
  double* S;        // [K]   per-rollout cost without the k = 0 state terms
  double* part_m;   // [P]   per-block minimum of S (+inf when the block has none finite)
  float* part_Z;    // [P]   sum_m exp(-(S - part_m)/lambda)
  float* part_Z2;   // [P]   sum_m exp(-2 (S - part_m)/lambda)
  float* part_N;    // [H*7][P] sum_m exp(-(S - part_m)/lambda) eps^(m)
};

struct LaunchConfig {
  int R;            // rollouts per K1 block
  int k1_threads;   // K1 block size (multiple of 64)
  int P;            // number of K1 blocks
  size_t k1_lds;    // dynamic LDS bytes of K1
  int k2_blocks;    // K2 grid
};

LaunchConfig plan_launch_config(int K, int H);
size_t workspace_bytes(int K, int H, int P);
Workspace carve_workspace(void* base, int K, int H, int P);

// Enqueue both kernels of one plan step.  Returns a hipError_t value (0 = success).
// When `events` is non-null, events[0..2] (hipEvent_t) are recorded before the
// rollout-cost kernel, between the kernels and after the merge kernel.
int launch_plan_step(const DevRobot* robot, const StepParams& p, const LaunchConfig& lc,
                     const Workspace& ws, const smpc_plan_args& args, void* stream,
                     void* events);

}  // namespace smpc
