// Signed Euclidean distance field from an occupancy grid (Sec. III-B) for gfx950.
//
// The field is built from two exact squared Euclidean distance transforms on the
// voxel lattice: D_out, the squared index distance from every voxel to the nearest
// occupied voxel, and D_in, to the nearest free voxel.  Each is separable: a 1-D
// transform along every axis in turn, D(p) = min_q ((p - q)^2 + f(q)), starting
// from 0 on the sources and "none" elsewhere.  The paper runs the 1-D
// Felzenszwalb-Huttenlocher (FH) lower-envelope transform along y, x, z on a layout
// whose contiguous axis is y, gathering each strided line into a per-thread buffer
// instead of transposing the grid.  The exact result does not depend on the order
// of the axes, so the same idea maps onto the planner's x-fastest layout as:
//
//   pass x  (contiguous axis, binary input): one wave per row; ballots of the
//           sources of each 64-voxel chunk give, by bit scans, the nearest source
//           on either side, i.e. the exact 1-D transform of a 0/none input;
//   pass y  FH, one thread per (x, z) line, lanes on consecutive x (coalesced),
//           lower-envelope stack in LDS, in place on both fields;
//   pass z  FH, one thread per (x, y) line, both fields in turn, fused with the
//           signed distance phi = voxel * (sqrt(D_out) - sqrt(D_in)).
//
// Integer-exact FH: a stack entry packs F = f(q) + q^2 (< 2^20) with q (< 2^9) in
// one word, and both envelope tests compare cross-multiplied integers instead of
// the floating intersection abscissae.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "smpc_internal.h"

namespace smpc {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;  // "no source on this line (yet)"
constexpr int kIdxBits = 9;              // q < 512
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;
constexpr int kFhLanes = 64;             // one wave per FH block
constexpr int kBatch = 8;                // line samples fetched per batch

// ---------------------------------------------------------------------------
// Pass x: per row, squared distance to the nearest occupied / free voxel.
// ---------------------------------------------------------------------------
constexpr int kRowWaves = 4;
constexpr int kMaxChunks = kEdtMaxSide / 64;

__global__ __launch_bounds__(64 * kRowWaves) void edt_rows_kernel(const uint8_t* __restrict__ occ,
                                                                 int nx, long long rows,
                                                                 long long nvox,
                                                                 uint32_t* __restrict__ work) {
  const int lane = threadIdx.x & 63;
  const long long row = (long long)blockIdx.x * kRowWaves + (threadIdx.x >> 6);
  if (row >= rows) return;  // whole wave leaves together
  const uint8_t* src = occ + row * nx;
  const int nch = (nx + 63) >> 6;
  uint64_t m_occ[kMaxChunks], m_free[kMaxChunks];
#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c) {
    m_occ[c] = m_free[c] = 0;
    if (c < nch) {
      const int p = c * 64 + lane;
      const bool in = p < nx;
      const bool o = in && src[in ? p : 0] != 0;
      m_occ[c] = __ballot(o);
      m_free[c] = __ballot(in && !o);
    }
  }
  // Nearest source strictly left of chunk c / strictly right of it (-1 / huge: none).
  int left_o[kMaxChunks], left_f[kMaxChunks], right_o[kMaxChunks], right_f[kMaxChunks];
  int lo = -1, lf = -1;
#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c) {
    left_o[c] = lo;
    left_f[c] = lf;
    if (m_occ[c]) lo = c * 64 + 63 - __clzll(m_occ[c]);
    if (m_free[c]) lf = c * 64 + 63 - __clzll(m_free[c]);
  }
  int ro = 1 << 30, rf = 1 << 30;
#pragma unroll
  for (int c = kMaxChunks - 1; c >= 0; --c) {
    right_o[c] = ro;
    right_f[c] = rf;
    if (m_occ[c]) ro = c * 64 + __ffsll((unsigned long long)m_occ[c]) - 1;
    if (m_free[c]) rf = c * 64 + __ffsll((unsigned long long)m_free[c]) - 1;
  }
  const uint64_t at_or_below = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const uint64_t at_or_above = ~0ull << lane;
  uint32_t* out_o = work + row * nx;
  uint32_t* out_f = out_o + nvox;
#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c) {
    if (c >= nch) break;
    const int p = c * 64 + lane;
    if (p >= nx) break;
    uint32_t d[2];
#pragma unroll
    for (int fld = 0; fld < 2; ++fld) {
      const uint64_t m = fld ? m_free[c] : m_occ[c];
      const uint64_t ml = m & at_or_below, mr = m & at_or_above;
      const int l = ml ? c * 64 + 63 - __clzll(ml) : (fld ? left_f[c] : left_o[c]);
      const int r = mr ? c * 64 + __ffsll((unsigned long long)mr) - 1
                       : (fld ? right_f[c] : right_o[c]);
      int dist = 1 << 30;
      if (l >= 0) dist = p - l;
      if (r < (1 << 30)) dist = min(dist, r - p);
      d[fld] = dist < (1 << 30) ? (uint32_t)(dist * dist) : kNone;
    }
    out_o[p] = d[0];
    out_f[p] = d[1];
  }
}

// ---------------------------------------------------------------------------
// FH along one strided line, by one thread.
// ---------------------------------------------------------------------------
struct Envelope {
  int k;  // parabolas kept
};

// Build the lower envelope of the parabolas rooted at the finite samples of
// line[q * stride], q < n.  st points at this lane's first stack word; entry i
// lives at st[i * kFhLanes] (lane-interleaved, so lanes never share a bank).
__device__ __forceinline__ int fh_build(const uint32_t* __restrict__ line, long long stride, int n,
                                        uint32_t* st) {
  int k = 0;
  int t = 0, Ft = 0;  // top of the stack
  int r = 0, Fr = 0;  // entry below the top (valid when k >= 2)
  uint32_t nxt[kBatch];
#pragma unroll
  for (int j = 0; j < kBatch; ++j) nxt[j] = j < n ? line[(long long)j * stride] : kNone;
  for (int q0 = 0; q0 < n; q0 += kBatch) {
    uint32_t cur[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) cur[j] = nxt[j];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int q = q0 + kBatch + j;
      nxt[j] = q < n ? line[(long long)q * stride] : kNone;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const uint32_t f = cur[j];
      if (f == kNone) continue;  // also covers q >= n
      const int q = q0 + j;
      const int Fq = (int)f + q * q;
      // Pop while the new parabola overtakes the top one no later than the top
      // overtook the one below it: s(t, q) <= s(r, t), cross-multiplied.
      while (k >= 2 && (Fq - Ft) * (t - r) <= (Ft - Fr) * (q - t)) {
        --k;
        t = r;
        Ft = Fr;
        if (k >= 2) {
          const uint32_t e = st[(k - 2) * kFhLanes];
          r = (int)(e & kIdxMask);
          Fr = (int)(e >> kIdxBits);
        }
      }
      st[k * kFhLanes] = ((uint32_t)Fq << kIdxBits) | (uint32_t)q;
      ++k;
      r = t;
      Fr = Ft;
      t = q;
      Ft = Fq;
    }
  }
  return k;
}

// Read the envelope off at p = 0..n-1 and hand (p, D(p)) to emit; D is kNone when
// the line has no finite sample.
template <class Emit>
__device__ __forceinline__ void fh_read(const uint32_t* st, int k, int n, Emit&& emit) {
  if (k == 0) {
    for (int p = 0; p < n; ++p) emit(p, kNone);
    return;
  }
  uint32_t e = st[0];
  int v = (int)(e & kIdxMask), F = (int)(e >> kIdxBits);
  int j = 0;
  int vn = 0, Fn = 0;
  if (k > 1) {
    e = st[kFhLanes];
    vn = (int)(e & kIdxMask);
    Fn = (int)(e >> kIdxBits);
  }
  for (int p = 0; p < n; ++p) {
    // Advance while the next parabola starts strictly left of p.
    while (j + 1 < k && Fn - F < 2 * p * (vn - v)) {
      ++j;
      v = vn;
      F = Fn;
      if (j + 1 < k) {
        e = st[(j + 1) * kFhLanes];
        vn = (int)(e & kIdxMask);
        Fn = (int)(e >> kIdxBits);
      }
    }
    emit(p, (uint32_t)(F + p * (p - 2 * v)));
  }
}

// Pass y: lines (x, z) of both fields, transformed in place.
__global__ __launch_bounds__(kFhLanes) void edt_fh_y_kernel(uint32_t* __restrict__ work, int nx,
                                                            int ny, int nz, long long nvox) {
  extern __shared__ uint32_t lds[];
  const long long lines = (long long)nx * nz;
  const long long i = (long long)blockIdx.x * kFhLanes + threadIdx.x;
  const int fld = blockIdx.y;
  if (i >= lines) return;
  const long long z = i / nx, x = i - z * nx;
  uint32_t* line = work + fld * nvox + z * (long long)nx * ny + x;
  uint32_t* st = lds + threadIdx.x;
  const int k = fh_build(line, nx, ny, st);
  fh_read(st, k, ny, [&](int p, uint32_t d) { line[(long long)p * nx] = d; });
}

// Pass z: lines (x, y); D_out then D_in, then phi.
__global__ __launch_bounds__(kFhLanes) void edt_fh_z_kernel(uint32_t* __restrict__ work, int nx,
                                                            int ny, int nz, long long nvox,
                                                            uint32_t none_value, double voxel,
                                                            float* __restrict__ phi) {
  extern __shared__ uint32_t lds[];
  const long long lines = (long long)nx * ny;
  const long long i = (long long)blockIdx.x * kFhLanes + threadIdx.x;
  if (i >= lines) return;
  const long long stride = lines;
  uint32_t* line_o = work + i;
  uint32_t* line_f = line_o + nvox;
  uint32_t* st = lds + threadIdx.x;
  int k = fh_build(line_o, stride, nz, st);
  fh_read(st, k, nz, [&](int p, uint32_t d) {
    line_o[(long long)p * stride] = d == kNone ? none_value : d;
  });
  k = fh_build(line_f, stride, nz, st);
  fh_read(st, k, nz, [&](int p, uint32_t d) {
    const long long at = (long long)p * stride;
    const uint32_t d_in = d == kNone ? none_value : d;
    line_f[at] = d_in;
    if (phi) {
      const uint32_t d_out = line_o[at];
      phi[i + at] = (float)(voxel * (__builtin_sqrt((double)d_out) -
                                     __builtin_sqrt((double)d_in)));
    }
  });
}

}  // namespace

int launch_edt(const uint8_t* occ, int nx, int ny, int nz, float voxel, float* phi,
               uint32_t* work, hipStream_t stream) {
  const long long nvox = (long long)nx * ny * nz;
  const long long rows = (long long)ny * nz;
  const uint32_t none_value = (uint32_t)nx * nx + (uint32_t)ny * ny + (uint32_t)nz * nz;
  hipLaunchKernelGGL(edt_rows_kernel, dim3((unsigned)((rows + kRowWaves - 1) / kRowWaves)),
                     dim3(64 * kRowWaves), 0, stream, occ, nx, rows, nvox, work);
  const long long ly = (long long)nx * nz;
  hipLaunchKernelGGL(edt_fh_y_kernel, dim3((unsigned)((ly + kFhLanes - 1) / kFhLanes), 2),
                     dim3(kFhLanes), (size_t)kFhLanes * ny * sizeof(uint32_t), stream, work, nx,
                     ny, nz, nvox);
  const long long lz = (long long)nx * ny;
  hipLaunchKernelGGL(edt_fh_z_kernel, dim3((unsigned)((lz + kFhLanes - 1) / kFhLanes)),
                     dim3(kFhLanes), (size_t)kFhLanes * nz * sizeof(uint32_t), stream, work, nx,
                     ny, nz, nvox, none_value, (double)voxel, phi);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace smpc
