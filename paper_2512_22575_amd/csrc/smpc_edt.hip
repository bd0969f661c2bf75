// Signed Euclidean distance field from an occupancy grid (Sec. III-B) for gfx950.
//
// The field is built from two exact squared Euclidean distance transforms on the
// voxel lattice: D_out, the squared index distance from every voxel to the nearest
// occupied voxel, and D_in, to the nearest free voxel.  Each is separable: a 1-D
// transform along every axis in turn, D(p) = min_q ((p - q)^2 + f(q)), starting
// from 0 on the sources and "none" elsewhere.  The paper runs the 1-D
// Felzenszwalb-Huttenlocher (FH) lower-envelope transform along y, x, z on a layout
// whose contiguous axis is y, gathering each strided line into a per-thread buffer.
// The exact result does not depend on the order of the axes; on the planner's
// x-fastest layout the same plan (contiguous axis first) is x, y, z:
//
//   pass x  (binary input): one wave per row; ballots of the sources of each
//           64-voxel chunk give the nearest source on either side by bit scans;
//   pass y  FH over 16 (x, z) lines per block, staged in LDS tiles;
//   pass z  FH over 16 (x, y) lines per block, one field per block;
//   phi     the signed distance phi = voxel * (sqrt(D_out) - sqrt(D_in)).
//
// Compact intermediates: after the x and y passes a voxel's value in its own
// field is 0 (a free voxel is a source of D_in, an occupied one of D_out), so one
// value per voxel plus its occupancy bit carries both fields: 16 bits after the x
// pass, 32 after the y pass.
//
// FH with 16 lanes per line.  Each lane builds the lower envelope of the samples of
// its band of the line (FH's stack, kept as a linked list in LDS); four rounds of
// pairwise merges join adjacent bands.  In the dual picture the envelope is the
// lower convex hull of the points (q, F_q), F_q = f(q) + q^2, so merging the hulls
// of two index-separated bands only removes points near the junction: pop the left
// tail and the right head until both turns there are strictly convex (the bridge).
// The read-off walks the merged list; along it the cost (p - q)^2 + f(q) is
// unimodal in the list position, so each output p starts from the winner of p - 1.
// All tests are integer cross-multiplications: F_q < 2^20 and index differences
// < 2^9 keep every product below 2^29.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "smpc_internal.h"

namespace smpc {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;  // "no source on this line (yet)"
constexpr uint16_t kNil = 0xFFFFu;       // end of a linked list
constexpr int kLines = 16;               // lines per FH block
constexpr int kG = 16;                   // lanes per line
constexpr int kFhThreads = kLines * kG;  // 256
constexpr int kTs = kLines + 1;          // LDS tile row stride (words), padded
constexpr int kMaxChunks = kEdtMaxSide / 64;

// Compact per-voxel records.
//   after x: bit 15 occupied, bit 14 "no source in the row", bits 0..13 distance
//   after y: bit 31 occupied, bit 30 "no source in the plane", bits 0..29 D
constexpr uint16_t kXOcc = 0x8000u, kXNone = 0x4000u;
constexpr uint32_t kYOcc = 0x80000000u, kYNone = 0x40000000u, kYVal = 0x3FFFFFFFu;

// Squared-distance sample of field `fld` (0: to occupied, 1: to free) from a record.
__device__ __forceinline__ uint32_t field_of_x(uint16_t r, int fld) {
  const bool occ = r & kXOcc;
  if (occ != (fld == 1)) return 0u;  // the voxel is a source of this field
  if (r & kXNone) return kNone;
  const uint32_t d = r & 0x3FFFu;
  return d * d;
}

__device__ __forceinline__ uint32_t field_of_y(uint32_t r, int fld) {
  const bool occ = r & kYOcc;
  if (occ != (fld == 1)) return 0u;
  return (r & kYNone) ? kNone : (r & kYVal);
}

// ---------------------------------------------------------------------------
// Pass x: per voxel, the distance along its row to the nearest voxel of the other
// kind (occupied for a free voxel, free for an occupied one).
// ---------------------------------------------------------------------------
constexpr int kRowWaves = 4;
constexpr int kRowsPerWave = 4;

__global__ __launch_bounds__(64 * kRowWaves) void edt_pass_x_kernel(
    const uint8_t* __restrict__ occ, int nx, long long rows, uint16_t* __restrict__ xrec) {
  const int lane = threadIdx.x & 63;
  const long long row0 =
      ((long long)blockIdx.x * kRowWaves + (threadIdx.x >> 6)) * kRowsPerWave;
  if (row0 >= rows) return;  // whole wave leaves together
  const int nch = (nx + 63) >> 6;
  // All loads of the wave's rows first, so their latencies overlap.
  uint8_t v[kRowsPerWave][kMaxChunks];
#pragma unroll
  for (int w = 0; w < kRowsPerWave; ++w) {
    const long long row = row0 + w;
    const uint8_t* src = occ + row * nx;
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) {
      const int p = c * 64 + lane;
      v[w][c] = (row < rows && c < nch && p < nx) ? src[p] : 0;
    }
  }
#pragma unroll
  for (int w = 0; w < kRowsPerWave; ++w) {
    const long long row = row0 + w;
    if (row >= rows) break;
    uint64_t m_occ[kMaxChunks], m_free[kMaxChunks];
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) {
      const int p = c * 64 + lane;
      m_occ[c] = __ballot(p < nx && v[w][c] != 0);
      m_free[c] = __ballot(p < nx && v[w][c] == 0);
    }
    // Nearest source strictly left of chunk c / strictly right of it (-1 / 2^30: none).
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
    uint16_t* out = xrec + row * nx;
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) {
      const int p = c * 64 + lane;
      if (c < nch && p < nx) {
        const bool o = v[w][c] != 0;
        const uint64_t m = o ? m_free[c] : m_occ[c];  // sources of the voxel's other field
        const uint64_t ml = m & at_or_below, mr = m & at_or_above;
        const int l = ml ? c * 64 + 63 - __clzll(ml) : (o ? left_f[c] : left_o[c]);
        const int r = mr ? c * 64 + __ffsll((unsigned long long)mr) - 1
                         : (o ? right_f[c] : right_o[c]);
        int dist = 1 << 30;
        if (l >= 0) dist = p - l;
        if (r < (1 << 30)) dist = min(dist, r - p);
        out[p] = (uint16_t)((o ? kXOcc : 0u) | (dist < (1 << 30) ? (uint32_t)dist : kXNone));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FH on a tile of kLines lines held in LDS, kG lanes per line.
// ---------------------------------------------------------------------------
struct Tile {
  uint32_t* f;    // [n][kTs]: f(q); kNone for no sample and for points dropped
  uint16_t* prv;  // [n][kTs]: previous kept point of the list
  uint16_t* nxt;  // [n][kTs]: next kept point of the list
};

constexpr size_t tile_bytes(int n) {
  return (size_t)n * kTs * (sizeof(uint32_t) + 2 * sizeof(uint16_t));
}

__device__ __forceinline__ Tile carve_tile(uint32_t* lds, int n) {
  Tile t;
  t.f = lds;
  t.prv = reinterpret_cast<uint16_t*>(lds + n * kTs);
  t.nxt = t.prv + n * kTs;
  return t;
}

// Point y lies strictly below the segment from x to z (x < y < z, values F).
__device__ __forceinline__ bool below(int x, int Fx, int y, int Fy, int z, int Fz) {
  return (Fy - Fx) * (z - y) < (Fz - Fy) * (y - x);
}

// Every thread of the block calls this (it holds block barriers).  The thread
// works on line threadIdx.x / kG, band threadIdx.x % kG; `active` is false for
// lines past the end of the grid.  emit(p, D) receives each output of the band
// (kNone when the line holds no sample).
template <class Emit>
__device__ __forceinline__ void tile_fh(const Tile& T, int n, bool active, Emit&& emit) {
  const int lane = threadIdx.x & 63;
  const int line = threadIdx.x / kG;
  const int band = threadIdx.x % kG;
  const int b = (n + kG - 1) / kG;
  const int lo = min(n, band * b), hi = min(n, lo + b);
  uint32_t* f = T.f + line;
  uint16_t* prv = T.prv + line;
  uint16_t* nxt = T.nxt + line;
  auto F = [&](int q) { return (int)f[q * kTs] + q * q; };

  // Phase A: lower envelope of the band, as a list head..tail.
  int head = kNil, tail = kNil;
  if (active) {
    int k = 0, t = 0, Ft = 0, r = 0, Fr = 0;
    for (int q = lo; q < hi; ++q) {
      const uint32_t fq = f[q * kTs];
      if (fq == kNone) continue;
      const int Fq = (int)fq + q * q;
      while (k >= 2 && !below(r, Fr, t, Ft, q, Fq)) {
        f[t * kTs] = kNone;
        t = r;
        Ft = Fr;
        --k;
        if (k >= 2) {
          r = prv[t * kTs];
          Fr = F(r);
        }
      }
      prv[q * kTs] = (uint16_t)(k ? t : kNil);
      if (k)
        nxt[t * kTs] = (uint16_t)q;
      else
        head = q;
      r = t;
      Fr = Ft;
      t = q;
      Ft = Fq;
      ++k;
    }
    if (k) {
      nxt[t * kTs] = kNil;
      tail = t;
    }
  }
  __syncthreads();

  // Phase B: merge groups of s bands pairwise, s = 1, 2, 4, 8.
#pragma unroll
  for (int s = 1; s < kG; s <<= 1) {
    const int rh = __shfl(head, lane + 1);
    const int rt = __shfl(tail, lane + 1);
    int nh = head, nt = tail;
    if (active && (band & (2 * s - 1)) == s - 1) {
      if (tail == kNil) {
        nh = rh;
        nt = rt;
      } else if (rh != kNil) {
        int a = tail, Fa = F(a), c = rh, Fc = F(c);
        for (;;) {
          bool moved = false;
          for (;;) {  // drop the left tail while it is not strictly convex
            const int pa = prv[a * kTs];
            if (pa == kNil) break;
            const int Fpa = F(pa);
            if (below(pa, Fpa, a, Fa, c, Fc)) break;
            f[a * kTs] = kNone;
            a = pa;
            Fa = Fpa;
            moved = true;
          }
          for (;;) {  // drop the right head while it is not strictly convex
            const int nc = nxt[c * kTs];
            if (nc == kNil) break;
            const int Fnc = F(nc);
            if (below(a, Fa, c, Fc, nc, Fnc)) break;
            f[c * kTs] = kNone;
            c = nc;
            Fc = Fnc;
            moved = true;
          }
          if (!moved) break;
        }
        nxt[a * kTs] = (uint16_t)c;
        prv[c * kTs] = (uint16_t)a;
        nt = rt;  // the extreme points of a group are never dropped
      }
    }
    const int src = lane - band + (band & ~(2 * s - 1)) + s - 1;
    head = __shfl(nh, src);
    tail = __shfl(nt, src);
  }
  __syncthreads();

  // Phase C: a kept point near the band, then the read-off.
  int fm = kNil, lm = kNil;
  if (active) {
    for (int q = lo; q < hi; ++q) {
      if (f[q * kTs] != kNone) {
        if (fm == kNil) fm = q;
        lm = q;
      }
    }
  }
  int start = fm;
#pragma unroll
  for (int d = 1; d < kG; ++d) {
    const int v = __shfl(lm, lane - d);
    if (start == kNil && band - d >= 0) start = v;
  }
#pragma unroll
  for (int d = 1; d < kG; ++d) {
    const int v = __shfl(fm, lane + d);
    if (start == kNil && band + d < kG) start = v;
  }
  if (!active) return;
  if (start == kNil) {
    for (int p = lo; p < hi; ++p) emit(p, kNone);
    return;
  }
  int c = start, Fc = F(c);
  for (int p = lo; p < hi; ++p) {
    for (;;) {
      const int nc = nxt[c * kTs];
      if (nc == kNil) break;
      const int Fn = F(nc);
      if (Fn + p * (p - 2 * nc) > Fc + p * (p - 2 * c)) break;
      c = nc;
      Fc = Fn;
    }
    if (p == lo) {
      for (;;) {
        const int pc = prv[c * kTs];
        if (pc == kNil) break;
        const int Fp = F(pc);
        if (Fp + p * (p - 2 * pc) >= Fc + p * (p - 2 * c)) break;
        c = pc;
        Fc = Fp;
      }
    }
    emit(p, (uint32_t)(Fc + p * (p - 2 * c)));
  }
}

// Stage samples q = 0..n-1 of the block's lines into the f tile: thread t takes
// line t % kLines at q = t / kLines + (kFhThreads / kLines) k.  Eight loads are
// issued before any is used (indices clamped into range, so no load sits behind a
// branch); decode(raw, q) turns a record into the sample.  Threads of lines past the grid pass ok = false
// and a valid base; their samples become kNone.
template <class Rec, class Decode>
__device__ __forceinline__ void stage_tile(uint32_t* f, int n, const Rec* base, long long stride,
                                           bool ok, Decode&& decode) {
  constexpr int kRowsPerPass = kFhThreads / kLines;  // 8
  constexpr int kBatch = 8;
  const int l = threadIdx.x % kLines;
  for (int q0 = threadIdx.x / kLines; q0 < n; q0 += kRowsPerPass * kBatch) {
    Rec v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int q = min(q0 + j * kRowsPerPass, n - 1);
      v[j] = base[q * stride];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int q = q0 + j * kRowsPerPass;
      if (q < n) f[q * kTs + l] = ok ? decode(v[j], q) : kNone;
    }
  }
}

// Pass y: block = 16 consecutive lines (x, z) of one field (blockIdx.y).
__global__ __launch_bounds__(kFhThreads) void edt_pass_y_kernel(
    const uint16_t* __restrict__ xrec, uint32_t* __restrict__ yrec, int nx, int ny, int nz) {
  extern __shared__ uint32_t lds[];
  const int fld = blockIdx.y;
  const int line0 = blockIdx.x * kLines;  // flattened (z, x) < 2^18
  Tile T = carve_tile(lds, ny);
  uint32_t* occ_bits = lds + tile_bytes(ny) / sizeof(uint32_t);  // [ny], bit = line
  const int lines = nx * nz;
  const long long plane = (long long)nx * ny;
  for (int i = threadIdx.x; i < ny; i += kFhThreads) occ_bits[i] = 0u;
  __syncthreads();
  {
    const int li = line0 + (int)(threadIdx.x % kLines);
    const bool ok = li < lines;
    const int z = ok ? li / nx : 0, x = ok ? li - z * nx : 0;
    const uint32_t bit = 1u << (threadIdx.x % kLines);
    stage_tile(T.f, ny, xrec + z * plane + x, nx, ok, [&](uint16_t r, int y) -> uint32_t {
      if (r & kXOcc) atomicOr(&occ_bits[y], bit);
      return field_of_x(r, fld);
    });
  }
  __syncthreads();
  const int line = threadIdx.x / kG;
  const int li = line0 + line;
  const bool active = li < lines;
  const int z = active ? li / nx : 0, x = active ? li - z * nx : 0;
  uint32_t* out = yrec + z * plane + x;
  tile_fh(T, ny, active, [&](int p, uint32_t d) {
    const bool o = (occ_bits[p] >> line) & 1u;
    if (o != (fld == 1)) return;  // a source of this field: the other field's block writes it
    out[(long long)p * nx] = (o ? kYOcc : 0u) | (d == kNone ? kYNone : d);
  });
}

// Pass z: block = 16 consecutive lines (x, y) of one field (blockIdx.y).  Without
// d2, D_out is parked in the phi buffer (as bits) and D_in in the workspace region
// of the x-pass records, which is dead once the y pass has finished; the y records
// are only read (the blocks of the two fields run concurrently).
__global__ __launch_bounds__(kFhThreads) void edt_pass_z_kernel(
    const uint32_t* __restrict__ yrec, int nx, int ny, int nz, uint32_t none_value, float* phi,
    uint32_t* d2, uint32_t* d_in_scratch) {
  extern __shared__ uint32_t lds[];
  const int fld = blockIdx.y;
  const long long plane = (long long)nx * ny;
  const long long nvox = plane * nz;
  const long long line0 = (long long)blockIdx.x * kLines;  // flattened (y, x)
  Tile T = carve_tile(lds, nz);
  const int line = threadIdx.x / kG;
  const long long li = line0 + line;
  const bool active = li < plane;
  uint32_t* dst =
      fld == 0 ? (d2 ? d2 : reinterpret_cast<uint32_t*>(phi)) : (d2 ? d2 + nvox : d_in_scratch);
  {
    const long long i = line0 + (long long)(threadIdx.x % kLines);
    stage_tile(T.f, nz, yrec + (i < plane ? i : 0), plane, i < plane,
               [&](uint32_t r, int) { return field_of_y(r, fld); });
  }
  __syncthreads();
  uint32_t* out = dst + li;
  tile_fh(T, nz, active, [&](int p, uint32_t d) {
    out[p * plane] = d == kNone ? none_value : d;
  });
}

// phi = voxel * (sqrt(D_out) - sqrt(D_in)), in float64, rounded to float32 once.  At
// most one of the two is nonzero (a voxel is a source of one field), and then the
// formula is exactly +-voxel * sqrt(D) (subtracting sqrt(0) = 0 and negating are
// exact), so one square root suffices.
__global__ __launch_bounds__(256) void edt_phi_kernel(const uint32_t* d_out,
                                                      const uint32_t* d_in, long long nvox,
                                                      double voxel, float* phi) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= nvox) return;
  const uint32_t a = d_out[i], b = d_in[i];
  double v;
  if (a == 0u)
    v = -(voxel * __builtin_sqrt((double)b));
  else if (b == 0u)
    v = voxel * __builtin_sqrt((double)a);
  else
    v = voxel * (__builtin_sqrt((double)a) - __builtin_sqrt((double)b));
  phi[i] = (float)v;
}

}  // namespace

size_t edt_workspace_bytes(long long nvox) {
  // y-pass records, then the x-pass records (u16) later reused for D_in (u32).
  return (size_t)nvox * (2 * sizeof(uint32_t));
}

size_t edt_lds_bytes(int n_line) { return tile_bytes(n_line) + (size_t)n_line * sizeof(uint32_t); }

int launch_edt(const uint8_t* occ, int nx, int ny, int nz, float voxel, float* phi,
               uint32_t* d2, void* work, hipStream_t stream) {
  const long long plane = (long long)nx * ny;
  const long long nvox = plane * nz;
  uint32_t* yrec = static_cast<uint32_t*>(work);
  uint16_t* xrec = reinterpret_cast<uint16_t*>(yrec + nvox);
  const long long rows = (long long)ny * nz;
  const uint32_t none_value = (uint32_t)nx * nx + (uint32_t)ny * ny + (uint32_t)nz * nz;
  const long long rows_per_block = (long long)kRowWaves * kRowsPerWave;
  hipLaunchKernelGGL(edt_pass_x_kernel,
                     dim3((unsigned)((rows + rows_per_block - 1) / rows_per_block)),
                     dim3(64 * kRowWaves), 0, stream, occ, nx, rows, xrec);
  const long long ly = (long long)nx * nz;
  hipLaunchKernelGGL(edt_pass_y_kernel, dim3((unsigned)((ly + kLines - 1) / kLines), 2),
                     dim3(kFhThreads), edt_lds_bytes(ny), stream, xrec, yrec, nx, ny, nz);
  uint32_t* d_in_scratch = yrec + nvox;  // over the x-pass records, dead after pass y
  hipLaunchKernelGGL(edt_pass_z_kernel, dim3((unsigned)((plane + kLines - 1) / kLines), 2),
                     dim3(kFhThreads), tile_bytes(nz), stream, yrec, nx, ny, nz, none_value, phi,
                     d2, d_in_scratch);
  if (phi) {
    const uint32_t* d_out = d2 ? d2 : reinterpret_cast<const uint32_t*>(phi);
    const uint32_t* d_in = d2 ? d2 + nvox : d_in_scratch;
    hipLaunchKernelGGL(edt_phi_kernel, dim3((unsigned)((nvox + 255) / 256)), dim3(256), 0, stream,
                       d_out, d_in, nvox, (double)voxel, phi);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace smpc
