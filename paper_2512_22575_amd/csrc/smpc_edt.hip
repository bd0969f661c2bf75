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
//   pass y  16 (x, z) lines of one field per block, staged in an LDS tile: D_out by
//           FH, D_in by a bounded search around each occupied voxel (FH when an
//           obstacle is too thick for it);
//   pass z  the same over 16 (x, y) lines per block, writing the outputs: phi =
//           voxel * (sqrt(D_out) - sqrt(D_in)) and/or the two squared fields.
//
// Compact intermediates: after every pass a voxel's value in its own field is 0 (a
// free voxel is a source of D_in, an occupied one of D_out), so one value per voxel
// plus its occupancy bit carries both fields: 16 bits after the x pass, 32 after the
// y pass.
//
// FH with 16 lanes per line.  Each lane builds the lower envelope of the samples of
// its band of the line (FH's stack, kept as a linked list in LDS); four rounds of
// pairwise merges join adjacent bands.  In the dual picture the envelope is the lower
// convex hull of the points (q, F_q), F_q = f(q) + q^2, so merging the hulls
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
constexpr int kLines = 16;               // lines per FH block
constexpr int kG = 16;                   // lanes per line
constexpr int kFhThreads = kLines * kG;  // 256
constexpr int kTs = kLines + 1;          // LDS tile row stride (words), padded

// Compact per-voxel records.
//   after x: bit 15 occupied, bit 14 "no source in the row", bits 0..13 distance
//   after y: bit 31 occupied, bit 30 "no source in the plane", bits 0..29 D
constexpr uint16_t kXOcc = 0x8000u, kXNone = 0x4000u;
constexpr uint32_t kYOcc = 0x80000000u, kYNone = 0x40000000u, kYVal = 0x3FFFFFFFu;

// ---------------------------------------------------------------------------
// Pass x: per voxel, the distance along its row to the nearest voxel of the other
// kind (occupied for a free voxel, free for an occupied one).
// ---------------------------------------------------------------------------
constexpr int kRowWaves = 4;
constexpr int kRowsPerWave = 4;

// kChunks: 64-voxel chunks a row may hold (nx <= 64 kChunks).
template <int kChunks>
__global__ __launch_bounds__(64 * kRowWaves) void edt_pass_x_kernel(
    const uint8_t* __restrict__ occ, int nx, long long rows, uint16_t* __restrict__ xrec) {
  const int lane = threadIdx.x & 63;
  const long long row0 =
      ((long long)blockIdx.x * kRowWaves + (threadIdx.x >> 6)) * kRowsPerWave;
  if (row0 >= rows) return;  // whole wave leaves together
  const int nch = (nx + 63) >> 6;
  // All loads of the wave's rows first, so their latencies overlap.
  uint8_t v[kRowsPerWave][kChunks];
#pragma unroll
  for (int w = 0; w < kRowsPerWave; ++w) {
    const long long row = row0 + w;
    const uint8_t* src = occ + row * nx;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const int p = c * 64 + lane;
      v[w][c] = (row < rows && c < nch && p < nx) ? src[p] : 0;
    }
  }
#pragma unroll
  for (int w = 0; w < kRowsPerWave; ++w) {
    const long long row = row0 + w;
    if (row >= rows) break;
    uint64_t m_occ[kChunks], m_free[kChunks];
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const int p = c * 64 + lane;
      m_occ[c] = __ballot(p < nx && v[w][c] != 0);
      m_free[c] = __ballot(p < nx && v[w][c] == 0);
    }
    // Nearest source strictly left of chunk c / strictly right of it (-1 / 2^30: none).
    int left_o[kChunks], left_f[kChunks], right_o[kChunks], right_f[kChunks];
    int lo = -1, lf = -1;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      left_o[c] = lo;
      left_f[c] = lf;
      if (m_occ[c]) lo = c * 64 + 63 - __clzll(m_occ[c]);
      if (m_free[c]) lf = c * 64 + 63 - __clzll(m_free[c]);
    }
    int ro = 1 << 30, rf = 1 << 30;
#pragma unroll
    for (int c = kChunks - 1; c >= 0; --c) {
      right_o[c] = ro;
      right_f[c] = rf;
      if (m_occ[c]) ro = c * 64 + __ffsll((unsigned long long)m_occ[c]) - 1;
      if (m_free[c]) rf = c * 64 + __ffsll((unsigned long long)m_free[c]) - 1;
    }
    const uint64_t at_or_below = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const uint64_t at_or_above = ~0ull << lane;
    uint16_t* out = xrec + row * nx;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
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

// Rows whose length is a multiple of 4, at most 256 voxels, in a 4-byte-aligned grid
// (records 8-byte aligned): lane l holds voxels 4l .. 4l + 3 of a row, read as one
// 32-bit word and written as one 8-byte record group.  The nearest voxel of the other
// kind is found in the lane's own four voxels, else in the nearest lane on that side
// holding one (a ballot of the lanes holding each kind, then a lane shuffle of that
// lane's first or last such voxel).
__device__ __forceinline__ int last_bit4(uint32_t m) { return 31 - __clz(m); }  // m != 0
__device__ __forceinline__ int first_bit4(uint32_t m) { return __ffs(m) - 1; }  // m != 0

constexpr int kWordRows = 2;  // rows per wave of the word-per-lane kernel

__global__ __launch_bounds__(64 * kRowWaves) void edt_pass_x_words_kernel(
    const uint8_t* __restrict__ occ, int nx, long long rows, uint16_t* __restrict__ xrec) {
  const int lane = threadIdx.x & 63;
  const long long row0 =
      ((long long)blockIdx.x * kRowWaves + (threadIdx.x >> 6)) * kWordRows;
  if (row0 >= rows) return;  // whole wave leaves together
  const int nw = nx >> 2;    // 32-bit words per row
  const bool has = lane < nw;
  uint32_t word[kWordRows];
#pragma unroll
  for (int w = 0; w < kWordRows; ++w) {
    const long long row = row0 + w;
    word[w] = (row < rows && has)
                  ? *reinterpret_cast<const uint32_t*>(occ + row * nx + 4 * lane)
                  : 0u;
  }
  const uint64_t below = (1ull << lane) - 1ull;               // lanes left of this one
  const uint64_t above = lane == 63 ? 0ull : ~0ull << (lane + 1);
  // "None" on the left / right: p - kNoLeft and kNoRight - p are >= 2^20 for every p.
  constexpr int kNoLeft = -(1 << 20), kNoRight = 1 << 21;
#pragma unroll
  for (int w = 0; w < kWordRows; ++w) {
    const long long row = row0 + w;
    if (row >= rows) break;
    uint32_t mo = 0u;  // bit k: voxel 4 lane + k occupied
#pragma unroll
    for (int k = 0; k < 4; ++k) mo |= (((word[w] >> (8 * k)) & 0xFFu) != 0u ? 1u : 0u) << k;
    const uint32_t mf = has ? (~mo & 0xFu) : 0u;              // free voxels
    const uint64_t lanes_o = __ballot(mo != 0u), lanes_f = __ballot(mf != 0u);
    // This lane's first and last voxel of each kind (absolute indices).
    const int fo = mo ? 4 * lane + first_bit4(mo) : 0, lo = mo ? 4 * lane + last_bit4(mo) : 0;
    const int ff = mf ? 4 * lane + first_bit4(mf) : 0, lf = mf ? 4 * lane + last_bit4(mf) : 0;
    // Nearest lane on each side holding each kind, and its nearest voxel of that kind.
    const uint64_t lo_m = lanes_o & below, ro_m = lanes_o & above;
    const uint64_t lf_m = lanes_f & below, rf_m = lanes_f & above;
    const int lo_src = lo_m ? 63 - __clzll(lo_m) : lane;
    const int ro_src = ro_m ? __ffsll((unsigned long long)ro_m) - 1 : lane;
    const int lf_src = lf_m ? 63 - __clzll(lf_m) : lane;
    const int rf_src = rf_m ? __ffsll((unsigned long long)rf_m) - 1 : lane;
    const int sh_lo = __shfl(lo, lo_src), sh_fo = __shfl(fo, ro_src);
    const int sh_lf = __shfl(lf, lf_src), sh_ff = __shfl(ff, rf_src);
    const int left_o = lo_m ? sh_lo : kNoLeft, right_o = ro_m ? sh_fo : kNoRight;
    const int left_f = lf_m ? sh_lf : kNoLeft, right_f = rf_m ? sh_ff : kNoRight;
    if (!has) continue;
    uint16_t rec[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int p = 4 * lane + k;
      const bool o = (mo >> k) & 1u;
      const uint32_t m = o ? mf : mo;                          // sources of the other kind
      const uint32_t ml = m & ((1u << k) - 1u), mr = m & (0xEu << k) & 0xFu;
      const int l = ml ? 4 * lane + last_bit4(ml) : (o ? left_f : left_o);
      const int r = mr ? 4 * lane + first_bit4(mr) : (o ? right_f : right_o);
      const int dist = min(p - l, r - p);
      rec[k] = (uint16_t)((o ? kXOcc : 0u) | (dist < (1 << 20) ? (uint32_t)dist : kXNone));
    }
    uint2 out;
    out.x = (uint32_t)rec[0] | ((uint32_t)rec[1] << 16);
    out.y = (uint32_t)rec[2] | ((uint32_t)rec[3] << 16);
    *reinterpret_cast<uint2*>(xrec + row * nx + 4 * lane) = out;
  }
}

// ---------------------------------------------------------------------------
// FH on a tile of kLines lines held in LDS, kG lanes per line.  Samples are of type
// Val (uint16_t when every finite sample is below 0xFFFF, else uint32_t; the
// all-ones value marks "no sample" and dropped points) and list links are sample
// indices of type Link (uint8_t for lines of at most 255 samples, index 255 ending a
// list, else uint16_t), so that more tiles fit in a CU's LDS.
// ---------------------------------------------------------------------------
template <class Val, class Link>
struct Tile {
  static constexpr int kNil = (int)(Link)(-1);  // end of a linked list
  static constexpr uint32_t kNoVal = (Val)(-1);
  Val* f;     // [n][kTs]: f(q); kNoVal for no sample and for points dropped
  Link* prv;  // [n][kTs]: previous kept point of the list
  Link* nxt;  // [n][kTs]: next kept point of the list
};

// LDS bytes of a tile of n samples per line, rounded up to whole words.
template <class Val, class Link>
constexpr size_t tile_bytes(int n) {
  return ((size_t)n * kTs * (sizeof(Val) + 2 * sizeof(Link)) + 3) & ~size_t(3);
}

template <class Val, class Link>
__device__ __forceinline__ Tile<Val, Link> carve_tile(uint32_t* lds, int n) {
  Tile<Val, Link> t;
  t.f = reinterpret_cast<Val*>(lds);
  t.prv = reinterpret_cast<Link*>(t.f + n * kTs);
  t.nxt = t.prv + n * kTs;
  return t;
}

// Point y lies strictly below the segment from x to z (x < y < z, values F).
__device__ __forceinline__ bool below(int x, int Fx, int y, int Fy, int z, int Fz) {
  return (Fy - Fx) * (z - y) < (Fz - Fy) * (y - x);
}

// Band [lo, hi) of the calling thread's line: kG bands of ceil(n / kG) samples.
struct Band {
  int line, band, lo, hi;
};
__device__ __forceinline__ Band my_band(int n) {
  Band b;
  b.line = threadIdx.x / kG;
  b.band = threadIdx.x % kG;
  const int len = (n + kG - 1) / kG;
  b.lo = min(n, b.band * len);
  b.hi = min(n, b.lo + len);
  return b;
}
static_assert((kEdtMaxSide + kG - 1) / kG <= 64, "a band's occupancy fits 64 bits");

// Occupancy of the thread's band, bit q - lo (occ_bits[q] holds bit `line`).
__device__ __forceinline__ uint64_t band_occupancy(const uint32_t* occ_bits, const Band& B) {
  uint64_t m = 0;
  for (int q = B.lo; q < B.hi; ++q) m |= (uint64_t)((occ_bits[q] >> B.line) & 1u) << (q - B.lo);
  return m;
}

// Every thread of the block calls this (it holds block barriers).  The thread
// works on line threadIdx.x / kG, band threadIdx.x % kG; `active` is false for
// lines past the end of the grid and for lines with no output to write (a wave
// whose lines are all inactive skips the work).  emit(p, D, occupied) receives
// each output of the band (D = kNone when the line holds no sample).
template <class Val, class Link, class Emit>
__device__ __forceinline__ void tile_fh(const Tile<Val, Link>& T, int n, bool active,
                                        const uint32_t* occ_bits, Emit&& emit) {
  constexpr int kNil = Tile<Val, Link>::kNil;
  constexpr uint32_t kNoVal = Tile<Val, Link>::kNoVal;
  const int lane = threadIdx.x & 63;
  const Band B = my_band(n);
  const int band = B.band, lo = B.lo, hi = B.hi;
  Val* f = T.f + B.line;
  Link* prv = T.prv + B.line;
  Link* nxt = T.nxt + B.line;
  auto F = [&](int q) { return (int)f[q * kTs] + q * q; };

  // Phase A: lower envelope of the band, as a list head..tail.  The samples are
  // read kAhead at a time (the pops only overwrite samples already read).
  constexpr int kAhead = 8;
  int head = kNil, tail = kNil;
  if (active) {
    int k = 0, t = 0, Ft = 0, r = 0, Fr = 0;
    for (int q0 = lo; q0 < hi; q0 += kAhead) {
      uint32_t fv[kAhead];
#pragma unroll
      for (int j = 0; j < kAhead; ++j) fv[j] = f[min(q0 + j, hi - 1) * kTs];
#pragma unroll
      for (int j = 0; j < kAhead; ++j) {
        const int q = q0 + j;
        if (q >= hi || fv[j] == kNoVal) continue;
        const int Fq = (int)fv[j] + q * q;
        while (k >= 2 && !below(r, Fr, t, Ft, q, Fq)) {
          f[t * kTs] = (Val)kNoVal;
          t = r;
          Ft = Fr;
          --k;
          if (k >= 2) {
            r = prv[t * kTs];
            Fr = F(r);
          }
        }
        prv[q * kTs] = (Link)(k ? t : kNil);
        if (k)
          nxt[t * kTs] = (Link)q;
        else
          head = q;
        r = t;
        Fr = Ft;
        t = q;
        Ft = Fq;
        ++k;
      }
    }
    if (k) {
      nxt[t * kTs] = (Link)kNil;
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
            f[a * kTs] = (Val)kNoVal;
            a = pa;
            Fa = Fpa;
            moved = true;
          }
          for (;;) {  // drop the right head while it is not strictly convex
            const int nc = nxt[c * kTs];
            if (nc == kNil) break;
            const int Fnc = F(nc);
            if (below(a, Fa, c, Fc, nc, Fnc)) break;
            f[c * kTs] = (Val)kNoVal;
            c = nc;
            Fc = Fnc;
            moved = true;
          }
          if (!moved) break;
        }
        nxt[a * kTs] = (Link)c;
        prv[c * kTs] = (Link)a;
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
      if (f[q * kTs] != kNoVal) {
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
  const uint64_t occ = band_occupancy(occ_bits, B);
  if (start == kNil) {
    for (int p = lo; p < hi; ++p) emit(p, kNone, (occ >> (p - lo)) & 1u);
    return;
  }
  // The winner c and its successor nc (with their F) stay in registers, so an output
  // whose winner does not change reads no LDS.
  int c = start, Fc = F(c);
  int nc = nxt[c * kTs], Fn = nc == kNil ? 0 : F(nc);
  for (int p = lo; p < hi; ++p) {
    while (nc != kNil && Fn + p * (p - 2 * nc) <= Fc + p * (p - 2 * c)) {
      c = nc;
      Fc = Fn;
      nc = nxt[c * kTs];
      if (nc != kNil) Fn = F(nc);
    }
    if (p == lo) {
      bool moved = false;
      for (;;) {
        const int pc = prv[c * kTs];
        if (pc == kNil) break;
        const int Fp = F(pc);
        if (Fp + p * (p - 2 * pc) >= Fc + p * (p - 2 * c)) break;
        c = pc;
        Fc = Fp;
        moved = true;
      }
      if (moved) {
        nc = nxt[c * kTs];
        Fn = nc == kNil ? 0 : F(nc);
      }
    }
    emit(p, (uint32_t)(Fc + p * (p - 2 * c)), (occ >> (p - lo)) & 1u);
  }
}

// One field of kLines lines, one block (fld 0: D_out, 1: D_in).  A voxel's record
// after the previous pass holds its occupancy and one value v: the sample of the
// field it is not a source of (D_out's for a free voxel, D_in's for an occupied one;
// its own field is 0 there).
//   1. Stage the samples into the tile (thread t: line t % kLines, q = t / kLines +
//      (kFhThreads / kLines) k, kBatch loads in flight) and the occupancy into
//      occ_bits[q] (bit = line).  decode(raw, occ) returns v as a 32-bit value
//      (kNone: no sample).
//   2. D_out: FH over the lines that hold a free voxel, written at the free voxels.
//   3. D_in: at each occupied voxel p a search outward from p: candidates q = p +- d
//      for d = 1, 2, ... (f_in(q) = 0 on free q, v(q) on occupied q), stopping once d^2
//      reaches the best value found, which is then exact since every farther q costs
//      at least d^2.  Obstacles are thin against a line, so the search ends after a
//      few steps.  The occupied voxels of the tile are listed during staging and
//      shared out evenly over the block's threads; a tile with more than kInList of
//      them, or a search that would pass kInReach, is transformed by FH instead.
// write(p, D) stores the result of the thread's line and write_at(line, p, D) that of
// line `line` of the block (D = kNone: no source of the field on the line).
constexpr int kInReach = 64;
constexpr int kInList = 2048;  // occupied voxels listed per tile, (q << 4) | line
static_assert(kLines <= 16 && kEdtMaxSide <= 4096, "a list entry fits 16 bits");

template <class Val, class Link, class Rec, class Decode, class Write, class WriteAt>
__device__ __forceinline__ void fh_lines(uint32_t* lds, int n, const Rec* base, long long stride,
                                         bool stage_ok, bool line_ok, int fld,
                                         Decode&& decode, Write&& write, WriteAt&& write_at) {
  constexpr uint32_t kNoVal = Tile<Val, Link>::kNoVal;
  Tile<Val, Link> T = carve_tile<Val, Link>(lds, n);
  uint32_t* occ_bits = lds + tile_bytes<Val, Link>(n) / sizeof(uint32_t);  // [n], bit = line
  // Lines with an output (a voxel that is not a source of the field), voxels listed.
  uint32_t* flags = occ_bits + n;
  uint16_t* list = reinterpret_cast<uint16_t*>(flags + 2);  // [kInList]
  for (int i = threadIdx.x; i < n + 2; i += kFhThreads) occ_bits[i] = 0u;
  __syncthreads();

  constexpr int kRowsPerPass = kFhThreads / kLines;  // 16
  constexpr int kBatch = 16;
  const int sl = threadIdx.x % kLines;
  const uint32_t sbit = 1u << sl;
  {
    bool has_output = false;
    for (int q0 = threadIdx.x / kLines; q0 < n; q0 += kRowsPerPass * kBatch) {
      Rec v[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) v[j] = base[min(q0 + j * kRowsPerPass, n - 1) * stride];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int q = q0 + j * kRowsPerPass;
        if (q < n) {
          bool occ = false;
          const uint32_t x = decode(v[j], occ);
          // D_out's sample is 0 on occupied voxels; D_in keeps v and tells the
          // sources (free voxels, sample 0) by their occupancy bit.
          const uint32_t sample = (fld == 0 && occ) ? 0u : x;
          T.f[q * kTs + sl] = (Val)(stage_ok && sample != kNone ? sample : kNoVal);
          if (stage_ok && occ) {
            atomicOr(&occ_bits[q], sbit);
            if (fld == 1) {
              const uint32_t at = atomicAdd(&flags[1], 1u);
              if (at < (uint32_t)kInList) list[at] = (uint16_t)((q << 4) | sl);
            }
          }
          has_output |= stage_ok && (occ == (fld == 1));
        }
      }
    }
    if (has_output) atomicOr(&flags[0], sbit);
  }
  __syncthreads();
  const Band B = my_band(n);
  const uint32_t with_output = flags[0];
  if (with_output == 0u) return;  // uniform across the block
  const bool active = line_ok && ((with_output >> B.line) & 1u);
  if (fld == 0) {
    tile_fh(T, n, active, occ_bits, [&](int p, uint32_t d, bool o) {
      if (!o) write(p, d);
    });
    return;
  }

  // D_in by the bounded search, listed voxel i on thread i mod kFhThreads.
  const uint32_t n_occ = flags[1];
  bool unresolved = n_occ > (uint32_t)kInList;
  for (int i = threadIdx.x; !unresolved && i < (int)n_occ; i += kFhThreads) {
    const int e = list[i];
    const int line = e & 15, p = e >> 4;
    const Val* f = T.f + line;
    const uint32_t fp = f[p * kTs];
    uint32_t best = fp == kNoVal ? kNone : fp;
    const int dmax = max(p, n - 1 - p);  // beyond it no candidate is left
    // kStep distances per round, all loads of a round issued together; after a
    // round every candidate left costs at least (d0 + kStep)^2.
    constexpr int kStep = 4;
    bool done = false;
    for (int d0 = 1; d0 <= kInReach; d0 += kStep) {
      uint32_t ob[2 * kStep], fb[2 * kStep];
#pragma unroll
      for (int c = 0; c < kStep; ++c) {
        const int qa = max(p - d0 - c, 0), qb = min(p + d0 + c, n - 1);
        ob[2 * c] = occ_bits[qa];
        fb[2 * c] = f[qa * kTs];
        ob[2 * c + 1] = occ_bits[qb];
        fb[2 * c + 1] = f[qb * kTs];
      }
#pragma unroll
      for (int c = 0; c < 2 * kStep; ++c) {
        const int d = d0 + c / 2;
        const int q = (c & 1) ? p + d : p - d;
        const uint32_t fq = ((ob[c] >> line) & 1u) ? fb[c] : 0u;
        if (q >= 0 && q < n && fq != kNoVal) best = min(best, (uint32_t)(d * d) + fq);
      }
      const int dn = d0 + kStep;  // nearest distance not yet searched
      if (dn > dmax || (uint32_t)(dn * dn) >= best) {
        done = true;
        break;
      }
    }
    if (done)
      write_at(line, p, best);
    else
      unresolved = true;  // the search would pass kInReach
  }
  if (!__syncthreads_or(unresolved)) return;
  // FH on f_in: the free voxels' samples become 0 (each thread rewrites the entries
  // it staged).
  for (int q = threadIdx.x / kLines; q < n; q += kRowsPerPass)
    if (!((occ_bits[q] >> sl) & 1u)) T.f[q * kTs + sl] = (Val)0;
  __syncthreads();
  tile_fh(T, n, active, occ_bits, [&](int p, uint32_t d, bool o) {
    if (o) write(p, d);
  });
}

// Work item (tile, field) of block b.  All D_out items come first (they take longest,
// so the short D_in blocks fill the end of the launch).  Within a field, blocks are
// dispatched to XCD b mod 8; the G neighbouring tiles that share 128-byte lines of the
// records form a group that runs on one XCD, so each line is fetched into one L2 once,
// and consecutive groups go to consecutive XCDs, so that every XCD gets a share of
// every region of the grid (a contiguous run per XCD leaves the XCDs holding the
// obstacle-dense regions to finish last).  Returns false for the padding blocks.
template <int G>
__host__ __device__ __forceinline__ long long xcd_half(long long tiles) {
  return 8 * (((tiles + G - 1) / G + 7) / 8) * G;  // blocks per field, a multiple of 8
}
template <int G>
__device__ __forceinline__ bool xcd_item(long long tiles, long long& tile, int& fld) {
  const long long half = xcd_half<G>(tiles);
  fld = blockIdx.x >= half;
  const long long b = blockIdx.x - (fld ? half : 0);
  const long long k = b / 8;  // k-th item of this XCD
  tile = ((b % 8) + 8 * (k / G)) * G + k % G;
  return tile < tiles;
}
template <int G>
unsigned xcd_grid(long long tiles) {
  return (unsigned)(2 * xcd_half<G>(tiles));
}
// Tiles per 128-byte line: 16 lines x 2-byte x-records, 16 lines x 4-byte y-records.
constexpr int kGroupY = 4, kGroupZ = 2;

// Pass y: block = 16 consecutive lines (x, z) of one field.
template <class Val, class Link>
__global__ __launch_bounds__(kFhThreads) void edt_pass_y_kernel(
    const uint16_t* __restrict__ xrec, uint32_t* __restrict__ yrec, int nx, int ny, int nz) {
  extern __shared__ uint32_t lds[];
  const int lines = nx * nz;
  long long tile;
  int fld;
  if (!xcd_item<kGroupY>((lines + kLines - 1) / kLines, tile, fld)) return;  // whole block
  const int line0 = (int)tile * kLines;  // flattened (z, x) < 2^18
  const long long plane = (long long)nx * ny;
  auto line_out = [&](int l) {  // records of block line l (clamped into the grid)
    const int i = min(line0 + l, lines - 1);
    const int z = i / nx;
    return yrec + z * plane + (i - z * nx);
  };
  const int si = line0 + (int)(threadIdx.x % kLines);
  const bool stage_ok = si < lines;
  const int sz = stage_ok ? si / nx : 0, sx = stage_ok ? si - sz * nx : 0;
  const int line = (int)(threadIdx.x / kG);
  uint32_t* out = line_out(line);
  const uint32_t occ_flag = fld == 1 ? kYOcc : 0u;
  fh_lines<Val, Link>(
      lds, ny, xrec + sz * plane + sx, nx, stage_ok, line0 + line < lines, fld,
      [](uint16_t r, bool& occ) -> uint32_t {
        occ = r & kXOcc;
        if (r & kXNone) return kNone;
        const uint32_t d = r & 0x3FFFu;
        return d * d;
      },
      [&](int p, uint32_t d) { out[(long long)p * nx] = occ_flag | (d == kNone ? kYNone : d); },
      [&](int l, int p, uint32_t d) {
        line_out(l)[(long long)p * nx] = occ_flag | (d == kNone ? kYNone : d);
      });
}

// The outputs of voxel i, which is occupied or not and has squared distance D to the
// nearest voxel of the other kind (none_value: none in the grid): phi = voxel *
// (sqrt(D_out) - sqrt(D_in)), in float64 and rounded to float32 once, and/or the two
// squared fields.  One of D_out, D_in is 0 (a voxel is a source of one field), so phi
// is exactly +-voxel * sqrt(D) (subtracting sqrt(0) = 0 and negating are exact).
struct FieldOut {
  float* phi;     // [nvox] or null
  uint32_t* d2;   // [2][nvox] or null
  long long nvox;
  double voxel;
  uint32_t none_value;
  __device__ __forceinline__ void put(long long i, bool occ, uint32_t d) const {
    const uint32_t D = d == kNone ? none_value : d;
    if (d2) {
      d2[i] = occ ? 0u : D;
      d2[nvox + i] = occ ? D : 0u;
    }
    if (phi) {
      const double v = voxel * __builtin_sqrt((double)D);
      phi[i] = (float)(occ ? -v : v);
    }
  }
};

// Pass z: block = 16 consecutive lines (x, y) of one field; the D_out block writes the
// outputs of the free voxels, the D_in block those of the occupied ones.
template <class Link>
__global__ __launch_bounds__(kFhThreads) void edt_pass_z_kernel(
    const uint32_t* __restrict__ yrec, int nx, int ny, int nz, FieldOut fo) {
  extern __shared__ uint32_t lds[];
  const long long plane = (long long)nx * ny;
  long long tile;
  int fld;
  if (!xcd_item<kGroupZ>((plane + kLines - 1) / kLines, tile, fld)) return;  // whole block
  const long long line0 = tile * kLines;  // flattened (y, x)
  const long long si = line0 + (long long)(threadIdx.x % kLines);
  const long long li = line0 + (long long)(threadIdx.x / kG);
  const long long out0 = li < plane ? li : 0;
  const bool occ = fld == 1;
  fh_lines<uint32_t, Link>(
      lds, nz, yrec + (si < plane ? si : 0), plane, si < plane, li < plane, fld,
      [](uint32_t r, bool& o) -> uint32_t {
        o = r & kYOcc;
        return (r & kYNone) ? kNone : (r & kYVal);
      },
      [&](int p, uint32_t d) { fo.put(out0 + p * plane, occ, d); },
      [&](int l, int p, uint32_t d) {
        const long long i = line0 + l < plane ? line0 + l : plane - 1;
        fo.put(i + p * plane, occ, d);
      });
}

template <class Val, class Link>
size_t fh_lds_bytes(int n) {
  return tile_bytes<Val, Link>(n) + (size_t)(n + 2) * sizeof(uint32_t) +
         (size_t)kInList * sizeof(uint16_t);
}

template <class Link>
void launch_fh_passes(const uint16_t* xrec, uint32_t* yrec, int nx, int ny, int nz,
                      const FieldOut& fo, hipStream_t stream) {
  const long long plane = (long long)nx * ny;
  const long long ly = (long long)nx * nz;
  const dim3 ygrid(xcd_grid<kGroupY>((ly + kLines - 1) / kLines));
  // x-pass distances are at most nx - 1: their squares fit 16 bits below 0xFFFF
  // when nx <= 256.
  if (nx <= 256)
    edt_pass_y_kernel<uint16_t, Link><<<ygrid, kFhThreads, fh_lds_bytes<uint16_t, Link>(ny),
                                        stream>>>(xrec, yrec, nx, ny, nz);
  else
    edt_pass_y_kernel<uint32_t, Link><<<ygrid, kFhThreads, fh_lds_bytes<uint32_t, Link>(ny),
                                        stream>>>(xrec, yrec, nx, ny, nz);
  edt_pass_z_kernel<Link><<<dim3(xcd_grid<kGroupZ>((plane + kLines - 1) / kLines)), kFhThreads,
                            fh_lds_bytes<uint32_t, Link>(nz), stream>>>(yrec, nx, ny, nz, fo);
}

}  // namespace

size_t edt_workspace_bytes(long long nvox) {
  // y-pass records (u32), then the x-pass records (u16).
  return (size_t)nvox * (2 * sizeof(uint32_t));
}

size_t edt_lds_bytes(int n_line) {
  return n_line <= 255 ? fh_lds_bytes<uint32_t, uint8_t>(n_line)
                       : fh_lds_bytes<uint32_t, uint16_t>(n_line);
}

int launch_edt(const uint8_t* occ, int nx, int ny, int nz, float voxel, float* phi,
               uint32_t* d2, void* work, hipStream_t stream) {
  const long long plane = (long long)nx * ny;
  const long long nvox = plane * nz;
  uint32_t* yrec = static_cast<uint32_t*>(work);
  uint16_t* xrec = reinterpret_cast<uint16_t*>(yrec + nvox);
  const long long rows = (long long)ny * nz;
  const uint32_t none_value = (uint32_t)nx * nx + (uint32_t)ny * ny + (uint32_t)nz * nz;
  const long long rows_per_block = (long long)kRowWaves * kRowsPerWave;
  const dim3 xgrid((unsigned)((rows + rows_per_block - 1) / rows_per_block));
  const long long word_rows_per_block = (long long)kRowWaves * kWordRows;
  if (nx <= 256 && nx % 4 == 0 && reinterpret_cast<uintptr_t>(occ) % 4 == 0 &&
      reinterpret_cast<uintptr_t>(xrec) % 8 == 0)
    hipLaunchKernelGGL(edt_pass_x_words_kernel,
                       dim3((unsigned)((rows + word_rows_per_block - 1) / word_rows_per_block)),
                       dim3(64 * kRowWaves), 0, stream, occ, nx, rows, xrec);
  else if (nx <= 256)
    hipLaunchKernelGGL(edt_pass_x_kernel<4>, xgrid, dim3(64 * kRowWaves), 0, stream, occ, nx,
                       rows, xrec);
  else
    hipLaunchKernelGGL(edt_pass_x_kernel<kEdtMaxSide / 64>, xgrid, dim3(64 * kRowWaves), 0,
                       stream, occ, nx, rows, xrec);
  const FieldOut fo{phi, d2, nvox, (double)voxel, none_value};
  if (ny <= 255 && nz <= 255)
    launch_fh_passes<uint8_t>(xrec, yrec, nx, ny, nz, fo, stream);
  else
    launch_fh_passes<uint16_t>(xrec, yrec, nx, ny, nz, fo, stream);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace smpc
