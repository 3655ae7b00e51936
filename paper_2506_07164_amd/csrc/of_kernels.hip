// of_kernels.hip -- gfx950 kernels of the Oriented FAST pipeline.
//
// Steps (one launch each, over every level of every frame of a call):
//   k_prologue       -- per-(frame, level) plan (cached behind a signature), zeroed
//                       counters and cell flags
//   k_pyramid        -- fixed-point bilinear levels (plain path and of_pyramid_build)
//   k_mark           -- segment test (Eq. 1, run of 9 of 16) at both thresholds over LDS
//                       tiles; the fused form resamples its tile from the input frame
//   k_detect         -- cell-aligned tiles: candidates at each cell's threshold, Harris R'
//                       (Sec. 3.2 / Eq. 4, 7x7 window), 3x3 NMS, per-cell top-K
//   k_select_orient  -- per-level top-N_l by (R' desc, y asc, x asc) through rank counts,
//                       fused with the intensity-centroid orientation of each winner
//   k_select         -- radix select of the best N_l of levels with very many candidates
//                       into a short list, which a second k_select_orient launch ranks
// Wave64 throughout; nothing here is a dense contraction, so there is no MFMA use.
#include <hip/hip_runtime.h>

#include <hip/hip_ext.h>

#include <mutex>

#include "of_kernels.h"

namespace ofk {

template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> G(T* p) {
  return (gptr<T>)p;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Read-only memory of a launch (the per-level plans and their signature, written by the
// prologue): a wave-uniform address in the constant address space is read with scalar
// loads, one request per wave, instead of a vector load per field that every wave of
// the launch aims at the same few cache lines.
template <class T>
using cptr = const __attribute__((address_space(4))) T*;

__device__ __forceinline__ LevelPlan plan_at(const LevelPlan* plan, int e) {
  static_assert(sizeof(LevelPlan) % 4 == 0, "plan copied as 32-bit words");
  LevelPlan P;
  const cptr<uint32_t> src = (cptr<uint32_t>)plan +
                             (size_t)__builtin_amdgcn_readfirstlane(e) * (sizeof(LevelPlan) / 4);
  uint32_t* dst = (uint32_t*)&P;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(LevelPlan) / 4); ++i) dst[i] = src[i];
  return P;
}

__device__ __forceinline__ int32_t plan_quota(const LevelPlan* plan, int e) {
  return ((cptr<LevelPlan>)plan)[e].quota;
}


// 16-byte candidate records and 32-byte keypoints move as native vectors (class types
// cannot be copied across address spaces).
__device__ __forceinline__ Cand load_cand(gptr<const Cand> p) {
  const u32x4 v = *(gptr<const u32x4>)p;
  Cand c;
  c.score = (int64_t)(((uint64_t)v.y << 32) | v.x);
  c.pos = v.z;
  c.pad = 0;
  return c;
}

__device__ __forceinline__ void store_cand(gptr<Cand> p, int64_t score, uint32_t pos) {
  u32x4 v;
  v.x = (uint32_t)(uint64_t)score;
  v.y = (uint32_t)((uint64_t)score >> 32);
  v.z = pos;
  v.w = 0u;
  *(gptr<u32x4>)p = v;
}

__device__ __forceinline__ void store_keypoint(gptr<of_keypoint> p, int x, int y, int level,
                                               int m10, int m01, float angle, int64_t score) {
  u32x4 a, b;
  a.x = (uint32_t)x;
  a.y = (uint32_t)y;
  a.z = (uint32_t)level;
  a.w = (uint32_t)m10;
  b.x = (uint32_t)m01;
  b.y = __float_as_uint(angle);
  b.z = (uint32_t)(uint64_t)score;
  b.w = (uint32_t)((uint64_t)score >> 32);
  gptr<u32x4> q = (gptr<u32x4>)p;
  q[0] = a;
  q[1] = b;
}

// ---------------------------------------------------------------- helpers --

__device__ __forceinline__ int imin3(int a, int b, int c) { return min(min(a, b), c); }
__device__ __forceinline__ int imax3(int a, int b, int c) { return max(max(a, b), c); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Byte offset of row y in a buffer of `stride` bytes per row, by one full-rate 24-bit
// multiply: every frame (stride < 2^24, at most 2^31 bytes, checked by the host), level
// buffer, bitmap and slot table here has rows and strides below 2^24 and spans below
// 2^32 bytes.
__device__ __forceinline__ uint32_t row_off(int y, int stride) {
  return (uint32_t)__umul24((uint32_t)y, (uint32_t)stride);
}

// floor(i / d) for small operands: recip16(d) = ceil(2^16 / d), and (i * recip16(d)) >> 16
// is exact while i * d < 2^16 (its error i (recip16(d) d - 2^16) / (d 2^16) stays below
// 1 / d, under the distance from i / d to the next integer).
__device__ __forceinline__ uint32_t recip16(int d) {
  return (65536u + (uint32_t)d - 1u) / (uint32_t)d;
}
__device__ __forceinline__ int div16(int i, uint32_t r) {
  return (int)((uint32_t)__umul24((uint32_t)i, r) >> 16);
}

// Per-level counters spread over kCountSpread sub-counters (see kCountSpread).
__device__ __forceinline__ void count_add(uint32_t* c, int stride, uint32_t v) {
  atomicAdd(c + (int)(blockIdx.x % (unsigned)kCountSpread) * stride, v);
}
__device__ __forceinline__ uint32_t count_sum(gptr<const uint32_t> c, int stride) {
  uint32_t v[kCountSpread];
#pragma unroll
  for (int k = 0; k < kCountSpread; ++k) v[k] = c[k * stride];
  uint32_t t = 0;
#pragma unroll
  for (int k = 0; k < kCountSpread; ++k) t += v[k];
  return t;
}

// Ranking order: higher R' first; equal R' -> smaller y, then smaller x (pos = y<<16|x).
__device__ __forceinline__ bool better(int64_t sa, uint32_t pa, int64_t sb, uint32_t pb) {
  return sa > sb || (sa == sb && pa < pb);
}


// Launch-wide values every block needs before its first tile.  They are read together,
// before any branch depends on them, so their scalar loads share one trip to memory
// rather than forming a chain of dependent trips (each a full memory latency at kernel
// start, when the caches are cold).  b is row `row` of the small-batch prefix table.
// Threads per block of the tile kernels, the selection and the helpers below (their
// launches use exactly this; a constant saves reading the launch size from memory).
constexpr int kBlock = 256;

struct Head {
  LevelPlan* plan;
  const uint64_t* ws_sig;
  uint64_t sig;
  int32_t n_entries, total, entry, persistent, bands, small;
  uint32_t* qctr;
  int32_t cell;
  Tune t;
  uint32_t* counters;
  uint8_t* flags;
  int32_t b[kSmallEntries + 1];
};

__device__ __forceinline__ Head read_head(const KArgs& a, int row) {
  Head h;
  h.plan = a.plan;
  h.ws_sig = a.ws_sig;
  h.sig = a.sig;
  h.n_entries = a.n_entries;
  h.total = a.total;
  h.entry = a.entry;
  h.persistent = a.persistent;
  h.bands = a.bands;
  h.small = a.small;
  h.qctr = a.qctr;
  h.cell = a.cell;
  h.t = a.t;
  h.counters = a.counters;
  h.flags = a.flags;
#pragma unroll
  for (int i = 0; i <= kSmallEntries; ++i) h.b[i] = a.sbase[row * (kSmallEntries + 1) + i];
  // every value in a scalar register here: no load is left for after a branch
  asm volatile("" ::"s"(h.plan), "s"(h.ws_sig), "s"(h.sig), "s"(h.n_entries), "s"(h.total),
               "s"(h.entry), "s"(h.persistent), "s"(h.bands), "s"(h.small), "s"(h.qctr),
               "s"(h.cell), "s"(h.counters), "s"(h.flags));
  asm volatile("" ::"s"(h.t.mark_words), "s"(h.t.mark_rows), "s"(h.t.det_cx), "s"(h.t.det_cy),
               "s"(h.t.det_w), "s"(h.t.det_h));
  asm volatile("" ::"s"(h.b[0]), "s"(h.b[1]), "s"(h.b[2]), "s"(h.b[3]), "s"(h.b[4]),
               "s"(h.b[5]), "s"(h.b[6]), "s"(h.b[7]), "s"(h.b[8]));
  asm volatile("" ::"s"(h.b[9]), "s"(h.b[10]), "s"(h.b[11]), "s"(h.b[12]), "s"(h.b[13]),
               "s"(h.b[14]), "s"(h.b[15]), "s"(h.b[16]));
  return h;
}

// Entry of unit g and the entry's first unit, from a small-batch prefix row (entries
// past the last hold INT32_MAX).  Unrolled: the row is in scalar registers.
__device__ __forceinline__ void small_entry(const int32_t (&b)[kSmallEntries + 1], int g, int* e,
                                            int* start) {
  int ee = 0, st = 0;
#pragma unroll
  for (int i = 1; i < kSmallEntries; ++i) {
    if (g >= b[i]) {
      ee = i;
      st = b[i];
    }
  }
  *e = ee;
  *start = st;
}

// The same with the entry's end: its successor's first unit, or the launch's total.
__device__ __forceinline__ void small_entry(const int32_t (&b)[kSmallEntries + 1], int g, int* e,
                                            int* start, int* end) {
  int ee = 0, st = 0, en = b[kSmallEntries];
#pragma unroll
  for (int i = 1; i < kSmallEntries; ++i) {
    if (g >= b[i]) {
      ee = i;
      st = b[i];
    } else {
      en = min(en, b[i]);
    }
  }
  *e = ee;
  *start = st;
  *end = en;
}

// Cross-lane sums by DPP (every lane of the wave active): lane exchanges inside rows of
// 16 lanes ride on the adds, with no LDS round trip.  quad_perm [1,0,3,2] and
// [2,3,0,1] give each lane its quad's sum, row_half_mirror pairs the two quads of an
// 8-lane group, row_mirror the two halves of a row.
template <int CTRL>
__device__ __forceinline__ int dpp_add(int v) {
  return v + __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

// Sum over each aligned group of 8 lanes, in every lane of the group.
__device__ __forceinline__ int group8_sum(int v) {
  v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
  return dpp_add<0x141>(v);  // row_half_mirror
}

// Inclusive prefix sum over the 64 lanes (every lane active): sums of 4 lanes from the
// original values shifted right 1..3 within the row, then the row prefix doubled by
// shifts of 4 and 8, then row 15's lane broadcast into rows 1 and 3 and lane 31 into
// rows 2 and 3.  Lanes a shift moves out of a row add zero.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v0) {
  const int x = (int)v0;
  int t = x + __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  t += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);         // row_shr:2
  t += __builtin_amdgcn_update_dpp(0, x, 0x113, 0xf, 0xf, true);         // row_shr:3
  t += __builtin_amdgcn_update_dpp(0, t, 0x114, 0xf, 0xe, false);        // row_shr:4
  t += __builtin_amdgcn_update_dpp(0, t, 0x118, 0xf, 0xc, false);        // row_shr:8
  t += __builtin_amdgcn_update_dpp(0, t, 0x142, 0xa, 0xf, false);        // row_bcast:15
  t += __builtin_amdgcn_update_dpp(0, t, 0x143, 0xc, 0xf, false);        // row_bcast:31
  return (uint32_t)t;
}

// Sum over the 64 lanes, wave-uniform: the four row sums read into scalar registers.
__device__ __forceinline__ int wave_sum(int v) {
  v = dpp_add<0x140>(group8_sum(v));  // row_mirror
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

// Segment test at two thresholds from the 16 circle pixels c[i] and the centre p.  A
// bright run of 9 at threshold t exists iff max_s min_{k<9} c[s+k] - p >= t; a dark run
// iff p - min_s max_{k<9} c[s+k] >= t (the centre is one constant of every difference,
// so the windows are taken over the pixels themselves).  Both come from 3-input min/max
// over cyclic windows (3 x 3 = 9 positions), folded over the 16 starts 3 at a time.
// Returns bit 0 = corner at t_lo, bit 1 = at t_hi.
__device__ __forceinline__ uint32_t segment_test_px(const int (&c)[16], int p, int t_lo,
                                                    int t_hi) {
  int mn3[16], mx3[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    mn3[i] = imin3(c[i], c[(i + 1) & 15], c[(i + 2) & 15]);
    mx3[i] = imax3(c[i], c[(i + 1) & 15], c[(i + 2) & 15]);
  }
  int m9[16], M9[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    m9[i] = imin3(mn3[i], mn3[(i + 3) & 15], mn3[(i + 6) & 15]);
    M9[i] = imax3(mx3[i], mx3[(i + 3) & 15], mx3[(i + 6) & 15]);
  }
  int sb = imax3(m9[0], m9[1], m9[2]), sd = imin3(M9[0], M9[1], M9[2]);
#pragma unroll
  for (int i = 3; i < 15; i += 2) {
    sb = imax3(sb, m9[i], m9[i + 1]);
    sd = imin3(sd, M9[i], M9[i + 1]);
  }
  sb = max(sb, m9[15]);
  sd = min(sd, M9[15]);
  const int s = max(sb - p, p - sd);
  return (s >= t_lo ? 1u : 0u) | (s >= t_hi ? 2u : 0u);
}

// The same from the 16 differences d[i] = I_i - I_p (a centre of 0).
__device__ __forceinline__ uint32_t segment_test2(const int (&d)[16], int t_lo, int t_hi) {
  return segment_test_px(d, 0, t_lo, t_hi);
}

// Circle differences around pixel c of an LDS tile with row pitch P.  Positions 1..16
// of the radius-3 Bresenham circle, clockwise from the top, y down.
__device__ __forceinline__ void circle_diffs(const uint8_t* c, int P, int (&d)[16]) {
  const int p = c[0];
  d[0] = c[-3 * P] - p;
  d[1] = c[-3 * P + 1] - p;
  d[2] = c[-2 * P + 2] - p;
  d[3] = c[-P + 3] - p;
  d[4] = c[3] - p;
  d[5] = c[P + 3] - p;
  d[6] = c[2 * P + 2] - p;
  d[7] = c[3 * P + 1] - p;
  d[8] = c[3 * P] - p;
  d[9] = c[3 * P - 1] - p;
  d[10] = c[2 * P - 2] - p;
  d[11] = c[P - 3] - p;
  d[12] = c[-3] - p;
  d[13] = c[-P - 3] - p;
  d[14] = c[-2 * P - 2] - p;
  d[15] = c[-3 * P - 1] - p;
}

// Bytes p[0..3] of a row as one little-endian word, zero past the row's last readable
// byte (room = bytes left in the row, >= 1): one dword load at any alignment, moved back
// so that it ends at the row's limit when fewer than 4 bytes remain.
typedef uint32_t u32_any_align_g __attribute__((aligned(1)));
__device__ __forceinline__ uint32_t load_word(gptr<const uint8_t> p, int room) {
  const int back = room >= 4 ? 0 : 4 - room;
  return *(gptr<const u32_any_align_g>)(p - back) >> (8 * back);
}

// Bytes p[0] (low) and p[1] (high) with one 16-bit load at any alignment.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// (lo, hi) as two 16-bit lanes (both < 2^16).
__device__ __forceinline__ u16x2 pair16(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(u16x2, lo | (hi << 16));
}

// Bytes 0 and 1 of v as two 16-bit lanes.
__device__ __forceinline__ u16x2 bytes16(uint32_t v) {
  return __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(0u, v, 0x0c010c00u));
}

// R4's blend from the tap bytes: bytes 0, 1 of t (row y0) and b (row y0 + 1) with
// weights wx = (256 - wx, wx) and wy = (256 - wy, wy), by 16-bit dot products: the
// horizontal blends are at most 256 * 255, so they pack into one word for the vertical
// blend; all exact.
__device__ __forceinline__ uint32_t blend_q8(uint32_t t, uint32_t b, u16x2 wx, u16x2 wy) {
  const uint32_t top = __builtin_amdgcn_udot2(bytes16(t), wx, 0u, false);
  const uint32_t bot = __builtin_amdgcn_udot2(bytes16(b), wx, 0u, false);
  return __builtin_amdgcn_udot2(pair16(top, bot), wy, 32768u, false) >> 16;
}

typedef uint16_t u16_any_align __attribute__((aligned(1)));
typedef uint32_t u32_any_align __attribute__((aligned(1)));
__device__ __forceinline__ uint32_t load_pair(gptr<const uint8_t> p) {
  return *(gptr<const u16_any_align>)p;
}

// Rows [y0, y1) x columns [x0, x1) of a level into LDS (row pitch lp), as 32-bit words
// (x0 a multiple of 4; bytes past the row's readable limit read as zero), or as 16-byte
// chunks where stage_wide allows (bytes past x1 up to the chunk's end are staged too).
// The block's threads take the units in order, U words' worth per thread per pass.
// stage_issue loads the first pass into registers and stage_store writes it to LDS
// (then loads and stores any further passes), so that a caller can issue other loads in
// between and wait for all of them at once: a tile of up to U * kBlock words costs one
// round trip to memory.
// s_waitcnt operand (gfx9 encoding) that waits for every vector memory operation of the
// wave: vmcnt 0, expcnt and lgkmcnt at their maxima (no wait).
constexpr int kWaitVmem = 0x0F70;

typedef u32x4 u32x4_any_align_g __attribute__((aligned(1)));

// CHUNKS: the 16-byte form is compiled in (U a multiple of 4).
template <int U, bool CHUNKS>
struct Stage {
  static_assert(!CHUNKS || U % 4 == 0, "whole chunks per pass");
  uint32_t v[U];
  int nw, total, drow, dw;  // units per row, in all; walk advance per kBlock units
  int row, w, i0;           // walk position of this thread's next unit; first unit of the pass
  bool wide;                // 16-byte units (U / 4 per thread and pass), else words
};

// Words i = i0 + u * kBlock + threadIdx.x of a pass: (row, word) advanced by (drow, dw)
// per kBlock words, so only the first needs a division.  Every load is issued without a
// branch, so the U loads of a pass are all in flight before the first wait (a caller can
// issue other loads between stage_issue and stage_store and wait for all of them at
// once).  A word past the region re-reads the region's first word and is dropped;
// stage_store waits for every load of the pass, dropped ones included, so that none is
// still in flight when its register is next written in a later step.
template <int U, bool CHUNKS>
__device__ __forceinline__ void stage_begin(Stage<U, CHUNKS>& st, int x0, int x1, int y0,
                                            int y1, int row_limit, int lp) {
  st.wide = CHUNKS && stage_wide(x0, x1, row_limit, lp);  // the same for the block
  st.nw = st.wide ? (x1 - x0 + 15) >> 4 : (x1 - x0 + 3) >> 2;
  st.total = st.nw * (y1 - y0);
  st.drow = (int)((uint32_t)kBlock / (uint32_t)st.nw);
  st.dw = kBlock - st.drow * st.nw;
  st.row = (int)(threadIdx.x / (uint32_t)st.nw);
  st.w = (int)threadIdx.x - st.row * st.nw;
  st.i0 = 0;
}

template <int U, bool CHUNKS>
__device__ __forceinline__ void stage_issue(Stage<U, CHUNKS>& st, gptr<const uint8_t> src,
                                            int stride, int row_limit, int x0, int y0) {
  int row = st.row, w = st.w;
  const gptr<const uint8_t> first = src + (row_off(y0, stride) + x0);
  if constexpr (CHUNKS) {
    if (st.wide) {
#pragma unroll
      for (int c = 0; c < U / 4; ++c) {
        const bool in = st.i0 + c * kBlock + (int)threadIdx.x < st.total;
        const gptr<const uint8_t> p = in ? src + (row_off(y0 + row, stride) + x0 + 16 * w)
                                         : first;
        const u32x4 q = *(gptr<const u32x4_any_align_g>)p;
        st.v[4 * c] = q.x;
        st.v[4 * c + 1] = q.y;
        st.v[4 * c + 2] = q.z;
        st.v[4 * c + 3] = q.w;
        row += st.drow;
        w += st.dw;
        if (w >= st.nw) {
          w -= st.nw;
          ++row;
        }
      }
      return;
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool in = st.i0 + u * kBlock + (int)threadIdx.x < st.total;
    const int x = x0 + 4 * w;
    const int room = in ? row_limit - x : 4;
    const int back = room >= 4 ? 0 : 4 - room;
    const gptr<const uint8_t> p = in ? src + (row_off(y0 + row, stride) + x - back) : first;
    st.v[u] = *(gptr<const u32_any_align_g>)p >> (8 * back);
    row += st.drow;
    w += st.dw;
    if (w >= st.nw) {
      w -= st.nw;
      ++row;
    }
  }
}

template <int U, bool CHUNKS>
__device__ __forceinline__ void stage_store(Stage<U, CHUNKS>& st, uint8_t* lds, int lp) {
  int row = st.row, w = st.w;
  if constexpr (CHUNKS) {
    if (st.wide) {
#pragma unroll
      for (int c = 0; c < U / 4; ++c) {
        if (st.i0 + c * kBlock + (int)threadIdx.x < st.total) {
          uint32_t* d = (uint32_t*)(lds + row * lp + 16 * w);  // 4-byte aligned
          d[0] = st.v[4 * c];
          d[1] = st.v[4 * c + 1];
          d[2] = st.v[4 * c + 2];
          d[3] = st.v[4 * c + 3];
        }
        row += st.drow;
        w += st.dw;
        if (w >= st.nw) {
          w -= st.nw;
          ++row;
        }
      }
      __builtin_amdgcn_s_waitcnt(kWaitVmem);  // the dropped loads too
      st.row = row;
      st.w = w;
      st.i0 += U / 4 * kBlock;
      return;
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (st.i0 + u * kBlock + (int)threadIdx.x < st.total)
      *(uint32_t*)(lds + row * lp + 4 * w) = st.v[u];
    row += st.drow;
    w += st.dw;
    if (w >= st.nw) {
      w -= st.nw;
      ++row;
    }
  }
  __builtin_amdgcn_s_waitcnt(kWaitVmem);  // the dropped loads too
  st.row = row;
  st.w = w;
  st.i0 += U * kBlock;
}

// The passes left after the first (regions larger than U * kBlock words).
template <int U, bool CHUNKS>
__device__ __forceinline__ void stage_rest(Stage<U, CHUNKS>& st, uint8_t* lds, int lp,
                                           gptr<const uint8_t> src, int stride, int row_limit,
                                           int x0, int y0) {
  while (st.i0 < st.total) {
    stage_issue(st, src, stride, row_limit, x0, y0);
    stage_store(st, lds, lp);
  }
}

// A whole region, pass by pass.
template <int U, bool CHUNKS>
__device__ __forceinline__ void stage_all(uint8_t* lds, int lp, gptr<const uint8_t> src,
                                          int stride, int row_limit, int x0, int x1, int y0,
                                          int y1) {
  Stage<U, CHUNKS> st;
  stage_begin(st, x0, x1, y0, y1, row_limit, lp);
  stage_rest(st, lds, lp, src, stride, row_limit, x0, y0);
}

// Harris R' at LDS pixel (cx, cy) by one lane, in 16-bit pairs of window columns: the
// 9 x 9 neighbourhood is read as three aligned 32-bit words per row (bytes moved into
// 16-bit lanes by byte permutes), the horizontal differences hd = I[c+1] - I[c-1] and
// smoothings hs = I[c-1] + 2 I[c] + I[c+1] are formed for columns (0,1), (2,3), (4,5), (6,-)
// of the window, three rows are kept for G_x = hd[r-1] + 2 hd[r] + hd[r+1] and
// G_y = hs[r+1] - hs[r-1] (Eq. 4, separable), and the sums of products take one
// dot2 (two 16 x 16-bit products added to 32 bits) per pair.  Every intermediate fits
// 16 bits (|hd| <= 255, hs <= 1020, |G| <= 1020) and every sum 32 bits (49 * 2 * 1020^2),
// so the integers are those of the plain definition.  pix and the row pitch P are
// 4-aligned.
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void harris_row_pairs(const uint8_t* row, int s, s16x2 (&hd)[4],
                                                 s16x2 (&hs)[4]) {
  const uint32_t* w = (const uint32_t*)row;
  const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
  const uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)s);   // bytes 0..3
  const uint32_t mid = __builtin_amdgcn_alignbyte(w2, w1, (uint32_t)s);  // bytes 4..7
  const uint32_t b8 = (w2 >> (8 * s)) & 255u;                           // byte 8
  // p[k] = bytes (2k, 2k+1), q[k] = bytes (2k+1, 2k+2), each in two 16-bit lanes
  s16x2 p[5], q[4];
  p[0] = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(0u, lo, 0x0c010c00u));
  p[1] = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(0u, lo, 0x0c030c02u));
  p[2] = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(0u, mid, 0x0c010c00u));
  p[3] = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(0u, mid, 0x0c030c02u));
  p[4] = __builtin_bit_cast(s16x2, b8);
  q[0] = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(0u, lo, 0x0c020c01u));
  q[1] = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(mid, lo, 0x0c040c03u));
  q[2] = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(0u, mid, 0x0c020c01u));
  q[3] = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(b8, mid, 0x0c040c03u));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    hd[k] = p[k + 1] - p[k];
    hs[k] = p[k] + p[k + 1] + (s16x2)2 * q[k];
  }
  // column 7 is outside the window: its lanes are cleared
  hd[3] = __builtin_bit_cast(s16x2, __builtin_bit_cast(uint32_t, hd[3]) & 0xffffu);
  hs[3] = __builtin_bit_cast(s16x2, __builtin_bit_cast(uint32_t, hs[3]) & 0xffffu);
}

// Sums of G_x^2, G_y^2 and G_x G_y over window rows w0 .. w0 + nr - 1 (0 .. 6 from the
// top) of the 7x7 window at LDS pixel (cx, cy); NR >= nr rows are unrolled.
template <int NR>
__device__ __forceinline__ void harris_part(const uint8_t* pix, int P, int cx, int cy, int w0,
                                            int nr, int& sxx, int& syy, int& sxy) {
  const int a = cx - 4, s = a & 3;
  const uint8_t* row = pix + (cy - 4 + w0) * P + (a - s);
  s16x2 hd0[4], hs0[4], hd1[4], hs1[4];
  harris_row_pairs(row, s, hd0, hs0);
  harris_row_pairs(row + P, s, hd1, hs1);
  sxx = syy = sxy = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nr) {
      s16x2 hd2[4], hs2[4];
      harris_row_pairs(row + (r + 2) * P, s, hd2, hs2);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const s16x2 gx = hd0[k] + (s16x2)2 * hd1[k] + hd2[k];
        const s16x2 gy = hs2[k] - hs0[k];
        sxx = __builtin_amdgcn_sdot2(gx, gx, sxx, false);
        syy = __builtin_amdgcn_sdot2(gy, gy, syy, false);
        sxy = __builtin_amdgcn_sdot2(gx, gy, sxy, false);
        hd0[k] = hd1[k];
        hd1[k] = hd2[k];
        hs0[k] = hs1[k];
        hs1[k] = hs2[k];
      }
    }
  }
}

__device__ __forceinline__ int64_t harris_r(int sxx, int syy, int sxy) {
  const int64_t A = sxx, B = syy, C = sxy;
  return 25 * (A * B - C * C) - (A + B) * (A + B);
}

// Out of line: the rare path (candidates past the tile's score cache) has one copy, not
// one per call site, so the tile kernel's hot code stays compact.
__device__ __noinline__ int64_t harris_point(const uint8_t* pix, int P, int cx, int cy) {
  int sxx, syy, sxy;
  harris_part<7>(pix, P, cx, cy, 0, 7, sxx, syy, sxy);
  return harris_r(sxx, syy, sxy);
}

// R' of the n cached candidates (positions y << 16 | x, pixels staged from (sx0, sy0)),
// 2^lg adjacent lanes per candidate, each taking ceil(7 / 2^lg) window rows; the partial
// sums are added across the group.  Few candidates per tile: more lanes each, so that
// the step's latency is a few window rows rather than the whole window.  One code path
// for every group size (rows past a lane's share are skipped by uniform branches where
// no lane of the wave needs them), so that it stays in the instruction cache.
__device__ __forceinline__ void harris_cache(const uint8_t* pix, int P, const uint32_t* cpos,
                                             int64_t* crs, int n, int sx0, int sy0, int lg) {
  const int G = 1 << lg, nr_max = (7 + G - 1) >> lg;
  for (int i = (int)threadIdx.x; i < (n << lg); i += kBlock) {
    const int c = i >> lg, j = i & (G - 1);
    const uint32_t ps = cpos[c];
    const int w0 = j * nr_max, nr = min(nr_max, 7 - w0);
    int sxx, syy, sxy;
    harris_part<7>(pix, P, (int)(ps & 0xffff) - sx0, (int)(ps >> 16) - sy0, w0, nr, sxx, syy,
                   sxy);
    for (int o = 1; o < G; o <<= 1) {
      sxx += __shfl_xor(sxx, o, 64);
      syy += __shfl_xor(syy, o, 64);
      sxy += __shfl_xor(sxy, o, 64);
    }
    if (j == 0) crs[c] = harris_r(sxx, syy, sxy);
  }
}

// Block barrier that orders LDS accesses only.  __syncthreads() also waits for the
// block's global stores to complete; tiles that never read back their own global
// stores use this one so that stores drain while the next step runs.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Exclusive scan of cnt[0..n) into pre[0..n], pre[n] = total, by the whole block.
__device__ void block_scan_u32(const uint32_t* cnt, uint32_t* pre, int n, uint32_t* s_wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = kBlock >> 6;
  uint32_t carry = 0;
  for (int base = 0; base < n; base += kBlock) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < n ? cnt[i] : 0u;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) s_wsum[wave] = inc;
    lds_barrier();
    uint32_t woff = 0, total = 0;
    for (int w = 0; w < nwave; ++w) {
      const uint32_t s = s_wsum[w];
      if (w < wave) woff += s;
      total += s;
    }
    if (i < n) pre[i] = carry + woff + inc - v;
    carry += total;
    lds_barrier();
  }
  if (threadIdx.x == 0) pre[n] = carry;
  lds_barrier();
}

// m10 = sum dx I and m01 = sum dy I over the disk dx^2 + dy^2 <= r^2 around (x, y), by
// one wave.  For r <= 15 the 2r+1 square box is read with one 32-bit load per lane and
// box row: lane (row group lane / 8, column group lane % 8) reads 4 consecutive pixels
// starting at box column min(4 (lane % 8), 2r - 3), so every load stays inside the box,
// and counts only the pixels no lower column group holds; rows lane / 8 + 8k past the
// box are not read.  Larger radii take rows and columns in passes of 8 loads.
__device__ __forceinline__ void wave_moments(gptr<const uint8_t> lvl, int stride, int x, int y,
                                             int r, int lane, int* m10, int* m01) {
  const int span = 2 * r + 1;
  const int r2 = r * r;
  int a = 0, b = 0;
  if (r <= 15) {
    const int lr = lane >> 3, lc4 = (lane & 7) * 4;
    const int c0 = min(lc4, span - 4);  // first box column of this lane's load
    gptr<const uint8_t> base = lvl + (row_off(y - r, stride) + x - r + c0);
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int row = lr + 8 * k;
      v[k] = row < span ? *(gptr<const u32_any_align>)(base + row_off(row, stride)) : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int dy = lr + 8 * k - r;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = c0 + q;
        const int dx = c - r;
        const int px = (int)((v[k] >> (8 * q)) & 255u);
        const bool in = c >= lc4 && dx * dx + dy * dy <= r2;  // rows past the box read 0
        a += in ? dx * px : 0;
        b += in ? dy * px : 0;
      }
    }
  } else {
    const int cspan = min(span, 64);
    const int rows_per = 64 / cspan;
    const int lr = lane / cspan, lc = lane - lr * cspan;
    if (lr < rows_per) {
      for (int c0 = 0; c0 < span; c0 += cspan) {
        const int dx = c0 + lc - r;
        for (int k0 = 0; k0 * rows_per < span; k0 += 8) {
          int v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int dy = (k0 + k) * rows_per + lr - r;
            const bool in = dy <= r && dx <= r && dx * dx + dy * dy <= r2;
            v[k] = in ? (int)lvl[(size_t)(y + dy) * stride + x + dx] : 0;
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int dy = (k0 + k) * rows_per + lr - r;
            a += dx * v[k];
            b += dy * v[k];
          }
        }
      }
    }
  }
  *m10 = wave_sum(a);
  *m01 = wave_sum(b);
}

// Tile index: blockIdx.x once, or from the queue counter.  The next index is drawn
// when a tile starts and parked in LDS only when it ends, so the atomic's round trip
// overlaps the tile instead of stalling the block.
__device__ __forceinline__ void queue_start(const Head& h, uint32_t* ctr, int* s_next) {
  if (h.persistent && threadIdx.x == 0) *s_next = (int)atomicAdd(ctr, 1u);
}

__device__ __forceinline__ int queue_take(const Head& h, int iter, int* s_next) {
  if (!h.persistent) return iter == 0 ? (int)blockIdx.x : h.total;
  lds_barrier();
  return *s_next;
}

__device__ __forceinline__ int queue_prefetch(const Head& h, int g, uint32_t* ctr) {
  return (h.persistent && threadIdx.x == 0 && g < h.total) ? (int)atomicAdd(ctr, 1u) : 0;
}

__device__ __forceinline__ void queue_park(const Head& h, int next, int* s_next) {
  if (h.persistent && threadIdx.x == 0) *s_next = next;
}

// Copy of an exclusive prefix (n + 1 values) into LDS for entry lookups.
__device__ __forceinline__ void load_bases(int32_t* s_base, const int32_t* base, int n) {
  for (int i = threadIdx.x; i <= n; i += kBlock) s_base[i] = G(base)[i];
  lds_barrier();
}

// ---------------------------------------------------------------- prologue --

// Every block zeroes a share of the counters and cell flags.  Block 0 also checks the
// signature of the call shape stored in the workspace and rebuilds the plan only when
// it changed (new frames, sizes, pointers, parameters or tuning).
__global__ __launch_bounds__(1024) void k_prologue(PrologueArgs a) {
  __shared__ int64_t s_scan[1024];
  __shared__ int64_t s_tot;
  __shared__ int s_same;
  uint8_t* ws = a.ws;
  uint32_t* qctr = (uint32_t*)(ws + a.lay.off_hdr);
  uint64_t* sig = (uint64_t*)(ws + a.lay.off_hdr + 128);
  {
    uint32_t* counters = (uint32_t*)(ws + a.lay.off_counters);
    const int64_t ncnt = counter_words(a.lay.n_entries);
    uint4* fl = (uint4*)(ws + a.lay.off_flags);
    const int64_t nq = a.lay.flag_bytes / 16;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t k = t0; k < ncnt; k += stride) G(counters)[k] = 0u;
    const u32x4 zero = {0u, 0u, 0u, 0u};
    for (int64_t k = t0; k < nq; k += stride) ((gptr<u32x4>)G(fl))[k] = zero;
  }
  if (blockIdx.x != 0) return;
  if (threadIdx.x < 32) G(qctr)[threadIdx.x] = 0u;
  if (threadIdx.x == 0) s_same = *G(sig) == a.sig;
  __syncthreads();
  if (s_same) return;

  const int L = a.p.n_levels;
  const int nL = a.n * L;
  const int i = threadIdx.x;
  FrameGeom g;
  EntrySize s = {};
  int f = 0, l = 0;
  if (i < nL) {
    f = i / L;
    l = i - f * L;
    frame_geom(a.f[f].w, a.f[f].h, a.p, &g);
    entry_size(g, a.p, a.t, l, &s);
  }
  auto scan = [&](int64_t v) -> int64_t {
    s_scan[i] = i < nL ? v : 0;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t t = i >= o ? s_scan[i - o] : 0;
      __syncthreads();
      s_scan[i] += t;
      __syncthreads();
    }
    const int64_t incl = s_scan[i];
    if (i == 1023) s_tot = incl;
    __syncthreads();
    const int64_t r = incl - (i < nL ? v : 0);
    __syncthreads();
    return r;
  };
  const int64_t o_mark = scan(s.mark_tiles);
  const int64_t t_mark = s_tot;
  const int64_t o_det = scan(s.det_tiles);
  const int64_t t_det = s_tot;
  const int64_t o_sl = scan(s.sel_slots);
  const int64_t t_sl = s_tot;
  const int64_t o_flag = scan(s.flag_bytes);
  const int64_t o_bm = scan(s.bm_words);
  const int64_t o_cand = scan(s.cand_cap);
  const int64_t o_rank = scan(s.rank_slots);
  const int64_t t_rank = s_tot;
  const int64_t o_sel = scan(s.sel_cap);
  const int64_t o_lvl = scan(s.lvl_bytes);
  const int64_t o_pyr = scan(s.pyr_blocks);
  const int64_t t_pyr = s_tot;
  const int32_t rot = (int32_t)(scan(s.mark_ty % kXcds) % kXcds);
  int32_t* band_base = (int32_t*)(ws + a.lay.off_band_base);
  for (int k = 0; k < kXcds; ++k) {
    const int32_t rows = band_rows(s.mark_ty, rot, k);
    const int64_t o_band = scan(i < nL ? (int64_t)s.mark_tx * rows : 0);
    if (i < nL) band_base[k * (nL + 1) + i] = (int32_t)o_band;
    if (i == 0) band_base[k * (nL + 1) + nL] = (int32_t)s_tot;
  }
  const int32_t drot = (int32_t)(scan(s.det_ty % kXcds) % kXcds);
  int32_t* det_band_base = (int32_t*)(ws + a.lay.off_det_band_base);
  for (int k = 0; k < kXcds; ++k) {
    const int32_t rows = band_rows(s.det_ty, drot, k);
    const int64_t o_band = scan(i < nL ? (int64_t)s.det_tx * rows : 0);
    if (i < nL) det_band_base[k * (nL + 1) + i] = (int32_t)o_band;
    if (i == 0) det_band_base[k * (nL + 1) + nL] = (int32_t)s_tot;
  }

  LevelPlan* plan = (LevelPlan*)(ws + a.lay.off_plan);
  int32_t* mark_base = (int32_t*)(ws + a.lay.off_mark_base);
  int32_t* det_base = (int32_t*)(ws + a.lay.off_det_base);
  int32_t* sl_base = (int32_t*)(ws + a.lay.off_sel_base);
  int32_t* rank_base = (int32_t*)(ws + a.lay.off_rank_base);
  int32_t* pyr_base = (int32_t*)(ws + a.lay.off_pyr_base);
  uint32_t* counters = (uint32_t*)(ws + a.lay.off_counters);

  if (i < nL) {
    LevelPlan P;
    const EntryOffsets eo = {o_flag, o_bm, o_cand, o_sel, o_lvl, rot, drot, counters};
    fill_level_plan(P, a, ws, g, s, i, f, l, eo);
    plan[i] = P;
    mark_base[i] = (int32_t)o_mark;
    det_base[i] = (int32_t)o_det;
    sl_base[i] = (int32_t)o_sl;
    rank_base[i] = (int32_t)o_rank;
    pyr_base[i] = (int32_t)o_pyr;
  }
  if (i == 0) {
    mark_base[nL] = (int32_t)t_mark;
    det_base[nL] = (int32_t)t_det;
    sl_base[nL] = (int32_t)t_sl;
    rank_base[nL] = (int32_t)t_rank;
    pyr_base[nL] = (int32_t)t_pyr;
  }
  __threadfence();
  __syncthreads();
  if (i == 0) *sig = a.sig;
}

// ----------------------------------------------------------------- pyramid --

// One block = 64 x 16 output pixels of one level; the tap tables of its columns and rows
// are computed once in LDS.  Weights are Q8; one rounding at the end.
__device__ __forceinline__ void resample_block(gptr<const uint8_t> src, int src_w, int src_h,
                                               int src_stride, gptr<uint8_t> dst, int w, int h,
                                               int stride, int bx, int by, uint32_t* xt,
                                               uint32_t* yt) {
  const int t = threadIdx.x;
  if (t < 64 && bx + t < w) xt[t] = resample_tap(bx + t, src_w, w);
  if (t >= 64 && t < 80 && by + t - 64 < h) yt[t - 64] = resample_tap(by + t - 64, src_h, h);
  lds_barrier();
  const int lx = t & 63;
  const int x = bx + lx;
  if (x >= w) return;
  const uint32_t tx = xt[lx];
  const int x0 = tx >> 9, wx = tx & 511;
  const int x1 = min(x0 + 1, src_w - 1);
  int v[4][4];
  int wy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int ly = min((t >> 6) * 4 + k, h - 1 - by);
    const uint32_t ty = yt[ly];
    const int y0 = ty >> 9;
    wy[k] = ty & 511;
    const int y1 = min(y0 + 1, src_h - 1);
    v[k][0] = src[(size_t)y0 * src_stride + x0];
    v[k][1] = src[(size_t)y0 * src_stride + x1];
    v[k][2] = src[(size_t)y1 * src_stride + x0];
    v[k][3] = src[(size_t)y1 * src_stride + x1];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int y = by + (t >> 6) * 4 + k;
    if (y >= h) break;
    const int top = (256 - wx) * v[k][0] + wx * v[k][1];
    const int bot = (256 - wx) * v[k][2] + wx * v[k][3];
    dst[(size_t)y * stride + x] = (uint8_t)(((256 - wy[k]) * top + wy[k] * bot + 32768) >> 16);
  }
}

// Levels of one frame: blockIdx.z is the level.
__global__ __launch_bounds__(256) void k_pyramid(PyrArgs a) {
  __shared__ uint32_t xt[64], yt[16];
  const PyrLevel L = a.lv[blockIdx.z];
  const int bx = blockIdx.x * 64, by = blockIdx.y * 16;
  if (bx >= L.w || by >= L.h) return;
  resample_block(G(a.src), a.src_w, a.src_h, a.src_stride, G(L.dst), L.w, L.h, L.stride, bx, by,
                 xt, yt);
}

// Levels >= 1 of every frame of a batch: blocks are numbered through pyr_base.
__global__ __launch_bounds__(256) void k_pyramid_batch(KArgs a) {
  __shared__ uint32_t xt[64], yt[16];
  __shared__ int32_t s_base[kMaxEntries + 1];
  const Head h = read_head(a, 0);
  const uint64_t wsig = *(cptr<uint64_t>)h.ws_sig;  // compared before the plan's pointers are used
  const int g = (int)blockIdx.x;
  int e, b;
  if (h.small) {
    int st;
    small_entry(h.b, g, &e, &st);
    b = g - st;
  } else {
    load_bases(s_base, a.pyr_base, h.n_entries);
    e = uniform(prefix_entry(s_base, h.n_entries, g));
    b = g - s_base[e];
  }
  const LevelPlan P = plan_at(h.plan, e);
  if (wsig != h.sig) return;  // not the plan this launch was made for
  const int nbx = (P.W + 63) >> 6;
  const int by = b / nbx, bx = b - by * nbx;
  resample_block(G(P.base), P.base_w, P.base_h, P.base_stride, G(P.lvl_w), P.W, P.H,
                 P.lvl_stride, bx * 64, by * 16, xt, yt);
}

// ------------------------------------------------------------ segment test --

// Resampled pixels of a segment-test tile, K adjacent output columns per lane: columns
// [4, 4 + TW) of the tile (the 7 side columns are left to the caller).  The taps of K
// adjacent output columns lie within 8 bytes of a frame row when (K - 1) * bw < 6 * W
// (K = 4 below scale 2, K = 2 below scale 6), so one unaligned 64-bit load per source
// row serves all K (moved back from the row's end where 8 bytes would pass it); a byte
// permute takes each column's two tap bytes out of it into 16-bit lanes, and the K
// resampled bytes go to LDS in one 32- or 16-bit store.  The taps come from the tile's
// LDS tables: column i has x0 cx[i] and weights cw[i], row j source row offsets
// ro[2j], ro[2j + 1] and weights rwy[j].  Each wave step covers R tile rows
// (64 / (TW / K) lanes per row); RPI steps' loads are in flight at once.
template <int K, int TW, int RPI>
__device__ __forceinline__ void resample_groups(uint8_t* pix, int pitch, gptr<const uint8_t> base,
                                                int bw, int nx, int ny, const uint32_t* cx,
                                                const uint32_t* cw, const uint32_t* ro,
                                                const uint32_t* rwy, int lane, int wave) {
  constexpr int G = TW / K;                // lane groups per tile row
  constexpr int R = G <= 64 ? 64 / G : 1;  // tile rows per wave step
  constexpr int C = G <= 64 ? 1 : G / 64;  // column groups per lane
  typedef uint64_t u64_any_align __attribute__((aligned(1)));
  const int r = G <= 64 ? lane / G : 0;
  const int q0 = G <= 64 ? lane - r * G : lane;
  uint32_t b[C], sel[C][K];
  u16x2 wx[C][K];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int i0 = 4 + K * (q0 + 64 * c);
    uint32_t x0[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const int i = min(i0 + m, nx - 1);
      x0[m] = cx[i];
      wx[c][m] = __builtin_bit_cast(u16x2, cw[i]);
    }
    b[c] = min(x0[0], (uint32_t)(bw - 8));
    // bytes s and s + 1 of the 8 loaded (s <= 6) into the low bytes of the two halves
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const uint32_t sb = x0[m] - b[c];
      sel[c][m] = 0x0c000c00u | sb | ((sb + 1u) << 16);
    }
  }
  for (int j0 = R * RPI * wave; j0 < ny; j0 += R * RPI * 4) {
    uint64_t v[RPI][C][2];
    u16x2 wy[RPI];
#pragma unroll
    for (int h = 0; h < RPI; ++h) {
      const int j = min(j0 + h * R + r, ny - 1);
      const uint32_t o0 = ro[2 * j], o1 = ro[2 * j + 1];
      wy[h] = __builtin_bit_cast(u16x2, rwy[j]);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        v[h][c][0] = *(gptr<const u64_any_align>)(base + (o0 + b[c]));
        v[h][c][1] = *(gptr<const u64_any_align>)(base + (o1 + b[c]));
      }
    }
#pragma unroll
    for (int h = 0; h < RPI; ++h) {
      const int j = j0 + h * R + r;
      if (j >= ny) continue;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        // R4's blend: horizontal 16-bit dot products per source row, packed into one
        // word for the vertical one; the result (< 2^24) is byte 2 of res
        uint32_t res[K];
#pragma unroll
        for (int m = 0; m < K; ++m) {
          const u16x2 t = __builtin_bit_cast(
              u16x2, __builtin_amdgcn_perm((uint32_t)(v[h][c][0] >> 32), (uint32_t)v[h][c][0],
                                           sel[c][m]));
          const u16x2 u = __builtin_bit_cast(
              u16x2, __builtin_amdgcn_perm((uint32_t)(v[h][c][1] >> 32), (uint32_t)v[h][c][1],
                                           sel[c][m]));
          const uint32_t top = __builtin_amdgcn_udot2(t, wx[c][m], 0u, false);
          const uint32_t bot = __builtin_amdgcn_udot2(u, wx[c][m], 0u, false);
          res[m] = __builtin_amdgcn_udot2(pair16(top, bot), wy[h], 32768u, false);
        }
        uint8_t* dst = pix + j * pitch + 4 + K * (q0 + 64 * c);
        if constexpr (K == 4) {
          *(uint32_t*)dst = __builtin_amdgcn_perm(res[1], res[0], 0x0c0c0602u) |
                            __builtin_amdgcn_perm(res[3], res[2], 0x06020c0cu);
        } else {
          *(uint16_t*)dst = (uint16_t)__builtin_amdgcn_perm(res[1], res[0], 0x0c0c0602u);
        }
      }
    }
  }
}


// One block per segment-test tile of 64*TWW x mark_rows level pixels.  TWW fixes the
// LDS row pitch at compile time, so every circle and compass offset below is a
// ds_read immediate.
template <bool FUSED, int TWW, bool PERSIST>
__global__ __launch_bounds__(256, 5) void k_mark(KArgs a) {
  constexpr int TW = 64 * TWW;
  constexpr int PITCH = TW + 16;  // the staged width (TW + 7) in whole 16-byte chunks
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ int s_next, s_qcnt[4];
  __shared__ uint8_t s_cf[kMarkCellFlags];  // cells of the tile that hold a fast_t corner
  const int band = (int)(blockIdx.x % kXcds);  // used in the band order only
  Head h = read_head(a, band);
  h.persistent = PERSIST;  // one tile per block otherwise: straight-line code, no loop state
  const MarkLds& M = a.ml;  // computed by the host
  uint8_t* pix = smem;
  uint16_t* queue = (uint16_t*)(smem + M.off_queue);
  uint32_t* bml = (uint32_t*)(smem + M.off_bml);
  uint32_t* bmh = (uint32_t*)(smem + M.off_bmh);
  int32_t* s_base = (int32_t*)(smem + M.bytes);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = kBlock >> 6;
  // XCD bands: block b runs on XCD b % kXcds and takes tile b / kXcds of band b % kXcds
  // (the same rows of every level of every frame), so each XCD's L2 holds one band of
  // the frames that its tiles resample from.
  const uint64_t wsig = *(cptr<uint64_t>)h.ws_sig;  // compared before the plan's pointers are used
  if (h.entry < 0 && blockIdx.x == 0) {  // counters of this call (read after this kernel)
    const int ncnt = (int)counter_words(h.n_entries);
    for (int i = threadIdx.x; i < ncnt; i += kBlock) G(h.counters)[i] = 0u;
    if (threadIdx.x == 0) G(h.qctr)[2] = 0u;
  }
  if (h.entry < 0 && !h.small)
    load_bases(s_base, h.bands ? a.band_base + band * (h.n_entries + 1) : a.mark_base,
               h.n_entries);
  queue_start(h, h.qctr + 0, &s_next);

  for (int iter = 0; PERSIST || iter == 0; ++iter) {
    const int g0 = uniform(queue_take(h, iter, &s_next));
    // in the band order a band may hold fewer tiles than the launch gives it blocks
    const int g = launch_tile(g0, h.total, h.bands,
                              h.bands ? (h.small ? h.b[kSmallEntries] : s_base[h.n_entries]) : 0,
                              a.mark_rev);
    if (g < 0) break;
    if (h.persistent) lds_barrier();  // every thread has read s_next
    const int next = queue_prefetch(h, g0, h.qctr + 0);
    int e, t;
    if (h.entry >= 0) {
      e = h.entry;
      t = g;
    } else if (h.small) {
      int st;
      small_entry(h.b, g, &e, &st);
      t = g - st;
    } else {
      e = uniform(prefix_entry(s_base, h.n_entries, g));
      t = g - s_base[e];
    }
    const LevelPlan P = plan_at(h.plan, e);
    if (wsig != h.sig) break;  // not the plan this launch was made for
    const int W = P.W, H = P.H, B = P.B;
    const int tx = t % P.mark_tx;
    const int ty = t / P.mark_tx + (h.bands ? band_row0(P.mark_ty, P.band_rot, band) : 0);
    const MarkTile T = mark_tile(W, H, TW, M.th, tx, ty);
    const int x_t0 = T.x_t0, x_t1 = T.x_t1, y_t0 = T.y_t0, y_t1 = T.y_t1;
    const int ox = T.ox, oy = T.oy, ex = T.ex, ey = T.ey;
    const int nx = ex - ox, ny = ey - oy;

    // 1. level pixels of the tile and its 3-pixel halo
    if (FUSED && P.level > 0) {
      // A column tap keeps x0 + 1 inside the source row (at the right border x0 = w - 2
      // with weight 256: the same value as x0 = x1 = w - 1), so one 16-bit load fetches
      // both horizontal neighbours.  The 7 side columns (the left halo and the last 3)
      // are spread over the lanes by (row, column), so no lane slot holds a column for a
      // few lanes only.
      gptr<const uint8_t> base = G(P.base);
      const int bs = P.base_stride, bw = P.base_w, bh1 = P.base_h - 1;
      constexpr int NC = TWW;  // tile columns per lane
      const double rw = 1.0 / (double)(2 * W), rh = 1.0 / (double)(2 * H);
      auto col_tap = [&](int i, uint32_t* x0, u16x2* w) {
        const uint32_t txx = resample_tap_r(ox + min(i, nx - 1), bw, W, rw);
        int xx = (int)(txx >> 9), wx = (int)(txx & 511);
        if (xx >= bw - 1) {
          xx = bw - 2;
          wx = 256;
        }
        *x0 = (uint32_t)xx;
        *w = pair16((uint32_t)(256 - wx), (uint32_t)wx);  // (256 - wx, wx)
      };
      // Adjacent output columns whose taps share 8 bytes of a frame row: 4 below scale 2,
      // 2 below scale 6 (one 64-bit load per source row for all of them), else one
      // 16-bit gather per column and source row.
      const int kgrp = 3 * bw < 6 * W ? 4 : (bw < 6 * W ? 2 : 1);
      if (kgrp > 1) {
        // The tile's taps, once per block, in the queue's region (free until step 2):
        // per column x0 and (256 - wx, wx), per row the offsets of source rows y0 and
        // min(y0 + 1, h - 1) and (256 - wy, wy).
        uint32_t* tcx = (uint32_t*)(smem + M.off_queue);
        uint32_t* tcw = tcx + M.tcols;
        uint32_t* tro = tcw + M.tcols;
        uint32_t* trw = tro + 2 * M.rows;
        for (int i = threadIdx.x; i < nx + ny; i += kBlock) {
          if (i < nx) {
            uint32_t x0;
            u16x2 w;
            col_tap(i, &x0, &w);
            tcx[i] = x0;
            tcw[i] = __builtin_bit_cast(uint32_t, w);
          } else {
            const int j = i - nx;
            const uint32_t tyy = resample_tap_r(oy + j, P.base_h, H, rh);
            const int y0 = (int)(tyy >> 9);
            tro[2 * j] = (uint32_t)(y0 * bs);
            tro[2 * j + 1] = (uint32_t)(min(y0 + 1, bh1) * bs);
            trw[j] = (256u - (tyy & 511u)) | ((tyy & 511u) << 16);
          }
        }
        lds_barrier();
        if (kgrp == 4) {
          constexpr int G4 = TW / 4, R4 = G4 <= 64 ? 64 / G4 : 1;
          resample_groups<4, TW, (R4 >= 4 ? 2 : (R4 == 2 ? 4 : 8))>(
              pix, PITCH, base, bw, nx, ny, tcx, tcw, tro, trw, lane, wave);
        } else {
          constexpr int G2 = TW / 2, R2 = G2 <= 64 ? 64 / G2 : 1, C2 = G2 <= 64 ? 1 : G2 / 64;
          resample_groups<2, TW, (R2 * C2 >= 4 ? 2 : (R2 * C2 == 2 ? 4 : 8))>(
              pix, PITCH, base, bw, nx, ny, tcx, tcw, tro, trw, lane, wave);
        }
        // the left halo and the last 3 columns, by (row, column)
        for (int t0 = 0; t0 < 7 * ny; t0 += kBlock) {
          const int t = t0 + (int)threadIdx.x;
          const int j = t / 7, k = t - j * 7;
          const int col = k < 4 ? k : TW + k;
          if (j < ny && col < nx) {
            const uint32_t x0 = tcx[col];
            const uint32_t v0 = load_pair(base + (tro[2 * j] + x0));
            const uint32_t v1 = load_pair(base + (tro[2 * j + 1] + x0));
            pix[j * PITCH + col] = (uint8_t)blend_q8(v0, v1, __builtin_bit_cast(u16x2, tcw[col]),
                                                     __builtin_bit_cast(u16x2, trw[j]));
          }
        }
      } else {
      // Taps in registers: lane owns the columns 4 + lane + 64c (c < TWW: the tile's
      // width from the left halo's end), and lane j holds the row tap of tile row j
      // (j + 64 in the second value), read per row with readlane.  Each wave takes RPI
      // consecutive rows per round trip.
      const uint32_t ty_a = resample_tap_r(oy + min(lane, ny - 1), P.base_h, H, rh);
      const uint32_t ty_b = ny > 64 ? resample_tap_r(oy + min(lane + 64, ny - 1), P.base_h, H, rh)
                                    : 0u;
      uint32_t cx[NC];
      u16x2 cwx[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) col_tap(4 + lane + 64 * c, &cx[c], &cwx[c]);
      // 2 * RPI * NC loads in flight, plus 2 for the side columns; the most that fit the
      // registers without spilling (a one-tile block keeps fewer values live)
      constexpr int RPI = TWW == 1 ? 6 : (TWW == 2 ? (PERSIST ? 5 : 7) : (TWW == 3 ? 3 : 2));
      static_assert(7 * RPI <= 64, "side columns of a round exceed the wave");
      const int hrow = lane / 7, hk = lane - 7 * hrow;
      const int hcol = hk < 4 ? hk : TW + hk;  // side column of this lane
      uint32_t hx;
      u16x2 hwx;
      col_tap(hcol, &hx, &hwx);
      const bool hlane = lane < 7 * RPI && hcol < nx;
      auto tap_pair = [&](int y, uint32_t x) -> uint32_t {
        return load_pair(base + ((uint32_t)(y * bs) + x));
      };
      for (int j0 = RPI * wave; j0 < ny; j0 += RPI * nwave) {
        uint32_t v[RPI][NC][2];
        u16x2 wyr[RPI];  // (256 - wy, wy)
#pragma unroll
        for (int h = 0; h < RPI; ++h) {
          const int j = min(j0 + h, ny - 1);
          const uint32_t tyy =
              (uint32_t)__builtin_amdgcn_readlane((int)(j < 64 ? ty_a : ty_b), j & 63);
          const int y0 = (int)(tyy >> 9);
          wyr[h] = pair16(256u - (tyy & 511u), tyy & 511u);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            v[h][c][0] = tap_pair(y0, cx[c]);
            v[h][c][1] = tap_pair(min(y0 + 1, bh1), cx[c]);
          }
        }
        // side columns: lane takes row j0 + hrow
        const int hj = min(j0 + hrow, ny - 1);
        const int hta = __shfl((int)ty_a, hj & 63, 64), htb = __shfl((int)ty_b, hj & 63, 64);
        const uint32_t hty = (uint32_t)(hj < 64 ? hta : htb);
        uint32_t hv0 = 0, hv1 = 0;
        if (hlane) {
          const int y0 = (int)(hty >> 9);
          hv0 = tap_pair(y0, hx);
          hv1 = tap_pair(min(y0 + 1, bh1), hx);
        }
#pragma unroll
        for (int h = 0; h < RPI; ++h) {
          const int j = j0 + h;
          if (j >= ny) break;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const int i = 4 + lane + 64 * c;
            if (i < nx) pix[j * PITCH + i] = (uint8_t)blend_q8(v[h][c][0], v[h][c][1], cwx[c], wyr[h]);
          }
        }
        if (hlane && j0 + hrow < ny) {
          const int j = j0 + hrow;
          const u16x2 wy = pair16(256u - (hty & 511u), hty & 511u);
          pix[j * PITCH + hcol] = (uint8_t)blend_q8(hv0, hv1, hwx, wy);
        }
      }
      }
    } else {
      const int limit = P.level == 0 ? W : P.lvl_stride;
      stage_all<8, true>(pix, PITCH, G(P.lvl), P.lvl_stride, limit, ox, ex, oy, ey);
    }
    for (int i = threadIdx.x; i < 2 * M.th * 2 * TWW; i += kBlock) bml[i] = 0u;  // lo, hi
    // cells of the tile's pixels: flagged in LDS by the full test, written once at the end
    const int cx_t0 = (int)div_by((uint32_t)x_t0, P.csd), cy_t0 = (int)div_by((uint32_t)y_t0, P.csd);
    const int ncx_t = (int)div_by((uint32_t)(x_t1 - 1), P.csd) - cx_t0 + 1;
    const int ncf = ncx_t * ((int)div_by((uint32_t)(y_t1 - 1), P.csd) - cy_t0 + 1);
    for (int i = threadIdx.x; i < ncf; i += kBlock) s_cf[i] = 0;
    lds_barrier();
    // 2. compass pre-test at fast_t_min: a run of 9 holds two cyclically adjacent
    //    compass points (positions 1/5/9/13), so (n|s) & (e|w) per polarity is
    //    necessary; (n >= hi | s >= hi) & (e >= hi | w >= hi) is
    //    min(max(n, s), max(e, w)) >= hi, and likewise for dark.  Each wave takes rows
    //    and appends the pixels that pass to its own quarter of the queue.
    const int tlo = P.fast_t_min, thi = P.fast_t;
    {
      const int ya = max(y_t0, B), yb = min(y_t1, H - B);
      uint16_t* myq = queue + wave * M.qseg;
      int qn = 0;
      int lxk[TWW];
      bool vk[TWW];
#pragma unroll
      for (int k = 0; k < TWW; ++k) {
        const int x = x_t0 + 64 * k + lane;
        lxk[k] = x - ox;
        vk[k] = x >= B && x < W - B;
      }
      if constexpr (TWW % 2 == 0) {
        // Two horizontally adjacent pixels per lane (columns x, x + 1 with x even) in
        // 16-bit lanes: row words are read aligned and the compass pairs picked with
        // byte permutes; bright holds iff sat(p + t - min(max(n,s), max(e,w))) == 0 and
        // dark iff sat(max(min(n,s), min(e,w)) + t - p) == 0, both pixels at once.
        constexpr int NP = TWW / 2;
        int lxp[NP];
        bool v0[NP], v1[NP];
        uint64_t vm0[NP], vm1[NP];  // the same as lane masks
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int x = x_t0 + 128 * q + 2 * lane;
          lxp[q] = x - ox;  // even; ox is a multiple of 4
          v0[q] = x >= B && x < W - B;
          v1[q] = x + 1 >= B && x + 1 < W - B;
          vm0[q] = __ballot(v0[q]);
          vm1[q] = __ballot(v1[q]);
        }
        const u16x2 t2 = pair16((uint32_t)tlo, (uint32_t)tlo);
        for (int y = ya + wave; y < yb; y += nwave) {
          const int ly = y - oy;
          const uint8_t* r0 = pix + ly * PITCH;
#pragma unroll
          for (int q = 0; q < NP; ++q) {
            const int lx = lxp[q];
            const uint32_t* wr = (const uint32_t*)(r0 + (lx & ~3));
            const uint32_t wm = wr[-1], w0 = wr[0], w1 = wr[1];  // bytes lx-4.. lx+7 (aligned)
            const uint32_t vn = *(const uint16_t*)(r0 - 3 * PITCH + lx);
            const uint32_t vs = *(const uint16_t*)(r0 + 3 * PITCH + lx);
            const bool odd = (lx & 2) != 0;  // lx % 4 == 2
            const u16x2 pp = __builtin_bit_cast(
                u16x2, __builtin_amdgcn_perm(0u, w0, odd ? 0x0c030c02u : 0x0c010c00u));
            const u16x2 pw = __builtin_bit_cast(
                u16x2, __builtin_amdgcn_perm(w0, wm, odd ? 0x0c040c03u : 0x0c020c01u));
            const u16x2 pe = __builtin_bit_cast(
                u16x2, __builtin_amdgcn_perm(w1, w0, odd ? 0x0c060c05u : 0x0c040c03u));
            const u16x2 pn = bytes16(vn), ps = bytes16(vs);
            const u16x2 hb = __builtin_elementwise_min(__builtin_elementwise_max(pn, ps),
                                                       __builtin_elementwise_max(pe, pw));
            const u16x2 hd = __builtin_elementwise_max(__builtin_elementwise_min(pn, ps),
                                                       __builtin_elementwise_min(pe, pw));
            const u16x2 zb = __builtin_elementwise_sub_sat(pp + t2, hb);
            const u16x2 zd = __builtin_elementwise_sub_sat(hd + t2, pp);
            const uint32_t z = __builtin_bit_cast(uint32_t, __builtin_elementwise_min(zb, zd));
            // One append for both pixels: a lane's entries follow those of the lanes below
            // it (pixel order in the queue does not matter).  The lane masks come from
            // the compares themselves (ICMP_EQ 32, ICMP_ULT 36) and the fixed column masks.
            const uint64_t m0 = __builtin_amdgcn_uicmp(z & 0xffffu, 0u, 32) & vm0[q];
            const uint64_t m1 = __builtin_amdgcn_uicmp(z, 0x10000u, 36) & vm1[q];
            if (m0 | m1) {
              const bool pass0 = v0[q] && (z & 0xffffu) == 0u;
              const bool pass1 = v1[q] && z < 0x10000u;
              const int slot = qn + (int)(lanes_below(m0) + lanes_below(m1));
              const uint32_t e = (uint32_t)(lx | (ly << 9));
              if (pass0) myq[slot] = (uint16_t)e;
              if (pass1) myq[slot + (pass0 ? 1 : 0)] = (uint16_t)(e + 1u);
              qn += __popcll(m0) + __popcll(m1);
            }
          }
        }
      } else {
        for (int y = ya + wave; y < yb; y += nwave) {
          const int ly = y - oy;
          const uint8_t* rowp = pix + (ly - 3) * PITCH;  // compass north row
#pragma unroll
          for (int k = 0; k < TWW; ++k) {
            const uint8_t* c = rowp + lxk[k];
            const int vn = c[0], vw = c[3 * PITCH - 3], p = c[3 * PITCH], ve = c[3 * PITCH + 3];
            const int vs = c[6 * PITCH];
            const bool pass = vk[k] && (min(max(vn, vs), max(ve, vw)) >= p + tlo ||
                                        max(min(vn, vs), min(ve, vw)) <= p - tlo);
            const uint64_t m = __ballot(pass);
            if (m) {
              if (pass) myq[qn + lanes_below(m)] = (uint16_t)(lxk[k] | (ly << 9));
              qn += __popcll(m);
            }
          }
        }
      }
      // 2b. the same necessary condition on the diagonal points (positions 2/6/10/14,
      //     (+-2, +-2)): a run of 9 holds two cyclically adjacent ones too.  Each wave
      //     filters its own queue segment in place (a lane writes at or below the entry it
      //     read, and all reads of a step come before its writes), at either polarity: on
      //     textured frames the compass test passes most pixels and this one few of them.
      {
        int kept = 0;
        for (int q0 = 0; q0 < qn; q0 += 64) {
          const int q = q0 + lane;
          const int ent = q < qn ? myq[q] : 0;
          bool keep = false;
          if (q < qn) {
            const uint8_t* c = pix + (ent >> 9) * PITCH + (ent & 511);
            const int p = c[0], ne = c[2 - 2 * PITCH], se = c[2 + 2 * PITCH];
            const int sw = c[2 * PITCH - 2], nw = c[-2 - 2 * PITCH];
            keep = min(max(ne, sw), max(se, nw)) >= p + tlo ||
                   max(min(ne, sw), min(se, nw)) <= p - tlo;
          }
          const uint64_t m = __ballot(keep);
          if (keep) myq[kept + lanes_below(m)] = (uint16_t)ent;
          kept += __popcll(m);
        }
        qn = kept;
      }
      // 2c. the same on the other two sets of four (positions 1/5/9/13 and 3/7/11/15),
      //     both at once and per polarity: a bright run of 9 holds two cyclically
      //     adjacent points of each set at >= p + t, a dark one at <= p - t.  It runs on
      //     what the first two stages left, where it drops about a third, and only in a
      //     wave left with more than two full-test steps' worth (128 entries): with
      //     fewer the block's full test takes about as long without it.
      if (qn > 128) {
        int kept = 0;
        for (int q0 = 0; q0 < qn; q0 += 64) {
          const int q = q0 + lane;
          const int ent = q < qn ? myq[q] : 0;
          bool keep = false;
          if (q < qn) {
            const uint8_t* c = pix + (ent >> 9) * PITCH + (ent & 511);
            const int p = c[0];
            const int a1 = c[1 - 3 * PITCH], a5 = c[3 + PITCH], a9 = c[3 * PITCH - 1];
            const int a13 = c[-3 - PITCH], b3 = c[3 - PITCH], b7 = c[1 + 3 * PITCH];
            const int b11 = c[PITCH - 3], b15 = c[-1 - 3 * PITCH];
            const int hi = p + tlo, lo = p - tlo;
            keep = (imin3(max(a1, a9), max(a5, a13), max(b3, b11)) >= hi &&
                    max(b7, b15) >= hi) ||
                   (imax3(min(a1, a9), min(a5, a13), min(b3, b11)) <= lo &&
                    min(b7, b15) <= lo);
          }
          const uint64_t m = __ballot(keep);
          if (keep) myq[kept + lanes_below(m)] = (uint16_t)ent;
          kept += __popcll(m);
        }
        qn = kept;
      }
      if (lane == 0) s_qcnt[wave] = qn;
    }
    lds_barrier();

    // 3. full segment test of the queued pixels at both thresholds
    int qoff[4];
    int qtot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      qoff[w] = qtot;
      qtot += w < nwave ? s_qcnt[w] : 0;
    }
    for (int q = threadIdx.x; q < qtot; q += kBlock) {
      int w = 0;
#pragma unroll
      for (int k = 1; k < 4; ++k) w += q >= qoff[k] ? 1 : 0;
      const int ent = queue[w * M.qseg + (q - qoff[w])];
      const int lx = ent & 511, ly = ent >> 9;
      const uint8_t* c0 = pix + (ly - 3) * PITCH + (lx - 3);  // top-left of the 7x7 box
      const int p = c0[3 * PITCH + 3];
      int c[16];
      c[0] = c0[3];
      c[1] = c0[4];
      c[2] = c0[PITCH + 5];
      c[3] = c0[2 * PITCH + 6];
      c[4] = c0[3 * PITCH + 6];
      c[5] = c0[4 * PITCH + 6];
      c[6] = c0[5 * PITCH + 5];
      c[7] = c0[6 * PITCH + 4];
      c[8] = c0[6 * PITCH + 3];
      c[9] = c0[6 * PITCH + 2];
      c[10] = c0[5 * PITCH + 1];
      c[11] = c0[4 * PITCH];
      c[12] = c0[3 * PITCH];
      c[13] = c0[2 * PITCH];
      c[14] = c0[PITCH + 1];
      c[15] = c0[2];
      const uint32_t r = segment_test_px(c, p, tlo, thi);
      if (r) {
        const int x = ox + lx, y = oy + ly;
        const int bit = x - x_t0;
        const int word = (y - y_t0) * 2 * TWW + (bit >> 5);
        atomicOr(&bml[word], 1u << (bit & 31));
        if (r & 2u) {
          atomicOr(&bmh[word], 1u << (bit & 31));
          s_cf[((int)div_by((uint32_t)y, P.csd) - cy_t0) * ncx_t +
               ((int)div_by((uint32_t)x, P.csd) - cx_t0)] = 1;
        }
      }
    }
    lds_barrier();

    // 4. bitmap words of the tile rows (zero outside the valid region)
    const int w0 = x_t0 >> 5;
    const int nwd = min(2 * TWW, P.wpr - w0);
    gptr<uint32_t> glo = G(P.bm_lo), ghi = G(P.bm_hi);
    {
      const int k = threadIdx.x & 7;  // at most 8 words per tile row
      for (int r = threadIdx.x >> 3; r < y_t1 - y_t0; r += kBlock >> 3) {
        if (k < nwd) {
          const uint32_t gi = row_off(y_t0 + r, P.wpr) + w0 + k;
          glo[gi] = bml[r * 2 * TWW + k];
          ghi[gi] = bmh[r * 2 * TWW + k];
        }
      }
    }
    // 5. the tile's flagged cells and (fused) its level pixels.  Global stores come last:
    //    a store's registers are reused only after it completes, so a store issued
    //    before a later step would hold that step up.
    {
      gptr<uint8_t> flags = G(P.flags);
      for (int i = threadIdx.x; i < ncf; i += kBlock)
        if (s_cf[i]) {
          const int r = (int)((uint32_t)i / (uint32_t)ncx_t);
          flags[(cy_t0 + r) * P.ncx + cx_t0 + (i - r * ncx_t)] = 1;
        }
    }
    if (FUSED && P.level > 0) {
      // The tile's own pixels to the level buffer, 16 bytes per store (level rows are
      // 64-byte aligned and tiles start at multiples of 64; a ragged right end goes
      // byte by byte).
      const int ow = x_t1 - x_t0, nfull = ow >> 4;
      gptr<uint8_t> lv = G(P.lvl_w) + (row_off(y_t0, P.lvl_stride) + x_t0);
      const uint8_t* own = pix + (y_t0 - oy) * PITCH + (x_t0 - ox);  // 4-byte aligned
      for (int q = threadIdx.x; q < (y_t1 - y_t0) * (TW / 16); q += kBlock) {
        const int r = q / (TW / 16), k = q - r * (TW / 16);
        const uint8_t* src = own + r * PITCH + 16 * k;
        gptr<uint8_t> dst = lv + (row_off(r, P.lvl_stride) + 16 * k);
        if (k < nfull) {
          const uint32_t* s4 = (const uint32_t*)src;
          *(gptr<u32x4>)dst = u32x4{s4[0], s4[1], s4[2], s4[3]};
        } else {
          for (int b = 0; b < ow - 16 * k; ++b) dst[b] = src[b];
        }
      }
    }
    queue_park(h, next, &s_next);
  }
}

// ------------------------------------------------------- Harris / NMS / cells --

// Bits [a, b) of a 32-bit word, 0 <= a <= b <= 32.
__device__ __forceinline__ uint32_t bit_range(int a, int b) {
  const uint32_t hi = b >= 32 ? 0xffffffffu : ((1u << b) - 1u);
  return a >= 32 ? 0u : hi & ~((1u << a) - 1u);
}

// One block per Harris/NMS tile (whole cells, or det_w x det_h pixels when the level is
// one cell).  Candidates of the tile and a 1-pixel ring are found word-parallel from
// the segment-test bitmaps, scored with Harris from LDS, suppressed against their
// candidate neighbours, and the per-cell best are written to the cells' fixed slots.
// LA > 0 compiles the tile shape in (LA x LB cells of side LCELL, or LA x LB pixels when
// LCELL == 0): its LDS layout and tile geometry are then constants rather than values held
// in scalar registers (which spilled); LA == 0 takes the shape from the arguments.
template <bool PERSIST, int LA, int LB, int LCELL>
__global__ __launch_bounds__(256, 4) void k_detect(KArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ int s_next, s_ns, s_ne, s_nin;
  __shared__ uint32_t s_wsum[16];
  const int band = (int)(blockIdx.x % kXcds);  // used in the band order only
  Head h = read_head(a, band);
  h.persistent = PERSIST;  // one tile per block otherwise: straight-line code, no loop state
  constexpr Tune kT = det_shape_tune(LA, LB, LCELL);
  constexpr DetLds kD = det_lds(kT, LCELL);
  const DetLds& D = LA > 0 ? kD : a.dl;  // else computed by the host
  const Tune& TT = LA > 0 ? kT : h.t;     // the tile shape's fields
  const int cellm = LA > 0 ? LCELL : h.cell;
  uint8_t* pix = smem;
  uint32_t* cw = (uint32_t*)(smem + D.off_cw);
  uint32_t* ucnt = (uint32_t*)(smem + D.off_ucnt);
  uint32_t* cpre = (uint32_t*)(smem + D.off_cpre);
  int64_t* crs = (int64_t*)(smem + D.off_crs);
  uint32_t* cpos = (uint32_t*)(smem + D.off_cpos);
  uint16_t* sci = (uint16_t*)(smem + D.off_sci);
  uint16_t* scell = (uint16_t*)(smem + D.off_scell);  // cell of each survivor (multi only)
  const bool multi = D.max_cells > 1;
  uint16_t* order = (uint16_t*)(smem + D.off_order);  // cells: grouped survivors; else block flags
  uint32_t* ccnt = (uint32_t*)(smem + D.off_ccnt);
  uint32_t* coff = (uint32_t*)(smem + D.off_coff);
  uint32_t* cfill = (uint32_t*)(smem + D.off_cfill);
  uint32_t* ckept = (uint32_t*)(smem + D.off_ckept);
  int64_t* cbest = (int64_t*)(smem + D.off_cbest);
  uint32_t* cwin = (uint32_t*)(smem + D.off_cwin);
  uint8_t* lfl = smem + D.off_lfl;
  uint32_t* fmt = (uint32_t*)(smem + D.off_fm);  // candidate-word masks per flag row and word
  int32_t* s_base = (int32_t*)(smem + D.bytes);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = kBlock >> 6;
  const int bd = (int)kBlock, tid = (int)threadIdx.x;
  const uint64_t wsig = *(cptr<uint64_t>)h.ws_sig;  // compared before the plan's pointers are used
  if (h.entry < 0 && !h.small)
    load_bases(s_base, h.bands ? a.det_band_base + band * (h.n_entries + 1) : a.det_base,
               h.n_entries);
  queue_start(h, h.qctr + 2, &s_next);

  for (int iter = 0; PERSIST || iter == 0; ++iter) {
    const int g0 = uniform(queue_take(h, iter, &s_next));
    const int g = launch_tile(g0, h.total, h.bands,
                              h.bands ? (h.small ? h.b[kSmallEntries] : s_base[h.n_entries]) : 0,
                              a.det_rev);
    if (g < 0) break;
    if (h.persistent) lds_barrier();  // every thread has read s_next
    const int next = queue_prefetch(h, g0, h.qctr + 2);
    int e, t;
    if (h.entry >= 0) {
      e = h.entry;
      t = g;
    } else if (h.small) {
      int st;
      small_entry(h.b, g, &e, &st);
      t = g - st;
    } else {
      e = uniform(prefix_entry(s_base, h.n_entries, g));
      t = g - s_base[e];
    }
    const LevelPlan P = plan_at(h.plan, e);
    if (wsig != h.sig) break;  // not the plan this launch was made for
    const int W = P.W, H = P.H, B = P.B, cs = P.cs;
    const int tx = t % P.det_tx;
    const int ty = t / P.det_tx + (h.bands ? band_row0(P.det_ty, P.det_band_rot, band) : 0);
    const DetTile T = det_tile(P, TT, cellm, tx, ty);
    const int vx0 = T.vx0, vx1 = T.vx1, vy0 = T.vy0, vy1 = T.vy1;
    const int cxa = T.cxa, cya = T.cya, nlcx = T.nlcx, nlcy = T.nlcy;
    const int rx0 = T.rx0, ry0 = T.ry0, rw = T.rw;
    const int sx0 = T.sx0, sy0 = T.sy0, sx1 = T.sx1, sy1 = T.sy1;
    const int bw0 = T.bw0, nbw = T.nbw, nunits = T.nunits;
    const int fcx0 = T.fcx0, fcy0 = T.fcy0, nfx = T.nfx, nfy = T.nfy;
    const int ncell = nlcx * nlcy;
    const int nvx = P.det_xend - P.det_x0;
    const int nbx = (vx1 - vx0 + 1) >> 1, nby = (vy1 - vy0 + 1) >> 1;  // 2x2 blocks
    // divisions by the words per ring row and the ring's flag columns (i * d < 2^16 for
    // every index here: at most 2 * 256 + (mth + 2) * nbw words and flags, nbw <= 10)
    const uint32_t rnbw = recip16(nbw), rnfx = recip16(nfx);

    // 1. loads: the thread's bitmap words (kept in registers) and the cell flags first,
    //    then the tile's pixels, which stay in flight through the candidate words
    gptr<const uint32_t> glo = G((const uint32_t*)P.bm_lo), ghi = G((const uint32_t*)P.bm_hi);
    uint32_t vlo[2], vhi[2];
    int vr[2], vk[2];
    const int limit = P.level == 0 ? W : P.lvl_stride;
    Stage<12, true> st;
    {
      gptr<const uint8_t> gfl = G((const uint8_t*)P.flags);
      const int nfl = nfx * nfy;
      uint32_t vfl[2];
      // no branches: an index past its region loads the region's last element, dropped
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = u * bd + tid;
        vr[u] = div16(i, rnbw);
        vk[u] = i - vr[u] * nbw;
        const int iu = min(i, nunits - 1), ru = div16(iu, rnbw);
        const uint32_t gi = row_off(ry0 + ru, P.wpr) + bw0 + (iu - ru * nbw);
        vlo[u] = glo[gi];
        vhi[u] = ghi[gi];
        const int jf = min(i, nfl - 1), rf = div16(jf, rnfx);
        vfl[u] = gfl[row_off(fcy0 + rf, P.ncx) + fcx0 + (jf - rf * nfx)];
      }
      stage_begin(st, sx0, sx1, sy0, sy1, limit, D.pitch);
      stage_issue(st, G(P.lvl), P.lvl_stride, limit, sx0, sy0);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = u * bd + tid;
        if (i < nfl) lfl[i] = (uint8_t)vfl[u];
        if (i >= nunits) vlo[u] = vhi[u] = 0;
      }
      for (int i = 2 * bd + tid; i < nfl; i += bd) {
        const int r = i / nfx, k = i - r * nfx;
        lfl[i] = gfl[(fcy0 + r) * P.ncx + fcx0 + k];
      }
    }
    if (tid == 0) {
      s_ns = 0;
      s_ne = 0;
      s_nin = 0;
    }
    // one survivor kept per cell: the cell's winner is found with LDS atomics
    const bool best1 = cellm > 0 && P.kcell == 1;
    if (cellm > 0) {
      for (int c = tid; c < ncell; c += bd) {
        ccnt[c] = 0;
        cfill[c] = 0;
        ckept[c] = 0;
        cbest[c] = INT64_MIN;
        cwin[c] = kNoPos;
      }
    } else {
      for (int i = tid; i < nbx * nby; i += bd) order[i] = 0;
    }
    lds_barrier();

    // 2. candidate words, 32 pixels per thread and step, and their counts.  A pixel is a
    //    candidate at the threshold of its own cell: fast_t where the cell holds a fast_t
    //    corner, else fast_t_min.  Per flag row and word column of the tile, the table
    //    holds the word's columns inside [xa, xb) (hi bitmap) and those of them in cells
    //    without a fast_t corner (lo bitmap); a 32-pixel span meets at most 5 cells.
    const int xa = max(rx0, B), xb = min(rx0 + rw, W - B);
    for (int i = tid; i < nfy * nbw; i += bd) {
      const int fr = div16(i, rnbw), k = i - fr * nbw;
      const int x0 = (bw0 + k) << 5;
      const int a0 = max(x0, xa), b0 = min(x0 + 32, xb);
      uint32_t valid = 0, fm = 0;
      if (a0 < b0) {
        valid = bit_range(a0 - x0, b0 - x0);
        const int c0 = (int)div_by((uint32_t)a0, P.csd);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const int c = c0 + q, ca = max(c * cs, a0), cb = min(c * cs + cs, b0);
          if (ca < cb && lfl[fr * nfx + c - fcx0]) fm |= bit_range(ca - x0, cb - x0);
        }
      }
      fmt[2 * i] = valid;
      fmt[2 * i + 1] = valid & ~fm;
    }
    lds_barrier();
    auto cand_word = [&](uint32_t lo, uint32_t hi, int y, int k) -> uint32_t {
      if (y < B || y >= H - B) return 0u;
      const uint32_t* m = fmt + 2 * (((int)div_by((uint32_t)y, P.csd) - fcy0) * nbw + k);
      return (hi & m[0]) | (lo & m[1]);
    };
    uint32_t cwr[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = u * bd + tid;
      cwr[u] = 0;
      if (i < nunits) {
        cwr[u] = cand_word(vlo[u], vhi[u], ry0 + vr[u], vk[u]);
        cw[i] = cwr[u];
        ucnt[i] = (uint32_t)__popc(cwr[u]);
      }
    }
    for (int i = 2 * bd + tid; i < nunits; i += bd) {
      const int r = div16(i, rnbw), k = i - r * nbw;
      const uint32_t gi = row_off(ry0 + r, P.wpr) + bw0 + k;
      const uint32_t c = cand_word(glo[gi], ghi[gi], ry0 + r, k);
      cw[i] = c;
      ucnt[i] = (uint32_t)__popc(c);
    }
    // prefix counts of the candidate words (raster order)
    uint32_t pre[2];
    int ncand;
    if (nunits <= 2 * bd) {
      // words tid and tid + bd are in registers: one wave scan per half, one barrier
      const uint32_t inc0 = wave_incl_scan((uint32_t)__popc(cwr[0]));
      const uint32_t inc1 = wave_incl_scan((uint32_t)__popc(cwr[1]));
      if (lane == 63) {
        s_wsum[wave] = inc0;
        s_wsum[8 + wave] = inc1;
      }
      lds_barrier();
      uint32_t off0 = 0, off1 = 0, tot0 = 0, tot1 = 0;
      for (int w = 0; w < nwave; ++w) {
        const uint32_t a0 = s_wsum[w], a1 = s_wsum[8 + w];
        off0 += w < wave ? a0 : 0u;
        off1 += w < wave ? a1 : 0u;
        tot0 += a0;
        tot1 += a1;
      }
      pre[0] = off0 + inc0 - (uint32_t)__popc(cwr[0]);
      pre[1] = tot0 + off1 + inc1 - (uint32_t)__popc(cwr[1]);
      if (tid < nunits) cpre[tid] = pre[0];
      if (bd + tid < nunits) cpre[bd + tid] = pre[1];
      if (tid == 0) cpre[nunits] = tot0 + tot1;
      ncand = (int)(tot0 + tot1);
    } else {
      lds_barrier();
      block_scan_u32(ucnt, cpre, nunits, s_wsum);
      ncand = (int)cpre[nunits];
      pre[0] = tid < nunits ? cpre[tid] : 0u;
      pre[1] = bd + tid < nunits ? cpre[bd + tid] : 0u;
    }

    // 3. cached candidate positions (raster order) and their Harris scores
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = u * bd + tid;
      uint32_t m = cwr[u];
      if (i < nunits && m) {
        uint32_t idx = pre[u];
        const uint32_t yx = ((uint32_t)(ry0 + vr[u]) << 16) | (uint32_t)((bw0 + vk[u]) << 5);
        for (; m && idx < (uint32_t)kCandCache; m &= m - 1u) cpos[idx++] = yx + __builtin_ctz(m);
      }
    }
    for (int i = 2 * bd + tid; i < nunits; i += bd) {
      uint32_t m = cw[i];
      uint32_t idx = cpre[i];
      const int r = div16(i, rnbw), k = i - r * nbw;
      const uint32_t yx = ((uint32_t)(ry0 + r) << 16) | (uint32_t)((bw0 + k) << 5);
      for (; m && idx < (uint32_t)kCandCache; m &= m - 1u) cpos[idx++] = yx + __builtin_ctz(m);
    }
    stage_store(st, pix, D.pitch);
    stage_rest(st, pix, D.pitch, G(P.lvl), P.lvl_stride, limit, sx0, sy0);
    lds_barrier();
    const int ncache = min(ncand, kCandCache);
    harris_cache(pix, D.pitch, cpos, crs, ncache, sx0, sy0,
                 ncache <= kBlock / 8 ? 3 : (ncache <= kBlock / 4 ? 2 : (ncache <= kBlock / 2 ? 1 : 0)));
    lds_barrier();

    // Position and R' of candidate ci (raster order); beyond the cache the position is
    // found from the word prefix counts and R' is recomputed from the staged pixels.
    auto cand_pos = [&](int ci) -> uint32_t {
      if (ci < kCandCache) return cpos[ci];
      int lo = 0, hi = nunits - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cpre[mid] <= (uint32_t)ci) lo = mid; else hi = mid - 1;
      }
      uint32_t m = cw[lo];
      for (uint32_t k = cpre[lo]; k < (uint32_t)ci; ++k) m &= m - 1u;
      const int r = lo / nbw, k = lo - r * nbw;
      return ((uint32_t)(ry0 + r) << 16) | (uint32_t)(((bw0 + k) << 5) + __builtin_ctz(m));
    };
    auto cand_score = [&](int ci, uint32_t pos) -> int64_t {
      if (ci < kCandCache) return crs[ci];
      return harris_point(pix, D.pitch, (int)(pos & 0xffff) - sx0, (int)(pos >> 16) - sy0);
    };

    // 4. NMS: a tile candidate survives when it ranks above every candidate neighbour.
    for (int ci0 = 0; ci0 < ncand; ci0 += bd) {
      const int ci = ci0 + tid;
      uint32_t pos = 0;
      bool inside = false;
      if (ci < ncand) {
        pos = cand_pos(ci);
        const int x = (int)(pos & 0xffff), y = (int)(pos >> 16);
        inside = x >= vx0 && x < vx1 && y >= vy0 && y < vy1;  // not the ring
      }
      const uint64_t im = __ballot(inside);
      if (lane == 0 && im) atomicAdd(&s_nin, (int)__popcll(im));
      if (!inside) continue;
      const int x = (int)(pos & 0xffff), y = (int)(pos >> 16);
      // The 8 neighbours' lookups in three rounds of independent LDS reads (candidate
      // words and their prefix counts, then scores), with no branch between them, so
      // that their latencies overlap; a neighbour past the score cache (rare) is
      // recomputed afterwards.
      const int64_t R0 = crs[min(ci, kCandCache - 1)];
      uint32_t qm[8], qp[8];
      int qb[8];
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        const int dx = nb < 3 ? nb - 1 : (nb < 5 ? (nb == 3 ? -1 : 1) : nb - 6);
        const int dy = nb < 3 ? -1 : (nb < 5 ? 0 : 1);
        const int qx = x + dx, qy = y + dy;
        const int qu = (qy - ry0) * nbw + (qx >> 5) - bw0;
        qb[nb] = qx & 31;
        qm[nb] = cw[qu];
        qp[nb] = cpre[qu];
      }
      int qi[8];
      int64_t qs[8];
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        qi[nb] = (int)(qp[nb] + (uint32_t)__popc(qm[nb] & ((1u << qb[nb]) - 1u)));
        qs[nb] = crs[min(qi[nb], kCandCache - 1)];
      }
      const int64_t R = ci < kCandCache ? R0 : cand_score(ci, pos);
      bool alive = true, far = false;
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        const int dx = nb < 3 ? nb - 1 : (nb < 5 ? (nb == 3 ? -1 : 1) : nb - 6);
        const int dy = nb < 3 ? -1 : (nb < 5 ? 0 : 1);
        const uint32_t qpos = ((uint32_t)(y + dy) << 16) | (uint32_t)(x + dx);
        const bool isc = (qm[nb] >> qb[nb]) & 1u;
        far = far || (isc && qi[nb] >= kCandCache);
        alive = alive && !(isc && qi[nb] < kCandCache && !better(R, pos, qs[nb], qpos));
      }
      if (far) {  // neighbours past the score cache: recomputed from the staged pixels
#pragma unroll 1
        for (int nb = 0; nb < 8; ++nb) {
          const int dx = nb < 3 ? nb - 1 : (nb < 5 ? (nb == 3 ? -1 : 1) : nb - 6);
          const int dy = nb < 3 ? -1 : (nb < 5 ? 0 : 1);
          const uint32_t qpos = ((uint32_t)(y + dy) << 16) | (uint32_t)(x + dx);
          if (((qm[nb] >> qb[nb]) & 1u) && qi[nb] >= kCandCache)
            alive = alive && better(R, pos, cand_score(qi[nb], qpos), qpos);
        }
      }
      if (alive) {
        const int si = atomicAdd(&s_ns, 1);
        const int c = multi ? ((int)div_by((uint32_t)y, P.csd) - cya) * nlcx +
                                  ((int)div_by((uint32_t)x, P.csd) - cxa)
                            : 0;
        sci[si] = (uint16_t)ci;
        if (multi) scell[si] = (uint16_t)c;
        if (best1) atomicMax((long long*)&cbest[c], (long long)R);
      }
    }
    lds_barrier();
    const int ns = s_ns;
    if (tid == 0 && s_nin > 0) count_add(P.ncand_count, P.count_stride, (uint32_t)s_nin);
    // 5. per-cell top-K (K = quota when the whole level is one cell), written to fixed
    //    slots: K' = min(K, survivors a cell can hold) per cell, or one per 2x2 block
    //    when there are no cells.  Slots left empty get the sentinel.
    const int K = P.kcell;
    gptr<Cand> out = G(P.cand);
    if (best1) {
      // K = 1: among the survivors holding their cell's best R', the smallest (y, x) wins
      for (int s = tid; s < ns; s += bd) {
        const int ci = sci[s];
        const uint32_t pos = cand_pos(ci);
        const int c = multi ? scell[s] : 0;
        if (cand_score(ci, pos) == cbest[c]) atomicMin(&cwin[c], pos);
      }
      lds_barrier();
      for (int c0 = 0; c0 < ncell; c0 += bd) {
        const int c = c0 + tid;
        bool filled = false;
        if (c < ncell) {
          const int lcy = c / nlcx, lcx = c - lcy * nlcx;
          const int slot = (cya + lcy - P.det_y0) * nvx + (cxa + lcx - P.det_x0);
          filled = cwin[c] != kNoPos;
          store_cand(out + slot, filled ? cbest[c] : INT64_MIN, cwin[c]);
        }
        const uint64_t m = __ballot(filled);
        if (lane == 0 && m) count_add(P.cand_count, P.count_stride, (uint32_t)__popcll(m));
      }
      queue_park(h, next, &s_next);
      continue;
    }
    if (ns > 0) {
      if (cellm > 0) {
        for (int s2 = tid; s2 < ns; s2 += bd) atomicAdd(&ccnt[multi ? scell[s2] : 0], 1u);
        lds_barrier();
        if (tid == 0) {
          uint32_t o = 0;
          for (int c = 0; c < ncell; ++c) {
            coff[c] = o;
            o += ccnt[c];
          }
        }
        lds_barrier();
        for (int s2 = tid; s2 < ns; s2 += bd) {
          const int c = multi ? scell[s2] : 0;
          order[coff[c] + atomicAdd(&cfill[c], 1u)] = (uint16_t)s2;
        }
        lds_barrier();
      }
      for (int s = tid; s < ns; s += bd) {
        const int ci = sci[s];
        const uint32_t pos = cand_pos(ci);
        const int64_t R = cand_score(ci, pos);
        const int c = multi ? scell[s] : 0;
        const int n = cellm > 0 ? (int)ccnt[c] : ns;
        bool keep = true;
        if (n > K) {
          int rank = 0;
          const int o = cellm > 0 ? (int)coff[c] : 0;
          for (int q = 0; q < n && rank < K; ++q) {
            const int s2 = cellm > 0 ? order[o + q] : q;
            const int ci2 = sci[s2];
            const uint32_t pos2 = cand_pos(ci2);
            rank += better(cand_score(ci2, pos2), pos2, R, pos) ? 1 : 0;
          }
          keep = rank < K;
        }
        if (keep) {
          const int x = (int)(pos & 0xffff), y = (int)(pos >> 16);
          int slot;
          if (cellm > 0) {
            const int r = (int)atomicAdd(&ckept[c], 1u);
            slot = (((int)div_by((uint32_t)y, P.csd) - P.det_y0) * nvx +
                    ((int)div_by((uint32_t)x, P.csd) - P.det_x0)) * P.kslot + r;
          } else if (P.compact) {  // listed here, appended below
            order[atomicAdd(&s_ne, 1)] = (uint16_t)s;
            continue;
          } else {
            slot = ((y - B) >> 1) * P.slot_w + ((x - B) >> 1);
            order[((y - vy0) >> 1) * nbx + ((x - vx0) >> 1)] = 1;
          }
          store_cand(out + slot, R, pos);
          atomicAdd(&s_ne, 1);
        }
      }
    }
    lds_barrier();
    if (P.compact) {
      // Levels with more candidate slots than the rank path takes: the kept survivors
      // are appended after the level's filled count (one reserving atomic per tile, on
      // sub-counter 0, which alone counts such a level), so the radix select reads
      // filled entries only.
      if (tid == 0) s_ns = s_ne > 0 ? (int)atomicAdd(P.cand_count, (uint32_t)s_ne) : 0;
      lds_barrier();
      const int base = s_ns, ne = s_ne;
      for (int k = tid; k < ne; k += bd) {
        const int ci = sci[order[k]];
        const uint32_t pos = cand_pos(ci);
        if (base + k < P.cand_cap) store_cand(out + base + k, cand_score(ci, pos), pos);
      }
      queue_park(h, next, &s_next);
      continue;
    }
    if (cellm > 0) {
      const int ks = P.kslot;
      for (int i = tid; i < ncell * ks; i += bd) {
        const int c = ks == 1 ? i : i / ks;
        const int r = i - c * ks;
        if (r >= (int)ckept[c]) {
          const int lcy = c / nlcx, lcx = c - lcy * nlcx;
          const int slot = ((cya + lcy - P.det_y0) * nvx + (cxa + lcx - P.det_x0)) * ks + r;
          store_cand(out + slot, INT64_MIN, kNoPos);
        }
      }
    } else {
      const int srow = (vy0 - B) >> 1, scol = (vx0 - B) >> 1;
      for (int by = wave; by < nby; by += nwave)
        for (int bx = lane; bx < nbx; bx += 64)
          if (!order[by * nbx + bx])
            store_cand(out + (row_off(srow + by, P.slot_w) + scol + bx), INT64_MIN, kNoPos);
    }
    if (tid == 0 && s_ne > 0) count_add(P.cand_count, P.count_stride, (uint32_t)s_ne);
    queue_park(h, next, &s_next);
  }
}

// ------------------------------------------- level selection + orientation --

// Sum over levels 0 .. upto-1 of the frame of min(filled slots, quota): the first output
// index of level `upto` (upto = n_levels: the frame's keypoint count).  counts0 is level
// 0's sub-counter 0.  Every lane of the wave takes part (16 lanes per level, one
// sub-counter each); the result is the same in every lane.
__device__ __forceinline__ int level_prefix(const LevelPlan* plan, int entry0,
                                            gptr<const uint32_t> counts0, int stride, int upto) {
  const int lane = (int)(threadIdx.x & 63);
  int acc = 0;
  for (int l0 = 0; l0 < upto; l0 += 64 / kCountSpread) {
    const int l = l0 + lane / kCountSpread, k = lane % kCountSpread;
    uint32_t v = l < upto ? counts0[l + k * stride] : 0u;
#pragma unroll
    for (int o = 1; o < kCountSpread; o <<= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    if (k == 0 && l < upto) acc += min((int)v, plan_quota(plan, entry0 + l));
  }
  return wave_sum(acc);
}

// One wave per candidate slot.  A candidate's rank is the number of candidates of its
// level that rank above it; ranks of the N_l best are exactly their sorted positions, so
// the wave that holds rank < N_l computes the orientation and writes its keypoint at
// out[level prefix + rank].  Levels whose candidate count exceeds the call's rank cap
// are left to the radix select, which lists their best N_l for a second launch of this
// kernel (from_sel) to rank the same way.
__global__ __launch_bounds__(256) void k_select_orient(KArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];  // the level's R' when staged
  __shared__ int32_t s_base[kMaxEntries + 1];
  const Head h = read_head(a, 0);
  const uint64_t wsig = *(cptr<uint64_t>)h.ws_sig;  // compared before the plan's pointers are used
  if (blockIdx.x == 0 && wsig != h.sig) {  // not the plan this launch was made for
    if ((int)threadIdx.x < a.n_frames) G(a.frame_counts)[threadIdx.x] = -1;
    return;
  }
  if (h.flags) {  // cell flags and the segment-test queue counter, zero for the next call
    const int nq = (int)(a.flag_bytes / 16);
    const u32x4 zero = {0u, 0u, 0u, 0u};
    for (int q = (int)(blockIdx.x * kBlock + threadIdx.x); q < nq; q += (int)(gridDim.x * kBlock))
      ((gptr<u32x4>)G(h.flags))[q] = zero;
    if (blockIdx.x == 0 && threadIdx.x == 0) G(h.qctr)[0] = 0u;
  }
  if (!h.small) load_bases(s_base, a.rank_base, h.n_entries);
  const int lane = threadIdx.x & 63, wave = uniform((int)(threadIdx.x >> 6));
  const int slot0 = (int)blockIdx.x * (kBlock >> 6), slot = slot0 + wave;
  const int nslots = h.small ? h.b[kSmallEntries] : s_base[h.n_entries];
  if (slot0 >= nslots) return;  // the whole block
  // Entry of the block's first slot and where that entry's slots end; a wave's own slot
  // falls in a later entry only at an entry boundary.
  auto entry_of = [&](int sl, int* e, int* st, int* en) {
    if (h.small) {
      small_entry(h.b, sl, e, st, en);
    } else {
      *e = uniform(prefix_entry(s_base, h.n_entries, sl));
      *st = s_base[*e];
      *en = s_base[*e + 1];
    }
  };
  int e0, st0, en0;
  entry_of(slot0, &e0, &st0, &en0);
  const int ms = min(slot, nslots - 1);
  int e = e0, i = ms - st0;
  if (ms >= en0) {
    int st, en;
    entry_of(ms, &e, &st, &en);
    i = ms - st;
  }
  // the block's four slots in one entry
  const bool one = min(slot0 + (kBlock >> 6) - 1, nslots - 1) < en0;
  const bool live = slot < nslots;
  const LevelPlan P = plan_at(h.plan, e);
  if (wsig != h.sig) return;
  gptr<const uint32_t> counts = G((const uint32_t*)P.cand_count) - e;  // all entries
  // empty slots hold the sentinel; only an appended level's count bounds its list (and
  // a radix-selected list its own count)
  const int C = a.from_sel ? min((int)*G((const uint32_t*)P.sel_count), P.quota)
                : P.compact ? ranked_candidates(P, count_sum(counts + e, P.count_stride))
                            : P.cand_cap;
  if (live && P.level == 0 && i == 0) {
    const int total =
        level_prefix(a.plan, P.entry0, counts + P.entry0, P.count_stride, P.n_levels);
    if (lane == 0) *G(P.count_out) = total;
  }
  if (one && slot0 - st0 >= C) return;  // the block's slots are past the level's list
  gptr<const Cand> cand = G((const Cand*)(a.from_sel ? P.sel : P.cand));
  // A block whose slots all belong to one level that fits the LDS stages the level's
  // R' once (one load per 256 slots per thread, all in flight) and ranks from there.
  const bool staged = a.sel_lds > 0 && one && C <= a.sel_lds;
  Cand me;
  me.score = INT64_MIN;
  me.pos = kNoPos;
  if (live && i < C && (a.from_sel || C <= h.t.rank_cap)) me = load_cand(cand + i);
  int cnt = 0;
  if (staged) {
    int64_t* s_sc = (int64_t*)smem;
    // Padded to a multiple of 256 with the empty slots' INT64_MIN (below every
    // candidate's R'), so that every lane takes the same steps, four reads at a time,
    // with no bounds test and no per-lane loop exit (sel_lds is a multiple of 256).
    const int Cp = uniform((C + 255) & ~255);
    for (int k = threadIdx.x; k < Cp; k += kBlock)
      s_sc[k] = k < C ? *(gptr<const int64_t>)(cand + k) : INT64_MIN;
    lds_barrier();
    if (me.pos == kNoPos) return;
    int eq = 0;  // candidates with the same R', the wave's own included
    for (int j0 = 0; j0 < Cp; j0 += 256) {
      int64_t sj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) sj[u] = s_sc[j0 + 64 * u + lane];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        cnt += sj[u] > me.score ? 1 : 0;
        eq += __popcll(__ballot(sj[u] == me.score));
      }
    }
    if (eq > 1) {  // equal R' (rare): ordered by position
      for (int j = lane; j < C; j += 64) {
        const Cand o = load_cand(cand + j);
        cnt += (o.score == me.score && o.pos < me.pos) ? 1 : 0;
      }
    }
  } else {
    if (me.pos == kNoPos) return;
    // Count better candidates, 8 slots in flight per lane (score and position only, few
    // registers: every slot's wave of a call stays resident); a wave whose partial count
    // already reaches the quota cannot be selected and stops.
    for (int j0 = 0; j0 < C; j0 += 8 * 64) {
      int64_t sc[8];
      uint32_t ps[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        gptr<const Cand> q = cand + min(j0 + u * 64 + lane, C - 1);
        sc[u] = *(gptr<const int64_t>)q;
        ps[u] = *((gptr<const uint32_t>)q + 2);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + u * 64 + lane;
        cnt += (j < C && better(sc[u], ps[u], me.score, me.pos)) ? 1 : 0;
      }
      if (j0 + 8 * 64 < C && wave_sum(cnt) >= P.quota) return;
    }
  }
  const int rank = wave_sum(cnt);
  if (rank >= P.quota) return;
  const int prefix = level_prefix(a.plan, P.entry0, counts + P.entry0, P.count_stride, P.level);
  const int x = (int)(me.pos & 0xffff), y = (int)(me.pos >> 16);
  int m10, m01;
  wave_moments(G(P.lvl), P.lvl_stride, x, y, P.B, lane, &m10, &m01);
  if (lane == 0)
    store_keypoint(G(P.out) + prefix + rank, x, y, P.level, m10, m01,
                   atan2f((float)m01, (float)m10), me.score);
}

// ----------------------------------------------- radix-select fallback path --

__device__ __forceinline__ uint64_t score_key(int64_t s) {
  return (uint64_t)s ^ 0x8000000000000000ull;
}

// Adds 1 to bin b of an LDS histogram for every active lane (act): a wave whose active
// lanes share one bin adds its count once (the high digits of nearby scores mostly
// agree, and same-address LDS atomics are performed one lane at a time); otherwise each
// lane adds its own.
__device__ __forceinline__ void hist_add(uint32_t* hist, uint32_t b, bool act) {
  const uint64_t m = __ballot(act);
  if (!m) return;
  const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)b, __builtin_ctzll(m));
  if (__ballot(act && b == b0) == m) {
    if (act && lanes_below(m) == 0) atomicAdd(&hist[b0], (uint32_t)__popcll(m));
  } else if (act) {
    atomicAdd(&hist[b], 1u);
  }
}

// Slot in an LDS list for every active lane: one counter atomic per wave, lanes placed in
// lane order after it.
__device__ __forceinline__ uint32_t list_slot(uint32_t* count, bool act) {
  const uint64_t m = __ballot(act);
  uint32_t base = 0;
  if (m) {
    const int first = __builtin_ctzll(m);
    if ((int)(threadIdx.x & 63) == first) base = atomicAdd(count, (uint32_t)__popcll(m));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, first);
  }
  return base + lanes_below(m);
}

// Digit of a 256-bin histogram at which the running count, taken from the high digits
// down (desc) or from the low digits up, first reaches k (k >= 1, at most the total), and
// the count of the digits before it.  Run by one whole wave: lane l sums four bins, a
// wave scan gives each lane the count before its bins, and the first lane whose bins
// reach k walks them.
__device__ __forceinline__ void hist_find(const uint32_t* hist, uint32_t k, bool desc, int* digit,
                                          uint32_t* before) {
  const int lane = (int)(threadIdx.x & 63);
  uint32_t h[4], sum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    h[j] = hist[desc ? 255 - 4 * lane - j : 4 * lane + j];
    sum += h[j];
  }
  const uint32_t incl = wave_incl_scan(sum);
  const uint64_t m = __ballot(incl >= k);
  const int L = m ? __builtin_ctzll(m) : 63;
  int d = 0;
  uint32_t acc = incl - sum;
  if (lane == L) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      d = desc ? 255 - 4 * lane - j : 4 * lane + j;
      if (acc + h[j] >= k) break;
      acc += h[j];
    }
  }
  *digit = __builtin_amdgcn_readlane(d, L);
  *before = (uint32_t)__builtin_amdgcn_readlane((int)acc, L);
}

// Threshold of the best k of a level's candidates, by radix select: the k-th best score
// key T (8 bits at a time from the top), and, when more candidates than the k needed
// hold T, the largest position pcut among the smallest positions that complete the k
// (8 bits at a time from the top); else pcut = 0xffffffff.  The best k are those with
// key > T, or key == T and position <= pcut.  get(i, &key, &pos) reads candidate i < n
// (false: an empty slot); every thread of the block calls this.
template <class Get>
__device__ void radix_threshold(Get get, int n, uint32_t k, uint32_t* hist, uint64_t* s_key,
                                uint32_t* s_k, uint32_t* s_eq, uint64_t* T, uint32_t* pcut) {
  const int tid = (int)threadIdx.x, bd = (int)blockDim.x;
  if (tid == 0) {
    *s_key = 0;
    *s_k = k;
    *s_eq = 0;
  }
  uint64_t mask = 0;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int i = tid; i < 256; i += bd) hist[i] = 0;
    __syncthreads();
    const uint64_t prefix = *s_key;
    for (int i0 = 0; i0 < n; i0 += bd) {  // whole waves in every step
      uint64_t u = 0;
      uint32_t pos = 0;
      const bool ok = i0 + tid < n && get(i0 + tid, &u, &pos);
      hist_add(hist, (uint32_t)(u >> shift) & 255u, ok && (u & mask) == prefix);
    }
    __syncthreads();
    if (tid < 64) {
      int dg;
      uint32_t before;
      hist_find(hist, *s_k, true, &dg, &before);
      if (tid == 0) {
        *s_k -= before;
        *s_key = prefix | ((uint64_t)dg << shift);
      }
    }
    mask |= 255ull << shift;
    __syncthreads();
  }
  *T = *s_key;
  const uint32_t k_eq = *s_k;  // candidates at T that the k still needs
  for (int i0 = 0; i0 < n; i0 += bd) {
    uint64_t u = 0;
    uint32_t pos = 0;
    const bool ok = i0 + tid < n && get(i0 + tid, &u, &pos);
    hist_add(s_eq, 0u, ok && u == *T);
  }
  __syncthreads();
  *pcut = 0xffffffffu;
  if (*s_eq <= k_eq) return;  // every candidate at T is needed (block-uniform)
  __syncthreads();  // every thread has read s_eq
  if (tid == 0) {
    *s_key = 0;
    *s_k = k_eq;
  }
  uint32_t pmask = 0;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int i = tid; i < 256; i += bd) hist[i] = 0;
    __syncthreads();
    const uint32_t pp = (uint32_t)*s_key;
    for (int i0 = 0; i0 < n; i0 += bd) {
      uint64_t u = 0;
      uint32_t pos = 0;
      const bool ok = i0 + tid < n && get(i0 + tid, &u, &pos);
      hist_add(hist, (pos >> shift) & 255u, ok && u == *T && (pos & pmask) == pp);
    }
    __syncthreads();
    if (tid < 64) {
      int dg;
      uint32_t before;
      hist_find(hist, *s_k, false, &dg, &before);
      if (tid == 0) {
        *s_k -= before;
        *s_key = pp | ((uint32_t)dg << shift);
      }
    }
    pmask |= 255u << shift;
    __syncthreads();
  }
  *pcut = (uint32_t)*s_key;
}

// Levels with more candidates than the call's rank cap (one block per level): the best
// min(filled, N_l) candidates, found by radix select from the level's slots (or from
// its filled slots gathered into LDS when they fit), are written unsorted to the level's
// selection list; k_select_orient then ranks that short list by counting.  A level that
// the first counting launch took gets an empty list.
__global__ __launch_bounds__(1024) void k_select(KArgs a) {
  __shared__ int64_t sc[kSortCap];
  __shared__ uint32_t ps[kSortCap];
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_key;
  __shared__ uint32_t s_k, s_n, s_eq;
  const int e = a.entry >= 0 ? a.entry : (int)blockIdx.x;
  const uint64_t wsig = *(cptr<uint64_t>)a.ws_sig;
  const LevelPlan P = plan_at(a.plan, e);
  if (wsig != a.sig) return;  // not the plan this launch was made for
  const int tid = (int)threadIdx.x, bd = (int)blockDim.x;
  const int N = P.quota;
  const int nfill = (int)count_sum(G((const uint32_t*)P.cand_count), P.count_stride);
  // slots (empty ones hold the sentinel and are skipped), or the appended entries
  const int C = ranked_candidates(P, (uint32_t)nfill);
  const int nout = min(nfill, N);
  if ((a.rank_path && C <= a.t.rank_cap) || nout <= 0) {  // nothing for the list
    if (tid == 0) *G(P.sel_count) = 0;
    return;
  }
  gptr<const Cand> cand = G((const Cand*)P.cand);
  gptr<Cand> sel = G(P.sel);
  if (tid == 0) s_n = 0;
  __syncthreads();
  if (nfill <= kSortCap) {
    // every filled slot fits: gather them all, then keep the best nout
    for (int i0 = 0; i0 < C; i0 += bd) {
      Cand cd;
      cd.pos = kNoPos;
      if (i0 + tid < C) cd = load_cand(cand + i0 + tid);
      const bool keep = cd.pos != kNoPos;
      const uint32_t slot = list_slot(&s_n, keep);
      if (keep && slot < (uint32_t)kSortCap) {
        sc[slot] = cd.score;
        ps[slot] = cd.pos;
      }
    }
    __syncthreads();
    const int n = min((int)s_n, kSortCap);
    uint64_t T = 0;
    uint32_t pcut = 0xffffffffu;
    if (n > nout) {
      auto get = [&](int i, uint64_t* u, uint32_t* pos) {
        *u = score_key(sc[i]);
        *pos = ps[i];
        return true;
      };
      radix_threshold(get, n, (uint32_t)nout, hist, &s_key, &s_k, &s_eq, &T, &pcut);
    }
    __syncthreads();
    if (tid == 0) s_n = 0;
    __syncthreads();
    for (int i0 = 0; i0 < n; i0 += bd) {
      const int i = i0 + tid;
      const uint64_t u = i < n ? score_key(sc[i]) : 0;
      const uint32_t pos = i < n ? ps[i] : 0u;
      const bool keep = i < n && (u > T || (u == T && pos <= pcut));
      const uint32_t slot = list_slot(&s_n, keep);
      if (keep && slot < (uint32_t)nout) store_cand(sel + slot, sc[i], pos);
    }
  } else {
    auto get = [&](int i, uint64_t* u, uint32_t* pos) {
      const Cand cd = load_cand(cand + i);
      *u = score_key(cd.score);
      *pos = cd.pos;
      return cd.pos != kNoPos;
    };
    uint64_t T;
    uint32_t pcut;
    radix_threshold(get, C, (uint32_t)nout, hist, &s_key, &s_k, &s_eq, &T, &pcut);
    __syncthreads();
    if (tid == 0) s_n = 0;
    __syncthreads();
    for (int i0 = 0; i0 < C; i0 += bd) {
      Cand cd;
      cd.pos = kNoPos;
      cd.score = 0;
      if (i0 + tid < C) cd = load_cand(cand + i0 + tid);
      const uint64_t u = score_key(cd.score);
      const bool keep = cd.pos != kNoPos && (u > T || (u == T && cd.pos <= pcut));
      const uint32_t slot = list_slot(&s_n, keep);
      if (keep && slot < (uint32_t)nout) store_cand(sel + slot, cd.score, cd.pos);
    }
  }
  if (tid == 0) *G(P.sel_count) = (uint32_t)nout;
}

// ------------------------------------------------------------ test kernel --

__global__ __launch_bounds__(256) void k_test_segment(const uint8_t* circles, int n, int t_lo,
                                                      int t_hi, uint8_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint8_t* c = circles + (size_t)i * 17;
  int cc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) cc[k] = c[1 + k];
  out[i] = (uint8_t)segment_test_px(cc, c[0], t_lo, t_hi);  // the segment-test tiles' routine
}

// ----------------------------------------------------------------- launches --

// ------------------------------------------------------------------- rBRIEF --

// One wave per keypoint slot.  The angle bin is the largest dot product of (m10, m01)
// with the 30 bin centres (lane k takes centre k; ties to the smaller k); the 31 x 31
// patch around the keypoint is staged in LDS; lane l evaluates tests l, l + 64, l + 128
// and l + 192 of the bin's rotated pattern (5x5 binomial sums compared), and the four
// ballots are the 256-bit descriptor.  Slots beyond the frame's count, or a workspace
// that does not hold the expected plan, are left untouched.
constexpr int kPatchPitch = 36;  // bytes per patch row
constexpr int kSumPitch = 28;    // uint16 per row of the sum tables

// LDS written by some lanes of a wave, read by others of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__global__ __launch_bounds__(256) void k_describe(DescArgs a) {
  __shared__ __align__(16) uint8_t patch[4][31 * kPatchPitch];
  __shared__ __align__(16) uint16_t hsum[4][31 * kSumPitch];  // horizontal 5-tap sums
  __shared__ __align__(16) uint16_t ssum[4][27 * kSumPitch];  // 5 x 5 binomial sums
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  const int slot = (int)blockIdx.x * 4 + wave;
  const int f = slot / a.cap, i = slot - f * a.cap;
  if (f >= a.n || i >= G(a.counts)[f] || *(cptr<uint64_t>)a.ws_sig != a.sig) return;
  const u32x4 k0 = *(gptr<const u32x4>)(G(a.kps) + a.off[f] + i);        // x, y, level, m10
  const int x = (int)k0.x, y = (int)k0.y, level = (int)k0.z, m10 = (int)k0.w;
  const int m01 = *(gptr<const int32_t>)((gptr<const uint8_t>)(G(a.kps) + a.off[f] + i) + 16);
  if (level < 0 || level >= a.L) return;
  const LevelPlan P = plan_at(a.plan, f * a.L + level);
  if (x < 15 || y < 15 || x >= P.W - 15 || y >= P.H - 15) return;
  // angle bin: max over lanes of (dot, -k), packed into one 64-bit key
  uint64_t key = 0;
  if (lane < 30) {
    const int64_t d = (int64_t)m10 * G(a.centres)[2 * lane] +
                      (int64_t)m01 * G(a.centres)[2 * lane + 1];
    key = ((uint64_t)(d + (1ll << 40)) << 5) | (uint64_t)(31 - lane);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t other = __shfl_xor(key, o, 64);
    key = other > key ? other : key;
  }
  const int bin = 31 - (int)(key & 31);
  // The 31 x 31 patch, row pitch 36 bytes (9 words: the rows a lane each reads below
  // start in distinct banks).
  uint8_t* pt = patch[wave];
  gptr<const uint8_t> lvl = G(P.lvl);
  uint8_t v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int idx = lane + 64 * k;
    v[k] = idx < 961 ? lvl[(size_t)(y - 15 + idx / 31) * P.lvl_stride + x - 15 + idx % 31] : 0;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int idx = lane + 64 * k;
    if (idx < 961) pt[(idx / 31) * kPatchPitch + idx % 31] = v[k];
  }
  wave_lds_sync();
  // Every test point lies within 13 pixels of the keypoint, so the 5 x 5 binomial sums
  // (weights 1 4 6 4 1 in each direction, not normalised) are needed at the 27 x 27
  // centres only: formed once per keypoint, separably and exactly in integers.
  // Horizontal pass: lane (row r, half h) sums patch columns c .. c+4 of row r for the
  // 14 (h = 0) or 13 (h = 1) centre columns c of its half.
  uint16_t* hs = hsum[wave];
  {
    const int r = lane & 31, h = lane >> 5;
    if (r < 31) {
      const uint32_t* row = (const uint32_t*)(pt + r * kPatchPitch) + 3 * h;
      uint32_t w[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) w[k] = row[k];  // bytes 12h .. 12h + 19 of the row
      int b[20];
#pragma unroll
      for (int k = 0; k < 20; ++k) b[k] = (int)((w[k >> 2] >> (8 * (k & 3))) & 0xffu);
      // centre column c = 14h + j takes bytes c .. c + 4, i.e. b[2h + j ..]
      uint32_t* out = (uint32_t*)(hs + r * kSumPitch) + 7 * h;
#pragma unroll
      for (int j = 0; j < 14; j += 2) {
        const int o = 2 * h + j;
        const int s0 = b[o] + 4 * b[o + 1] + 6 * b[o + 2] + 4 * b[o + 3] + b[o + 4];
        const int s1 = b[o + 1] + 4 * b[o + 2] + 6 * b[o + 3] + 4 * b[o + 4] + b[o + 5];
        out[j >> 1] = (uint32_t)s0 | ((uint32_t)s1 << 16);
      }
    }
  }
  wave_lds_sync();
  // Vertical pass: lane (column c, half h) sums rows w .. w+4 of the horizontal sums for
  // the 14 (h = 0) or 13 (h = 1) centre rows w of its half.
  uint16_t* ss = ssum[wave];
  if (lane < 54) {
    const int h = lane >= 27 ? 1 : 0, c = lane - 27 * h;
    const uint16_t* col = hs + 14 * h * kSumPitch + c;
    int hv[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) hv[k] = k < 17 + (h ^ 1) ? (int)col[k * kSumPitch] : 0;
#pragma unroll
    for (int j = 0; j < 14; ++j)
      if (j < 14 - h)
        ss[(14 * h + j) * kSumPitch + c] =
            (uint16_t)(hv[j] + 4 * hv[j + 1] + 6 * hv[j + 2] + 4 * hv[j + 3] + hv[j + 4]);
  }
  wave_lds_sync();
  gptr<const uint32_t> tbl = (gptr<const uint32_t>)(G(a.rot) + (size_t)bin * 256 * 4);
  uint64_t words[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t t = tbl[r * 64 + lane];
    // clamped so that no entry reads outside the table
    const int x1 = min(max((int)(int8_t)(t & 0xff), -13), 13);
    const int y1 = min(max((int)(int8_t)((t >> 8) & 0xff), -13), 13);
    const int x2 = min(max((int)(int8_t)((t >> 16) & 0xff), -13), 13);
    const int y2 = min(max((int)(int8_t)(t >> 24), -13), 13);
    words[r] = __ballot(ss[(y1 + 13) * kSumPitch + x1 + 13] < ss[(y2 + 13) * kSumPitch + x2 + 13]);
  }
  if (lane == 0) {
    gptr<uint64_t> d = (gptr<uint64_t>)(G(a.desc) + (size_t)(a.off[f] + i) * 32);
#pragma unroll
    for (int r = 0; r < 4; ++r) d[r] = words[r];
  }
}

// ----------------------------------------------------------------- ablation --
// Kernels of the ablation ladder.  Each computes one step of one pyramid level the way
// an earlier design does, so that the gain of every design decision can be measured on
// the same inputs: FAST with branchy per-circle-pixel logic and global reads, with
// bright/dark bit masks (global, then LDS), and the production scheme (LDS, compass
// pre-test, min/max windows); Harris per candidate with 2D Sobel, separable Sobel, 8
// lanes per candidate, and a dense map from sliding column sums.

// Level of block g and the block's index within it (the level table is in the kernel
// arguments: scalar loads, no memory search).
__device__ __forceinline__ int ab_level(const AbArgs& a, int g, int* local) {
  int e = 0;
#pragma unroll
  for (int i = 1; i < kAbMaxLevels; ++i)
    if (i < a.n_levels && g >= a.lv[i].base) e = i;
  *local = g - a.lv[e].base;
  return e;
}

__constant__ int8_t kCircleX[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
__constant__ int8_t kCircleY[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

// Nine contiguous set bits on the 16-bit circle, with wrap-around: 2, 4, 8, then 9.
__device__ __forceinline__ bool run9_bits(uint32_t m) {
  const uint32_t x = m | (m << 16);
  uint32_t a = x & (x >> 1);
  a &= a >> 2;
  a &= a >> 4;
  a &= x >> 8;
  return (a & 0xffffu) != 0;
}

// Branchy: per circle pixel, classify and count the current bright or dark run while
// walking the circle once and a half (a run of nine that wraps is seen whole).
__global__ __launch_bounds__(256) void k_ab_fast_branchy(AbArgs a) {
  int b;
  const AbLevel& L = a.lv[ab_level(a, (int)blockIdx.x, &b)];
  const uint8_t* img = L.img;
  uint8_t* out = (uint8_t*)L.out;
  const int W = L.W, H = L.H, stride = L.stride, t = a.t, B = a.B;
  const int bx = b % cdiv(W, 64), by = b / cdiv(W, 64);
  const int x = bx * 64 + (int)(threadIdx.x & 63);
  const int y = by * 4 + (int)(threadIdx.x >> 6);
  if (x >= W || y >= H) return;
  uint8_t r = 0;
  if (x >= B && x < W - B && y >= B && y < H - B) {
    gptr<const uint8_t> g = G(img);
    const int p = g[(size_t)y * stride + x];
    int rb = 0, rd = 0;
    for (int k = 0; k < 25; ++k) {
      const int i = k & 15;
      const int v = g[(size_t)(y + kCircleY[i]) * stride + x + kCircleX[i]];
      if (v >= p + t) {
        ++rb;
        rd = 0;
      } else if (v <= p - t) {
        ++rd;
        rb = 0;
      } else {
        rb = rd = 0;
      }
      if (rb >= 9 || rd >= 9) {
        r = 1;
        break;
      }
    }
  }
  G(out)[(size_t)y * W + x] = r;
}

template <bool LDS>
__global__ __launch_bounds__(256) void k_ab_fast_masks(AbArgs a) {
  int b;
  const AbLevel& L = a.lv[ab_level(a, (int)blockIdx.x, &b)];
  const uint8_t* img = L.img;
  uint8_t* out = (uint8_t*)L.out;
  const int W = L.W, H = L.H, stride = L.stride, t = a.t, B = a.B;
  const int bx = b % cdiv(W, 64), by = b / cdiv(W, 64);
  // a block covers 64 x 16 pixels, 4 rows per thread; LDS: the block's pixels and a
  // 3-pixel halo, staged first
  __shared__ uint8_t tile[22][72];
  const int lx = (int)(threadIdx.x & 63), ly0 = (int)(threadIdx.x >> 6) * 4;
  const int x = bx * 64 + lx;
  gptr<const uint8_t> g = G(img);
  if (LDS) {
    const int x0 = bx * 64 - 3, y0 = by * 16 - 3;
    for (int i = (int)threadIdx.x; i < 22 * 70; i += 256) {
      const int r = i / 70, c = i - r * 70;
      const int gx = x0 + c, gy = y0 + r;
      tile[r][c] = (gx >= 0 && gx < W && gy >= 0 && gy < H) ? g[(size_t)gy * stride + gx] : 0;
    }
    lds_barrier();
  }
  for (int k = 0; k < 4; ++k) {
    const int ly = ly0 + k, y = by * 16 + ly;
    if (x >= W || y >= H) continue;
    uint8_t r = 0;
    if (x >= B && x < W - B && y >= B && y < H - B) {
      const int p = LDS ? tile[ly + 3][lx + 3] : g[(size_t)y * stride + x];
      uint32_t mb = 0, md = 0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        constexpr int8_t cx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
        constexpr int8_t cy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};
        const int v = LDS ? tile[ly + 3 + cy[i]][lx + 3 + cx[i]]
                          : g[(size_t)(y + cy[i]) * stride + x + cx[i]];
        mb |= (v >= p + t ? 1u : 0u) << i;
        md |= (v <= p - t ? 1u : 0u) << i;
      }
      r = (run9_bits(mb) || run9_bits(md)) ? 1 : 0;
    }
    G(out)[(size_t)y * W + x] = r;
  }
}

// Production scheme on one level: LDS tile (64 x 16 pixels, 4 rows per thread), exact
// compass pre-test as a wave-wide early-out, min/max windows (the segment-test kernel
// without pyramid, queue and bitmaps).  MASKS: the same tile and pre-test, then bright
// and dark masks and the shift-and run test instead of the min/max windows.
template <bool MASKS>
__global__ __launch_bounds__(256) void k_ab_fast_minmax(AbArgs a) {
  int b;
  const AbLevel& L = a.lv[ab_level(a, (int)blockIdx.x, &b)];
  const uint8_t* img = L.img;
  uint8_t* out = (uint8_t*)L.out;
  const int W = L.W, H = L.H, stride = L.stride, t = a.t, B = a.B;
  const int bx = b % cdiv(W, 64), by = b / cdiv(W, 64);
  __shared__ uint8_t tile[22][72];
  const int lx = (int)(threadIdx.x & 63), ly0 = (int)(threadIdx.x >> 6) * 4;
  const int x = bx * 64 + lx;
  gptr<const uint8_t> g = G(img);
  const int x0 = bx * 64 - 3, y0 = by * 16 - 3;
  for (int i = (int)threadIdx.x; i < 22 * 70; i += 256) {
    const int r = i / 70, c = i - r * 70;
    const int gx = x0 + c, gy = y0 + r;
    tile[r][c] = (gx >= 0 && gx < W && gy >= 0 && gy < H) ? g[(size_t)gy * stride + gx] : 0;
  }
  lds_barrier();
  for (int k = 0; k < 4; ++k) {
    const int ly = ly0 + k, y = by * 16 + ly;
    const bool in = x < W && y < H && x >= B && x < W - B && y >= B && y < H - B;
    bool pass = false;
    int p = 0;
    if (in) {
      const uint8_t* c = &tile[ly + 3][lx + 3];
      p = c[0];
      const int vn = c[-3 * 72], vs = c[3 * 72], ve = c[3], vw = c[-3];
      pass = min(max(vn, vs), max(ve, vw)) >= p + t || max(min(vn, vs), min(ve, vw)) <= p - t;
    }
    uint8_t r = 0;
    if (__ballot(pass) != 0 && pass) {
      int d[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        constexpr int8_t cx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
        constexpr int8_t cy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};
        d[i] = (int)tile[ly + 3 + cy[i]][lx + 3 + cx[i]] - p;
      }
      if (MASKS) {
        uint32_t mb = 0, md = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          mb |= (d[i] >= t ? 1u : 0u) << i;
          md |= (d[i] <= -t ? 1u : 0u) << i;
        }
        r = (run9_bits(mb) || run9_bits(md)) ? 1 : 0;
      } else {
        r = (uint8_t)(segment_test2(d, t, t) & 1u);
      }
    }
    if (x < W && y < H) G(out)[(size_t)y * W + x] = r;
  }
}

// Harris at candidate positions.  variant 0: one thread, 2D Sobel per window pixel;
// 1: one thread, separable Sobel over the 9 x 9 neighbourhood row by row; 2: 8 lanes,
// one window row each, sums added across the group.  Out-of-range positions get 0.
__device__ __forceinline__ bool harris_in(int x, int y, int W, int H) {
  return x >= 4 && y >= 4 && x < W - 4 && y < H - 4;
}

__global__ __launch_bounds__(256) void k_ab_harris_2d(AbArgs a) {
  int b;
  const AbLevel& L = a.lv[ab_level(a, (int)blockIdx.x, &b)];
  const uint8_t* img = L.img;
  int64_t* out = (int64_t*)L.out;
  const uint32_t* pos = L.pos;
  const int W = L.W, H = L.H, stride = L.stride, n = L.n;
  const int i = b * (int)blockDim.x + (int)threadIdx.x;
  if (i >= n) return;
  const uint32_t ps = G(pos)[i];
  const int x = (int)(ps & 0xffff), y = (int)(ps >> 16);
  int64_t R = 0;
  if (harris_in(x, y, W, H)) {
    gptr<const uint8_t> g = G(img);
    int sxx = 0, syy = 0, sxy = 0;
    for (int dy = -3; dy <= 3; ++dy)
      for (int dx = -3; dx <= 3; ++dx) {
        auto I = [&](int u, int v) { return (int)g[(size_t)(y + dy + v) * stride + x + dx + u]; };
        const int gx = (I(1, -1) + 2 * I(1, 0) + I(1, 1)) - (I(-1, -1) + 2 * I(-1, 0) + I(-1, 1));
        const int gy = (I(-1, 1) + 2 * I(0, 1) + I(1, 1)) - (I(-1, -1) + 2 * I(0, -1) + I(1, -1));
        sxx += gx * gx;
        syy += gy * gy;
        sxy += gx * gy;
      }
    const int64_t A = sxx, Bv = syy, C = sxy;
    R = 25 * (A * Bv - C * C) - (A + Bv) * (A + Bv);
  }
  G(out)[i] = R;
}

__global__ __launch_bounds__(256) void k_ab_harris_sep(AbArgs a) {
  int b;
  const AbLevel& L = a.lv[ab_level(a, (int)blockIdx.x, &b)];
  const uint8_t* img = L.img;
  int64_t* out = (int64_t*)L.out;
  const uint32_t* pos = L.pos;
  const int W = L.W, H = L.H, stride = L.stride, n = L.n;
  const int i = b * (int)blockDim.x + (int)threadIdx.x;
  if (i >= n) return;
  const uint32_t ps = G(pos)[i];
  const int x = (int)(ps & 0xffff), y = (int)(ps >> 16);
  int64_t R = 0;
  if (harris_in(x, y, W, H)) {
    gptr<const uint8_t> g = G(img);
    int hx[3][7], hs[3][7];  // rolling rows of [-1 0 1] and [1 2 1] along x
    int sxx = 0, syy = 0, sxy = 0;
    for (int r = 0; r < 9; ++r) {
      int a[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) a[k] = g[(size_t)(y - 4 + r) * stride + x - 4 + k];
      const int slot = r % 3;
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        hx[slot][k] = a[k + 2] - a[k];
        hs[slot][k] = a[k] + 2 * a[k + 1] + a[k + 2];
      }
      if (r >= 2) {  // window row r - 1 (rows r - 2, r - 1, r are held)
        const int s0 = (r - 2) % 3, s1 = (r - 1) % 3, s2 = r % 3;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
          const int gx = hx[s0][k] + 2 * hx[s1][k] + hx[s2][k];
          const int gy = hs[s2][k] - hs[s0][k];
          sxx += gx * gx;
          syy += gy * gy;
          sxy += gx * gy;
        }
      }
    }
    const int64_t A = sxx, Bv = syy, C = sxy;
    R = 25 * (A * Bv - C * C) - (A + Bv) * (A + Bv);
  }
  G(out)[i] = R;
}

__global__ __launch_bounds__(256) void k_ab_harris_groups(AbArgs a) {
  int b;
  const AbLevel& L = a.lv[ab_level(a, (int)blockIdx.x, &b)];
  const uint8_t* img = L.img;
  int64_t* out = (int64_t*)L.out;
  const uint32_t* pos = L.pos;
  const int W = L.W, H = L.H, stride = L.stride, n = L.n;
  const int c = b * (int)(blockDim.x >> 3) + (int)(threadIdx.x >> 3);
  const int s = (int)(threadIdx.x & 7);
  int sxx = 0, syy = 0, sxy = 0;
  bool ok = false;
  if (c < n) {
    const uint32_t ps = G(pos)[c];
    const int x = (int)(ps & 0xffff), y = (int)(ps >> 16);
    ok = harris_in(x, y, W, H);
    if (ok && s < 7) {
      gptr<const uint8_t> r0 = G(img) + (size_t)(y + s - 4) * stride + (x - 4);
      int a[9], b[9], d[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        a[k] = r0[k];
        b[k] = r0[stride + k];
        d[k] = r0[2 * stride + k];
      }
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        const int gx = (a[k + 1] - a[k - 1]) + 2 * (b[k + 1] - b[k - 1]) + (d[k + 1] - d[k - 1]);
        const int gy = (d[k - 1] + 2 * d[k] + d[k + 1]) - (a[k - 1] + 2 * a[k] + a[k + 1]);
        sxx += gx * gx;
        syy += gy * gy;
        sxy += gx * gy;
      }
    }
  }
  sxx = group8_sum(sxx);
  syy = group8_sum(syy);
  sxy = group8_sum(sxy);
  if (c < n && s == 0) {
    const int64_t A = sxx, Bv = syy, C = sxy;
    G(out)[c] = ok ? 25 * (A * Bv - C * C) - (A + Bv) * (A + Bv) : 0;
  }
}

// Dense R' over the whole level by sliding sums: per 64 x 32 output tile, Sobel at every
// pixel of the tile and a 3-pixel ring (LDS), products summed down 7-row columns, then
// along 7-column rows.  Pixels closer than 4 to the border get 0.
__global__ __launch_bounds__(256) void k_ab_harris_dense(AbArgs a) {
  int b;
  const AbLevel& L = a.lv[ab_level(a, (int)blockIdx.x, &b)];
  const uint8_t* img = L.img;
  int64_t* out = (int64_t*)L.out;
  const int W = L.W, H = L.H, stride = L.stride;
  constexpr int TW = 64, TH = 32, GW = TW + 6, GH = TH + 6, PW = TW + 8, PH = TH + 8;
  __shared__ uint8_t pix[PH][PW];
  __shared__ int16_t sgx[GH][GW], sgy[GH][GW];
  __shared__ int32_t col[3][TH][GW];
  const int tx0 = (b % cdiv(W, TW)) * TW, ty0 = (b / cdiv(W, TW)) * TH;
  gptr<const uint8_t> g = G(img);
  for (int i = (int)threadIdx.x; i < PH * PW; i += 256) {
    const int r = i / PW, c = i - r * PW;
    const int gx = min(max(tx0 - 4 + c, 0), W - 1), gy = min(max(ty0 - 4 + r, 0), H - 1);
    pix[r][c] = g[(size_t)gy * stride + gx];
  }
  lds_barrier();
  for (int i = (int)threadIdx.x; i < GH * GW; i += 256) {
    const int r = i / GW, c = i - r * GW;
    auto I = [&](int u, int v) { return (int)pix[r + 1 + v][c + 1 + u]; };
    sgx[r][c] = (int16_t)((I(1, -1) + 2 * I(1, 0) + I(1, 1)) - (I(-1, -1) + 2 * I(-1, 0) + I(-1, 1)));
    sgy[r][c] = (int16_t)((I(-1, 1) + 2 * I(0, 1) + I(1, 1)) - (I(-1, -1) + 2 * I(0, -1) + I(1, -1)));
  }
  lds_barrier();
  // column sums: one thread per (column, product), sliding down the rows
  for (int i = (int)threadIdx.x; i < 3 * GW; i += 256) {
    const int k = i / GW, c = i - k * GW;
    auto prod = [&](int r) {
      const int a = sgx[r][c], b = sgy[r][c];
      return k == 0 ? a * a : (k == 1 ? b * b : a * b);
    };
    int acc = 0;
    for (int r = 0; r < 7; ++r) acc += prod(r);
    col[k][0][c] = acc;
    for (int r = 1; r < TH; ++r) {
      acc += prod(r + 6) - prod(r - 1);
      col[k][r][c] = acc;
    }
  }
  lds_barrier();
  // row sums: one thread per output row segment of 8 pixels, sliding along the row
  for (int i = (int)threadIdx.x; i < TH * (TW / 8); i += 256) {
    const int r = i / (TW / 8), c0 = (i - r * (TW / 8)) * 8;
    int a = 0, b = 0, d = 0;
    for (int c = c0; c < c0 + 7; ++c) {
      a += col[0][r][c];
      b += col[1][r][c];
      d += col[2][r][c];
    }
    for (int c = c0; c < c0 + 8; ++c) {
      if (c > c0) {
        a += col[0][r][c + 6] - col[0][r][c - 1];
        b += col[1][r][c + 6] - col[1][r][c - 1];
        d += col[2][r][c + 6] - col[2][r][c - 1];
      }
      const int x = tx0 + c, y = ty0 + r;
      if (x < W && y < H) {
        const int64_t A = a, Bv = b, C = d;
        G(out)[(size_t)y * W + x] =
            harris_in(x, y, W, H) ? 25 * (A * Bv - C * C) - (A + Bv) * (A + Bv) : 0;
      }
    }
  }
}

// ------------------------------------------------------- static workspace --

// The workspace of of_detect_batch_scratch: device memory of the library itself, for
// callers that cannot allocate (code under graph capture, tight serving loops).  Each
// device holds its own copy from the library's load until the process ends.  Host code
// never passes the array's name to a kernel or a copy: the name is a host-side stand-in;
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) uint8_t scratch[OF_SCRATCH_BYTES];

hipError_t scratch_workspace(void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // with device `dev` current
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// Events attached to the next launch (profiling): recorded by the dispatch itself, so
// they time the kernel alone.
thread_local LaunchEvents g_launch_ev;

void set_launch_events(hipEvent_t start, hipEvent_t stop) { g_launch_ev = {start, stop}; }

#define OF_LAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                   \
  do {                                                                                      \
    if (g_launch_ev.start || g_launch_ev.stop) {                                            \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, g_launch_ev.start,          \
                            g_launch_ev.stop, 0, __VA_ARGS__);                              \
      g_launch_ev = {};                                                                     \
    } else {                                                                                \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                  \
    }                                                                                       \
  } while (0)

hipError_t launch_prologue(const PrologueArgs& a, int grid, hipStream_t s) {
  OF_LAUNCH(k_prologue, dim3(grid), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pyramid(const PyrArgs& a, int n_levels, int max_w, int max_h, hipStream_t s) {
  dim3 grid(cdiv(max_w, 64), cdiv(max_h, 16), n_levels);
  OF_LAUNCH(k_pyramid, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pyramid_batch(const KArgs& a, int blocks, hipStream_t s) {
  OF_LAUNCH(k_pyramid_batch, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int TWW>
void launch_mark_w(const KArgs& a, bool fused, int grid, int bytes, hipStream_t s) {
  if (fused && a.persistent)
    OF_LAUNCH((k_mark<true, TWW, true>), dim3(grid), dim3(256), bytes, s, a);
  else if (fused)
    OF_LAUNCH((k_mark<true, TWW, false>), dim3(grid), dim3(256), bytes, s, a);
  else if (a.persistent)
    OF_LAUNCH((k_mark<false, TWW, true>), dim3(grid), dim3(256), bytes, s, a);
  else
    OF_LAUNCH((k_mark<false, TWW, false>), dim3(grid), dim3(256), bytes, s, a);
}

hipError_t launch_mark(const KArgs& a, bool fused, int grid, hipStream_t s) {
  const int bytes = a.ml.bytes + base_table_bytes(a.n_entries);
  switch (a.t.mark_words) {
    case 1: launch_mark_w<1>(a, fused, grid, bytes, s); break;
    case 2: launch_mark_w<2>(a, fused, grid, bytes, s); break;
    case 3: launch_mark_w<3>(a, fused, grid, bytes, s); break;
    default: launch_mark_w<4>(a, fused, grid, bytes, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_detect(const KArgs& a, int grid, hipStream_t s) {
  const int bytes = a.dl.bytes + base_table_bytes(a.n_entries);
  // the shipped and default tile shapes with their layout compiled in
  const bool cells = a.cell > 0;
  const int sa = cells ? a.t.det_cx : a.t.det_w, sb = cells ? a.t.det_cy : a.t.det_h;
  if (a.persistent)
    OF_LAUNCH((k_detect<true, 0, 0, 0>), dim3(grid), dim3(256), bytes, s, a);
  else if (a.cell == 30 && sa == 8 && sb == 1)
    OF_LAUNCH((k_detect<false, 8, 1, 30>), dim3(grid), dim3(256), bytes, s, a);
  else if (a.cell == 30 && sa == 4 && sb == 2)
    OF_LAUNCH((k_detect<false, 4, 2, 30>), dim3(grid), dim3(256), bytes, s, a);
  else if (!cells && sa == 128 && sb == 32)
    OF_LAUNCH((k_detect<false, 128, 32, 0>), dim3(grid), dim3(256), bytes, s, a);
  else if (!cells && sa == 64 && sb == 32)
    OF_LAUNCH((k_detect<false, 64, 32, 0>), dim3(grid), dim3(256), bytes, s, a);
  else
    OF_LAUNCH((k_detect<false, 0, 0, 0>), dim3(grid), dim3(256), bytes, s, a);
  return hipGetLastError();
}

// Candidate counters of the entries (one, or all when entry < 0) divided by `times`:
// after a Harris/NMS launch issued `times` times back to back for profiling, each count
// is exactly `times` times its value (every issue adds the same amount).
// Every sub-counter of the filled slots and FAST candidates divided by the number of
// repeated issues (each issue adds the same amounts to the same sub-counters).
__global__ __launch_bounds__(256) void k_scale_counters(uint32_t* counters, int n, int entry,
                                                        int times) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int e = entry >= 0 ? entry : i;
  if ((entry >= 0 && i > 0) || e >= n) return;
  const int cs = count_stride(n);
  for (int k = 0; k < 2 * kCountSpread; ++k) G(counters)[k * cs + e] /= (uint32_t)times;
}

hipError_t launch_scale_counters(const KArgs& a, int times, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_counters, dim3(cdiv(a.n_entries, 256)), dim3(256), 0, s, a.counters,
                     a.n_entries, a.entry, times);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sum_fast_counts(const uint32_t* counters, int n,
                                                         int32_t* out) {
  const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (e >= n) return;
  const int cs = count_stride(n);
  G(out)[e] = (int32_t)count_sum(G(counters) + kCountSpread * cs + e, cs);
}

hipError_t launch_sum_fast_counts(const uint32_t* counters, int n, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_fast_counts, dim3(cdiv(n, 256)), dim3(256), 0, s, counters, n, out);
  return hipGetLastError();
}

hipError_t launch_select_orient(const KArgs& a, int slots, hipStream_t s) {
  OF_LAUNCH(k_select_orient, dim3(cdiv(slots, 4)), dim3(256), 8 * a.sel_lds, s, a);
  return hipGetLastError();
}

hipError_t launch_select(const KArgs& a, int grid, hipStream_t s) {
  OF_LAUNCH(k_select, dim3(grid), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_test_segment(const uint8_t* circles, int n, int t_lo, int t_hi, uint8_t* out,
                               hipStream_t s) {
  OF_LAUNCH(k_test_segment, dim3(cdiv(n, 256)), dim3(256), 0, s, circles, n, t_lo, t_hi,
                     out);
  return hipGetLastError();
}

int ablate_fast_blocks(int variant, int W, int H) {
  return cdiv(W, 64) * cdiv(H, variant == 0 ? 4 : 16);
}

int ablate_harris_blocks(int variant, int W, int H, int n) {
  switch (variant) {
    case 0:
    case 1: return cdiv(n, 256);
    case 2: return cdiv(n, 32);
    default: return cdiv(W, 64) * cdiv(H, 32);
  }
}

static int ab_total(const AbArgs& a, int variant, bool fast) {
  const AbLevel& L = a.lv[a.n_levels - 1];
  return L.base + (fast ? ablate_fast_blocks(variant, L.W, L.H)
                        : ablate_harris_blocks(variant, L.W, L.H, L.n));
}

hipError_t launch_ablate_fast(const AbArgs& a, int variant, hipStream_t s) {
  const dim3 grid(ab_total(a, variant, true));
  switch (variant) {
    case 0: OF_LAUNCH(k_ab_fast_branchy, grid, dim3(256), 0, s, a); break;
    case 1: OF_LAUNCH((k_ab_fast_masks<false>), grid, dim3(256), 0, s, a); break;
    case 2: OF_LAUNCH((k_ab_fast_masks<true>), grid, dim3(256), 0, s, a); break;
    case 3: OF_LAUNCH((k_ab_fast_minmax<false>), grid, dim3(256), 0, s, a); break;
    default: OF_LAUNCH((k_ab_fast_minmax<true>), grid, dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_ablate_harris(const AbArgs& a, int variant, hipStream_t s) {
  const dim3 grid(ab_total(a, variant, false));
  switch (variant) {
    case 0: OF_LAUNCH(k_ab_harris_2d, grid, dim3(256), 0, s, a); break;
    case 1: OF_LAUNCH(k_ab_harris_sep, grid, dim3(256), 0, s, a); break;
    case 2: OF_LAUNCH(k_ab_harris_groups, grid, dim3(256), 0, s, a); break;
    default: OF_LAUNCH(k_ab_harris_dense, grid, dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_describe(const DescArgs& a, hipStream_t s) {
  OF_LAUNCH(k_describe, dim3(cdiv(a.n * a.cap, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ofk
