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
//   k_select, k_orient -- radix-select fallback for levels with very many candidates
// Wave64 throughout; nothing here is a dense contraction, so there is no MFMA use.
#include <hip/hip_runtime.h>

#include "of_kernels.h"

namespace ofk {

template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> G(T* p) {
  return (gptr<T>)p;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

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

// Ranking order: higher R' first; equal R' -> smaller y, then smaller x (pos = y<<16|x).
__device__ __forceinline__ bool better(int64_t sa, uint32_t pa, int64_t sb, uint32_t pb) {
  return sa > sb || (sa == sb && pa < pb);
}

// Last index e with base[e] <= g, base non-decreasing with n + 1 entries.
__device__ __forceinline__ int find_entry(const int32_t* base, int n, int g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Segment test at two thresholds from the 16 circle differences d[i] = I_i - I_p.
// A bright run of 9 at threshold t exists iff max_s min_{k<9} d[s+k] >= t; a dark run
// iff -(min_s max_{k<9} d[s+k]) >= t.  Both come from 3-input min/max over cyclic
// windows (3 x 3 = 9 positions).  Returns bit 0 = corner at t_lo, bit 1 = at t_hi.
__device__ __forceinline__ uint32_t segment_test2(const int (&d)[16], int t_lo, int t_hi) {
  int mn3[16], mx3[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    mn3[i] = imin3(d[i], d[(i + 1) & 15], d[(i + 2) & 15]);
    mx3[i] = imax3(d[i], d[(i + 1) & 15], d[(i + 2) & 15]);
  }
  int sb = -1024, sd = 1024;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    sb = max(sb, imin3(mn3[i], mn3[(i + 3) & 15], mn3[(i + 6) & 15]));
    sd = min(sd, imax3(mx3[i], mx3[(i + 3) & 15], mx3[(i + 6) & 15]));
  }
  const int s = max(sb, -sd);
  return (s >= t_lo ? 1u : 0u) | (s >= t_hi ? 2u : 0u);
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

// Copy rows [y0, y1) x cols [x0, x1) of an 8-bit image into LDS (row pitch lp, origin
// (x0, y0)); x0 is a multiple of 4.  Waves take rows (row base in scalar registers),
// lanes take 32-bit words; each wave keeps four rows of loads in flight.  Whole words
// where the source row allows, bytes at a ragged right edge.
__device__ __forceinline__ uint32_t load_word(gptr<const uint8_t> s, bool whole, int n) {
  if (whole) return *(gptr<const uint32_t>)s;
  uint32_t v = 0;
  for (int k = 0; k < n; ++k) v |= (uint32_t)s[k] << (8 * k);
  return v;
}

__device__ __forceinline__ void stage_rows(uint8_t* lds, int lp, gptr<const uint8_t> src,
                                           int stride, int row_limit, int x0, int x1, int y0,
                                           int y1) {
  constexpr int U = 4;
  const bool aligned = ((((uintptr_t)src) | (uintptr_t)stride) & 3) == 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int nw = (x1 - x0 + 3) >> 2;
  const int nrow = y1 - y0;
  for (int r0 = wave * U; r0 < nrow; r0 += nwave * U) {
    for (int w0 = 0; w0 < nw; w0 += 64) {
      const int w = w0 + lane;
      const int x = x0 + 4 * w;
      const bool in_x = w < nw;
      const bool whole = aligned && x + 4 <= row_limit;
      const int nb = min(4, x1 - x);
      uint32_t v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = 0;
        if (in_x && r0 + u < nrow)
          v[u] = load_word(src + (size_t)(y0 + r0 + u) * stride + x, whole, nb);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (in_x && r0 + u < nrow) *(uint32_t*)(lds + (r0 + u) * lp + 4 * w) = v[u];
    }
  }
}

// Harris R' at LDS pixel (cx, cy): Sobel G_x, G_y (Eq. 4) at the 49 pixels of the 7x7
// window, summed as Sxx, Syy, Sxy (int32), R' = 25 (Sxx Syy - Sxy^2) - (Sxx + Syy)^2.
// Separable form: each of the 9 rows gives horizontal differences hd = I[c+1] - I[c-1]
// and smoothings hs = I[c-1] + 2 I[c] + I[c+1]; two earlier rows stay in registers and
// G_x = hd[r-1] + 2 hd[r] + hd[r+1], G_y = hs[r+1] - hs[r-1].
__device__ __forceinline__ void harris_row(const uint8_t* row, int (&hd)[7], int (&hs)[7]) {
  int v[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) v[k] = row[k];
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    hd[c] = v[c + 2] - v[c];
    hs[c] = v[c] + 2 * v[c + 1] + v[c + 2];
  }
}

__device__ __forceinline__ int64_t harris_lds(const uint8_t* pix, int P, int cx, int cy) {
  int hd0[7], hs0[7], hd1[7], hs1[7];
  const uint8_t* row = pix + (cy - 4) * P + (cx - 4);
  harris_row(row, hd0, hs0);
  harris_row(row + P, hd1, hs1);
  int sxx = 0, syy = 0, sxy = 0;
#pragma unroll 1
  for (int r = 2; r < 9; ++r) {
    int hd2[7], hs2[7];
    harris_row(row + r * P, hd2, hs2);
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      const int gx = hd0[c] + 2 * hd1[c] + hd2[c];
      const int gy = hs2[c] - hs0[c];
      sxx += gx * gx;
      syy += gy * gy;
      sxy += gx * gy;
      hd0[c] = hd1[c];
      hd1[c] = hd2[c];
      hs0[c] = hs1[c];
      hs1[c] = hs2[c];
    }
  }
  const int64_t a = sxx, b = syy, c = sxy;
  return 25 * (a * b - c * c) - (a + b) * (a + b);
}

// Out-of-line Harris for the rare candidates beyond the per-tile score cache.
__device__ __noinline__ int64_t harris_lds_uncached(const uint8_t* pix, int P, int cx, int cy) {
  return harris_lds(pix, P, cx, cy);
}

// Harris R' of candidates by groups of 8 lanes: lane s < 7 of a group forms the Sobel
// gradients (Eq. 4) at the 7 pixels of window row dy = s - 3 from 3 staged rows and
// sums gx^2, gy^2, gx*gy; the 7 row sums are added across the group and R' is formed
// by lane 0.  Every lane of the block runs the same number of rounds.
__device__ __forceinline__ void harris_groups(const uint8_t* pix, int P, const uint32_t* cpos,
                                              int64_t* crs, int n, int sx0, int sy0) {
  const int s = threadIdx.x & 7;
  const int groups = blockDim.x >> 3;
  for (int cb = 0; cb < n; cb += groups) {
    const int c = cb + (threadIdx.x >> 3);
    int sxx = 0, syy = 0, sxy = 0;
    if (c < n && s < 7) {
      const uint32_t pos = cpos[c];
      const int cx = (int)(pos & 0xffff) - sx0, cy = (int)(pos >> 16) - sy0;
      const uint8_t* r0 = pix + (cy + s - 4) * P + (cx - 4);
      int a[9], b[9], d[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        a[k] = r0[k];
        b[k] = r0[P + k];
        d[k] = r0[2 * P + k];
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
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      sxx += __shfl_xor(sxx, o, 8);
      syy += __shfl_xor(syy, o, 8);
      sxy += __shfl_xor(sxy, o, 8);
    }
    if (c < n && s == 0) {
      const int64_t A = sxx, B = syy, C = sxy;
      crs[c] = 25 * (A * B - C * C) - (A + B) * (A + B);
    }
  }
}

// Exclusive scan of cnt[0..n) into pre[0..n], pre[n] = total, by the whole block.
__device__ void block_scan_u32(const uint32_t* cnt, uint32_t* pre, int n, uint32_t* s_wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  uint32_t carry = 0;
  for (int base = 0; base < n; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < n ? cnt[i] : 0u;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    if (lane == 63) s_wsum[wave] = inc;
    __syncthreads();
    uint32_t woff = 0, total = 0;
    for (int w = 0; w < nwave; ++w) {
      const uint32_t s = s_wsum[w];
      if (w < wave) woff += s;
      total += s;
    }
    if (i < n) pre[i] = carry + woff + inc - v;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) pre[n] = carry;
  __syncthreads();
}

// Intensity-centroid moments over the disk dx^2 + dy^2 <= r^2 around (x, y), one wave
// cooperating: lanes cover rows of the disk, all loads of a batch are issued first.
__device__ __forceinline__ void wave_moments(gptr<const uint8_t> lvl, int stride, int x, int y,
                                             int r, int lane, int* m10, int* m01) {
  const int span = 2 * r + 1;
  const int cspan = min(span, 64);
  const int rows_per = 64 / cspan;
  const int lr = lane / cspan, lc = lane - lr * cspan;
  const int r2 = r * r;
  int a = 0, b = 0;
  if (lr < rows_per) {
    for (int c0 = 0; c0 < span; c0 += cspan) {
      const int dx = c0 + lc - r;
      for (int k0 = 0; k0 * rows_per < span; k0 += 16) {
        int v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int dy = (k0 + k) * rows_per + lr - r;
          const bool in = dy <= r && dx <= r && dx * dx + dy * dy <= r2;
          v[k] = in ? (int)lvl[(size_t)(y + dy) * stride + x + dx] : 0;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int dy = (k0 + k) * rows_per + lr - r;
          a += dx * v[k];
          b += dy * v[k];
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
__device__ __forceinline__ void queue_start(const KArgs& a, uint32_t* ctr, int* s_next) {
  if (a.persistent && threadIdx.x == 0) *s_next = (int)atomicAdd(ctr, 1u);
}

__device__ __forceinline__ int queue_take(const KArgs& a, int iter, int* s_next) {
  if (!a.persistent) return iter == 0 ? (int)blockIdx.x : a.total;
  __syncthreads();
  return *s_next;
}

__device__ __forceinline__ int queue_prefetch(const KArgs& a, int g, uint32_t* ctr) {
  return (a.persistent && threadIdx.x == 0 && g < a.total) ? (int)atomicAdd(ctr, 1u) : 0;
}

__device__ __forceinline__ void queue_park(const KArgs& a, int next, int* s_next) {
  if (a.persistent && threadIdx.x == 0) *s_next = next;
}

// Copy of an exclusive prefix (n + 1 values) into LDS for entry lookups.
__device__ __forceinline__ void load_bases(int32_t* s_base, const int32_t* base, int n) {
  for (int i = threadIdx.x; i <= n; i += blockDim.x) s_base[i] = G(base)[i];
  __syncthreads();
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
    const int64_t ncnt = 2 * (int64_t)a.lay.n_entries;
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
  const int64_t o_or = scan(s.orient_blocks);
  const int64_t t_or = s_tot;
  const int64_t o_flag = scan(s.flag_bytes);
  const int64_t o_bm = scan(s.bm_words);
  const int64_t o_cand = scan(s.cand_cap);
  const int64_t o_rank = scan(s.cand_cap < kRankCap ? s.cand_cap : kRankCap);
  const int64_t t_rank = s_tot;
  const int64_t o_sel = scan(s.sel_cap);
  const int64_t o_lvl = scan(s.lvl_bytes);

  LevelPlan* plan = (LevelPlan*)(ws + a.lay.off_plan);
  int32_t* mark_base = (int32_t*)(ws + a.lay.off_mark_base);
  int32_t* det_base = (int32_t*)(ws + a.lay.off_det_base);
  int32_t* or_base = (int32_t*)(ws + a.lay.off_orient_base);
  int32_t* rank_base = (int32_t*)(ws + a.lay.off_rank_base);
  uint32_t* counters = (uint32_t*)(ws + a.lay.off_counters);

  if (i < nL) {
    LevelPlan P;
    P.W = g.W[l];
    P.H = g.H[l];
    P.B = a.p.patch_radius;
    P.level = l;
    P.frame = f;
    P.n_levels = L;
    P.cs = g.cs[l];
    P.ncx = g.ncx[l];
    P.ncy = g.ncy[l];
    P.quota = g.quota[l];
    P.kcell = g.kcell[l];
    P.fast_t = a.p.fast_t;
    P.fast_t_min = a.p.fast_t_min;
    P.base = a.f[f].data;
    P.base_w = a.f[f].w;
    P.base_h = a.f[f].h;
    P.base_stride = a.f[f].stride;
    if (l == 0) {
      P.lvl = a.f[f].data;
      P.lvl_w = nullptr;
      P.lvl_stride = a.f[f].stride;
    } else {
      P.lvl_w = ws + a.lay.off_lvl + o_lvl;
      P.lvl = P.lvl_w;
      P.lvl_stride = level_stride(P.W);
    }
    P.wpr = s.wpr;
    P.bm_lo = (uint32_t*)(ws + a.lay.off_bm) + o_bm;
    P.bm_hi = P.bm_lo + (int64_t)s.wpr * P.H;
    P.flags = ws + a.lay.off_flags + o_flag;
    P.cand = (Cand*)(ws + a.lay.off_cand) + o_cand;
    P.cand_count = counters + i;
    P.cand_cap = (int32_t)s.cand_cap;
    P.sel = (Cand*)(ws + a.lay.off_sel) + o_sel;
    P.sel_count = counters + a.lay.n_entries + i;
    P.mark_tx = s.mark_tx;
    P.mark_ty = s.mark_ty;
    P.det_tx = s.det_tx;
    P.det_ty = s.det_ty;
    P.det_x0 = s.det_x0;
    P.det_y0 = s.det_y0;
    P.det_xend = s.det_xend;
    P.det_yend = s.det_yend;
    P.orient_blocks = s.orient_blocks;
    P.entry0 = f * L;
    P.out = a.out + a.f[f].out_off;
    P.count_out = a.counts + f;
    plan[i] = P;
    mark_base[i] = (int32_t)o_mark;
    det_base[i] = (int32_t)o_det;
    or_base[i] = (int32_t)o_or;
    rank_base[i] = (int32_t)o_rank;
  }
  if (i == 0) {
    mark_base[nL] = (int32_t)t_mark;
    det_base[nL] = (int32_t)t_det;
    or_base[nL] = (int32_t)t_or;
    rank_base[nL] = (int32_t)t_rank;
  }
  __threadfence();
  __syncthreads();
  if (i == 0) *sig = a.sig;
}

// ----------------------------------------------------------------- pyramid --

// One block = 64 x 16 output pixels of level blockIdx.z; the tap tables of its columns
// and rows are computed once in LDS.  Weights are Q8; one rounding at the end.
__global__ __launch_bounds__(256) void k_pyramid(PyrArgs a) {
  __shared__ uint32_t xt[64], yt[16];
  const PyrLevel L = a.lv[blockIdx.z];
  const int bx = blockIdx.x * 64, by = blockIdx.y * 16;
  if (bx >= L.w || by >= L.h) return;
  const int t = threadIdx.x;
  if (t < 64 && bx + t < L.w) xt[t] = resample_tap(bx + t, a.src_w, L.w);
  if (t >= 64 && t < 80 && by + t - 64 < L.h) yt[t - 64] = resample_tap(by + t - 64, a.src_h, L.h);
  __syncthreads();
  const int lx = t & 63;
  const int x = bx + lx;
  if (x >= L.w) return;
  gptr<const uint8_t> src = G(a.src);
  const uint32_t tx = xt[lx];
  const int x0 = tx >> 9, wx = tx & 511;
  const int x1 = min(x0 + 1, a.src_w - 1);
  int v[4][4];
  int wy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int ly = min((t >> 6) * 4 + k, L.h - 1 - by);
    const uint32_t ty = yt[ly];
    const int y0 = ty >> 9;
    wy[k] = ty & 511;
    const int y1 = min(y0 + 1, a.src_h - 1);
    v[k][0] = src[(size_t)y0 * a.src_stride + x0];
    v[k][1] = src[(size_t)y0 * a.src_stride + x1];
    v[k][2] = src[(size_t)y1 * a.src_stride + x0];
    v[k][3] = src[(size_t)y1 * a.src_stride + x1];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int y = by + (t >> 6) * 4 + k;
    if (y >= L.h) break;
    const int top = (256 - wx) * v[k][0] + wx * v[k][1];
    const int bot = (256 - wx) * v[k][2] + wx * v[k][3];
    G(L.dst)[(size_t)y * L.stride + x] = (uint8_t)(((256 - wy[k]) * top + wy[k] * bot + 32768) >> 16);
  }
}

// ------------------------------------------------------------ segment test --

// One block per segment-test tile of 64*TWW x mark_rows level pixels.  TWW fixes the
// LDS row pitch at compile time, so every circle and compass offset below is a
// ds_read immediate.
template <bool FUSED, int TWW>
__global__ __launch_bounds__(256) void k_mark(KArgs a) {
  constexpr int TW = 64 * TWW;
  constexpr int PITCH = TW + 8;
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ int s_next, s_qcnt[4];
  __shared__ int32_t s_base[kMaxEntries + 1];
  const MarkLds M = mark_lds(a.t);
  uint8_t* pix = smem;
  uint16_t* queue = (uint16_t*)(smem + M.off_queue);
  uint32_t* bml = (uint32_t*)(smem + M.off_bml);
  uint32_t* bmh = (uint32_t*)(smem + M.off_bmh);
  uint32_t* xt = (uint32_t*)(smem + M.off_xt);
  uint32_t* yt = (uint32_t*)(smem + M.off_yt);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  if (a.entry < 0) load_bases(s_base, a.mark_base, a.n_entries);
  queue_start(a, a.qctr + 0, &s_next);

  for (int iter = 0;; ++iter) {
    const int g = uniform(queue_take(a, iter, &s_next));
    if (g >= a.total) break;
    __syncthreads();  // every thread has read s_next
    const int next = queue_prefetch(a, g, a.qctr + 0);
    const int e = a.entry >= 0 ? a.entry : uniform(find_entry(s_base, a.n_entries, g));
    const int t = a.entry >= 0 ? g : g - s_base[e];
    const LevelPlan P = a.plan[e];
    const int W = P.W, H = P.H, B = P.B;
    const int tx = t % P.mark_tx, ty = t / P.mark_tx;
    const int x_t0 = tx * TW, x_t1 = min(W, x_t0 + TW);
    const int y_t0 = ty * M.th, y_t1 = min(H, y_t0 + M.th);
    const int ox = max(0, x_t0 - 4), oy = max(0, y_t0 - 3);
    const int ex = min(W, x_t1 + 3), ey = min(H, y_t1 + 3);
    const int nx = ex - ox, ny = ey - oy;

    // 1. level pixels of the tile and its 3-pixel halo
    if (FUSED && P.level > 0) {
      for (int i = threadIdx.x; i < nx; i += blockDim.x) xt[i] = resample_tap(ox + i, P.base_w, W);
      for (int j = threadIdx.x; j < ny; j += blockDim.x) yt[j] = resample_tap(oy + j, P.base_h, H);
      __syncthreads();
      // Column taps stay in registers (lane owns columns lane + 64c); each wave takes two
      // consecutive output rows at a time with their base-row pointers in scalar
      // registers, so a tap costs its load and the blend only.
      gptr<const uint8_t> base = G(P.base);
      const int bs = P.base_stride, bw1 = P.base_w - 1, bh1 = P.base_h - 1;
      constexpr int NC = TWW + 1;  // columns per lane: nx <= TW + 7
      int cx0[NC], cx1[NC], cwx[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const uint32_t txx = xt[min(lane + 64 * c, nx - 1)];
        cx0[c] = txx >> 9;
        cx1[c] = min(cx0[c] + 1, bw1);
        cwx[c] = txx & 511;
      }
      for (int j0 = 2 * wave; j0 < ny; j0 += 2 * nwave) {
        int v[2][NC][4];
        int wyr[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t tyy = (uint32_t)uniform((int)yt[min(j0 + h, ny - 1)]);
          const int y0 = tyy >> 9;
          wyr[h] = tyy & 511;
          gptr<const uint8_t> r0 = base + (size_t)y0 * bs;
          gptr<const uint8_t> r1 = base + (size_t)min(y0 + 1, bh1) * bs;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            v[h][c][0] = r0[cx0[c]];
            v[h][c][1] = r0[cx1[c]];
            v[h][c][2] = r1[cx0[c]];
            v[h][c][3] = r1[cx1[c]];
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = j0 + h;
          if (j >= ny) break;
          const int wy = wyr[h];
          uint8_t* prow = pix + j * PITCH;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const int i = lane + 64 * c;
            if (i < nx) {
              const int wx = cwx[c];
              const int top = (256 - wx) * v[h][c][0] + wx * v[h][c][1];
              const int bot = (256 - wx) * v[h][c][2] + wx * v[h][c][3];
              prow[i] = (uint8_t)(((256 - wy) * top + wy * bot + 32768) >> 16);
            }
          }
        }
      }
      __syncthreads();
      // the tile's own pixels go to the level buffer for the later steps
      const int lx0 = x_t0 - ox;
      const int nwd = (x_t1 - x_t0 + 3) >> 2;
      gptr<uint8_t> lw = G(P.lvl_w);
      for (int r = wave; r < y_t1 - y_t0; r += nwave) {
        const int y = y_t0 + r;
        for (int w0 = 0; w0 < nwd; w0 += 64) {
          const int w = w0 + lane;
          if (w < nwd)
            *(gptr<uint32_t>)(lw + (size_t)y * P.lvl_stride + x_t0 + 4 * w) =
                *(const uint32_t*)(pix + (y - oy) * PITCH + lx0 + 4 * w);
        }
      }
    } else {
      const int limit = P.level == 0 ? W : P.lvl_stride;
      stage_rows(pix, PITCH, G(P.lvl), P.lvl_stride, limit, ox, ex, oy, ey);
    }
    for (int i = threadIdx.x; i < 2 * M.th * 2 * TWW; i += blockDim.x) bml[i] = 0u;  // lo, hi
    __syncthreads();

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
      if (lane == 0) s_qcnt[wave] = qn;
    }
    __syncthreads();

    // 3. full segment test of the queued pixels at both thresholds
    int qoff[4];
    int qtot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      qoff[w] = qtot;
      qtot += w < nwave ? s_qcnt[w] : 0;
    }
    gptr<uint8_t> flags = G(P.flags);
    for (int q = threadIdx.x; q < qtot; q += blockDim.x) {
      int w = 0;
#pragma unroll
      for (int k = 1; k < 4; ++k) w += q >= qoff[k] ? 1 : 0;
      const int ent = queue[w * M.qseg + (q - qoff[w])];
      const int lx = ent & 511, ly = ent >> 9;
      const uint8_t* c0 = pix + (ly - 3) * PITCH + (lx - 3);  // top-left of the 7x7 box
      const int p = c0[3 * PITCH + 3];
      int d[16];
      d[0] = c0[3] - p;
      d[1] = c0[4] - p;
      d[2] = c0[PITCH + 5] - p;
      d[3] = c0[2 * PITCH + 6] - p;
      d[4] = c0[3 * PITCH + 6] - p;
      d[5] = c0[4 * PITCH + 6] - p;
      d[6] = c0[5 * PITCH + 5] - p;
      d[7] = c0[6 * PITCH + 4] - p;
      d[8] = c0[6 * PITCH + 3] - p;
      d[9] = c0[6 * PITCH + 2] - p;
      d[10] = c0[5 * PITCH + 1] - p;
      d[11] = c0[4 * PITCH] - p;
      d[12] = c0[3 * PITCH] - p;
      d[13] = c0[2 * PITCH] - p;
      d[14] = c0[PITCH + 1] - p;
      d[15] = c0[2] - p;
      const uint32_t r = segment_test2(d, tlo, thi);
      if (r) {
        const int x = ox + lx, y = oy + ly;
        const int bit = x - x_t0;
        const int word = (y - y_t0) * 2 * TWW + (bit >> 5);
        atomicOr(&bml[word], 1u << (bit & 31));
        if (r & 2u) {
          atomicOr(&bmh[word], 1u << (bit & 31));
          flags[(y / P.cs) * P.ncx + x / P.cs] = 1;
        }
      }
    }
    __syncthreads();

    // 4. bitmap words of the tile rows (zero outside the valid region)
    const int w0 = x_t0 >> 5;
    const int nwd = min(2 * TWW, P.wpr - w0);
    gptr<uint32_t> glo = G(P.bm_lo), ghi = G(P.bm_hi);
    {
      const int k = threadIdx.x & 7;  // at most 8 words per tile row
      for (int r = threadIdx.x >> 3; r < y_t1 - y_t0; r += blockDim.x >> 3) {
        if (k < nwd) {
          const size_t gi = (size_t)(y_t0 + r) * P.wpr + w0 + k;
          glo[gi] = bml[r * 2 * TWW + k];
          ghi[gi] = bmh[r * 2 * TWW + k];
        }
      }
    }
    queue_park(a, next, &s_next);
  }
}

// ------------------------------------------------------- Harris / NMS / cells --

__global__ __launch_bounds__(256) void k_detect(KArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ int s_next, s_ns, s_ne, s_base_out;
  __shared__ uint32_t s_wsum[16];
  __shared__ int32_t s_base[kMaxEntries + 1];
  const DetLds D = det_lds(a.t, a.cell);
  uint8_t* pix = smem;
  uint64_t* cw = (uint64_t*)(smem + D.off_cw);
  uint32_t* ucnt = (uint32_t*)(smem + D.off_ucnt);
  uint32_t* cpre = (uint32_t*)(smem + D.off_cpre);
  int64_t* crs = (int64_t*)(smem + D.off_crs);
  uint32_t* cpos = (uint32_t*)(smem + D.off_cpos);
  int64_t* srs = (int64_t*)(smem + D.off_srs);
  uint32_t* spos = (uint32_t*)(smem + D.off_spos);
  uint16_t* scell = (uint16_t*)(smem + D.off_scell);
  uint16_t* order = (uint16_t*)(smem + D.off_order);
  uint16_t* emit = (uint16_t*)(smem + D.off_emit);
  uint32_t* ccnt = (uint32_t*)(smem + D.off_ccnt);
  uint32_t* coff = (uint32_t*)(smem + D.off_coff);
  uint32_t* cfill = (uint32_t*)(smem + D.off_cfill);
  uint32_t* wlo = (uint32_t*)(smem + D.off_wlo);
  uint32_t* whi = (uint32_t*)(smem + D.off_whi);
  uint8_t* lfl = smem + D.off_lfl;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  if (a.entry < 0) load_bases(s_base, a.det_base, a.n_entries);
  queue_start(a, a.qctr + 2, &s_next);

  for (int iter = 0;; ++iter) {
    const int g = uniform(queue_take(a, iter, &s_next));
    if (g >= a.total) break;
    __syncthreads();  // every thread has read s_next
    const int next = queue_prefetch(a, g, a.qctr + 2);
    const int e = a.entry >= 0 ? a.entry : uniform(find_entry(s_base, a.n_entries, g));
    const int t = a.entry >= 0 ? g : g - s_base[e];
    const LevelPlan P = a.plan[e];
    const int W = P.W, H = P.H, B = P.B, cs = P.cs;
    const int tx = t % P.det_tx, ty = t / P.det_tx;
    int vx0, vx1, vy0, vy1, cxa = 0, cya = 0, nlcx = 1, nlcy = 1;
    if (a.cell > 0) {
      cxa = P.det_x0 + tx * a.t.det_cx;
      cya = P.det_y0 + ty * a.t.det_cy;
      const int cxb = min(cxa + a.t.det_cx, P.det_xend), cyb = min(cya + a.t.det_cy, P.det_yend);
      nlcx = cxb - cxa;
      nlcy = cyb - cya;
      vx0 = max(cxa * cs, B);
      vx1 = min(cxb * cs, W - B);
      vy0 = max(cya * cs, B);
      vy1 = min(cyb * cs, H - B);
    } else {
      vx0 = P.det_x0 + tx * a.t.det_w;
      vx1 = min(vx0 + a.t.det_w, P.det_xend);
      vy0 = P.det_y0 + ty * a.t.det_h;
      vy1 = min(vy0 + a.t.det_h, P.det_yend);
    }
    const int rx0 = vx0 - 1, ry0 = vy0 - 1;
    const int rw = vx1 - vx0 + 2, rh = vy1 - vy0 + 2;
    const int sx0 = max(0, vx0 - 5) & ~3, sy0 = max(0, vy0 - 5);
    const int sx1 = min(W, vx1 + 5), sy1 = min(H, vy1 + 5);
    const int nwr = (rw + 63) >> 6;
    const int nunits = rh * nwr;
    // bitmap words and cells touched by the tile and its 1-pixel ring
    const int bw0 = rx0 >> 5, nbw = ((rx0 + rw - 1) >> 5) - bw0 + 1;
    const int fcx0 = rx0 / cs, fcy0 = ry0 / cs;
    const int nfx = (rx0 + rw - 1) / cs - fcx0 + 1, nfy = (ry0 + rh - 1) / cs - fcy0 + 1;

    // 1. one batch of independent loads: bitmap words, flags, pixels (5-pixel halo)
    {
      gptr<const uint32_t> glo = G((const uint32_t*)P.bm_lo), ghi = G((const uint32_t*)P.bm_hi);
      gptr<const uint8_t> gfl = G((const uint8_t*)P.flags);
      const int nbm = rh * nbw, nfl = nfx * nfy;
      uint32_t vlo[2], vhi[2], vfl[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = u * (int)blockDim.x + (int)threadIdx.x;
        vlo[u] = vhi[u] = vfl[u] = 0;
        if (i < nbm) {
          const int r = i / nbw, k = i - r * nbw;
          const size_t gi = (size_t)(ry0 + r) * P.wpr + bw0 + k;
          vlo[u] = glo[gi];
          vhi[u] = ghi[gi];
        }
        if (i < nfl) {
          const int r = i / nfx, k = i - r * nfx;
          vfl[u] = gfl[(fcy0 + r) * P.ncx + fcx0 + k];
        }
      }
      stage_rows(pix, D.pitch, G(P.lvl), P.lvl_stride, P.level == 0 ? W : P.lvl_stride, sx0,
                 sx1, sy0, sy1);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = u * (int)blockDim.x + (int)threadIdx.x;
        if (i < nbm) {
          wlo[i] = vlo[u];
          whi[i] = vhi[u];
        }
        if (i < nfl) lfl[i] = (uint8_t)vfl[u];
      }
      for (int i = 2 * (int)blockDim.x + (int)threadIdx.x; i < nbm; i += blockDim.x) {
        const int r = i / nbw, k = i - r * nbw;
        const size_t gi = (size_t)(ry0 + r) * P.wpr + bw0 + k;
        wlo[i] = glo[gi];
        whi[i] = ghi[gi];
      }
      for (int i = 2 * (int)blockDim.x + (int)threadIdx.x; i < nfl; i += blockDim.x) {
        const int r = i / nfx, k = i - r * nfx;
        lfl[i] = gfl[(fcy0 + r) * P.ncx + fcx0 + k];
      }
    }
    if (threadIdx.x == 0) {
      s_ns = 0;
      s_ne = 0;
    }
    __syncthreads();
    // 2. candidate words over tile + ring: corner at the threshold of its own cell.
    //    Cell columns of a lane's pixels are fixed for the tile (nwr <= 5 words), cell
    //    rows advance with the row, so no division runs per pixel.
    {
      int lcx[5];
      bool xok[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const int lxr = 64 * k + lane;
        const int x = rx0 + lxr;
        xok[k] = k < nwr && lxr < rw && x >= B && x < W - B;
        lcx[k] = xok[k] ? x / cs - fcx0 : 0;
      }
      for (int j = wave; j < rh; j += nwave) {
        const int y = ry0 + j;
        const bool yok = y >= B && y < H - B;
        const uint8_t* frow = lfl + (y / cs - fcy0) * nfx;
        const uint32_t* rlo = wlo + j * nbw - bw0;
        const uint32_t* rhi = whi + j * nbw - bw0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          if (k >= nwr) break;
          const int x = rx0 + 64 * k + lane;
          bool c = false;
          if (yok && xok[k]) {
            const uint32_t bit = 1u << (x & 31);
            c = (rhi[x >> 5] & bit) != 0 || ((rlo[x >> 5] & bit) != 0 && frow[lcx[k]] == 0);
          }
          const uint64_t m = __ballot(c);
          if (lane == 0) {
            cw[j * nwr + k] = m;
            ucnt[j * nwr + k] = (uint32_t)__popcll(m);
          }
        }
      }
    }
    __syncthreads();
    block_scan_u32(ucnt, cpre, nunits, s_wsum);
    const int ncand = (int)cpre[nunits];
    // 3. cached candidate positions (raster order) and their Harris scores
    for (int j = wave; j < rh; j += nwave) {
      for (int k = 0; k < nwr; ++k) {
        const int u = j * nwr + k;
        const uint64_t m = cw[u];
        if ((m >> lane) & 1ull) {
          const uint32_t idx = cpre[u] + lanes_below(m);
          if (idx < (uint32_t)kCandCache)
            cpos[idx] = ((uint32_t)(ry0 + j) << 16) | (uint32_t)(rx0 + 64 * k + lane);
        }
      }
    }
    __syncthreads();
    const int ncache = min(ncand, kCandCache);
    harris_groups(pix, D.pitch, cpos, crs, ncache, sx0, sy0);
    __syncthreads();
    // 4. NMS: a tile candidate survives when it ranks above every candidate neighbour.
    //    One thread per candidate; neighbours are found through the candidate words.
    for (int ci = threadIdx.x; ci < ncand; ci += blockDim.x) {
      uint32_t pos;
      if (ci < kCandCache) {
        pos = cpos[ci];
      } else {  // beyond the cache: locate the ci-th candidate in raster order
        int lo = 0, hi = nunits - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (cpre[mid] <= (uint32_t)ci) lo = mid; else hi = mid - 1;
        }
        uint64_t m = cw[lo];
        for (uint32_t k = cpre[lo]; k < (uint32_t)ci; ++k) m &= m - 1ull;
        const int j = lo / nwr, k = lo - j * nwr;
        pos = ((uint32_t)(ry0 + j) << 16) | (uint32_t)(rx0 + 64 * k + __builtin_ctzll(m));
      }
      const int x = (int)(pos & 0xffff), y = (int)(pos >> 16);
      const int lxr = x - rx0, j = y - ry0;
      if (j == 0 || j == rh - 1 || lxr == 0 || lxr >= rw - 1) continue;  // ring only
      const int64_t R = ci < kCandCache ? crs[ci]
                                        : harris_lds_uncached(pix, D.pitch, x - sx0, y - sy0);
      bool alive = true;
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        const int dx = nb < 3 ? nb - 1 : (nb < 5 ? (nb == 3 ? -1 : 1) : nb - 6);
        const int dy = nb < 3 ? -1 : (nb < 5 ? 0 : 1);
        const int ql = lxr + dx;
        const int qu = (j + dy) * nwr + (ql >> 6);
        const uint64_t qm = cw[qu];
        const int qb = ql & 63;
        if ((qm >> qb) & 1ull) {
          const uint32_t qidx = cpre[qu] + (uint32_t)__popcll(qm & ((1ull << qb) - 1ull));
          const int qx = x + dx, qy = y + dy;
          const int64_t Rq = qidx < (uint32_t)kCandCache
                                 ? crs[qidx]
                                 : harris_lds_uncached(pix, D.pitch, qx - sx0, qy - sy0);
          alive = alive && better(R, pos, Rq, ((uint32_t)qy << 16) | (uint32_t)qx);
        }
      }
      if (alive) {
        const int si = atomicAdd(&s_ns, 1);
        srs[si] = R;
        spos[si] = pos;
        scell[si] = a.cell > 0 ? (uint16_t)((y / cs - cya) * nlcx + (x / cs - cxa)) : 0;
      }
    }
    __syncthreads();
    const int ns = s_ns;
    // 5. per-cell top-K (K = quota when the whole level is one cell)
    if (ns > 0) {
      const int K = P.kcell;
      const int ncell = nlcx * nlcy;
      for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
        ccnt[c] = 0;
        cfill[c] = 0;
      }
      __syncthreads();
      for (int s = threadIdx.x; s < ns; s += blockDim.x) atomicAdd(&ccnt[scell[s]], 1u);
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t o = 0;
        for (int c = 0; c < ncell; ++c) {
          coff[c] = o;
          o += ccnt[c];
        }
      }
      __syncthreads();
      for (int s = threadIdx.x; s < ns; s += blockDim.x) {
        const int c = scell[s];
        order[coff[c] + atomicAdd(&cfill[c], 1u)] = (uint16_t)s;
      }
      __syncthreads();
      for (int s = threadIdx.x; s < ns; s += blockDim.x) {
        const int c = scell[s];
        const uint32_t n = ccnt[c];
        bool keep = true;
        if ((int)n > K) {
          const int64_t R = srs[s];
          const uint32_t pos = spos[s];
          int rank = 0;
          const uint32_t o = coff[c];
          for (uint32_t q = 0; q < n && rank < K; ++q) {
            const int s2 = order[o + q];
            rank += better(srs[s2], spos[s2], R, pos) ? 1 : 0;
          }
          keep = rank < K;
        }
        if (keep) emit[atomicAdd(&s_ne, 1)] = (uint16_t)s;
      }
      __syncthreads();
      const int ne = s_ne;
      if (threadIdx.x == 0) s_base_out = (int)atomicAdd(P.cand_count, (uint32_t)ne);
      __syncthreads();
      const int base = s_base_out;
      gptr<Cand> out = G(P.cand);
      for (int i = threadIdx.x; i < ne; i += blockDim.x) {
        if (base + i < P.cand_cap) {
          const int s = emit[i];
          store_cand(out + base + i, srs[s], spos[s]);
        }
      }
    }
    queue_park(a, next, &s_next);
  }
}

// ------------------------------------------- level selection + orientation --

// One wave per candidate slot.  A candidate's rank is the number of candidates of its
// level that rank above it; ranks of the N_l best are exactly their sorted positions, so
// the wave that holds rank < N_l computes the orientation and writes its keypoint at
// out[level prefix + rank].  Levels whose candidate count exceeds kRankCap are left to
// the radix-select path.
__global__ __launch_bounds__(256) void k_select_orient(KArgs a) {
  __shared__ int32_t s_base[kMaxEntries + 1];
  load_bases(s_base, a.rank_base, a.n_entries);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot = (int)blockIdx.x * (blockDim.x >> 6) + wave;
  if (slot >= s_base[a.n_entries]) return;
  const int e = uniform(find_entry(s_base, a.n_entries, slot));
  const int i = slot - s_base[e];
  const LevelPlan P = a.plan[e];
  gptr<const uint32_t> counts = G((const uint32_t*)P.cand_count) - e;  // all entries
  const int C = min((int)counts[e], P.cand_cap);
  if (P.level == 0 && i == 0 && lane == 0) {
    int total = 0;
    for (int l = 0; l < P.n_levels; ++l) {
      const LevelPlan& Q = a.plan[P.entry0 + l];
      total += min(min((int)counts[P.entry0 + l], Q.cand_cap), Q.quota);
    }
    *G(P.count_out) = total;
  }
  if (i >= C || C > kRankCap) return;
  gptr<const Cand> cand = G((const Cand*)P.cand);
  const Cand me = load_cand(cand + i);
  // Count better candidates, 8 loads in flight per lane; a wave whose partial count
  // already reaches the quota cannot be selected and stops early.
  int cnt = 0;
  for (int j0 = 0; j0 < C; j0 += 8 * 64) {
    Cand o[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) o[u] = load_cand(cand + min(j0 + u * 64 + lane, C - 1));
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * 64 + lane;
      cnt += (j < C && better(o[u].score, o[u].pos, me.score, me.pos)) ? 1 : 0;
    }
    if (j0 + 8 * 64 < C && wave_sum(cnt) >= P.quota) return;
  }
  const int rank = wave_sum(cnt);
  if (rank >= P.quota) return;
  int prefix = 0;
  for (int l = 0; l < P.level; ++l) {
    const LevelPlan& Q = a.plan[P.entry0 + l];
    prefix += min(min((int)counts[P.entry0 + l], Q.cand_cap), Q.quota);
  }
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

// Bitonic sort of n (power of two) entries in LDS, best first.
__device__ void bitonic_best_first(int64_t* sc, uint32_t* ps, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int64_t x = sc[i], y = sc[ixj];
          const uint32_t px = ps[i], py = ps[ixj];
          const bool first_half = (i & k) == 0;
          const bool swap = first_half ? better(y, py, x, px) : better(x, px, y, py);
          if (swap) {
            sc[i] = y;
            sc[ixj] = x;
            ps[i] = py;
            ps[ixj] = px;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Levels with more than kRankCap candidates: the N-th best score by radix select (8
// bits at a time), ties at that score by the smallest positions, then a sort.
__global__ __launch_bounds__(1024) void k_select(KArgs a) {
  __shared__ int64_t sc[kSortCap];
  __shared__ uint32_t ps[kSortCap];
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_k, s_n, s_eq;
  const int e = a.entry >= 0 ? a.entry : (int)blockIdx.x;
  const LevelPlan P = a.plan[e];
  const int N = P.quota;
  const int C = min((int)*G(P.cand_count), P.cand_cap);
  if (a.rank_path && C <= kRankCap) return;  // handled by k_select_orient
  const int nout = min(C, N);
  if (N <= 0 || C <= 0) {
    if (threadIdx.x == 0) *G(P.sel_count) = 0;
    return;
  }
  gptr<const Cand> cand = G((const Cand*)P.cand);
  int nsort;
  if (C <= kSortCap) {
    nsort = C;
    for (int i = threadIdx.x; i < C; i += blockDim.x) {
      const Cand cd = load_cand(cand + i);
      sc[i] = cd.score;
      ps[i] = cd.pos;
    }
  } else {
    if (threadIdx.x == 0) {
      s_prefix = 0;
      s_k = (uint32_t)N;
    }
    uint64_t mask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
      __syncthreads();
      const uint64_t prefix = s_prefix;
      for (int i = threadIdx.x; i < C; i += blockDim.x) {
        const uint64_t u = score_key(load_cand(cand + i).score);
        if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t acc = 0, k = s_k;
        int dsel = 0;
        for (int dgt = 255; dgt >= 0; --dgt) {
          if (acc + hist[dgt] >= k) {
            dsel = dgt;
            break;
          }
          acc += hist[dgt];
        }
        s_k = k - acc;
        s_prefix = prefix | ((uint64_t)dsel << shift);
      }
      mask |= 255ull << shift;
      __syncthreads();
    }
    const uint64_t T = s_prefix;
    const uint32_t k_eq = s_k;
    if (threadIdx.x == 0) s_eq = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < C; i += blockDim.x)
      if (score_key(load_cand(cand + i).score) == T) atomicAdd(&s_eq, 1u);
    __syncthreads();
    uint32_t pcut = 0xffffffffu;
    if (s_eq > k_eq) {
      if (threadIdx.x == 0) {
        s_prefix = 0;
        s_k = k_eq;
      }
      uint32_t pmask = 0;
      for (int shift = 24; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        const uint32_t pp = (uint32_t)s_prefix;
        for (int i = threadIdx.x; i < C; i += blockDim.x) {
          const Cand cd = load_cand(cand + i);
          if (score_key(cd.score) == T && (cd.pos & pmask) == pp)
            atomicAdd(&hist[(cd.pos >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
          uint32_t acc = 0, k = s_k;
          int dsel = 0;
          for (int dgt = 0; dgt < 256; ++dgt) {
            if (acc + hist[dgt] >= k) {
              dsel = dgt;
              break;
            }
            acc += hist[dgt];
          }
          s_k = k - acc;
          s_prefix = pp | ((uint32_t)dsel << shift);
        }
        pmask |= 255u << shift;
        __syncthreads();
      }
      pcut = (uint32_t)s_prefix;
    }
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < C; i += blockDim.x) {
      const Cand cd = load_cand(cand + i);
      const uint64_t u = score_key(cd.score);
      if (u > T || (u == T && cd.pos <= pcut)) {
        const uint32_t slot = atomicAdd(&s_n, 1u);
        if (slot < (uint32_t)kSortCap) {
          sc[slot] = cd.score;
          ps[slot] = cd.pos;
        }
      }
    }
    __syncthreads();
    nsort = min((int)s_n, kSortCap);
  }
  int n2 = 1;
  while (n2 < nsort) n2 <<= 1;
  for (int i = nsort + threadIdx.x; i < n2; i += blockDim.x) {
    sc[i] = INT64_MIN;
    ps[i] = 0xffffffffu;
  }
  __syncthreads();
  bitonic_best_first(sc, ps, n2);
  gptr<Cand> sel = G(P.sel);
  for (int i = threadIdx.x; i < nout; i += blockDim.x) store_cand(sel + i, sc[i], ps[i]);
  if (threadIdx.x == 0) *G(P.sel_count) = (uint32_t)nout;
}

// Orientation of the radix-selected keypoints: one wave per keypoint.
__global__ __launch_bounds__(256) void k_orient(KArgs a) {
  const int b = (int)blockIdx.x;
  const int e = a.entry >= 0 ? a.entry : find_entry(a.orient_base, a.n_entries, b);
  const int chunk = a.entry >= 0 ? b : b - a.orient_base[e];
  const LevelPlan P = a.plan[e];
  gptr<const uint32_t> counts = G((const uint32_t*)P.cand_count) - e;
  const int C = min((int)counts[e], P.cand_cap);
  if (a.rank_path && C <= kRankCap) return;  // written by k_select_orient
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nsel = (int)*G(P.sel_count);
  int prefix = 0;
  for (int l = 0; l < P.level; ++l) {
    const LevelPlan& Q = a.plan[P.entry0 + l];
    prefix += min(min((int)counts[P.entry0 + l], Q.cand_cap), Q.quota);
  }
  if (!a.rank_path && P.level == 0 && chunk == 0 && threadIdx.x == 0) {
    int total = 0;
    for (int l = 0; l < P.n_levels; ++l) {
      const LevelPlan& Q = a.plan[P.entry0 + l];
      total += min(min((int)counts[P.entry0 + l], Q.cand_cap), Q.quota);
    }
    *G(P.count_out) = total;
  }
  gptr<const Cand> sel = G((const Cand*)P.sel);
  for (int kk = 0; kk < kOrientPerBlock / 4; ++kk) {
    const int i = chunk * kOrientPerBlock + wave * (kOrientPerBlock / 4) + kk;
    if (i >= nsel) break;
    const Cand cd = load_cand(sel + i);
    const int x = (int)(cd.pos & 0xffff), y = (int)(cd.pos >> 16);
    int m10, m01;
    wave_moments(G(P.lvl), P.lvl_stride, x, y, P.B, lane, &m10, &m01);
    if (lane == 0)
      store_keypoint(G(P.out) + prefix + i, x, y, P.level, m10, m01,
                     atan2f((float)m01, (float)m10), cd.score);
  }
}

// ------------------------------------------------------------ test kernel --

__global__ __launch_bounds__(256) void k_test_segment(const uint8_t* circles, int n, int t_lo,
                                                      int t_hi, uint8_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint8_t* c = circles + (size_t)i * 17;
  int d[16];
  for (int k = 0; k < 16; ++k) d[k] = (int)c[1 + k] - (int)c[0];
  out[i] = (uint8_t)segment_test2(d, t_lo, t_hi);
}

// ----------------------------------------------------------------- launches --

hipError_t launch_prologue(const PrologueArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_prologue, dim3(grid), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pyramid(const PyrArgs& a, int n_levels, int max_w, int max_h, hipStream_t s) {
  dim3 grid(cdiv(max_w, 64), cdiv(max_h, 16), n_levels);
  hipLaunchKernelGGL(k_pyramid, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int TWW>
void launch_mark_w(const KArgs& a, bool fused, int grid, int bytes, hipStream_t s) {
  if (fused)
    hipLaunchKernelGGL((k_mark<true, TWW>), dim3(grid), dim3(256), bytes, s, a);
  else
    hipLaunchKernelGGL((k_mark<false, TWW>), dim3(grid), dim3(256), bytes, s, a);
}

hipError_t launch_mark(const KArgs& a, bool fused, int grid, hipStream_t s) {
  const MarkLds M = mark_lds(a.t);
  switch (a.t.mark_words) {
    case 1: launch_mark_w<1>(a, fused, grid, M.bytes, s); break;
    case 2: launch_mark_w<2>(a, fused, grid, M.bytes, s); break;
    case 3: launch_mark_w<3>(a, fused, grid, M.bytes, s); break;
    default: launch_mark_w<4>(a, fused, grid, M.bytes, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_detect(const KArgs& a, int grid, hipStream_t s) {
  const DetLds D = det_lds(a.t, a.cell);
  hipLaunchKernelGGL(k_detect, dim3(grid), dim3(256), D.bytes, s, a);
  return hipGetLastError();
}

hipError_t launch_select_orient(const KArgs& a, int slots, hipStream_t s) {
  hipLaunchKernelGGL(k_select_orient, dim3(cdiv(slots, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_select(const KArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(grid), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_orient(const KArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_orient, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_test_segment(const uint8_t* circles, int n, int t_lo, int t_hi, uint8_t* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_test_segment, dim3(cdiv(n, 256)), dim3(256), 0, s, circles, n, t_lo, t_hi,
                     out);
  return hipGetLastError();
}

}  // namespace ofk
