// of_plan.h -- launch plan shared by the host library and the gfx950 kernels.
//
// The same __host__ __device__ functions size the workspace on the host and fill the
// per-(frame, level) plan on the device, so both sides agree on every offset.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/of.h"

#define OF_HD __host__ __device__ inline

namespace ofk {

constexpr int kMaxLevels = OF_MAX_LEVELS;
constexpr int kMaxBatch = OF_MAX_BATCH;
constexpr int kMaxEntries = kMaxLevels * kMaxBatch;  // (frame, level) pairs per call
constexpr int kMaxQuota = 4096;                      // keypoints per level
constexpr int kSortCap = 4096;                       // candidates sorted in LDS at once
constexpr int kMaxDetW = 256, kMaxDetH = 128;        // Harris/NMS tile limits (pixels)
constexpr int kCandCache = 1024;                     // Harris scores cached per tile
constexpr int kMarkCellFlags = 320;  // cells a segment-test tile meets (cell >= 8: 33 x 9)
constexpr int kRankCap = 16384;                      // levels ranked by counting, not radix
constexpr int kSelLdsCap = 2560;                     // level R' staged in LDS for ranking
static_assert(kSelLdsCap % 256 == 0 && kSortCap % 256 == 0, "staged copies padded to 256");
constexpr uint32_t kNoPos = 0xffffffffu;              // position of an empty candidate slot
// Per-level counters that many tiles add to are split into kCountSpread sub-counters in
// separate 128-byte lines (a tile adds to sub-counter blockIdx mod kCountSpread; readers
// sum them): device-wide atomics on one address are serialised where they are
// performed, and the last of them hold the launch's completion.
constexpr int kCountSpread = 16;

struct Tune {
  int32_t mark_words, mark_rows;
  int32_t det_cx, det_cy, det_w, det_h;
  int32_t mark_grid, det_grid;
  int32_t pyr_pass;  // 1: levels are resampled by a separate pass before the segment test
  int32_t mark_order;  // 1: segment-test tiles in XCD bands (block b on XCD b % 8)
  int32_t plan_resident;  // 1: skip the prologue when this workspace holds this plan
  int32_t det_order;  // 1: Harris/NMS tiles in the segment test's XCD bands
  // Largest candidate count of a level that the selection ranks by counting (at most
  // kRankCap); larger levels take the radix select.  Set per call from its size: counting
  // costs C^2 per level but runs every slot's wave at once (shortest for a few frames),
  // the radix select costs a few passes over C in one block per level.
  int32_t rank_cap;
};

constexpr int kXcds = 8;  // blocks are dispatched to the XCDs round-robin by block index

// First tile row of band k when a level's mark_ty tile rows are split over the XCDs.
// Every band takes mark_ty / 8 consecutive rows; the mark_ty % 8 rows left over go one
// each to bands rot, rot + 1, ... (mod 8).  rot carries on from entry to entry (the sum
// of the leftovers of the entries before, mod 8), so the leftovers of a batch of levels
// spread over all XCDs instead of piling onto the same few.
OF_HD int32_t band_row0(int32_t mark_ty, int32_t rot, int32_t k) {
  const int32_t q = mark_ty / kXcds, r = mark_ty % kXcds, hi = rot + r;
  int32_t c = k - rot < 0 ? 0 : (k - rot < r ? k - rot : r);  // bands rot .. min(hi, 8) - 1
  if (hi > kXcds) c += k < hi - kXcds ? k : hi - kXcds;      // wrapped: bands 0 .. hi - 9
  return q * k + c;
}

OF_HD int32_t band_rows(int32_t mark_ty, int32_t rot, int32_t k) {
  return band_row0(mark_ty, rot, k + 1) - band_row0(mark_ty, rot, k);
}

// Division of small non-negative numerators by a divisor fixed for a whole tile:
// q = n / d as a multiply-high by m = ceil(2^32 / d) (the low 32 bits of it; d = 1, whose
// m is 2^32, adds n itself).  Exact for n * d < 2^32, which every use here satisfies
// (numerators and divisors below 2^16).
struct FastDiv {
  uint32_t mlo, one;  // one = 0xffffffff when d == 1
};

OF_HD FastDiv fast_div(uint32_t d) {
  const uint64_t m = ((1ull << 32) + d - 1) / d;
  FastDiv f;
  f.mlo = (uint32_t)m;
  f.one = d == 1 ? 0xffffffffu : 0u;
  return f;
}

OF_HD uint32_t div_by(uint32_t n, const FastDiv& f) {
#ifdef __HIP_DEVICE_COMPILE__
  return __umulhi(n, f.mlo) + (n & f.one);
#else
  return (uint32_t)(((uint64_t)n * f.mlo) >> 32) + (n & f.one);
#endif
}

// One ranked candidate: R' and (y << 16 | x) in level coordinates.
struct Cand {
  int64_t score;
  uint32_t pos;
  uint32_t pad;
};

// Everything a kernel needs about one (frame, level) pair.  Written by the prologue.
struct LevelPlan {
  int32_t W, H, B, level, frame, n_levels;
  int32_t cs, ncx, ncy;        // cell side (whole level when cell == 0) and cell grid
  FastDiv csd;                 // division by cs
  int32_t quota, kcell;
  int32_t fast_t, fast_t_min;
  const uint8_t* base;         // input frame
  int32_t base_w, base_h, base_stride;
  const uint8_t* lvl;          // level pixels (the input frame for level 0)
  uint8_t* lvl_w;              // writable level buffer (nullptr for level 0)
  int32_t lvl_stride;
  uint32_t* bm_lo;             // segment-test bitmaps: bit x of row y in 32-bit words,
  uint32_t* bm_hi;             //   wpr words per row; lo = corner at fast_t_min
  int32_t wpr;
  uint8_t* flags;              // ncx * ncy bytes: 1 = cell holds a fast_t corner
  Cand* cand;                  // candidate slots written by the Harris/NMS tiles
  uint32_t* cand_count;        // filled slots: sub-counter 0 (count_stride apart)
  int32_t cand_cap;            // slots (filled or holding the kNoPos sentinel)
  int32_t kslot;               // slots per cell (cell > 0)
  int32_t compact;             // 1: no fixed slots; tiles append (level past kRankCap, cell 0)
  Cand* sel;                   // level selection, sorted, quota entries
  uint32_t* sel_count;
  uint32_t* ncand_count;       // FAST candidates of the level (statistics), sub-counter 0
  int32_t count_stride;        // words between sub-counters
  int32_t mark_tx, mark_ty;    // segment-test tile grid (covers the whole level)
  int32_t band_rot;            // first band that takes one of the leftover tile rows
  int32_t det_band_rot;        // the same for the Harris/NMS tile rows
  int32_t det_tx, det_ty;      // Harris/NMS tile grid (covers the valid region)
  int32_t det_x0, det_y0;      // first cell column/row (cell > 0) or first pixel (cell == 0)
  int32_t det_xend, det_yend;  // one past the last cell column/row, or W-B / H-B
  int32_t slot_w;              // output slots per row of 2x2 blocks (no cells)
  int32_t entry0;              // plan index of this frame's level 0
  of_keypoint* out;            // this frame's output
  int32_t* count_out;
};

// ------------------------------------------------------------------ geometry --

OF_HD int32_t cdiv(int32_t a, int32_t b) { return (a + b - 1) / b; }
OF_HD int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Counter region of a call with n entries: kCountSpread sub-counters of the filled slots
// and of the FAST candidates (one 128-byte-aligned array of n words each), then one
// selected count per entry.
OF_HD int32_t count_stride(int32_t n_entries) { return (int32_t)align_up(n_entries, 32); }
OF_HD int64_t counter_words(int32_t n_entries) {
  return 2 * (int64_t)kCountSpread * count_stride(n_entries) + n_entries;
}

// The same for the LDS layouts that every wave of a tile kernel computes at its start:
// non-negative 32-bit values, so unsigned arithmetic (a power-of-two divisor is a shift).
constexpr OF_HD int32_t align16(int32_t v) { return (int32_t)(((uint32_t)v + 15u) & ~15u); }
constexpr OF_HD int32_t cdiv_u(int32_t a, int32_t b) {
  return (int32_t)(((uint32_t)a + (uint32_t)b - 1u) / (uint32_t)b);
}

// Level size: round-half-up of n / s^l with s = num / den, exact in 64-bit integers.
OF_HD int32_t level_extent(int32_t n, int l, int32_t num, int32_t den) {
  int64_t a = 1, b = 1;
  for (int i = 0; i < l; ++i) {
    a *= num;
    b *= den;
  }
  return (int32_t)((2 * (int64_t)n * b + a) / (2 * a));
}

struct FrameGeom {
  int32_t L;
  int32_t W[kMaxLevels], H[kMaxLevels], quota[kMaxLevels], kcell[kMaxLevels];
  int32_t ncx[kMaxLevels], ncy[kMaxLevels], cs[kMaxLevels];
};

// Level sizes, quotas N_l (area-proportional, floor, level 0 takes the rest) and the
// per-cell keep count K_l = max(1, ceil(N_l / cells_l)).
OF_HD void frame_geom(int32_t W0, int32_t H0, const of_params& p, FrameGeom* g) {
  g->L = p.n_levels;
  int64_t area = 0;
  for (int l = 0; l < p.n_levels; ++l) {
    g->W[l] = level_extent(W0, l, p.scale_num, p.scale_den);
    g->H[l] = level_extent(H0, l, p.scale_num, p.scale_den);
    area += (int64_t)g->W[l] * g->H[l];
  }
  int32_t rest = p.n_features;
  for (int l = 1; l < p.n_levels; ++l) {
    g->quota[l] = (int32_t)(((int64_t)p.n_features * g->W[l] * g->H[l]) / area);
    rest -= g->quota[l];
  }
  g->quota[0] = rest;
  for (int l = 0; l < p.n_levels; ++l) {
    int32_t cs = p.cell > 0 ? p.cell : (g->W[l] > g->H[l] ? g->W[l] : g->H[l]);
    g->cs[l] = cs;
    g->ncx[l] = cdiv(g->W[l], cs);
    g->ncy[l] = cdiv(g->H[l], cs);
    int32_t nc = g->ncx[l] * g->ncy[l];
    int32_t k = (g->quota[l] + nc - 1) / nc;
    g->kcell[l] = k < 1 ? 1 : k;
  }
}

OF_HD int32_t level_stride(int32_t W) { return (int32_t)align_up(W, 64); }

// Sizes of one (frame, level) entry inside each workspace region.
struct EntrySize {
  int32_t mark_tiles, det_tiles;
  int64_t bm_words;   // 32-bit words of both bitmaps
  int64_t flag_bytes;
  int64_t cand_cap;
  int64_t sel_cap;
  int64_t lvl_bytes;
  // tile grids
  int32_t mark_tx, mark_ty, det_tx, det_ty, det_x0, det_y0, det_xend, det_yend, wpr;
  int32_t slot_w;       // slots per row of 2x2 blocks (no cells)
  int32_t kslot;        // slots per cell (cells): K_l capped by the survivors a cell holds
  int32_t pyr_blocks;   // 64 x 16 resample blocks of a level >= 1
  int32_t rank_slots;   // waves of the counting selection: the slots of a level it ranks,
                        // none past the rank cap (an appended list: up to the cap)
  int32_t sel_slots;    // waves of the second counting pass over a radix-selected list:
                        // N_l for a level that can take the radix path, else none
};

OF_HD void entry_size(const FrameGeom& g, const of_params& p, const Tune& t, int l,
                      EntrySize* s) {
  const int32_t W = g.W[l], H = g.H[l], B = p.patch_radius, cs = g.cs[l];
  s->mark_tx = cdiv(W, 64 * t.mark_words);
  s->mark_ty = cdiv(H, t.mark_rows);
  s->mark_tiles = s->mark_tx * s->mark_ty;
  s->wpr = 2 * cdiv(W, 64);
  s->bm_words = 2 * (int64_t)s->wpr * H;
  s->flag_bytes = align_up((int64_t)g.ncx[l] * g.ncy[l], 16);
  if (p.cell > 0) {
    s->det_x0 = B / cs;
    s->det_y0 = B / cs;
    s->det_xend = (W - 1 - B) / cs + 1;
    s->det_yend = (H - 1 - B) / cs + 1;
    s->det_tx = cdiv(s->det_xend - s->det_x0, t.det_cx);
    s->det_ty = cdiv(s->det_yend - s->det_y0, t.det_cy);
  } else {
    s->det_x0 = B;
    s->det_y0 = B;
    s->det_xend = W - B;
    s->det_yend = H - B;
    s->det_tx = cdiv(W - 2 * B, t.det_w);
    s->det_ty = cdiv(H - 2 * B, t.det_h);
  }
  // Output slots of the Harris/NMS tiles, fixed for any tiling so that no block needs
  // a returned atomic to place its results.  With cells: K_l slots per cell of the
  // valid region, cell-major.  Without cells: one slot per 2x2 block of the valid
  // region, which can hold at most one NMS survivor (all four pixels are neighbours).
  // NMS survivors are never neighbours, so a cs x cs cell holds at most ceil(cs/2)^2 of
  // them and K_l beyond that needs no slots.  Unused slots hold a sentinel that ranks
  // below every real candidate.
  {
    s->slot_w = cdiv(W - 2 * B, 2);
    const int64_t hc = cdiv(cs, 2);
    s->kslot = (int32_t)(g.kcell[l] < hc * hc ? g.kcell[l] : hc * hc);
    if (p.cell > 0) {
      const int64_t nvx = s->det_xend - s->det_x0, nvy = s->det_yend - s->det_y0;
      s->cand_cap = nvx * nvy * s->kslot;
    } else {
      s->cand_cap = (int64_t)s->slot_w * cdiv(H - 2 * B, 2);
    }
  }
  s->det_tiles = s->det_tx * s->det_ty;
  // Fixed slots are ranked by counting only up to the rank cap; an appended list (a
  // whole-level cell past kRankCap) has a length known only on the device, so it gets
  // the cap's waves and takes whichever path its length falls to.
  const bool appended = p.cell == 0 && s->cand_cap > kRankCap;
  s->rank_slots = appended ? t.rank_cap : (s->cand_cap <= t.rank_cap ? (int32_t)s->cand_cap : 0);
  s->sel_slots = appended || s->cand_cap > t.rank_cap ? g.quota[l] : 0;
  s->sel_cap = g.quota[l];
  s->lvl_bytes = l == 0 ? 0 : align_up((int64_t)level_stride(W) * H, 256);
  s->pyr_blocks = l == 0 ? 0 : cdiv(W, 64) * cdiv(H, 16);
}

// Candidates the level selection ranks for a level: its slots (fixed slots, empty ones
// holding the sentinel), or the survivors its tiles appended (a whole-level cell past the
// rank cap: a dense list of `filled` entries).  Levels with at most the call's rank cap
// (Tune::rank_cap) of them are ranked by counting (k_select_orient); the rest take the
// radix select.
OF_HD int32_t ranked_candidates(const LevelPlan& P, uint32_t filled) {
  return P.compact ? ((int64_t)filled < P.cand_cap ? (int32_t)filled : P.cand_cap) : P.cand_cap;
}

// ------------------------------------------------------------ workspace layout --

// Region sizes of a whole call; offsets are from the workspace base (256-aligned).
struct WsLayout {
  int64_t off_hdr, off_plan, off_mark_base, off_det_base, off_sel_base, off_rank_base;
  int64_t off_pyr_base;
  int64_t off_band_base;   // kXcds prefix tables of segment-test tiles per entry, by band
  int64_t off_det_band_base;  // the same for Harris/NMS tiles
  int64_t off_counters, off_flags, off_bm, off_cand, off_sel, off_lvl, total;
  int32_t n_entries, mark_tiles, det_tiles, sel_slots, rank_slots, max_cand_cap, pyr_blocks;
  int32_t band_tiles[kXcds];
  int32_t det_band_tiles[kXcds];
  int32_t band_rot;        // rotation of the next entry's leftover rows
  int32_t det_band_rot;    // the same for Harris/NMS tile rows
  int64_t flag_bytes, bm_words, cand_entries, sel_entries, lvl_bytes;
};

OF_HD void ws_layout_accumulate(WsLayout* w, const EntrySize& s) {
  w->n_entries += 1;
  w->mark_tiles += s.mark_tiles;
  w->det_tiles += s.det_tiles;
  w->sel_slots += s.sel_slots;
  w->pyr_blocks += s.pyr_blocks;
  for (int k = 0; k < kXcds; ++k) {
    w->band_tiles[k] += s.mark_tx * band_rows(s.mark_ty, w->band_rot, k);
    w->det_band_tiles[k] += s.det_tx * band_rows(s.det_ty, w->det_band_rot, k);
  }
  w->band_rot = (w->band_rot + s.mark_ty % kXcds) % kXcds;
  w->det_band_rot = (w->det_band_rot + s.det_ty % kXcds) % kXcds;
  w->flag_bytes += s.flag_bytes;
  w->bm_words += s.bm_words;
  w->cand_entries += s.cand_cap;
  w->rank_slots += s.rank_slots;
  if (s.cand_cap > w->max_cand_cap) w->max_cand_cap = (int32_t)s.cand_cap;
  w->sel_entries += s.sel_cap;
  w->lvl_bytes += s.lvl_bytes;
}

OF_HD void ws_layout_finish(WsLayout* w) {
  int64_t o = 0;
  w->off_hdr = o;          o += 256;  // queue counters [0, 128), plan signature at 128
  w->off_plan = o;         o = align_up(o + (int64_t)w->n_entries * sizeof(LevelPlan), 256);
  w->off_mark_base = o;    o = align_up(o + 4 * ((int64_t)w->n_entries + 1), 256);
  w->off_det_base = o;     o = align_up(o + 4 * ((int64_t)w->n_entries + 1), 256);
  w->off_sel_base = o;     o = align_up(o + 4 * ((int64_t)w->n_entries + 1), 256);
  w->off_rank_base = o;    o = align_up(o + 4 * ((int64_t)w->n_entries + 1), 256);
  w->off_pyr_base = o;     o = align_up(o + 4 * ((int64_t)w->n_entries + 1), 256);
  w->off_band_base = o;    o = align_up(o + 4 * kXcds * ((int64_t)w->n_entries + 1), 256);
  w->off_det_band_base = o;  o = align_up(o + 4 * kXcds * ((int64_t)w->n_entries + 1), 256);
  // counters: filled candidate slots and FAST candidates (spread), selected (radix path)
  w->off_counters = o;     o = align_up(o + 4 * counter_words(w->n_entries), 256);
  w->off_flags = o;        o = align_up(o + w->flag_bytes, 256);
  w->off_bm = o;           o = align_up(o + 4 * w->bm_words, 256);
  w->off_cand = o;         o = align_up(o + (int64_t)sizeof(Cand) * w->cand_entries, 256);
  w->off_sel = o;          o = align_up(o + (int64_t)sizeof(Cand) * w->sel_entries, 256);
  w->off_lvl = o;          o = align_up(o + w->lvl_bytes, 256);
  w->total = o;
}

// ------------------------------------------------------------------ resample --

// Source tap of output coordinate i on an axis of n_src -> n_dst pixels: pixel centres
// aligned, position ((2i+1) n_src - n_dst) / (2 n_dst); returns the integer part in the
// high bits and the Q8 weight (fraction * 256 rounded half to even, 0..256) in the low 9.
OF_HD uint32_t resample_tap(int32_t i, int32_t n_src, int32_t n_dst) {
  int32_t num = (2 * i + 1) * n_src - n_dst;
  int32_t den = 2 * n_dst;
  int32_t i0 = num / den;
  int32_t r = num - i0 * den;
  int32_t a = 256 * r;
  int32_t q = a / den;
  int32_t rr = a - q * den;
  if (2 * rr > den || (2 * rr == den && (q & 1))) ++q;
  return ((uint32_t)i0 << 9) | (uint32_t)q;
}


// The same tap with both divisions by den = 2 n_dst done as a multiply by rden, the double
// nearest 1 / den, and one correction step.  Exact: num / den < 2^25 and num * rden is
// within 2^-27 of num / den, while a non-integer num / den sits at least 1 / den >= 2^-16
// from the next integer, so the truncated product is the floor or (num / den an integer)
// one less, which the remainder test fixes; the same holds for 256 r / den < 256.
OF_HD uint32_t resample_tap_r(int32_t i, int32_t n_src, int32_t n_dst, double rden) {
  const int32_t num = (2 * i + 1) * n_src - n_dst;
  const int32_t den = 2 * n_dst;
  int32_t i0 = (int32_t)((double)num * rden);
  int32_t r = num - i0 * den;
  if (r >= den) {
    ++i0;
    r -= den;
  }
  const int32_t a = 256 * r;
  int32_t q = (int32_t)((double)a * rden);
  int32_t rr = a - q * den;
  if (rr >= den) {
    ++q;
    rr -= den;
  }
  if (2 * rr > den || (2 * rr == den && (q & 1))) ++q;
  return ((uint32_t)i0 << 9) | (uint32_t)q;
}

// ------------------------------------------------------------- tile geometry --

// Whether columns [x0, x1) of a row (x0 a multiple of 4) are staged in whole 16-byte
// chunks: when the last chunk ends inside the row's readable bytes (row_limit) and
// inside an LDS row of lp bytes; otherwise the staging goes word by word.
OF_HD bool stage_wide(int32_t x0, int32_t x1, int32_t row_limit, int32_t lp) {
  const int32_t span = 16 * ((x1 - x0 + 15) >> 4);
  return x0 + span <= row_limit && span <= lp;
}
// The same functions place every tile in the kernels and in the CPU launch model of the
// tests, so both check one arithmetic.

// Tile (in the launch's numbering) that block or queue draw g0 takes, or -1 when it
// takes none.  In the band order block b takes the (b / kXcds)-th tile of band
// b % kXcds, which holds band_tiles; a grid the device holds at once runs its tiles last
// first (rev).
OF_HD int32_t launch_tile(int32_t g0, int32_t total, int32_t bands, int32_t band_tiles,
                          int32_t rev) {
  if (g0 >= total) return -1;
  const int32_t gb = bands ? g0 / kXcds : g0;
  const int32_t ng = bands ? band_tiles : total;
  if (gb >= ng) return -1;
  return rev ? ng - 1 - gb : gb;
}

// Last index e < n with base[e] <= g, for a non-decreasing exclusive prefix base.
OF_HD int32_t prefix_entry(const int32_t* base, int32_t n, int32_t g) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (base[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Segment-test tile (tx, ty) of a W x H level: the tile's pixels [x_t0, x_t1) x
// [y_t0, y_t1) and the staged region [ox, ex) x [oy, ey) with its 3-pixel halo (ox a
// multiple of 4, one pixel more on the left).
struct MarkTile {
  int32_t x_t0, x_t1, y_t0, y_t1, ox, oy, ex, ey;
};

OF_HD MarkTile mark_tile(int32_t W, int32_t H, int32_t tw, int32_t th, int32_t tx, int32_t ty) {
  MarkTile m;
  m.x_t0 = tx * tw;
  m.x_t1 = m.x_t0 + tw < W ? m.x_t0 + tw : W;
  m.y_t0 = ty * th;
  m.y_t1 = m.y_t0 + th < H ? m.y_t0 + th : H;
  m.ox = m.x_t0 - 4 > 0 ? m.x_t0 - 4 : 0;
  m.oy = m.y_t0 - 3 > 0 ? m.y_t0 - 3 : 0;
  m.ex = m.x_t1 + 3 < W ? m.x_t1 + 3 : W;
  m.ey = m.y_t1 + 3 < H ? m.y_t1 + 3 : H;
  return m;
}

// Harris/NMS tile (tx, ty) of a level: its valid pixels [vx0, vx1) x [vy0, vy1) (whole
// cells cxa.. / cya.. when there are cells), the 1-pixel ring of candidates around them
// (origin rx0, ry0, size rw x rh), the staged pixels [sx0, sx1) x [sy0, sy1) (5-pixel
// halo, sx0 a multiple of 4), the bitmap words that hold ring columns (bw0, nbw per
// ring row, nunits in all) and the cell flags of the ring (fcx0, fcy0, nfx x nfy).
struct DetTile {
  int32_t vx0, vx1, vy0, vy1, cxa, cya, nlcx, nlcy;
  int32_t rx0, ry0, rw, rh, sx0, sy0, sx1, sy1;
  int32_t bw0, nbw, nunits, fcx0, fcy0, nfx, nfy;
};

OF_HD DetTile det_tile(const LevelPlan& P, const Tune& t, int32_t cell, int32_t tx, int32_t ty) {
  DetTile d;
  const int32_t W = P.W, H = P.H, B = P.B, cs = P.cs;
  d.cxa = d.cya = 0;
  d.nlcx = d.nlcy = 1;
  if (cell > 0) {
    d.cxa = P.det_x0 + tx * t.det_cx;
    d.cya = P.det_y0 + ty * t.det_cy;
    const int32_t cxb = d.cxa + t.det_cx < P.det_xend ? d.cxa + t.det_cx : P.det_xend;
    const int32_t cyb = d.cya + t.det_cy < P.det_yend ? d.cya + t.det_cy : P.det_yend;
    d.nlcx = cxb - d.cxa;
    d.nlcy = cyb - d.cya;
    d.vx0 = d.cxa * cs > B ? d.cxa * cs : B;
    d.vx1 = cxb * cs < W - B ? cxb * cs : W - B;
    d.vy0 = d.cya * cs > B ? d.cya * cs : B;
    d.vy1 = cyb * cs < H - B ? cyb * cs : H - B;
  } else {
    d.vx0 = P.det_x0 + tx * t.det_w;
    d.vx1 = d.vx0 + t.det_w < P.det_xend ? d.vx0 + t.det_w : P.det_xend;
    d.vy0 = P.det_y0 + ty * t.det_h;
    d.vy1 = d.vy0 + t.det_h < P.det_yend ? d.vy0 + t.det_h : P.det_yend;
  }
  d.rx0 = d.vx0 - 1;
  d.ry0 = d.vy0 - 1;
  d.rw = d.vx1 - d.vx0 + 2;
  d.rh = d.vy1 - d.vy0 + 2;
  d.sx0 = (d.vx0 - 5 > 0 ? d.vx0 - 5 : 0) & ~3;
  d.sy0 = d.vy0 - 5 > 0 ? d.vy0 - 5 : 0;
  d.sx1 = d.vx1 + 5 < W ? d.vx1 + 5 : W;
  d.sy1 = d.vy1 + 5 < H ? d.vy1 + 5 : H;
  d.bw0 = d.rx0 >> 5;
  d.nbw = ((d.rx0 + d.rw - 1) >> 5) - d.bw0 + 1;
  d.nunits = d.rh * d.nbw;
  d.fcx0 = d.rx0 / cs;
  d.fcy0 = d.ry0 / cs;
  d.nfx = (d.rx0 + d.rw - 1) / cs - d.fcx0 + 1;
  d.nfy = (d.ry0 + d.rh - 1) / cs - d.fcy0 + 1;
  return d;
}

// ------------------------------------------------------------- LDS layouts --

// LDS of the entry base table that tile kernels keep after their own layout.
OF_HD int32_t base_table_bytes(int32_t n_entries) {
  return (int32_t)align_up(4 * ((int64_t)n_entries + 1), 16);
}

// Segment-test tile: pixels (tile + 3-pixel halo, 4-aligned origin), the queue of
// pixels that pass the compass pre-test and both bitmaps.
struct MarkLds {
  int32_t tw, th, pitch, rows, qseg;
  int32_t off_queue, off_bml, off_bmh, bytes;
  int32_t tcols;  // resample taps of the tile's columns (in the queue's region, before its use)
};

OF_HD MarkLds mark_lds(const Tune& t) {
  MarkLds m;
  m.tw = 64 * t.mark_words;
  m.th = t.mark_rows;
  m.pitch = m.tw + 16;  // the staged width (tw + 7) rounded up to 16-byte chunks
  m.rows = m.th + 6;
  int32_t o = align16(m.pitch * m.rows);
  // four per-wave queue segments: wave w tests tile rows w, w + 4, ..., at most
  // ceil(rows / 4) of them, and each row appends at most 64 * mark_words pixels
  m.qseg = 64 * t.mark_words * cdiv_u(m.th, 4);
  // the same region holds the resample taps while the tile is resampled: per column
  // x0 and (256 - wx, wx), per row two source row offsets and (256 - wy, wy)
  m.tcols = m.tw + 7;
  const int32_t taps = 4 * (2 * m.tcols + 3 * m.rows);
  m.off_queue = o;  o += align16(2 * 4 * m.qseg > taps ? 2 * 4 * m.qseg : taps);
  m.off_bml = o;    o += 4 * m.th * 2 * t.mark_words;
  m.off_bmh = o;    o += 4 * m.th * 2 * t.mark_words;
  m.bytes = align16(o);
  return m;
}

// Harris/NMS tile: staged pixels (tile + 5-pixel halo), 32-bit candidate words of the
// tile plus a 1-pixel ring and their prefix counts, the Harris score cache, survivors
// (candidate index; cell only when the tile holds several), the cell-grouped survivor list (or 2x2 block flags when the
// level is one cell), per-cell counters and the cell flags of the ring.
struct DetLds {
  int32_t mtw, mth;          // largest tile (pixels)
  int32_t pitch, rows;       // staged pixels
  int32_t nbw, nunits;       // candidate words per ring row (at most), total words
  int32_t max_surv, max_cells;
  int32_t off_cw, off_ucnt, off_cpre, off_crs, off_cpos, off_sci, off_scell, off_order, off_ccnt,
      off_coff, off_cfill, off_ckept, off_cbest, off_cwin, off_lfl, fm_rows, off_fm, bytes;
};

// The tuning fields of a Harris/NMS tile shape known at compile time: a x b cells
// (cell > 0) or a x b pixels (whole-level cells, cell == 0); the rest zero.
constexpr OF_HD Tune det_shape_tune(int32_t a, int32_t b, int32_t cell) {
  Tune t{};
  if (cell > 0) {
    t.det_cx = a;
    t.det_cy = b;
  } else {
    t.det_w = a;
    t.det_h = b;
  }
  return t;
}

constexpr OF_HD DetLds det_lds(const Tune& t, int32_t cell) {
  DetLds d{};
  if (cell > 0) {
    d.mtw = t.det_cx * cell;
    d.mth = t.det_cy * cell;
    d.max_cells = t.det_cx * t.det_cy;
  } else {
    d.mtw = t.det_w;
    d.mth = t.det_h;
    d.max_cells = 1;
  }
  // The staged width (at most mtw + 13 bytes) rounded up to 16-byte chunks, plus one word:
  // an odd number of 32-bit words per row, so the rows of a Harris window fall in
  // distinct banks, and room for whole chunks (stage_wide).
  d.pitch = (int32_t)(((uint32_t)d.mtw + 13u + 15u) & ~15u) + 4;
  d.rows = d.mth + 10;
  d.nbw = cdiv_u(d.mtw + 2, 32) + 1;
  d.nunits = (d.mth + 2) * d.nbw;
  d.max_surv = cdiv_u(d.mtw, 2) * cdiv_u(d.mth, 2);
  int32_t o = align16(d.pitch * d.rows);
  d.off_cw = o;     o += align16(4 * d.nunits);
  d.off_ucnt = o;   o += align16(4 * d.nunits);
  d.off_cpre = o;   o += align16(4 * (d.nunits + 1));
  d.off_crs = o;    o += 8 * kCandCache;
  d.off_cpos = o;   o += 4 * kCandCache;
  d.off_sci = o;    o += align16(2 * d.max_surv);
  d.off_scell = o;  o += d.max_cells > 1 ? align16(2 * d.max_surv) : 0;
  d.off_order = o;  o += align16(2 * d.max_surv);
  d.off_ccnt = o;   o += align16(4 * d.max_cells);
  d.off_coff = o;   o += align16(4 * d.max_cells);
  d.off_cfill = o;  o += align16(4 * d.max_cells);
  d.off_ckept = o;  o += align16(4 * d.max_cells);
  d.off_cbest = o;  o += align16(8 * d.max_cells);   // K = 1: best R' per cell
  d.off_cwin = o;   o += align16(4 * d.max_cells);   // K = 1: its position
  const int32_t nfl = cell > 0 ? (t.det_cx + 2) * (t.det_cy + 2) : 4;  // cells of the ring
  d.off_lfl = o;    o += align16(nfl);
  d.fm_rows = cell > 0 ? t.det_cy + 2 : 4;  // flag rows of the ring
  d.off_fm = o;     o += 8 * d.fm_rows * d.nbw;  // candidate-word masks (hi, lo)
  d.bytes = o;      // + the entry base table of the launch
  return d;
}


}  // namespace ofk
