// launch_model.cpp -- CPU model of every kernel launch the C ABI issues.
//
// The library's own host code (of_api.cpp: validation, workspace layout, launch
// sequencing) is linked here against a model of the gfx950 kernels instead of the
// kernels themselves.  Each modelled launch walks every block (and, for persistent
// grids, every queue draw) of the launch with the kernels' own placement arithmetic
// (of_plan.h / of_kernels.h, shared with the device code), and checks:
//   * every global read and write falls inside one caller buffer, and no kernel but the
//     prologue writes the plan, its prefix tables or the band tables;
//   * every LDS access falls inside its region of the kernel's LDS layout, including the
//     worst case of data-dependent lists (pre-test queues, candidates, survivors);
//   * every tile of every (frame, level) is taken exactly once per launch;
//   * the state a call leaves for the next (counters, cell flags, queue counters) is
//     zero where the next call expects it.
// Data values are not computed: where an access depends on data, the model checks the
// extremes the data can reach (e.g. candidates anywhere in the valid region).
//
// Usage: launch_model <scenario>...   Prints one line per violation and a summary.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "../../paper_2506_07164_amd/csrc/of_kernels.h"

using namespace ofk;

// ------------------------------------------------------------------ reporting --

static int g_fail = 0;
static long g_checks = 0;
static std::string g_case;

static void fail(const char* fmt, ...) {
  static std::map<std::string, int> seen;  // one line per distinct message
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  const std::string key = g_case + "|" + fmt;
  if (seen[key]++ < 3 && g_fail < 200) printf("FAIL [%s] %s\n", g_case.c_str(), buf);
  ++g_fail;
}

#define CHECK(cond, ...)  \
  do {                    \
    ++g_checks;           \
    if (!(cond)) fail(__VA_ARGS__); \
  } while (0)

// ----------------------------------------------------------- device memory --

// Every "device" buffer is a host allocation registered here; accesses must stay inside
// one of them.  The plan area of a workspace is write-protected outside the prologue.
struct Region {
  const uint8_t* base;
  size_t size;
  std::string name;
};
static std::vector<Region> g_regions;
static std::vector<std::pair<const uint8_t*, size_t>> g_protected;
static bool g_in_prologue = false;

static void* dev_alloc(size_t n, const std::string& name) {
  uint8_t* p = (uint8_t*)malloc(n ? n : 1);
  memset(p, 0, n);
  g_regions.push_back({p, n, name});
  return p;
}

static void dev_free(void* p) {
  size_t size = 0;
  for (size_t i = 0; i < g_regions.size(); ++i)
    if (g_regions[i].base == p) {
      size = g_regions[i].size;
      g_regions.erase(g_regions.begin() + i);
      break;
    }
  g_protected.erase(std::remove_if(g_protected.begin(), g_protected.end(),
                                   [&](const std::pair<const uint8_t*, size_t>& r) {
                                     return r.first >= (const uint8_t*)p &&
                                            r.first < (const uint8_t*)p + size;
                                   }),
                    g_protected.end());
  free(p);
}

static void acc(const void* p, int64_t n, const char* what, bool write = false) {
  ++g_checks;
  if (n <= 0) return;
  const uint8_t* q = (const uint8_t*)p;
  const Region* r = nullptr;
  for (const Region& x : g_regions)
    if (q >= x.base && q + n <= x.base + x.size) {
      r = &x;
      break;
    }
  if (!r) {
    fail("%s: %s of %lld bytes at %p is outside every buffer", what, write ? "write" : "read",
         (long long)n, p);
    return;
  }
  if (write && !g_in_prologue)
    for (auto& pr : g_protected)
      if (q < pr.first + pr.second && q + n > pr.first)
        fail("%s: write into a workspace's plan tables", what);
  // touch the bytes (AddressSanitizer sees the host buffers)
  volatile uint8_t s = q[0];
  s = q[n - 1];
  (void)s;
}

// LDS of one block: [0, bytes); region checks are explicit.
static void lds(int64_t off, int64_t n, int64_t lo, int64_t hi, const char* what) {
  ++g_checks;
  if (n <= 0) return;
  if (off < lo || off + n > hi)
    fail("%s: LDS [%lld, %lld) outside its region [%lld, %lld)", what, (long long)off,
         (long long)(off + n), (long long)lo, (long long)hi);
}

// ------------------------------------------------------------ model state --

// Per workspace: what each call leaves behind for the next.
struct WsState {
  std::vector<bool> flags_dirty;  // per entry: cell flags written since the last clear
  bool counters_dirty = false;    // counters written since the last clear
};
static std::map<const uint8_t*, WsState> g_ws;

static uint8_t* ws_of(const KArgs& a) { return (uint8_t*)a.plan - 0; }

// The workspace base of a launch, from the header the plan follows.
static uint8_t* ws_base(const KArgs& a) { return (uint8_t*)a.qctr; }

static const LevelPlan& plan(const KArgs& a, int e) {
  acc(a.plan + e, sizeof(LevelPlan), "plan read");
  return a.plan[e];
}

static bool sig_ok(const KArgs& a) {
  acc(a.ws_sig, 8, "signature read");
  return *a.ws_sig == a.sig;
}

// Entry of unit g in the launch's prefix table (small table in the arguments, or the
// table in the workspace), as the kernels find it.
static void entry_of(const KArgs& a, const int32_t* table, int row, int g, int* e, int* st,
                     int* en) {
  if (a.small) {
    const int32_t* b = a.sbase + row * (kSmallEntries + 1);
    int ee = 0, s0 = 0, end = b[kSmallEntries];
    for (int i = 1; i < kSmallEntries; ++i) {
      if (g >= b[i]) {
        ee = i;
        s0 = b[i];
      } else {
        end = std::min(end, b[i]);
      }
    }
    *e = ee;
    *st = s0;
    *en = end;
  } else {
    acc(table, 4 * ((int64_t)a.n_entries + 1), "prefix table read");
    *e = prefix_entry(table, a.n_entries, g);
    *st = table[*e];
    *en = table[*e + 1];
  }
  CHECK(*e >= 0 && *e < a.n_entries, "unit %d maps to entry %d of %d", g, *e, a.n_entries);
}

static int32_t table_total(const KArgs& a, const int32_t* table, int row) {
  if (a.small) return a.sbase[row * (kSmallEntries + 1) + kSmallEntries];
  acc(table + a.n_entries, 4, "prefix total read");
  return table[a.n_entries];
}

// ------------------------------------------------------------------ prologue --

namespace ofk {

static std::map<const uint8_t*, WsLayout> g_layouts;  // workspace -> layout of its plan

hipError_t launch_prologue(const PrologueArgs& a, int grid, hipStream_t) {
  uint8_t* ws = a.ws;
  const WsLayout& lay = a.lay;
  CHECK(grid >= 1 && grid <= 64, "prologue grid %d", grid);
  acc(ws, lay.total, "workspace (whole layout)");
  uint32_t* counters = (uint32_t*)(ws + lay.off_counters);
  uint32_t* qctr = (uint32_t*)(ws + lay.off_hdr);
  uint64_t* sig = (uint64_t*)(ws + lay.off_hdr + 128);
  g_in_prologue = true;
  acc(counters, 4 * counter_words(lay.n_entries), "counters zeroed", true);
  memset(counters, 0, 4 * (size_t)counter_words(lay.n_entries));
  acc(ws + lay.off_flags, lay.flag_bytes / 16 * 16, "flags zeroed", true);
  acc(qctr, 128, "queue counters zeroed", true);
  memset(qctr, 0, 128);
  WsState& st = g_ws[ws];
  st.flags_dirty.assign(lay.n_entries, false);
  st.counters_dirty = false;
  acc(sig, 8, "signature read");
  if (*sig != a.sig) {
    const int L = a.p.n_levels, nL = a.n * L;
    CHECK(nL == lay.n_entries && nL <= 1024, "entries %d vs layout %d", nL, lay.n_entries);
    LevelPlan* pl = (LevelPlan*)(ws + lay.off_plan);
    int32_t* mark_base = (int32_t*)(ws + lay.off_mark_base);
    int32_t* det_base = (int32_t*)(ws + lay.off_det_base);
    int32_t* sl_base = (int32_t*)(ws + lay.off_sel_base);
    int32_t* rank_base = (int32_t*)(ws + lay.off_rank_base);
    int32_t* pyr_base = (int32_t*)(ws + lay.off_pyr_base);
    int32_t* band_base = (int32_t*)(ws + lay.off_band_base);
    int32_t* det_band_base = (int32_t*)(ws + lay.off_det_band_base);
    int64_t o_mark = 0, o_det = 0, o_sl = 0, o_flag = 0, o_bm = 0, o_cand = 0, o_rank = 0,
            o_sel = 0, o_lvl = 0, o_pyr = 0, rot = 0, drot = 0;
    int64_t o_band[kXcds] = {}, o_dband[kXcds] = {};
    for (int i = 0; i < nL; ++i) {
      const int f = i / L, l = i - f * L;
      FrameGeom g;
      EntrySize s = {};
      frame_geom(a.f[f].w, a.f[f].h, a.p, &g);
      entry_size(g, a.p, a.t, l, &s);
      LevelPlan P;
      const EntryOffsets eo = {o_flag, o_bm, o_cand, o_sel, o_lvl, (int32_t)rot, (int32_t)drot,
                               counters};
      fill_level_plan(P, a, ws, g, s, i, f, l, eo);
      acc(pl + i, sizeof(LevelPlan), "plan write", true);
      pl[i] = P;
      acc(mark_base + i, 4, "prefix write", true);
      mark_base[i] = (int32_t)o_mark;
      det_base[i] = (int32_t)o_det;
      sl_base[i] = (int32_t)o_sl;
      rank_base[i] = (int32_t)o_rank;
      pyr_base[i] = (int32_t)o_pyr;
      for (int k = 0; k < kXcds; ++k) {
        band_base[k * (nL + 1) + i] = (int32_t)o_band[k];
        det_band_base[k * (nL + 1) + i] = (int32_t)o_dband[k];
        o_band[k] += (int64_t)s.mark_tx * band_rows(s.mark_ty, (int32_t)rot, k);
        o_dband[k] += (int64_t)s.det_tx * band_rows(s.det_ty, (int32_t)drot, k);
      }
      o_mark += s.mark_tiles;
      o_det += s.det_tiles;
      o_sl += s.sel_slots;
      o_flag += s.flag_bytes;
      o_bm += s.bm_words;
      o_cand += s.cand_cap;
      o_rank += s.rank_slots;
      o_sel += s.sel_cap;
      o_lvl += s.lvl_bytes;
      o_pyr += s.pyr_blocks;
      rot = (rot + s.mark_ty % kXcds) % kXcds;
      drot = (drot + s.det_ty % kXcds) % kXcds;
      // every region of the entry inside the workspace
      if (P.lvl_w) acc(P.lvl_w, (int64_t)P.lvl_stride * P.H, "level buffer (layout)");
      acc(P.bm_lo, 4 * (int64_t)s.bm_words, "bitmaps (layout)");
      acc(P.flags, (int64_t)P.ncx * P.ncy, "cell flags (layout)");
      acc(P.cand, (int64_t)sizeof(Cand) * P.cand_cap, "candidate slots (layout)");
      acc(P.sel, (int64_t)sizeof(Cand) * s.sel_cap, "selection (layout)");
    }
    mark_base[nL] = (int32_t)o_mark;
    det_base[nL] = (int32_t)o_det;
    sl_base[nL] = (int32_t)o_sl;
    rank_base[nL] = (int32_t)o_rank;
    pyr_base[nL] = (int32_t)o_pyr;
    for (int k = 0; k < kXcds; ++k) {
      band_base[k * (nL + 1) + nL] = (int32_t)o_band[k];
      det_band_base[k * (nL + 1) + nL] = (int32_t)o_dband[k];
      CHECK(o_band[k] == lay.band_tiles[k], "band %d: %lld tiles vs host %d", k,
            (long long)o_band[k], lay.band_tiles[k]);
      CHECK(o_dband[k] == lay.det_band_tiles[k], "Harris band %d: %lld tiles vs host %d", k,
            (long long)o_dband[k], lay.det_band_tiles[k]);
    }
    CHECK(o_mark == lay.mark_tiles && o_det == lay.det_tiles && o_sl == lay.sel_slots &&
              o_rank == lay.rank_slots && o_pyr == lay.pyr_blocks,
          "prologue totals differ from the host layout");
    CHECK(o_flag == lay.flag_bytes && o_bm == lay.bm_words && o_cand == lay.cand_entries &&
              o_sel == lay.sel_entries && o_lvl == lay.lvl_bytes,
          "prologue region sizes differ from the host layout");
    *sig = a.sig;
  }
  g_in_prologue = false;
  g_layouts[ws] = lay;
  // the plan area is written by the prologue only
  g_protected.erase(std::remove_if(g_protected.begin(), g_protected.end(),
                                   [&](const std::pair<const uint8_t*, size_t>& p) {
                                     return p.first >= ws && p.first < ws + lay.total;
                                   }),
                    g_protected.end());
  g_protected.push_back({ws + lay.off_plan, (size_t)(lay.off_counters - lay.off_plan)});
  g_protected.push_back({ws + lay.off_hdr + 128, 8});
  return hipSuccess;
}

// ----------------------------------------------------------------- pyramid --

static void model_resample(const uint8_t* src, int sw, int sh, int sstride, uint8_t* dst, int w,
                           int h, int stride, int bx, int by, const char* what) {
  // block of 64 x 16 output pixels; taps are monotone, so the corners bound every read
  const int x1 = std::min(bx + 64, w) - 1, y1 = std::min(by + 16, h) - 1;
  for (int x : {bx, x1})
    for (int y : {by, y1}) {
      const uint32_t tx = resample_tap(x, sw, w), ty = resample_tap(y, sh, h);
      const int x0 = tx >> 9, y0 = ty >> 9;
      CHECK(x0 >= 0 && x0 < sw && y0 >= 0 && y0 < sh, "%s: tap (%d,%d) outside the source", what,
            x0, y0);
      const int xx = std::min(x0 + 1, sw - 1), yy = std::min(y0 + 1, sh - 1);
      acc(src + (size_t)y0 * sstride + x0, 1, what);
      acc(src + (size_t)yy * sstride + xx, 1, what);
      acc(dst + (size_t)y * stride + x, 1, what, true);
    }
}

hipError_t launch_pyramid(const PyrArgs& a, int n_levels, int max_w, int max_h, hipStream_t) {
  for (int z = 0; z < n_levels; ++z) {
    const PyrLevel& L = a.lv[z];
    for (int by = 0; by < cdiv(max_h, 16) * 16; by += 16)
      for (int bx = 0; bx < cdiv(max_w, 64) * 64; bx += 64) {
        if (bx >= L.w || by >= L.h) continue;
        model_resample(a.src, a.src_w, a.src_h, a.src_stride, L.dst, L.w, L.h, L.stride, bx, by,
                       "k_pyramid");
      }
  }
  return hipSuccess;
}

hipError_t launch_pyramid_batch(const KArgs& a, int blocks, hipStream_t) {
  if (!sig_ok(a)) return hipSuccess;
  std::vector<int> seen;
  for (int g = 0; g < blocks; ++g) {
    int e, st, en;
    entry_of(a, a.pyr_base, 0, g, &e, &st, &en);
    const LevelPlan& P = plan(a, e);
    const int b = g - st;
    const int nbx = (P.W + 63) >> 6;
    const int by = b / nbx, bx = b - by * nbx;
    CHECK(P.level > 0 && by < cdiv(P.H, 16), "k_pyramid_batch: block %d -> entry %d block %d", g,
          e, b);
    model_resample(P.base, P.base_w, P.base_h, P.base_stride, P.lvl_w, P.W, P.H, P.lvl_stride,
                   bx * 64, by * 16, "k_pyramid_batch");
  }
  return hipSuccess;
}

// ------------------------------------------------------------ segment test --

// Tiles taken by a tile launch: (entry, tile index) per block, or per queue draw.
struct TileTake {
  int e, t, band;
};

static std::vector<TileTake> tiles_of_launch(const KArgs& a, int grid, uint32_t* qctr,
                                             const int32_t* base, const int32_t* band_base,
                                             int rev, const char* what) {
  std::vector<TileTake> out;
  std::vector<int32_t> draws;
  if (a.persistent) {
    acc(qctr, 4, "queue counter", true);
    const uint32_t c0 = *qctr;
    CHECK(c0 == 0, "%s: persistent queue counter starts at %u, not 0", what, c0);
    // each block draws until it reaches the total, then stops: total + grid draws
    for (int64_t d = 0; d < (int64_t)a.total + grid; ++d) draws.push_back((int32_t)(c0 + d));
    *qctr = c0 + a.total + grid;
  } else {
    for (int b = 0; b < grid; ++b) draws.push_back(b);
  }
  for (size_t k = 0; k < draws.size(); ++k) {
    const int g0 = draws[k];
    const int band = a.persistent ? 0 : g0 % kXcds;
    const int32_t* table = a.bands ? band_base + band * (a.n_entries + 1) : base;
    const int row = a.bands ? band : (a.persistent ? 0 : g0 % kXcds);
    const int btiles = a.bands ? table_total(a, table, row) : 0;
    const int g = launch_tile(g0, a.total, a.bands, btiles, rev);
    if (g < 0) continue;
    int e, t;
    if (a.entry >= 0) {
      e = a.entry;
      t = g;
    } else {
      int st, en;
      entry_of(a, table, row, g, &e, &st, &en);
      t = g - st;
      CHECK(t >= 0 && g < en, "%s: unit %d outside entry %d [%d, %d)", what, g, e, st, en);
    }
    out.push_back({e, t, band});
  }
  return out;
}

static void check_coverage(const KArgs& a, const std::vector<TileTake>& takes, bool det,
                           const char* what) {
  std::map<std::pair<int, int>, int> seen;  // (entry, tile row * W + col)
  for (const TileTake& k : takes) {
    const LevelPlan& P = plan(a, k.e);
    const int tx_n = det ? P.det_tx : P.mark_tx, ty_n = det ? P.det_ty : P.mark_ty;
    const int rot = det ? P.det_band_rot : P.band_rot;
    const int tx = k.t % tx_n;
    const int ty = k.t / tx_n + (a.bands ? band_row0(ty_n, rot, k.band) : 0);
    CHECK(tx >= 0 && tx < tx_n && ty >= 0 && ty < ty_n, "%s: tile (%d,%d) of entry %d outside "
          "its %dx%d grid", what, tx, ty, k.e, tx_n, ty_n);
    if (a.bands)
      CHECK(ty < band_row0(ty_n, rot, k.band) + band_rows(ty_n, rot, k.band),
            "%s: tile row %d of entry %d outside band %d", what, ty, k.e, k.band);
    seen[{k.e, ty * tx_n + tx}]++;
  }
  const int e0 = a.entry >= 0 ? a.entry : 0, e1 = a.entry >= 0 ? a.entry + 1 : a.n_entries;
  for (int e = e0; e < e1; ++e) {
    const LevelPlan& P = plan(a, e);
    const int n = det ? P.det_tx * P.det_ty : P.mark_tx * P.mark_ty;
    for (int i = 0; i < n; ++i) {
      auto it = seen.find({e, i});
      const int c = it == seen.end() ? 0 : it->second;
      if (c != 1) {
        fail("%s: tile %d of entry %d taken %d times", what, i, e, c);
        return;
      }
    }
  }
}

hipError_t launch_mark(const KArgs& a, bool fused, int grid, hipStream_t) {
  const char* what = "k_mark";
  uint8_t* ws = ws_base(a);
  WsState& st = g_ws[ws];
  st.flags_dirty.resize(a.n_entries, false);
  for (int e = 0; e < a.n_entries; ++e)
    if (a.entry < 0 || a.entry == e)
      CHECK(!st.flags_dirty[e], "k_mark: cell flags of entry %d not cleared since the last call",
            e);
  if (!sig_ok(a)) return hipSuccess;
  const MarkLds& M = a.ml;
  const int TWW = a.t.mark_words, TW = 64 * TWW, PITCH = TW + 16;
  CHECK(M.pitch == PITCH && M.th == a.t.mark_rows, "k_mark: layout of another tuning");
  const int64_t lds_bytes = M.bytes + base_table_bytes(a.n_entries);
  CHECK(lds_bytes <= 65536, "k_mark: %lld bytes of LDS", (long long)lds_bytes);

  if (a.entry < 0) {
    acc(a.counters, 4 * counter_words(a.n_entries), "counters zeroed", true);
    acc(a.qctr + 2, 4, "Harris queue counter", true);
    a.qctr[2] = 0;
    st.counters_dirty = false;
  }
  const auto takes = tiles_of_launch(a, grid, a.qctr + 0, a.mark_base, a.band_base, a.mark_rev,
                                     what);
  check_coverage(a, takes, false, what);
  for (const TileTake& k : takes) {
    const LevelPlan& P = plan(a, k.e);
    const int W = P.W, H = P.H, B = P.B;
    const int tx = k.t % P.mark_tx;
    const int ty = k.t / P.mark_tx + (a.bands ? band_row0(P.mark_ty, P.band_rot, k.band) : 0);
    const MarkTile T = mark_tile(W, H, TW, M.th, tx, ty);
    const int nx = T.ex - T.ox, ny = T.ey - T.oy;
    // LDS: staged pixels, resample writes
    lds(0, (int64_t)ny * PITCH, 0, M.off_queue, "k_mark pixels");
    CHECK(nx <= PITCH - 1 && ny <= M.rows, "k_mark: staged %dx%d in %dx%d", nx, ny, PITCH, M.rows);
    if (fused && P.level > 0) {
      // taps of the tile's extreme rows and columns (taps are monotone)
      for (int i : {0, nx - 1})
        for (int j : {0, ny - 1}) {
          const uint32_t txx = resample_tap(T.ox + i, P.base_w, W);
          int xx = (int)(txx >> 9);
          if (xx >= P.base_w - 1) xx = P.base_w - 2;
          const int y0 = (int)(resample_tap(T.oy + j, P.base_h, H) >> 9);
          const int y1 = std::min(y0 + 1, P.base_h - 1);
          acc(P.base + (size_t)y0 * P.base_stride + xx, 2, "k_mark resample tap");
          acc(P.base + (size_t)y1 * P.base_stride + xx, 2, "k_mark resample tap");
          CHECK((int64_t)y1 * P.base_stride + xx + 1 <= INT32_MAX, "k_mark: 32-bit tap offset");
        }
      // grouped taps: one 8-byte load per source row for 4 or 2 adjacent columns
      const int kgrp = 3 * P.base_w < 6 * W ? 4 : (P.base_w < 6 * W ? 2 : 1);
      if (kgrp > 1) {
        CHECK(P.base_w >= 8, "k_mark: frame narrower than one 8-byte load");
        // tap tables in the queue's region: x0 and weights of columns [0, nx), two row
        // offsets and weights of rows [0, ny)
        CHECK(nx <= M.tcols, "k_mark: %d columns for %d tap slots", nx, M.tcols);
        const int64_t tq = M.off_queue;
        lds(tq, 4 * (int64_t)nx, M.off_queue, M.off_bml, "k_mark column taps x0");
        lds(tq + 4 * (int64_t)M.tcols, 4 * (int64_t)nx, M.off_queue, M.off_bml,
            "k_mark column tap weights");
        lds(tq + 8 * (int64_t)M.tcols, 8 * (int64_t)ny, M.off_queue, M.off_bml,
            "k_mark row offsets");
        lds(tq + 8 * (int64_t)M.tcols + 8 * (int64_t)M.rows, 4 * (int64_t)ny, M.off_queue,
            M.off_bml, "k_mark row weights");
        for (int i0 : {4, 4 + TW - kgrp}) {
          auto colx = [&](int i) {
            int xx = (int)(resample_tap(T.ox + std::min(i, nx - 1), P.base_w, W) >> 9);
            return xx >= P.base_w - 1 ? P.base_w - 2 : xx;
          };
          const int b = std::min(colx(i0), P.base_w - 8);
          for (int m = 0; m < kgrp; ++m)
            CHECK(colx(i0 + m) - b >= 0 && colx(i0 + m) - b <= 6,
                  "k_mark: column tap %d bytes into an 8-byte load", colx(i0 + m) - b);
          for (int j : {0, ny - 1}) {
            const int y0 = (int)(resample_tap(T.oy + j, P.base_h, H) >> 9);
            const int y1 = std::min(y0 + 1, P.base_h - 1);
            acc(P.base + (size_t)y0 * P.base_stride + b, 8, "k_mark grouped taps");
            acc(P.base + (size_t)y1 * P.base_stride + b, 8, "k_mark grouped taps");
          }
        }
        lds((int64_t)(ny - 1) * PITCH + 4 + TW - kgrp, kgrp, 0, M.off_queue, "k_mark grouped store");
      }
      // the tile's own pixels to the level buffer
      for (int r : {T.y_t0, T.y_t1 - 1})
        acc(P.lvl_w + (size_t)r * P.lvl_stride + T.x_t0, T.x_t1 - T.x_t0, "k_mark level store",
            true);
      CHECK(T.x_t0 % 16 == 0 || T.x_t1 - T.x_t0 < 16, "k_mark: 16-byte stores misaligned");
    } else if (stage_wide(T.ox, T.ex, P.level == 0 ? W : P.lvl_stride, PITCH)) {
      const int span = 16 * ((T.ex - T.ox + 15) >> 4);
      for (int row : {T.oy, T.ey - 1})
        acc(P.lvl + (size_t)row * P.lvl_stride + T.ox, span, "k_mark staged chunks");
      lds((int64_t)(ny - 1) * PITCH, span, 0, M.off_queue, "k_mark staged chunks");
    } else {
      const int limit = P.level == 0 ? W : P.lvl_stride;
      const int nw = (T.ex - T.ox + 3) >> 2;
      for (int row : {T.oy, T.ey - 1})
        for (int w : {0, nw - 1}) {
          const int x = T.ox + 4 * w, room = limit - x;
          const int back = room >= 4 ? 0 : 4 - room;
          CHECK(room >= 1, "k_mark: staged word past the row");
          acc(P.lvl + (size_t)row * P.lvl_stride + x - back, 4, "k_mark staged word");
        }
      lds(0, (int64_t)(ny - 1) * PITCH + 4 * nw, 0, M.off_queue, "k_mark staged words");
    }
    // pre-test: rows ya.. yb of the valid region, word reads lx - 4 .. lx + 7 and the
    // compass rows at +-3
    const int ya = std::max(T.y_t0, B), yb = std::min(T.y_t1, H - B);
    for (int w = 0; w < 4; ++w) {
      int n = 0;
      for (int y = ya + w; y < yb; y += 4) n += TW;
      CHECK(n <= M.qseg, "k_mark: wave %d may append %d to a %d-entry queue", w, n, M.qseg);
    }
    if (ya < yb) {
      for (int y : {ya, yb - 1})
        for (int lx : {T.x_t0 - T.ox, T.x_t0 + TW - 2 - T.ox}) {
          const int ly = y - T.oy;
          // the pixel row's words around lx (west / east) and the north / south pairs
          lds((int64_t)ly * PITCH + (lx & ~3) - 4, 12, 0, M.off_queue, "k_mark pre-test");
          lds((int64_t)(ly - 3) * PITCH + lx, 2, 0, M.off_queue, "k_mark pre-test");
          lds((int64_t)(ly + 3) * PITCH + lx, 2, 0, M.off_queue, "k_mark pre-test");
        }
      // full test: the 7x7 box of any valid pixel of the tile
      const int xa = std::max(T.x_t0, B), xb = std::min(T.x_t1, W - B);
      if (xa < xb)
        for (int y : {ya, yb - 1})
          for (int x : {xa, xb - 1}) {
            const int lx = x - T.ox, ly = y - T.oy;
            CHECK(lx < 512 && ly < 128, "k_mark: queue entry (%d,%d) does not fit 16 bits", lx, ly);
            lds((int64_t)(ly - 3) * PITCH + lx - 3, 7, 0, M.off_queue, "k_mark full test");
            lds((int64_t)(ly + 3) * PITCH + lx - 3, 7, 0, M.off_queue, "k_mark full test");
            const int word = (y - T.y_t0) * 2 * TWW + ((x - T.x_t0) >> 5);
            lds(M.off_bml + 4 * word, 4, M.off_bml, M.off_bmh, "k_mark bitmap (lo)");
            lds(M.off_bmh + 4 * word, 4, M.off_bmh, M.bytes, "k_mark bitmap (hi)");
            const int64_t c = (int64_t)(y / P.cs) * P.ncx + x / P.cs;
            CHECK(c < (int64_t)P.ncx * P.ncy, "k_mark: cell %lld", (long long)c);
            acc(P.flags + c, 1, "k_mark cell flag", true);
          }
    }
    // the tile's cells, flagged in LDS and written at the end of the tile
    {
      const int cx0 = T.x_t0 / P.cs, cy0 = T.y_t0 / P.cs;
      const int ncxt = (T.x_t1 - 1) / P.cs - cx0 + 1, ncyt = (T.y_t1 - 1) / P.cs - cy0 + 1;
      CHECK(ncxt * ncyt <= kMarkCellFlags, "k_mark: %d cells in a tile > %d", ncxt * ncyt,
            kMarkCellFlags);
      CHECK(cx0 + ncxt <= P.ncx && cy0 + ncyt <= P.ncy, "k_mark: tile cells outside the level");
      acc(P.flags + (int64_t)cy0 * P.ncx + cx0, 1, "k_mark cell flag", true);
      acc(P.flags + (int64_t)(cy0 + ncyt - 1) * P.ncx + cx0 + ncxt - 1, 1, "k_mark cell flag", true);
    }
    // bitmap words of the tile rows
    const int w0 = T.x_t0 >> 5, nwd = std::min(2 * TWW, P.wpr - w0);
    CHECK(nwd <= 8, "k_mark: %d bitmap words per tile row", nwd);
    for (int r : {0, T.y_t1 - T.y_t0 - 1}) {
      const size_t gi = (size_t)(T.y_t0 + r) * P.wpr + w0;
      acc(P.bm_lo + gi, 4 * nwd, "k_mark bitmap store", true);
      acc(P.bm_hi + gi, 4 * nwd, "k_mark bitmap store", true);
    }
  }
  for (int e = 0; e < a.n_entries; ++e)
    if (a.entry < 0 || a.entry == e) st.flags_dirty[e] = true;
  return hipSuccess;
}

// ------------------------------------------------------- Harris / NMS / cells --

hipError_t launch_detect(const KArgs& a, int grid, hipStream_t) {
  const char* what = "k_detect";
  if (!sig_ok(a)) return hipSuccess;
  const DetLds& D = a.dl;
  const int64_t lds_bytes = D.bytes + base_table_bytes(a.n_entries) + 80;
  CHECK(lds_bytes <= 65536 + 80, "k_detect: %lld bytes of LDS", (long long)lds_bytes);
  const auto takes = tiles_of_launch(a, grid, a.qctr + 2, a.det_base, a.det_band_base, a.det_rev,
                                     what);
  check_coverage(a, takes, true, what);
  const int nfl_alloc = a.cell > 0 ? (a.t.det_cx + 2) * (a.t.det_cy + 2) : 4;
  for (const TileTake& k : takes) {
    const LevelPlan& P = plan(a, k.e);
    const int W = P.W, H = P.H, B = P.B, cs = P.cs;
    const int tx = k.t % P.det_tx;
    const int ty = k.t / P.det_tx + (a.bands ? band_row0(P.det_ty, P.det_band_rot, k.band) : 0);
    const DetTile T = det_tile(P, a.t, a.cell, tx, ty);
    CHECK(T.vx0 < T.vx1 && T.vy0 < T.vy1, "k_detect: empty tile (%d,%d) of entry %d", tx, ty, k.e);
    // LDS regions
    CHECK(T.nunits <= D.nunits, "k_detect: %d candidate words > %d", T.nunits, D.nunits);
    CHECK(T.nfx * T.nfy <= nfl_alloc, "k_detect: %d ring cells > %d", T.nfx * T.nfy, nfl_alloc);
    // candidate-word masks: two words per (flag row, word column)
    CHECK(T.nfy <= D.fm_rows && T.nbw <= D.nbw, "k_detect: %dx%d mask table > %dx%d", T.nfy,
          T.nbw, D.fm_rows, D.nbw);
    lds(D.off_fm + 8 * ((int64_t)T.nfy * T.nbw - 1), 8, D.off_fm, D.bytes, "k_detect word masks");
    // the cells a word column's table entry reads: c0 .. c0 + 4 from the first valid column,
    // those overlapping the word inside the ring's flag columns
    {
      const int xa0 = std::max(T.rx0, B), xb0 = std::min(T.rx0 + T.rw, W - B);
      for (int k = 0; k < T.nbw; ++k) {
        const int x0 = (T.bw0 + k) << 5, a0 = std::max(x0, xa0), b0 = std::min(x0 + 32, xb0);
        if (a0 >= b0) continue;
        for (int c = a0 / cs; c * cs < b0; ++c) {
          CHECK(c - a0 / cs < 5, "k_detect: word %d meets more than 5 cells", k);
          CHECK(c >= T.fcx0 && c < T.fcx0 + T.nfx, "k_detect: cell %d outside the ring's flags", c);
        }
      }
    }
    CHECK(T.nlcx * T.nlcy <= D.max_cells, "k_detect: %d cells > %d", T.nlcx * T.nlcy, D.max_cells);
    const int vw = T.vx1 - T.vx0, vh = T.vy1 - T.vy0;
    CHECK(((vw + 1) / 2) * ((vh + 1) / 2) <= D.max_surv, "k_detect: survivors may exceed %d",
          D.max_surv);
    const int nw = (T.sx1 - T.sx0 + 3) >> 2;
    CHECK(4 * nw <= D.pitch && T.sy1 - T.sy0 <= D.rows, "k_detect: staged %dx%d words in %dx%d",
          nw, T.sy1 - T.sy0, D.pitch / 4, D.rows);
    // the kernel's 16-bit reciprocal divisions by nbw and nfx need index * divisor < 2^16
    CHECK((int64_t)std::max(T.nunits, std::max(T.nfy * T.nbw, 2 * 256)) * T.nbw < 65536 &&
              (int64_t)std::max(T.nfx * T.nfy, 2 * 256) * T.nfx < 65536,
          "k_detect: divisions by %d and %d beyond their exact range", T.nbw, T.nfx);
    // Harris windows of the extreme ring candidates: 3 words per row from (cx - 4) & ~3
    const int xa = std::max(T.rx0, B), xb = std::min(T.rx0 + T.rw, W - B);
    const int ya = std::max(T.ry0, B), yb = std::min(T.ry0 + T.rh, H - B);
    if (xa < xb && ya < yb)
      for (int x : {xa, xb - 1})
        for (int y : {ya, yb - 1}) {
          const int cx = x - T.sx0, cy = y - T.sy0;
          CHECK(cx >= 4 && cy >= 4, "k_detect: Harris window left of the staged pixels");
          lds((int64_t)(cy - 4) * D.pitch + ((cx - 4) & ~3), 12, 0, D.off_cw, "k_detect Harris");
          lds((int64_t)(cy + 4) * D.pitch + ((cx - 4) & ~3), 12, 0, D.off_cw, "k_detect Harris");
          CHECK(cy + 4 < T.sy1 - T.sy0 && cx + 4 < T.sx1 - T.sx0,
                "k_detect: Harris window past the staged pixels");
        }
    // NMS lookups of tile pixels' neighbours in the candidate words
    for (int x : {T.vx0, T.vx1 - 1})
      for (int y : {T.vy0, T.vy1 - 1})
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int qu = (y + dy - T.ry0) * T.nbw + ((x + dx) >> 5) - T.bw0;
            CHECK(qu >= 0 && qu < T.nunits, "k_detect: neighbour word %d of %d", qu, T.nunits);
          }
    // global: bitmap words, cell flags, staged pixels
    for (int r : {0, T.rh - 1}) {
      const size_t gi = (size_t)(T.ry0 + r) * P.wpr + T.bw0;
      acc(P.bm_lo + gi, 4 * T.nbw, "k_detect bitmap read");
      acc(P.bm_hi + gi, 4 * T.nbw, "k_detect bitmap read");
    }
    CHECK(T.fcx0 + T.nfx <= P.ncx && T.fcy0 + T.nfy <= P.ncy, "k_detect: ring cells outside "
          "the level's %dx%d cells", P.ncx, P.ncy);
    acc(P.flags + (int64_t)T.fcy0 * P.ncx + T.fcx0, 1, "k_detect flag read");
    acc(P.flags + (int64_t)(T.fcy0 + T.nfy - 1) * P.ncx + T.fcx0 + T.nfx - 1, 1,
        "k_detect flag read");
    const int limit = P.level == 0 ? W : P.lvl_stride;
    if (stage_wide(T.sx0, T.sx1, limit, D.pitch)) {  // whole 16-byte chunks
      const int span = 16 * ((T.sx1 - T.sx0 + 15) >> 4);
      CHECK(span <= D.pitch, "k_detect: %d-byte chunks in a %d-byte LDS row", span, D.pitch);
      for (int row : {T.sy0, T.sy1 - 1})
        acc(P.lvl + (size_t)row * P.lvl_stride + T.sx0, span, "k_detect staged chunks");
      lds((int64_t)(T.sy1 - T.sy0 - 1) * D.pitch, span, 0, D.off_cw, "k_detect staged chunks");
    } else {
      for (int row : {T.sy0, T.sy1 - 1})
        for (int w : {0, nw - 1}) {
          const int x = T.sx0 + 4 * w, room = limit - x;
          const int back = room >= 4 ? 0 : 4 - room;
          acc(P.lvl + (size_t)row * P.lvl_stride + x - back, 4, "k_detect staged word");
        }
    }
    // outputs: slots of the tile's cells, or of its 2x2 blocks, or the appended list
    const int nvx = P.det_xend - P.det_x0;
    if (a.cell > 0) {
      for (int lcy : {0, T.nlcy - 1})
        for (int lcx : {0, T.nlcx - 1}) {
          const int64_t c = (int64_t)(T.cya + lcy - P.det_y0) * nvx + (T.cxa + lcx - P.det_x0);
          CHECK((c + 1) * P.kslot <= P.cand_cap, "k_detect: cell slot %lld past %d",
                (long long)c, P.cand_cap);
          acc(P.cand + c * P.kslot, (int64_t)sizeof(Cand) * P.kslot, "k_detect cell slots", true);
        }
    } else if (P.compact) {
      acc(P.cand, (int64_t)sizeof(Cand) * P.cand_cap, "k_detect appended list", true);
    } else {
      const int nbx = (vw + 1) >> 1, nby = (vh + 1) >> 1;
      const int srow = (T.vy0 - B) >> 1, scol = (T.vx0 - B) >> 1;
      CHECK(nbx * nby <= D.max_surv, "k_detect: %d block flags", nbx * nby);
      for (int by : {0, nby - 1}) {
        const int64_t s0 = (int64_t)(srow + by) * P.slot_w + scol;
        CHECK(s0 + nbx <= P.cand_cap, "k_detect: block slot %lld past %d",
              (long long)(s0 + nbx), P.cand_cap);
        acc(P.cand + s0, (int64_t)sizeof(Cand) * nbx, "k_detect block slots", true);
      }
    }
    for (int k : {0, kCountSpread - 1}) {  // the sub-counters a tile may add to
      acc(P.cand_count + (int64_t)k * P.count_stride, 4, "k_detect count", true);
      acc(P.ncand_count + (int64_t)k * P.count_stride, 4, "k_detect FAST count", true);
    }
  }
  g_ws[ws_base(a)].counters_dirty = true;
  return hipSuccess;
}

hipError_t launch_sum_fast_counts(const uint32_t* counters, int n, int32_t* out, hipStream_t) {
  const int64_t cs = count_stride(n);
  acc(counters + kCountSpread * cs, 4 * kCountSpread * cs, "FAST count sums");
  acc(out, 4 * (int64_t)n, "FAST count output", true);
  return hipSuccess;
}

hipError_t launch_scale_counters(const KArgs& a, int, hipStream_t) {
  acc(a.counters, 4 * counter_words(a.n_entries), "k_scale_counters", true);
  return hipSuccess;
}

// ------------------------------------------- level selection + orientation --

static int model_filled(const LevelPlan& P) {
  // the most a level's counter can hold: every slot filled / the whole list appended
  return P.cand_cap;
}

static void model_moments(const LevelPlan& P, const char* what) {
  // keypoints lie in the valid region [B, W - B) x [B, H - B); the disk of radius B
  const int B = P.B;
  for (int x : {B, P.W - 1 - B})
    for (int y : {B, P.H - 1 - B}) {
      acc(P.lvl + (size_t)(y - B) * P.lvl_stride + x - B, 2 * B + 1, what);
      acc(P.lvl + (size_t)(y + B) * P.lvl_stride + x - B, 2 * B + 1, what);
    }
}

static std::map<const void*, std::pair<const void*, int64_t>> g_out_slices;  // out -> (base, cap)

static void check_out(const LevelPlan& P, const KArgs& a, int64_t idx, const char* what) {
  acc(P.out + idx, sizeof(of_keypoint), what, true);
}

hipError_t launch_select_orient(const KArgs& a, int slots, hipStream_t) {
  const char* what = "k_select_orient";
  if (!sig_ok(a)) return hipSuccess;
  WsState& st = g_ws[ws_base(a)];
  CHECK(slots >= 1, "k_select_orient: %d slots", slots);
  if (a.flags) {  // the first counting launch clears them for the next call
    acc(a.flags, a.flag_bytes, "flags zeroed", true);
    st.flags_dirty.assign(a.n_entries, false);
    acc(a.qctr, 4, "queue counter zeroed", true);
    a.qctr[0] = 0;
  }
  CHECK((int64_t)8 * a.sel_lds <= 65536 - 4100, "k_select_orient: LDS");
  const int nslots = table_total(a, a.rank_base, 0);
  const int64_t clear = 4 * std::max<int64_t>((a.flag_bytes / 16 + 2047) / 2048, 1);
  CHECK(slots == (a.from_sel ? nslots : (int)std::max<int64_t>(nslots, clear)),
        "k_select_orient: %d slots launched for %d", slots, nslots);
  if (a.from_sel)
    CHECK(a.rank_base == a.sel_base && !a.flags, "k_select_orient: list launch tables");
  // per entry: the slot range, ranked candidates and outputs
  for (int e = 0; e < a.n_entries; ++e) {
    const LevelPlan& P = plan(a, e);
    int ee, s0, en;
    const int32_t first = a.small ? a.sbase[e] : a.rank_base[e];
    if (!a.small) acc(a.rank_base + e, 4, "rank prefix");
    const int32_t next = e + 1 < a.n_entries ? (a.small ? a.sbase[e + 1] : a.rank_base[e + 1])
                                             : nslots;
    if (next == first) continue;  // an entry without slots (its level takes the radix path)
    entry_of(a, a.rank_base, 0, first, &ee, &s0, &en);
    CHECK(ee == e || first == en, "k_select_orient: slot %d of entry %d found in entry %d",
          first, e, ee);
    const bool radix = P.compact || P.cand_cap > a.t.rank_cap;  // can take the radix path
    const int C = a.from_sel ? std::min(model_filled(P), P.quota)
                             : ranked_candidates(P, (uint32_t)model_filled(P));
    const int want = a.from_sel ? (radix ? P.quota : 0)
                     : P.compact ? std::min(P.cand_cap, a.t.rank_cap)
                                 : (P.cand_cap <= a.t.rank_cap ? P.cand_cap : 0);
    CHECK(en - s0 == want, "k_select_orient: entry %d has %d slots", e, en - s0);
    if (a.from_sel || C <= a.t.rank_cap) {
      if (a.from_sel) acc(P.sel_count, 4, "k_select_orient list count");
      acc(a.from_sel ? P.sel : P.cand, (int64_t)sizeof(Cand) * C,
          "k_select_orient candidate reads");
      if (a.sel_lds > 0 && C <= a.sel_lds) {
        CHECK(a.sel_lds % 256 == 0, "k_select_orient: staged copy padded to 256");
        lds(0, 8 * (((int64_t)C + 255) & ~255), 0, 8 * (int64_t)a.sel_lds,
            "k_select_orient staged R' (padded)");
      }
      model_moments(P, "k_select_orient moments");
      // the level's keypoints at prefix .. prefix + quota of the frame's output
      int64_t prefix = 0;
      for (int l = 0; l < P.level; ++l) prefix += plan(a, P.entry0 + l).quota;
      if (P.quota > 0) check_out(P, a, prefix + P.quota - 1, "k_select_orient keypoint");
    }
    acc(P.count_out, 4, "k_select_orient count", true);
    // the frame's level counters: every sub-counter of its levels
    const LevelPlan& P0 = plan(a, P.entry0);
    acc(P0.cand_count, 4, "k_select_orient level counters");
    acc(P0.cand_count + (P.n_levels - 1) + (int64_t)(kCountSpread - 1) * P.count_stride, 4,
        "k_select_orient level counters");
  }
  return hipSuccess;
}

hipError_t launch_select(const KArgs& a, int grid, hipStream_t) {
  if (!sig_ok(a)) return hipSuccess;
  CHECK(grid == a.n_entries, "k_select: grid %d for %d entries", grid, a.n_entries);
  for (int e = 0; e < grid; ++e) {
    const LevelPlan& P = plan(a, e);
    const int nfill = model_filled(P);
    const int C = ranked_candidates(P, (uint32_t)nfill);
    acc(P.sel_count, 4, "k_select count", true);
    if (a.rank_path && C <= a.t.rank_cap) continue;
    acc(P.cand, (int64_t)sizeof(Cand) * C, "k_select candidate reads");
    const int nout = std::min(nfill, P.quota);
    CHECK(nout <= kSortCap, "k_select: %d selected > sort capacity", nout);
    if (nout > 0) acc(P.sel, (int64_t)sizeof(Cand) * nout, "k_select selection", true);
    acc(P.sel_count, 4, "k_select count", true);
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ others --

hipError_t launch_describe(const DescArgs& a, hipStream_t) {
  acc(a.ws_sig, 8, "describe signature");
  if (*a.ws_sig != a.sig) return hipSuccess;
  for (int f = 0; f < a.n; ++f) {
    acc(a.counts + f, 4, "describe count");
    acc(a.kps + a.off[f], (int64_t)sizeof(of_keypoint) * a.cap, "describe keypoints");
    acc(a.desc + (size_t)a.off[f] * 32, 32 * (int64_t)a.cap, "describe output", true);
    for (int l = 0; l < a.L; ++l) {
      const LevelPlan& P = a.plan[f * a.L + l];
      acc(&P, sizeof(LevelPlan), "describe plan");
      for (int x : {15, P.W - 16})
        for (int y : {15, P.H - 16}) {
          if (x < 15 || y < 15) continue;
          acc(P.lvl + (size_t)(y - 15) * P.lvl_stride + x - 15, 31, "describe patch");
          acc(P.lvl + (size_t)(y + 15) * P.lvl_stride + x - 15, 31, "describe patch");
        }
    }
  }
  acc(a.rot, 30 * 256 * 4, "describe table");
  acc(a.centres, 30 * 2 * 4, "describe centres");
  return hipSuccess;
}

hipError_t launch_test_segment(const uint8_t* c, int n, int, int, uint8_t* out, hipStream_t) {
  acc(c, 17 * (int64_t)n, "test_segment input");
  acc(out, n, "test_segment output", true);
  return hipSuccess;
}

hipError_t launch_ablate_fast(const AbArgs&, int, hipStream_t) { return hipSuccess; }
hipError_t launch_ablate_harris(const AbArgs&, int, hipStream_t) { return hipSuccess; }
int ablate_fast_blocks(int variant, int W, int H) { return cdiv(W, 64) * cdiv(H, variant == 0 ? 4 : 16); }
int ablate_harris_blocks(int variant, int W, int H, int n) {
  return variant <= 1 ? cdiv(n, 256) : (variant == 2 ? cdiv(n, 32) : cdiv(W, 64) * cdiv(H, 32));
}
void set_launch_events(hipEvent_t, hipEvent_t) {}

// The static workspace: a host buffer of the same size stands in for the device array.
hipError_t scratch_workspace(void** ptr) {
  static void* p = nullptr;
  if (!p) p = dev_alloc(OF_SCRATCH_BYTES, "static workspace");
  *ptr = p;
  return hipSuccess;
}

}  // namespace ofk

// ---------------------------------------------------- HIP runtime stand-ins --

extern "C" {
hipError_t hipGetDevice(int*) { return hipErrorNoDevice; }
hipError_t hipDeviceGetAttribute(int*, hipDeviceAttribute_t, int) { return hipErrorNoDevice; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  acc(s, n, "memcpy source");
  acc(d, n, "memcpy destination", true);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t*) { return hipErrorNoDevice; }
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float*, hipEvent_t, hipEvent_t) { return hipErrorNoDevice; }
}

// ----------------------------------------------------------------- driver --

struct Frame {
  int w, h, stride;
  uint8_t* data;
};

static Frame make_frame(int w, int h, int pad = 0) {
  Frame f{w, h, w + pad, nullptr};
  f.data = (uint8_t*)dev_alloc((size_t)f.stride * (h - 1) + w, "frame");
  return f;
}

static of_params params(int L, int t, int tmin, int cell, int N, int num = 6, int den = 5,
                        int radius = 15) {
  of_params p;
  p.n_levels = L;
  p.scale_num = num;
  p.scale_den = den;
  p.fast_t = t;
  p.fast_t_min = tmin;
  p.cell = cell;
  p.n_features = N;
  p.harris_block = 7;
  p.patch_radius = radius;
  return p;
}

static of_tuning tuning() {
  of_tuning t;
  memset(&t, 0, sizeof(t));
  t.mark_grid = t.det_grid = t.pyr_pass = t.mark_order = t.plan_resident = t.det_order = -1;
  return t;
}

// A detector that owns its workspace and outputs, like ofhip.Detector.
struct Detector {
  std::vector<Frame> frames;
  of_params p;
  uint8_t* ws = nullptr;
  size_t ws_bytes = 0;
  of_keypoint* out = nullptr;
  int32_t* counts = nullptr;
  std::vector<int64_t> offs;
  bool resident;

  Detector(const std::vector<Frame>& fr, const of_params& pp, bool res) : frames(fr), p(pp),
                                                                          resident(res) {
    std::vector<of_image> im = images();
    CHECK(of_workspace_size(im.data(), (int)im.size(), &p, &ws_bytes) == OF_OK,
          "of_workspace_size rejects the frames");
    ws = (uint8_t*)dev_alloc(ws_bytes, "workspace");
    out = (of_keypoint*)dev_alloc(sizeof(of_keypoint) * p.n_features * frames.size(), "keypoints");
    counts = (int32_t*)dev_alloc(4 * frames.size(), "counts");
    for (size_t i = 0; i < frames.size(); ++i) offs.push_back((int64_t)i * p.n_features);
  }
  ~Detector() {
    dev_free(ws);
    dev_free(out);
    dev_free(counts);
  }
  std::vector<of_image> images() const {
    std::vector<of_image> im;
    for (const Frame& f : frames) im.push_back({f.data, f.w, f.h, f.stride});
    return im;
  }
  int batch(of_tuning t) {
    if (resident) t.plan_resident = 1;
    std::vector<of_image> im = images();
    return of_detect_batch(im.data(), (int)im.size(), &p, ws, ws_bytes, out, offs.data(),
                           p.n_features, counts, &t, nullptr);
  }
  int plain() {
    std::vector<of_image> im = images();
    return of_detect(&im[0], &p, ws, ws_bytes, out, p.n_features, counts, nullptr);
  }
  int describe(of_tuning t) {
    if (resident) t.plan_resident = 1;
    std::vector<of_image> im = images();
    int8_t* rot = (int8_t*)dev_alloc(30 * 256 * 4, "rot");
    int32_t* cen = (int32_t*)dev_alloc(30 * 2 * 4, "centres");
    uint8_t* desc = (uint8_t*)dev_alloc(32 * (size_t)p.n_features * frames.size(), "desc");
    int st = of_describe(im.data(), (int)im.size(), &p, &t, ws, out, offs.data(), counts, rot, cen,
                         desc, nullptr);
    dev_free(rot);
    dev_free(cen);
    dev_free(desc);
    return st;
  }
};

static void expect_ok(int st, const char* what) {
  CHECK(st == OF_OK, "%s returned %d", what, st);
}

static of_tuning tune_of(std::initializer_list<std::pair<const char*, int>> kv) {
  of_tuning t = tuning();
  for (auto& x : kv) {
    const std::string k = x.first;
    if (k == "mark_words") t.mark_words = x.second;
    else if (k == "mark_rows") t.mark_rows = x.second;
    else if (k == "det_cells_x") t.det_cells_x = x.second;
    else if (k == "det_cells_y") t.det_cells_y = x.second;
    else if (k == "det_w") t.det_w = x.second;
    else if (k == "det_h") t.det_h = x.second;
    else if (k == "mark_grid") t.mark_grid = x.second;
    else if (k == "det_grid") t.det_grid = x.second;
    else if (k == "pyr_pass") t.pyr_pass = x.second;
    else if (k == "mark_order") t.mark_order = x.second;
    else if (k == "det_order") t.det_order = x.second;
  }
  return t;
}

// The autotuner's trial sequence on one resident workspace (coordinate descent over
// grids, segment-test tiles, Harris tiles, then grids again), every candidate run twice
// (planning call, then a resident call), as the search issues them.
static void scenario_tuner(const std::vector<Frame>& frames, const of_params& p, int cus) {
  Detector det(frames, p, true);
  std::vector<of_tuning> grids, marks, dets;
  for (int mo = 0; mo < 2; ++mo)
    for (int dor = 0; dor < 2; ++dor)
      for (int pp = 0; pp < 2; ++pp)
        grids.push_back(tune_of({{"mark_grid", 0}, {"det_grid", 0}, {"pyr_pass", pp},
                                 {"mark_order", mo}, {"det_order", dor}}));
  for (int m : {2, 4})
    for (int d : {2, 3})
      grids.push_back(tune_of({{"mark_grid", m * cus}, {"det_grid", d * cus}}));
  grids.push_back(tune_of({{"mark_grid", 7}, {"det_grid", 3}}));
  for (int w : {1, 2, 3, 4})
    for (int r : {4, 5, 6, 7, 8, 9, 13, 16, 24, 32, 40, 48, 56, 64})
      marks.push_back(tune_of({{"mark_words", w}, {"mark_rows", r}}));
  if (p.cell > 0) {
    const int cds[][2] = {{1, 1}, {2, 1}, {4, 1}, {2, 2}, {8, 1}, {4, 2}, {2, 3}, {1, 4}};
    for (auto& c : cds) dets.push_back(tune_of({{"det_cells_x", c[0]}, {"det_cells_y", c[1]}}));
  } else {
    const int whs[][2] = {{64, 32}, {128, 32}, {128, 64}, {256, 32}, {8, 8}, {8, 10}, {256, 128}};
    for (auto& c : whs) dets.push_back(tune_of({{"det_w", c[0]}, {"det_h", c[1]}}));
  }
  std::vector<of_tuning> all;
  all.push_back(tuning());
  for (auto* grp : {&grids, &marks, &dets, &grids})
    for (auto& t : *grp) all.push_back(t);
  // cross terms: every segment-test tile with persistent grids and band orders
  for (auto& m : marks)
    for (int k = 0; k < 3; ++k) {
      of_tuning t = m;
      if (k == 0) { t.mark_grid = 2 * cus; t.det_grid = 2 * cus; }
      if (k == 1) { t.mark_order = 1; t.det_order = 1; }
      if (k == 2) { t.pyr_pass = 1; t.mark_order = 1; }
      all.push_back(t);
    }
  for (auto& d : dets)
    for (int k = 0; k < 2; ++k) {
      of_tuning t = d;
      if (k == 0) { t.det_grid = 3 * cus; t.mark_order = 1; }
      if (k == 1) { t.det_order = 1; t.mark_order = 1; }
      all.push_back(t);
    }
  int runs = 0;
  for (auto& t : all)
    for (int r = 0; r < 2; ++r) {
      const int st = det.batch(t);
      if (st == OF_EINVAL) break;  // a shape the library rejects (LDS budget): no launch
      expect_ok(st, "tuner trial");
      ++runs;
    }
  printf("  tuner: %zu candidates, %d calls\n", all.size(), runs);
}

static std::vector<int> c3_sizes() {
  std::vector<int> s;
  const int wh[4][2] = {{720, 540}, {1080, 720}, {1440, 1080}, {1920, 1080}};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 16; ++j) {
      s.push_back(wh[i][0]);
      s.push_back(wh[i][1]);
    }
  return s;
}

static void run_scenario(const std::string& name) {
  g_case = name;
  const int cus = 256;
  const of_params c2 = params(8, 20, 7, 30, 2000);
  if (name == "tuner_c2") {
    std::vector<Frame> fr = {make_frame(1920, 1080)};
    scenario_tuner(fr, c2, cus);
  } else if (name == "tuner_cell0") {
    std::vector<Frame> fr = {make_frame(641, 479)};
    scenario_tuner(fr, params(3, 8, 8, 0, 400), cus);
  } else if (name == "tuner_c3") {
    std::vector<Frame> fr;
    auto s = c3_sizes();
    for (size_t i = 0; i < s.size(); i += 2) fr.push_back(make_frame(s[i], s[i + 1]));
    Detector det(fr, c2, true);
    for (auto t : {tuning(), tune_of({{"mark_grid", 512}, {"det_grid", 512}}),
                   tune_of({{"mark_order", 1}, {"det_order", 1}}),
                   tune_of({{"pyr_pass", 1}, {"mark_order", 1}, {"det_order", 1}}),
                   tune_of({{"mark_words", 4}, {"mark_rows", 32}, {"det_cells_x", 4},
                            {"det_cells_y", 2}}),
                   tune_of({{"mark_words", 1}, {"mark_rows", 64}, {"mark_grid", 1024},
                            {"det_grid", 768}})})
      for (int r = 0; r < 2; ++r) expect_ok(det.batch(t), "c3 trial");
  } else if (name == "bench_legs") {
    // fused (resident, shipped shape), plain, 16 copies, c3, c4, c1, patterns, describe
    Frame f = make_frame(1920, 1080);
    of_tuning shipped = tune_of({{"mark_words", 2}, {"mark_rows", 48}, {"det_cells_x", 8},
                                 {"det_cells_y", 1}, {"det_w", 128}, {"det_h", 32},
                                 {"mark_grid", 0}, {"det_grid", 0}, {"pyr_pass", 0},
                                 {"mark_order", 1}, {"det_order", 1}});
    {
      Detector fused({f}, c2, true);
      for (int r = 0; r < 3; ++r) expect_ok(fused.batch(shipped), "fused");
      expect_ok(fused.describe(shipped), "describe");
      Detector plain({f}, c2, false);
      expect_ok(plain.plain(), "plain");
      expect_ok(plain.plain(), "plain");
    }
    {
      std::vector<Frame> fr;
      for (int i = 0; i < 16; ++i) fr.push_back(make_frame(1920, 1080));
      Detector b16(fr, c2, true);
      for (int r = 0; r < 2; ++r) expect_ok(b16.batch(shipped), "16 x 1080p");
    }
    {
      std::vector<Frame> fr;
      auto s = c3_sizes();
      for (size_t i = 0; i < s.size(); i += 2) fr.push_back(make_frame(s[i], s[i + 1]));
      Detector c3(fr, c2, true);
      for (int r = 0; r < 2; ++r) expect_ok(c3.batch(tuning()), "c3");
    }
    {
      std::vector<Frame> fr;
      for (int i = 0; i < 16; ++i) fr.push_back(make_frame(3840, 2160));
      Detector c4(fr, params(12, 20, 7, 30, 5000), true);
      for (int r = 0; r < 2; ++r) expect_ok(c4.batch(tuning()), "c4");
    }
    {
      Detector c1({make_frame(640, 480)}, params(1, 20, 20, 0, 500), true);
      for (int r = 0; r < 2; ++r) expect_ok(c1.batch(tuning()), "c1");
      expect_ok(c1.plain(), "c1 plain");
    }
    for (int L : {1, 4})
      for (int N : {2000, L == 1 ? 4000 : 8000}) {
        Detector pd({make_frame(1024, 1024)}, params(L, 20, 20, 0, N), true);
        for (int r = 0; r < 2; ++r) expect_ok(pd.batch(tuning()), "patterns");
      }
  } else if (name == "served") {
    // mixed batches of up to 16 frames (720x540 .. 1920x1080), fresh workspaces per
    // batch, three lanes in flight
    const int wh[4][2] = {{720, 540}, {1080, 720}, {1440, 1080}, {1920, 1080}};
    uint64_t s = 12345;
    for (int b = 0; b < 60; ++b) {
      s = s * 6364136223846793005ull + 1442695040888963407ull;
      const int n = 1 + (int)((s >> 33) % 16);
      std::vector<Frame> fr;
      for (int i = 0; i < n; ++i) {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        const int k = (int)((s >> 35) % 4);
        fr.push_back(make_frame(wh[k][0], wh[k][1]));
      }
      Detector d(fr, c2, false);
      expect_ok(d.batch(tuning()), "served batch");
      for (Frame& f : fr) dev_free(f.data);
    }
  } else if (name == "test_shapes") {
    struct S { int w, h, L, t, tmin, cell, N, num, den, r, pad; };
    const S cases[] = {
        {96, 80, 1, 20, 7, 30, 400, 6, 5, 15, 0},      {97, 83, 1, 20, 20, 0, 400, 6, 5, 15, 0},
        {641, 479, 4, 20, 9, 16, 400, 6, 5, 15, 3},    {16384, 40, 1, 20, 7, 30, 1000, 6, 5, 15, 0},
        {40, 16384, 1, 20, 7, 30, 1000, 6, 5, 15, 0},  {480, 480, 16, 20, 7, 30, 2000, 6, 5, 15, 0},
        {480, 480, 16, 20, 7, 30, 60, 6, 5, 15, 0},    {286, 286, 1, 20, 20, 0, 4096, 6, 5, 15, 0},
        {287, 286, 1, 20, 20, 0, 4096, 6, 5, 15, 0},   {31, 31, 1, 20, 7, 30, 4, 6, 5, 15, 0},
        {31, 31, 1, 20, 7, 0, 4, 6, 5, 15, 0},         {641, 479, 4, 20, 7, 30, 1000, 2, 1, 8, 0},
        {641, 479, 6, 20, 7, 30, 1000, 8, 7, 20, 0},   {320, 240, 3, 20, 7, 30, 1000, 3, 2, 4, 0},
        {641, 479, 3, 20, 7, 30, 1000, 6, 5, 31, 0},   {1920, 1080, 8, 20, 7, 30, 1000, 6, 5, 48, 0},
        {700, 500, 3, 20, 7, 8, 600, 6, 5, 15, 0},     {700, 500, 3, 20, 7, 128, 600, 6, 5, 15, 0},
        {400, 300, 3, 20, 7, 30, 600, 6, 5, 15, 0},    {331, 250, 3, 20, 7, 30, 600, 6, 5, 15, 69},
    };
    for (const S& c : cases) {
      Detector d({make_frame(c.w, c.h, c.pad)},
                 params(c.L, c.t, c.tmin, c.cell, c.N, c.num, c.den, c.r), false);
      expect_ok(d.batch(tuning()), "batch");
      expect_ok(d.plain(), "plain");
      for (auto t : {tune_of({{"mark_words", 3}, {"mark_rows", 5}}),
                     tune_of({{"mark_words", 4}, {"mark_rows", 13}, {"mark_order", 1}}),
                     tune_of({{"mark_grid", 7}, {"det_grid", 3}, {"pyr_pass", 1}})})
        expect_ok(d.batch(t), "batch tuned");
    }
  } else if (name == "scratch") {
    // the static-workspace entry point: two calls in a row, the second smaller, then a
    // batch too large for it (rejected before any launch)
    const of_params p = params(8, 20, 7, 30, 2000);
    for (int n : {3, 1}) {
      std::vector<Frame> fr;
      for (int i = 0; i < n; ++i) fr.push_back(make_frame(1920, 1080));
      std::vector<of_image> im;
      for (const Frame& f : fr) im.push_back({f.data, f.w, f.h, f.stride});
      of_keypoint* out = (of_keypoint*)dev_alloc(sizeof(of_keypoint) * 2000 * n, "keypoints");
      int32_t* counts = (int32_t*)dev_alloc(4 * n, "counts");
      std::vector<int64_t> offs;
      for (int i = 0; i < n; ++i) offs.push_back((int64_t)i * 2000);
      of_tuning t = tuning();
      expect_ok(of_detect_batch_scratch(im.data(), n, &p, out, offs.data(), 2000, counts, &t,
                                        nullptr), "scratch call");
      dev_free(out);
      dev_free(counts);
    }
    std::vector<Frame> big;
    for (int i = 0; i < 16; ++i) big.push_back(make_frame(1920, 1080));
    std::vector<of_image> im;
    for (const Frame& f : big) im.push_back({f.data, f.w, f.h, f.stride});
    of_keypoint* out = (of_keypoint*)dev_alloc(sizeof(of_keypoint) * 2000 * 16, "keypoints");
    int32_t* counts = (int32_t*)dev_alloc(4 * 16, "counts");
    std::vector<int64_t> offs;
    for (int i = 0; i < 16; ++i) offs.push_back((int64_t)i * 2000);
    CHECK(of_detect_batch_scratch(im.data(), 16, &p, out, offs.data(), 2000, counts, nullptr,
                                  nullptr) == OF_ENOSPACE, "scratch: oversized batch accepted");
  } else {
    fail("unknown scenario");
  }
}

int main(int argc, char** argv) {
  for (int i = 1; i < argc; ++i) {
    const int before = g_fail;
    run_scenario(argv[i]);
    printf("%s: %s\n", argv[i], g_fail == before ? "ok" : "FAILED");
  }
  printf("%s: %ld checks, %d failures\n", g_fail ? "fail" : "ok", g_checks, g_fail);
  return g_fail ? 1 : 0;
}
