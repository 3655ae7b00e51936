// of_kernels.h -- kernel argument blocks and launch functions (internal).
#pragma once

#include "of_plan.h"

namespace ofk {

constexpr int kSmallEntries = 16;

struct FrameIn {
  const uint8_t* data;
  int32_t w, h, stride, pad;
  int64_t out_off;
};

struct PrologueArgs {
  uint64_t sig;                // hash of this struct (sig = 0) plus a tag; caches the plan
  of_params p;
  Tune t;
  int32_t n;
  int32_t pad;
  FrameIn f[kMaxBatch];
  uint8_t* ws;
  WsLayout lay;
  of_keypoint* out;
  int32_t* counts;
};

// Plan of entry i = (frame f, level l) of a call, from the frame's geometry, the entry's
// sizes and its offsets in the workspace regions (exclusive prefixes over the entries
// before it).  Used by the prologue kernel and by the CPU launch model of the tests.
struct EntryOffsets {
  int64_t flag, bm, cand, sel, lvl;
  int32_t band_rot, det_band_rot;
  uint32_t* counters;  // the workspace's counter region
};

OF_HD void fill_level_plan(LevelPlan& P, const PrologueArgs& a, uint8_t* ws, const FrameGeom& g,
                           const EntrySize& s, int i, int f, int l, const EntryOffsets& o) {
  const int L = a.p.n_levels;
  P.W = g.W[l];
  P.H = g.H[l];
  P.B = a.p.patch_radius;
  P.level = l;
  P.frame = f;
  P.n_levels = L;
  P.cs = g.cs[l];
  P.csd = fast_div((uint32_t)g.cs[l]);
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
    P.lvl_w = ws + a.lay.off_lvl + o.lvl;
    P.lvl = P.lvl_w;
    P.lvl_stride = level_stride(P.W);
  }
  P.wpr = s.wpr;
  P.bm_lo = (uint32_t*)(ws + a.lay.off_bm) + o.bm;
  P.bm_hi = P.bm_lo + (int64_t)s.wpr * P.H;
  P.flags = ws + a.lay.off_flags + o.flag;
  P.cand = (Cand*)(ws + a.lay.off_cand) + o.cand;
  const int32_t cstride = count_stride(a.lay.n_entries);
  P.cand_count = o.counters + i;
  P.count_stride = cstride;
  P.cand_cap = (int32_t)s.cand_cap;
  P.kslot = s.kslot;
  P.compact = a.p.cell == 0 && s.cand_cap > kRankCap;
  P.slot_w = s.slot_w;
  P.sel = (Cand*)(ws + a.lay.off_sel) + o.sel;
  P.sel_count = o.counters + 2 * (int64_t)kCountSpread * cstride + i;
  P.ncand_count = o.counters + (int64_t)kCountSpread * cstride + i;
  P.mark_tx = s.mark_tx;
  P.mark_ty = s.mark_ty;
  P.band_rot = o.band_rot;
  P.det_band_rot = o.det_band_rot;
  P.det_tx = s.det_tx;
  P.det_ty = s.det_ty;
  P.det_x0 = s.det_x0;
  P.det_y0 = s.det_y0;
  P.det_xend = s.det_xend;
  P.det_yend = s.det_yend;
  P.entry0 = f * L;
  P.out = a.out + a.f[f].out_off;
  P.count_out = a.counts + f;
}

// Arguments of the tile kernels, selection and orientation.
struct KArgs {
  // Read by every block before its first tile, together (the first cache lines of the
  // argument segment).
  LevelPlan* plan;
  // The plan signature the workspace must hold: blocks of a workspace with another plan
  // do nothing (the selection then sets every frame's count to -1).
  const uint64_t* ws_sig;      // the workspace's copy, written by the prologue
  uint64_t sig;
  int32_t n_entries;
  int32_t total;               // tiles (or blocks) of this launch
  int32_t entry;               // >= 0: one entry only, tile = blockIdx.x
  int32_t persistent;          // 1: blocks draw tiles from qctr until exhausted
  int32_t bands;               // 1: block b takes band b % kXcds, tile b / kXcds of it
  int32_t small;               // 1: the prefix table of this launch is in sbase
  uint32_t* qctr;              // queue counters: [0] segment-test tiles, [2] Harris tiles
  int32_t cell;                // params.cell
  int32_t rank_path;           // 1: k_select_orient ranks levels with <= t.rank_cap candidates
  Tune t;
  int32_t pad;
  MarkLds ml;                  // LDS layouts of the tile kernels for this tuning (host-made)
  DetLds dl;
  // The state each call leaves zeroed for the next: k_mark clears the counters, the
  // selection clears the cell flags and the segment-test queue counter.
  uint32_t* counters;          // counter_words(n_entries)
  uint8_t* flags;
  int64_t flag_bytes;          // multiple of 16
  int32_t* frame_counts;
  const int32_t* mark_base;    // exclusive prefix of tiles per entry (n_entries + 1)
  const int32_t* det_base;
  const int32_t* sel_base;     // exclusive prefix of selection-list slots per entry
  const int32_t* rank_base;    // exclusive prefix of the slots a counting launch ranks per
                               // entry (rank_slots, or sel_slots for a from_sel launch)
  const int32_t* pyr_base;     // exclusive prefix of resample blocks per entry
  const int32_t* band_base;    // kXcds tables: prefix of segment-test tiles per entry in band k
  const int32_t* det_band_base;  // the same for Harris/NMS tiles
  int32_t n_frames;
  int32_t sel_lds;             // level R' the selection stages in LDS (0: none)
  int32_t from_sel;            // 1: k_select_orient ranks each level's radix-selected list
  int32_t det_rev;             // 1: Harris/NMS tiles taken last first (grid resident at once)
  int32_t mark_rev;            // 1: segment-test tiles taken last first (grid resident at once)
  // Batches of at most kSmallEntries entries carry the launch's prefix table here, so
  // blocks find their entry without a memory load: entries 0 .. n_entries - 1, INT32_MAX
  // up to index kSmallEntries - 1 and the launch's total at index kSmallEntries.  The
  // segment-test launch fills kXcds rows (one per band, or the same row kXcds times),
  // the others row 0.
  int32_t sbase[kXcds * (kSmallEntries + 1)];
};

struct PyrLevel {
  uint8_t* dst;
  int32_t w, h, stride, pad;
};

struct PyrArgs {
  const uint8_t* src;
  int32_t src_w, src_h, src_stride, pad;
  PyrLevel lv[kMaxLevels];
};

struct LaunchEvents {
  hipEvent_t start, stop;
};

// The next launch records `start` as it begins and `stop` as it ends (either may be
// null); later launches record nothing.
void set_launch_events(hipEvent_t start, hipEvent_t stop);

hipError_t launch_prologue(const PrologueArgs& a, int grid, hipStream_t s);
hipError_t launch_pyramid(const PyrArgs& a, int n_levels, int max_w, int max_h, hipStream_t s);
hipError_t launch_pyramid_batch(const KArgs& a, int blocks, hipStream_t s);
hipError_t launch_mark(const KArgs& a, bool fused, int grid, hipStream_t s);
hipError_t launch_detect(const KArgs& a, int grid, hipStream_t s);
hipError_t launch_scale_counters(const KArgs& a, int times, hipStream_t s);
// out[e] = the FAST candidates of entry e (the sum of its sub-counters), n entries.
hipError_t launch_sum_fast_counts(const uint32_t* counters, int n, int32_t* out, hipStream_t s);
hipError_t launch_select_orient(const KArgs& a, int slots, hipStream_t s);
hipError_t launch_select(const KArgs& a, int grid, hipStream_t s);
// Arguments of the rBRIEF launch: keypoints of n frames (cap slots each) described on
// the levels of the plan in the workspace, which must carry signature `sig`.
struct DescArgs {
  const LevelPlan* plan;
  const uint64_t* ws_sig;
  uint64_t sig;
  int32_t n, L, cap, pad;
  const of_keypoint* kps;
  const int32_t* counts;
  const int8_t* rot;       // 30 x 256 x 4
  const int32_t* centres;  // 30 x 2
  uint8_t* desc;           // 32 bytes per keypoint slot, indexed like kps
  int64_t off[kMaxBatch];  // first keypoint of each frame
};

hipError_t launch_describe(const DescArgs& a, hipStream_t s);

// Device address of this device's static workspace (OF_SCRATCH_BYTES), looked up once per
// device.
constexpr int kMaxDevices = 64;
hipError_t scratch_workspace(void** ptr);

// Levels of one ablation launch (in the kernel arguments).
constexpr int kAbMaxLevels = 64;
struct AbLevel {
  const uint8_t* img;
  void* out;               // uint8 map (FAST), int64 scores or map (Harris)
  const uint32_t* pos;     // Harris positions (point variants)
  int32_t W, H, stride, n; // n: Harris positions
  int32_t base;            // first block of this level
  int32_t pad;
};
struct AbArgs {
  int32_t n_levels, t, B, pad;
  AbLevel lv[kAbMaxLevels];
};

hipError_t launch_ablate_fast(const AbArgs& a, int variant, hipStream_t s);
hipError_t launch_ablate_harris(const AbArgs& a, int variant, hipStream_t s);
// Blocks a level needs in an ablation launch (the launch functions and the host agree).
int ablate_fast_blocks(int variant, int W, int H);
int ablate_harris_blocks(int variant, int W, int H, int n);
hipError_t launch_test_segment(const uint8_t* circles, int n, int t_lo, int t_hi, uint8_t* out,
                               hipStream_t s);

}  // namespace ofk
