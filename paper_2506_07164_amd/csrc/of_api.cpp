// of_api.cpp -- the C ABI declared in include/of.h: validation, workspace layout and
// launch sequencing.  Every step of the detector runs in the kernels of
// of_kernels.hip; this file only checks arguments and queues launches.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "of_kernels.h"

using namespace ofk;

namespace {

thread_local int g_last_hip = 0;

// ------------------------------------------------------------ step profiling --

constexpr int kEventPool = 8192;

struct Profiler {
  std::mutex mu;
  bool on = false;
  int repeat = 1;   // back-to-back issues of a repeatable launch between its events
  bool created = false;
  hipEvent_t ev[2 * kEventPool];
  int step_of[kEventPool];
  int used = 0;
  int64_t launches[OF_PROFILE_STEPS] = {};
};

Profiler g_prof;

// Runs `launch` with profiling events attached to its dispatch (start as the kernel
// begins, stop as it ends).  A repeatable launch (one that gives the same results when
// issued again, or whose only accumulation the caller scales back: it does not draw
// from a queue) is issued `repeat` times back to back, start on the first dispatch and
// stop on the last; *issued reports how many times it ran.
template <class F>
hipError_t timed(int step, hipStream_t s, F&& launch, bool repeatable = false,
                 int* issued = nullptr) {
  if (issued) *issued = 1;
  if (!g_prof.on) return launch();
  std::lock_guard<std::mutex> lk(g_prof.mu);
  const int times = repeatable ? g_prof.repeat : 1;
  g_prof.launches[step] += times;
  if (g_prof.used >= kEventPool) {
    g_prof.launches[step] += 1 - times;
    return launch();
  }
  if (issued) *issued = times;
  const int k = g_prof.used++;
  g_prof.step_of[k] = step;
  hipError_t e = hipSuccess;
  for (int r = 0; r < times && e == hipSuccess; ++r) {
    set_launch_events(r == 0 ? g_prof.ev[2 * k] : nullptr,
                      r == times - 1 ? g_prof.ev[2 * k + 1] : nullptr);
    e = launch();
  }
  set_launch_events(nullptr, nullptr);
  return e;
}

// Last plan built on each workspace (by any call's prologue), for calls that keep their
// plan resident: the prologue is skipped when the workspace already holds this plan.
struct ResidentPlans {
  std::mutex mu;
  const void* ws[64] = {};
  uint64_t sig[64] = {};
  int next = 0;
};

ResidentPlans g_resident;

bool resident_holds(const void* ws, uint64_t sig) {
  std::lock_guard<std::mutex> lk(g_resident.mu);
  for (int i = 0; i < 64; ++i)
    if (g_resident.ws[i] == ws) return g_resident.sig[i] == sig;
  return false;
}

void resident_record(const void* ws, uint64_t sig) {
  std::lock_guard<std::mutex> lk(g_resident.mu);
  for (int i = 0; i < 64; ++i)
    if (g_resident.ws[i] == ws) {
      g_resident.sig[i] = sig;
      return;
    }
  g_resident.ws[g_resident.next] = ws;
  g_resident.sig[g_resident.next] = sig;
  g_resident.next = (g_resident.next + 1) % 64;
}

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return OF_EHIP;
}

int check_params(const of_params* p) {
  if (!p) return OF_EINVAL;
  if (p->n_levels < 1 || p->n_levels > kMaxLevels) return OF_EINVAL;
  if (p->scale_den < 1 || p->scale_num <= p->scale_den || p->scale_num > 8) return OF_EINVAL;
  if (p->fast_t < 1 || p->fast_t > 255) return OF_EINVAL;
  if (p->fast_t_min < 1 || p->fast_t_min > p->fast_t) return OF_EINVAL;
  if (p->cell != 0 && (p->cell < 8 || p->cell > 128)) return OF_EINVAL;
  if (p->n_features < 1 || p->n_features > 65536) return OF_EINVAL;
  if (p->harris_block != 7) return OF_EINVAL;
  if (p->patch_radius < 4 || p->patch_radius > 48) return OF_EINVAL;
  return OF_OK;
}

int check_frame_size(int32_t W, int32_t H, const of_params& p) {
  if (W < 1 || H < 1 || W > 16384 || H > 16384) return OF_EINVAL;
  FrameGeom g;
  frame_geom(W, H, p, &g);
  for (int l = 0; l < p.n_levels; ++l) {
    if (g.W[l] < 2 * p.patch_radius + 1 || g.H[l] < 2 * p.patch_radius + 1) return OF_EINVAL;
    if (g.quota[l] > kMaxQuota) return OF_EINVAL;
  }
  return OF_OK;
}

int check_image(const of_image* im, const of_params& p) {
  if (!im || !im->data) return OF_EINVAL;
  if (im->stride < im->width || im->stride >= (1 << 24)) return OF_EINVAL;  // 24-bit row math
  int st = check_frame_size(im->width, im->height, p);
  if (st) return st;
  // The fused resample addresses the frame by 32-bit signed offsets from its first byte.
  if ((int64_t)im->stride * (im->height - 1) + im->width > (int64_t)INT32_MAX) return OF_EINVAL;
  return OF_OK;
}

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
  }
  return cus;
}

// Defaults: 256 x 16 segment-test tiles; Harris/NMS tiles of about 240 x 30 pixels
// (whole cells), or 128 x 32 pixels when the level is one cell.
Tune default_tune(const of_params& p) {
  Tune t;
  t.mark_words = 2;
  t.mark_rows = 56;
  if (p.cell > 0) {
    t.det_cx = 240 / p.cell > 0 ? 240 / p.cell : 1;
    t.det_cy = 30 / p.cell > 0 ? 30 / p.cell : 1;
  } else {
    t.det_cx = t.det_cy = 1;
  }
  t.det_w = 128;
  t.det_h = 32;
  // One block per tile by default: a shared queue counter hit from all eight XCDs
  // costs more than the hardware dispatcher on this chip (the tuner can still pick a
  // persistent grid).
  t.mark_grid = 0;
  t.det_grid = 0;
  t.pyr_pass = 0;
  t.mark_order = 1;  // XCD bands: measured faster on every workload here
  t.plan_resident = 0;
  t.det_order = 0;
  t.rank_cap = kRankCap;  // per call: set_rank_cap
  // narrower Harris tiles where large cells would exceed the LDS budget
  while (p.cell > 0 && t.det_cx > 1 &&
         det_lds(t, p.cell).bytes + base_table_bytes(kMaxEntries) > 65536)
    --t.det_cx;
  return t;
}

int resolve_tune(const of_tuning* user, const of_params& p, Tune* out) {
  Tune t = default_tune(p);
  if (user) {
    if (user->mark_words) t.mark_words = user->mark_words;
    if (user->mark_rows) t.mark_rows = user->mark_rows;
    if (user->det_cells_x) t.det_cx = user->det_cells_x;
    if (user->det_cells_y) t.det_cy = user->det_cells_y;
    if (user->det_w) t.det_w = user->det_w;
    if (user->det_h) t.det_h = user->det_h;
    if (user->mark_grid >= 0) t.mark_grid = user->mark_grid;
    if (user->det_grid >= 0) t.det_grid = user->det_grid;
    if (user->pyr_pass >= 0) t.pyr_pass = user->pyr_pass != 0;
    if (user->mark_order >= 0) t.mark_order = user->mark_order != 0;
    if (user->plan_resident >= 0) t.plan_resident = user->plan_resident != 0;
    if (user->det_order >= 0) t.det_order = user->det_order != 0;
  }
  if (t.mark_words < 1 || t.mark_words > 4 || t.mark_rows < 4 || t.mark_rows > 64)
    return OF_EINVAL;
  if (p.cell > 0) {
    if (t.det_cx < 1 || t.det_cy < 1 || t.det_cx * p.cell > kMaxDetW ||
        t.det_cy * p.cell > kMaxDetH)
      return OF_EINVAL;
  }
  // det_w, det_h even: tiles then start on the 2x2 blocks that own the output slots
  if (t.det_w < 8 || t.det_w > kMaxDetW || t.det_h < 8 || t.det_h > kMaxDetH ||
      (t.det_w & 1) || (t.det_h & 1))
    return OF_EINVAL;
  const int32_t bases = base_table_bytes(kMaxEntries);
  if (mark_lds(t).bytes + bases > 65536 || det_lds(t, p.cell).bytes + bases > 65536)
    return OF_EINVAL;
  *out = t;
  return OF_OK;
}

// The counting selection's cap for a call (Tune::rank_cap).  Ranking by counting takes
// C^2 compares per level of C candidate slots but runs every slot's wave at once, which is
// the shortest path while the call's counting work is small (up to a few 1080p frames:
// about 10M compares each); past that, the radix select (a few passes over C in one
// block per level, every level at once, then a count over the N_l it keeps) takes every
// level above kRankCapBusy slots.  On a single 1080p frame the radix path takes 60 us
// per call against 43.5 for counting; on 16 such frames 385 us against 422, and 2.07 ms
// against 2.65 on 16 frames of 3840 x 2160 (caps of 512 and 4096 were slower there).
// Levels with appended lists (whole-level cells past kRankCap) count no work here:
// their length is known only on the device, which takes the radix path when it
// exceeds the cap.
constexpr int64_t kRankWorkFew = 40000000;
constexpr int32_t kRankCapBusy = 128;

void set_rank_cap(const of_image* frames, int n, const of_params& p, Tune* t) {
  t->rank_cap = kRankCap;
  int64_t work = 0;
  for (int f = 0; f < n; ++f) {
    FrameGeom g;
    frame_geom(frames[f].width, frames[f].height, p, &g);
    for (int l = 0; l < p.n_levels; ++l) {
      EntrySize s;
      entry_size(g, p, *t, l, &s);
      if (p.cell == 0 && s.cand_cap > kRankCap) continue;
      const int64_t c = std::min<int64_t>(s.cand_cap, kRankCap);
      work += c * c;
    }
  }
  if (work > kRankWorkFew) t->rank_cap = kRankCapBusy;
}

struct CallPlan {
  WsLayout lay;
  EntrySize es[kMaxEntries];
  int64_t lvl_off[kMaxEntries];
  FrameGeom geo[kMaxBatch];
};

// Host-side planning state of one call (about 140 KB): a single static instance, held
// under its lock for the host part of a call, so that no call allocates host memory.
// Calls from several threads take turns for that part only; their launches overlap.
struct HostScratch {
  std::mutex mu;
  CallPlan c;
  PrologueArgs pa;
};

HostScratch g_host;

void plan_call(const of_image* frames, int n, const of_params& p, const Tune& t, CallPlan* c) {
  memset(&c->lay, 0, sizeof(c->lay));
  int64_t lvl = 0;
  for (int f = 0; f < n; ++f) {
    frame_geom(frames[f].width, frames[f].height, p, &c->geo[f]);
    for (int l = 0; l < p.n_levels; ++l) {
      const int e = f * p.n_levels + l;
      entry_size(c->geo[f], p, t, l, &c->es[e]);
      c->lvl_off[e] = lvl;
      lvl += c->es[e].lvl_bytes;
      ws_layout_accumulate(&c->lay, c->es[e]);
    }
  }
  ws_layout_finish(&c->lay);
}

int check_frames(const of_image* frames, int32_t n, const of_params* params) {
  int st = check_params(params);
  if (st) return st;
  if (!frames || n < 1 || n > kMaxBatch) return OF_EINVAL;
  for (int f = 0; f < n; ++f) {
    st = check_frame_size(frames[f].width, frames[f].height, *params);
    if (st) return st;
  }
  return OF_OK;
}

void fill_prologue(PrologueArgs* pa, const of_image* frames, int n, const of_params& p,
                   const Tune& t, void* ws, const WsLayout& lay, of_keypoint* out,
                   const int64_t* out_offset, int32_t* counts) {
  memset(pa, 0, sizeof(*pa));
  pa->p = p;
  pa->t = t;
  pa->n = n;
  for (int f = 0; f < n; ++f) {
    pa->f[f].data = frames[f].data;
    pa->f[f].w = frames[f].width;
    pa->f[f].h = frames[f].height;
    pa->f[f].stride = frames[f].stride;
    pa->f[f].out_off = out_offset ? out_offset[f] : 0;
  }
  pa->ws = (uint8_t*)ws;
  pa->lay = lay;
  pa->out = out;
  pa->counts = counts;
  // FNV-1a over every byte the plan depends on (the struct is zero-filled first, so
  // padding is deterministic); the prologue rebuilds the plan when this changes.
  uint64_t h = 1469598103934665603ull;
  const uint8_t* b = (const uint8_t*)pa;
  for (size_t i = 0; i < sizeof(*pa); ++i) h = (h ^ b[i]) * 1099511628211ull;
  pa->sig = h ^ 0x4f46504c414e3031ull;
}

int prologue_grid(const WsLayout& lay) {
  const int64_t items = lay.flag_bytes / 16 + 2 * (int64_t)lay.n_entries;
  const int64_t g = 1 + items / (1024 * 8);
  return (int)(g < 64 ? g : 64);
}

KArgs kargs(void* ws, const WsLayout& lay, const Tune& t, const of_params& p) {
  KArgs k;
  memset(&k, 0, sizeof(k));
  uint8_t* b = (uint8_t*)ws;
  k.plan = (LevelPlan*)(b + lay.off_plan);
  k.mark_base = (const int32_t*)(b + lay.off_mark_base);
  k.det_base = (const int32_t*)(b + lay.off_det_base);
  k.sel_base = (const int32_t*)(b + lay.off_sel_base);
  k.rank_base = (const int32_t*)(b + lay.off_rank_base);
  k.pyr_base = (const int32_t*)(b + lay.off_pyr_base);
  k.counters = (uint32_t*)(b + lay.off_counters);
  k.flags = b + lay.off_flags;
  k.flag_bytes = lay.flag_bytes;
  k.band_base = (const int32_t*)(b + lay.off_band_base);
  k.det_band_base = (const int32_t*)(b + lay.off_det_band_base);
  k.rank_path = 1;
  k.qctr = (uint32_t*)(b + lay.off_hdr);
  k.ws_sig = (const uint64_t*)(b + lay.off_hdr + 128);
  k.n_entries = lay.n_entries;
  k.entry = -1;
  k.cell = p.cell;
  k.t = t;
  k.ml = mark_lds(t);
  k.dl = det_lds(t, p.cell);
  return k;
}

enum BaseKind { kMarkTiles, kMarkBands, kDetTiles, kDetBands, kRankSlots, kSelSlots, kPyrBlocks };

// The launch's prefix table (units per entry), copied into the kernel arguments when the
// call has at most kSmallEntries entries; the kernels then skip loading it.
void set_small_bases(KArgs& k, const CallPlan& c, BaseKind kind) {
  const int n = c.lay.n_entries;
  k.small = n <= kSmallEntries;
  if (!k.small) return;
  // the tile kernels read row blockIdx % kXcds (their band, or a copy of row 0)
  const int rows = kind == kRankSlots || kind == kSelSlots || kind == kPyrBlocks ? 1 : kXcds;
  for (int r = 0; r < rows; ++r) {
    int32_t* b = k.sbase + r * (kSmallEntries + 1);
    int32_t acc = 0, rot = 0, drot = 0;
    for (int e = 0; e < n; ++e) {
      b[e] = acc;
      const EntrySize& s = c.es[e];
      switch (kind) {
        case kMarkTiles: acc += s.mark_tiles; break;
        case kMarkBands:
          acc += s.mark_tx * band_rows(s.mark_ty, rot, r);
          rot = (rot + s.mark_ty % kXcds) % kXcds;
          break;
        case kDetTiles: acc += s.det_tiles; break;
        case kDetBands:
          acc += s.det_tx * band_rows(s.det_ty, drot, r);
          drot = (drot + s.det_ty % kXcds) % kXcds;
          break;
        case kRankSlots: acc += s.rank_slots; break;
        case kSelSlots: acc += s.sel_slots; break;
        case kPyrBlocks: acc += s.pyr_blocks; break;
      }
    }
    b[n] = acc;
    for (int e = n + 1; e < kSmallEntries; ++e) b[e] = INT32_MAX;  // never reached
    b[kSmallEntries] = acc;
  }
}

// Level selection + orientation: ranks by counting for every level up to the call's
// rank cap; when some level can exceed it, the radix select lists the best N_l of each
// such level and a second counting launch ranks those lists.
hipError_t launch_selection(KArgs k, const CallPlan& c, hipStream_t stream) {
  const WsLayout& lay = c.lay;
  k.entry = -1;
  k.persistent = 0;
  set_small_bases(k, c, kRankSlots);
  // Stage each level's R' in LDS when every slot's wave of the call is resident at once
  // (latency then sets the time, and a staged level is ranked without round trips);
  // otherwise waves rank from memory and most stop early, which takes less work.
  int32_t widest = 0;  // largest level the rank path takes (appended lists: up to the cap)
  for (int i = 0; i < lay.n_entries; ++i) widest = std::max(widest, c.es[i].rank_slots);
  // (a staged copy is padded to a multiple of 256)
  k.sel_lds = std::min((int32_t)align_up(widest, 256), kSelLdsCap);
  const int64_t blocks_per_cu = std::min<int64_t>(8, 163840 / (8 * (int64_t)k.sel_lds + 4352));
  if ((int64_t)lay.rank_slots > (int64_t)device_cus() * 4 * blocks_per_cu) k.sel_lds = 0;
  // Besides ranking, the launch clears the cell flags and the segment-test queue counter
  // for the next call, so it keeps enough blocks for that (8 16-byte stores per thread)
  // also when every level takes the radix path and nothing is ranked here.
  const int64_t clear_blocks = (lay.flag_bytes / 16 + 8 * 256 - 1) / (8 * 256);
  const int32_t slots =
      (int32_t)std::max<int64_t>(lay.rank_slots, 4 * std::max<int64_t>(clear_blocks, 1));
  hipError_t e = timed(4, stream, [&] { return launch_select_orient(k, slots, stream); }, true);
  if (e == hipSuccess && lay.sel_slots > 0) {
    k.total = lay.n_entries;
    e = timed(4, stream, [&] { return launch_select(k, lay.n_entries, stream); });
    if (e == hipSuccess) {
      // the lists (at most N_l <= kSortCap long) ranked by the same kernel, staged
      k.from_sel = 1;
      k.flags = nullptr;  // cleared by the first launch
      k.rank_base = k.sel_base;
      set_small_bases(k, c, kSelSlots);
      int32_t longest = 0;
      for (int i = 0; i < lay.n_entries; ++i) longest = std::max(longest, c.es[i].sel_slots);
      k.sel_lds = std::min((int32_t)align_up(longest, 256), kSortCap);
      e = timed(5, stream, [&] { return launch_select_orient(k, lay.sel_slots, stream); }, true);
    }
  }
  return e;
}

}  // namespace

extern "C" {

int of_pyramid_desc_get(int32_t width, int32_t height, const of_params* params,
                        of_pyramid_desc* out) {
  int st = check_params(params);
  if (st) return st;
  if (!out) return OF_EINVAL;
  st = check_frame_size(width, height, *params);
  if (st) return st;
  FrameGeom g;
  frame_geom(width, height, *params, &g);
  memset(out, 0, sizeof(*out));
  out->n_levels = params->n_levels;
  int64_t off = 0;
  for (int l = 0; l < params->n_levels; ++l) {
    out->width[l] = g.W[l];
    out->height[l] = g.H[l];
    out->stride[l] = level_stride(g.W[l]);
    out->quota[l] = g.quota[l];
    out->offset[l] = off;
    off += align_up((int64_t)out->stride[l] * g.H[l], 256);
  }
  out->total_bytes = off;
  return OF_OK;
}

int of_pyramid_build(const of_image* in, const of_params* params, uint8_t* levels,
                     hipStream_t stream) {
  of_pyramid_desc d;
  int st = check_params(params);
  if (st) return st;
  st = check_image(in, *params);
  if (st) return st;
  if (!levels) return OF_EINVAL;
  st = of_pyramid_desc_get(in->width, in->height, params, &d);
  if (st) return st;
  PyrArgs a;
  memset(&a, 0, sizeof(a));
  a.src = in->data;
  a.src_w = in->width;
  a.src_h = in->height;
  a.src_stride = in->stride;
  for (int l = 0; l < d.n_levels; ++l) {
    a.lv[l].dst = levels + d.offset[l];
    a.lv[l].w = d.width[l];
    a.lv[l].h = d.height[l];
    a.lv[l].stride = d.stride[l];
  }
  hipError_t e = launch_pyramid(a, d.n_levels, d.width[0], d.height[0], stream);
  return e == hipSuccess ? OF_OK : hip_fail(e);
}

int of_workspace_size(const of_image* frames, int32_t n, const of_params* params, size_t* bytes) {
  if (!bytes) return OF_EINVAL;
  int st = check_frames(frames, n, params);
  if (st) return st;
  std::lock_guard<std::mutex> lk(g_host.mu);
  CallPlan* cp = &g_host.c;  // the layout does not depend on the tuning
  plan_call(frames, n, *params, default_tune(*params), cp);
  *bytes = (size_t)cp->lay.total;
  return OF_OK;
}

int of_tuning_default(const of_image* frames, int32_t n, const of_params* params,
                      of_tuning* out) {
  if (!out) return OF_EINVAL;
  int st = check_frames(frames, n, params);
  if (st) return st;
  const Tune t = default_tune(*params);
  out->mark_words = t.mark_words;
  out->mark_rows = t.mark_rows;
  out->det_cells_x = t.det_cx;
  out->det_cells_y = t.det_cy;
  out->det_w = t.det_w;
  out->det_h = t.det_h;
  out->mark_grid = t.mark_grid;
  out->det_grid = t.det_grid;
  out->pyr_pass = t.pyr_pass;
  out->mark_order = t.mark_order;
  out->plan_resident = t.plan_resident;
  out->det_order = t.det_order;
  return OF_OK;
}

int of_detect(const of_image* in, const of_params* params, void* ws, size_t ws_bytes,
              of_keypoint* out, int32_t cap, int32_t* count, hipStream_t stream) {
  int st = check_params(params);
  if (st) return st;
  st = check_image(in, *params);
  if (st) return st;
  if (!ws || !out || !count || cap < params->n_features) return OF_EINVAL;
  const of_params& p = *params;
  Tune t = default_tune(p);
  set_rank_cap(in, 1, p, &t);
  std::lock_guard<std::mutex> lk(g_host.mu);
  CallPlan* c = &g_host.c;
  plan_call(in, 1, p, t, c);
  if ((size_t)c->lay.total > ws_bytes) return OF_ENOSPACE;
  PrologueArgs* pa = &g_host.pa;
  fill_prologue(pa, in, 1, p, t, ws, c->lay, out, nullptr, count);
  hipError_t e = timed(0, stream, [&] { return launch_prologue(*pa, prologue_grid(c->lay), stream); });
  resident_record(ws, pa->sig);
  const uint64_t sig = pa->sig;
  const int L = p.n_levels;
  // levels 1.. from the input frame, one launch per level
  for (int l = 1; l < L && e == hipSuccess; ++l) {
    PyrArgs a;
    memset(&a, 0, sizeof(a));
    a.src = in->data;
    a.src_w = in->width;
    a.src_h = in->height;
    a.src_stride = in->stride;
    a.lv[0].dst = (uint8_t*)ws + c->lay.off_lvl + c->lvl_off[l];
    a.lv[0].w = c->geo[0].W[l];
    a.lv[0].h = c->geo[0].H[l];
    a.lv[0].stride = level_stride(c->geo[0].W[l]);
    e = timed(1, stream, [&] { return launch_pyramid(a, 1, a.lv[0].w, a.lv[0].h, stream); }, true);
  }
  KArgs k = kargs(ws, c->lay, t, p);
  k.sig = sig;
  k.persistent = 0;
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    k.entry = l;
    k.total = c->es[l].mark_tiles;
    e = timed(2, stream, [&] { return launch_mark(k, false, k.total, stream); }, true);
  }
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    k.entry = l;
    k.total = c->es[l].det_tiles;
    int issued = 1;
    e = timed(3, stream, [&] { return launch_detect(k, k.total, stream); }, true, &issued);
    if (e == hipSuccess && issued > 1) e = launch_scale_counters(k, issued, stream);
  }
  if (e == hipSuccess) e = launch_selection(k, *c, stream);
  return e == hipSuccess ? OF_OK : hip_fail(e);
}

}  // extern "C"

namespace {

// Validation of a batched call's arguments (everything but the workspace), on the host
// before any launch.
int check_batch(const of_image* frames, int32_t n, const of_params* params, of_keypoint* out,
                const int64_t* out_offset, int32_t cap_per_frame, int32_t* counts,
                const of_tuning* tuning, Tune* t) {
  int st = check_frames(frames, n, params);
  if (st) return st;
  for (int f = 0; f < n; ++f) {
    st = check_image(&frames[f], *params);
    if (st) return st;
  }
  if (!out || !out_offset || !counts || cap_per_frame < params->n_features) return OF_EINVAL;
  st = resolve_tune(tuning, *params, t);
  if (st) return st;
  set_rank_cap(frames, n, *params, t);
  return OF_OK;
}

// The batched path on a workspace of ws_bytes (the caller holds g_host.mu; c holds the
// call's plan).
int detect_batch_planned(const of_image* frames, int32_t n, const of_params& p, const Tune& t,
                         CallPlan* c, void* ws, of_keypoint* out, const int64_t* out_offset,
                         int32_t* counts, hipStream_t stream) {
  PrologueArgs* pa = &g_host.pa;
  fill_prologue(pa, frames, n, p, t, ws, c->lay, out, out_offset, counts);
  const uint64_t sig = pa->sig;
  hipError_t e = hipSuccess;
  if (!(t.plan_resident && resident_holds(ws, sig))) {
    e = timed(0, stream, [&] { return launch_prologue(*pa, prologue_grid(c->lay), stream); });
    resident_record(ws, sig);
  }
  KArgs k = kargs(ws, c->lay, t, p);
  k.sig = sig;
  k.frame_counts = counts;
  k.n_frames = n;
  const bool fused = !t.pyr_pass || c->lay.pyr_blocks == 0;
  if (e == hipSuccess && !fused) {
    k.total = c->lay.pyr_blocks;
    set_small_bases(k, *c, kPyrBlocks);
    e = timed(1, stream, [&] { return launch_pyramid_batch(k, c->lay.pyr_blocks, stream); }, true);
  }
  if (e == hipSuccess) {
    k.total = c->lay.mark_tiles;
    k.persistent = t.mark_grid > 0 && t.mark_grid < k.total;
    set_small_bases(k, *c, kMarkTiles);
    if (!k.persistent && t.mark_order == 1) {
      int32_t widest = 0;
      for (int b = 0; b < kXcds; ++b) widest = std::max(widest, c->lay.band_tiles[b]);
      k.bands = 1;
      k.total = kXcds * widest;
      set_small_bases(k, *c, kMarkBands);
    }
    // A grid that the device holds at once (launch bounds: 5 blocks per CU) runs its
    // tiles last first.
    k.mark_rev = !k.persistent && (int64_t)k.total <= (int64_t)device_cus() * 5;
    e = timed(2, stream, [&] { return launch_mark(k, fused, k.persistent ? t.mark_grid : k.total, stream); },
              !k.persistent);
    k.bands = 0;
    k.mark_rev = 0;
  }
  if (e == hipSuccess) {
    k.total = c->lay.det_tiles;
    set_small_bases(k, *c, kDetTiles);
    k.persistent = t.det_grid > 0 && t.det_grid < k.total;
    if (!k.persistent && t.det_order == 1) {
      int32_t widest = 0;
      for (int b = 0; b < kXcds; ++b) widest = std::max(widest, c->lay.det_band_tiles[b]);
      k.bands = 1;
      k.total = kXcds * widest;
      set_small_bases(k, *c, kDetBands);
    }
    // A grid that the device holds at once (launch bounds: 4 blocks per CU) runs its
    // tiles last first.
    k.det_rev = !k.persistent && (int64_t)k.total <= (int64_t)device_cus() * 4;
    // Repeated for profiling only without a persistent grid; its candidate counters are
    // then divided back by the number of issues.
    int issued = 1;
    e = timed(3, stream, [&] { return launch_detect(k, k.persistent ? t.det_grid : k.total, stream); },
              !k.persistent, &issued);
    if (e == hipSuccess && issued > 1) e = launch_scale_counters(k, issued, stream);
    k.bands = 0;
    k.det_rev = 0;
  }
  if (e == hipSuccess) e = launch_selection(k, *c, stream);
  return e == hipSuccess ? OF_OK : hip_fail(e);
}

}  // namespace

extern "C" {

int of_detect_batch(const of_image* frames, int32_t n, const of_params* params, void* ws,
                    size_t ws_bytes, of_keypoint* out, const int64_t* out_offset,
                    int32_t cap_per_frame, int32_t* counts, const of_tuning* tuning,
                    hipStream_t stream) {
  Tune t;
  int st = check_batch(frames, n, params, out, out_offset, cap_per_frame, counts, tuning, &t);
  if (st) return st;
  if (!ws) return OF_EINVAL;
  std::lock_guard<std::mutex> lk(g_host.mu);
  CallPlan* c = &g_host.c;
  plan_call(frames, n, *params, t, c);
  if ((size_t)c->lay.total > ws_bytes) return OF_ENOSPACE;
  return detect_batch_planned(frames, n, *params, t, c, ws, out, out_offset, counts, stream);
}

int of_detect_batch_scratch(const of_image* frames, int32_t n, const of_params* params,
                            of_keypoint* out, const int64_t* out_offset, int32_t cap_per_frame,
                            int32_t* counts, const of_tuning* tuning, hipStream_t stream) {
  Tune t;
  int st = check_batch(frames, n, params, out, out_offset, cap_per_frame, counts, tuning, &t);
  if (st) return st;
  std::lock_guard<std::mutex> lk(g_host.mu);
  CallPlan* c = &g_host.c;
  plan_call(frames, n, *params, t, c);
  if ((uint64_t)c->lay.total > (uint64_t)OF_SCRATCH_BYTES) return OF_ENOSPACE;
  void* ws = nullptr;
  const hipError_t e = scratch_workspace(&ws);
  if (e != hipSuccess) return hip_fail(e);
  return detect_batch_planned(frames, n, *params, t, c, ws, out, out_offset, counts, stream);
}

int of_candidate_counts(const of_image* frames, int32_t n, const of_params* params,
                        const void* ws, int32_t* out, hipStream_t stream) {
  int st = check_frames(frames, n, params);
  if (st) return st;
  if (!ws || !out) return OF_EINVAL;
  std::lock_guard<std::mutex> lk(g_host.mu);
  CallPlan* c = &g_host.c;
  plan_call(frames, n, *params, default_tune(*params), c);
  const uint32_t* counters = (const uint32_t*)((const uint8_t*)ws + c->lay.off_counters);
  hipError_t e = launch_sum_fast_counts(counters, c->lay.n_entries, out, stream);
  return e == hipSuccess ? OF_OK : hip_fail(e);
}

static bool ab_level_ok(const of_image& L) {
  return L.data && L.width >= 1 && L.height >= 1 && L.width <= 16384 && L.height <= 16384 &&
         L.stride >= L.width;
}

int of_ablate_fast(const of_image* levels, int32_t n, int32_t t, int32_t border,
                   int32_t variant, uint8_t* const* outs, hipStream_t stream) {
  if (!levels || !outs || n < 1 || n > kAbMaxLevels) return OF_EINVAL;
  if (t < 1 || t > 255 || border < 3 || variant < 0 || variant > OF_AB_FAST_MASKS_PRETEST_LDS)
    return OF_EINVAL;
  AbArgs a;
  memset(&a, 0, sizeof(a));
  a.n_levels = n;
  a.t = t;
  a.B = border;
  int32_t base = 0;
  for (int i = 0; i < n; ++i) {
    if (!ab_level_ok(levels[i]) || !outs[i]) return OF_EINVAL;
    AbLevel& L = a.lv[i];
    L.img = levels[i].data;
    L.out = outs[i];
    L.W = levels[i].width;
    L.H = levels[i].height;
    L.stride = levels[i].stride;
    L.base = base;
    base += ablate_fast_blocks(variant, L.W, L.H);
  }
  hipError_t e = timed(6, stream, [&] { return launch_ablate_fast(a, variant, stream); }, true);
  return e == hipSuccess ? OF_OK : hip_fail(e);
}

int of_ablate_harris(const of_image* levels, int32_t n, const uint32_t* const* pos,
                     const int32_t* counts, int32_t variant, int64_t* const* outs,
                     hipStream_t stream) {
  if (!levels || !outs || n < 1 || n > kAbMaxLevels) return OF_EINVAL;
  if (variant < 0 || variant > OF_AB_HARRIS_DENSE_SLIDING) return OF_EINVAL;
  const bool dense = variant == OF_AB_HARRIS_DENSE_SLIDING;
  if (!dense && (!pos || !counts)) return OF_EINVAL;
  AbArgs a;
  memset(&a, 0, sizeof(a));
  a.n_levels = n;
  int32_t base = 0;
  for (int i = 0; i < n; ++i) {
    if (!ab_level_ok(levels[i]) || !outs[i]) return OF_EINVAL;
    AbLevel& L = a.lv[i];
    L.img = levels[i].data;
    L.out = outs[i];
    L.W = levels[i].width;
    L.H = levels[i].height;
    L.stride = levels[i].stride;
    if (!dense) {
      if (counts[i] < 0 || (counts[i] > 0 && !pos[i])) return OF_EINVAL;
      L.pos = pos[i];
      L.n = counts[i];
    }
    L.base = base;
    base += ablate_harris_blocks(variant, L.W, L.H, L.n);
  }
  if (base == 0) return OF_OK;  // no positions to score
  hipError_t e = timed(7, stream, [&] { return launch_ablate_harris(a, variant, stream); }, true);
  return e == hipSuccess ? OF_OK : hip_fail(e);
}

int of_brief_tables(const int8_t* pattern, int8_t* rot, int32_t* centres) {
  if (!pattern || !rot || !centres) return OF_EINVAL;
  // std::nearbyint rounds half to even in the default rounding mode
  const double turn = 6.283185307179586476925286766559;
  for (int k = 0; k < 15; ++k) {
    double c = std::cos(turn * k / 30.0), s = std::sin(turn * k / 30.0);
    if (k == 0) {
      c = 1.0;
      s = 0.0;
    } else if (k == 5 || k == 10) {
      c = k == 5 ? 0.5 : -0.5;  // the rational cosines, exactly
    }
    centres[2 * k] = (int32_t)std::nearbyint(16384.0 * c);
    centres[2 * k + 1] = (int32_t)std::nearbyint(16384.0 * s);
    centres[2 * (k + 15)] = -centres[2 * k];
    centres[2 * (k + 15) + 1] = -centres[2 * k + 1];
    for (int i = 0; i < 256; ++i) {
      for (int j = 0; j < 2; ++j) {
        const double px = pattern[4 * i + 2 * j], py = pattern[4 * i + 2 * j + 1];
        const int8_t rx = (int8_t)std::nearbyint(c * px - s * py);
        const int8_t ry = (int8_t)std::nearbyint(s * px + c * py);
        int8_t* a = rot + ((size_t)k * 256 + i) * 4 + 2 * j;
        int8_t* b = rot + ((size_t)(k + 15) * 256 + i) * 4 + 2 * j;
        a[0] = rx;
        a[1] = ry;
        b[0] = (int8_t)-rx;  // half a turn further: exact negation
        b[1] = (int8_t)-ry;
      }
    }
  }
  return OF_OK;
}

int of_describe(const of_image* frames, int32_t n, const of_params* params,
                const of_tuning* tuning, const void* ws, const of_keypoint* kps,
                const int64_t* kp_offset, const int32_t* counts, const int8_t* rot,
                const int32_t* centres, uint8_t* desc, hipStream_t stream) {
  int st = check_frames(frames, n, params);
  if (st) return st;
  for (int f = 0; f < n; ++f) {
    st = check_image(&frames[f], *params);
    if (st) return st;
  }
  if (!ws || !kps || !kp_offset || !counts || !rot || !centres || !desc) return OF_EINVAL;
  // The descriptor reads the 31 x 31 patch around each keypoint, which stays inside its
  // level only when the detection border (the patch radius) is at least 15.
  if (params->patch_radius < 15) return OF_EINVAL;
  Tune t;
  st = resolve_tune(tuning, *params, &t);
  if (st) return st;
  set_rank_cap(frames, n, *params, &t);  // the plan of_detect_batch made for these frames
  std::lock_guard<std::mutex> lk(g_host.mu);
  CallPlan* c = &g_host.c;
  plan_call(frames, n, *params, t, c);
  PrologueArgs* pa = &g_host.pa;
  fill_prologue(pa, frames, n, *params, t, const_cast<void*>(ws), c->lay,
                const_cast<of_keypoint*>(kps), kp_offset, const_cast<int32_t*>(counts));
  DescArgs a;
  memset(&a, 0, sizeof(a));
  const uint8_t* b = (const uint8_t*)ws;
  a.plan = (const LevelPlan*)(b + c->lay.off_plan);
  a.ws_sig = (const uint64_t*)(b + c->lay.off_hdr + 128);
  a.sig = pa->sig;
  a.n = n;
  a.L = params->n_levels;
  a.cap = params->n_features;
  a.kps = kps;
  a.counts = counts;
  a.rot = rot;
  a.centres = centres;
  a.desc = desc;
  for (int f = 0; f < n; ++f) a.off[f] = kp_offset[f];
  hipError_t e = launch_describe(a, stream);
  return e == hipSuccess ? OF_OK : hip_fail(e);
}

int of_test_segment(const uint8_t* circles, int32_t n, int32_t t_lo, int32_t t_hi,
                    uint8_t* out, hipStream_t stream) {
  if (!circles || !out || n < 0 || t_lo < 1 || t_hi < t_lo || t_hi > 255) return OF_EINVAL;
  if (n == 0) return OF_OK;
  hipError_t e = launch_test_segment(circles, n, t_lo, t_hi, out, stream);
  return e == hipSuccess ? OF_OK : hip_fail(e);
}

int of_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (on && !g_prof.created) {
    for (int i = 0; i < 2 * kEventPool; ++i) {
      hipError_t e = hipEventCreate(&g_prof.ev[i]);
      if (e != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(g_prof.ev[j]);
        return hip_fail(e);
      }
    }
    g_prof.created = true;
  }
  g_prof.on = on != 0;
  g_prof.repeat = on > 1 ? on : 1;
  return OF_OK;
}

int of_profile_read(double* ms, int64_t* launches, int32_t n) {
  if (!ms || !launches || n < 0 || n > OF_PROFILE_STEPS) return OF_EINVAL;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  double acc[OF_PROFILE_STEPS] = {};
  for (int k = 0; k < g_prof.used; ++k) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(g_prof.ev[2 * k + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, g_prof.ev[2 * k], g_prof.ev[2 * k + 1]);
    if (e != hipSuccess) return hip_fail(e);
    acc[g_prof.step_of[k]] += t;
  }
  for (int i = 0; i < n; ++i) {
    ms[i] = acc[i];
    launches[i] = g_prof.launches[i];
  }
  g_prof.used = 0;
  for (int i = 0; i < OF_PROFILE_STEPS; ++i) g_prof.launches[i] = 0;
  return OF_OK;
}

const char* of_status_string(int status) {
  switch (status) {
    case OF_OK: return "ok";
    case OF_EINVAL: return "invalid argument (pointer, frame size, parameter, capacity or tuning)";
    case OF_ENOSPACE: return "workspace smaller than of_workspace_size()";
    case OF_EHIP: return "HIP launch failed (see of_last_hip_error)";
    default: return "unknown status";
  }
}

int of_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
