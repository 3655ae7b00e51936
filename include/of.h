/*
 * of.h -- C ABI of the MI355X (gfx950) Oriented FAST detector.
 *
 * The library detects oriented FAST keypoints over a multi-level image pyramid and keeps
 * the ones the Harris response ranks highest, as in the Oriented-FAST stage of ORB that
 * the paper accelerates (Sec. 1: pyramid, FAST, Harris, NMS and centroid steps of Fig. 1).
 * Steps, in order:
 *   1. pyramid      -- levels at scale s^-l (s = scale_num/scale_den), each sampled from
 *                      the input frame with fixed-point bilinear weights;
 *   2. segment test -- Eq. (1) with the "9 or more contiguous" rule (Sec. 3.1), at
 *                      fast_t, or at fast_t_min inside cells that hold no fast_t corner;
 *   3. Harris       -- Sec. 3.2 / Eq. (4): 3x3 Sobel gradients summed over a 7x7 window,
 *                      ranked by R' = 25 det(M) - tr(M)^2 (= 25 x score with k = 0.04);
 *   4. 3x3 non-maximum suppression under the order (R' desc, y asc, x asc);
 *   5. per-cell top-K then per-level top-N_l, N_l proportional to level area;
 *   6. intensity-centroid orientation over a disk of radius patch_radius.
 * Every step is exact integer arithmetic except the final atan2 (float).
 *
 * Conventions for every entry point:
 *   - Pointers to pixels, keypoints, counts and workspace are DEVICE pointers unless the
 *     argument says "host".  The caller owns every buffer; the library never allocates,
 *     frees or synchronises on these calls and never throws across the ABI.
 *   - Work is queued on `stream` (a hipStream_t; NULL = the default stream) and is
 *     asynchronous; results are valid once the stream has reached that point.
 *     Calls contain no memset or memcpy nodes, so a sequence can be captured in a
 *     HIP graph and replayed.
 *   - Concurrent calls must use distinct workspaces.
 *   - Return 0 (OF_OK) or a negative status; of_status_string() explains it.  On
 *     OF_EHIP the HIP error of the failing launch is kept per thread (of_last_hip_error).
 */
#ifndef OF_H
#define OF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hipStream_t;

#define OF_OK 0
#define OF_EINVAL (-1)   /* bad argument: null pointer, size, parameter, capacity */
#define OF_ENOSPACE (-2) /* workspace smaller than of_workspace_size() */
#define OF_EHIP (-3)     /* a HIP launch failed */

#define OF_MAX_LEVELS 16
#define OF_MAX_BATCH 64  /* frames per of_detect_batch call */

/* 8-bit grey frame, row-major, `stride` bytes between rows (width <= stride < 2^24).
 * 1 <= width, height <= 16384, and the frame spans at most 2^31 - 1 bytes:
 * stride * (height - 1) + width <= 2147483647 (else OF_EINVAL from every call that
 * reads frame pixels). */
typedef struct {
  const uint8_t* data;
  int32_t width, height, stride;
} of_image;

/* Detector parameters.  Accepted ranges (else OF_EINVAL):
 *   n_levels 1..16; 1 <= scale_den < scale_num <= 8;
 *   fast_t 1..255; 1 <= fast_t_min <= fast_t (equal = no fallback);
 *   cell 0 (the whole level is one cell) or 8..128;
 *   n_features 1..65536, and every level quota N_l <= 4096;
 *   harris_block 7; patch_radius 4..48;
 *   every level at least 2*patch_radius+1 pixels in both directions. */
typedef struct {
  int32_t n_levels;
  int32_t scale_num, scale_den; /* 6, 5 = scale 1.2 */
  int32_t fast_t, fast_t_min;   /* 20, 7 */
  int32_t cell;                 /* 30 */
  int32_t n_features;           /* keypoints per frame over all levels */
  int32_t harris_block;         /* 7 */
  int32_t patch_radius;         /* 15: orientation radius and detection border */
} of_params;

/* One keypoint, 32 bytes.  (x, y) are in the coordinates of `level`. */
typedef struct {
  int32_t x, y, level;
  int32_t m10, m01; /* intensity moments over the disk (y down) */
  float angle;      /* atan2(m01, m10), radians in (-pi, pi] */
  int64_t score;    /* R' */
} of_keypoint;

/* Pyramid layout as written by of_pyramid_build: level l is height[l] rows of
 * width[l] pixels, row stride stride[l], starting at byte offset[l] of the buffer.
 * quota[l] is the level's keypoint quota N_l. */
typedef struct {
  int32_t n_levels;
  int32_t width[OF_MAX_LEVELS], height[OF_MAX_LEVELS], stride[OF_MAX_LEVELS];
  int32_t quota[OF_MAX_LEVELS];
  int64_t offset[OF_MAX_LEVELS];
  int64_t total_bytes;
} of_pyramid_desc;

/* Launch shape of the batched path (tile sizes, grid sizes, pyramid pass).  Tile fields
 * set to 0 take the default; grid, pyr_pass, mark_order, plan_resident and det_order
 * fields take the default when negative.
 * of_tuning_default() reports the defaults for a batch.  det_w and det_h must be even. */
typedef struct {
  int32_t mark_words; /* segment-test tile width in 64-pixel words, 1..4 */
  int32_t mark_rows;  /* segment-test tile height, 4..64 */
  int32_t det_cells_x, det_cells_y; /* Harris/NMS tile in cells (cell > 0); w*cell <= 256, h*cell <= 128 */
  int32_t det_w, det_h;             /* Harris/NMS tile in pixels when cell == 0; <= 256 x 128 */
  int32_t mark_grid;  /* workgroups of the persistent segment-test launch (0 = one per tile) */
  int32_t det_grid;   /* workgroups of the persistent Harris/NMS launch (0 = one per tile) */
  int32_t pyr_pass;   /* 1 = resample the levels in a pass of their own before the segment
                         test; 0 = the segment-test tiles resample their own pixels */
  int32_t mark_order; /* 1 = segment-test tiles ordered by XCD band (block b takes band
                         b % 8 of every level, so each XCD's L2 holds one band of each
                         frame); 0 = entry-major order.  Ignored with a persistent grid. */
  int32_t plan_resident; /* 1 = the caller keeps `ws` for this library's calls only: the
                         plan (built by a first launch whenever the frames, sizes,
                         parameters or tuning change) is then reused without that launch
                         when this workspace already holds it.  Every kernel checks the
                         plan's signature; if ws was overwritten in between, nothing is
                         computed and every frame's count reads -1.  0 = always re-check
                         with a launch of its own (any workspace). */
  int32_t det_order;  /* 1 = Harris/NMS tiles ordered by XCD band like the segment-test
                         tiles (block b takes band b % 8 of the tile rows of every level),
                         so with mark_order 1 a tile mostly reads pixels and bitmaps that
                         its own XCD's L2 holds from the segment test; 0 = entry-major
                         order.  Ignored with a persistent grid. */
} of_tuning;

/* Host only.  Level sizes, strides and offsets of the pyramid of a W x H frame. */
int of_pyramid_desc_get(int32_t width, int32_t height, const of_params* params,
                        of_pyramid_desc* out);

/* Build every level of `in` (level 0 copied) into `levels` (device, at least
 * desc.total_bytes, laid out as of_pyramid_desc_get reports). */
int of_pyramid_build(const of_image* in, const of_params* params, uint8_t* levels,
                     hipStream_t stream);

/* Host only.  Workspace bytes needed by of_detect (n = 1) or of_detect_batch for these
 * frames (host array of n descriptors; only width and height are read). */
int of_workspace_size(const of_image* frames, int32_t n, const of_params* params,
                      size_t* bytes);

/* Plain path: one frame, one launch per pyramid level and step.  Writes up to
 * n_features keypoints to `out` in the order (level asc, R' desc, y asc, x asc) and
 * their number to *count (device int32).  cap >= n_features is required.
 * ws: device workspace of ws_bytes >= of_workspace_size(in, 1, params). */
int of_detect(const of_image* in, const of_params* params, void* ws, size_t ws_bytes,
              of_keypoint* out, int32_t cap, int32_t* count, hipStream_t stream);

/* Batched path: n frames (host array of descriptors, 1 <= n <= OF_MAX_BATCH, sizes may
 * differ) through one launch per step over every level of every frame: the fused
 * pyramid + segment-test kernel, the Harris/NMS/cell-selection kernel (one block per
 * tile, or a persistent grid drawing tiles from a queue with the tuning's grids), and
 * the level selection with the orientation.  Frame i writes its keypoints (same order as
 * of_detect) at out + out_offset[i] (host array, in keypoints) and its count to
 * counts[i] (device).  cap_per_frame >= n_features is required and the caller keeps
 * the n output ranges disjoint.  `tuning` may be NULL (defaults). */
int of_detect_batch(const of_image* frames, int32_t n, const of_params* params, void* ws,
                    size_t ws_bytes, of_keypoint* out, const int64_t* out_offset,
                    int32_t cap_per_frame, int32_t* counts, const of_tuning* tuning,
                    hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): of_detect_batch on the library's own
 * static workspace of OF_SCRATCH_BYTES per device, held from the library's load until the
 * process ends, instead of a caller workspace.  Same arguments, results and errors as
 * of_detect_batch otherwise; OF_ENOSPACE when the batch needs a larger workspace than
 * OF_SCRATCH_BYTES (of_workspace_size tells).  The call allocates nothing: no device
 * memory, no host memory.  Every call on one device shares that device's workspace and
 * leaves its contents to the next call, so calls that overlap on one device race: issue
 * them on one stream, or order them.  A caller that owns the device can pass
 * plan_resident = 1 to skip re-planning repeated calls of one shape. */
#define OF_SCRATCH_BYTES (64 * 1024 * 1024)
int of_detect_batch_scratch(const of_image* frames, int32_t n, const of_params* params,
                            of_keypoint* out, const int64_t* out_offset, int32_t cap_per_frame,
                            int32_t* counts, const of_tuning* tuning, hipStream_t stream);

/* Host only.  The tuning of_detect_batch uses when given NULL (or zero fields). */
int of_tuning_default(const of_image* frames, int32_t n, const of_params* params,
                      of_tuning* out);

/* Statistics of the last detection on `ws` (same frames and params as that call):
 * copies, on `stream`, the number of FAST candidates of every (frame, level) -- pixels
 * of the valid region that pass the segment test (Sec. 3.1, Eq. 1) at their cell's
 * threshold -- to `out` (device int32, n * n_levels, frame-major).  Enqueue it after
 * the detection on the same stream.  OF_EINVAL on bad arguments. */
int of_candidate_counts(const of_image* frames, int32_t n, const of_params* params,
                        const void* ws, int32_t* out, hipStream_t stream);

/* Steered rBRIEF, the descriptor ORB attaches to each oriented keypoint (Sec. 1).
 *
 * of_brief_tables (host only): the 256 test pairs of `pattern` (host, 256 x 4 int8,
 * (x1, y1, x2, y2), every point within 13 of the origin) rotated to 30 angle bins of
 * 12 degrees, rounded half to even (host, rot: 30 x 256 x 4 int8), and the bins'
 * centre directions round(2^14 (cos, sin)) (host, centres: 30 x 2 int32).  The cosine is
 * exact where rational (bins 5 and 10) and bins 15..29 negate bins 0..14.
 *
 * of_describe: 256-bit descriptors of the keypoints of the last detection on `ws` (same
 * frames, params and tuning as that call, and the same kps / kp_offset / counts buffers
 * it wrote).  Per keypoint the bin is the k maximising m10 * centres[k][0] +
 * m01 * centres[k][1] (ties: smallest k), and bit i (byte i / 8, bit i % 8) is set iff
 * the 5x5 binomial sum (weights 1 4 6 4 1 per axis) on the keypoint's level at p + a_i
 * is smaller than at p + b_i, (a_i, b_i) = rot[k][i].  rot and centres are device copies
 * of of_brief_tables' output; desc (device) holds 32 bytes per keypoint slot, indexed
 * like kps.  Slots beyond counts[f] are not written; if ws does not hold the plan of
 * that detection nothing is written.  The 31 x 31 patch must lie inside the level, so
 * params->patch_radius (the detection border) must be at least 15.  OF_EINVAL on bad
 * arguments (nothing launched). */
int of_brief_tables(const int8_t* pattern, int8_t* rot, int32_t* centres);
int of_describe(const of_image* frames, int32_t n, const of_params* params,
                const of_tuning* tuning, const void* ws, const of_keypoint* kps,
                const int64_t* kp_offset, const int32_t* counts, const int8_t* rot,
                const int32_t* centres, uint8_t* desc, hipStream_t stream);

/* Ablation ladder: the same step computed the way earlier designs do, to measure the
 * gain of each design decision.  One call covers n pyramid levels (1 <= n <= 64, host
 * arrays of device image descriptors and device output pointers) in one launch.
 *
 * of_ablate_fast: the FAST-9 segment test (Sec. 3.1, Eq. 1: bright I_i >= I_p + t, dark
 * I_i <= I_p - t, corner iff 9 contiguous of the 16 circle pixels are bright or dark)
 * of every pixel of each level at threshold t:
 *   OF_AB_FAST_BRANCHY      one thread per pixel, global reads, a branch per circle
 *                           pixel counting the current run (the scheme Alg. 1 sketches)
 *   OF_AB_FAST_MASKS        global reads, bright and dark 16-bit masks and a shift-and
 *                           test for nine contiguous bits (the binary encoding of
 *                           Sec. 5.1 / Alg. 2)
 *   OF_AB_FAST_MASKS_LDS    the same reading 64 x 16 tiles staged in LDS
 *   OF_AB_FAST_MINMAX_LDS   the production scheme: LDS tiles, exact compass pre-test as a
 *                           wave-wide early-out, min/max windows
 *   OF_AB_FAST_MASKS_PRETEST_LDS  LDS tiles and the same compass pre-test, then the masks
 *                           and shift-and test of OF_AB_FAST_MASKS instead of min/max
 * outs[i] (device, width * height bytes, row pitch = width) gets 1 for corners of the
 * region x, y in [border, size - border) and 0 elsewhere.  border >= 3, 1 <= t <= 255.
 *
 * of_ablate_harris: R' = 25 (Sxx Syy - Sxy^2) - (Sxx + Syy)^2 over the 7x7 window of
 * Sobel gradients (Sec. 3.2, Eqs. 2-4) at counts[i] positions pos[i][k] = (y << 16 | x)
 * of level i (device):
 *   OF_AB_HARRIS_2D          one thread per position, 2D Sobel at each window pixel
 *   OF_AB_HARRIS_SEPARABLE   one thread per position, separable Sobel row by row (Eq. 4)
 *   OF_AB_HARRIS_GROUPS      8 lanes per position, one window row each
 * outs[i][k] (device int64) gets R', or 0 when x or y is closer than 4 to the border.
 *   OF_AB_HARRIS_DENSE_SLIDING  R' at every pixel by sliding column and row sums (the
 *                           structure of Alg. 3); pos and counts are ignored (may be NULL)
 *                           and outs[i] holds width * height int64.
 * Both return OF_EINVAL on bad arguments and launch nothing then. */
#define OF_AB_FAST_BRANCHY 0
#define OF_AB_FAST_MASKS 1
#define OF_AB_FAST_MASKS_LDS 2
#define OF_AB_FAST_MINMAX_LDS 3
#define OF_AB_FAST_MASKS_PRETEST_LDS 4
#define OF_AB_HARRIS_2D 0
#define OF_AB_HARRIS_SEPARABLE 1
#define OF_AB_HARRIS_GROUPS 2
#define OF_AB_HARRIS_DENSE_SLIDING 3
int of_ablate_fast(const of_image* levels, int32_t n, int32_t t, int32_t border,
                   int32_t variant, uint8_t* const* outs, hipStream_t stream);
int of_ablate_harris(const of_image* levels, int32_t n, const uint32_t* const* pos,
                     const int32_t* counts, int32_t variant, int64_t* const* outs,
                     hipStream_t stream);

/* Test entry point for the segment test alone: for each of n pixels, `circles` holds 17
 * bytes (the centre, then circle positions 1..16 clockwise from the top) and out[i]
 * gets bit 0 = corner at t_lo, bit 1 = corner at t_hi.  Device pointers. */
int of_test_segment(const uint8_t* circles, int32_t n, int32_t t_lo, int32_t t_hi,
                    uint8_t* out, hipStream_t stream);

/* Step timing.  While enabled (host call, not during graph capture), of_detect and
 * of_detect_batch attach two HIP events to each step launch's dispatch on their stream,
 * recorded as the kernel begins and as it ends:
 * step 0 prologue, 1 pyramid, 2 segment test, 3 Harris/NMS/cells, 4 level selection
 * (counting, and the radix select of levels past the call's rank cap), 5 ranking of the
 * radix-selected lists; the ablation entry points are steps 6 (segment test) and 7
 * (Harris).  of_profile_read waits for the recorded events, writes the summed
 * milliseconds and launch counts of the first n steps (host arrays) and clears them.
 * Events come from a fixed pool created on the first enable; launches beyond the pool
 * are not timed (their count is still reported in launches[]).  on > 1 also issues each
 * repeatable launch (pyramid, segment test and Harris/NMS without a persistent grid,
 * level selection: launches that give the same results when issued again, the
 * Harris/NMS candidate counters being divided back afterwards) `on` times back to back
 * between its events, so that ms / launches is the kernel's own duration; results are
 * unchanged.  on = 0 disables. */
#define OF_PROFILE_STEPS 8
int of_profile_enable(int on);
int of_profile_read(double* ms, int64_t* launches, int32_t n);

const char* of_status_string(int status);
int of_last_hip_error(void); /* hipError_t of the last OF_EHIP on this thread */

#ifdef __cplusplus
}
#endif
#endif
