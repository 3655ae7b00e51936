/*
 * ofref.h -- CPU oracle for Oriented FAST detection over an image pyramid.
 *
 * TEST INFRASTRUCTURE ONLY.  The detector product never loads, links or calls this
 * library; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no code, header, table or constant with the GPU path.
 *
 * Every function is a plain, single-threaded definition in exact integers (the angle is
 * the only floating-point output, computed in double).  All pointers are host pointers;
 * images are 8-bit grey, row-major, with an explicit row stride in bytes.
 *
 * Steps and the passages they follow:
 *   pyramid      -- Sec. 1 (multi-level pyramid); each level is sampled from the input
 *                   frame itself, as in the related-work pyramid of Sec. 2.1
 *   segment test -- Eq. (1) and the "9 or more contiguous" rule of Sec. 3.1
 *   Harris       -- Sec. 3.2 (second-moment matrix, Score = det - k tr^2, k = 0.04), with
 *                   the 3x3 Sobel operator of Eq. (4) over a 7x7 window (Sec. 4.2)
 *   NMS, centroid -- the NMS and Centroid steps named in Fig. 1
 *   selection    -- per-cell and per-level top-N; the paper only says that Harris keeps
 *                   the most robust FAST points (Sec. 3.2), so the cell, quota and
 *                   tie-break rules are stated readings, given where each is used
 */
#ifndef OFREF_H
#define OFREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OFREF_MAX_LEVELS 16

typedef struct {
  int32_t n_levels;     /* 1..16 */
  int32_t scale_num;    /* level scale = scale_num / scale_den (6/5) */
  int32_t scale_den;
  int32_t fast_t;       /* segment-test threshold (20) */
  int32_t fast_t_min;   /* fallback threshold for cells without a fast_t corner (7) */
  int32_t cell;         /* cell side in level pixels; 0 = the whole level is one cell */
  int32_t n_features;   /* keypoints per frame over all levels */
  int32_t harris_block; /* Harris window side, 7 */
  int32_t patch_radius; /* orientation disk radius, also the detection border */
} ofref_params;

typedef struct {
  int32_t x, y, level; /* position in level coordinates */
  int32_t m10, m01;    /* intensity moments over the disk */
  int32_t pad;
  double angle;        /* atan2(m01, m10), radians */
  int64_t score;       /* R' = 25 (Sxx Syy - Sxy^2) - (Sxx + Syy)^2 */
} ofref_keypoint;

/* 0 if the parameters and frame size are accepted, -1 otherwise. */
int ofref_check(int32_t W, int32_t H, const ofref_params* p);

/* Per-level width, height, keypoint quota N_l and per-cell keep count K_l.
 * Any output pointer may be NULL.  Returns the level count or -1. */
int ofref_geometry(int32_t W, int32_t H, const ofref_params* p, int32_t* widths,
                   int32_t* heights, int32_t* quotas, int32_t* kcell, int32_t* ncells);

/* Bilinear resample of a W x H frame to Wl x Hl (dst row stride Wl). */
void ofref_resample(const uint8_t* src, int32_t W, int32_t H, int32_t stride,
                    uint8_t* dst, int32_t Wl, int32_t Hl);

/* 1 if the 16-bit circle mask (bit i = circle position i) holds 9 or more
 * cyclically contiguous ones. */
int ofref_run9(uint32_t mask16);

/* Segment test of pixel (x, y) at threshold t: 1 = corner. */
int ofref_segment_test(const uint8_t* img, int32_t stride, int32_t x, int32_t y, int32_t t);

/* Harris response R' at (x, y) over a block x block window. */
int64_t ofref_harris(const uint8_t* img, int32_t stride, int32_t x, int32_t y, int32_t block);

/* Moments over the disk of radius r centred on (x, y). */
/* Steered rBRIEF tables: for bin k of 30 (12 degrees each, angle measured like
 * atan2(m01, m10) with y down), the pattern's points rotated by 2 pi k / 30 and rounded
 * half to even: rot[k][i] = (x1, y1, x2, y2) of pair i; centres[k] = the bin's
 * direction, round(2^14 (cos, sin)).  The cosine is taken exactly where it is rational
 * (1/2 at 60 and 300 degrees, -1/2 at 120 and 240) and bins 15..29 are the exact
 * negations of bins 0..14.  pattern: 256 * 4 int8 (input). */
void ofref_brief_tables(const int8_t* pattern, int8_t* rot, int32_t* centres);

/* rBRIEF (the descriptor ORB attaches to each oriented keypoint, Sec. 1): the angle
 * bin is the k maximising m10 * centres[k][0] + m01 * centres[k][1] (ties: smallest k);
 * bit i of out (byte i / 8, bit i % 8) is set iff S(p + a_i) < S(p + b_i), with
 * (a_i, b_i) = rot[k][i] = (x1, y1, x2, y2) and S the 5x5 binomial smoothing
 * sum_{|u|,|v| <= 2} w_u w_v I(y + v, x + u), w = (1, 4, 6, 4, 1).  Every point of rot
 * must lie within 13 of (x, y) and (x, y) at least 15 from the border.  rot: 30 * 256
 * * 4 int8, centres: 30 * 2 int32 (inputs). */
void ofref_describe(const uint8_t* img, int32_t stride, int32_t x, int32_t y, int32_t m10,
                    int32_t m01, const int8_t* rot, const int32_t* centres, uint8_t* out);

void ofref_moments(const uint8_t* img, int32_t stride, int32_t x, int32_t y, int32_t r,
                   int32_t* m10, int32_t* m01);

/* One level: candidates, scores, survivors and the selected keypoints of that level
 * (sorted by R' desc, y asc, x asc; moments and angle not filled).  The map outputs
 * are Wl*Hl arrays (row stride Wl) and may be NULL; score_map is 0 off candidates.
 * cell_flags (may be NULL) receives one byte per cell: 1 = holds a fast_t corner.
 * Returns the number of keypoints written to out (at most n_keep), or -1. */
int ofref_level_detect(const uint8_t* lvl, int32_t Wl, int32_t Hl, int32_t stride,
                       const ofref_params* p, int32_t level, int32_t k_cell, int32_t n_keep,
                       uint8_t* cand_map, uint8_t* surv_map, int64_t* score_map,
                       uint8_t* cell_flags, ofref_keypoint* out);

/* Build level l (1 <= l < n_levels) of the pyramid into dst (row stride = level width). */
int ofref_pyramid_level(const uint8_t* img, int32_t W, int32_t H, int32_t stride,
                        const ofref_params* p, int32_t l, uint8_t* dst);

/* Whole pipeline for one frame.  Writes at most cap keypoints in the order
 * (level asc, R' desc, y asc, x asc).  Returns the count or -1. */
int ofref_detect(const uint8_t* img, int32_t W, int32_t H, int32_t stride,
                 const ofref_params* p, ofref_keypoint* out, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif
