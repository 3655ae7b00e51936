/*
 * ofref.c -- CPU oracle for Oriented FAST detection over an image pyramid.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU-baseline
 * leg of the benchmark, never by the detector product.  It shares no code with the
 * GPU path.  Plain C99, one thread, exact integer arithmetic (the angle is double).
 *
 * Each step is written as its plain definition, in the order the paper's Oriented-FAST
 * pipeline runs it (Fig. 1): pyramid, segment test, Harris response, NMS, selection,
 * centroid orientation.  Where the paper leaves a step undefined the reading used is
 * stated beside the code as "Reading:".
 */
#include "ofref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ geometry -- */

static int64_t ipow64(int64_t b, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}

/* Reading: level l has size round-half-up(n / s^l), s = num/den, in exact integers. */
static int32_t level_extent(int32_t n, int l, int32_t num, int32_t den) {
  int64_t a = ipow64(num, l), b = ipow64(den, l);
  return (int32_t)((2 * (int64_t)n * b + a) / (2 * a));
}

static int32_t ceil_div(int32_t a, int32_t b) { return (a + b - 1) / b; }

int ofref_check(int32_t W, int32_t H, const ofref_params* p) {
  if (!p) return -1;
  if (p->n_levels < 1 || p->n_levels > OFREF_MAX_LEVELS) return -1;
  if (p->scale_den < 1 || p->scale_num <= p->scale_den || p->scale_num > 8) return -1;
  if (p->fast_t < 1 || p->fast_t > 255) return -1;
  if (p->fast_t_min < 1 || p->fast_t_min > p->fast_t) return -1;
  if (p->cell != 0 && (p->cell < 8 || p->cell > 128)) return -1;
  if (p->n_features < 1 || p->n_features > 65536) return -1;
  if (p->harris_block != 7) return -1;
  if (p->patch_radius < 4 || p->patch_radius > 48) return -1;
  if (W < 1 || H < 1 || W > 16384 || H > 16384) return -1;
  for (int l = 0; l < p->n_levels; ++l) {
    int32_t wl = level_extent(W, l, p->scale_num, p->scale_den);
    int32_t hl = level_extent(H, l, p->scale_num, p->scale_den);
    if (wl < 2 * p->patch_radius + 1 || hl < 2 * p->patch_radius + 1) return -1;
  }
  return 0;
}

int ofref_geometry(int32_t W, int32_t H, const ofref_params* p, int32_t* widths,
                   int32_t* heights, int32_t* quotas, int32_t* kcell, int32_t* ncells) {
  if (ofref_check(W, H, p) != 0) return -1;
  int L = p->n_levels;
  int32_t w[OFREF_MAX_LEVELS], h[OFREF_MAX_LEVELS], q[OFREF_MAX_LEVELS];
  int64_t area_sum = 0;
  for (int l = 0; l < L; ++l) {
    w[l] = level_extent(W, l, p->scale_num, p->scale_den);
    h[l] = level_extent(H, l, p->scale_num, p->scale_den);
    area_sum += (int64_t)w[l] * h[l];
  }
  /* Reading: quota N_l = floor(N A_l / sum A) for l >= 1; level 0 takes the rest. */
  int32_t rest = p->n_features;
  for (int l = 1; l < L; ++l) {
    q[l] = (int32_t)(((int64_t)p->n_features * w[l] * h[l]) / area_sum);
    rest -= q[l];
  }
  q[0] = rest;
  for (int l = 0; l < L; ++l) {
    /* Reading: K_l = max(1, ceil(N_l / cells_l)); cell 0 = one cell per level. */
    int32_t nc = p->cell > 0 ? ceil_div(w[l], p->cell) * ceil_div(h[l], p->cell) : 1;
    int32_t k = (q[l] + nc - 1) / nc;
    if (k < 1) k = 1;
    if (widths) widths[l] = w[l];
    if (heights) heights[l] = h[l];
    if (quotas) quotas[l] = q[l];
    if (kcell) kcell[l] = k;
    if (ncells) ncells[l] = nc;
  }
  return L;
}

/* ------------------------------------------------------------------- pyramid -- */

/* Round-half-to-even of a / b for a >= 0, b > 0. */
static int32_t div_rhe(int64_t a, int64_t b) {
  int64_t q = a / b, r = a % b;
  if (2 * r > b || (2 * r == b && (q & 1))) ++q;
  return (int32_t)q;
}

/*
 * Reading: every level is sampled from the input frame (not from the level above).
 * Output pixel x sits at source position ((2x+1) W - Wl) / (2 Wl) (pixel centres
 * aligned).  Its integer part x0 and the fraction, rounded half-even to 1/256, give
 * Q8 weights; the four taps are blended in integers and rounded once.
 */
void ofref_resample(const uint8_t* src, int32_t W, int32_t H, int32_t stride,
                    uint8_t* dst, int32_t Wl, int32_t Hl) {
  for (int32_t y = 0; y < Hl; ++y) {
    int64_t ny = (int64_t)(2 * y + 1) * H - Hl, ey = 2 * (int64_t)Hl;
    int32_t y0 = (int32_t)(ny / ey);
    int32_t wy = div_rhe(256 * (ny - (int64_t)y0 * ey), ey);
    int32_t y1 = y0 + 1 < H ? y0 + 1 : H - 1;
    for (int32_t x = 0; x < Wl; ++x) {
      int64_t nx = (int64_t)(2 * x + 1) * W - Wl, ex = 2 * (int64_t)Wl;
      int32_t x0 = (int32_t)(nx / ex);
      int32_t wx = div_rhe(256 * (nx - (int64_t)x0 * ex), ex);
      int32_t x1 = x0 + 1 < W ? x0 + 1 : W - 1;
      int32_t p00 = src[(size_t)y0 * stride + x0], p01 = src[(size_t)y0 * stride + x1];
      int32_t p10 = src[(size_t)y1 * stride + x0], p11 = src[(size_t)y1 * stride + x1];
      int32_t top = (256 - wx) * p00 + wx * p01;
      int32_t bot = (256 - wx) * p10 + wx * p11;
      dst[(size_t)y * Wl + x] = (uint8_t)(((256 - wy) * top + wy * bot + 32768) >> 16);
    }
  }
}

int ofref_pyramid_level(const uint8_t* img, int32_t W, int32_t H, int32_t stride,
                        const ofref_params* p, int32_t l, uint8_t* dst) {
  int32_t w[OFREF_MAX_LEVELS], h[OFREF_MAX_LEVELS];
  if (ofref_geometry(W, H, p, w, h, NULL, NULL, NULL) < 0) return -1;
  if (l < 1 || l >= p->n_levels) return -1;
  ofref_resample(img, W, H, stride, dst, w[l], h[l]);
  return 0;
}

/* -------------------------------------------------------------- segment test -- */

/* The 16 circle positions (radius-3 Bresenham circle), clockwise from the top, y down. */
static const int kCircleDx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
static const int kCircleDy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

int ofref_run9(uint32_t mask16) {
  for (int s = 0; s < 16; ++s) {
    int all = 1;
    for (int k = 0; k < 9; ++k) all &= (int)((mask16 >> ((s + k) & 15)) & 1u);
    if (all) return 1;
  }
  return 0;
}

/* Eq. (1): circle pixel i is dark if I_i <= I_p - t, bright if I_i >= I_p + t.  The
 * pixel is a corner when 9 or more contiguous circle pixels are all dark or all bright. */
int ofref_segment_test(const uint8_t* img, int32_t stride, int32_t x, int32_t y, int32_t t) {
  int32_t ip = img[(size_t)y * stride + x];
  uint32_t dark = 0, bright = 0;
  for (int i = 0; i < 16; ++i) {
    int32_t ii = img[(size_t)(y + kCircleDy[i]) * stride + (x + kCircleDx[i])];
    if (ii <= ip - t) dark |= 1u << i;
    if (ii >= ip + t) bright |= 1u << i;
  }
  return ofref_run9(dark) || ofref_run9(bright);
}

/* -------------------------------------------------------------------- Harris -- */

/* Eq. (4): the 3x3 Sobel kernels, applied as sum_{i,j} K[j][i] I(x+i-1, y+j-1).
 * (The printed G_y has +1 in its top-right entry; the factorisation printed beside it,
 * [-1 0 1]^T [1 2 1], fixes that entry to -1.) */
static const int kSobelX[3][3] = {{-1, 0, 1}, {-2, 0, 2}, {-1, 0, 1}};
static const int kSobelY[3][3] = {{-1, -2, -1}, {0, 0, 0}, {1, 2, 1}};

/* Sec. 3.2: M summed over the window; Score = det(M) - k tr(M)^2 with k = 0.04.  The
 * oracle returns R' = 25 det - tr^2 = 25 Score, exact in int64 and ordered like Score. */
int64_t ofref_harris(const uint8_t* img, int32_t stride, int32_t x, int32_t y, int32_t block) {
  int32_t r = block / 2;
  int64_t sxx = 0, syy = 0, sxy = 0;
  for (int32_t wy = y - r; wy <= y + r; ++wy) {
    for (int32_t wx = x - r; wx <= x + r; ++wx) {
      int32_t gx = 0, gy = 0;
      for (int j = 0; j < 3; ++j) {
        for (int i = 0; i < 3; ++i) {
          int32_t v = img[(size_t)(wy + j - 1) * stride + (wx + i - 1)];
          gx += kSobelX[j][i] * v;
          gy += kSobelY[j][i] * v;
        }
      }
      sxx += (int64_t)gx * gx;
      syy += (int64_t)gy * gy;
      sxy += (int64_t)gx * gy;
    }
  }
  return 25 * (sxx * syy - sxy * sxy) - (sxx + syy) * (sxx + syy);
}

/* --------------------------------------------------------------- orientation -- */

/* Reading: intensity centroid over the disk dx^2 + dy^2 <= r^2 on the keypoint's level:
 * m10 = sum dx I, m01 = sum dy I (y down); angle = atan2(m01, m10). */
/* Round half to even of a double (the values here are small). */
static int32_t round_half_even(double v) {
  double f = floor(v);
  double r = v - f;
  int32_t i = (int32_t)f;
  if (r > 0.5) return i + 1;
  if (r < 0.5) return i;
  return (i % 2 == 0) ? i : i + 1;
}

void ofref_brief_tables(const int8_t* pattern, int8_t* rot, int32_t* centres) {
  const double pi = 3.14159265358979323846;
  for (int32_t k = 0; k < 15; ++k) {
    /* the exact value where the cosine is rational (0, 60, 120 degrees) */
    double c = k == 0 ? 1.0 : (k == 5 ? 0.5 : (k == 10 ? -0.5 : cos(2.0 * pi * k / 30.0)));
    double s = k == 0 ? 0.0 : sin(2.0 * pi * k / 30.0);
    centres[2 * k] = round_half_even(c * 16384.0);
    centres[2 * k + 1] = round_half_even(s * 16384.0);
    for (int32_t i = 0; i < 256; ++i) {
      for (int32_t j = 0; j < 4; j += 2) {
        const double x = pattern[4 * i + j], y = pattern[4 * i + j + 1];
        rot[((size_t)k * 256 + i) * 4 + j] = (int8_t)round_half_even(c * x - s * y);
        rot[((size_t)k * 256 + i) * 4 + j + 1] = (int8_t)round_half_even(s * x + c * y);
      }
    }
  }
  /* a half turn further: the exact negation (rounding half to even is odd-symmetric) */
  for (int32_t k = 15; k < 30; ++k) {
    centres[2 * k] = -centres[2 * (k - 15)];
    centres[2 * k + 1] = -centres[2 * (k - 15) + 1];
    for (int32_t i = 0; i < 256 * 4; ++i)
      rot[(size_t)k * 256 * 4 + i] = (int8_t)-rot[(size_t)(k - 15) * 256 * 4 + i];
  }
}

/* 5x5 binomial smoothing sum at (x, y): separable weights 1 4 6 4 1, not normalised
 * (the tests compare two sums, so no rounding enters). */
static int32_t smooth5(const uint8_t* img, int32_t stride, int32_t x, int32_t y) {
  static const int32_t w[5] = {1, 4, 6, 4, 1};
  int32_t s = 0;
  for (int32_t v = -2; v <= 2; ++v)
    for (int32_t u = -2; u <= 2; ++u)
      s += w[u + 2] * w[v + 2] * img[(size_t)(y + v) * stride + (x + u)];
  return s;
}

void ofref_describe(const uint8_t* img, int32_t stride, int32_t x, int32_t y, int32_t m10,
                    int32_t m01, const int8_t* rot, const int32_t* centres, uint8_t* out) {
  int32_t bin = 0;
  int64_t best = 0;
  for (int32_t k = 0; k < 30; ++k) {
    int64_t d = (int64_t)m10 * centres[2 * k] + (int64_t)m01 * centres[2 * k + 1];
    if (k == 0 || d > best) {
      best = d;
      bin = k;
    }
  }
  const int8_t* t = rot + (size_t)bin * 256 * 4;
  for (int32_t i = 0; i < 32; ++i) out[i] = 0;
  for (int32_t i = 0; i < 256; ++i) {
    int32_t s1 = smooth5(img, stride, x + t[4 * i], y + t[4 * i + 1]);
    int32_t s2 = smooth5(img, stride, x + t[4 * i + 2], y + t[4 * i + 3]);
    if (s1 < s2) out[i >> 3] |= (uint8_t)(1u << (i & 7));
  }
}

void ofref_moments(const uint8_t* img, int32_t stride, int32_t x, int32_t y, int32_t r,
                   int32_t* m10, int32_t* m01) {
  int32_t a = 0, b = 0;
  for (int32_t dy = -r; dy <= r; ++dy) {
    for (int32_t dx = -r; dx <= r; ++dx) {
      if (dx * dx + dy * dy > r * r) continue;
      int32_t v = img[(size_t)(y + dy) * stride + (x + dx)];
      a += dx * v;
      b += dy * v;
    }
  }
  *m10 = a;
  *m01 = b;
}

/* ------------------------------------------------------------------ ordering -- */

/* Reading: keypoints are ranked by R' (higher first), ties by y then x (smaller first). */
static int key_better(int64_t sa, int32_t ya, int32_t xa, int64_t sb, int32_t yb, int32_t xb) {
  if (sa != sb) return sa > sb;
  if (ya != yb) return ya < yb;
  return xa < xb;
}

static int cmp_keypoint(const void* pa, const void* pb) {
  const ofref_keypoint* a = (const ofref_keypoint*)pa;
  const ofref_keypoint* b = (const ofref_keypoint*)pb;
  if (a->level != b->level) return a->level < b->level ? -1 : 1;
  if (key_better(a->score, a->y, a->x, b->score, b->y, b->x)) return -1;
  if (key_better(b->score, b->y, b->x, a->score, a->y, a->x)) return 1;
  return 0;
}

/* --------------------------------------------------------------- level stage -- */

int ofref_level_detect(const uint8_t* lvl, int32_t Wl, int32_t Hl, int32_t stride,
                       const ofref_params* p, int32_t level, int32_t k_cell, int32_t n_keep,
                       uint8_t* cand_map, uint8_t* surv_map, int64_t* score_map,
                       uint8_t* cell_flags, ofref_keypoint* out) {
  const int32_t B = p->patch_radius;
  /* Reading: cells of side `cell` anchored at the level origin; cell 0 = one cell. */
  const int32_t cs = p->cell > 0 ? p->cell : (Wl > Hl ? Wl : Hl);
  const int32_t ncx = ceil_div(Wl, cs), ncy = ceil_div(Hl, cs);
  const size_t npx = (size_t)Wl * Hl;
  uint8_t* cand = (uint8_t*)calloc(npx, 1);
  int64_t* score = (int64_t*)calloc(npx, sizeof(int64_t));
  uint8_t* surv = (uint8_t*)calloc(npx, 1);
  uint8_t* flag = (uint8_t*)calloc((size_t)ncx * ncy, 1);
  ofref_keypoint* kept = NULL;
  int32_t n_out = 0;
  if (!cand || !score || !surv || !flag) goto fail;

  /* Reading: only pixels at least B from every edge are examined (B = patch radius). */
  /* Reading: a cell with no corner at fast_t is examined again at fast_t_min. */
  for (int32_t y = B; y <= Hl - 1 - B; ++y)
    for (int32_t x = B; x <= Wl - 1 - B; ++x)
      if (ofref_segment_test(lvl, stride, x, y, p->fast_t)) flag[(y / cs) * ncx + x / cs] = 1;
  for (int32_t y = B; y <= Hl - 1 - B; ++y) {
    for (int32_t x = B; x <= Wl - 1 - B; ++x) {
      int32_t t = flag[(y / cs) * ncx + x / cs] ? p->fast_t : p->fast_t_min;
      if (ofref_segment_test(lvl, stride, x, y, t)) {
        cand[(size_t)y * Wl + x] = 1;
        score[(size_t)y * Wl + x] = ofref_harris(lvl, stride, x, y, p->harris_block);
      }
    }
  }

  /* Reading: 3x3 NMS -- a candidate survives when it ranks above every candidate among
   * its 8 neighbours (non-candidates never suppress). */
  size_t n_surv = 0;
  for (int32_t y = 0; y < Hl; ++y) {
    for (int32_t x = 0; x < Wl; ++x) {
      size_t i = (size_t)y * Wl + x;
      if (!cand[i]) continue;
      int alive = 1;
      for (int32_t dy = -1; dy <= 1; ++dy) {
        for (int32_t dx = -1; dx <= 1; ++dx) {
          int32_t qx = x + dx, qy = y + dy;
          if ((dx == 0 && dy == 0) || qx < 0 || qy < 0 || qx >= Wl || qy >= Hl) continue;
          size_t j = (size_t)qy * Wl + qx;
          if (cand[j] && !key_better(score[i], y, x, score[j], qy, qx)) alive = 0;
        }
      }
      surv[i] = (uint8_t)alive;
      n_surv += (size_t)alive;
    }
  }

  /* Per cell keep the k_cell best survivors, then the n_keep best of those. */
  kept = (ofref_keypoint*)malloc((n_surv ? n_surv : 1) * sizeof(ofref_keypoint));
  if (!kept) goto fail;
  size_t n_kept = 0;
  for (int32_t cy = 0; cy < ncy; ++cy) {
    for (int32_t cx = 0; cx < ncx; ++cx) {
      size_t first = n_kept;
      int32_t x0 = cx * cs, y0 = cy * cs;
      for (int32_t y = y0; y < y0 + cs && y < Hl; ++y) {
        for (int32_t x = x0; x < x0 + cs && x < Wl; ++x) {
          size_t i = (size_t)y * Wl + x;
          if (!surv[i]) continue;
          ofref_keypoint k;
          memset(&k, 0, sizeof k);
          k.x = x; k.y = y; k.level = level; k.score = score[i];
          kept[n_kept++] = k;
        }
      }
      size_t nc = n_kept - first;
      qsort(kept + first, nc, sizeof(ofref_keypoint), cmp_keypoint);
      if (nc > (size_t)k_cell) n_kept = first + (size_t)k_cell;
    }
  }
  qsort(kept, n_kept, sizeof(ofref_keypoint), cmp_keypoint);
  n_out = n_kept < (size_t)n_keep ? (int32_t)n_kept : n_keep;
  for (int32_t i = 0; i < n_out; ++i) out[i] = kept[i];

  if (cand_map) memcpy(cand_map, cand, npx);
  if (surv_map) memcpy(surv_map, surv, npx);
  if (score_map) memcpy(score_map, score, npx * sizeof(int64_t));
  if (cell_flags) memcpy(cell_flags, flag, (size_t)ncx * ncy);
  free(kept);
  free(cand);
  free(score);
  free(surv);
  free(flag);
  return n_out;
fail:
  free(kept);
  free(cand);
  free(score);
  free(surv);
  free(flag);
  return -1;
}

/* ------------------------------------------------------------- whole frame -- */

int ofref_detect(const uint8_t* img, int32_t W, int32_t H, int32_t stride,
                 const ofref_params* p, ofref_keypoint* out, int32_t cap) {
  int32_t w[OFREF_MAX_LEVELS], h[OFREF_MAX_LEVELS], q[OFREF_MAX_LEVELS], k[OFREF_MAX_LEVELS];
  int L = ofref_geometry(W, H, p, w, h, q, k, NULL);
  if (L < 0 || cap < p->n_features) return -1;
  int32_t total = 0;
  for (int l = 0; l < L; ++l) {
    const uint8_t* lvl = img;
    int32_t lstride = stride;
    uint8_t* buf = NULL;
    if (l > 0) {
      buf = (uint8_t*)malloc((size_t)w[l] * h[l]);
      if (!buf) return -1;
      ofref_resample(img, W, H, stride, buf, w[l], h[l]);
      lvl = buf;
      lstride = w[l];
    }
    int n = ofref_level_detect(lvl, w[l], h[l], lstride, p, l, k[l], q[l], NULL, NULL, NULL,
                               NULL, out + total);
    if (n < 0) {
      free(buf);
      return -1;
    }
    for (int i = 0; i < n; ++i) {
      ofref_keypoint* kp = out + total + i;
      ofref_moments(lvl, lstride, kp->x, kp->y, p->patch_radius, &kp->m10, &kp->m01);
      kp->angle = atan2((double)kp->m01, (double)kp->m10);
    }
    total += n;
    free(buf);
  }
  return total;
}
