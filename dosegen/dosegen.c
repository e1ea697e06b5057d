/*
 * dosegen.c — seeded, row-random-access generator of synthetic dose-deposition
 * matrices (voxels x beam spots) and spot-weight vectors.
 *
 * This module only draws inputs.  It contains none of the dose computation:
 * no encoding, no products, no reductions.  Both the CPU oracle and the GPU
 * library receive exactly the arrays produced here.
 *
 * Structure (Sec. II-A and II-B of the paper):
 *   - rows are voxels of an nx*ny*nz dose grid, columns are pencil-beam spots
 *     laid out in n_lines scanlines of n_spots spots each (column index
 *     line*n_spots + pos), seen in the beam's-eye view;
 *   - a voxel outside the beam footprint receives no dose (empty row);
 *   - a voxel inside receives dose from spots near its beam's-eye-view
 *     position: 2-4 contiguous runs of columns on adjacent scanlines;
 *   - row lengths are lognormal around the non-empty mean, values are
 *     lognormal(mu, sigma) clipped to [0, 1] and rounded once to FP32.
 *
 * Randomness is counter based: every draw is SplitMix64's output mixing
 * function (Steele, Lea & Flood, OOPSLA 2014; the finaliser of Vigna's
 * splitmix64.c) applied to a key built from (seed, matrix id, row, counter).
 * Any row can therefore be regenerated on its own, in any order, by any
 * thread.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t nx, ny, nz;        /* dose grid; n_rows = nx*ny*nz, row = ix + nx*(iy + ny*iz) */
  int32_t n_lines, n_spots;  /* spot grid; n_cols = n_lines*n_spots                     */
  double mean_len;           /* mean length of a non-empty row                          */
  double sigma_len;          /* lognormal sigma of the row length                       */
  int32_t max_len;           /* cap on a row's length (0: n_cols)                       */
  int32_t beam_axis;         /* 0: beam along y, 1: beam along x                        */
  double empty_frac;         /* fraction of voxels outside the footprint (0 or >=0.215) */
  double shift_u, shift_v;   /* footprint centre shift in the beam's-eye view           */
  double val_mu, val_sigma;  /* lognormal value distribution                            */
  uint64_t seed;
  uint64_t matrix_id;
} dg_spec;

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* One 64-bit draw for (key, counter): the splitmix64 sequence of state `key`
 * read at position `ctr`. */
static inline uint64_t draw(uint64_t key, uint64_t ctr) {
  return sm64_mix(key + (ctr + 1) * 0x9E3779B97F4A7C15ULL);
}

static inline uint64_t row_key(const dg_spec* s, int64_t row) {
  uint64_t k = sm64_mix(s->seed ^ 0x6A09E667F3BCC909ULL);
  k = sm64_mix(k ^ (s->matrix_id * 0xD1B54A32D192ED03ULL));
  return sm64_mix(k ^ ((uint64_t)row * 0x8CB92BA72F3D8DD7ULL));
}

/* Standard normal from one 64-bit draw (Box-Muller, cosine branch). */
static inline double normal_from(uint64_t r) {
  double u1 = ((double)(r >> 32) + 0.5) * (1.0 / 4294967296.0);
  double u2 = (double)(r & 0xFFFFFFFFULL) * (1.0 / 4294967296.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

typedef struct {
  int nonempty;
  double us, vs; /* position on the spot grid, each in [0,1) */
} bev_t;

static bev_t bev_of(const dg_spec* s, int64_t row) {
  bev_t b;
  int64_t ix = row % s->nx;
  int64_t iy = (row / s->nx) % s->ny;
  int64_t iz = row / ((int64_t)s->nx * s->ny);
  double u = s->beam_axis == 0 ? (ix + 0.5) / s->nx : (iy + 0.5) / s->ny;
  double v = (iz + 0.5) / s->nz;
  if (s->empty_frac <= 0.0) {
    b.nonempty = 1;
    b.us = u;
    b.vs = v;
    return b;
  }
  double r = sqrt((1.0 - s->empty_frac) / 3.141592653589793);
  if (r > 0.5) r = 0.5;
  double cu = 0.5 + s->shift_u, cv = 0.5 + s->shift_v;
  double du = u - cu, dv = v - cv;
  b.nonempty = (du * du + dv * dv) <= r * r;
  /* spots cover the footprint's bounding box */
  b.us = (du + r) / (2.0 * r);
  b.vs = (dv + r) / (2.0 * r);
  if (b.us < 0.0) b.us = 0.0;
  if (b.vs < 0.0) b.vs = 0.0;
  if (b.us >= 1.0) b.us = 0.999999999;
  if (b.vs >= 1.0) b.vs = 0.999999999;
  return b;
}

static int64_t row_len_of(const dg_spec* s, int64_t row, const bev_t* b) {
  if (!b->nonempty) return 0;
  int64_t nc = (int64_t)s->n_lines * s->n_spots;
  int64_t cap = s->max_len > 0 && s->max_len < nc ? s->max_len : nc;
  uint64_t key = row_key(s, row);
  double z = normal_from(draw(key, 0));
  double len = s->mean_len * exp(s->sigma_len * z - 0.5 * s->sigma_len * s->sigma_len);
  int64_t n = (int64_t)llround(len);
  if (n < 1) n = 1;
  if (n > cap) n = cap;
  return n;
}

int64_t dg_row_len(const dg_spec* s, int64_t row) {
  bev_t b = bev_of(s, row);
  return row_len_of(s, row, &b);
}

/* Lengths of rows [r0, r1) into out[0 .. r1-r0). */
void dg_row_lens(const dg_spec* s, int64_t r0, int64_t r1, int32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = r0; r < r1; ++r) out[r - r0] = (int32_t)dg_row_len(s, r);
}

/* Columns and values of one row; returns its length.  cols/vals must hold
 * dg_row_len(s,row) entries. */
int64_t dg_row(const dg_spec* s, int64_t row, int32_t* cols, float* vals) {
  bev_t b = bev_of(s, row);
  int64_t n = row_len_of(s, row, &b);
  if (n == 0) return 0;
  const int64_t L = s->n_lines, S = s->n_spots;
  uint64_t key = row_key(s, row);
  int64_t k = 2 + (int64_t)(draw(key, 1) % 3u); /* 2, 3 or 4 runs */
  if (k > L) k = L;
  if (n > k * S) k = (n + S - 1) / S;
  int64_t lc = (int64_t)(b.vs * L);
  int64_t sc = (int64_t)(b.us * S);
  int64_t l0 = lc - (k - 1) / 2;
  if (l0 > L - k) l0 = L - k;
  if (l0 < 0) l0 = 0;
  int64_t base = n / k, rem = n % k, t = 0;
  for (int64_t run = 0; run < k; ++run) {
    int64_t len = base + (run < rem ? 1 : 0);
    int64_t start = sc - len / 2;
    if (start > S - len) start = S - len;
    if (start < 0) start = 0;
    for (int64_t p = 0; p < len; ++p) cols[t++] = (int32_t)((l0 + run) * S + start + p);
  }
  for (int64_t j = 0; j < n; ++j) {
    double z = normal_from(draw(key, 2 + (uint64_t)j));
    double v = exp(s->val_mu + s->val_sigma * z);
    if (v > 1.0) v = 1.0;
    vals[j] = (float)v;
  }
  return n;
}

/* Rows [r0, r1) into caller arrays; row_ptr holds r1-r0+1 offsets into
 * cols/vals (row_ptr[0] may be non-zero: cols/vals are indexed by it). */
void dg_fill_rows(const dg_spec* s, int64_t r0, int64_t r1, const int64_t* row_ptr,
                  int32_t* cols, float* vals) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t r = r0; r < r1; ++r) {
    int64_t o = row_ptr[r - r0];
    dg_row(s, r, cols + o, vals + o);
  }
}

/* Spot weights: x_j = (u32 >> 8) * 2^-24, uniform in [0,1) and exact in FP32. */
void dg_fill_x(uint64_t seed, uint64_t stream, int64_t n, float* x) {
  uint64_t key = sm64_mix(sm64_mix(seed ^ 0xBB67AE8584CAA73BULL) ^ (stream * 0xA0761D6478BD642FULL));
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    uint32_t u = (uint32_t)(draw(key, (uint64_t)j) >> 32);
    x[j] = (float)(u >> 8) * (1.0f / 16777216.0f);
  }
}

/* Signed uniform values in [-1,1) with 8 significant bits (exact in FP32),
 * for adjoint seeds and invariant tests. */
void dg_fill_signed(uint64_t seed, uint64_t stream, int64_t n, float* x) {
  uint64_t key = sm64_mix(sm64_mix(seed ^ 0x3C6EF372FE94F82BULL) ^ (stream * 0xE7037ED1A0B428DBULL));
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    uint32_t u = (uint32_t)(draw(key, (uint64_t)j) >> 32);
    x[j] = (float)((int32_t)(u >> 24) - 128) * (1.0f / 128.0f);
  }
}

/* Number of rows of the grid inside the beam footprint. */
int64_t dg_count_nonempty(const dg_spec* s) {
  int64_t n_rows = (int64_t)s->nx * s->ny * s->nz, c = 0;
#pragma omp parallel for reduction(+ : c) schedule(static)
  for (int64_t r = 0; r < n_rows; ++r) c += bev_of(s, r).nonempty;
  return c;
}

int dg_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
