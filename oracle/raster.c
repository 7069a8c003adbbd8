/*
 * ORACLE -- test infrastructure only.  Nothing in the product path may link,
 * load or call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.
 *
 * Visibility of the render loop (paper Sec. 3 and Sec. 5.2: the latent mesh is
 * rasterized from each sampled camera; the paper delegates this to the
 * rasterization primitive of Laine et al. 2020, which runs on fixed-function
 * hardware).  The paper fixes no sub-pixel precision, fill rule or depth
 * format, so this file is the definition adopted for them:
 *
 *   R1  clip = MVP [p,1] evaluated in float32 as ((m0 x + m1 y) + m2 z) + m3,
 *       every operation rounded to float32.  X = rint(((x/w) 0.5 + 0.5) W 256),
 *       Y likewise with H, Z = clamp(rint(((z/w) 0.5 + 0.5) 2^24), 0, 2^24-1),
 *       each step rounded to float32, rint = round half to even.
 *   R2  a vertex is unusable if w <= 1e-6, |x/w| > 8 or |y/w| > 8 (or NaN);
 *       a triangle with an unusable vertex or zero integer area is dropped.
 *   R3  no back-face culling: a clockwise triangle has its last two corners
 *       swapped before the coverage test.
 *   R4  coverage of pixel (i, j), centre (256 i + 128, 256 j + 128) with row 0
 *       at the bottom, by integer edge functions and the top-left rule.
 *   R5  depth = clamp(rint(z), 0, 2^24-1) with z the float32 plane through the
 *       three snapped (X, Y, Z) evaluated as (Z0 + a dx) + b dy, where
 *       a = (dz1 dy2 - dz2 dy1) / A, b = (dz2 dx1 - dz1 dx2) / A and
 *       A = dx1 dy2 - dy1 dx2, all in float32 in that order.
 *   R6  key = depth << 32 | (triangle + 1); the smallest key wins, so equal
 *       depth goes to the smaller triangle index.  Empty pixels hold
 *       0xFFFFFFFF00000000 (triangle id 0).
 *
 * Compiled with gcc -O2 -fno-fast-math -ffp-contract=off on x86-64, where
 * float arithmetic is IEEE single precision with round-to-nearest-even.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define KEY_EMPTY 0xFFFFFFFF00000000ull
#define ZMAX 16777215

typedef struct { int32_t x, y, z, ok; } snap_t;

/* R1/R2 for one vertex. */
static snap_t snap_vertex(const float* m, const float* p, int W, int H) {
  snap_t s;
  float c[4];
  for (int r = 0; r < 4; ++r) {
    float a = m[4 * r + 0] * p[0];
    float b = m[4 * r + 1] * p[1];
    float t = a + b;
    float d = m[4 * r + 2] * p[2];
    t = t + d;
    t = t + m[4 * r + 3];
    c[r] = t;
  }
  s.x = s.y = s.z = 0;
  s.ok = 0;
  float w = c[3];
  if (!(w > 1e-6f)) return s;
  float qx = c[0] / w, qy = c[1] / w, qz = c[2] / w;
  if (!(fabsf(qx) <= 8.0f) || !(fabsf(qy) <= 8.0f) || isnan(qz)) return s;
  float sx = qx * 0.5f; sx = sx + 0.5f; sx = sx * (float)(W * 256);
  float sy = qy * 0.5f; sy = sy + 0.5f; sy = sy * (float)(H * 256);
  float sz = qz * 0.5f; sz = sz + 0.5f; sz = sz * 16777216.0f;
  s.x = (int32_t)rintf(sx);
  s.y = (int32_t)rintf(sy);
  float rz = rintf(sz);
  s.z = rz <= 0.0f ? 0 : (rz >= (float)ZMAX ? ZMAX : (int32_t)rz);
  s.ok = 1;
  return s;
}

/* Snapped vertices of one view: out[V*4] = (X, Y, Z, usable). */
void oracle_snap(const float* pos, int32_t n_pos, const float* mvp, int32_t W, int32_t H,
                 int32_t* out) {
  for (int32_t v = 0; v < n_pos; ++v) {
    snap_t s = snap_vertex(mvp, pos + 3 * v, W, H);
    out[4 * v + 0] = s.x; out[4 * v + 1] = s.y; out[4 * v + 2] = s.z; out[4 * v + 3] = s.ok;
  }
}

/* Float32 clip coordinates as R1 evaluates them (used by tests). */
void oracle_clip32(const float* pos, int32_t n_pos, const float* m, float* out) {
  for (int32_t v = 0; v < n_pos; ++v) {
    const float* p = pos + 3 * v;
    for (int r = 0; r < 4; ++r) {
      float a = m[4 * r + 0] * p[0];
      float b = m[4 * r + 1] * p[1];
      float t = a + b;
      float d = m[4 * r + 2] * p[2];
      t = t + d;
      t = t + m[4 * r + 3];
      out[4 * v + r] = t;
    }
  }
}

typedef struct {
  int64_t X[3], Y[3];
  int32_t Z[3];
  int64_t A;
  int32_t flip;           /* 1 if corners 1 and 2 were swapped */
  int32_t vid[3];         /* original corner index of each oriented corner */
  float a, b;             /* R5 plane slopes */
} tri_setup_t;

/* Oriented setup of one triangle; returns 0 if it is dropped (R2). */
static int setup_triangle(const int32_t* snapv, const int32_t* t, tri_setup_t* s) {
  const int32_t* v0 = snapv + 4 * t[0];
  const int32_t* v1 = snapv + 4 * t[1];
  const int32_t* v2 = snapv + 4 * t[2];
  if (!v0[3] || !v1[3] || !v2[3]) return 0;
  int64_t A = (int64_t)(v1[0] - v0[0]) * (v2[1] - v0[1]) - (int64_t)(v1[1] - v0[1]) * (v2[0] - v0[0]);
  if (A == 0) return 0;
  int order[3] = {0, 1, 2};
  s->flip = 0;
  if (A < 0) { order[1] = 2; order[2] = 1; A = -A; s->flip = 1; }
  const int32_t* vv[3] = {v0, v1, v2};
  for (int k = 0; k < 3; ++k) {
    s->X[k] = vv[order[k]][0];
    s->Y[k] = vv[order[k]][1];
    s->Z[k] = vv[order[k]][2];
    s->vid[k] = order[k];
  }
  s->A = A;
  float dx1 = (float)(s->X[1] - s->X[0]), dy1 = (float)(s->Y[1] - s->Y[0]);
  float dx2 = (float)(s->X[2] - s->X[0]), dy2 = (float)(s->Y[2] - s->Y[0]);
  float dz1 = (float)(s->Z[1] - s->Z[0]), dz2 = (float)(s->Z[2] - s->Z[0]);
  float p1 = dx1 * dy2, p2 = dy1 * dx2;
  float Af = p1 - p2;
  float n1 = dz1 * dy2, n2 = dz2 * dy1;
  float nx = n1 - n2;
  float m1 = dz2 * dx1, m2 = dz1 * dx2;
  float ny = m1 - m2;
  s->a = nx / Af;
  s->b = ny / Af;
  return 1;
}

/* Edge function of the oriented edge opposite corner k at (px, py). */
static int64_t edge_fn(const tri_setup_t* s, int k, int64_t px, int64_t py) {
  int j = (k + 1) % 3, l = (k + 2) % 3;
  return (s->X[l] - s->X[j]) * (py - s->Y[j]) - (s->Y[l] - s->Y[j]) * (px - s->X[j]);
}

/* R4: top-left edges include their boundary. */
static int edge_is_top_left(const tri_setup_t* s, int k) {
  int j = (k + 1) % 3, l = (k + 2) % 3;
  int64_t dy = s->Y[l] - s->Y[j], dx = s->X[l] - s->X[j];
  return dy < 0 || (dy == 0 && dx < 0);
}

static int covers(const tri_setup_t* s, int64_t px, int64_t py) {
  for (int k = 0; k < 3; ++k) {
    int64_t e = edge_fn(s, k, px, py);
    if (e < 0 || (e == 0 && !edge_is_top_left(s, k))) return 0;
  }
  return 1;
}

static uint32_t depth_at(const tri_setup_t* s, int64_t px, int64_t py) {
  float t = (float)s->Z[0];
  float u = s->a * (float)(px - s->X[0]);
  t = t + u;
  float w = s->b * (float)(py - s->Y[0]);
  t = t + w;
  float r = rintf(t);
  if (!(r > 0.0f)) return 0;
  if (r >= (float)ZMAX) return ZMAX;
  return (uint32_t)r;
}

static int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

/*
 * Rasterize one view.  snapv: [V*4] from oracle_snap.  keys: [H*W] (row j at
 * offset j*W), coverage: [H*W] or NULL (number of covering triangles before
 * the depth test), orient: [T] or NULL (+1 counter-clockwise, -1 clockwise, 0
 * dropped).  brute != 0 tests every pixel against every triangle instead of
 * walking bounding boxes (a check of the bounding-box walk).
 */
void oracle_raster(const int32_t* tri, int32_t n_tri, const int32_t* snapv, int32_t W, int32_t H,
                   uint64_t* keys, uint32_t* coverage, int8_t* orient, int32_t brute) {
  for (int64_t i = 0; i < (int64_t)W * H; ++i) keys[i] = KEY_EMPTY;
  if (coverage) memset(coverage, 0, sizeof(uint32_t) * (size_t)W * H);
  for (int32_t t = 0; t < n_tri; ++t) {
    tri_setup_t s;
    int ok = setup_triangle(snapv, tri + 3 * t, &s);
    if (orient) orient[t] = ok ? (s.flip ? -1 : 1) : 0;
    if (!ok) continue;
    int64_t i0 = 0, i1 = W - 1, j0 = 0, j1 = H - 1;
    if (!brute) {
      int64_t mnx = s.X[0], mxx = s.X[0], mny = s.Y[0], mxy = s.Y[0];
      for (int k = 1; k < 3; ++k) {
        if (s.X[k] < mnx) mnx = s.X[k];
        if (s.X[k] > mxx) mxx = s.X[k];
        if (s.Y[k] < mny) mny = s.Y[k];
        if (s.Y[k] > mxy) mxy = s.Y[k];
      }
      i0 = floor_div(mnx - 128 + 255, 256); i1 = floor_div(mxx - 128, 256);
      j0 = floor_div(mny - 128 + 255, 256); j1 = floor_div(mxy - 128, 256);
      if (i0 < 0) i0 = 0;
      if (j0 < 0) j0 = 0;
      if (i1 > W - 1) i1 = W - 1;
      if (j1 > H - 1) j1 = H - 1;
    }
    for (int64_t j = j0; j <= j1; ++j) {
      for (int64_t i = i0; i <= i1; ++i) {
        int64_t px = 256 * i + 128, py = 256 * j + 128;
        if (!covers(&s, px, py)) continue;
        uint64_t key = ((uint64_t)depth_at(&s, px, py) << 32) | (uint32_t)(t + 1);
        int64_t o = j * W + i;
        if (coverage) coverage[o] += 1;
        if (key < keys[o]) keys[o] = key;
      }
    }
  }
}

/*
 * One depth-peeling pass of one view (Sec. 5.2, "Order-independent
 * transparency"): keys[o] receives the smallest key strictly greater than
 * floor[o] among the fragments covering pixel o (the two-sided test against
 * the previous layer), KEY_EMPTY if there is none.  floor: [H*W] or NULL (no
 * lower bound: the plain front layer).  brute as for oracle_raster.
 */
void oracle_raster_peel(const int32_t* tri, int32_t n_tri, const int32_t* snapv, int32_t W, int32_t H,
                        const uint64_t* floor_keys, uint64_t* keys, int32_t brute) {
  for (int64_t i = 0; i < (int64_t)W * H; ++i) keys[i] = KEY_EMPTY;
  for (int32_t t = 0; t < n_tri; ++t) {
    tri_setup_t s;
    if (!setup_triangle(snapv, tri + 3 * t, &s)) continue;
    int64_t i0 = 0, i1 = W - 1, j0 = 0, j1 = H - 1;
    if (!brute) {
      int64_t mnx = s.X[0], mxx = s.X[0], mny = s.Y[0], mxy = s.Y[0];
      for (int k = 1; k < 3; ++k) {
        if (s.X[k] < mnx) mnx = s.X[k];
        if (s.X[k] > mxx) mxx = s.X[k];
        if (s.Y[k] < mny) mny = s.Y[k];
        if (s.Y[k] > mxy) mxy = s.Y[k];
      }
      i0 = floor_div(mnx - 128 + 255, 256); i1 = floor_div(mxx - 128, 256);
      j0 = floor_div(mny - 128 + 255, 256); j1 = floor_div(mxy - 128, 256);
      if (i0 < 0) i0 = 0;
      if (j0 < 0) j0 = 0;
      if (i1 > W - 1) i1 = W - 1;
      if (j1 > H - 1) j1 = H - 1;
    }
    for (int64_t j = j0; j <= j1; ++j) {
      for (int64_t i = i0; i <= i1; ++i) {
        int64_t px = 256 * i + 128, py = 256 * j + 128;
        if (!covers(&s, px, py)) continue;
        uint64_t key = ((uint64_t)depth_at(&s, px, py) << 32) | (uint32_t)(t + 1);
        int64_t o = j * W + i;
        if (floor_keys && key <= floor_keys[o]) continue;
        if (key < keys[o]) keys[o] = key;
      }
    }
  }
}

/*
 * Integer inside test of the oriented edges of triangle t at pixel (i, j):
 * bit k of the result is set if the pixel centre is on the inside of the
 * oriented edge opposite oriented corner k (top-left rule included).  Also
 * returns, through vid, the original corner index of each oriented corner.
 * Returns -1 if the triangle is dropped.
 */
int32_t oracle_edge_inside(const int32_t* tri, int32_t t, const int32_t* snapv, int32_t i, int32_t j,
                           int32_t* vid) {
  tri_setup_t s;
  if (!setup_triangle(snapv, tri + 3 * t, &s)) return -1;
  int64_t px = 256 * (int64_t)i + 128, py = 256 * (int64_t)j + 128;
  int32_t bits = 0;
  for (int k = 0; k < 3; ++k) {
    int64_t e = edge_fn(&s, k, px, py);
    if (e > 0 || (e == 0 && edge_is_top_left(&s, k))) bits |= 1 << k;
    vid[k] = s.vid[k];
  }
  return bits;
}

/* oracle_edge_inside for n (triangle, pixel) queries; vid is [n*3]. */
void oracle_edge_inside_batch(const int32_t* tri, const int32_t* snapv, int32_t n, const int32_t* t,
                              const int32_t* i, const int32_t* j, int32_t* bits, int32_t* vid) {
  for (int32_t q = 0; q < n; ++q) bits[q] = oracle_edge_inside(tri, t[q], snapv, i[q], j[q], vid + 3 * q);
}
