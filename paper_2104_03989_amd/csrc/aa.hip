// Silhouette antialiasing (Sec. 5.2, "Antialiasing": the operator of Laine et
// al. 2020 that gives visibility gradients at silhouettes), fused with the
// image loss of Sec. 5.3, and its adjoint.
//
// For two horizontally or vertically adjacent pixels whose triangle ids
// differ, the front triangle F is the one with the smaller visibility key
// (empty pixels have the largest key); P is the pixel F is visible at, Q the
// other one.  Among F's oriented edges 0, 1, 2 the first one that Q lies
// outside of (integer edge test with the top-left rule) and that is a
// silhouette edge (a boundary edge, or one whose neighbouring triangle has
// the other screen orientation in this view) is the crossing edge a->b.
// With e(X) the float edge function of the projected edge at the NDC centre
// of pixel X, s = clamp(e(P) / (e(P) - e(Q)), 0, 1); a box filter one pixel
// wide gives out(Q) += (s - 1/2)(c(P) - c(Q)) if s > 1/2 and
// out(P) += (1/2 - s)(c(Q) - c(P)) if s < 1/2.  All terms use the colours
// before antialiasing, so each pixel gathers its own four pairs and no
// atomics or ordering are involved in the forward pass.
//
// Loss: mean over B*H*W*3 of |T(out) - T(ref)| (or the square), with
// T(x) = Gamma(log(x + 1)) and Gamma the sRGB transfer function
// (12.92 x for x <= 0.0031308, 1.055 x^(1/2.4) - 0.055 above), or T(x) = x.
#include "dev.h"

namespace adr {


// The crossing edge of pair (P, Q) for front triangle F, or false.
struct Cross {
  int va, vb;    // vertex indices, F on the left of a->b
  float s;       // crossing parameter from P towards Q (clamped)
  bool clamped;  // s was outside [0, 1]
  double eP, eQ, den;
  double aP[2], bP[2], aQ[2], bQ[2];  // projected a, b relative to the centres of P and Q
};

// Projected corner relative to the NDC point X: (x - w X.x) / w, (y - w X.y) / w
// (float64, from the float64 clip coordinates: edges of pixel-sized
// triangles are short, and their edge functions cancel in float32); iw is
// 1 / w, shared by the corner's two uses.
__device__ __forceinline__ void rel_proj(double4 c, double iw, double Xx, double Xy, double out[2]) {
  out[0] = (c.x - c.w * Xx) * iw;
  out[1] = (c.y - c.w * Xy) * iw;
}

// The front triangle F of a pair as read from memory: its vertex indices and
// their snapped coordinates in this view, its orientation and, for each
// vertex c, the orientation of the neighbour across the edge opposite c (2,
// which no orientation takes, where there is none).
struct Front {
  int v[3];
  int2 s[3];
  int of, on[3];
};
// The accesses that depend on F only, then those that depend on them.
__device__ __forceinline__ void front_ids(const AAArgs& a, int b, int F, Front& f, int nb[3]) {
  const int* tri = a.m.tri + 3 * F;
  const int* adj = a.m.adj + 3 * F;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    f.v[c] = tri[c];
    nb[c] = adj[c];
  }
  f.of = a.orient[(int64_t)b * a.m.n_tri + F];
}
__device__ __forceinline__ void front_coords(const AAArgs& a, int b, const int nb[3], Front& f) {
  const int2* sv = reinterpret_cast<const int2*>(a.snap + (int64_t)b * a.m.n_pos);
  const int8_t* ov = a.orient + (int64_t)b * a.m.n_tri;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    f.s[c] = sv[2 * f.v[c]];
    f.on[c] = nb[c] < 0 ? 2 : (int)ov[nb[c]];
  }
}

// Among F's edges 0, 1, 2 (counter-clockwise order) the first one that pixel
// (Qi, Qj) lies outside of and that is a silhouette edge: its vertices a -> b
// with F on the left, or false.
__device__ __forceinline__ bool cross_edge(const Front& f, int Qi, int Qj, int& va, int& vb) {
  const int64_t A = (int64_t)(f.s[1].x - f.s[0].x) * (f.s[2].y - f.s[0].y) -
                    (int64_t)(f.s[1].y - f.s[0].y) * (f.s[2].x - f.s[0].x);
  // vertices 1 and 2 exchanged for a clockwise F (the edge opposite a vertex
  // goes with it); every index below is then a constant
  const bool sw = A < 0;
  const int V[3] = {f.v[0], sw ? f.v[2] : f.v[1], sw ? f.v[1] : f.v[2]};
  const int O[3] = {f.on[0], sw ? f.on[2] : f.on[1], sw ? f.on[1] : f.on[2]};
  const int X[3] = {f.s[0].x, sw ? f.s[2].x : f.s[1].x, sw ? f.s[1].x : f.s[2].x};
  const int Y[3] = {f.s[0].y, sw ? f.s[2].y : f.s[1].y, sw ? f.s[1].y : f.s[2].y};
  const int64_t qx = 256 * (int64_t)Qi + 128, qy = 256 * (int64_t)Qj + 128;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int j = k == 2 ? 0 : k + 1, l = k == 0 ? 2 : k - 1;
    const int64_t dx = (int64_t)X[l] - X[j], dy = (int64_t)Y[l] - Y[j];
    const int64_t e = dx * (qy - Y[j]) - dy * (qx - X[j]);
    const bool tl = dy < 0 || (dy == 0 && dx < 0);
    const bool inside = e > 0 || (e == 0 && tl);
    if (inside) continue;
    if (O[k] == f.of) continue;  // both sides face the same way: no silhouette
    va = V[j];
    vb = V[l];
    return true;
  }
  return false;
}

// The crossing parameter of pair (P, Q) on the projected edge with clip
// coordinates ca -> cb; false if the edge is parallel to the pair.
__device__ __forceinline__ bool cross_param(const AAArgs& a, double4 ca, double4 cb, int Pi, int Pj, int Qi,
                                            int Qj, Cross& x) {
  const double Px = ((double)Pi + 0.5) * a.v.sxs - 1.0;
  const double Py = ((double)Pj + 0.5) * a.v.sys - 1.0;
  const double Qx = ((double)Qi + 0.5) * a.v.sxs - 1.0;
  const double Qy = ((double)Qj + 0.5) * a.v.sys - 1.0;
  // e(X) = (b - a) x (X - a) = a' x b' with a' = a - X, b' = b - X
  const double iwa = 1.0 / ca.w, iwb = 1.0 / cb.w;
  rel_proj(ca, iwa, Px, Py, x.aP);
  rel_proj(cb, iwb, Px, Py, x.bP);
  rel_proj(ca, iwa, Qx, Qy, x.aQ);
  rel_proj(cb, iwb, Qx, Qy, x.bQ);
  x.eP = x.aP[0] * x.bP[1] - x.aP[1] * x.bP[0];
  x.eQ = x.aQ[0] * x.bQ[1] - x.aQ[1] * x.bQ[0];
  x.den = x.eP - x.eQ;
  if (x.den == 0.0) return false;
  const double s = x.eP / x.den;
  x.clamped = !(s >= 0.0 && s <= 1.0);
  x.s = (float)fmin(fmax(s, 0.0), 1.0);
  return true;
}

__device__ __forceinline__ bool find_cross(const AAArgs& a, int b, int F, int Pi, int Pj, int Qi, int Qj,
                                           Cross& x) {
  Front f;
  int nb[3];
  front_ids(a, b, F, f, nb);
  front_coords(a, b, nb, f);
  if (!cross_edge(f, Qi, Qj, x.va, x.vb)) return false;
  return cross_param(a, clip_d(a.m.pos, a.v.mvpd, b, x.va), clip_d(a.m.pos, a.v.mvpd, b, x.vb), Pi, Pj, Qi,
                     Qj, x);
}

// A pair's code: -1 if it does not blend, else its crossing parameter s in
// [0, 1], plus 2 if s was clamped.  Every pair is evaluated once, by its left
// or lower pixel; both pixels then read its code.
__device__ __forceinline__ float pair_code(const Cross& x) { return x.clamped ? x.s + 2.f : x.s; }

// Pair between pixel (i,j) and its neighbour (ni,nj): which side is P and
// the crossing, or false if the pair does not blend.
struct Pair {
  bool self_is_P;
  Cross x;
};
__device__ __forceinline__ bool eval_pair(const AAArgs& a, int b, int i, int j, uint64_t kself, int ni,
                                          int nj, uint64_t knb, Pair& pr) {
  if ((uint32_t)kself == (uint32_t)knb) return false;
  bool selfP = kself < knb;
  uint64_t kF = selfP ? kself : knb;
  int F = (int)(uint32_t)kF - 1;
  pr.self_is_P = selfP;
  if (selfP) return find_cross(a, b, F, i, j, ni, nj, pr.x);
  return find_cross(a, b, F, ni, nj, i, j, pr.x);
}

__device__ __forceinline__ f3 ldc(const float* c, int64_t o) { return mk(c[3 * o], c[3 * o + 1], c[3 * o + 2]); }

// x^(1/2.4) for the power branch of the sRGB curve (x > 0.0031308, a normal
// float) through the hardware base-2 logarithm and exponential (each within
// about one unit in the last place; the general powf costs several times
// more and is evaluated six times per pixel by the tone-mapped loss).
__device__ __forceinline__ float pow_inv24(float x) {
  return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 2.4f));
}
__device__ __forceinline__ float srgb(float x) {
  return x <= 0.0031308f ? 12.92f * x : 1.055f * pow_inv24(x) - 0.055f;
}
// log(1 + a) for a >= 0: with u = 1 + a rounded, log(u) a / (u - 1) makes up
// for the rounding of u (D. Goldberg, "What every computer scientist should
// know about floating-point arithmetic", 1991), a few units in the last
// place with the hardware logarithm and reciprocal; a itself where u rounds
// to 1.
__device__ __forceinline__ float log1p_pos(float a) {
  const float u = 1.0f + a;
  const float d = u - 1.0f;
  return d == 0.f ? a : (__builtin_amdgcn_logf(u) * 0.693147180559945309f) * (a * __builtin_amdgcn_rcpf(d));
}
// T(x) = sign(x) Gamma(log(1 + |x|)): the paper's tone map for x >= 0,
// extended as an odd function to the negative radiance that freely optimised
// texels can produce.
__device__ __forceinline__ float tmap(float x) { return copysignf(srgb(log1p_pos(fabsf(x))), x); }
// T(x) and T'(x) together: with y = log(1 + |x|), Gamma'(y) = 12.92 below the
// knee, else (1.055 / 2.4) y^(1/2.4) / y, and T'(x) = Gamma'(y) / (1 + |x|).
__device__ __forceinline__ float tmap_and_d(float x, float& d) {
  const float a = fabsf(x);
  const float y = log1p_pos(a);
  float t;
  if (y <= 0.0031308f) {
    t = 12.92f * y;
    d = 12.92f * __builtin_amdgcn_rcpf(1.0f + a);
  } else {
    const float p = pow_inv24(y);
    t = 1.055f * p - 0.055f;
    d = (1.055f / 2.4f) * p * __builtin_amdgcn_rcpf(y * (1.0f + a));
  }
  return copysignf(t, x);
}

// Code of the pair between pixel (i, j) and its neighbour in direction q
// (0 left, 1 right, 2 down, 3 up); the neighbour must be inside the image.
__device__ __forceinline__ float code_of(const AAArgs& a, int64_t base, int i, int j, int q) {
  const int ci = q == 0 ? i - 1 : i, cj = q == 2 ? j - 1 : j;
  return a.codes[a.code_stride * (base + (int64_t)cj * a.v.W + ci) + (q >= 2 ? 1 : 0)];
}

// Weight a pixel receives from a pair with code c, given whether it is the
// pair's front pixel P.
__device__ __forceinline__ float received_from(float c, bool self_is_P) {
  if (c < 0.f) return 0.f;
  const float s = c >= 2.f ? c - 2.f : c;
  if (self_is_P) return s < 0.5f ? 0.5f - s : 0.f;
  return s > 0.5f ? s - 0.5f : 0.f;
}

// Weight pixel (i, j) receives from the pair with its neighbour, and the
// neighbour's index; 0 if the pair does not blend into this pixel.
__device__ __forceinline__ float received(const AAArgs& a, int b, int i, int j, uint64_t k, int ni, int nj,
                                          uint64_t kn) {
  Pair pr;
  if (!eval_pair(a, b, i, j, k, ni, nj, kn, pr)) return 0.f;
  float s = pr.x.s;
  if (pr.self_is_P) return s < 0.5f ? 0.5f - s : 0.f;
  return s > 0.5f ? s - 0.5f : 0.f;
}

// Received antialiasing of pixel (i, j): total weight W and
// acc = sum_k w_k (c_k - c); the output is c + acc / max(1, W), a convex
// blend even where several edges of sub-pixel triangles cross.
struct Recv {
  float W;
  f3 acc;
};
__device__ __forceinline__ Recv recv_stats(const AAArgs& a, int b, int i, int j) {
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  int64_t base = (int64_t)b * a.v.H * a.v.W;
  int64_t o = base + (int64_t)j * a.v.W + i;
  uint64_t k = a.vis[o];
  f3 c = ldc(a.color, o);
  Recv r{0.f, mk(0.f, 0.f, 0.f)};
  for (int q = 0; q < 4; ++q) {
    int ni = i + di[q], nj = j + dj[q];
    if (ni < 0 || nj < 0 || ni >= a.v.W || nj >= a.v.H) continue;
    int64_t on = base + (int64_t)nj * a.v.W + ni;
    const uint64_t kn = a.vis[on];
    float w = a.codes ? ((uint32_t)k == (uint32_t)kn ? 0.f : received_from(code_of(a, base, i, j, q), k < kn))
                      : received(a, b, i, j, k, ni, nj, kn);
    if (w > 0.f) {
      r.W += w;
      r.acc += w * (ldc(a.color, on) - c);
    }
  }
  return r;
}

__device__ __forceinline__ Recv recv_load(const float4* st, int64_t o) {
  const float4 q = st[o];
  return Recv{q.x, mk(q.y, q.z, q.w)};
}

// Loss term of one pixel (Sec. 5.3) and its gradient, written to dimage[o].
__device__ __forceinline__ float pixel_loss(f3 out, f3 r, int loss_kind, float inv_n, float* dimage, int64_t o) {
  const bool tm = loss_kind == ADR_LOSS_L1_TONEMAP || loss_kind == ADR_LOSS_L2_TONEMAP;
  const bool l1 = loss_kind == ADR_LOSS_L1 || loss_kind == ADR_LOSS_L1_TONEMAP;
  float ov[3] = {out.x, out.y, out.z}, rv[3] = {r.x, r.y, r.z}, gd[3];
  float lsum = 0.f;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float dt = 1.0f, d;
    if (tm) d = tmap_and_d(ov[ch], dt) - tmap(rv[ch]);
    else d = ov[ch] - rv[ch];
    if (l1) {
      lsum += fabsf(d);
      gd[ch] = (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f)) * dt * inv_n;
    } else {
      lsum += d * d;
      gd[ch] = 2.f * d * dt * inv_n;
    }
  }
  st3(dimage, o, mk(gd[0], gd[1], gd[2]));
  return lsum;
}

// Multisample resolve (Sec. 5.2, "Antialiasing"): a pixel is the mean of its
// ms x ms antialiased samples; the loss is taken on the resolved pixels.
__global__ __launch_bounds__(256) void k_msaa_resolve(ViewsD v, const float* __restrict__ image_s,
                                                      const float* __restrict__ ref, int loss_kind,
                                                      float* __restrict__ image, float* __restrict__ dimage,
                                                      float* __restrict__ partial) {
  __shared__ float red[4];
  const int Wp = v.W / v.ms, Hp = v.H / v.ms;
  const int64_t n = (int64_t)v.B * Hp * Wp;
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float lsum = 0.f;
  if (o < n) {
    const int64_t b = o / ((int64_t)Hp * Wp);
    const int64_t r = o - b * Hp * Wp;
    const int jp = (int)(r / Wp), ip = (int)(r - (int64_t)jp * Wp);
    f3 acc = mk(0.f, 0.f, 0.f);
    for (int sj = 0; sj < v.ms; ++sj)
      for (int si = 0; si < v.ms; ++si)
        acc += ldc(image_s, (b * v.H + jp * v.ms + sj) * v.W + ip * v.ms + si);
    const f3 out = (1.0f / (float)(v.ms * v.ms)) * acc;
    if (image) st3(image, o, out);
    if (ref) lsum = pixel_loss(out, ldc(ref, o), loss_kind, 1.0f / (3.0f * (float)n), dimage, o);
  }
  if (ref) {
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// dL/d(antialiased sample): a sample carries 1/ms^2 of its pixel's gradient.
__device__ __forceinline__ f3 sample_grad(const AAArgs& a, const float* dimage, int b, int i, int j) {
  if (a.v.ms == 1) return ldc(dimage, ((int64_t)b * a.v.H + j) * a.v.W + i);
  const int64_t op = ((int64_t)b * a.v.Hp + (j >> a.v.msh)) * a.v.Wp + (i >> a.v.msh);
  return (1.0f / (float)(a.v.ms * a.v.ms)) * ldc(dimage, op);
}

// Antialiasing, image and loss of one 16x16 tile of pixels (Sec. 5.2, 5.3).
// Every pair of neighbours is evaluated once: each pixel evaluates its pairs
// with its right and upper neighbours, and 32 threads the pairs that link
// the tile to its left and lower neighbours (which the neighbouring tiles
// evaluate too, with the same arguments and so the same code); the codes
// meet in LDS, where each pixel gathers its four: hc[r][c] is the code of the
// pair (x0 + c - 1, x0 + c) in row y0 + r, vc[r][c] that of (y0 + r - 1,
// y0 + r) in column x0 + c.  With a stats buffer the pixels' own codes also
// go to it for the adjoint.
__device__ __forceinline__ void aa_fwd_body(const AAFwdArgs& f, int bid, int nb) {
  __shared__ float hc[16][17], vc[17][16];
  __shared__ float red[4];
  const AAArgs& a = f.a;
  const float* __restrict__ ref = f.ref;
  const int loss_kind = f.loss_kind;
  float* __restrict__ image = f.image;
  float* __restrict__ dimage = f.dimage;
  const int tile = xcd_tile(bid, nb);
  const Pix p = tile_pixel(tile, threadIdx.x, a.tiles_x, a.tiles_y, a.v.W, a.v.H);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lx = (wave & 1) * 8 + (lane & 7), ly = (wave >> 1) * 8 + (lane >> 3);
  const int x0 = p.i - lx, y0 = p.j - ly;
  const int64_t base = (int64_t)p.b * a.v.H * a.v.W;
  const int64_t o = base + (int64_t)p.j * a.v.W + p.i;
  // every load of the pixel issued up front, so that their latencies overlap:
  // its key, its four neighbours' keys (a missing neighbour takes the
  // pixel's own key, which pairs with nothing), its colour and reference
  const uint64_t k = p.ok ? a.vis[o] : 0ull;
  const bool aa_on = p.ok && !a.no_aa;
  const uint64_t kl = aa_on && p.i > 0 ? a.vis[o - 1] : k;
  const uint64_t kr = aa_on && p.i + 1 < a.v.W ? a.vis[o + 1] : k;
  const uint64_t kd = aa_on && p.j > 0 ? a.vis[o - a.v.W] : k;
  const uint64_t ku = aa_on && p.j + 1 < a.v.H ? a.vis[o + a.v.W] : k;
  const f3 c = p.ok ? ldc(a.color, o) : mk(0.f, 0.f, 0.f);
  const f3 rv = p.ok && ref ? ldc(ref, o) : mk(0.f, 0.f, 0.f);
  // the pair that links the tile to its left (threads 0..15) or lower
  // (16..31) neighbour tile: its left (lower) pixel and that pixel's
  // neighbour, with their keys loaded up front as well
  const bool edge_thread = !a.no_aa && threadIdx.x < 32;  // whether or not its own pixel is inside
  const bool left = threadIdx.x < 16;
  const int er = threadIdx.x & 15;
  const int ei = left ? x0 - 1 : x0 + er, ej = left ? y0 + er : y0 - 1;
  const int eni = left ? ei + 1 : ei, enj = left ? ej : ej + 1;
  const bool e_ok = edge_thread && ei >= 0 && ej >= 0 && eni < a.v.W && enj < a.v.H;
  const uint64_t ke = e_ok ? a.vis[base + (int64_t)ej * a.v.W + ei] : 0ull;
  const uint64_t ken = e_ok ? a.vis[base + (int64_t)enj * a.v.W + eni] : 0ull;
  if (!a.no_aa) {
    // A thread's pairs (with its right and its upper neighbour, and the
    // linking pair above) go through their memory accesses together, one
    // stage after the other, so that their latencies overlap: the front
    // triangle, its vertices and neighbours, the crossing edge, the edge's
    // positions.  PI, PJ is the front pixel P, QI, QJ the other one, F = -1
    // for a pair that does not blend.
    int PI[3], PJ[3], QI[3], QJ[3], F[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int si = q < 2 ? p.i : ei, sj = q < 2 ? p.j : ej;
      const int ni = q == 0 ? p.i + 1 : (q == 1 ? p.i : eni), nj = q == 0 ? p.j : (q == 1 ? p.j + 1 : enj);
      const uint64_t ks = q < 2 ? k : ke, kn = q == 0 ? kr : (q == 1 ? ku : ken);
      const bool on = (q < 2 ? aa_on : e_ok) && (uint32_t)ks != (uint32_t)kn;
      const bool selfP = ks < kn;
      F[q] = on ? (int)(uint32_t)(selfP ? ks : kn) - 1 : -1;
      PI[q] = selfP ? si : ni;
      PJ[q] = selfP ? sj : nj;
      QI[q] = selfP ? ni : si;
      QJ[q] = selfP ? nj : sj;
    }
    Front fr[3];
    int nb[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (F[q] >= 0) front_ids(a, p.b, F[q], fr[q], nb[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (F[q] >= 0) front_coords(a, p.b, nb[q], fr[q]);
    int va[3], vb[3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (F[q] >= 0 && !cross_edge(fr[q], QI[q], QJ[q], va[q], vb[q])) F[q] = -1;
    float pa[3][3], pb[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (F[q] >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          pa[q][c] = a.m.pos[3 * va[q] + c];
          pb[q][c] = a.m.pos[3 * vb[q] + c];
        }
      }
    float code[3];
    const double* M = a.v.mvpd + 16 * p.b;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      code[q] = -1.f;
      Cross x;
      if (F[q] >= 0 && cross_param(a, clip_from(M, pa[q][0], pa[q][1], pa[q][2]),
                                   clip_from(M, pb[q][0], pb[q][1], pb[q][2]), PI[q], PJ[q], QI[q], QJ[q], x))
        code[q] = pair_code(x);
    }
    if (p.ok && a.stats) {
      a.codes[a.code_stride * o] = code[0];
      a.codes[a.code_stride * o + 1] = code[1];
    }
    hc[ly][lx + 1] = code[0];
    vc[ly + 1][lx] = code[1];
    if (threadIdx.x < 32) {
      if (left) hc[er][0] = code[2];
      else vc[0][er] = code[2];
    }
    __syncthreads();
  }
  float lsum = 0.f;
  if (p.ok) {
    f3 out = c;
    if (!a.no_aa) {
      // received antialiasing: W and acc = sum_k w_k (c_k - c)
      Recv r{0.f, mk(0.f, 0.f, 0.f)};
      const int64_t dn[4] = {-1, 1, -(int64_t)a.v.W, (int64_t)a.v.W};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t on = o + dn[q];
        const uint64_t kn = q == 0 ? kl : (q == 1 ? kr : (q == 2 ? kd : ku));
        const float cq = q == 0 ? hc[ly][lx] : (q == 1 ? hc[ly][lx + 1] : (q == 2 ? vc[ly][lx] : vc[ly + 1][lx]));
        const float w = (uint32_t)k == (uint32_t)kn ? 0.f : received_from(cq, k < kn);
        if (w > 0.f) {
          r.W += w;
          r.acc += w * (ldc(a.color, on) - c);
        }
      }
      if (r.W > 0.f) out += (1.0f / fmaxf(r.W, 1.0f)) * r.acc;
      if (a.stats) a.stats[o] = make_float4(r.W, r.acc.x, r.acc.y, r.acc.z);
    }
    if (image) st3(image, o, out);
    if (ref) {
      const float inv_n = 1.0f / (3.0f * (float)a.v.B * (float)a.v.H * (float)a.v.W);
      lsum += pixel_loss(out, rv, loss_kind, inv_n, dimage, o);
    }
  }
  if (ref) {
    // block reduction in a fixed order (deterministic)
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
    if (lane == 0) red[wave] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) f.partial[bid] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}
// (5 waves per SIMD, 96 VGPRs: the three pairs' loads in flight together need the registers; at 6 or 7
// waves the spills double the time)
ADR_KERNEL(__launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))), k_aa_fwd, AAFwdArgs, aa_fwd_body)

__device__ __forceinline__ void loss_reduce_body(const LossReduceArgs& a, int, int) {
  __shared__ double red[4];
  // each thread's partials in a fixed order, sixteen loads in flight at a time
  double acc = 0.0;
  int i = threadIdx.x;
  for (; i + 15 * 256 < a.n; i += 16 * 256) {
    float x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = a.partial[i + q * 256];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += (double)x[q];
  }
  for (; i < a.n; i += 256) acc += (double)a.partial[i];
  // then a fixed tree: within each wave, then the four waves
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) a.loss[0] = (float)(((red[0] + red[1]) + (red[2] + red[3])) * (double)a.inv_n);
}
ADR_KERNEL(__launch_bounds__(256), k_loss_reduce, LossReduceArgs, loss_reduce_body)

// Adjoint.  With out(r) = c(r) + acc(r) / M(r), M = max(1, W):
//   d out(r) / d c(r) = 1 - W(r)/M(r),  d out(r) / d c(k) = w_k / M(r),
//   d out(r) / d w_k = (c(k) - c(r)) / M(r) - [W > 1] acc(r) / W(r)^2.
// Each pixel gathers dL/dc of its own colour (as receiver and as source of
// its four pairs; a receiver's W and acc are recomputed from its own pairs);
// the gradient of a pair's crossing parameter s w.r.t. the clip coordinates
// of its edge is scattered once, by the left (or lower) pixel of the pair.
__device__ __forceinline__ void aa_bwd_body(const AABwdArgs& b, int bid, int nb) {
  const AAArgs& a = b.a;
  const float* __restrict__ dimage = b.dimage;
  const float* __restrict__ dloss = b.dloss;
  unsigned long long* __restrict__ fclip = b.fclip;
  const bool det = b.det;
  int tile = xcd_tile(bid, nb);
  Pix p = tile_pixel(tile, threadIdx.x, a.tiles_x, a.tiles_y, a.v.W, a.v.H);
  if (!p.ok) return;
  float scale = dloss ? dloss[0] : 1.0f;
  int64_t base = (int64_t)p.b * a.v.H * a.v.W;
  int64_t o = base + (int64_t)p.j * a.v.W + p.i;
  f3 gself = scale * sample_grad(a, dimage, p.b, p.i, p.j);
  f3 gc = gself;
  if (!a.no_aa) {
    // the keys of the pixel and of its four neighbours, loaded together (a
    // missing neighbour takes the pixel's own key, which pairs with nothing)
    const uint64_t k = a.vis[o];
    const uint64_t kn[4] = {p.i > 0 ? a.vis[o - 1] : k, p.i + 1 < a.v.W ? a.vis[o + 1] : k,
                            p.j > 0 ? a.vis[o - a.v.W] : k, p.j + 1 < a.v.H ? a.vis[o + a.v.W] : k};
    const f3 c = ldc(a.color, o);
    const Recv rs = a.stats ? recv_load(a.stats, o) : recv_stats(a, p.b, p.i, p.j);
    const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
    // The four pairs go through their memory accesses together, one stage
    // after the other: their codes (from the forward, else the pairs
    // re-evaluated), then the neighbours' colours, gradients and sums for the
    // pairs that blend, then the edges of the two pairs this pixel owns.
    float cq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cq[q] = -1.f;
      if ((uint32_t)k == (uint32_t)kn[q]) continue;
      if (a.codes) {
        cq[q] = code_of(a, base, p.i, p.j, q);
      } else {
        Pair pr;
        if (eval_pair(a, p.b, p.i, p.j, k, p.i + di[q], p.j + dj[q], kn[q], pr)) cq[q] = pair_code(pr.x);
      }
    }
    f3 cn[4], gn[4];
    Recv rr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float s = cq[q] >= 2.f ? cq[q] - 2.f : cq[q];
      if (cq[q] < 0.f || s == 0.5f) continue;
      const int ni = p.i + di[q], nj = p.j + dj[q];
      const int64_t on = base + (int64_t)nj * a.v.W + ni;
      cn[q] = ldc(a.color, on);
      gn[q] = sample_grad(a, dimage, p.b, ni, nj);
      const bool selfP = k < kn[q];
      const bool self_recv = s > 0.5f ? !selfP : selfP;
      rr[q] = self_recv ? rs : (a.stats ? recv_load(a.stats, on) : recv_stats(a, p.b, ni, nj));
    }
    const float Ms = fmaxf(rs.W, 1.0f);
    gc = (1.0f - rs.W / Ms) * gself;
    float gs_own[2] = {0.f, 0.f};  // dL/ds of the pairs with the right and the upper neighbour
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float cc = cq[q];
      const float s = cc >= 2.f ? cc - 2.f : cc;
      if (cc < 0.f || s == 0.5f) continue;
      // the receiver is Q for s > 1/2 (w = s - 1/2) and P for s < 1/2 (w = 1/2 - s)
      const bool selfP = k < kn[q];
      const bool recv_Q = s > 0.5f;
      const bool self_recv = recv_Q ? !selfP : selfP;
      const float w = recv_Q ? s - 0.5f : 0.5f - s;
      const f3 gnq = scale * gn[q];
      const float Mr = fmaxf(rr[q].W, 1.0f);
      const f3 g_r = self_recv ? gself : gnq;   // dL/d out(receiver)
      const f3 c_r = self_recv ? c : cn[q], c_src = self_recv ? cn[q] : c;
      if (!self_recv) gc += (w / Mr) * gnq;     // this pixel is the source
      f3 dw = (1.0f / Mr) * (c_src - c_r);
      if (rr[q].W > 1.0f) dw -= (1.0f / (rr[q].W * rr[q].W)) * rr[q].acc;
      const float g_w = dot(g_r, dw);
      // s is taken from the edge only where it was not clamped
      if ((q == 1 || q == 3) && cc < 2.f) gs_own[q >> 1] = recv_Q ? g_w : -g_w;
    }
    // the gradient of s = eP / (eP - eQ) w.r.t. the clip coordinates of the
    // crossing edge of each pair this pixel owns (its edge found again, the
    // same s as the forward's)
    int F[2], PI[2], PJ[2], QI[2], QJ[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int q = 2 * t + 1, ni = p.i + di[q], nj = p.j + dj[q];
      const bool selfP = k < kn[q];
      F[t] = gs_own[t] != 0.f ? (int)(uint32_t)(selfP ? k : kn[q]) - 1 : -1;
      PI[t] = selfP ? p.i : ni;
      PJ[t] = selfP ? p.j : nj;
      QI[t] = selfP ? ni : p.i;
      QJ[t] = selfP ? nj : p.j;
    }
    Front fr[2];
    int nbr[2][3];
#pragma unroll
    for (int t = 0; t < 2; ++t)
      if (F[t] >= 0) front_ids(a, p.b, F[t], fr[t], nbr[t]);
#pragma unroll
    for (int t = 0; t < 2; ++t)
      if (F[t] >= 0) front_coords(a, p.b, nbr[t], fr[t]);
    int va[2], vb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
      if (F[t] >= 0 && !cross_edge(fr[t], QI[t], QJ[t], va[t], vb[t])) F[t] = -1;
    float pa[2][3], pb[2][3];
#pragma unroll
    for (int t = 0; t < 2; ++t)
      if (F[t] >= 0) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          pa[t][cc] = a.m.pos[3 * va[t] + cc];
          pb[t][cc] = a.m.pos[3 * vb[t] + cc];
        }
      }
    const double* M = a.v.mvpd + 16 * p.b;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if (F[t] < 0) continue;
      const double4 ca = clip_from(M, pa[t][0], pa[t][1], pa[t][2]);
      const double4 cb = clip_from(M, pb[t][0], pb[t][1], pb[t][2]);
      Cross x;
      if (!cross_param(a, ca, cb, PI[t], PJ[t], QI[t], QJ[t], x)) continue;
      const double g_s = gs_own[t];
      const double id2 = 1.0 / (x.den * x.den);
      const double g_eP = -g_s * x.eQ * id2, g_eQ = g_s * x.eP * id2;
      const double iwa = 1.0 / ca.w, iwb = 1.0 / cb.w;
      const double ax = ca.x * iwa, ay = ca.y * iwa, bx = cb.x * iwb, by = cb.y * iwb;
      // e(X) = a'_x b'_y - a'_y b'_x, a' = a - X, b' = b - X
      const double g_ax = g_eP * x.bP[1] + g_eQ * x.bQ[1];
      const double g_ay = -g_eP * x.bP[0] - g_eQ * x.bQ[0];
      const double g_bx = -g_eP * x.aP[1] - g_eQ * x.aQ[1];
      const double g_by = g_eP * x.aP[0] + g_eQ * x.aQ[0];
      const int64_t oa = 4 * ((int64_t)p.b * a.m.n_pos + va[t]);
      const int64_t ob = 4 * ((int64_t)p.b * a.m.n_pos + vb[t]);
      const double ga[3] = {g_ax * iwa, g_ay * iwa, -(g_ax * ax + g_ay * ay) * iwa};
      const double gb[3] = {g_bx * iwb, g_by * iwb, -(g_bx * bx + g_by * by) * iwb};
      const int comp[3] = {0, 1, 3};
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        acc_add(fclip + oa + comp[m], ga[m], det);
        acc_add(fclip + ob + comp[m], gb[m], det);
      }
    }
  }
  st3(b.gcolor, o, gc);
}
// (4 waves per SIMD, 128 VGPRs and 24 bytes of spills: 0.051 ms per step on the paper loop at 3 waves,
// 0.047 at 4; at 5 the spills double it)
ADR_KERNEL(__launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))), k_aa_bwd, AABwdArgs, aa_bwd_body)

// stats: the caller's buffer of 8 floats per pixel, two planes: the pixels'
// (W, acc) float4s, then their pair codes (2 floats each); without it the
// codes go to context scratch (forward) or are not used (adjoint: every pair
// is re-evaluated).
static AAArgs make_aa(const MeshD& m, const ViewsD& v, const Scratch& s, const uint64_t* vis,
                      const float* color, int no_aa, float* stats) {
  AAArgs a;
  const int64_t npx = (int64_t)v.B * v.H * v.W;
  a.stats = reinterpret_cast<float4*>(stats);
  a.code_stride = 2;
  a.codes = stats ? stats + 4 * npx : nullptr;
  a.m = m;
  a.v = v;
  a.snap = reinterpret_cast<const int4*>(s.snap);
  a.orient = s.orient;
  a.vis = vis;
  a.color = color;
  a.tiles_x = (v.W + 15) / 16;
  a.tiles_y = (v.H + 15) / 16;
  a.no_aa = no_aa;
  return a;
}

// The antialiasing and loss forward of one-sample pixels (0 blocks when there
// is neither an image nor a reference).
Plan<AAFwdArgs> plan_aa_fwd(const MeshD& m, const ViewsD& v, const Scratch& s, const uint64_t* vis,
                            const float* color, const float* ref, int loss_kind, int no_aa, float* image,
                            float* dimage, float* stats) {
  AAFwdArgs f{};
  f.a = make_aa(m, v, s, vis, color, no_aa, stats);
  f.ref = ref;
  f.loss_kind = loss_kind;
  f.image = image;
  f.dimage = dimage;
  f.partial = s.partial;
  return {f, (!image && !ref) ? 0u : (unsigned)(f.a.tiles_x * f.a.tiles_y * v.B)};
}

hipError_t launch_aa_loss_fwd(const MeshD& m, const ViewsD& v, const Scratch& s,
                              const uint64_t* vis, const float* color, const float* ref,
                              int loss_kind, int no_aa, float* image, float* dimage, float* loss,
                              hipStream_t st, float* stats) {
  if (!image && !ref) return hipSuccess;
  hipError_t e;
  if (v.ms > 1) {
    // antialiased samples, then the resolve and the loss per pixel
    ADR_LAUNCH_1(k_aa_fwd, plan_aa_fwd(m, v, s, vis, color, nullptr, loss_kind, no_aa, s.image_s, nullptr, stats), st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t n = (int64_t)v.B * (v.H / v.ms) * (v.W / v.ms);
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_msaa_resolve, dim3(nb), dim3(256), 0, st, v, s.image_s, ref, loss_kind, image, dimage,
                       s.partial);
  } else {
    ADR_LAUNCH_1(k_aa_fwd, plan_aa_fwd(m, v, s, vis, color, ref, loss_kind, no_aa, image, dimage, stats), st);
  }
  return hipGetLastError();
}

// The loss from the per-block partials of launch_aa_loss_fwd (a second,
// one-block launch; nothing to do without a reference).
Plan<LossReduceArgs> plan_loss_reduce(const ViewsD& v, const float* ref, const Scratch& s, float* loss) {
  int nb;
  if (v.ms > 1) {
    nb = (int)(((int64_t)v.B * v.Hp * v.Wp + 255) / 256);
  } else {
    nb = ((v.W + 15) / 16) * ((v.H + 15) / 16) * v.B;
  }
  // partials hold sums; the mean's 1/N is applied here
  const double n = 3.0 * (double)v.B * v.Hp * v.Wp;
  return {LossReduceArgs{s.partial, nb, (float)(1.0 / n), loss}, ref ? 1u : 0u};
}

hipError_t launch_loss_reduce(const ViewsD& v, const float* ref, const Scratch& s, float* loss, hipStream_t st) {
  ADR_LAUNCH_1(k_loss_reduce, plan_loss_reduce(v, ref, s, loss), st);
  return hipGetLastError();
}

Plan<AABwdArgs> plan_aa_bwd(const MeshD& m, const ViewsD& v, const Scratch& s, const uint64_t* vis,
                            const float* color, const float* dimage, const float* dloss, int no_aa,
                            const float* stats) {
  AABwdArgs b{};
  b.a = make_aa(m, v, s, vis, color, no_aa, const_cast<float*>(stats));
  b.dimage = dimage;
  b.dloss = dloss;
  b.gcolor = s.gcolor;
  b.fclip = s.fix_clip;
  b.det = s.det;
  return {b, (unsigned)(b.a.tiles_x * b.a.tiles_y * v.B)};
}

hipError_t launch_aa_bwd(const MeshD& m, const ViewsD& v, const Scratch& s, const uint64_t* vis,
                         const float* color, const float* dimage, const float* dloss, int no_aa,
                         hipStream_t st, const float* stats) {
  ADR_LAUNCH_1(k_aa_bwd, plan_aa_bwd(m, v, s, vis, color, dimage, dloss, no_aa, stats), st);
  return hipGetLastError();
}

// ---- batched launches ----
hipError_t launch_aa_fwd_n(const Stage<AAFwdArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_aa_fwd, s, st);
  return hipGetLastError();
}
hipError_t launch_loss_reduce_n(const Stage<LossReduceArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_loss_reduce, s, st);
  return hipGetLastError();
}
hipError_t launch_aa_bwd_n(const Stage<AABwdArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_aa_bwd, s, st);
  return hipGetLastError();
}

}  // namespace adr
