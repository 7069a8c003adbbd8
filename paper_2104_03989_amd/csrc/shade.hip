// Deferred shading of the rasterized views (Sec. 5.2) and its hand-written
// adjoint.  Per pixel the G-buffer (position, normal, tangent, bitangent,
// texture coordinates and their screen derivatives) is formed in registers
// from the visibility key and the clip coordinates and never stored: the
// backward kernel recomputes it.
//
// Interpolation: with h_k = (x, y, w) of corner k in clip space and the pixel
// centre p = (px, py, 1) in NDC, D_k = (h_{k+1} x h_{k+2}) . p and
// lambda_k = D_k / sum D are the perspective-correct barycentrics; their
// screen derivatives are (a_k - lambda_k sum a) / sum D with a_k the x
// component of h_{k+1} x h_{k+2} (likewise y), times 2/W (2/H) per pixel.
// The determinant is evaluated after moving every corner onto the pixel's
// ray, g_k = (x_k - w_k px, y_k - w_k py), which leaves it unchanged:
// D_k = g_{k+1} x g_{k+2} (2-D cross product); for pixel-sized triangles the
// plain triple product cancels badly.
// Textures: isotropic LOD = 0.5 log2 max(|duv/dx|^2, |duv/dy|^2) in level-0
// texels, trilinear lookups (wrap u, clamp v); the LOD is differentiated
// where it is not clamped.  Shading: normal-mapped frame N, T' =
// normalize(T - (N.T) N), B = N x T'; Blinn-Phong E max(0,n.l)(kd + 0.04
// max(0,n.h)^32) or the GGX model of Sec. 5.2 with k_s = (1-m) 0.04 + m k_d
// and k_s' = (1-gamma) k_s.
#include "dev.h"

namespace adr {

constexpr float kPi = 3.14159265358979323846f;

// The barycentric set-up runs in float64 from float64 clip coordinates:
// for pixel-sized or thin triangles the screen derivatives of lambda are
// ill-conditioned, and float32 clip coordinates alone move the texture LOD
// by ~1e-4 there.  It is ~60 float64 operations per pixel.
struct BaryD {
  double w[3];          // clip w
  double gx[3], gy[3];  // x - w px, y - w py
  double a[3], b[3];    // dD/dpx, dD/dpy
  double S, px, py;
};

// The float64 barycentric set-up of pixel (i, j) on the triangle with
// position indices v (the adjoint recomputes it at its end rather than
// keeping these 30 registers live through the shading).
__device__ __forceinline__ void bary_setup(const MeshD& m, const ViewsD& vw, int b, int i,
                                           int j, const int* v, BaryD& d) {
  // (i, j) is a visibility sample; shading is evaluated once per pixel, at
  // the centre of the sample's pixel, with derivatives per pixel
  d.px = ((double)(i >> vw.msh) + 0.5) * vw.pxs - 1.0;
  d.py = ((double)(j >> vw.msh) + 0.5) * vw.pys - 1.0;
  double D[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double4 q = clip_d(m.pos, vw.mvpd, b, v[c]);
    d.w[c] = q.w;
    d.gx[c] = q.x - q.w * d.px;
    d.gy[c] = q.y - q.w * d.py;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int j1 = c == 2 ? 0 : c + 1, k1 = c == 0 ? 2 : c - 1;
    D[c] = d.gx[j1] * d.gy[k1] - d.gy[j1] * d.gx[k1];
    d.a[c] = d.w[k1] * d.gy[j1] - d.w[j1] * d.gy[k1];
    d.b[c] = d.w[j1] * d.gx[k1] - d.w[k1] * d.gx[j1];
  }
  d.S = D[0] + D[1] + D[2];
}

struct PixelGeom {
  int v[3];        // position indices
  int t[3];        // uv indices
  float lam[3], lx[3], ly[3];
  float sx, sy;
  f3 x, Ni, T;
  float u, v_, ux, vx, uy, vy;
  float ul, vl;    // low parts: u + ul, v_ + vl are the coordinates to ~float64 precision
  f3 N, T1, Tp, Bt;
};

__device__ __forceinline__ void pixel_geom(const MeshD& m, const ViewsD& vw,
                                           const float* nrm, const float* tan, int b, int i,
                                           int j, int tri, PixelGeom& g) {
  g.sx = (float)vw.pxs;
  g.sy = (float)vw.pys;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    g.v[c] = m.tri[3 * tri + c];
    g.t[c] = m.uv_tri[3 * tri + c];
  }
  BaryD d;
  bary_setup(m, vw, b, i, j, g.v, d);
  double iS = 1.0 / d.S;
  double A = d.a[0] + d.a[1] + d.a[2];
  double Bs = d.b[0] + d.b[1] + d.b[2];
  const float u0 = m.uv[2 * g.t[0]], v0 = m.uv[2 * g.t[0] + 1];
  double ud = u0, vd = v0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int j1 = c == 2 ? 0 : c + 1, k1 = c == 0 ? 2 : c - 1;
    double lam = (d.gx[j1] * d.gy[k1] - d.gy[j1] * d.gx[k1]) * iS;
    g.lam[c] = (float)lam;
    g.lx[c] = (float)((d.a[c] - lam * A) * iS * vw.pxs);
    g.ly[c] = (float)((d.b[c] - lam * Bs) * iS * vw.pys);
    if (c > 0) {
      ud += lam * ((double)m.uv[2 * g.t[c]] - (double)u0);
      vd += lam * ((double)m.uv[2 * g.t[c] + 1] - (double)v0);
    }
  }
  g.u = (float)ud;
  g.v_ = (float)vd;
  g.ul = (float)(ud - (double)g.u);
  g.vl = (float)(vd - (double)g.v_);
  // attributes relative to corner 0 (sum lambda = 1, sum of derivatives = 0):
  // a = a0 + sum_c lambda_c (a_c - a0), da = sum_c dlambda_c (a_c - a0)
  g.x = ld3(m.pos, g.v[0]);
  g.Ni = ld3(nrm, g.v[0]);
  g.T = ld3(tan, g.v[0]);
  g.ux = g.vx = g.uy = g.vy = 0.f;
#pragma unroll
  for (int c = 1; c < 3; ++c) {
    g.x += g.lam[c] * (ld3(m.pos, g.v[c]) - ld3(m.pos, g.v[0]));
    g.Ni += g.lam[c] * (ld3(nrm, g.v[c]) - ld3(nrm, g.v[0]));
    g.T += g.lam[c] * (ld3(tan, g.v[c]) - ld3(tan, g.v[0]));
    float du = m.uv[2 * g.t[c]] - u0, dv = m.uv[2 * g.t[c] + 1] - v0;
    g.ux += g.lx[c] * du;
    g.vx += g.lx[c] * dv;
    g.uy += g.ly[c] * du;
    g.vy += g.ly[c] * dv;
  }
  g.N = safe_normalize(g.Ni);
  g.T1 = g.T - dot(g.N, g.T) * g.N;
  g.Tp = safe_normalize(g.T1);
  g.Bt = cross(g.N, g.Tp);
}

// ------------------------------------------------------------------ BRDFs

__device__ __forceinline__ f3 blinn_phong(f3 n, f3 v, f3 l, f3 kd, f3 E) {
  f3 h = safe_normalize(l + v);
  float nl = fmaxf(dot(n, l), 0.f);
  float nh = fmaxf(dot(n, h), 0.f);
  float nh2 = nh * nh, nh4 = nh2 * nh2, nh8 = nh4 * nh4, nh16 = nh8 * nh8, nh32 = nh16 * nh16;
  return nl * (E * (kd + mk(0.04f * nh32, 0.04f * nh32, 0.04f * nh32)));
}

__device__ __forceinline__ void blinn_phong_bwd(f3 n, f3 v, f3 l, f3 kd, f3 E, f3 gc, f3& gn,
                                                f3& gv, f3& gkd) {
  f3 hu = l + v;
  f3 h = safe_normalize(hu);
  float NL = dot(n, l), NH = dot(n, h);
  float nl = fmaxf(NL, 0.f), nh = fmaxf(NH, 0.f);
  float nh2 = nh * nh, nh4 = nh2 * nh2, nh8 = nh4 * nh4, nh16 = nh8 * nh8, nh31 = nh16 * nh8 * nh4 * nh2 * nh;
  float p32 = nh31 * nh;
  f3 Eg = E * gc;
  gkd = nl * Eg;
  float g_nl = dot(Eg, kd) + 0.04f * p32 * sum3(Eg);
  float g_nh = nl * 0.04f * sum3(Eg) * 32.f * nh31;
  float g_NL = NL >= 0.f ? g_nl : 0.f;
  float g_NH = NH >= 0.f ? g_nh : 0.f;
  gn = g_NL * l + g_NH * h;
  gv = safe_normalize_bwd(hu, g_NH * n);
}

struct GGX {
  f3 h, hu;
  float NL, NV, NH, VH, nl, nv, nh, vh, nlc;
  float r, alpha, a2, C, den, D, k, dl, dv, G1l, G1v, G, Q, w5;
  bool rok, nhpos;
  f3 ks, F0, F, diffuse, spec;
};

__device__ __forceinline__ void ggx_eval(f3 n, f3 v, f3 l, f3 kd, f3 orm, GGX& s) {
  float gamma = orm.x, rough = orm.y, metal = orm.z;
  s.rok = rough >= 0.08f && rough <= 1.0f;
  s.r = fminf(fmaxf(rough, 0.08f), 1.0f);
  s.alpha = s.r * s.r;
  s.a2 = s.alpha * s.alpha;
  s.hu = l + v;
  s.h = safe_normalize(s.hu);
  s.NL = dot(n, l);
  s.NV = dot(n, v);
  s.NH = dot(n, s.h);
  s.VH = dot(v, s.h);
  s.nl = fmaxf(s.NL, 0.f);
  s.nv = fmaxf(s.NV, 1e-4f);
  s.nh = fmaxf(s.NH, 0.f);
  s.vh = fmaxf(s.VH, 0.f);
  s.nlc = fmaxf(s.nl, 1e-4f);
  // (n.h)^2 (a^2 - 1) + 1 = a^2 (n.h)^2 + |n x h|^2 for unit n, h; the
  // second form avoids the cancellation of 1 - (n.h)^2 near the highlight.
  s.nhpos = s.NH > 0.f;
  f3 nxh = cross(n, s.h);
  s.C = dot(nxh, nxh);
  s.den = s.nhpos ? s.a2 * s.nh * s.nh + s.C : 1.0f;
  s.D = s.a2 / (kPi * s.den * s.den);
  s.k = 0.5f * s.alpha;
  s.dl = s.nl * (1.f - s.k) + s.k;
  s.dv = s.nv * (1.f - s.k) + s.k;
  s.G1l = s.nl / s.dl;
  s.G1v = s.nv / s.dv;
  s.G = s.G1l * s.G1v;
  s.ks = mk((1.f - metal) * 0.04f + metal * kd.x, (1.f - metal) * 0.04f + metal * kd.y,
            (1.f - metal) * 0.04f + metal * kd.z);
  s.F0 = (1.f - gamma) * s.ks;
  float om = 1.f - s.vh, om2 = om * om;
  s.w5 = om2 * om2 * om;
  s.F = s.F0 + s.w5 * (mk(1.f, 1.f, 1.f) - s.F0);
  s.Q = s.D * s.G / (4.f * s.nlc * s.nv);
  s.spec = s.Q * s.F;
  s.diffuse = ((1.f - metal) / kPi) * kd;
}

__device__ __forceinline__ f3 ggx(f3 n, f3 v, f3 l, f3 kd, f3 orm, f3 E) {
  GGX s;
  ggx_eval(n, v, l, kd, orm, s);
  return s.nl * (E * (s.diffuse + s.spec));
}

__device__ __forceinline__ void ggx_bwd(f3 n, f3 v, f3 l, f3 kd, f3 orm, f3 E, f3 gc, f3& gn,
                                        f3& gv, f3& gkd, f3& gorm) {
  GGX s;
  ggx_eval(n, v, l, kd, orm, s);
  float gamma = orm.x, metal = orm.z;
  f3 Eg = E * gc;
  f3 ginner = s.nl * Eg;
  float g_nl = dot(Eg, s.diffuse + s.spec);
  // diffuse = kd (1-m) / pi
  gkd = ((1.f - metal) / kPi) * ginner;
  float g_m = -dot(ginner, kd) / kPi;
  // spec = Q F
  f3 gF = s.Q * ginner;
  float gQ = dot(ginner, s.F);
  float inv4 = 1.f / (4.f * s.nlc * s.nv);
  float gD = gQ * s.G * inv4;
  float gG = gQ * s.D * inv4;
  float g_nlc = -gQ * s.Q / s.nlc;
  float g_nv = -gQ * s.Q / s.nv;
  // F = F0 + w5 (1 - F0)
  f3 gF0 = (1.f - s.w5) * gF;
  float g_w5 = dot(gF, mk(1.f, 1.f, 1.f) - s.F0);
  float om = 1.f - s.vh, om2 = om * om;
  float g_vh = -5.f * om2 * om2 * g_w5;
  // F0 = (1 - gamma) ks, ks = (1-m) 0.04 + m kd
  float g_gamma = -dot(gF0, s.ks);
  f3 gks = (1.f - gamma) * gF0;
  g_m += dot(gks, kd - mk(0.04f, 0.04f, 0.04f));
  gkd += metal * gks;
  // G = G1(nl) G1(nv), G1(x) = x / (x (1-k) + k)
  float gG1l = gG * s.G1v, gG1v = gG * s.G1l;
  g_nl += gG1l * s.k / (s.dl * s.dl);
  g_nv += gG1v * s.k / (s.dv * s.dv);
  float g_k = -gG1l * s.nl * (1.f - s.nl) / (s.dl * s.dl) - gG1v * s.nv * (1.f - s.nv) / (s.dv * s.dv);
  // D = a2 / (pi den^2)
  float g_a2 = gD / (kPi * s.den * s.den);
  float g_den = -2.f * gD * s.D / s.den;
  float g_NH = 0.f, g_C = 0.f;
  if (s.nhpos) {
    g_a2 += g_den * s.nh * s.nh;
    g_NH = g_den * 2.f * s.a2 * s.nh;
    g_C = g_den;
  }
  float g_alpha = 0.5f * g_k + 2.f * s.alpha * g_a2;
  float g_r = 2.f * s.r * g_alpha;
  gorm = mk(g_gamma, s.rok ? g_r : 0.f, g_m);
  // clamps
  if (s.nl >= 1e-4f) g_nl += g_nlc;
  float g_NL = s.NL >= 0.f ? g_nl : 0.f;
  float g_NV = s.NV >= 1e-4f ? g_nv : 0.f;
  float g_VH = s.VH >= 0.f ? g_vh : 0.f;
  // dot products and |n x h|^2
  gn = g_NL * l + g_NV * v + g_NH * s.h;
  gv = g_NV * n + g_VH * s.h;
  f3 gh = g_NH * n + g_VH * v;
  if (g_C != 0.f) {
    float nh_ = dot(n, s.h);
    gn += (2.f * g_C) * (dot(s.h, s.h) * n - nh_ * s.h);
    gh += (2.f * g_C) * (dot(n, n) * s.h - nh_ * n);
  }
  gv += safe_normalize_bwd(s.hu, gh);
}

// -------------------------------------------------------------- forward

// Alpha of a depth-peeled layer: clamp(alpha map, 0, 1), 1 without a map.
__device__ __forceinline__ float layer_alpha(const ShadeArgs& a, const PixelGeom& g) {
  if (!a.al.data) return 1.f;
  Lod La = lod_select(a.al, g.ux, g.vx, g.uy, g.vy);
  return fminf(fmaxf(tex_trilinear(a.al, g.u, g.v_, g.ul, g.vl, La).val.x, 0.f), 1.f);
}

__device__ __forceinline__ void shade_fwd_body(const ShadeFwdArgs& f, int bid, int nb) {
  const ShadeArgs& a = f.s;
  float* __restrict__ color = f.color;
  int32_t* __restrict__ tri_id = f.tri_id;
  float* __restrict__ alpha = f.alpha;
  int tile = xcd_tile(bid, nb);
  Pix p = tile_pixel(tile, threadIdx.x, a.tiles_x, a.tiles_y, a.v.W, a.v.H);
  if (!p.ok) return;
  int64_t o = ((int64_t)p.b * a.v.H + p.j) * a.v.W + p.i;
  uint64_t key = a.vis[o];
  uint32_t id = (uint32_t)key;
  if (tri_id) tri_id[o] = (int32_t)id;
  if (id == 0u) {
    st3(color, o, mk(0.f, 0.f, 0.f));
    if (alpha) alpha[o] = 0.f;
    return;
  }
  PixelGeom g;
  pixel_geom(a.m, a.v, a.nrm, a.tan, p.b, p.i, p.j, (int)id - 1, g);
  if (alpha) alpha[o] = layer_alpha(a, g);
  Lod Lk = lod_select(a.kd, g.ux, g.vx, g.uy, g.vy);
  f3 kd = tex_trilinear(a.kd, g.u, g.v_, g.ul, g.vl, Lk).val;
  Lod Ln = lod_select(a.nm, g.ux, g.vx, g.uy, g.vy);
  f3 nt = tex_trilinear(a.nm, g.u, g.v_, g.ul, g.vl, Ln).val;
  f3 n = safe_normalize(nt.x * g.Tp + nt.y * g.Bt + nt.z * g.N);
  f3 eye = ld3(a.v.eye, p.b);
  f3 vdir = safe_normalize(eye - g.x);
  f3 l = ld3(a.v.light_dir, p.b);
  f3 E = ld3(a.v.light_rgb, p.b);
  f3 c;
  if (a.model == ADR_SHADE_GGX) {
    Lod Lo = lod_select(a.orm, g.ux, g.vx, g.uy, g.vy);
    f3 orm = tex_trilinear(a.orm, g.u, g.v_, g.ul, g.vl, Lo).val;
    c = ggx(n, vdir, l, kd, orm, E);
  } else {
    c = blinn_phong(n, vdir, l, kd, E);
  }
  st3(color, o, c);
}
// 6 waves per SIMD (80 VGPRs, 16 bytes of spills): the compiler's own choice, 82 VGPRs, gives 5;
// 0.154 -> 0.139 ms per step for the two renders of the paper loop
ADR_KERNEL(__launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))), k_shade_fwd, ShadeFwdArgs,
           shade_fwd_body)

// -------------------------------------------------------------- backward

// ---- wave-aggregated texel-gradient scatter ----
//
// The 64 pixels of a wave (an 8x8 block) sample overlapping bilinear
// footprints: at the level the LOD picks, texels are about pixel-sized, so
// the wave touches roughly (8+1)^2 texels of a level where its lanes would
// issue 64 x 4 atomics per channel.  Per level present in the wave, the
// lanes' contributions are summed into an LDS window covering the wave's
// footprint (integer LDS atomics on fixed-point values, see window_pass), and
// the window's nonzero texel-channels are then added to HBM once each.  A
// footprint larger than the window (a UV seam, very oblique sampling,
// depth-peeled layers) is taken in groups of lanes whose cells fit a box of
// the window's size, one window pass per group.

// Window entries per wave (32-bit): 20 x 20 texels x 3 channels fit; 4 waves'
// windows take 20 KB of LDS, so 8 blocks (8 waves per SIMD) are resident per
// CU.
constexpr int kWinTex = 1280;
// side of the largest square box of texels whose window fits kWinTex entries
constexpr int win_side(int C) {
  int s = 1;
  while ((s + 1) * (s + 1) * C <= kWinTex) ++s;
  return s;
}

struct TexScatter {
  float u, v, ul, vl;
  int l0;
  float f;
  bool has1;
  f3 gs;
};

// Wave-wide min / max of an int, called from converged code (all 64 lanes
// active).  Within each row of 16 lanes two quad permutations and row
// rotations by 4 and 8 (DPP operands: VALU only, no LDS traffic) leave the
// row's result in every lane; the four rows are combined from scalar reads
// of lanes 0, 16, 32 and 48.
template <bool kMin>
__device__ __forceinline__ int wave_reduce_i(int x) {
  auto op = [](int a, int b) { return kMin ? min(a, b) : max(a, b); };
  x = op(x, __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  x = op(x, __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  x = op(x, __builtin_amdgcn_update_dpp(x, x, 0x124, 0xF, 0xF, false));  // row_ror:4
  x = op(x, __builtin_amdgcn_update_dpp(x, x, 0x128, 0xF, 0xF, false));  // row_ror:8
  const int a = __builtin_amdgcn_readlane(x, 0), b = __builtin_amdgcn_readlane(x, 16);
  const int c = __builtin_amdgcn_readlane(x, 32), d = __builtin_amdgcn_readlane(x, 48);
  return op(op(a, b), op(c, d));
}
__device__ __forceinline__ int wave_min_i(int x) { return wave_reduce_i<true>(x); }
__device__ __forceinline__ int wave_max_i(int x) { return wave_reduce_i<false>(x); }
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Unwrapped bilinear footprint at level l: rows r0 <= r1 (clamped), columns
// c0 and c0 + 1 with c0 in [0, s) (c0 + 1 may equal s: wraps to 0).
struct Foot {
  int r0, r1, c0, s;
  float fx, fy;
};
__device__ __forceinline__ Foot foot_at(const Tex& t, int l, float u, float v, float ul, float vl) {
  Foot q;
  int s = t.size >> l;
  if (s < 1) s = 1;
  q.s = s;
  int x0, y0;
  texel_coord(u, ul, s, x0, q.fx);
  texel_coord(v, vl, s, y0, q.fy);
  q.c0 = x0 & (s - 1);  // x0 mod s (s is a power of two), in [0, s) also for x0 < 0
  q.r0 = y0 < 0 ? 0 : (y0 > s - 1 ? s - 1 : y0);
  q.r1 = y0 + 1 < 0 ? 0 : (y0 + 1 > s - 1 ? s - 1 : y0 + 1);
  return q;
}

// Accumulates the contributions of the selected lanes (sel) at one level
// into an LDS window over their footprint (at most kWinTex entries), then
// adds the window's nonzero texel-channels to HBM and clears them, so the
// window is all zero again (it starts zeroed).  Converged code.
//
// The window sums in 32-bit fixed point: the pass scales every contribution
// by 2^k, k chosen from the largest magnitude in the wave so that each
// scaled value stays below 2^22, rounds it to an integer and adds it with an
// integer LDS atomic (on this chip a float LDS atomic costs some thirty
// times an integer one, a 64-bit one about twice a 32-bit one).  At most
// 64 lanes x 4 corners add to one entry, so its sum stays below 2^30.  A
// window texel-channel is converted back to float once: each contribution
// carries an error of at most 2^-23 of the wave's largest one, and the sum
// does not depend on the lanes' order.  A pass with a non-finite
// contribution adds markers instead and writes NaN to the texels it touches.
using WinT = unsigned int;

__device__ __forceinline__ WinT fix_of(float x, int k, bool finite) {
  return finite ? (WinT)(int)rintf(ldexpf(x, k)) : 1u;
}

__device__ __forceinline__ void window_pass(const Tex& t, float* __restrict__ gtex, WinT* win, bool sel,
                                            const Foot& q, float wl, const float (&gsv)[3], int off, int rmin,
                                            int rmax, int cmin, int cmax) {
  const int lane = threadIdx.x & 63;
  const int C = t.channels;
  const int ww = cmax - cmin + 1;
  const int n = (rmax - rmin + 1) * ww * C;
  // Per lane 4 corners x 3 channels.  (Merging lanes that share a bilinear
  // cell with DPP moves before the atomics paid off with float LDS atomics;
  // with integer ones it costs more than it saves.)
  const float w[4] = {(1.f - q.fx) * (1.f - q.fy), q.fx * (1.f - q.fy), (1.f - q.fx) * q.fy, q.fx * q.fy};
  float v[12];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float wk = sel ? wl * w[k] : 0.f;
    v[3 * k] = wk * gsv[0];
    v[3 * k + 1] = wk * gsv[1];
    v[3 * k + 2] = wk * gsv[2];
  }
  // the pass's scale from the largest magnitude still to be added (the bits
  // of non-negative floats order as the floats); amax < 2^e
  float amax = 0.f;
#pragma unroll
  for (int i = 0; i < 12; ++i) amax = fmaxf(amax, fabsf(v[i]));
  const int mb = wave_max_i(__float_as_int(amax));
  const bool finite = mb < 0x7F800000;
  const int e = ((mb >> 23) & 0xFF) - 126;
  const int ks = finite ? 22 - e : 0;
  wave_sync();
  if (sel && mb != 0) {
    // corner by corner (lanes sharing a cell add to the same entries in one
    // instruction: integer LDS atomics absorb that; rotating the corner and
    // channel order per lane against it cost more in selects than it saved)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int cell = (((k & 2 ? q.r1 : q.r0) - rmin) * ww + ((k & 1 ? q.c0 + 1 : q.c0) - cmin)) * C;
      atomicAdd(win + cell, fix_of(v[3 * k], ks, finite));
      if (C == 3) {
        atomicAdd(win + cell + 1, fix_of(v[3 * k + 1], ks, finite));
        atomicAdd(win + cell + 2, fix_of(v[3 * k + 2], ks, finite));
      }
    }
  }
  wave_sync();
  if (mb != 0) {
    // entry k = (row * ww + column) * C + channel; the row from a float
    // reciprocal of ww corrected by one either way (no integer division)
    const float inv_ww = 1.0f / (float)ww;
    for (int k = lane; k < n; k += 64) {
      const long long sum = (long long)(int)win[k];
      if (sum != 0) {
        win[k] = 0u;
        const float val = finite ? ldexpf((float)sum, -ks) : __int_as_float(0x7FC00000);
        const int texel = C == 3 ? k / 3 : k, ch = k - texel * C;
        int rr = (int)((float)texel * inv_ww);
        int cc = texel - rr * ww;
        if (cc < 0) {
          --rr;
          cc += ww;
        } else if (cc >= ww) {
          ++rr;
          cc -= ww;
        }
        int c = cmin + cc;
        if (c >= q.s) c -= q.s;
        atomicAdd(gtex + (int64_t)(off + (rmin + rr) * q.s + c) * C + ch, val);
      }
    }
  }
  wave_sync();
}

// Texel gradients of one map from the wave's samples, level by level.  When
// the footprint of all lanes at a level fits one window it is handled in one
// pass; otherwise (samples from far-apart parts of the map: a UV seam, or
// depth-peeled layers whose neighbouring pixels lie on different surfaces)
// the lanes are taken in groups: the first pending lane and every pending
// lane whose cell lies in a side x side box around it share a pass.
__device__ void wave_scatter_tex(const Tex& t, float* __restrict__ gtex, bool act, const TexScatter& ts,
                                 WinT* win) {
  const int BIG = 1 << 20;
  const int lane = threadIdx.x & 63;
  const int C = t.channels;
  const int side = C == 3 ? win_side(3) : win_side(1);  // side^2 C <= kWinTex
  bool done0 = !act, done1 = !(act && ts.has1);
  while (true) {
    int my = min(done0 ? BIG : ts.l0, done1 ? BIG : ts.l0 + 1);
    int lev = wave_min_i(my);
    if (lev >= BIG) break;
    bool use0 = !done0 && ts.l0 == lev;
    bool use1 = !done1 && ts.l0 + 1 == lev;
    bool part = use0 || use1;
    float wl = use0 ? (ts.has1 ? 1.f - ts.f : 1.f) : ts.f;
    done0 = done0 || use0;
    done1 = done1 || use1;
    const Foot q = foot_at(t, lev, ts.u, ts.v, ts.ul, ts.vl);
    const float gsv[3] = {ts.gs.x, ts.gs.y, ts.gs.z};
    const int off = t.off[lev];
    const int rmin = wave_min_i(part ? q.r0 : BIG), rmax = wave_max_i(part ? q.r1 : -1);
    const int cmin = wave_min_i(part ? q.c0 : BIG), cmax = wave_max_i(part ? q.c0 + 1 : -1);
    const bool whole = (rmax - rmin + 1) * (cmax - cmin + 1) * C <= kWinTex;
    bool pending = part;
    unsigned long long left = __ballot(pending);
    while (left) {
      bool in = pending;
      int r0 = rmin, r1 = rmax, c0 = cmin, c1 = cmax;
      if (!whole) {
        const int leader = __ffsll((long long)left) - 1;
        const int br = __builtin_amdgcn_readlane(q.r0, leader) - (side / 2 - 1);
        const int bc = __builtin_amdgcn_readlane(q.c0, leader) - (side / 2 - 1);
        in = pending && q.r0 >= br && q.r1 <= br + side - 1 && q.c0 >= bc && q.c0 + 1 <= bc + side - 1;
        r0 = wave_min_i(in ? q.r0 : BIG);
        r1 = wave_max_i(in ? q.r1 : -1);
        c0 = wave_min_i(in ? q.c0 : BIG);
        c1 = wave_max_i(in ? q.c0 + 1 : -1);
      }
      window_pass(t, gtex, win, in, q, wl, gsv, off, r0, r1, c0, c1);
      pending = pending && !in;
      left = __ballot(pending);
    }
  }
}

// The same for two 3-channel maps A and B of one size and layout whose
// lookups share level and weights: window entry (texel, c) holds channel c
// of A for c < 3 and channel c - 3 of B otherwise, and each map keeps a
// fixed-point scale of its own (from its own largest contribution), so each
// sum is what the map's own pass would give.
__device__ __forceinline__ void window_pass2(const Tex& t, float* __restrict__ ga, float* __restrict__ gb,
                                             WinT* win, bool sel, const Foot& q, float wl, const float (&gsa)[3],
                                             const float (&gsb)[3], int off, int rmin, int rmax, int cmin,
                                             int cmax) {
  const int lane = threadIdx.x & 63;
  const int ww = cmax - cmin + 1;
  const int n = (rmax - rmin + 1) * ww * 6;
  const float w[4] = {(1.f - q.fx) * (1.f - q.fy), q.fx * (1.f - q.fy), (1.f - q.fx) * q.fy, q.fx * q.fy};
  float va[12], vb[12];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float wk = sel ? wl * w[k] : 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      va[3 * k + c] = wk * gsa[c];
      vb[3 * k + c] = wk * gsb[c];
    }
  }
  float amax_a = 0.f, amax_b = 0.f;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    amax_a = fmaxf(amax_a, fabsf(va[i]));
    amax_b = fmaxf(amax_b, fabsf(vb[i]));
  }
  const int mba = wave_max_i(__float_as_int(amax_a)), mbb = wave_max_i(__float_as_int(amax_b));
  const bool fin_a = mba < 0x7F800000, fin_b = mbb < 0x7F800000;
  const int ks_a = fin_a ? 22 - (((mba >> 23) & 0xFF) - 126) : 0;
  const int ks_b = fin_b ? 22 - (((mbb >> 23) & 0xFF) - 126) : 0;
  wave_sync();
  if (sel && (mba | mbb) != 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int cell = (((k & 2 ? q.r1 : q.r0) - rmin) * ww + ((k & 1 ? q.c0 + 1 : q.c0) - cmin)) * 6;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        atomicAdd(win + cell + c, fix_of(va[3 * k + c], ks_a, fin_a));
        atomicAdd(win + cell + 3 + c, fix_of(vb[3 * k + c], ks_b, fin_b));
      }
    }
  }
  wave_sync();
  if ((mba | mbb) != 0) {
    const float inv_ww = 1.0f / (float)ww;
    for (int k = lane; k < n; k += 64) {
      const long long sum = (long long)(int)win[k];
      if (sum != 0) {
        win[k] = 0u;
        const int texel = k / 6, c6 = k - texel * 6;
        const bool is_b = c6 >= 3;
        const int ch = is_b ? c6 - 3 : c6;
        const bool fin = is_b ? fin_b : fin_a;
        const float val = fin ? ldexpf((float)sum, -(is_b ? ks_b : ks_a)) : __int_as_float(0x7FC00000);
        int rr = (int)((float)texel * inv_ww);
        int cc = texel - rr * ww;
        if (cc < 0) {
          --rr;
          cc += ww;
        } else if (cc >= ww) {
          ++rr;
          cc -= ww;
        }
        int c = cmin + cc;
        if (c >= q.s) c -= q.s;
        atomicAdd((is_b ? gb : ga) + (int64_t)(off + (rmin + rr) * q.s + c) * 3 + ch, val);
      }
    }
  }
  wave_sync();
}

// wave_scatter_tex for such a pair: one walk over the levels and lane
// groups for both maps (gsb: the lane's sample gradient of map B).
__device__ void wave_scatter_tex2(const Tex& t, float* __restrict__ ga, float* __restrict__ gb, bool act,
                                  const TexScatter& ts, f3 gsb, WinT* win) {
  const int BIG = 1 << 20;
  const int side = win_side(6);
  bool done0 = !act, done1 = !(act && ts.has1);
  while (true) {
    int my = min(done0 ? BIG : ts.l0, done1 ? BIG : ts.l0 + 1);
    int lev = wave_min_i(my);
    if (lev >= BIG) break;
    bool use0 = !done0 && ts.l0 == lev;
    bool use1 = !done1 && ts.l0 + 1 == lev;
    bool part = use0 || use1;
    float wl = use0 ? (ts.has1 ? 1.f - ts.f : 1.f) : ts.f;
    done0 = done0 || use0;
    done1 = done1 || use1;
    const Foot q = foot_at(t, lev, ts.u, ts.v, ts.ul, ts.vl);
    const float gsa_[3] = {ts.gs.x, ts.gs.y, ts.gs.z};
    const float gsb_[3] = {gsb.x, gsb.y, gsb.z};
    const int off = t.off[lev];
    const int rmin = wave_min_i(part ? q.r0 : BIG), rmax = wave_max_i(part ? q.r1 : -1);
    const int cmin = wave_min_i(part ? q.c0 : BIG), cmax = wave_max_i(part ? q.c0 + 1 : -1);
    const bool whole = (rmax - rmin + 1) * (cmax - cmin + 1) * 6 <= kWinTex;
    bool pending = part;
    unsigned long long left = __ballot(pending);
    while (left) {
      bool in = pending;
      int r0 = rmin, r1 = rmax, c0 = cmin, c1 = cmax;
      if (!whole) {
        const int leader = __ffsll((long long)left) - 1;
        const int br = __builtin_amdgcn_readlane(q.r0, leader) - (side / 2 - 1);
        const int bc = __builtin_amdgcn_readlane(q.c0, leader) - (side / 2 - 1);
        in = pending && q.r0 >= br && q.r1 <= br + side - 1 && q.c0 >= bc && q.c0 + 1 <= bc + side - 1;
        r0 = wave_min_i(in ? q.r0 : BIG);
        r1 = wave_max_i(in ? q.r1 : -1);
        c0 = wave_min_i(in ? q.c0 : BIG);
        c1 = wave_max_i(in ? q.c0 + 1 : -1);
      }
      window_pass2(t, ga, gb, win, in, q, wl, gsa_, gsb_, off, r0, r1, c0, c1);
      pending = pending && !in;
      left = __ballot(pending);
    }
  }
}

// Per-corner vertex gradients of one pixel: for corner c, acc[12c + 0..8]
// go to d(world position, normal, tangent) of vertex c and acc[12c + 9..11]
// to d(clip x, y, w) of vertex c in this view.
constexpr int kVtxAcc = 36;

// Column stride of the per-wave LDS table of vertex gradients (one column
// per lane, kVtxAcc rows; odd, against bank conflicts).
constexpr int kAccStride = 65;
constexpr int kVtxTable = kVtxAcc * kAccStride;  // floats per wave

// Where the texture-sample records of a pixel go: record 1 + slot of each
// map with a gradient buffer (slot < 0: none).
struct RecOut {
  float4* rec;
  int64_t P, o;
  int slot[4];
};

__device__ __forceinline__ void put_rec(const RecOut& ro, int m, const Lod& L, f3 gs, uint32_t& lv) {
  const int sl = ro.slot[m];
  if (sl < 0) return;
  lv &= ~(0xFFu << (8 * sl));
  lv |= (uint32_t)L.l0 << (8 * sl);
  st_nt(ro.rec + (1 + sl) * ro.P + ro.o, make_float4(gs.x, gs.y, gs.z, L.has1 ? L.f : 0.f));
}

// Adjoint of one pixel.  The vertex gradients are written to the pixel's
// column of the wave's LDS table (col[k * kAccStride], k < kVtxAcc) as they
// are computed, and each texture lookup's sample gradient record to HBM as
// soon as it is formed (neither is held in registers to the end); the maps'
// levels are returned in lv for the record header.  Returns false if the
// pixel contributes nothing.
// Gradient w.r.t. the texture coordinates and their screen derivatives.
struct UVGrad {
  float u, v, ux, vx, uy, vy;
};

// A lookup's derivatives parked in the pixel's LDS column between the
// lookups and the shading adjoint (the column is free then: the vertex
// gradients are written after), 3 rows per channel: d/du, d/dv and the level
// difference scaled by the LOD's derivative w.r.t. m (zero where the LOD is
// not differentiated).  Rows: kd 0-8, normal 9-17, orm 18-26, alpha 27-29;
// rows 30-35 keep the set-up's barycentrics and position indices until the
// end of the pixel's adjoint.
constexpr int kParkLam = 30;
__device__ __forceinline__ void stash_sample(float* col, int row, int ch, const TriSample& s, const Lod& L) {
  const float k = (L.has1 && L.grad) ? 0.5f / (L.m * 0.69314718055994531f) : 0.f;
  const float du[3] = {s.du.x, s.du.y, s.du.z}, dv[3] = {s.dv.x, s.dv.y, s.dv.z};
  const float dl[3] = {s.dl.x, s.dl.y, s.dl.z};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c >= ch) break;
    col[(row + 3 * c) * kAccStride] = du[c];
    col[(row + 3 * c + 1) * kAccStride] = dv[c];
    col[(row + 3 * c + 2) * kAccStride] = dl[c] * k;
  }
}

// Adjoint of one trilinear lookup w.r.t. (u, v) and, through the LOD, the
// screen derivatives, from the derivatives stash_sample parked.
__device__ __forceinline__ void uv_bwd_parked(const float* col, int row, int ch, const Tex& t, bool use_x,
                                              const PixelGeom& g, f3 gs, UVGrad& G) {
  if (t.size == 1) return;  // a one-texel map: nothing parked, no dependence on (u, v)
  const float gv[3] = {gs.x, gs.y, gs.z};
  float gu = 0.f, gw = 0.f, gm = 0.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c >= ch) break;
    gu += gv[c] * col[(row + 3 * c) * kAccStride];
    gw += gv[c] * col[(row + 3 * c + 1) * kAccStride];
    gm += gv[c] * col[(row + 3 * c + 2) * kAccStride];
  }
  G.u += gu;
  G.v += gw;
  // lod = 0.5 log2(m), m = max over x/y of |duv * size|^2 (gm is zero where
  // the LOD is not differentiated)
  const float S2 = (float)t.size * (float)t.size;
  if (use_x) {
    G.ux += gm * 2.f * g.ux * S2;
    G.vx += gm * 2.f * g.vx * S2;
  } else {
    G.uy += gm * 2.f * g.uy * S2;
    G.vy += gm * 2.f * g.vy * S2;
  }
}

// Adjoint of safe_normalize from the normalised vector y and inv = 1/|x|
// (0 when safe_normalize passed x through unchanged).
__device__ __forceinline__ f3 normalize_bwd_y(f3 y, float inv, f3 g) {
  return inv > 0.f ? inv * (g - dot(g, y) * y) : g;
}
__device__ __forceinline__ float inv_norm(f3 x) {
  float n2 = dot(x, x);
  return n2 > 1e-20f ? rsqrtf(n2) : 0.f;
}

// Adjoint of one pixel.  The vertex gradients are written to the pixel's
// column of the wave's LDS table (col[k * kAccStride], k < kVtxAcc) as they
// are computed, and each texture lookup's sample gradient record to HBM as
// soon as it is formed (neither is held in registers to the end); the maps'
// levels are returned in lv for the record header.  Returns false if the
// pixel contributes nothing.  Register pressure decides this kernel's
// speed (it runs latency-bound): the lookups' derivatives wait in LDS during
// the shading adjoint, and of the tangent frame only N, T', T and the two
// inverse lengths stay live.
template <bool ALPHA>
__device__ __forceinline__ bool shade_bwd_pixel(const ShadeArgs& a, const Pix& p,
                                                const float* __restrict__ gcolor, float* col,
                                                int& tri, int* vtx, const RecOut& ro, uint32_t& lv,
                                                float& u_out, float& v_out, float& lo_out) {
  int64_t o = ((int64_t)p.b * a.v.H + p.j) * a.v.W + p.i;
  uint32_t id = (uint32_t)a.vis[o];
  if (id == 0u) return false;
  f3 gc = mk(gcolor[3 * o], gcolor[3 * o + 1], gcolor[3 * o + 2]);
  const float g_alpha = ALPHA ? a.galpha[o] : 0.f;
  if (gc.x == 0.f && gc.y == 0.f && gc.z == 0.f && g_alpha == 0.f) return false;
  tri = (int)id - 1;
  PixelGeom g;
  pixel_geom(a.m, a.v, a.nrm, a.tan, p.b, p.i, p.j, (int)id - 1, g);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    col[(kParkLam + c) * kAccStride] = g.lam[c];
    col[(kParkLam + 3 + c) * kAccStride] = __int_as_float(g.v[c]);
  }
  const bool ggx_m = a.model == ADR_SHADE_GGX;
  // base colour and normal map: one level selection and one pair of
  // footprints when the two maps have one size
  const bool kn_same = same_layout(a.kd, a.nm);
  const Lod Lk = lod_select(a.kd, g.ux, g.vx, g.uy, g.vy);
  const Lod Ln = kn_same ? Lk : lod_select(a.nm, g.ux, g.vx, g.uy, g.vy);
  f3 kd, nt, ormv = mk(0.f, 0.f, 0.f);
  const TriFoot Fk = a.kd.size > 1 ? tri_foot(a.kd, g.u, g.v_, g.ul, g.vl, Lk) : TriFoot{};
  {
    const TriSample sk = tri_eval(a.kd, Fk, Lk);
    kd = sk.val;
    if (a.kd.size > 1) stash_sample(col, 0, 3, sk, Lk);
  }
  {
    const TriSample sn = kn_same ? tri_eval(a.nm, Fk, Ln) : tex_trilinear(a.nm, g.u, g.v_, g.ul, g.vl, Ln);
    nt = sn.val;
    if (a.nm.size > 1) stash_sample(col, 9, 3, sn, Ln);
  }
  Lod Lo{};
  if (ggx_m) {
    Lo = lod_select(a.orm, g.ux, g.vx, g.uy, g.vy);
    const TriSample so = tex_trilinear(a.orm, g.u, g.v_, g.ul, g.vl, Lo);
    ormv = so.val;
    if (a.orm.size > 1) stash_sample(col, 18, 3, so, Lo);
  }
  Lod La{};
  float alpha_t = 0.f;
  if (ALPHA && a.al.data) {
    La = lod_select(a.al, g.ux, g.vx, g.uy, g.vy);
    const TriSample sa = tex_trilinear(a.al, g.u, g.v_, g.ul, g.vl, La);
    alpha_t = sa.val.x;
    if (a.al.size > 1) stash_sample(col, 27, 1, sa, La);
  }
  // the tangent frame, compact: N, T', T and 1/|Ni|, 1/|T1| (B = N x T')
  const f3 N = g.N, Tp = g.Tp, T = g.T;
  const float invNi = inv_norm(g.Ni), invT1 = inv_norm(g.T1);
  f3 gkdv, gormv = mk(0.f, 0.f, 0.f), gm, gx;
  {
    const f3 Bt = cross(N, Tp);
    const f3 mraw = nt.x * Tp + nt.y * Bt + nt.z * N;
    const f3 n = safe_normalize(mraw);
    const f3 vraw = ld3(a.v.eye, p.b) - g.x;
    const f3 vdir = safe_normalize(vraw);
    const f3 l = ld3(a.v.light_dir, p.b);
    const f3 E = ld3(a.v.light_rgb, p.b);
    f3 gn, gv;
    if (ggx_m) {
      ggx_bwd(n, vdir, l, kd, ormv, E, gc, gn, gv, gkdv, gormv);
    } else {
      blinn_phong_bwd(n, vdir, l, kd, E, gc, gn, gv, gkdv);
    }
    // normal map: n = normalize(nt.x T' + nt.y B + nt.z N); view vector
    gm = safe_normalize_bwd(mraw, gn);
    gx = -safe_normalize_bwd(vraw, gv);
  }
  const f3 Bt = cross(N, Tp);
  const f3 gnt = mk(dot(gm, Tp), dot(gm, Bt), dot(gm, N));
  // textures
  UVGrad G{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  uv_bwd_parked(col, 0, 3, a.kd, Lk.use_x, g, gkdv, G);
  uv_bwd_parked(col, 9, 3, a.nm, Ln.use_x, g, gnt, G);
  if (ggx_m) uv_bwd_parked(col, 18, 3, a.orm, Lo.use_x, g, gormv, G);
  if (ALPHA && a.al.data) {
    // alpha = clamp(t, 0, 1): the gradient passes where t is inside [0, 1]
    const f3 gal = mk(alpha_t >= 0.f && alpha_t <= 1.f ? g_alpha : 0.f, 0.f, 0.f);
    uv_bwd_parked(col, 27, 1, a.al, La.use_x, g, gal, G);
    put_rec(ro, 3, La, gal, lv);
  }
  put_rec(ro, 0, Lk, gkdv, lv);
  put_rec(ro, 1, Ln, gnt, lv);
  if (ggx_m) put_rec(ro, 2, Lo, gormv, lv);
  u_out = g.u;
  v_out = g.v_;
  lo_out = pack_lo(g.ul, g.vl);
  // frame: B = N x T', T' = normalize(T1), T1 = T - (N.T) N, N = normalize(Ni)
  f3 gTp = nt.x * gm;
  f3 gBt = nt.y * gm;
  f3 gN = nt.z * gm;
  gN += cross(Tp, gBt);
  gTp += cross(gBt, N);
  f3 gT1 = normalize_bwd_y(Tp, invT1, gTp);
  float sNT = dot(N, T);
  f3 gT = gT1;
  float g_s = -dot(gT1, N);
  gN += (-sNT) * gT1;
  gN += g_s * T;
  gT += g_s * N;
  f3 gNi = normalize_bwd_y(N, invNi, gN);
  // interpolation: attributes -> barycentrics and vertex attribute gradients
  // (relative to corner 0, as in the forward pass: the barycentrics sum to
  // one, so a common offset of the three lambda gradients has no effect)
  // the barycentrics and corner indices parked after the set-up
  float lam[3];
  int vid[3], tid[3];
  int tri_o = tri;  // opaque, as the pixel below: no address kept live from the set-up
  asm volatile("" : "+v"(tri_o));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lam[c] = col[(kParkLam + c) * kAccStride];
    vid[c] = __float_as_int(col[(kParkLam + 3 + c) * kAccStride]);
    tid[c] = a.m.uv_tri[3 * tri_o + c];
  }
  float glam[3], glx[3], gly[3];
  f3 P0 = ld3(a.m.pos, vid[0]), N0 = ld3(a.nrm, vid[0]), T0 = ld3(a.tan, vid[0]);
  float u0 = a.m.uv[2 * tid[0]], v0 = a.m.uv[2 * tid[0] + 1];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int vi = vid[c];
    f3 P = ld3(a.m.pos, vi) - P0, Nv = ld3(a.nrm, vi) - N0, Tv = ld3(a.tan, vi) - T0;
    float uu = a.m.uv[2 * tid[c]] - u0, vv = a.m.uv[2 * tid[c] + 1] - v0;
    glam[c] = dot(P, gx) + dot(Nv, gNi) + dot(Tv, gT) + uu * G.u + vv * G.v;
    glx[c] = uu * G.ux + vv * G.vx;
    gly[c] = uu * G.uy + vv * G.vy;
    float lc = lam[c];
    float* da = col + 12 * c * kAccStride;
    da[0] = lc * gx.x; da[kAccStride] = lc * gx.y; da[2 * kAccStride] = lc * gx.z;
    da[3 * kAccStride] = lc * gNi.x; da[4 * kAccStride] = lc * gNi.y; da[5 * kAccStride] = lc * gNi.z;
    da[6 * kAccStride] = lc * gT.x; da[7 * kAccStride] = lc * gT.y; da[8 * kAccStride] = lc * gT.z;
    vtx[c] = vi;
  }
  // barycentrics (float64, like the forward set-up):
  // lambda_c = D_c / S, lx_c = (a_c - lambda_c A) / S * sx, ly_c likewise
  BaryD d;
  // the pixel made opaque to the compiler, which would otherwise keep the
  // set-up's pixel centre live from the first set-up to this one
  int pi = p.i, pj = p.j;
  asm volatile("" : "+v"(pi), "+v"(pj));
  bary_setup(a.m, a.v, p.b, pi, pj, vid, d);
  double iS = 1.0 / d.S;
  double A = d.a[0] + d.a[1] + d.a[2];
  double Bs = d.b[0] + d.b[1] + d.b[2];
  double gA = 0.0, gB = 0.0, gS = 0.0;
  double ga[3], gb[3], gD[3], dlam[3], dglam[3];
  const double sxd = a.v.pxs, syd = a.v.pys;  // per pixel
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int j1 = c == 2 ? 0 : c + 1, k1 = c == 0 ? 2 : c - 1;
    dlam[c] = (d.gx[j1] * d.gy[k1] - d.gy[j1] * d.gx[k1]) * iS;
    dglam[c] = glam[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double gu_ = glx[c] * sxd, gw_ = gly[c] * syd;
    double uc = (d.a[c] - dlam[c] * A) * iS, wc = (d.b[c] - dlam[c] * Bs) * iS;
    ga[c] = gu_ * iS;
    gb[c] = gw_ * iS;
    dglam[c] += -(gu_ * A + gw_ * Bs) * iS;
    gA += -gu_ * dlam[c] * iS;
    gB += -gw_ * dlam[c] * iS;
    gS += -(gu_ * uc + gw_ * wc) * iS;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ga[c] += gA;
    gb[c] += gB;
    gS += -dglam[c] * dlam[c] * iS;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) gD[c] = dglam[c] * iS + gS;
  // D_c = gx_j gy_k - gy_j gx_k, a_c = w_k gy_j - w_j gy_k, b_c = w_j gx_k - w_k gx_j
  double ggx[3] = {0.0, 0.0, 0.0}, ggy[3] = {0.0, 0.0, 0.0}, gw[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int j1 = c == 2 ? 0 : c + 1, k1 = c == 0 ? 2 : c - 1;
    ggx[j1] += gD[c] * d.gy[k1] - gb[c] * d.w[k1];
    ggx[k1] += -gD[c] * d.gy[j1] + gb[c] * d.w[j1];
    ggy[j1] += -gD[c] * d.gx[k1] + ga[c] * d.w[k1];
    ggy[k1] += gD[c] * d.gx[j1] - ga[c] * d.w[j1];
    gw[k1] += ga[c] * d.gy[j1] - gb[c] * d.gx[j1];
    gw[j1] += -ga[c] * d.gy[k1] + gb[c] * d.gx[k1];
  }
  // g = (x - w px, y - w py)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    col[(12 * c + 9) * kAccStride] = (float)ggx[c];
    col[(12 * c + 10) * kAccStride] = (float)ggy[c];
    col[(12 * c + 11) * kAccStride] = (float)(gw[c] - ggx[c] * d.px - ggy[c] * d.py);
  }
  return true;
}

// Pixels of one 64-wide wave (an 8x8 block) mostly lie on a few triangles,
// so their vertex gradients hit the same few addresses.  Each lane writes
// its 36 per-corner values to the wave's LDS window as a 36 x 64 table (row
// stride 65 floats: the 36 rows read by one instruction fall in different
// banks); then, per triangle present in the wave, lane k < 36 sums column
// entries of row k over the lanes on that triangle and issues one atomic.
// The member loops of all triangles together visit each lane once.

__device__ __forceinline__ void wave_vertex_scatter(const ShadeArgs& a, int b, bool act, int tri,
                                                    const int* vtx, const float* win,
                                                    unsigned long long* __restrict__ fclip,
                                                    unsigned long long* __restrict__ fattr, bool det) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(act);
  if (!todo) return;
  // the active lanes' columns of win were filled by the pixel adjoint
  wave_sync();
  while (todo) {
    int leader = __ffsll((long long)todo) - 1;
    int tl = __shfl(tri, leader);
    unsigned long long mine = __ballot(act && tri == tl);
    todo &= ~mine;
    int v0 = __shfl(vtx[0], leader), v1 = __shfl(vtx[1], leader), v2 = __shfl(vtx[2], leader);
    if (lane < kVtxAcc) {
      // four members per round, their LDS reads in flight together (a spent
      // mask reads the zero padding column kAccStride - 1)
      const float* row = win + lane * kAccStride;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
      unsigned long long m = mine;
      while (m) {
        const int j0 = __ffsll((long long)m) - 1;
        m &= m - 1;
        const int j1 = m ? __ffsll((long long)m) - 1 : kAccStride - 1;
        m &= m - 1;
        const int j2 = m ? __ffsll((long long)m) - 1 : kAccStride - 1;
        m &= m - 1;
        const int j3 = m ? __ffsll((long long)m) - 1 : kAccStride - 1;
        m &= m - 1;
        s0 += row[j0];
        s1 += row[j1];
        s2 += row[j2];
        s3 += row[j3];
      }
      const float sum = (s0 + s1) + (s2 + s3);
      if (sum != 0.f) {
        int c = lane / 12, comp = lane - 12 * c;
        int vi = c == 0 ? v0 : (c == 1 ? v1 : v2);
        const int64_t o = comp < 9 ? 9 * (int64_t)vi + comp
                                   : 4 * ((int64_t)b * a.m.n_pos + vi) + (comp == 11 ? 3 : comp - 9);
        acc_add(comp < 9 ? fattr + o : fclip + o, (double)sum, det);
      }
    }
  }
  wave_sync();
}

// Texture-sample records handed from the pixel adjoint to the texel
// scatter, per pixel of the view batch: rec[0] = (u, v, packed levels,
// packed low parts of u and v) with byte k of the packed levels the lower
// mip level l0 of gradient slot k (255: no contribution), and rec[1 + k] =
// (dL/dsample, weight of level l0 + 1) of slot k.
template <bool ALPHA>
__device__ __forceinline__ void shade_bwd_body(const ShadeBwdArgs& b, int bid, int nb) {
  __shared__ float table_all[4][kVtxTable];
  const ShadeArgs& a = b.s;
  const TexSlots& sl = b.sl;
  const float* __restrict__ gcolor = b.gcolor;
  float4* __restrict__ rec = b.rec;
  int tile = xcd_tile(bid, nb);
  Pix p = tile_pixel(tile, threadIdx.x, a.tiles_x, a.tiles_y, a.v.W, a.v.H);
  float* table = table_all[threadIdx.x >> 6];
  // the padding column stays zero (the pixel columns are 0..63)
  if ((threadIdx.x & 63) < kVtxAcc) table[(threadIdx.x & 63) * kAccStride + kAccStride - 1] = 0.f;
  int tri = -1;
  int vtx[3] = {0, 0, 0};
  const int64_t P = (int64_t)a.v.B * a.v.H * a.v.W;
  const int64_t o = ((int64_t)p.b * a.v.H + p.j) * a.v.W + p.i;
  const RecOut ro{rec, P, o, {sl.n > 0 ? sl.kd : -1, sl.n > 0 ? sl.nm : -1, sl.n > 0 ? sl.orm : -1,
                              ALPHA && sl.n > 0 ? sl.al : -1}};
  uint32_t lv = 0xFFFFFFFFu;
  float u = 0.f, v = 0.f, lo = 0.f;
  bool act = p.ok && shade_bwd_pixel<ALPHA>(a, p, gcolor, table + (threadIdx.x & 63), tri, vtx, ro, lv, u, v, lo);
  if (p.ok && sl.n > 0)
    st_nt(rec + o, make_float4(act ? u : 0.f, act ? v : 0.f, __uint_as_float(act ? lv : 0xFFFFFFFFu), act ? lo : 0.f));
  wave_vertex_scatter(a, p.b, act, tri, vtx, table, b.fclip, b.fattr, b.det);
}

// 4 waves per SIMD (128 VGPRs, 44 bytes of spills): 0.127 -> 0.119 ms on the paper loop; the
// compiler's own choice, 138 VGPRs, gives 3
template <bool ALPHA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_shade_bwd(ShadeBwdArgs b) {
  shade_bwd_body<ALPHA>(b, (int)blockIdx.x, (int)gridDim.x);
}
// the batched form (no alpha variant)
__device__ __forceinline__ void shade_bwd_body_opaque(const ShadeBwdArgs& b, int bid, int nb) {
  shade_bwd_body<false>(b, bid, nb);
}
ADR_KERNEL(__launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))), k_shade_bwd_opaque, ShadeBwdArgs,
           shade_bwd_body_opaque)

// Texel-gradient scatter of the recorded samples: a kernel of its own with
// few registers, so that enough waves are resident to hide the latency of
// the LDS atomics of the window accumulation.
__device__ __forceinline__ void tex_bwd_body(const TexBwdArgs& a, int bid, int nb) {
  __shared__ WinT win_all[4][kWinTex];
  int tile = xcd_tile(bid, nb);
  Pix p = tile_pixel(tile, threadIdx.x, a.tiles_x, a.tiles_y, a.v.W, a.v.H);
  const int64_t P = (int64_t)a.v.B * a.v.H * a.v.W;
  const int64_t o = ((int64_t)p.b * a.v.H + p.j) * a.v.W + p.i;
  float4 r0 = p.ok ? ld_nt(a.rec + o) : make_float4(0.f, 0.f, __uint_as_float(0xFFFFFFFFu), 0.f);
  const uint32_t lv = __float_as_uint(r0.z);
  WinT* win = win_all[threadIdx.x >> 6];
  for (int k = threadIdx.x & 63; k < kWinTex; k += 64) win[k] = 0u;
  float ul, vl;
  unpack_lo(r0.w, ul, vl);
  int k = 0;
  if (a.pair) {
    // slots 0 and 1 together where every lane looked both up at the same
    // level with the same weight (always, for maps of one size)
    const int l0 = (int)(lv & 0xFFu), l0b = (int)((lv >> 8) & 0xFFu);
    const bool act = p.ok && l0 != 0xFF, actb = p.ok && l0b != 0xFF;
    const float4 rk = act ? ld_nt(a.rec + P + o) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 rb = actb ? ld_nt(a.rec + 2 * P + o) : make_float4(0.f, 0.f, 0.f, 0.f);
    if (__ballot(act != actb || (act && (l0 != l0b || rk.w != rb.w))) == 0ull) {
      const TexScatter ts{r0.x, r0.y, ul, vl, l0, rk.w, rk.w > 0.f, mk(rk.x, rk.y, rk.z)};
      wave_scatter_tex2(a.t[0], a.g[0], a.g[1], act, ts, mk(rb.x, rb.y, rb.z), win);
      k = 2;
    }
  }
  for (; k < a.n; ++k) {
    const int l0 = (int)((lv >> (8 * k)) & 0xFFu);
    const bool act = p.ok && l0 != 0xFF;
    float4 rk = act ? ld_nt(a.rec + (1 + k) * P + o) : make_float4(0.f, 0.f, 0.f, 0.f);
    TexScatter ts{r0.x, r0.y, ul, vl, l0, rk.w, rk.w > 0.f, mk(rk.x, rk.y, rk.z)};
    wave_scatter_tex(a.t[k], a.g[k], act, ts, win);
  }
}
ADR_KERNEL(__launch_bounds__(256), k_tex_bwd, TexBwdArgs, tex_bwd_body)

static ShadeArgs make_args(const MeshD& m, const ViewsD& v, int model, const Tex& kd, const Tex& nm,
                           const Tex& orm, const Scratch& s, const uint64_t* vis) {
  ShadeArgs a{};
  a.m = m;
  a.v = v;
  a.model = model;
  a.kd = kd;
  a.nm = nm;
  a.orm = orm;
  a.nrm = s.nrm;
  a.tan = s.tan;
  a.vis = vis;
  a.tiles_x = (v.W + 15) / 16;
  a.tiles_y = (v.H + 15) / 16;
  return a;
}

Plan<ShadeFwdArgs> plan_shade_fwd(const MeshD& m, const ViewsD& v, int model, const Tex& kd, const Tex& nm,
                                   const Tex& orm, const Scratch& s, const uint64_t* vis, float* color,
                                   int32_t* tri_id, const Tex* al, float* alpha) {
  ShadeFwdArgs f{};
  f.s = make_args(m, v, model, kd, nm, orm, s, vis);
  if (al) f.s.al = *al;
  f.color = color;
  f.tri_id = tri_id;
  f.alpha = alpha;
  return {f, (unsigned)(f.s.tiles_x * f.s.tiles_y * v.B)};
}

hipError_t launch_shade_fwd(const MeshD& m, const ViewsD& v, int model, const Tex& kd,
                            const Tex& nm, const Tex& orm, const Scratch& s, const uint64_t* vis,
                            float* color, int32_t* tri_id, hipStream_t st, const Tex* al, float* alpha) {
  ADR_LAUNCH_1(k_shade_fwd, plan_shade_fwd(m, v, model, kd, nm, orm, s, vis, color, tri_id, al, alpha), st);
  return hipGetLastError();
}

int tex_slots(int model, const float* gkd, const float* gnm, const float* gorm, const float* gal) {
  return (gkd ? 1 : 0) + (gnm ? 1 : 0) + ((gorm && model == ADR_SHADE_GGX) ? 1 : 0) + (gal ? 1 : 0);
}

// Gradient slots in the order kd, normal, orm, alpha (maps with a gradient buffer).
static int make_slots(int model, const Tex& kd, const Tex& nm, const Tex& orm, float* gkd, float* gnm,
                      float* gorm, TexSlots& sl, TexBwdArgs& tb, const Tex* al = nullptr, float* gal = nullptr) {
  sl = TexSlots{-1, -1, -1, -1, 0};
  tb = TexBwdArgs{};
  auto add = [&](int& slot, const Tex& t, float* g) {
    slot = sl.n++;
    tb.t[slot] = t;
    tb.g[slot] = g;
  };
  if (gkd) add(sl.kd, kd, gkd);
  if (gnm) add(sl.nm, nm, gnm);
  if (gorm && model == ADR_SHADE_GGX) add(sl.orm, orm, gorm);
  if (gal && al && al->data) add(sl.al, *al, gal);
  tb.n = sl.n;
  // two maps of one size and level layout are looked up at the same levels
  // with the same weights (the level depends on the size only), so their
  // texel gradients can share the scatter's footprint
  tb.pair = 0;
  if (tb.n >= 2 && tb.t[0].size == tb.t[1].size && tb.t[0].levels == tb.t[1].levels && tb.t[0].channels == 3 &&
      tb.t[1].channels == 3) {
    tb.pair = 1;
    for (int l = 0; l <= tb.t[0].levels; ++l) tb.pair &= tb.t[0].off[l] == tb.t[1].off[l];
  }
  return sl.n;
}

Plan<ShadeBwdArgs> plan_shade_bwd(const MeshD& m, const ViewsD& v, int model, const Tex& kd, const Tex& nm,
                                   const Tex& orm, float* gkd, float* gnm, float* gorm, const Scratch& s,
                                   const uint64_t* vis, const Tex* al, float* gal, const float* galpha) {
  ShadeBwdArgs b{};
  b.s = make_args(m, v, model, kd, nm, orm, s, vis);
  TexBwdArgs tb;
  make_slots(model, kd, nm, orm, gkd, gnm, gorm, b.sl, tb, al, gal);
  if (galpha) {
    if (al) b.s.al = *al;
    b.s.galpha = galpha;
  }
  b.gcolor = s.gcolor;
  b.rec = s.texrec;
  b.fclip = s.fix_clip;
  b.fattr = s.fix_attr;
  b.det = s.det;
  return {b, (unsigned)(b.s.tiles_x * b.s.tiles_y * v.B)};
}

hipError_t launch_shade_bwd(const MeshD& m, const ViewsD& v, int model, const Tex& kd,
                            const Tex& nm, const Tex& orm, float* gkd, float* gnm, float* gorm,
                            const Scratch& s, const uint64_t* vis, hipStream_t st, const Tex* al, float* gal,
                            const float* galpha) {
  const Plan<ShadeBwdArgs> p = plan_shade_bwd(m, v, model, kd, nm, orm, gkd, gnm, gorm, s, vis, al, gal, galpha);
  if (galpha) ADR_LAUNCH_1(k_shade_bwd<true>, p, st);
  else ADR_LAUNCH_1(k_shade_bwd<false>, p, st);
  return hipGetLastError();
}

// ---- deterministic texel gradients: segmented reduction by bilinear cell ----
//
// Every (pixel, map, level) sample is one entry, written at a position fixed
// by those three indices and keyed by the bilinear cell of the sample: the
// 2x2 texels (x0, y0) .. (x0 + 1, y0 + 1) it reads, x0 wrapped and y0 in
// [-1, s - 1] (a row outside the level clamps to its edge, so a lower y0
// reads the same texels as -1 and a higher one the same as s - 1).  A level
// of size s has s (s + 1) cells, numbered (y0 + 1) s + x0 after the cells of
// the coarser... finer levels before it, the slots' chains one after the
// other; entries without a sample get the key `total`.  The value of an
// entry is the sample's adjoint times its level weight, a (3 floats), and
// its bilinear fractions fx, fy.  A stable radix sort by key groups each
// cell's entries in the fixed order of their positions; each group's four
// corner sums, c(cx, cy) = sum of (cx ? fx : 1 - fx) (cy ? fy : 1 - fy) a,
// are formed in that order (pieces within a tile of 2048 sorted entries by
// one thread each, groups that cross tiles joined tile after tile) and
// stored at the group's first sorted position.  Four passes then add corner
// (cx, cy) of every group to its texel (x0 + cx, y0 + cy).  Within one pass
// no two cells reach the same texel: a cell on row -1 holds both its rows'
// sums in its lower corners and one on row s - 1 in its upper corners (their
// two rows are the same texels), so each texel adds its at most four corner
// sums in pass order.  Keying by cell instead of by texel sorts a quarter of
// the entries.

struct TexDetArgs {
  TexBwdArgs tb;
  uint32_t base[5];               // first key of each slot; base[n] = total
  int coff[4][kMaxLevels + 1];    // first cell of each level within its slot
  int64_t E;                      // entries = n * P * 2
};

// Corner sums of a group, corner-major: (cx, cy) at 3 (2 cy + cx).
struct Corners {
  float v[12];
};

__device__ __forceinline__ void corners_add(Corners& c, float4 e, float fy) {
  const float wx[2] = {1.f - e.w, e.w}, wy[2] = {1.f - fy, fy};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float w = wx[q & 1] * wy[q >> 1];
    c.v[3 * q] += w * e.x;
    c.v[3 * q + 1] += w * e.y;
    c.v[3 * q + 2] += w * e.z;
  }
}

__device__ __forceinline__ void corners_store(float4* __restrict__ p, const Corners& c) {
  p[0] = make_float4(c.v[0], c.v[1], c.v[2], c.v[3]);
  p[1] = make_float4(c.v[4], c.v[5], c.v[6], c.v[7]);
  p[2] = make_float4(c.v[8], c.v[9], c.v[10], c.v[11]);
}

__device__ __forceinline__ Corners corners_load(const float4* __restrict__ p) {
  Corners c;
  const float4 a = p[0], b = p[1], d = p[2];
  c.v[0] = a.x; c.v[1] = a.y; c.v[2] = a.z; c.v[3] = a.w;
  c.v[4] = b.x; c.v[5] = b.y; c.v[6] = b.z; c.v[7] = b.w;
  c.v[8] = d.x; c.v[9] = d.y; c.v[10] = d.z; c.v[11] = d.w;
  return c;
}

__global__ __launch_bounds__(256) void k_tex_det_emit(TexDetArgs a, uint32_t* __restrict__ keys,
                                                      uint32_t* __restrict__ idx, float4* __restrict__ vals,
                                                      float* __restrict__ vfy) {
  const TexBwdArgs& tb = a.tb;
  const int64_t P = (int64_t)tb.v.B * tb.v.H * tb.v.W;
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= P) return;
  const float4 r0 = tb.rec[o];
  const uint32_t lv = __float_as_uint(r0.z);
  const uint32_t none = a.base[tb.n];
  float ul, vl;
  unpack_lo(r0.w, ul, vl);
  for (int k = 0; k < tb.n; ++k) {
    const int l0 = (int)((lv >> (8 * k)) & 0xFFu);
    float4 rk = make_float4(0.f, 0.f, 0.f, 0.f);
    if (l0 != 0xFF) rk = tb.rec[(1 + k) * P + o];
    const Tex& t = tb.t[k];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const bool on = l0 != 0xFF && (j == 0 || rk.w > 0.f);
      const int64_t e = ((int64_t)k * P + o) * 2 + j;
      uint32_t key = none;
      float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
      float fy = 0.f;
      if (on) {
        const int l = l0 + j;
        int sz = t.size >> l;
        if (sz < 1) sz = 1;
        int x0, y0;
        float fx;
        texel_coord(r0.x, ul, sz, x0, fx);
        texel_coord(r0.y, vl, sz, y0, fy);
        y0 = y0 < -1 ? -1 : (y0 > sz - 1 ? sz - 1 : y0);
        const float wl = j == 0 ? 1.f - rk.w : rk.w;
        key = a.base[k] + (uint32_t)(a.coff[k][l] + (y0 + 1) * sz + (x0 & (sz - 1)));
        val = make_float4(wl * rk.x, wl * rk.y, wl * rk.z, fx);
      }
      keys[e] = key;
      idx[e] = (uint32_t)e;
      vals[e] = val;
      vfy[e] = fy;
    }
  }
}

// Pieces of groups within each tile of 2048 sorted entries.  Each thread
// takes 8 consecutive entries (their value gathers issued together) and sums
// the runs of equal keys among them in order; a group whose entries all lie
// in one thread is stored at its first position.  A group that crosses
// threads is summed by the thread it starts in: its own run, then the first
// run of each following thread, in thread order.  part[2 tile] receives the
// sums of the tile's first piece when its group began in an earlier tile,
// part[2 tile + 1] those of its last piece when its group began in this tile
// and goes on into the next one (3 float4 each).
constexpr int kDetTile = 2048;
constexpr int kDetRun = kDetTile / 256;  // entries per thread

__global__ __launch_bounds__(256) void k_tex_det_pieces(TexDetArgs a, const uint32_t* __restrict__ sk,
                                                        const uint32_t* __restrict__ si,
                                                        const float4* __restrict__ vals,
                                                        const float* __restrict__ vfy,
                                                        float4* __restrict__ gsum, float4* __restrict__ part) {
  __shared__ float first_run[256][13];  // a thread's first run, when it continues an earlier thread's group
  __shared__ float last_run[256][13];   // a thread's last run, when its group starts there and goes on
  __shared__ int first_ends[256];       // first run: -1 none, 1 the group ends in this thread, 0 it goes on
  const int t = threadIdx.x;
  const int64_t tb0 = (int64_t)blockIdx.x * kDetTile;
  const int64_t te = min(tb0 + kDetTile, a.E);
  const uint32_t none = a.base[a.tb.n];
  const int64_t p0 = tb0 + (int64_t)kDetRun * t;
  uint32_t key[kDetRun], ix[kDetRun];
#pragma unroll
  for (int j = 0; j < kDetRun; ++j) {
    const int64_t q = p0 + j;
    key[j] = q < te ? sk[q] : none;
    ix[j] = q < te ? si[q] : 0u;
  }
  float4 v[kDetRun];
  float fy[kDetRun];
#pragma unroll
  for (int j = 0; j < kDetRun; ++j) {
    const bool on = key[j] < none;
    v[j] = on ? vals[ix[j]] : make_float4(0.f, 0.f, 0.f, 0.f);
    fy[j] = on ? vfy[ix[j]] : 0.f;
  }
  // the keys just before and just after this thread's entries
  const uint32_t kbefore = p0 > 0 && p0 < te ? sk[p0 - 1] : none;
  const uint32_t kafter = p0 + kDetRun < a.E ? sk[p0 + kDetRun] : none;
  Corners c;
#pragma unroll
  for (int q = 0; q < 12; ++q) c.v[q] = 0.f;
  int64_t run0 = p0;       // first position of the current run
  bool first = true;       // the current run is this thread's first
  bool open = false;       // a run is being summed
  int fend = -1;
#pragma unroll
  for (int j = 0; j < kDetRun; ++j) {
    if (key[j] < none) {
      corners_add(c, v[j], fy[j]);
      open = true;
      const uint32_t knext = j + 1 < kDetRun ? key[j + 1] : kafter;
      if (knext != key[j]) {  // the run ends here, and so does its group
        if (first && key[0] == kbefore) {
#pragma unroll
          for (int q = 0; q < 12; ++q) first_run[t][q] = c.v[q];
          fend = 1;
        } else {
          corners_store(gsum + 3 * run0, c);
        }
#pragma unroll
        for (int q = 0; q < 12; ++q) c.v[q] = 0.f;
        first = false;
        open = false;
        run0 = p0 + j + 1;
      }
    }
  }
  bool owner = false;  // a group that starts here goes on into the next thread
  if (open) {
    if (first && key[0] == kbefore) {
      // every entry of this thread continues an earlier group, which goes on
#pragma unroll
      for (int q = 0; q < 12; ++q) first_run[t][q] = c.v[q];
      fend = 0;
    } else {
#pragma unroll
      for (int q = 0; q < 12; ++q) last_run[t][q] = c.v[q];
      owner = true;
    }
  }
  first_ends[t] = fend;
  __syncthreads();
  // the tile's first piece, when its group began in an earlier tile: thread 0
  // adds the continuing first runs in thread order
  if (t == 0 && fend >= 0) {
#pragma unroll
    for (int q = 0; q < 12; ++q) c.v[q] = first_run[0][q];
    bool ended = fend == 1;
    for (int u = 1; !ended && u < 256; ++u) {
#pragma unroll
      for (int q = 0; q < 12; ++q) c.v[q] += first_run[u][q];
      ended = first_ends[u] == 1;
    }
    corners_store(part + 3 * (2 * blockIdx.x), c);
  }
  // a group that starts in this thread and goes on: its runs in thread
  // order, stored at its first position, or as the tile's last piece when it
  // goes on into the next tile
  if (owner) {
#pragma unroll
    for (int q = 0; q < 12; ++q) c.v[q] = last_run[t][q];
    bool ended = false;
    for (int u = t + 1; !ended && u < 256; ++u) {
#pragma unroll
      for (int q = 0; q < 12; ++q) c.v[q] += first_run[u][q];
      ended = first_ends[u] == 1;
    }
    if (ended) corners_store(gsum + 3 * run0, c);
    else corners_store(part + 3 * (2 * blockIdx.x + 1), c);
  }
}

// Groups that cross tiles: started in tile b, continued by the first pieces
// of the following tiles, added in tile order; stored at the group's first
// position.
__global__ __launch_bounds__(256) void k_tex_det_join(TexDetArgs a, const uint32_t* __restrict__ sk,
                                                      const float4* __restrict__ part, float4* __restrict__ gsum,
                                                      int64_t tiles) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= tiles) return;
  const int64_t te = min((b + 1) * kDetTile, a.E);
  if (te >= a.E) return;
  const uint32_t key = sk[te - 1];
  if (key >= a.base[a.tb.n] || sk[te] != key) return;
  // the group must start inside tile b: the keys are sorted, so if the key
  // before the tile is the same, the whole tile continues an earlier group
  const int64_t tb0 = b * kDetTile;
  if (tb0 > 0 && sk[tb0 - 1] == key) return;
  Corners c = corners_load(part + 3 * (2 * b + 1));
  for (int64_t t = b + 1; t < tiles; ++t) {
    const Corners d = corners_load(part + 3 * (2 * t));
#pragma unroll
    for (int q = 0; q < 12; ++q) c.v[q] += d.v[q];
    const int64_t ce = min((t + 1) * kDetTile, a.E);
    if (ce >= a.E || sk[ce] != key) break;
  }
  int64_t i = te - 1;
  while (i > tb0 && sk[i - 1] == key) --i;
  corners_store(gsum + 3 * i, c);
}

// Pass `corner` = 2 cy + cx: every group adds its corner (cx, cy) to its
// texel (see above for why no two groups of a pass reach the same texel).
__global__ __launch_bounds__(256) void k_tex_det_corner(TexDetArgs a, const uint32_t* __restrict__ sk,
                                                        const float4* __restrict__ gsum, int corner) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.E) return;
  const uint32_t key = sk[i];
  if (key >= a.base[a.tb.n] || (i > 0 && sk[i - 1] == key)) return;
  int k = 0;
  while (k + 1 < a.tb.n && key >= a.base[k + 1]) ++k;
  const Tex& t = a.tb.t[k];
  const int rel = (int)(key - a.base[k]);
  int l = 0;
  while (l + 1 < t.levels && rel >= a.coff[k][l + 1]) ++l;
  int sz = t.size >> l;
  if (sz < 1) sz = 1;
  const int cell = rel - a.coff[k][l];
  // sz is a power of two: the cell's row and column by shift and mask
  const int y0 = (cell >> __builtin_ctz((unsigned)sz)) - 1, x0 = cell & (sz - 1);
  const int cx = corner & 1, cy = corner >> 1;
  // only this pass's corner sums are read (two corners on a folded row)
  const float* cs = reinterpret_cast<const float*>(gsum + 3 * i);
  float g0, g1, g2;
  if (y0 == -1 || y0 == sz - 1) {
    // both rows are one row of texels: the lower corners of row -1, the
    // upper ones of row s - 1 carry the cell (row -1 wins when s = 1)
    const int keep = y0 == -1 ? 1 : 0;
    if (cy != keep) return;
    const int q0 = cx, q1 = 2 + cx;
    g0 = cs[3 * q0] + cs[3 * q1];
    g1 = cs[3 * q0 + 1] + cs[3 * q1 + 1];
    g2 = cs[3 * q0 + 2] + cs[3 * q1 + 2];
  } else {
    g0 = cs[3 * corner];
    g1 = cs[3 * corner + 1];
    g2 = cs[3 * corner + 2];
  }
  int row = y0 + cy;
  row = row < 0 ? 0 : (row > sz - 1 ? sz - 1 : row);
  const int col = (x0 + cx) & (sz - 1);
  float* g = a.tb.g[k] + (int64_t)(t.off[l] + row * sz + col) * t.channels;
  g[0] += g0;
  if (t.channels == 3) {
    g[1] += g1;
    g[2] += g2;
  }
}

hipError_t launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int bits,
                             uint32_t* hist, uint32_t* tmp, bool* in_first, hipStream_t st);

int64_t det_entries(const ViewsD& v, int slots) { return (int64_t)slots * v.B * v.H * v.W * 2; }

size_t det_vals_bytes(int64_t E) { return (size_t)E * 16 + (((size_t)E * 4 + 255) & ~(size_t)255) + (size_t)E * 48; }
size_t det_part_bytes(int64_t E) { return (size_t)((E + kDetTile - 1) / kDetTile) * 96; }

void det_carve(void* p, int64_t E, Scratch& s) {
  unsigned char* b = static_cast<unsigned char*>(p);
  s.det_vals = reinterpret_cast<float4*>(b);
  s.det_fy = reinterpret_cast<float*>(b + (size_t)E * 16);
  s.det_gsum = reinterpret_cast<float4*>(b + (size_t)E * 16 + (((size_t)E * 4 + 255) & ~(size_t)255));
}

hipError_t launch_tex_bwd_det(const ViewsD& v, int model, const Tex& kd, const Tex& nm, const Tex& orm,
                              float* gkd, float* gnm, float* gorm, const Scratch& s, hipStream_t st) {
  TexSlots sl;
  TexDetArgs a{};
  if (make_slots(model, kd, nm, orm, gkd, gnm, gorm, sl, a.tb) == 0) return hipSuccess;
  a.tb.rec = s.texrec;
  a.tb.v = v;
  uint32_t total = 0;
  for (int k = 0; k < a.tb.n; ++k) {
    const Tex& t = a.tb.t[k];
    a.base[k] = total;
    int c = 0;
    for (int l = 0; l <= kMaxLevels; ++l) {
      a.coff[k][l] = c;
      if (l < t.levels) {
        const int sz = (t.size >> l) < 1 ? 1 : (t.size >> l);
        c += sz * (sz + 1);
      }
    }
    total += (uint32_t)c;
  }
  a.base[a.tb.n] = total;
  a.E = det_entries(v, a.tb.n);
  const int64_t P = (int64_t)v.B * v.H * v.W;
  hipLaunchKernelGGL(k_tex_det_emit, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, a, s.det_k0, s.det_v0,
                     s.det_vals, s.det_fy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int bits = 1;
  while (bits < 32 && (1ull << bits) <= total) ++bits;
  bool first;
  if ((e = launch_radix_sort(s.det_k0, s.det_v0, s.det_k1, s.det_v1, a.E, bits, s.det_hist, s.det_tmp, &first,
                             st)) != hipSuccess)
    return e;
  const uint32_t* sk = first ? s.det_k0 : s.det_k1;
  const uint32_t* si = first ? s.det_v0 : s.det_v1;
  const int64_t tiles = (a.E + kDetTile - 1) / kDetTile;
  hipLaunchKernelGGL(k_tex_det_pieces, dim3((unsigned)tiles), dim3(256), 0, st, a, sk, si, s.det_vals, s.det_fy,
                     s.det_gsum, s.det_part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tex_det_join, dim3((unsigned)((tiles + 255) / 256)), dim3(256), 0, st, a, sk, s.det_part,
                     s.det_gsum, tiles);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int c = 0; c < 4; ++c) {
    hipLaunchKernelGGL(k_tex_det_corner, dim3((unsigned)((a.E + 255) / 256)), dim3(256), 0, st, a, sk, s.det_gsum,
                       c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// The atomic texel scatter (0 blocks without a gradient buffer).
Plan<TexBwdArgs> plan_tex_bwd(const ViewsD& v, int model, const Tex& kd, const Tex& nm, const Tex& orm, float* gkd,
                              float* gnm, float* gorm, const Scratch& s, const Tex* al, float* gal) {
  TexSlots sl;
  TexBwdArgs tb;
  const int n = make_slots(model, kd, nm, orm, gkd, gnm, gorm, sl, tb, al, gal);
  tb.rec = s.texrec;
  tb.v = v;
  tb.tiles_x = (v.W + 15) / 16;
  tb.tiles_y = (v.H + 15) / 16;
  return {tb, n == 0 ? 0u : (unsigned)(tb.tiles_x * tb.tiles_y * v.B)};
}

hipError_t launch_tex_bwd(const ViewsD& v, int model, const Tex& kd, const Tex& nm, const Tex& orm,
                          float* gkd, float* gnm, float* gorm, const Scratch& s, hipStream_t st, const Tex* al,
                          float* gal) {
  if (s.det) return launch_tex_bwd_det(v, model, kd, nm, orm, gkd, gnm, gorm, s, st);
  ADR_LAUNCH_1(k_tex_bwd, plan_tex_bwd(v, model, kd, nm, orm, gkd, gnm, gorm, s, al, gal), st);
  return hipGetLastError();
}

// ---- batched launches ----
hipError_t launch_shade_fwd_n(const Stage<ShadeFwdArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_shade_fwd, s, st);
  return hipGetLastError();
}
hipError_t launch_shade_bwd_n(const Stage<ShadeBwdArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_shade_bwd_opaque, s, st);
  return hipGetLastError();
}
hipError_t launch_tex_bwd_n(const Stage<TexBwdArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_tex_bwd, s, st);
  return hipGetLastError();
}

}  // namespace adr
