/*
 * adr.h -- C ABI of an MI355X (gfx950) implementation of the per-step
 * differentiable render loop of appearance-driven 3D model simplification
 * (Hasselgren, Munkberg, Lehtinen, Aittala, Laine: "Appearance-Driven
 * Automatic 3D Model Simplification").
 *
 * One optimisation step of the paper's objective (Sec. 3, Eq. 1) is
 *   adr_render_fwd(reference)  -> reference images I_ref(c, l)
 *   adr_render_fwd(latent)     -> latent images I_theta(c, l), image loss
 *   adr_render_bwd(latent)     -> dL/dtheta for vertex positions and texels
 *   adr_adam_step(theta)       -> Adam update (Sec. 5.3)
 * (adr_adam_step_maps updates mip-mapped maps with their chains' adjoint
 * and rebuild in the same launch), and adr_job_submit / adr_job_poll run whole optimisations (the paper's
 * statement of the problem: reference model, view/light distribution and
 * initial latent mesh and maps in, optimised mesh and maps out) inside the
 * library.
 *
 * Conventions
 *  - Pointers documented "device" are HIP device allocations (any allocator,
 *    e.g. PyTorch's); "host" pointers are ordinary CPU memory.
 *  - Every call validates its arguments before it launches anything and
 *    returns ADR_E_INVALID (with a message in adr_last_error()) on a bad
 *    shape, pointer or enum.  No C++ exception and no abort crosses the ABI.
 *  - render/adam calls enqueue work on `stream` and return without waiting;
 *    asynchronous HIP faults surface as ADR_E_HIP at the next synchronising
 *    call.  They BORROW caller memory until that stream work completes.
 *  - A context owns only scratch memory (grown on demand) and must be used
 *    by one host thread and one stream at a time; use one context per
 *    stream for concurrent work.
 *  - Images are [B, H, W, 3] float32 with row 0 at the bottom of the
 *    picture; vertex arrays are [n, 3] float32 row-major.
 */
#ifndef ADR_H
#define ADR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t adr_status;
#define ADR_OK 0
#define ADR_PENDING 1            /* job queued or running */
#define ADR_E_INVALID (-1)       /* bad shape, pointer or enum */
#define ADR_E_NOMEM (-2)         /* device or host allocation failed */
#define ADR_E_HIP (-3)           /* a HIP runtime call failed */
#define ADR_E_OVER_BUDGET (-4)   /* job can never fit the context's HBM budget */
#define ADR_E_NOTFOUND (-5)      /* unknown job id */
#define ADR_E_NONFINITE (-6)     /* job stopped on a non-finite loss or gradient */
#define ADR_E_UNIMPL (-7)        /* combination not implemented */

typedef struct adr_ctx adr_ctx;
typedef void* adr_stream;        /* hipStream_t; NULL = the legacy default stream */

/* Message of the last failing call on this thread ("" if none). */
const char* adr_last_error(void);

/* Context on HIP device `device`.  hbm_budget_bytes bounds the memory the job
 * server may keep resident (0 = free memory at creation minus 4 GiB). */
adr_status adr_ctx_create(int32_t device, uint64_t hbm_budget_bytes, adr_ctx** out);
adr_status adr_ctx_destroy(adr_ctx* ctx);

/* ------------------------------------------------------------------ data */

#define ADR_TEX_F32 0            /* float32 texels, `channels` of them */
#define ADR_TEX_RGBA8 1          /* 4 x uint8 unorm texels (x/255), rgb used */

/* A square power-of-two texture with its mip chain, level-major and
 * contiguous: level l has s_l = max(1, size >> l) rows of s_l texels, row r
 * holding texel rows v, starting at texel offset sum_{k<l} s_k^2.  Texel
 * centres sit at (i + 0.5) / s_l; lookups wrap in u and clamp in v. */
typedef struct adr_texture {
  void* data;                    /* device */
  int32_t size;                  /* level-0 width = height, power of two, 1..16384 */
  int32_t levels;                /* 1 .. log2(size) + 1 */
  int32_t channels;              /* F32: 1 or 3; RGBA8: 4 */
  int32_t format;                /* ADR_TEX_F32 or ADR_TEX_RGBA8 */
} adr_texture;

/* Triangle mesh with a separate UV index buffer (UV seams do not split
 * position vertices).  Triangles are listed counter-clockwise seen from
 * outside; both windings are rasterized. */
typedef struct adr_mesh {
  const float* pos;              /* device [n_pos, 3] */
  const int32_t* tri;            /* device [n_tri, 3] indices into pos */
  const float* uv;               /* device [n_uv, 2] */
  const int32_t* uv_tri;         /* device [n_tri, 3] indices into uv */
  const int32_t* adj;            /* device [n_tri, 3]: triangle across the edge opposite
                                    corner k, -1 on a boundary (adr_mesh_adjacency) */
  int32_t n_pos, n_tri, n_uv;
  /* Optional vertex frame (both or neither), device [n_pos, 3] unit smooth
   * normals and UV tangents as adr_mesh_frame returns them for these
   * positions (Sec. 5.1, "Tangent space").  When set, adr_render_fwd skips
   * the frame stage: for a mesh whose positions do not change, such as the
   * reference model.  adr_render_bwd always recomputes the frame. */
  const float* nrm;
  const float* tan;
} adr_mesh;

#define ADR_SHADE_BLINN_PHONG 0  /* E max(0,n.l) (kd + 0.04 max(0,n.h)^32) */
#define ADR_SHADE_GGX 1          /* diffuse + isotropic GGX lobe, Sec. 5.2 */

/* Materials of Sec. 5.2: base colour k_d, tangent-space normal map and, for
 * GGX, the (gamma, roughness, metalness) map with
 * k_s = (1-m) 0.04 + m k_d and k_s' = (1-gamma) k_s. */
typedef struct adr_material {
  int32_t model;                 /* ADR_SHADE_* */
  adr_texture kd;                /* F32 3 channels or RGBA8 */
  adr_texture normal;            /* F32 3 channels, tangent space (x along T, y along N x T, z along N) */
  adr_texture orm;               /* F32 3 channels (gamma, r, m); GGX only */
  adr_texture alpha;             /* F32 1 channel transparency, clamped to [0, 1]; optional (data NULL:
                                    opaque); read by the depth-peeled entry points only */
} adr_material;

/* B cameras and directional lights (Sec. 3: random camera and light per
 * iteration). */
typedef struct adr_views {
  const float* mvp;              /* device [B, 16], row-major clip = M [p, 1] (OpenGL clip space) */
  const float* eye;              /* device [B, 3] camera position */
  const float* light_dir;        /* device [B, 3] unit vector towards the light */
  const float* light_rgb;        /* device [B, 3] light radiance */
  int32_t n_views, width, height;/* 1..4096 views, 1..4096 pixels per side */
} adr_views;

#define ADR_LOSS_L1 0            /* mean |x - ref| */
#define ADR_LOSS_L1_TONEMAP 1    /* mean |T(x) - T(ref)|, T(x) = Gamma_sRGB(log(x + 1)), Sec. 5.3 */
#define ADR_LOSS_L2 2            /* mean (x - ref)^2 (aggregate geometry, Sec. 4.4) */
#define ADR_LOSS_L2_TONEMAP 3    /* mean (T(x) - T(ref))^2 */

/* Forward outputs, caller-owned device buffers.  vis, color and (when a
 * reference image is given) dimage are the state adr_render_bwd reads; the
 * G-buffer itself is never stored, the backward pass recomputes it. */
typedef struct adr_fwd_out {
  uint64_t* vis;                 /* [B,H,W] required: depth << 32 | (triangle + 1), empty
                                    pixels 0xFFFFFFFF00000000 */
  float* color;                  /* [B,H,W,3] required: shaded colour before antialiasing */
  float* image;                  /* [B,H,W,3] nullable: antialiased image */
  float* dimage;                 /* [B,H,W,3] required with a reference: dL/d image */
  float* loss;                   /* [1] required with a reference: the image loss */
  int32_t* tri_id;               /* [B,H,W] nullable: 0 empty, else triangle + 1 */
  uint32_t* coverage;            /* [B,H,W] nullable: covering triangles before the depth test */
  float* aa;                     /* 8 floats per (sample) pixel, nullable, in two planes: [B,H,W]
                                    float4 (W, acc), the antialiasing each pixel receives with
                                    out = c + acc / max(1, W), then [B,H,W] float2, the crossing
                                    parameters of its pairs with the right and upper neighbours
                                    (the rest unused); written by the forward when set, read by
                                    the backward when set (it then evaluates no pair edge twice) */
} adr_fwd_out;

#define ADR_FWD_BUILD_MIPS 1     /* rebuild levels 1.. of every F32 map from level 0 first */
#define ADR_FWD_NO_AA 2          /* skip silhouette antialiasing (image = color) */
#define ADR_MSAA_2X2 16          /* fwd and bwd: multisampled visibility (Sec. 5.2, "Antialiasing"):
                                    visibility on a 2x2 sample grid per pixel, each sample's
                                    triangle shaded once per pixel at the pixel centre, silhouette
                                    antialiasing between adjacent samples, pixel = mean of its
                                    samples.  vis, color, tri_id, coverage are then per sample
                                    ([B, 2H, 2W]); image, dimage, the loss and ref_image stay per
                                    pixel */
#define ADR_MSAA_4X4 32          /* as ADR_MSAA_2X2 with a 4x4 sample grid */
#define ADR_INDEPENDENT_MIPS 8   /* every mip level of the F32 maps is its own latent variable
                                    (Sec. 4.2): bwd leaves each level's gradient in place (no
                                    mip adjoint), so levels >= 1 of the gradients are outputs and
                                    Adam runs over whole chains; fwd rejects it together with
                                    ADR_FWD_BUILD_MIPS */
#define ADR_BWD_DEFER_MIP_ADJOINT 64 /* bwd (plain and depth-peeled): leave the mip adjoint of the
                                    map gradients to adr_adam_step_maps: each level of a gradient
                                    chain keeps the gradient w.r.t. its own texels (levels >= 1
                                    are then non-zero on exit).  Ignored by the forwards */
#define ADR_DETERMINISTIC 4      /* fwd and bwd: results identical bit for bit from run to run.
                                    Vertex-side sums (frame, clip and attribute adjoints, face
                                    terms) use 64-bit fixed point (2^-40 resolution, |sum| below
                                    2^23); texel gradients are a segmented reduction: all
                                    contributions sorted by texel (stable radix sort on a fixed
                                    emission order) and summed in that order.  Slower; the
                                    texel path needs 24 + 8 bytes per pixel, map, level and
                                    corner of scratch. */

/* Render B views of a mesh (Sec. 3 and 5.2): vertex normals and tangents
 * (Sec. 5.1), fixed-point rasterization, perspective-correct interpolation,
 * trilinear texture lookups, deferred shading, silhouette antialiasing and,
 * if ref_image is not NULL, the image loss of Sec. 5.3 against it.
 * ref_image: device [B,H,W,3] or NULL.  out: see adr_fwd_out.
 * Returns ADR_E_INVALID on bad arguments, ADR_E_NOMEM if scratch cannot
 * grow, ADR_E_HIP on a failed launch. */
adr_status adr_render_fwd(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                          const adr_views* views, const float* ref_image, int32_t loss_kind,
                          const adr_fwd_out* out, int32_t flags, adr_stream stream);

/* Forward render that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, checks, outputs and
 * kernels as adr_render_fwd.  Its scratch (snapped vertices, triangle
 * orientations, lists and queue, the vertex frame and its float64
 * accumulators, loss partials, the multisampled image) is carved from one
 * static device array of ADR_NOALLOC_SCRATCH_BYTES that every device the
 * library runs on holds until the process ends (its address is looked up
 * by adr_ctx_create).  That covers, e.g., 8 views of a 297,680-triangle mesh
 * (about 51 MB); an input that needs more returns ADR_E_INVALID before any
 * launch, with the size in adr_last_error().  All calls on one device share
 * that device's array, which keeps the last call's contents: calls that
 * overlap on one device (other host threads, or streams not ordered with
 * each other) race and give wrong results.  Stages are not timed
 * (adr_ctx_profile), and a following adr_render_bwd recomputes the
 * geometry instead of reusing this call's scratch. */
#define ADR_NOALLOC_SCRATCH_BYTES (64ull << 20)
adr_status adr_render_fwd_noalloc(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                                  const adr_views* views, const float* ref_image, int32_t loss_kind,
                                  const adr_fwd_out* out, int32_t flags, adr_stream stream);

/* Gradient buffers, caller-owned device memory.  Each is accumulated into
 * (+=).  Map gradients use the full mip-chain layout of their texture:
 * level 0 receives the gradient w.r.t. the level-0 texels (coarser levels
 * being box averages of level 0), levels 1.. are scratch that must be zero
 * on entry and are left zero; with ADR_INDEPENDENT_MIPS every level receives
 * the gradient w.r.t. its own texels. */
typedef struct adr_grads {
  float* pos;                    /* [n_pos,3] nullable */
  float* vnormal;                /* [n_pos,3] nullable: OVERWRITTEN with dL/d(smooth vertex
                                    normals), the part of pos's gradient that flows through them */
  float* kd;                     /* nullable; F32 kd only */
  float* normal;                 /* nullable */
  float* orm;                    /* nullable; GGX only */
  float* alpha;                  /* nullable; depth-peeled entry points with an alpha map only */
} adr_grads;

/* Hand-written adjoint of adr_render_fwd w.r.t. vertex positions and F32
 * texels (Sec. 3: gradients of the loss w.r.t. the latent parameters).
 * saved: the adr_fwd_out of the forward call with the same arguments
 * (vis, color and dimage are read).  When the context's previous call was
 * that forward (same mesh, views, deterministic flag and stream, and
 * saved->vis its out->vis), the vertex frame, snapped vertices and triangle
 * orientations it left in the context's scratch are reused instead of
 * recomputed; any other call in between makes the backward recompute them.  dloss: device [1] scale of the loss
 * gradient (NULL = 1).  Return values as adr_render_fwd. */
adr_status adr_render_bwd(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                          const adr_views* views, const adr_fwd_out* saved,
                          const float* dloss, const adr_grads* grads, int32_t flags,
                          adr_stream stream);

/* ----------------------------------------------------------------- batches */

/* Many renders of uneven size stepped together: the paper's optimisation
 * (Sec. 3, Eq. 1) run for independent meshes at once, each with its own
 * views, reference images and parameters.  A batch runs each stage of
 * adr_render_fwd (and of adr_render_bwd) as ONE launch over the work of all
 * its items: item k owns a contiguous range of the launch's blocks, found by
 * the blocks from a per-stage device table of argument blocks and block
 * offsets, so a small item costs a few blocks of a launch instead of
 * launches of its own, and the small and large items of a stage share the
 * chip.  Everything is planned and allocated at creation: adr_batch_fwd and
 * adr_batch_bwd only launch kernels (no allocation, no host
 * synchronisation), so a caller can capture them into a HIP graph.  Results
 * are those of adr_render_fwd / adr_render_bwd called item by item with the
 * same arguments (the same bits with ADR_DETERMINISTIC). */
typedef struct adr_batch adr_batch;

typedef struct adr_batch_item {
  const adr_mesh* mesh;          /* as adr_render_fwd; a precomputed frame (nrm, tan) is used by
                                    forward-only items */
  const adr_material* mat;
  const adr_views* views;
  const float* ref_image;        /* device [B,H,W,3] or NULL (no loss) */
  int32_t loss_kind;             /* ADR_LOSS_*, with ref_image */
  const adr_fwd_out* out;        /* as adr_render_fwd */
  const adr_grads* grads;        /* NULL: forward only; else as adr_render_bwd (needs ref_image) */
  const float* dloss;            /* device [1] scale of the loss gradient, NULL = 1 */
  int32_t flags;                 /* ADR_FWD_NO_AA, ADR_DETERMINISTIC, ADR_INDEPENDENT_MIPS,
                                    ADR_BWD_DEFER_MIP_ADJOINT */
  int32_t tiny_bbox, med_bbox;   /* the item's raster work split as adr_ctx_set_raster (0: the
                                    context's) */
} adr_batch_item;

/* Validates n items (host array; the structures are copied, the device
 * buffers they name are not: they must outlive the batch, and each call
 * reads their contents at that time), allocates every item's scratch and the
 * launch tables (device memory held until adr_batch_destroy) and uploads the
 * tables (synchronous).  ADR_E_INVALID for an item adr_render_fwd or
 * adr_render_bwd would reject, for multisampling or ADR_FWD_BUILD_MIPS
 * (rebuild chains with adr_mip_build or adr_adam_step_maps instead), or a
 * stage of 2^31 blocks or more; ADR_E_NOMEM when the scratch does not fit. */
adr_status adr_batch_create(adr_ctx* ctx, int32_t n, const adr_batch_item* items, adr_batch** out);
/* The forward of every item (adr_render_fwd with the item's arguments), in
 * 9 to 11 launches on `stream`. */
adr_status adr_batch_fwd(adr_batch* b, adr_stream stream);
/* The backward of every item with gradients (adr_render_bwd with the item's
 * arguments; gradients are accumulated into).  It reuses the vertex frame,
 * snapped vertices and triangle orientations that the batch's last
 * adr_batch_fwd left in the items' scratch, so it must follow that forward
 * on the same stream with the meshes and views unchanged in between;
 * ADR_E_INVALID before any forward or when no item has gradients.  The
 * texel adjoint of ADR_DETERMINISTIC items (a sort per item) and the mip
 * adjoint of items without ADR_BWD_DEFER_MIP_ADJOINT or
 * ADR_INDEPENDENT_MIPS run item after item. */
adr_status adr_batch_bwd(adr_batch* b, adr_stream stream);
/* Items and device bytes (scratch and tables) of a batch; either out may be NULL. */
adr_status adr_batch_info(const adr_batch* b, int32_t* n_items, uint64_t* scratch_bytes);
/* Frees the batch's device memory (waits for the device). */
adr_status adr_batch_destroy(adr_batch* b);

/* ------------------------------------ order-independent transparency */

/* Depth-peeled rendering (Sec. 5.2, "Order-independent transparency"; the
 * aggregate-geometry application, Sec. 4.4).  Layer 0 is the plain
 * visibility; layer k keeps per pixel the nearest fragment strictly behind
 * layer k-1's (the two-sided test, on the 64-bit keys: depth, then triangle
 * id, so layer k is the pixel's k-th smallest fragment key).  Each layer is
 * shaded (colour c_k, alpha a_k = clamp(alpha map, 0, 1), or 1 without a
 * map), then the layers are blended back to front from a black background:
 * B_k = a_k c_k + (1 - a_k) C_{k+1} where layer k covers the pixel, else
 * C_{k+1}; C_k = silhouette antialiasing of B_k with layer k's keys;
 * image = C_0.  All buffers are caller-owned device memory, layer-major. */
typedef struct adr_oit_out {
  int32_t n_layers;              /* 1..16 */
  uint64_t* vis;                 /* [L,B,H,W] required: keys of each layer (empty 0xFFFFFFFF00000000) */
  float* color;                  /* [L,B,H,W,3] required: c_k (0 where empty) */
  float* alpha;                  /* [L,B,H,W] required: a_k (0 where empty) */
  float* blend;                  /* [L,B,H,W,3] required: B_k */
  float* comp;                   /* [L,B,H,W,3] required: C_k; C_0 is the image */
  float* dimage;                 /* [B,H,W,3] required with a reference: dL/d image */
  float* loss;                   /* [1] required with a reference */
  float* aa;                     /* 8 L B H W floats, nullable: each layer's received antialiasing,
                                    laid out as adr_fwd_out.aa, layer after layer */
} adr_oit_out;

/* Forward of the depth-peeled render and, with ref_image, the image loss of
 * C_0.  flags: ADR_FWD_BUILD_MIPS (alpha map included), ADR_FWD_NO_AA,
 * ADR_INDEPENDENT_MIPS; ADR_E_UNIMPL with multisampling or
 * ADR_DETERMINISTIC.  Scratch as adr_render_fwd. */
adr_status adr_render_oit_fwd(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                              const adr_views* views, const float* ref_image, int32_t loss_kind,
                              const adr_oit_out* out, int32_t flags, adr_stream stream);
/* Adjoint of adr_render_oit_fwd (saved: its outputs; vis, color, alpha,
 * blend, comp and dimage are read), layer by layer from the front:
 * antialiasing adjoint of layer k, then the blend adjoint (dc_k = a_k dB_k,
 * da_k = dB_k . (c_k - C_{k+1}), dC_{k+1} = (1 - a_k) dB_k where covered),
 * then the shading and texel adjoints of the layer.  grads as adr_render_bwd
 * plus grads->alpha.  flags: ADR_FWD_NO_AA, ADR_INDEPENDENT_MIPS. */
adr_status adr_render_oit_bwd(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                              const adr_views* views, const adr_oit_out* saved, const float* dloss,
                              const adr_grads* grads, int32_t flags, adr_stream stream);

/* One optimised tensor for adr_adam_step: n floats each, device. */
typedef struct adr_param {
  float* param;
  float* grad;                   /* set to zero on exit */
  float* m;
  float* v;
  int64_t n;
} adr_param;

/* Bias-corrected Adam (Sec. 5.3, "with default parameters": beta1 0.9,
 * beta2 0.999, eps 1e-8) over n_params tensors in one launch; t is the
 * 1-based step.  params: host array of descriptors.  Zeroes each gradient. */
adr_status adr_adam_step(adr_ctx* ctx, const adr_param* params, int32_t n_params, int32_t t,
                         float lr, float beta1, float beta2, float eps, adr_stream stream);

/* One optimised F32 map for adr_adam_step_maps: the variable is level 0 of
 * `tex`; `grad` has the chain layout of `tex` and holds the per-level
 * gradients left by a backward with ADR_BWD_DEFER_MIP_ADJOINT (or a folded
 * level-0 gradient and zero levels >= 1); m and v: Adam moments of level 0,
 * size^2 x channels floats each.  All device memory. */
typedef struct adr_map_param {
  adr_texture tex;
  float* grad;                   /* whole chain set to zero on exit */
  float* m;
  float* v;
} adr_map_param;

/* Adam on the level-0 texels of mip-mapped maps (Sec. 5.3) fused with the
 * chain's adjoint before it and its rebuild after it (the mip chain is the
 * map's texture representation, Sec. 4.2): per map, the level-0 gradient
 * plus the coarser levels' gradients pushed down by the adjoint of the 2x2
 * box filter, the same Adam update as adr_adam_step, the gradient chain
 * cleared, and levels 1.. of the map rebuilt from the new level 0.  Gives
 * the same bits as adr_render_bwd's mip adjoint, adr_adam_step and a
 * forward with ADR_FWD_BUILD_MIPS, in two launches per four maps; a
 * forward after it needs no ADR_FWD_BUILD_MIPS.  maps: host array of n_maps
 * descriptors (F32 maps only, ADR_E_INVALID otherwise); t: 1-based step. */
adr_status adr_adam_step_maps(adr_ctx* ctx, const adr_map_param* maps, int32_t n_maps, int32_t t, float lr,
                              float beta1, float beta2, float eps, adr_stream stream);

/* Smooth vertex normals and UV tangents of a mesh (Sec. 5.1, "Tangent
 * space": normals from area-weighted face normals, tangents from the UV
 * Jacobian, both normalised), into device arrays nrm_out and tan_out
 * [n_pos, 3]; mesh->nrm and mesh->tan are ignored.  Device work on
 * `stream`. */
adr_status adr_mesh_frame(adr_ctx* ctx, const adr_mesh* mesh, float* nrm_out, float* tan_out,
                          adr_stream stream);

/* Rebuild levels 1.. of a texture from level 0 (2x2 box average; RGBA8
 * rounds (a+b+c+d+2)/4).  Device work on `stream`. */
adr_status adr_mip_build(adr_ctx* ctx, const adr_texture* tex, adr_stream stream);

/* ------------------------------------------------ tessellation + displacement */

/* Displacement mapping on a tessellated base mesh (Sec. 5.1 Eq. 3): each
 * tessellated vertex v is p = sum_c w_c P[vidx_c] displaced along
 * n = normalize(sum_c w_c N[vidx_c]) by a bilinear level-0 lookup of the
 * scalar displacement map at duv (N = smooth vertex normals of the base
 * mesh, recomputed from its positions).  The table comes from
 * adr_tess_build (edge-midpoint subdivision applied `levels` times; the
 * canonical numbering is documented in the implementation). */
typedef struct adr_tess {
  const int32_t* vidx;           /* device [n_vert,3] base vertices */
  const float* w;                /* device [n_vert,3] weights (dyadic, sum 1) */
  const float* duv;              /* device [n_vert,2] displacement-map coordinates */
  int32_t n_vert;
} adr_tess;

/* Host: sizes of the tessellated mesh (vertices, triangles = n_tri 4^levels,
 * UVs = n_tri (2^levels+1)(2^levels+2)/2).  levels 0..6. */
adr_status adr_tess_counts(const int32_t* tri, int32_t n_tri, int32_t n_pos, int32_t levels,
                           int64_t* n_vert, int64_t* n_tri_out, int64_t* n_uv_out);
/* Host: the table (vidx, w, duv) and the tessellated topology (tess_tri into
 * the tessellated vertices, tess_uv / tess_uv_tri), all host arrays sized by
 * adr_tess_counts.  Inputs: tri [n_tri,3] into n_pos positions, uv_tri
 * [n_tri,3] into uv [n_uv,2].  UVs of lattice points are the float32
 * rounding of their float64 barycentric combination.  ADR_E_INVALID for
 * out-of-range indices, levels outside 0..6 or outputs beyond int32 range;
 * nothing is written then. */
adr_status adr_tess_build(const int32_t* tri, const int32_t* uv_tri, const float* uv, int32_t n_tri,
                          int32_t n_pos, int32_t n_uv, int32_t levels, int32_t* vidx, float* w,
                          float* duv, int32_t* tess_tri, float* tess_uv, int32_t* tess_uv_tri);
/* Tessellated, displaced positions pos_out [n_vert,3] (device) from the base
 * mesh (pos, tri, uv, uv_tri used) and the F32 1-channel displacement map.
 * Computed in float64 and rounded once to float32.  Device work on `stream`;
 * scratch (base vertex frame) lives in the context. */
adr_status adr_tess_fwd(adr_ctx* ctx, const adr_mesh* base, const adr_tess* tess,
                        const adr_texture* disp, float* pos_out, adr_stream stream);
/* Adjoint: accumulates dL/d base positions (g_base_pos [n_pos,3], through the
 * base vertex normals too) and dL/d displacement texels (g_disp, level-0
 * layout, nullable) from dL/d pos_out (g_pos_out [n_vert,3], device), which
 * is consumed: set to zero on exit, ready for the next step's accumulation. */
adr_status adr_tess_bwd(adr_ctx* ctx, const adr_mesh* base, const adr_tess* tess,
                        const adr_texture* disp, float* g_pos_out, float* g_base_pos,
                        float* g_disp, adr_stream stream);

/* Box filter of a supersampled image: in [n_views, k height, k width, 3],
 * out [n_views, height, width, 3], each output pixel the mean of its k x k
 * input samples (device).  The reference of the prefiltering application
 * (Sec. 4.2) is rendered at k times the resolution and filtered so.
 * k in 1..64.  Device work on `stream`. */
adr_status adr_image_downsample(adr_ctx* ctx, const float* in, int32_t n_views, int32_t height, int32_t width,
                                int32_t k, float* out, adr_stream stream);

/* ------------------------------------------------ Laplacian regularizer */

/* One-ring neighbour lists (CSR) of a mesh's position vertices, device. */
typedef struct adr_one_ring {
  const int32_t* offs;           /* [n_pos + 1] */
  const int32_t* nbr;            /* [offs[n_pos]] neighbours of vertex i in offs[i]..offs[i+1], ascending */
  int32_t n_pos;
} adr_one_ring;

/* Host: the one-ring (vertices sharing an edge) of every vertex, sorted
 * ascending.  offs: host [n_pos + 1]; nbr: host array of at least the count
 * (at most 6 n_tri), or NULL to only count; *n_nbr receives the count.
 * ADR_E_INVALID on out-of-range indices. */
adr_status adr_mesh_one_ring(const int32_t* tri, int32_t n_tri, int32_t n_pos, int32_t* offs, int32_t* nbr,
                             int64_t* n_nbr);

/* Uniform Laplacian regularizer (Sec. 5.3, "Objective function"):
 * delta_i = v_i - mean of its one-ring, L = (1/n) sum |delta_i - delta_ref_i|^2
 * (delta_ref NULL: absolute, delta_ref = 0).  Optional outputs (device):
 * delta_out [n_pos,3] receives delta (e.g. of the initial mesh, for the
 * relative form), loss [1] receives L, g_pos [n_pos,3] is accumulated with
 * lambda dL/dpos.  pos, delta_ref: device [n_pos,3].  The adjoint is a gather
 * over the one-ring (no atomics).  Device work on `stream`. */
adr_status adr_laplacian(adr_ctx* ctx, const adr_one_ring* ring, const float* pos, const float* delta_ref,
                         float lambda, float* delta_out, float* loss, float* g_pos, adr_stream stream);

/* ---------------------------------------------------------------- skinning */

/* Dense linear blend skinning (Sec. 5.1, "Animation & skinning", Eq. 2):
 * pos_out[i] = sum_b weights[i,b] M_b (pos[i], 1), every weight a variable
 * (no normalisation is applied).  pos [n_pos,3] bind-pose positions,
 * weights [n_pos,n_bones] row-major, bones [n_bones,3,4] row-major top rows
 * of each bone's affine transform for the frame (constants), all device.
 * Outputs (device): pos_out [n_pos,3]; blend_out [n_pos,12] (nullable) the
 * blended matrix sum_b w_ib M_b of each vertex, which the adjoint needs.
 * Computed on the matrix cores in float64 and rounded once to float32.
 * n_bones in 1..4096.  ADR_E_INVALID on bad sizes or missing pointers.
 * Device work on `stream`; no scratch. */
adr_status adr_skin_fwd(adr_ctx* ctx, const float* pos, const float* weights, const float* bones, int32_t n_pos,
                        int32_t n_bones, float* pos_out, float* blend_out, adr_stream stream);
/* Adjoint of adr_skin_fwd from dL/d pos_out (g_pos_out [n_pos,3], device),
 * which is consumed (set to zero on exit).  Accumulates g_pos [n_pos,3] +=
 * dL/d pos and g_weights [n_pos,n_bones] += dL/d weights (each nullable, not
 * aliasing g_pos_out).  blend: the forward's blend_out for the same weights
 * and bones.  Each output row is written by one wave: no atomics, the same
 * bits on every run. */
adr_status adr_skin_bwd(adr_ctx* ctx, const float* pos, const float* bones, const float* blend, int32_t n_pos,
                        int32_t n_bones, float* g_pos_out, float* g_pos, float* g_weights, adr_stream stream);

/* Stage timing.  When enabled, every render/adam call brackets each of its
 * kernel stages with HIP events on the call's stream; adr_ctx_profile_read
 * waits for them, returns per stage the summed milliseconds and the number
 * of launches since the last read, and starts a new window.  Stages:
 * 0 vertex frame, 1 transform, 2 raster, 3 shade, 4 antialias+loss,
 * 5 antialias adjoint, 6 shade adjoint, 7 mip adjoint, 8 mesh adjoint,
 * 9 adam, 10 mip build, 11 texel adjoint, 12 buffer clears and
 * conversions, 13 skinning, 14 skinning adjoint, 15 layer blending and its
 * adjoint (depth peeling), 16 map Adam over level 0 with the adjoint and
 * rebuild of the levels inside its 32x32 tiles, 17 the levels above the
 * tiles (both adr_adam_step_maps), 18 the image loss's reduction of the
 * per-block partial sums.  ms and count: host arrays of ADR_N_STAGES. */
#define ADR_N_STAGES 19
adr_status adr_ctx_profile(adr_ctx* ctx, int32_t enable);
/* As adr_ctx_profile for the stages whose bits (1 << stage) are set in
 * stage_mask, the others untimed (0 disables).  Each bracketed stage stalls
 * its stream for a few microseconds at the two event records, so timing one
 * stage inside a timed loop costs far less than timing all of them.
 * ADR_E_INVALID for bits at or above ADR_N_STAGES. */
adr_status adr_ctx_profile_stages(adr_ctx* ctx, uint32_t stage_mask);

/* Raster work split of a context (a tuning knob, results do not change):
 * a triangle whose pixel bounding box holds at most tiny_bbox pixel centres
 * is walked by one thread, up to med_bbox by one wave from a chip-wide queue,
 * larger ones are binned to 16x16 tiles.  Defaults 64 and 4096; ranges
 * 1 <= tiny_bbox <= 1024, tiny_bbox <= med_bbox <= 65536. */
adr_status adr_ctx_set_raster(adr_ctx* ctx, int32_t tiny_bbox, int32_t med_bbox);
adr_status adr_ctx_profile_read(adr_ctx* ctx, double* ms, int64_t* count);

/* Host helpers (no device work). */
/* adj[t*3+k] = triangle sharing the edge opposite corner k of t, or -1. */
adr_status adr_mesh_adjacency(const int32_t* tri, int32_t n_tri, int32_t* adj);
/* Camera matrices for eye = dist * dir[b] / |dir[b]| looking at the origin,
 * up +y (+z when the view direction is within 0.999 of +-y), vertical field
 * of view fov_deg, aspect width/height, OpenGL projection with near 0.1,
 * far 10.  dirs [B,3] host; mvp [B,16] and eye [B,3] host outputs. */
adr_status adr_views_build(const float* dirs, int32_t n, float dist, float fov_deg,
                           int32_t width, int32_t height, float* mvp, float* eye);

/* ------------------------------------------------------------- job server */

/* A whole simplification job (host pointers, deep-copied at admission). */
typedef struct adr_job_desc {
  /* reference model (fixed) */
  const float* ref_pos; const int32_t* ref_tri; const float* ref_uv; const int32_t* ref_uv_tri;
  int32_t ref_n_pos, ref_n_tri, ref_n_uv;
  int32_t model;                 /* ADR_SHADE_* for both reference and latent */
  const void* ref_kd; int32_t ref_kd_size, ref_kd_format;     /* level 0 only */
  const float* ref_normal; int32_t ref_normal_size;           /* F32 x3 level 0 */
  const float* ref_orm; int32_t ref_orm_size;                 /* F32 x3 level 0, GGX */
  /* initial latent model */
  const float* lat_pos; const int32_t* lat_tri; const float* lat_uv; const int32_t* lat_uv_tri;
  int32_t lat_n_pos, lat_n_tri, lat_n_uv;
  const void* lat_kd; int32_t lat_kd_size, lat_kd_format;
  const float* lat_normal; int32_t lat_normal_size;
  const float* lat_orm; int32_t lat_orm_size;
  int32_t opt_mask;              /* bit 0 pos, 1 kd, 2 normal, 3 orm */
  /* view / light distribution: per step, n_views directions uniform on the
   * sphere at distance dist and one random unit light per view (or the same
   * light for all views if light_per_view == 0), drawn from a counter-based
   * generator seeded with `seed` */
  uint64_t seed;
  int32_t n_views, width, height, light_per_view;
  float dist, fov_deg;
  /* optimisation */
  int32_t n_steps, loss_kind;
  float lr0, lr_decay_k;         /* lr_t = lr0 10^(-k (t-1)) */
} adr_job_desc;

#define ADR_JOB_QUEUED 0
#define ADR_JOB_RUNNING 1
#define ADR_JOB_DONE 2
#define ADR_JOB_FAILED 3

typedef struct adr_job_status {
  int32_t state;                 /* ADR_JOB_* */
  int32_t step;                  /* completed steps */
  float last_loss;
  float p50_ms, p99_ms;          /* per-step latency, enqueue to completion */
  uint64_t device_bytes;         /* resident footprint */
} adr_job_status;

typedef struct adr_job_result {  /* host buffers the caller allocates */
  float* pos;                    /* [lat_n_pos,3] */
  void* kd;                      /* level 0 of the latent kd */
  float* normal;                 /* level 0 */
  float* orm;                    /* level 0 (if GGX) */
} adr_job_result;

/* The cameras and lights a job draws at step `step` (0-based): for view b,
 * direction and light are unit vectors from three normal deviates each
 * (Box-Muller on SplitMix64 uniforms u_i = (mix(seed + (i+1) 0x9E3779B97F4A7C15)
 * >> 11) 2^-53, i = (step n_views + b) 8 + k, k 0..3 for the direction and
 * 4..7 for the light; with light_per_view == 0 every view of a step uses
 * view 0's light).  dirs, lights: host [n_views,3].  Host-only. */
adr_status adr_job_views(uint64_t seed, int32_t step, int32_t n_views, int32_t light_per_view,
                         float* dirs, float* lights);

/* Queue a job.  Returns ADR_E_OVER_BUDGET if its footprint can never fit the
 * context's budget.  The server thread starts on the first submit. */
adr_status adr_job_submit(adr_ctx* ctx, const adr_job_desc* desc, uint64_t* job_id);

/* State of a job.  With out != NULL and state DONE, copies the optimised
 * latent model into the caller's host buffers and releases the job (a later
 * poll returns ADR_E_NOTFOUND).  Returns ADR_OK, ADR_PENDING (queued or
 * running), ADR_E_NONFINITE (stopped on a non-finite loss), ADR_E_HIP (could
 * not be admitted or stepped; adr_last_error says why), ADR_E_NOTFOUND.  A
 * failed job is released by the poll that reports it. */
adr_status adr_job_poll(adr_ctx* ctx, uint64_t job_id, adr_job_status* st, adr_job_result* out);

#ifdef __cplusplus
}
#endif

#endif /* ADR_H */
