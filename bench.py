#!/usr/bin/env python3
"""Throughput of the appearance-driven simplification step on one MI355X.

A step is one pass of the whole render loop: sample cameras and lights
(drawn ahead of time, resident in HBM), render the reference model, render
the latent model with its loss, run the hand-written backward pass into
vertex positions and texels, and apply Adam.  The workload is the
paper-scale loop: a ~300k-triangle fbm-displaced sphere with 2048^2 base
colour, normal and ORM maps under GGX as the reference, a ~7k-triangle
latent sphere with 2048^2 float32 base-colour and normal maps and full mip
chains, 8 views of 512x512 per step, one random directional light per view,
L1 loss on tone-mapped colours.  Inputs are seeded synthetic stand-ins for
the paper's scanned assets.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one
GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Stages whose timing brackets exactly one kernel (roofline candidates), with
# that kernel and the source files that define it.
SINGLE_KERNEL_STAGES = {
    "tex_bwd": ("adr::k_tex_bwd", ["shade.hip"]),
    "shade_bwd": ("adr::k_shade_bwd<false>", ["shade.hip"]),
    "aa_bwd": ("adr::k_aa_bwd", ["aa.hip"]),
    "shade": ("adr::k_shade_fwd", ["shade.hip"]),
    "aa_loss": ("adr::k_aa_fwd", ["aa.hip"]),
    "adam": ("adr::k_adam", ["adam.hip"]),
    "adam_maps": ("adr::k_adam_maps_tiles", ["tex.hip"]),
    "skin_bwd": ("adr::k_skin_bwd", ["skin.hip"]),
}
COMMON_SOURCES = ["dev.h", "internal.h"]


def _code_only(text):
    """C++ source without comments and with whitespace runs collapsed (string
    literals kept as they are): an edit of comments or layout leaves it."""
    import re
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"':                                       # string literal
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return re.sub(r"\s+", " ", "".join(out)).strip()


def kernel_sources_sha(files):
    """sha256 over a kernel's source files and the shared headers, comments
    and layout stripped (a change of the code itself voids stored counters)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2104_03989_amd", "csrc")
    paths = [os.path.join(csrc, f) for f in list(files) + COMMON_SOURCES] + [os.path.join(ROOT, "include", "adr.h")]
    for path in paths:
        with open(path, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()


def pmc_traffic(workload, stage):
    """HBM bytes per launch of a stage's kernel from the committed counter
    summary, or None if absent or if the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.json")
    if stage not in SINGLE_KERNEL_STAGES or not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    k = d.get("kernels", {}).get(SINGLE_KERNEL_STAGES[stage][0])
    if not k or k.get("sources_sha256") != kernel_sources_sha(SINGLE_KERNEL_STAGES[stage][1]):
        return None
    return k["hbm_bytes_per_launch"]


def summarize_pmc(workload, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """Writes profiles/pmc_traffic_<workload>.json from rocprofv3 --pmc runs:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the bench, each scaled by
    the ratio of known bytes to the same counter on a 1 GiB device copy."""
    import csv
    import re

    def load(d, counter):
        out = {}
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if r["Counter_Name"] != counter:
                continue
            n = re.sub(r"^void ", "", re.sub(r"\(.*", "", r["Kernel_Name"]))
            out.setdefault(n, []).append(float(r["Counter_Value"]) * 1024.0)
        return out

    def copy_scale(d, counter):
        v = load(d, counter).get("__amd_rocclr_copyBuffer", [])
        v = [x for x in v if x > 1e8]
        return (1 << 30) / (sum(v) / len(v))

    sf, sw = copy_scale(copy_fetch_dir, "FETCH_SIZE"), copy_scale(copy_write_dir, "WRITE_SIZE")
    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    kernels = {}
    for stage, (name, files) in SINGLE_KERNEL_STAGES.items():
        if name not in fetch or name not in write:
            continue
        f = sum(fetch[name]) / len(fetch[name]) * sf
        w = sum(write[name]) / len(write[name]) * sw
        kernels[name] = {"stage": stage, "fetch_bytes_per_launch": round(f), "write_bytes_per_launch": round(w),
                         "hbm_bytes_per_launch": round(f + w), "launches": len(fetch[name]),
                         "sources_sha256": kernel_sources_sha(files)}
    bench = f"python3 /root/repo/bench.py --workload {workload} --steps 2 --warmup 1 --no-cpu-baseline --no-profile"
    out = {"workload": workload, "copy_scale_fetch": round(sf, 4), "copy_scale_write": round(sw, 4),
           "counters": "rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE (KiB per dispatch)",
           "commands": [f"cd /tmp && rocprofv3 --pmc {c} -d <dir> -o run --output-format csv -- {b}"
                        for c in ("FETCH_SIZE", "WRITE_SIZE")
                        for b in (bench, "python3 /root/repo/bench.py --calibrate-copy")],
           "kernels": kernels}
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path)


def summarize_valu(workload, pmc_dir):
    """Writes profiles/pmc_valu_<workload>.json from a rocprofv3 --pmc
    SQ_WAVES SQ_INSTS_VALU run: VALU wave-instructions per launch of each
    single-kernel stage's kernel, with a hash of its sources."""
    import csv
    import re
    acc = {}
    for r in csv.DictReader(open(os.path.join(pmc_dir, "run_counter_collection.csv"))):
        n = re.sub(r"^void ", "", re.sub(r"\(.*", "", r["Kernel_Name"]))
        acc.setdefault(n, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    kernels = {}
    for stage, (name, files) in SINGLE_KERNEL_STAGES.items():
        c = acc.get(name)
        if not c or "SQ_INSTS_VALU" not in c or "SQ_WAVES" not in c:
            continue
        valu = sum(c["SQ_INSTS_VALU"]) / len(c["SQ_INSTS_VALU"])
        waves = sum(c["SQ_WAVES"]) / len(c["SQ_WAVES"])
        kernels[name] = {"stage": stage, "waves_per_launch": round(waves), "valu_per_wave": round(valu / waves, 1),
                         "valu_per_launch": round(valu), "launches": len(c["SQ_WAVES"]),
                         "sources_sha256": kernel_sources_sha(files)}
    bench = f"python3 /root/repo/bench.py --workload {workload} --steps 2 --warmup 1 --no-cpu-baseline --no-profile"
    out = {"workload": workload, "counters": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU (per dispatch)",
           "command": f"cd /tmp && rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU -d <dir> -o run --output-format csv -- {bench}",
           "valu_peak": "256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction = 614.4 G/s",
           "kernels": kernels}
    path = os.path.join(ROOT, "profiles", f"pmc_valu_{workload}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_step(w, ctx, adr, torch, np, n_steps, seed, det=False, laplacian=False, tune=True, ctx_ref=None):
    """Upload the workload and return (step(t) closure, state).

    With ctx_ref (a second context) the reference renders run on a stream of
    their own, double-buffered: the reference of step t + 1 depends only on
    that step's cameras, so it overlaps step t's backward and Adam; a
    latent forward waits for its reference, and a reference render waits
    until the latent forward that last read its buffer has run."""
    overlap = ctx_ref is not None
    rctx = ctx_ref if overlap else ctx
    ref_mesh = adr.DeviceMesh(w.ref.mesh)
    rig = None
    if w.rig is None:
        ref_mesh.precompute_frame(ctx)      # the reference does not move
    else:
        # skinned meshes (Eq. 2): bind poses, dense weights and the bone
        # transforms of every frame stay resident; one frame per step
        rig = dict(bones=torch.from_numpy(np.ascontiguousarray(w.rig.bones)).cuda(),
                   ref_bind=ref_mesh.pos.clone(),
                   ref_w=torch.from_numpy(np.ascontiguousarray(w.rig.ref_weights)).cuda())
    ref_mat = adr.DeviceMaterial(w.ref, ctx=ctx)
    ts = disp = None
    if w.tess_levels:
        ts = adr.DeviceTess(w.latent.mesh, w.tess_levels)
        disp = adr.DeviceTexture(w.disp.data, "f32", levels=1)
        lat_mesh = ts.mesh
        adr.tess_fwd(ctx, ts, disp)
    else:
        lat_mesh = adr.DeviceMesh(w.latent.mesh)
    lat_mat = adr.DeviceMaterial(w.latent, ctx=ctx)
    B, H, W = w.dirs.shape[0], w.height, w.width
    # cameras and lights of every step, drawn on the host ahead of time
    g = np.random.Generator(np.random.PCG64(seed))
    dirs = g.normal(size=(n_steps, B, 3))
    lights = g.normal(size=(n_steps, B, 3))
    lights /= np.linalg.norm(lights, axis=2, keepdims=True)
    mvps, eyes = [], []
    for t in range(n_steps):
        m, e = adr.views_build(dirs[t], w.dist, w.fov_deg, W, H)
        mvps.append(m)
        eyes.append(e)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    mvp_d, eye_d, light_d = dev(np.stack(mvps)), dev(np.stack(eyes)), dev(lights)
    rgb_d = dev(np.ones((n_steps, B, 3)))
    views = [adr.DeviceViews(mvp_d[t], eye_d[t], light_d[t], rgb_d[t], W, H) for t in range(n_steps)]
    k = w.ref_ssaa   # supersampled reference (prefiltering): same cameras, k times the resolution
    ref_views = views if k == 1 else [adr.DeviceViews(mvp_d[t], eye_d[t], light_d[t], rgb_d[t], W * k, H * k)
                                      for t in range(n_steps)]
    # optimised parameters: positions and level 0 of the F32 maps
    params = []
    grads = {"pos": torch.zeros_like(lat_mesh.pos)}
    if rig is not None:
        rig.update(bind=lat_mesh.pos.clone(), w=torch.from_numpy(np.ascontiguousarray(w.weights)).cuda(),
                   blend=torch.zeros(lat_mesh.pos.shape[0], 12, device="cuda"))
        rig.update(g_bind=torch.zeros_like(rig["bind"]), g_w=torch.zeros_like(rig["w"]))
        params += [(rig["bind"], rig["g_bind"]), (rig["w"], rig["g_w"])]
        n_frames = rig["bones"].shape[0]
        adr.skin_fwd(ctx, rig["ref_bind"], rig["ref_w"], rig["bones"][0], out=ref_mesh.pos)
        adr.skin_fwd(ctx, rig["bind"], rig["w"], rig["bones"][0], out=lat_mesh.pos, blend=rig["blend"])
    elif ts is None:
        params.append((lat_mesh.pos, grads["pos"]))
    else:
        # base positions and the displacement map (Eq. 3); the tessellated
        # positions are recomputed every step
        g_base = torch.zeros_like(ts.base.pos)
        g_disp = torch.zeros_like(disp.data)
        params += [(ts.base.pos, g_base), (disp.data, g_disp)]
    independent = False
    maps = []    # mip-mapped maps: Adam fused with the chain's adjoint and rebuild
    for name in ("kd", "normal", "orm", "alpha"):
        if name not in w.optimize:
            grads[name] = None
            continue
        tex = getattr(lat_mat, name)
        grads[name] = tex.grad_buffer()
        if getattr(getattr(w.latent, name), "chain", None) is not None:
            independent = True       # every mip level is a variable
            params.append((tex.data, grads[name]))
        else:
            n0 = tex.size * tex.size
            maps.append((tex, grads[name], torch.zeros_like(tex.data[:n0]), torch.zeros_like(tex.data[:n0])))
    adam = [(p, gr, torch.zeros_like(p), torch.zeros_like(p)) for p, gr in params]
    n_params = sum(p.numel() for p, _ in params) + sum(m.numel() for _, _, m, _ in maps)
    n_map_params = sum(m.numel() for _, _, m, _ in maps)
    # map Adam's tile kernel: 32 B per level-0 float as Adam, plus per float
    # of the levels inside a 32x32 level-0 tile (1..5) the gradient read and
    # cleared and the rebuilt texel written (the levels above the tiles, a
    # second small launch, are not counted)
    def tile_level_floats(tex, m):
        c = m.numel() // (tex.size * tex.size)
        return c * sum((tex.size >> l) ** 2 for l in range(1, 6) if tex.size >> l)
    map_adam_bytes = sum(32 * m.numel() + 12 * tile_level_floats(tex, m) for tex, _, m, _ in maps)
    dflag = adr.DETERMINISTIC if det else 0
    if w.msaa > 1:
        dflag |= adr.MSAA_4X4 if w.msaa == 4 else adr.MSAA_2X2
    lflag = dflag | (adr.INDEPENDENT_MIPS if independent else adr.FWD_BUILD_MIPS)
    # in the loop the map Adam keeps the chains built: the forward rebuilds
    # nothing and the backward leaves the chains' adjoint to it
    sflag = lflag & ~adr.FWD_BUILD_MIPS
    bflag = sflag | (adr.BWD_DEFER_MIP_ADJOINT if maps else 0)
    nbuf = 2 if overlap else 1
    ref_outs = [adr.render_fwd(rctx, ref_mesh, ref_mat, ref_views[0], flags=dflag & adr.DETERMINISTIC)
                for _ in range(nbuf)]
    ref_imgs = [o["image"] if k == 1 else adr.image_downsample(rctx, o["image"], k) for o in ref_outs]
    ref_out, ref_img = ref_outs[0], ref_imgs[0]
    s_ref = torch.cuda.Stream() if overlap else None         # default priority
    ev_ref = [torch.cuda.Event() for _ in range(nbuf)]       # reference i rendered
    ev_used = [torch.cuda.Event() for _ in range(nbuf)]      # latent forward read reference i
    L = w.oit_layers
    if L:
        # depth-peeled latent (order-independent transparency)
        lat_out = adr.render_oit_fwd(ctx, lat_mesh, lat_mat, views[0], L, ref=ref_img, loss=w.loss, flags=lflag)
    else:
        lat_out = adr.render_fwd(ctx, lat_mesh, lat_mat, views[0], ref=ref_img, loss=w.loss,
                                 flags=lflag, want_image=False, want_tri_id=True)

    # the rasterizer's work split of each render from the autotuner (cached
    # per shape bucket; the split changes only the speed)
    from paper_2104_03989_amd.autotune import DEFAULT, Tuner
    split_ref = split_lat = DEFAULT
    if tune:
        tuner = Tuner()
        split_ref = tuner.pick(rctx, "ref", int(w.ref.mesh.tri.shape[0]), B, W * k,
                               lambda: adr.render_fwd(rctx, ref_mesh, ref_mat, ref_views[0], outputs=ref_out,
                                                      flags=dflag & adr.DETERMINISTIC))
        if L:
            split_lat = tuner.pick(ctx, f"latent_peel{L}", int(lat_mesh.tri.shape[0]), B, W * w.msaa,
                                   lambda: adr.render_oit_fwd(ctx, lat_mesh, lat_mat, views[0], L, ref=ref_img,
                                                              loss=w.loss, flags=sflag, outputs=lat_out))
        else:
            split_lat = tuner.pick(ctx, "latent", int(lat_mesh.tri.shape[0]), B, W * w.msaa,
                                   lambda: adr.render_fwd(ctx, lat_mesh, lat_mat, views[0], ref=ref_img, loss=w.loss,
                                                          flags=sflag, outputs=lat_out))
        tuner.save()

    # uniform Laplacian regularizer (absolute form: the latent starts as a
    # resampled sphere), lambda_0 by the heuristic, then the recursive decay
    lap = None
    if laplacian:
        base = ts.base if ts is not None else lat_mesh
        base_pos = rig["bind"] if rig is not None else base.pos
        ring = adr.DeviceOneRing(base.tri.cpu().numpy(), base.pos.shape[0])
        ld = torch.zeros(1, device="cuda")
        adr.laplacian(ctx, ring, base_pos, loss=ld)
        torch.cuda.synchronize()
        lam0 = 0.25 * float(lat_out["loss"][0]) / max(float(ld[0]), 1e-30)
        lams = [lam0]
        for i in range(1, n_steps):
            lams.append((lams[-1] - 0.02 * lam0) * 10.0 ** (-1e-6 * i) + 0.02 * lam0)
        g_lap = g_base if ts is not None else (rig["g_bind"] if rig is not None else grads["pos"])
        lap = (ring, base_pos, lams, g_lap)

    def render_reference(t, i, stream):
        if rig is not None:
            adr.skin_fwd(rctx, rig["ref_bind"], rig["ref_w"], rig["bones"][t % n_frames], out=ref_mesh.pos,
                         stream=stream)
        rctx.set_raster(*split_ref)
        adr.render_fwd(rctx, ref_mesh, ref_mat, ref_views[t % n_steps], outputs=ref_outs[i],
                       flags=dflag & adr.DETERMINISTIC, stream=stream)
        if k > 1:
            adr.image_downsample(rctx, ref_outs[i]["image"], k, out=ref_imgs[i], stream=stream)

    def step(t, with_reference=True):
        """One step; without the reference render it reuses the reference
        image already in its buffer (the latent-only rate)."""
        v = views[t % n_steps]
        i = t % nbuf
        cur = torch.cuda.current_stream()
        if not with_reference:
            pass
        elif overlap:
            s_ref.wait_event(ev_used[i])
            render_reference(t, i, s_ref)
            ev_ref[i].record(s_ref)
            cur.wait_event(ev_ref[i])
        else:
            render_reference(t, i, None)
        ref_img = ref_imgs[i]
        if ts is not None:
            adr.tess_fwd(ctx, ts, disp)
        if rig is not None:
            bones = rig["bones"][t % n_frames]
            adr.skin_fwd(ctx, rig["bind"], rig["w"], bones, out=lat_mesh.pos, blend=rig["blend"])
        ctx.set_raster(*split_lat)
        if L:
            adr.render_oit_fwd(ctx, lat_mesh, lat_mat, v, L, ref=ref_img, loss=w.loss, flags=sflag, outputs=lat_out)
            ev_used[i].record(cur)
            adr.render_oit_bwd(ctx, lat_mesh, lat_mat, v, lat_out, grads, flags=bflag)
        else:
            adr.render_fwd(ctx, lat_mesh, lat_mat, v, ref=ref_img, loss=w.loss, flags=sflag, outputs=lat_out)
            ev_used[i].record(cur)
            adr.render_bwd(ctx, lat_mesh, lat_mat, v, lat_out, grads, flags=bflag)
        if ts is not None:
            adr.tess_bwd(ctx, ts, disp, grads["pos"], g_base, g_disp)
        if rig is not None:
            adr.skin_bwd(ctx, rig["bind"], bones, rig["blend"], grads["pos"], g_pos=rig["g_bind"], g_weights=rig["g_w"])
        if lap is not None:
            ring, base_pos, lams, g_lap = lap
            adr.laplacian(ctx, ring, base_pos, None, lams[t % n_steps], g_pos=g_lap)
        lr = w.lr * 10.0 ** (-0.0002 * t)
        adr.adam_step(ctx, adam, t + 1, lr)
        if maps:
            adr.adam_step_maps(ctx, maps, t + 1, lr)

    state = dict(ref_mesh=ref_mesh, lat_mesh=lat_mesh, lat_mat=lat_mat, lat_out=lat_out,
                 ref_out=ref_out, n_params=n_params, n_map_params=n_map_params,
                 map_adam_bytes=map_adam_bytes, raster_split={"ref": list(split_ref), "latent": list(split_lat)},
                 views=views, adam=adam,
                 skin=None if rig is None else tuple(rig["w"].shape))
    return step, state


TEXEL_C = 1.25   # compulsory texels per covered pixel per mip level at ~1 texel per pixel


def lookup_bytes(scene):
    """Compulsory texel bytes of one pixel's trilinear lookups of every map
    of a scene larger than 1x1: TEXEL_C texels at each of two levels."""
    total = 0.0
    for name in ("kd", "normal", "orm", "alpha"):
        tex = getattr(scene, name, None)
        if tex is None or tex.data.shape[0] <= 1:
            continue
        bt = 4 if getattr(tex, "fmt", "f32") == "rgba8" else 4 * tex.data.shape[2]
        total += 2 * TEXEL_C * bt
    return total


def optimised_maps(w):
    """(name, bytes per texel) of the optimised F32 maps larger than 1x1."""
    out = []
    for name in ("kd", "normal", "orm", "alpha"):
        tex = getattr(w.latent, name, None)
        if name in w.optimize and tex is not None and tex.data.shape[0] > 1:
            out.append((name, 4 * tex.data.shape[2]))
    return out


def algorithmic_bytes(stage, w, st, covered_latent, covered_ref=0):
    """Compulsory HBM bytes of one launch of a stage's kernel.

    shade (k_shade_fwd, one launch per render, averaged over the reference
    and latent renders of a step): per visibility sample its key (8 B) and
    colour (12 B); per covered pixel the texels of its trilinear lookups
    (TEXEL_C per level, two levels, every map of that render's material).
    aa_loss (k_aa_fwd, averaged over the two renders): per pixel key and
    colour (20 B); the reference writes its image (12 B); the latent reads
    the reference image (12 B) and writes dL/dimage (12 B) and the received
    antialiasing it keeps for the adjoint (24 B).
    aa_bwd (k_aa_bwd): per pixel key, colour, dL/dimage, the kept
    antialiasing (8 + 12 + 12 + 24 B) and dL/dcolour written (12 B).
    shade_bwd (pixel adjoint): per pixel its visibility key (8 B) and the
    record header it writes (16 B); per covered pixel dL/dcolour (12 B), a
    16-B sample record per optimised map and the texels of its trilinear
    lookups (TEXEL_C per level, two levels, every latent map).
    tex_bwd (texel scatter): the records back (16 B per pixel, 16 B per
    covered pixel and map) and, per covered pixel and map, TEXEL_C texels at
    each of the two trilinear levels, each a read-modify-write of its
    gradient (2 x B_t)."""
    B, H, W = w.dirs.shape[0], w.height, w.width
    px = B * H * W
    maps = optimised_maps(w)
    if stage == "adam":
        return 32.0 * (st["n_params"] - st.get("n_map_params", 0))   # read p,g,m,v; write p,m,v,g
    if stage == "adam_maps":
        return float(st["map_adam_bytes"]) if st.get("map_adam_bytes") else None
    L = w.oit_layers
    if L:
        # depth-peeled latent: one launch per layer; covered_latent counts the
        # covered pixels of all layers; the average launch is returned
        if stage == "shade_bwd":
            return (L * px * (8 + 16 + 4) + covered_latent * (12 + 16 * len(maps) + lookup_bytes(w.latent))) / L
        if stage == "tex_bwd":
            return (L * px * 16 + covered_latent * sum(16 + 2 * TEXEL_C * 2 * bt for _, bt in maps)) / L
        if stage == "aa_bwd":
            return px * (8 + 12 + 12 + 24 + 12)
        return None
    if stage == "shade_bwd":
        return px * (8 + 16) + covered_latent * (12 + 16 * len(maps) + lookup_bytes(w.latent))
    if stage == "tex_bwd":
        return px * 16 + covered_latent * sum(16 + 2 * TEXEL_C * 2 * bt for _, bt in maps)
    if stage == "aa_bwd":
        return px * (8 + 12 + 12 + 24 + 12)
    if stage == "aa_loss":
        if w.msaa > 1 or w.ref_ssaa > 1:
            return None                                   # the resolve or downsample is a second kernel
        return (px * (20 + 12) + px * (20 + 12 + 12 + 24)) / 2.0
    if stage == "shade":
        ref = px * w.ref_ssaa ** 2 * (8 + 12) + covered_ref * lookup_bytes(w.ref)
        lat = px * w.msaa ** 2 * (8 + 12) + covered_latent * lookup_bytes(w.latent)
        return (ref + lat) / 2.0
    if stage == "skin_bwd" and st.get("skin"):
        V, nb = st["skin"]
        # per vertex: dL/dskinned read + cleared, bind position, blended
        # matrix, dL/dweights and dL/dpos read-modify-write; the bones once
        return V * (12 + 12 + 12 + 48 + 8 * nb + 24) + 48 * nb
    return None


TRI_VIEW_BYTES = 100   # per triangle and view: transform, set-up and bin entry (the scope's model)


def step_model_bytes(w, st, covered_latent, covered_ref, launches):
    """Algorithmic bytes of one step: every stage with a byte model, times
    its launches per step, plus the triangle set-up of both renders."""
    total = 0.0
    for stage, n in launches.items():
        by = algorithmic_bytes(stage, w, st, covered_latent, covered_ref)
        if by:
            total += by * n
    B = w.dirs.shape[0]
    total += TRI_VIEW_BYTES * B * (int(w.ref.mesh.tri.shape[0]) + int(st["lat_mesh"].tri.shape[0]))
    return total


VALU_PEAK = 256 * 4 * 2.4e9 / 4 / 1e9   # wave64 VALU instructions per second: 16-lane SIMDs, 4 cycles each


def pmc_valu(workload, stage):
    """VALU instructions per launch of a stage's kernel from the committed
    counter summary (SQ_INSTS_VALU x SQ_WAVES), or None if absent or stale."""
    path = os.path.join(ROOT, "profiles", f"pmc_valu_{workload}.json")
    if stage not in SINGLE_KERNEL_STAGES or not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    k = d.get("kernels", {}).get(SINGLE_KERNEL_STAGES[stage][0])
    if not k or k.get("sources_sha256") != kernel_sources_sha(SINGLE_KERNEL_STAGES[stage][1]):
        return None
    return k["valu_per_launch"]


def stage_rooflines(w, st, covered, covered_ref, stages, workload):
    """HBM (and, where VALU counters are committed, VALU-issue) fraction of
    every single-kernel stage from the profiled pass."""
    out = {}
    for stage, (ms, cnt) in stages.items():
        if stage not in SINGLE_KERNEL_STAGES or not cnt:
            continue
        avg_ms = ms / cnt
        rec = {"kernel": SINGLE_KERNEL_STAGES[stage][0], "avg_launch_ms": round(avg_ms, 4)}
        by = algorithmic_bytes(stage, w, st, covered, covered_ref)
        if by:
            ach = by / (avg_ms * 1e-3) / 1e9
            rec["hbm"] = {"achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": round(by)}
        # (with multisampling the antialiasing stage also holds the resolve)
        valu = pmc_valu(workload, stage) if not (stage == "aa_loss" and w.msaa > 1) else None
        if valu:
            ach = valu / (avg_ms * 1e-3) / 1e9
            rec["valu"] = {"achieved": round(ach, 1), "peak": VALU_PEAK, "unit": "G wave-instr/s",
                           "frac": round(ach / VALU_PEAK, 4), "instr_per_launch": round(valu)}
        out[stage] = rec
    return out


def cpu_baseline(w, np, torch, views, min_seconds=10.0, max_steps=4):
    """The FP64 oracle on whole steps of the workload (``views`` of its
    views, full meshes and maps), repeated until about min_seconds."""
    from oracle import loop as OL
    from paper_2104_03989_amd import synth
    w1 = synth.scaled(w, views=views)
    t0 = time.perf_counter()
    steps = 0
    state = {}
    params = OL.latent_params(w1)
    while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < min_seconds):
        mvp32, eye = OL.cameras(w1)
        ref = OL.reference_image(w1, mvp32, eye)
        loss, grads, _ = OL.loss_and_grads(w1, ref, mvp32, eye, params)
        new, state = OL.adam_update(params, grads, state, steps + 1, w1.lr)
        params = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in new.items()}
        steps += 1
    dt = time.perf_counter() - t0
    B = w.dirs.shape[0]
    return dict(value=round(steps * views * w1.width * w1.height / dt / 1e6, 4), unit="Mpix/s",
                cores=torch.get_num_threads(), kind="oracle", host=host_cpu(),
                sample=f"{steps} full steps ({views} of the {B} views each, full-size meshes and maps): "
                       "reference render, latent render, loss, backward, Adam", seconds=round(dt, 2))


def host_cpu():
    """nproc and the CPU model line of lscpu (the oracle's host)."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Thread(s) per core", "Core(s) per socket", "Socket(s)"):
                info[k.strip()] = v.strip()
    except OSError:
        pass
    return info


def oracle_step_seconds(w, np, torch, steps):
    """Seconds per whole oracle step (reference render, latent render, loss,
    backward, Adam) of a workload, one value per step."""
    from oracle import loop as OL
    params = OL.latent_params(w)
    state, out = {}, []
    for t in range(steps):
        t0 = time.perf_counter()
        mvp32, eye = OL.cameras(w)
        ref = OL.reference_image(w, mvp32, eye)
        loss, grads, _ = OL.loss_and_grads(w, ref, mvp32, eye, params)
        new, state = OL.adam_update(params, grads, state, t + 1, w.lr)
        params = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in new.items()}
        out.append(time.perf_counter() - t0)
        _log(f"  oracle step {t + 1}/{steps}: {out[-1]:.2f} s")
    return out


def oracle_timing(args):
    """The FP64 oracle's per-step time on this host: the plain step as a
    median of 5, the paper-scale and displacement loops over 3 steps, one
    mesh-step of the batched and of the served mixes, each at one thread and
    at every core; writes profiles/oracle_timing.md."""
    import numpy as np
    import torch

    from paper_2104_03989_amd import synth
    host = host_cpu()
    n_all = host["nproc"]
    disp = synth.workload_displacement()
    disp.disp = synth.Texture(np.random.default_rng(12).normal(0.0, 0.01, size=(1024, 1024, 1)).astype(np.float32), "f32")
    batched = synth.workload_batched(n_meshes=1)[0]
    served = serve_pool(1, np.random.Generator(np.random.PCG64(synth.seed_for(5, 0))))[0]
    cases = [("plain step (4 x 256^2, 1,280 / 20,480 tris)", synth.workload_plain_step(), 5, "median"),
             ("paper-scale loop (8 x 512^2, 7,220 / 297,680 tris, 2048^2 maps)", synth.workload_paper_loop(), 3, "mean"),
             ("displacement loop (8 x 512^2, 62,720 / 369,920 tris)", disp, 3, "mean"),
             ("batched: one mesh-step (mesh 0 of the 64)", batched, 1, "mean"),
             ("served: one job-step (job 0 of the pool)", served, 1, "mean")]
    lines = ["# FP64 oracle timing on the host (a baseline, not a target)", "",
             "Command: `python3 bench.py --oracle-timing` on the GPU box's host.  Host: " +
             ", ".join(f"{k} {v}" for k, v in host.items()) + ".", "",
             "A step is the whole oracle step: reference render, latent render, image loss, backward (autograd of "
             "the float64 forward) and Adam.  The integer rasterizer is single-threaded C; the float64 stages use "
             "torch's CPU threads.", "",
             "| workload | threads | steps | s per step | Mpix/s |", "|---|---|---|---|---|"]
    print("\n".join(lines), flush=True)
    for name, w, steps, how in cases:
        px = w.dirs.shape[0] * w.width * w.height
        for threads in (1, n_all):
            torch.set_num_threads(threads)
            _log(f"oracle timing: {name}, {threads} thread(s)")
            ts = oracle_step_seconds(w, np, torch, steps)
            sec = float(np.median(ts)) if how == "median" else float(np.mean(ts))
            lines.append(f"| {name} | {torch.get_num_threads()} | {steps} ({how}) | {sec:.3f} | {px / sec / 1e6:.4f} |")
            print(lines[-1], flush=True)
    path = args.oracle_timing_out or os.path.join(ROOT, "profiles", "oracle_timing.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(path)


def serve_pool(n, g):
    """Workloads of the served mix: reference 20k-735k and target 1k-20k
    triangles (log-uniform), 1024^2 maps, 8 views of 512x512."""
    from paper_2104_03989_amd import synth

    def nu_for(tris):
        return max(2, int(round(math.sqrt(tris / 20.0))))
    pool = []
    for _ in range(n):
        rt = math.exp(g.uniform(math.log(20e3), math.log(735e3)))
        lt = math.exp(g.uniform(math.log(1e3), math.log(20e3)))
        pool.append(synth.workload_paper_loop(views=8, res=512, map_size=1024, ref_nu=nu_for(rt),
                                              lat_nu=nu_for(lt)))
    return pool


def serve(args):
    """Served mode: jobs shaped like the served workload arrive as a Poisson
    stream; the job server admits them by HBM budget and interleaves their
    steps.  Reports jobs/hr, steps/s and per-step p50/p99 latency, and the
    steps/s of the same jobs run one at a time."""
    import numpy as np
    from paper_2104_03989_amd import adr, synth

    g = np.random.Generator(np.random.PCG64(synth.seed_for(5, 0)))
    pool = serve_pool(args.serve_pool, g)
    n_jobs = args.serve_jobs
    arrivals = np.cumsum(g.exponential(1.0 / args.serve_rate, size=n_jobs))
    ctx = adr.Context(0)
    # one job alone first (warm-up, and the one-at-a-time reference)
    t0 = time.perf_counter()
    jid = adr.job_submit(ctx, pool[0], n_steps=args.serve_steps, seed=1)
    while True:
        st, _ = adr.job_poll(ctx, jid)
        if st["state"] == adr.JOB_DONE:
            break
        if st["code"] < 0:
            raise RuntimeError(st.get("error"))
        time.sleep(0.002)
    adr.job_poll(ctx, jid, pool[0])
    alone_steps_s = args.serve_steps / (time.perf_counter() - t0)
    _log(f"one job alone: {alone_steps_s:.1f} steps/s")
    t0 = time.perf_counter()
    submitted, done, lat = {}, {}, []
    k = 0
    while len(done) < n_jobs:
        now = time.perf_counter() - t0
        while k < n_jobs and arrivals[k] <= now:
            w = pool[k % len(pool)]
            submitted[adr.job_submit(ctx, w, n_steps=args.serve_steps, seed=1000 + k)] = w
            k += 1
        for jid, w in list(submitted.items()):
            if jid in done:
                continue
            st, res = adr.job_poll(ctx, jid, w)
            if st["code"] < 0:
                _log(f"job {jid} failed: {st.get('error')}")
                done[jid] = st
            elif st["state"] == adr.JOB_DONE:
                done[jid] = st
        time.sleep(0.002)
    wall = time.perf_counter() - t0
    steps = sum(s["step"] for s in done.values())
    p50 = float(np.median([s["p50_ms"] for s in done.values()]))
    p99 = float(np.max([s["p99_ms"] for s in done.values()]))
    rec = {"metric": "served jobs/hr with p50/p99 step ms", "value": round(n_jobs / wall * 3600, 1),
           "unit": "jobs/hr", "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "steps_per_s": round(steps / wall, 1), "one_at_a_time_steps_per_s": round(alone_steps_s, 1),
           "p50_step_ms": round(p50, 3), "p99_step_ms": round(p99, 3), "wall_s": round(wall, 2),
           "config": {"workload": "served: Poisson arrivals, reference 20k-735k tris, target 1k-20k tris, "
                                  "1024^2 maps, 8 views x 512x512, GGX, tone-mapped L1",
                      "rate_per_s": args.serve_rate, "jobs": n_jobs, "steps_per_job": args.serve_steps,
                      "mesh_pool": len(pool)}}
    print(json.dumps(rec), flush=True)
    ctx.close()


WORKLOADS = {
    "paper": ("paper-scale loop: 297,680-tri GGX reference, 7,220-tri latent, 2048^2 maps, "
              "8 views x 512x512, tone-mapped L1, Adam"),
    "displacement": ("displacement loop: 369,920-tri reference, 980-tri base tessellated to 62,720 tris "
                     "and displaced by a 1024^2 map, 1024^2 normal map, 8 views x 512x512, L1, Adam"),
    "plain": ("plain single step: 20,480-tri SH reference, 1,280-tri latent, 256^2 maps, 4 views x 256x256, "
              "Blinn-Phong, L1, Adam"),
    "animation": ("animation: 19,220-tri GGX reference skinned to a 32-bone rig (40 frames, one per step), "
                  "5,120-tri latent with dense 32-bone weights, bind pose and 1024^2 maps optimised, "
                  "8 views x 512x512, tone-mapped L1, Adam"),
    "batched": ("batched: 64 meshes, latent 1k-50k tris (log-uniform), reference at 4x the sphere frequency "
                "(at most 737k tris), 4-16 views at 256^2-1024^2, 512^2-2048^2 FP32 normal and ORM maps, GGX, L1, "
                "one launch per render stage over all meshes, graph-captured, with one Adam launch, against the "
                "same meshes one at a time"),
    "aggregate": ("aggregate geometry: 1.2M-tri leaf cloud reference, 4,800 transparent quads (9,600 tris) "
                  "with 8 depth-peeled layers, 2048^2 base colour, normal and alpha maps optimised with positions, "
                  "8 views x 512x512, L2, Adam"),
    "prefilter": ("prefiltering: 297,680-tri GGX reference with 8x8 supersampling, 7,220-tri latent with 4x4 "
                  "multisampled visibility and independent-mip 512^2 maps, 8 views x 128x128, tone-mapped L1, Adam"),
}


def make_workload(name):
    from paper_2104_03989_amd import synth
    if name == "paper":
        return synth.workload_paper_loop(), 2
    if name == "displacement":
        return synth.workload_displacement(), 3
    if name == "prefilter":
        return synth.workload_prefilter(), 6
    if name == "animation":
        return synth.workload_animation(), 7
    if name == "aggregate":
        return synth.workload_aggregate(), 8
    return synth.workload_plain_step(), 1


def batched(args):
    """Batched form: 64 uneven meshes stepped one at a time (plain) and as a
    graph-captured batch (--batch-form launch: one launch per render stage
    over all meshes; streams: every mesh's launches over 4 streams) with one
    Adam launch, from the same state; reports mesh-steps/s of both and their
    losses."""
    import numpy as np
    import torch

    from paper_2104_03989_amd import synth
    from paper_2104_03989_amd.batch import Batch

    torch.cuda.set_device(0)
    _log("generating 64 meshes")
    ws = synth.workload_batched(progress=lambda k, w: _log(f"  mesh {k}: {w.latent.mesh.tri.shape[0]} / "
                                                            f"{w.ref.mesh.tri.shape[0]} tris, {w.dirs.shape[0]} x "
                                                            f"{w.width}^2"))
    W, K = args.warmup, args.steps
    n_steps = W + K + 1
    _log("uploading and tuning")
    b = Batch(ws, n_steps, n_streams=4, det=args.deterministic, tune=True, progress=lambda k: None,
              form=args.batch_form)
    px = sum(w.dirs.shape[0] * w.width * w.height for w in ws)
    # both forms run steps 0 .. W+K-1 from the same state (the optimised
    # parameters, maps and Adam moments restored in between), so their last
    # losses are comparable
    snap = b.snapshot()
    t = 0
    _log("plain warm-up")
    for _ in range(W):
        b.step_plain(t)
        t += 1
    torch.cuda.synchronize()
    _log(f"plain: timing {K} steps")
    t0 = time.perf_counter()
    for _ in range(K):
        b.step_plain(t)
        t += 1
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    loss_plain = float(np.mean(b.losses()))
    _log("batched: warm-up and capture")
    b.restore(snap)
    del snap
    t = 0
    b.step_eager(t)
    t += 1
    b.capture()
    for _ in range(W - 1):
        b.step(t)
        t += 1
    torch.cuda.synchronize()
    _log(f"batched: timing {K} steps")
    t0 = time.perf_counter()
    for _ in range(K):
        b.step(t)
        t += 1
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    loss_b = float(np.mean(b.losses()))
    n = len(ws)
    rec = {
        "metric": "optimizer steps/s (mesh-steps, batched form) with fwd+bwd Mpix/s",
        "value": round(n * K / dt_b, 2), "unit": "mesh-steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(dt_b / K * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "mpix_per_s": round(px * K / dt_b / 1e6, 1),
        "plain": {"mesh_steps_per_s": round(n * K / dt_plain, 2), "ms_per_step": round(dt_plain / K * 1e3, 3),
                  "mpix_per_s": round(px * K / dt_plain / 1e6, 1), "mean_loss_last_step": round(loss_plain, 6)},
        "speedup_vs_plain": round(dt_plain / dt_b, 3),
        "config": {"workload": WORKLOADS["batched"], "meshes": n, "latent_tris": int(sum(w.latent.mesh.tri.shape[0] for w in ws)),
                   "ref_tris": int(sum(w.ref.mesh.tri.shape[0] for w in ws)), "pixels_per_step": px,
                   "gradient_mode": "deterministic" if args.deterministic else "atomic",
                   "form": args.batch_form, "streams": 1 if args.batch_form == "launch" else 4,
                   "batch_scratch_gib": round(b.scratch_bytes() / 2**30, 2), "mean_loss_last_step": round(loss_b, 6),
                   "raster_splits": sorted({str(m.split_ref) + "/" + str(m.split_lat) for m in b.meshes})},
    }
    print(json.dumps(rec), flush=True)
    b.close()


def calibrate_copy(np, torch, nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling HBM byte counters."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                      "launches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="paper")
    ap.add_argument("--cpu-views", type=int, default=8, help="views of the oracle's timed step")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device copy three times (HBM counter scale) and exit")
    ap.add_argument("--deterministic", action="store_true",
                    help="bit-reproducible gradients (fixed-point vertex sums, sorted texel sums)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write profiles/pmc_traffic_<workload>.json from rocprofv3 --pmc output and exit")
    ap.add_argument("--pmc-valu-summary", metavar="PMC_DIR",
                    help="write profiles/pmc_valu_<workload>.json from a rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU run "
                         "and exit")
    ap.add_argument("--laplacian", action="store_true",
                    help="add the uniform Laplacian regularizer with the heuristic lambda_0 and its schedule")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without stage events")
    ap.add_argument("--no-tune", action="store_true", help="default raster work split instead of the autotuner's")
    ap.add_argument("--overlap", action="store_true",
                    help="render each step's reference on a stream of its own, overlapping the previous step's "
                         "backward and Adam (kernel times then include the concurrent work)")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="time the FP64 oracle per step on this host (1 thread and all cores) and write "
                         "profiles/oracle_timing.md")
    ap.add_argument("--oracle-timing-out", metavar="PATH", help="where --oracle-timing writes its table")
    ap.add_argument("--batch-form", choices=("launch", "streams"), default="launch",
                    help="batched workload: one launch per render stage over all meshes (launch) or every mesh's "
                         "launches over 4 streams (streams), both graph-captured")
    ap.add_argument("--serve", action="store_true", help="served mode (job server, Poisson arrivals)")
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-jobs", type=int, default=16)
    ap.add_argument("--serve-steps", type=int, default=200)
    ap.add_argument("--serve-pool", type=int, default=4)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.serve:
        serve(args)
        return
    if args.oracle_timing:
        oracle_timing(args)
        return
    if args.pmc_summary:
        summarize_pmc(args.workload, *args.pmc_summary)
        return
    if args.pmc_valu_summary:
        summarize_valu(args.workload, args.pmc_valu_summary)
        return
    if args.workload == "batched":
        batched(args)
        return

    import numpy as np
    import torch

    from paper_2104_03989_amd import adr, synth

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy(np, torch)
        return
    _log("generating workload")
    w, cfg = make_workload(args.workload)
    B, H, W = w.dirs.shape[0], w.height, w.width
    ctx = adr.Context(0)
    ctx_ref = adr.Context(0) if args.overlap else None
    ctxs = [c for c in (ctx, ctx_ref) if c is not None]
    n_steps = args.warmup + args.steps
    step, st = build_step(w, ctx, adr, torch, np, n_steps, seed=synth.seed_for(cfg, 100), det=args.deterministic,
                          laplacian=args.laplacian, tune=not args.no_tune, ctx_ref=ctx_ref)
    torch.cuda.synchronize()
    if w.oit_layers:
        covered = int(((st["lat_out"]["vis"] & 0xFFFFFFFF) != 0).sum())
    else:
        covered = int((st["lat_out"]["tri_id"] > 0).sum()) // (w.msaa * w.msaa)
        st["lat_out"]["tri_id"] = None     # read for the count above only: the steps do not write it
    covered_ref = int(((st["ref_out"]["vis"] & 0xFFFFFFFF) != 0).sum())
    _log(f"warmup {args.warmup}")
    for t in range(args.warmup):
        step(t)
    torch.cuda.synchronize()
    # Stage breakdown: a profiled pass outside the timed region (every stage
    # bracketed by events, which stall the stream a few microseconds each).
    # In the timed region only the dominant single-kernel stage is bracketed,
    # for its roofline.
    stages, dom, n_prof = {}, None, 0
    def read_stages():
        # both contexts' spans, per stage (summed milliseconds, launches)
        out = {}
        for c in ctxs:
            for k_, (ms_, cnt_) in c.profile_read().items():
                a_, b_ = out.get(k_, (0.0, 0))
                out[k_] = (a_ + ms_, b_ + cnt_)
        return out

    if not args.no_profile:
        for c in ctxs:
            c.profile(True)
        read_stages()
        n_prof = max(3, min(10, args.warmup))
        _log(f"profiled pass {n_prof}")
        for t in range(n_prof):
            step(t)
        stages = read_stages()
        cands = {k: v[0] for k, v in stages.items()
                 if v[1] > 0 and k in SINGLE_KERNEL_STAGES and algorithmic_bytes(k, w, st, covered, covered_ref) is not None}
        dom = max(cands, key=cands.get)
        for c in ctxs:
            c.profile_stages([dom])
        read_stages()
    _log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.warmup, n_steps):
        step(t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timed = read_stages() if dom else {}
    for c in ctxs:
        c.profile(False)
    loss = float(st["lat_out"]["loss"][0])
    ms_step = dt / args.steps * 1e3
    mpix = B * H * W * args.steps / dt / 1e6
    # the same steps without the reference render (latent forward, backward
    # and Adam only, against the last reference images)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for t in range(args.warmup, n_steps):
        step(t, with_reference=False)
    torch.cuda.synchronize()
    dt_lat = time.perf_counter() - t1
    # a device copy of 1 GiB: the measured HBM ceiling beside the nominal one
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    copy_gbs = 2.0 * (1 << 30) * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    roof = None
    prof, stage_step = {}, {}
    if stages:
        prof = {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1] > 0}
        stage_step = {k: round(v[0] / n_prof, 4) for k, v in stages.items() if v[1] > 0}
    if dom:
        ms, cnt = timed[dom]
        avg_ms = ms / cnt
        by = algorithmic_bytes(dom, w, st, covered, covered_ref)
        ach = by / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": SINGLE_KERNEL_STAGES[dom][0], "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": pmc_traffic(args.workload, dom), "avg_launch_ms": round(avg_ms, 4),
                "launches": cnt, "bytes_per_launch": by,
                "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(ach / copy_gbs, 4)}
    # achieved GB/s of every stage with an algorithmic byte count (profiled pass)
    stage_gbs = {}
    for k, (ms_k, cnt_k) in stages.items():
        by_k = algorithmic_bytes(k, w, st, covered, covered_ref) if cnt_k else None
        if by_k:
            stage_gbs[k] = round(by_k / (ms_k / cnt_k * 1e-3) / 1e9, 1)
    # every single-kernel stage against its roofline(s), and the whole step
    # against the HBM ceiling of its algorithmic bytes
    roofs = stage_rooflines(w, st, covered, covered_ref, stages, args.workload) if stages else {}
    step_roof = None
    if stages:
        launches = {k: v[1] / n_prof for k, v in stages.items() if v[1] > 0}
        sb = step_model_bytes(w, st, covered, covered_ref, launches)
        ach = sb / (ms_step * 1e-3) / 1e9
        step_roof = {"bytes_per_step": round(sb), "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "ceiling_ms": round(sb / (HBM_PEAK_GBS * 1e9) * 1e3, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        _log("oracle baseline")
        cpu = cpu_baseline(w, np, torch, min(args.cpu_views, B))
    rec = {
        "metric": "fwd+bwd Mpix/s (latent pixels per second, reference render and Adam included)",
        "value": round(mpix, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "mpix_per_s_without_reference": round(B * H * W * args.steps / dt_lat / 1e6, 2),
        "ms_per_step_without_reference": round(dt_lat / args.steps * 1e3, 3),
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "steps_per_s": round(1e3 / ms_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "views": B, "res": [W, H], "ref_tris": int(w.ref.mesh.tri.shape[0]),
                   "latent_tris": int(st["lat_mesh"].tri.shape[0]), "params": st["n_params"],
                   "gradient_mode": "deterministic" if args.deterministic else "atomic",
                   "laplacian": bool(args.laplacian), "raster_split": st["raster_split"],
                   "reference_stream": "overlapped" if ctx_ref is not None else "same",
                   "final_loss": round(loss, 6)},
        "roofline": roof, "cpu_baseline": cpu, "roofline_stages": roofs, "step_roofline": step_roof,
        "stage_avg_ms": prof, "stage_ms_per_step": stage_step, "stage_gbs": stage_gbs,
        "stage_pass_steps": n_prof if stages else 0,
    }
    print(json.dumps(rec), flush=True)
    for c in ctxs:
        c.close()


if __name__ == "__main__":
    main()
