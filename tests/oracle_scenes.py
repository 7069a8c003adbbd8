"""Small hand-built scenes for the oracle pins (input layout only)."""
import numpy as np

from paper_2104_03989_amd import synth


def const_tex(value, size=4):
    v = np.asarray(value, dtype=np.float32)
    return synth.Texture(np.tile(v, (size, size, 1)), "f32")


def flat_normals(size=4):
    return synth.Texture(synth.flat_normal_map(size).astype(np.float32), "f32")


def quad_mesh(z=0.0, half=1.0):
    pos = np.array([(-half, -half, z), (half, -half, z), (-half, half, z), (half, half, z)],
                   dtype=np.float32)
    tri = np.array([(0, 1, 3), (0, 3, 2)], dtype=np.int32)
    uv = ((pos[:, :2] / half + 1.0) / 2.0).astype(np.float32)
    return synth.Mesh(pos, tri, uv, tri.copy())


def workload(ref, latent, dirs, light, W, H, loss="l1", optimize=("pos",), light_rgb=None):
    dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    B = dirs.shape[0]
    light = np.asarray(light, dtype=np.float64).reshape(-1, 3)
    light = light / np.linalg.norm(light, axis=1, keepdims=True)
    if light.shape[0] == 1:
        light = np.repeat(light, B, axis=0)
    rgb = np.ones((B, 3)) if light_rgb is None else np.asarray(light_rgb, dtype=np.float64)
    return synth.Workload("test", ref, latent, dirs, light, rgb, W, H, 3.0, 45.0, loss, 1e-3,
                          tuple(optimize))


def tiny_sphere_workload(model="blinn_phong", nu=2, res=24, views=1, tex=8, loss="l1",
                         seed=0):
    g = np.random.default_rng(seed)
    ref_mesh = synth.sphere_mesh(nu + 1, lambda d: synth.sh_radius(d, 100 + seed, lmax=3, sigma=0.08))
    lat_mesh = synth.sphere_mesh(nu, lambda d: synth.sh_radius(d, 200 + seed, lmax=3, sigma=0.05))
    def tex3(lo, hi):
        return synth.Texture(g.uniform(lo, hi, size=(tex, tex, 3)).astype(np.float32), "f32")
    def nmap(tilt):
        return synth.Texture(synth.detail_normal_map(tex, 300 + seed, tilt).astype(np.float32), "f32")
    orm_ref = orm_lat = None
    if model == "ggx":
        orm_ref = synth.Texture(synth.orm_map(tex, 400 + seed).astype(np.float32), "f32")
        o = synth.orm_map(tex, 500 + seed)
        o[..., 0] = g.uniform(0.0, 0.3, size=(tex, tex))
        orm_lat = synth.Texture(o.astype(np.float32), "f32")
    ref = synth.Scene(ref_mesh, model, tex3(0.1, 0.9), nmap(0.2), orm_ref)
    lat = synth.Scene(lat_mesh, model, tex3(0.1, 0.9), nmap(0.1), orm_lat)
    dirs = synth.random_unit(views, 600 + seed)
    light = synth.random_unit(views, 700 + seed)
    # light roughly from the camera side so that most pixels are lit
    light = light + 1.5 * dirs
    opt = ("pos", "kd", "normal", "orm") if model == "ggx" else ("pos", "kd", "normal")
    return workload(ref, lat, dirs, light, res, res, loss=loss, optimize=opt)


def tess_crop_workload(res=32, views=2, disp_size=16, seed=0, levels=3):
    """The 64-triangle crop of the displacement loop: one base triangle
    (tessellated `levels` times) displaced by a random map, against a tilted
    textured reference triangle."""
    g = np.random.default_rng(seed)
    pos = np.array([[-0.9, -0.8, 0.0], [1.0, -0.6, 0.1], [-0.3, 0.9, -0.05]], np.float32)
    tri = np.array([[0, 1, 2]], np.int32)
    uv = np.array([[0.1, 0.1], [0.9, 0.2], [0.3, 0.85]], np.float32)
    base = synth.Mesh(pos, tri, uv, tri.copy())
    ref_pos = pos * np.float32(0.95) + np.array([0.03, -0.02, 0.1], np.float32)
    ref_mesh = synth.Mesh(ref_pos.astype(np.float32), tri, uv, tri.copy())
    kd_ref = synth.Texture(g.uniform(0.2, 0.9, size=(8, 8, 3)).astype(np.float32), "f32")
    ref = synth.Scene(ref_mesh, "blinn_phong", kd_ref, flat_normals(), None)
    nm = synth.Texture(synth.detail_normal_map(disp_size, 900 + seed, 0.1).astype(np.float32), "f32")
    lat = synth.Scene(base, "blinn_phong", const_tex((0.6, 0.5, 0.4)), nm, None)
    disp = synth.Texture(g.normal(0.0, 0.04, size=(disp_size, disp_size, 1)).astype(np.float32), "f32")
    dirs = np.array([[0.1, 0.15, 1.0], [-0.25, 0.1, 1.0], [0.2, -0.3, 1.0]])[:views]
    light = np.array([[0.3, 0.4, 1.0]])
    w = workload(ref, lat, dirs, light, res, res, loss="l1", optimize=("pos", "disp", "normal"))
    w.disp = disp
    w.tess_levels = levels
    return w


def rig_workload(w, n_bones=6, n_frames=4, frame=1, seed=0, identity=False):
    """Attach a small synthetic rig to a workload: reference weights from the
    rig's falloff, latent weights random and normalised per vertex.  With
    ``identity`` every bone transform is the identity."""
    rig = synth.synthetic_rig(w.ref.mesh.pos, n_bones, n_frames, 800 + seed, chains=2, reach=0.6)
    g = np.random.default_rng(900 + seed)
    n_lat = w.latent.mesh.pos.shape[0]
    if identity:
        # identity bones, and weights that sum to one exactly: multiples of
        # 1/64 for the latent, one-hot rows for the reference
        rig.bones[:] = np.eye(3, 4, dtype=np.float32)
        rig.ref_weights[:] = 0.0
        rig.ref_weights[np.arange(rig.ref_weights.shape[0]), g.integers(0, n_bones, rig.ref_weights.shape[0])] = 1.0
        cuts = np.sort(g.integers(0, 65, size=(n_lat, n_bones - 1)), axis=1)
        parts = np.diff(np.concatenate([np.zeros((n_lat, 1)), cuts, np.full((n_lat, 1), 64)], 1), axis=1)
        w.weights = (parts / 64.0).astype(np.float32)
    else:
        wt = g.uniform(0.0, 1.0, size=(n_lat, n_bones))
        w.weights = (wt / wt.sum(1, keepdims=True)).astype(np.float32)
    w.rig = rig
    w.frame = frame
    w.optimize = tuple(w.optimize) + ("weights",)
    return w


def aggregate_case(res=24, views=1, n_leaves=60, n_quads=6, tex=8, layers=4, seed=0):
    """A small aggregate scene: leaves against textured, transparent quads."""
    g = np.random.default_rng(seed)
    leaves = synth.leaf_cloud(n_leaves, 1000 + seed, radius=0.6, size=0.15)
    kd_ref = synth.Texture(g.uniform(0.1, 0.9, size=(tex, tex, 3)).astype(np.float32), "f32")
    ref = synth.Scene(leaves, "blinn_phong", kd_ref, flat_normals(), None)
    quads = synth.quad_cloud(n_quads, 2000 + seed, radius=0.4, size=0.6)
    lat = synth.Scene(quads, "blinn_phong", synth.Texture(g.uniform(0.2, 0.8, (tex, tex, 3)).astype(np.float32), "f32"),
                      synth.Texture(synth.detail_normal_map(tex, 3000 + seed, 0.1).astype(np.float32), "f32"), None,
                      synth.Texture(g.uniform(0.2, 0.8, (tex, tex, 1)).astype(np.float32), "f32"))
    dirs = synth.random_unit(views, 4000 + seed) + np.array([0.0, 0.0, 1.5])
    light = synth.random_unit(views, 5000 + seed) + 1.5 * dirs
    w = workload(ref, lat, dirs, light, res, res, loss="l2", optimize=("pos", "kd", "normal", "alpha"))
    w.oit_layers = layers
    return w
