"""Seeded synthetic inputs for the pyramid Gaussian-splatting rasterizer.

This module only draws random numbers and lays them out; it holds none of the
rendering, loss or gradient arithmetic, so that the CPU oracle (tests) and the
HIP library (package, benchmark) can both be fed from it without sharing any of
the method's code.

Scenes stand in for the RGB-D sequences the paper evaluates on (Replica and
ScanNet, Sec. IV-A), which are not available here: a room-shaped box with
furniture boxes inside, seen by pinhole cameras of the same frame shapes
(1200x680 and 640x480) and with the pyramid depth the paper uses (3 levels,
Sec. IV-A "Parameters").

Parameter conventions (the primitive of Sec. III-B, generalised to per-axis
scales and a rotation):
  mean       [N,3]  float32, world metres, z up
  log_scale  [N,3]  float32, natural log of the per-axis standard deviation
  quat       [N,4]  float32, (w, x, y, z), normalised at generation time
  opacity    [N]    float32, logit (the rasterizer applies a sigmoid)
  rgb        [N,3]  float32, raw colour feature (no activation)
  sem        [N,C]  float32, raw per-class logits   (plain semantic mode)
  emb        [N,16] uint16, bfloat16 bit patterns   (learned semantic mode)
Views: R [3,3], t [3] float32 with x_cam = R @ x_world + t (OpenCV axes:
x right, y down, z forward), base intrinsics fx, fy, cx, cy, base size W, H
and a pyramid depth `levels` (level l has size W/2^l x H/2^l).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Seeds (PCG64): scene 1000+k, views 2000+k, perturbation 3000+k,
# config-0 targets 4000, sampling draws 5000+k, head training 6000.
SEED_SCENE = 1000
SEED_VIEWS = 2000
SEED_PERTURB = 3000
SEED_TARGETS = 4000


@dataclasses.dataclass
class View:
    R: np.ndarray          # [3,3] float32, world -> camera rotation
    t: np.ndarray          # [3]   float32
    fx: float
    fy: float
    cx: float
    cy: float
    W: int
    H: int
    levels: int


@dataclasses.dataclass
class Scene:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    rgb: np.ndarray
    sem: np.ndarray | None = None        # [N,C] float32 (plain)
    emb: np.ndarray | None = None        # [N,16] uint16 bf16 bits (learned)
    n_classes: int = 0

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    def copy(self) -> "Scene":
        return Scene(**{f.name: (getattr(self, f.name).copy()
                                 if isinstance(getattr(self, f.name), np.ndarray)
                                 else getattr(self, f.name))
                        for f in dataclasses.fields(self)})


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (round to nearest, ties to even); return bits."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    return ((u + rounding) >> 16).astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def _normalise_rows(q: np.ndarray) -> np.ndarray:
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _common_params(rng, n, log_mu, log_sd):
    log_scale = rng.normal(log_mu, log_sd, size=(n, 3))
    quat = _normalise_rows(rng.normal(size=(n, 4)))
    opacity = rng.normal(size=n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    return log_scale, quat, opacity, rgb


# --------------------------------------------------------------------------
# Tiny scene: Gaussians in a slab in front of an identity camera.
# --------------------------------------------------------------------------
def tiny_scene(n=2000, n_classes=8, seed=SEED_SCENE, log_mu=-3.0, log_sd=0.3,
               z_range=(2.0, 4.0), xy=1.0):
    rng = np.random.default_rng(seed)
    mean = np.empty((n, 3))
    mean[:, 0] = rng.uniform(-xy, xy, n)
    mean[:, 1] = rng.uniform(-xy, xy, n)
    mean[:, 2] = rng.uniform(z_range[0], z_range[1], n)
    log_scale, quat, opacity, rgb = _common_params(rng, n, log_mu, log_sd)
    sem = rng.normal(size=(n, n_classes))
    return Scene(mean.astype(np.float32), log_scale.astype(np.float32),
                 quat.astype(np.float32), opacity.astype(np.float32),
                 rgb.astype(np.float32), sem.astype(np.float32), None, n_classes)


def identity_view(W=128, H=96, fx=100.0, fy=100.0, cx=None, cy=None, levels=1):
    return View(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), float(fx), float(fy),
                float(W / 2 if cx is None else cx), float(H / 2 if cy is None else cy),
                int(W), int(H), int(levels))


def random_targets(n_pixels_per_item, n_classes, seed=SEED_TARGETS, depth_max=3.0,
                   invalid_frac=0.0):
    """Per item: rgb [3,H*W] ~U(0,1), depth [H*W] ~U(0,depth_max), labels ~U{0..C-1}.

    `invalid_frac` of the depth pixels are set to 0 (missing depth)."""
    rng = np.random.default_rng(seed)
    out = []
    for npx in n_pixels_per_item:
        rgb = rng.uniform(0, 1, size=(3, npx)).astype(np.float32)
        depth = rng.uniform(0, depth_max, size=npx).astype(np.float32)
        if invalid_frac > 0:
            depth[rng.uniform(size=npx) < invalid_frac] = 0.0
        labels = rng.integers(0, n_classes, size=npx).astype(np.int32)
        out.append((rgb, depth, labels))
    return out


# --------------------------------------------------------------------------
# Room-shaped scenes.
# --------------------------------------------------------------------------
def _sample_on_faces(rng, faces, n):
    """faces: list of (origin, u_vec, v_vec, surface_id). Uniform by area."""
    areas = np.array([np.linalg.norm(np.cross(u, v)) for _, u, v, _ in faces])
    which = rng.choice(len(faces), size=n, p=areas / areas.sum())
    a = rng.uniform(size=n)
    b = rng.uniform(size=n)
    pts = np.empty((n, 3))
    sid = np.empty(n, np.int64)
    for k, (o, u, v, s) in enumerate(faces):
        m = which == k
        pts[m] = o + a[m, None] * u + b[m, None] * v
        sid[m] = s
    return pts, sid


def _box_faces(lo, hi, with_bottom):
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    d = hi - lo
    ex, ey, ez = np.array([d[0], 0, 0]), np.array([0, d[1], 0]), np.array([0, 0, d[2]])
    faces = [
        (lo + ez, ex, ey),           # top
        (lo, ex, ez),                # y = lo
        (lo + ey, ex, ez),           # y = hi
        (lo, ey, ez),                # x = lo
        (lo + ex, ey, ez),           # x = hi
    ]
    if with_bottom:
        faces.append((lo, ex, ey))
    return faces


def room_scene(n=200_000, n_classes=52, seed=SEED_SCENE + 1, size=(6.0, 5.0, 3.0),
               n_boxes=20, surface_frac=0.7, log_mu=-4.5, log_sd=0.5, embed=False,
               partition_x=None):
    """Gaussians on the inner faces of a room box plus furniture boxes on the floor.

    Surfaces are numbered floor, ceiling, 4 walls, (the two faces of an optional
    partition wall at x=partition_x,) then the boxes; surface k carries class
    k mod C.  Logits are N(0,1)^C + 3*onehot(class).  With embed=True each
    Gaussian instead carries a 16-dim bfloat16 embedding ~N(0, 0.1)."""
    rng = np.random.default_rng(seed)
    X, Y, Z = size
    o = np.zeros(3)
    ex, ey, ez = np.array([X, 0, 0.]), np.array([0, Y, 0.]), np.array([0, 0, Z])
    room = [(o, ex, ey), (o + ez, ex, ey), (o, ex, ez), (o + ey, ex, ez), (o, ey, ez), (o + ex, ey, ez)]
    if partition_x is not None:
        px = np.array([partition_x, 0, 0.])
        # a wall with a 1.0 m x 2.1 m door centred in y
        y0 = Y / 2 - 0.5
        for side in (0, 1):
            off = px + np.array([0.0 if side == 0 else 1e-3, 0, 0])
            room.append((off, np.array([0, y0, 0.]), ez))
            room.append((off + np.array([0, y0 + 1.0, 0]), np.array([0, Y - y0 - 1.0, 0.]), ez))
            room.append((off + np.array([0, y0, 2.1]), np.array([0, 1.0, 0.]), np.array([0, 0, Z - 2.1])))
    faces = []
    sid = 0
    for k, (oo, u, v) in enumerate(room):
        if partition_x is not None and k >= 6:
            s = 6 + (k - 6) // 3          # the three pieces of one partition side share a surface
        else:
            s = k
        faces.append((oo, u, v, s))
    n_room_surfaces = 6 if partition_x is None else 8
    boxes = []
    for b in range(n_boxes):
        w = rng.uniform(0.3, 1.5, size=2)
        h = rng.uniform(0.3, 2.0)
        x0 = rng.uniform(0, X - w[0])
        y0 = rng.uniform(0, Y - w[1])
        lo = np.array([x0, y0, 0.0])
        hi = np.array([x0 + w[0], y0 + w[1], h])
        boxes.append((lo, hi))
    n_surf = int(round(n * surface_frac))
    pts_a, sid_a = _sample_on_faces(rng, faces, n_surf)
    box_faces = []
    for b, (lo, hi) in enumerate(boxes):
        for (oo, u, v) in _box_faces(lo, hi, with_bottom=False):
            box_faces.append((oo, u, v, n_room_surfaces + b))
    pts_b, sid_b = _sample_on_faces(rng, box_faces, n - n_surf)
    mean = np.concatenate([pts_a, pts_b])
    surf = np.concatenate([sid_a, sid_b])
    log_scale, quat, opacity, rgb = _common_params(rng, n, log_mu, log_sd)
    cls = surf % n_classes
    emb = None
    # class logits are drawn in every mode: in learned mode they define the plain
    # C-class render the head is fitted to
    sem = rng.normal(size=(n, n_classes))
    sem[np.arange(n), cls] += 3.0
    sem = sem.astype(np.float32)
    if embed:
        emb = f32_to_bf16_bits(rng.normal(0.0, 0.1, size=(n, 16)).astype(np.float32))
    sc = Scene(mean.astype(np.float32), log_scale.astype(np.float32), quat.astype(np.float32),
               opacity.astype(np.float32), rgb.astype(np.float32), sem, emb, n_classes)
    sc.boxes = boxes
    sc.room_size = size
    sc.surface_class = cls.astype(np.int32)
    return sc


def _rot(axis, ang):
    c, s = math.cos(ang), math.sin(ang)
    if axis == 'x':
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == 'y':
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def room_views(scene, n_views, W, H, fx=None, fy=None, cx=None, cy=None, levels=1,
               seed=SEED_VIEWS, level_choices=None):
    """Cameras uniform in the room shrunk by 0.5 m, at least 0.2 m from every box,
    yaw towards the room centre +- U(-60,60) deg (keyframes look into the room, not
    into the nearest wall), pitch U(-30,30) deg, roll U(-10,10) deg.

    `levels` is a fixed pyramid depth, or `level_choices` a tuple to draw from per view."""
    rng = np.random.default_rng(seed)
    X, Y, Z = scene.room_size
    fx = W / 2 if fx is None else fx
    fy = fx if fy is None else fy
    cx = W / 2 if cx is None else cx
    cy = H / 2 if cy is None else cy
    # camera looking along world +x, z up  ->  OpenCV axes (x right, y down, z forward)
    base_wc = np.array([[0, 0, 1], [-1, 0, 0], [0, -1, 0]], float)  # columns: cam x,y,z in world
    views = []
    while len(views) < n_views:
        c = rng.uniform([0.5, 0.5, 0.5], [X - 0.5, Y - 0.5, Z - 0.5])
        bad = False
        for lo, hi in scene.boxes:
            if np.all(c > lo - 0.2) and np.all(c < hi + 0.2):
                bad = True
        # keyframes look into the room: yaw towards the room centre +- 60 degrees
        yaw = math.atan2(Y / 2 - c[1], X / 2 - c[0]) + math.radians(rng.uniform(-60, 60))
        pitch = math.radians(rng.uniform(-30, 30))
        roll = math.radians(rng.uniform(-10, 10))
        lv = levels if level_choices is None else int(rng.choice(level_choices))
        if bad:
            continue
        R_wc = _rot('z', yaw) @ base_wc @ _rot('x', pitch) @ _rot('z', roll)
        R_cw = R_wc.T
        t_cw = -R_cw @ c
        views.append(View(R_cw.astype(np.float32), t_cw.astype(np.float32), float(fx), float(fy),
                          float(cx), float(cy), int(W), int(H), int(lv)))
    return views


def perturbed(scene: Scene, seed=SEED_PERTURB):
    """A perturbed copy used to render target images: mean += N(0,0.01 m),
    log_scale += N(0,0.1), quat += N(0,0.05) (renormalised), opacity += N(0,0.3),
    rgb += N(0,0.05) clipped to [0,1], logits += N(0,0.3)."""
    rng = np.random.default_rng(seed)
    s = scene.copy()
    n = s.n
    s.mean = (s.mean + rng.normal(0, 0.01, (n, 3))).astype(np.float32)
    s.log_scale = (s.log_scale + rng.normal(0, 0.1, (n, 3))).astype(np.float32)
    s.quat = _normalise_rows(s.quat + rng.normal(0, 0.05, (n, 4))).astype(np.float32)
    s.opacity = (s.opacity + rng.normal(0, 0.3, n)).astype(np.float32)
    s.rgb = np.clip(s.rgb + rng.normal(0, 0.05, (n, 3)), 0, 1).astype(np.float32)
    if s.sem is not None:
        s.sem = (s.sem + rng.normal(0, 0.3, s.sem.shape)).astype(np.float32)
    for a in ('boxes', 'room_size', 'surface_class'):
        if hasattr(scene, a):
            setattr(s, a, getattr(scene, a))
    return s


# --------------------------------------------------------------------------
# Named workloads.
# --------------------------------------------------------------------------
def config_tiny():
    """2,000 Gaussians, C=8, one 128x96 view (fx=fy=100, cx=64, cy=48), 1 level."""
    sc = tiny_scene()
    return sc, [identity_view(128, 96, 100.0, 100.0, 64.0, 48.0, 1)]


def config_room(n=200_000, n_classes=52):
    """200k Gaussians in a 6x5x3 m room, C=52, one 1200x680 view (fx=fy=600), 3 levels."""
    sc = room_scene(n=n, n_classes=n_classes)
    views = room_views(sc, 1, 1200, 680, 600.0, 600.0, 600.0, 340.0, levels=3)
    return sc, views


def config_batch(n=500_000, n_classes=20, n_views=8, embed=False):
    """500k-Gaussian room, 8 views at 640x480, each with 1-3 pyramid levels."""
    sc = room_scene(n=n, n_classes=n_classes, seed=SEED_SCENE + 2, embed=embed)
    views = room_views(sc, n_views, 640, 480, seed=SEED_VIEWS + 2, level_choices=(1, 2, 3))
    return sc, views


def synthetic_projection(item_sizes, n, seed=5000, tie_depths=True, cull_frac=0.2, max_radius=40):
    """Per (item, Gaussian) projected means (hi, lo float pairs), integer radii and
    float32 depths for testing the binning stage alone.

    item_sizes: list of (W, H). Means are spread over and beyond each image, a fraction
    of entries is culled (radius 0) and, with tie_depths, depths come from a small set
    so that many entries tie and the index tie-break decides."""
    rng = np.random.default_rng(seed)
    E = len(item_sizes) * n
    hi = np.empty((E, 2), np.float32)
    for k, (W, H) in enumerate(item_sizes):
        s = slice(k * n, (k + 1) * n)
        hi[s, 0] = rng.uniform(-0.2 * W, 1.2 * W, n)
        hi[s, 1] = rng.uniform(-0.2 * H, 1.2 * H, n)
    lo = (rng.normal(size=(E, 2)) * np.abs(hi) * 2.0 ** -26).astype(np.float32)
    radius = rng.integers(1, max_radius, E).astype(np.int32)
    radius[rng.uniform(size=E) < cull_frac] = 0
    if tie_depths:
        depth = rng.choice(np.float32([0.5, 1.0, 1.25, 2.0, 3.5, 7.0]), E).astype(np.float32)
    else:
        depth = rng.uniform(0.25, 20.0, E).astype(np.float32)
    return hi, lo, radius, depth


def semantic_colour_scene(sc: Scene, seed=SEED_SCENE + 50, noise=0.05) -> Scene:
    """A copy of sc whose semantic feature is a colour (3 channels, Sec. III-B's semantic
    colour): each Gaussian takes its class's colour, the class being the argmax of its
    logits, from a seeded palette of uniform colours, plus N(0, noise^2), clipped to [0, 1]."""
    rng = np.random.default_rng(seed)
    palette = rng.uniform(0.0, 1.0, size=(max(sc.n_classes, 1), 3))
    cls = np.argmax(sc.sem, axis=1) if sc.sem is not None and sc.n_classes > 0 else np.zeros(sc.n, np.int64)
    col = np.clip(palette[cls] + rng.normal(0.0, noise, size=(sc.n, 3)), 0.0, 1.0)
    out = sc.copy()
    out.sem = col.astype(np.float32)
    out.emb = None
    out.n_classes = 3
    return out


def random_image(n_pixels, K, seed=5100, scale=1.0):
    """Planar K-channel image of n_pixels pixels, N(0, scale^2)."""
    rng = np.random.default_rng(seed)
    return (rng.normal(size=n_pixels * K) * scale).astype(np.float32)


def head_weights(n_classes, seed=6000, d_in=16, d_hidden=64):
    """Initial learned-head weights: W1 ~ N(0, 1/d_in), W2 ~ N(0, 1/d_hidden) as bfloat16
    bits, biases zero (float32)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, 1.0 / math.sqrt(d_in), size=(d_hidden, d_in)).astype(np.float32)
    W2 = rng.normal(0.0, 1.0 / math.sqrt(d_hidden), size=(n_classes, d_hidden)).astype(np.float32)
    return dict(W1=f32_to_bf16_bits(W1), b1=np.zeros(d_hidden, np.float32), W2=f32_to_bf16_bits(W2),
                b2=np.zeros(n_classes, np.float32))


def config_learned(n=500_000, n_classes=52, n_views=8):
    """The batched room scene with a 16-dim bfloat16 embedding per Gaussian (and the
    52-class logits that define the plain render), 8 views at 640x480, 1-3 levels."""
    sc = room_scene(n=n, n_classes=n_classes, seed=SEED_SCENE + 2, embed=True)
    views = room_views(sc, n_views, 640, 480, seed=SEED_VIEWS + 2, level_choices=(1, 2, 3))
    return sc, views


def config_large(n=2_000_000, n_classes=52, n_views=16):
    """Two rooms (12x10x3 m, a partition at x = 6 m with a 1.0 x 2.1 m door), 40 boxes,
    2M Gaussians, 52 classes with a 16-dim bfloat16 embedding each; 16 views at 1920x1080
    (fx = fy = 960 at the image centre), 4 pyramid levels each."""
    sc = room_scene(n=n, n_classes=n_classes, seed=SEED_SCENE + 4, size=(12.0, 10.0, 3.0), n_boxes=40,
                    partition_x=6.0, embed=True)
    views = room_views(sc, n_views, 1920, 1080, levels=4, seed=SEED_VIEWS + 4)
    return sc, views
