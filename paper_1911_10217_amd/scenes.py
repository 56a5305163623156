"""Seeded synthetic scenes for the many-light direct-lighting workloads.

This module only makes inputs: emissive triangles, their emission, occluder
boxes, shading points with normals, and the method parameters each workload
runs with.  It holds none of the method's arithmetic; the GPU library and the
CPU oracle both take these arrays as they are.

The paper's scenes (a bathroom with Cornell boxes lit by a sky dome and area
lights, and a sky-lit architectural interior) are not available, so these
scenes stand in for them:

* ``tiny``     - 1,024 random triangles in a ceiling band over a unit box,
                 4,096 random points with cosine-distributed normals about +y,
                 64 random boxes; an 8^3 dense grid, cut size 16, 16 spp,
                 8 static frames.
* ``static``   - 65,536 triangles in 256 Gaussian clusters (sigma 0.02) under
                 the ceiling of a unit room and 4,096 box occluders: 3,456
                 cluttering the floor, 384 louvres just below the lights (the
                 lights are seen only through the gaps between them) and 256
                 in mid-air; the shading points are the 1920x1080 primary hits
                 of a pinhole camera looking down across the room (about
                 5,800 cells of the 64^3 hashed grid), listed in 16x16 pixel
                 tiles of 8x8 sub-tiles as a tiled renderer emits them.  Cut size 64, 1 spp,
                 32 frames.  It plays the paper's visibility-dominated
                 interior lit through small openings.
* ``dynamic``  - 16 walled compartments (4x4), each with its own cluster of
                 65,536 triangles under its ceiling (1,048,576 in total),
                 1,048,576 points on floors and walls, 16,384 wall bricks;
                 emission per cluster animated as Le * (1 + sin(2 pi f t +
                 phi)), f ~ U[0.1, 1] cycles per frame, phi ~ U[0, 2 pi).
                 The compartments stand in for the paper's Cornell boxes, each
                 lit only by its own light.

Every array is float32 (uint32 for indices) and C-contiguous.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

# Seeds: 19111021700 + workload number.
SEED_BASE = 19111021700

DEFAULT_PARAMS = dict(
    M=16,
    alpha=0.1,
    T=2.0,
    eps=0.05,
    fx_shift=32,
    reward_max=65536.0,
    t_lo=1e-4,
    reward_mode=0,
    two_sided=1,
    albedo=0.7,
    grid_lo=(0.0, 0.0, 0.0),
    grid_hi=(1.0, 1.0, 1.0),
    grid_dims=(8, 8, 8),
    hashed=0,
    capacity=0,
    max_cells=0,
    adapt=1,
    temporal=1,
    split_steps=1,
    normal_bits=0,
    jitter=0.0,
    scene_id=0,
    seed=SEED_BASE + 1,
    occ_grid_res=0,
    spp=1,
    frames=1,
)


@dataclasses.dataclass
class Scene:
    name: str
    tri: np.ndarray        # (N, 9) v0 v1 v2
    emit: np.ndarray       # (N, 3) RGB emission
    boxes: np.ndarray      # (K, 6) min xyz, max xyz
    pos: np.ndarray        # (P, 3) shading points
    nrm: np.ndarray        # (P, 3) unit normals
    params: dict
    emission_at: Optional[Callable[[int], np.ndarray]] = None  # frame -> (N, 3)
    image_size: Optional[tuple] = None
    pixel: Optional[np.ndarray] = None   # image position (row * width + col) of each point
    footprint: Optional[np.ndarray] = None  # (P,) side of each primary hit's pixel footprint

    def to_image(self, values: np.ndarray) -> np.ndarray:
        """Per-point values (P, ...) laid out as the (height, width, ...) image."""
        h, w = self.image_size
        out = np.zeros((h * w,) + values.shape[1:], values.dtype)
        out[self.pixel] = values
        return out.reshape((h, w) + values.shape[1:])

    @property
    def N(self) -> int:
        return int(self.tri.shape[0])

    @property
    def K(self) -> int:
        return int(self.boxes.shape[0])

    @property
    def P(self) -> int:
        return int(self.pos.shape[0])


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _cosine_normals(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit normals distributed as cos(theta) about +y."""
    u1 = rng.random(n)
    u2 = rng.random(n)
    r = np.sqrt(u1)
    phi = 2.0 * np.pi * u2
    v = np.stack([r * np.cos(phi), np.sqrt(np.maximum(0.0, 1.0 - u1)), r * np.sin(phi)], axis=1)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return _f32(v)


def _random_boxes(rng, k, centre_lo, centre_hi, side_lo=0.02, side_hi=0.1) -> np.ndarray:
    c = rng.uniform(centre_lo, centre_hi, size=(k, 3))
    h = 0.5 * rng.uniform(side_lo, side_hi, size=(k, 3))
    return _f32(np.concatenate([c - h, c + h], axis=1))


def params_for(**overrides) -> dict:
    p = dict(DEFAULT_PARAMS)
    p.update(overrides)
    return p


# --------------------------------------------------------------------------
# tiny: the small plain-method workload
# --------------------------------------------------------------------------
def make_tiny(n_lights=1024, n_points=4096, n_boxes=64, M=16, spp=16, frames=8,
              seed=SEED_BASE + 1, **overrides) -> Scene:
    rng = np.random.default_rng(seed)
    v = rng.uniform([0.0, 0.9, 0.0], [1.0, 1.0, 1.0], size=(n_lights, 3, 3))
    tri = _f32(v.reshape(n_lights, 9))
    emit = _f32(rng.random((n_lights, 3)))
    pos = _f32(rng.random((n_points, 3)))
    nrm = _cosine_normals(rng, n_points)
    boxes = _random_boxes(rng, n_boxes, 0.0, 1.0) if n_boxes else np.zeros((0, 6), np.float32)
    params = params_for(M=M, spp=spp, frames=frames, grid_dims=(8, 8, 8), hashed=0,
                        seed=seed)
    params.update(overrides)
    return Scene("tiny", tri, emit, boxes, pos, nrm, params)


# --------------------------------------------------------------------------
# Primary hits of a pinhole camera in a unit room with box occluders.
# --------------------------------------------------------------------------
def _primary_hits(boxes: np.ndarray, width: int, height: int, cam=(0.5, 0.45, 0.02), look=None,
                  vfov_deg=60.0, room_lo=(0.0, 0.0, 0.0), room_hi=(1.0, 1.0, 1.0)):
    """Cast one ray through every pixel centre of a pinhole camera at `cam`
    looking at `look` (default: along +z), +y up.

    Returns float32 positions snapped onto the face that was hit, the
    axis-aligned face normal pointing back towards the camera, and the side
    of each hit's pixel footprint: the square root of the surface area the
    pixel covers, t s sqrt(cos^3(alpha) / cos(theta)) for a hit at distance
    t, pixel pitch s on the image plane at distance 1, alpha the ray's angle
    to the optical axis and theta its angle to the surface normal.  Pixels
    are in row-major order, top row first.
    """
    o = np.asarray(cam, dtype=np.float64)
    fwd = (np.asarray(look, np.float64) - o) if look is not None else np.array([0.0, 0.0, 1.0])
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    tan_h = math.tan(math.radians(vfov_deg) * 0.5)
    aspect = width / height
    px = (np.arange(width) + 0.5) / width * 2.0 - 1.0
    py = 1.0 - (np.arange(height) + 0.5) / height * 2.0
    sx = np.broadcast_to(px[None, :] * tan_h * aspect, (height, width)).reshape(-1)
    sy = np.broadcast_to(py[:, None] * tan_h, (height, width)).reshape(-1)
    d = sx[:, None] * right[None, :] + sy[:, None] * up[None, :] + fwd[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    n_pix = d.shape[0]
    with np.errstate(divide="ignore"):
        inv = 1.0 / d

    # room walls (inside faces); the camera is inside the room
    lo = np.asarray(room_lo, np.float64)
    hi = np.asarray(room_hi, np.float64)
    t_best = np.full(n_pix, np.inf)
    axis_best = np.zeros(n_pix, np.int64)
    plane_best = np.zeros(n_pix)
    for a in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            t_hi = np.where(d[:, a] > 0, (hi[a] - o[a]) * inv[:, a], np.inf)
            t_lo = np.where(d[:, a] < 0, (lo[a] - o[a]) * inv[:, a], np.inf)
        for t, plane in ((t_hi, hi[a]), (t_lo, lo[a])):
            better = t < t_best
            t_best = np.where(better, t, t_best)
            axis_best = np.where(better, a, axis_best)
            plane_best = np.where(better, plane, plane_best)

    # boxes: test each box against the pixels inside its screen-space bound
    bx = boxes.astype(np.float64)
    corners = np.stack([np.stack([bx[:, 0 if (c & 1) == 0 else 3],
                                  bx[:, 1 if (c & 2) == 0 else 4],
                                  bx[:, 2 if (c & 4) == 0 else 5]], axis=1) for c in range(8)], axis=1)
    rel = corners - o[None, None, :]
    zc = rel @ fwd
    xc = rel @ right
    yc = rel @ up
    all_pix = np.arange(n_pix)
    for b in range(bx.shape[0]):
        if np.all(zc[b] <= 0):
            continue  # behind the camera
        if np.any(zc[b] <= 1e-6):
            idx = all_pix
        else:
            qx = xc[b] / zc[b] / (tan_h * aspect)
            qy = yc[b] / zc[b] / tan_h
            c0 = int(max(0, math.floor((qx.min() + 1.0) * 0.5 * width) - 1))
            c1 = int(min(width, math.ceil((qx.max() + 1.0) * 0.5 * width) + 1))
            r0 = int(max(0, math.floor((1.0 - qy.max()) * 0.5 * height) - 1))
            r1 = int(min(height, math.ceil((1.0 - qy.min()) * 0.5 * height) + 1))
            if c0 >= c1 or r0 >= r1:
                continue
            idx = (np.arange(r0, r1)[:, None] * width + np.arange(c0, c1)[None, :]).reshape(-1)
        dd = d[idx]
        iv = inv[idx]
        tn = np.zeros(idx.size)
        tf = np.full(idx.size, np.inf)
        ax = np.zeros(idx.size, np.int64)
        pl = np.zeros(idx.size)
        with np.errstate(invalid="ignore"):
            for a in range(3):
                t0 = (bx[b, a] - o[a]) * iv[:, a]
                t1 = (bx[b, 3 + a] - o[a]) * iv[:, a]
                near = np.minimum(t0, t1)
                enter_plane = np.where(dd[:, a] > 0, bx[b, a], bx[b, 3 + a])
                upd = near > tn
                tn = np.where(upd, near, tn)
                ax = np.where(upd, a, ax)
                pl = np.where(upd, enter_plane, pl)
                tf = np.minimum(tf, np.maximum(t0, t1))
        hit = (tn < tf) & (tn > 0) & (tn < t_best[idx])
        sel = idx[hit]
        t_best[sel] = tn[hit]
        axis_best[sel] = ax[hit]
        plane_best[sel] = pl[hit]

    p = o[None, :] + t_best[:, None] * d
    nrm = np.zeros_like(p)
    rows = np.arange(n_pix)
    p[rows, axis_best] = plane_best
    nrm[rows, axis_best] = -np.sign(d[rows, axis_best])
    pitch = 2.0 * tan_h / height
    cos_a = d @ fwd
    cos_t = np.maximum(np.abs(d[rows, axis_best]), 1e-6)
    fp = t_best * pitch * np.sqrt(cos_a ** 3 / cos_t)
    return _f32(p), _f32(nrm), _f32(fp)


def tiled_pixel_order(width: int, height: int, tile: int = 16, sub: int = 8) -> np.ndarray:
    """Row-major pixel indices reordered into tile x tile blocks made of
    sub x sub blocks (the order a tiled renderer emits its primary hits in);
    partial tiles at the right and bottom edges keep the same nesting."""
    y, x = np.divmod(np.arange(width * height), width)
    order = np.lexsort((x % sub, y % sub, (x % tile) // sub, (y % tile) // sub, x // tile, y // tile))
    return order


def _clustered_lights(rng, n_clusters, per_cluster, centre_lo, centre_hi, sigma=0.02, half=0.005):
    centres = rng.uniform(centre_lo, centre_hi, size=(n_clusters, 3))
    cen = centres[:, None, :] + sigma * rng.standard_normal((n_clusters, per_cluster, 3))
    verts = cen[:, :, None, :] + rng.uniform(-half, half, size=(n_clusters, per_cluster, 3, 3))
    tri = _f32(verts.reshape(n_clusters * per_cluster, 9))
    le_cluster = rng.random((n_clusters, 3))
    emit = _f32(np.repeat(le_cluster, per_cluster, axis=0))
    return tri, emit, centres, le_cluster


# --------------------------------------------------------------------------
# static: the large static workload (the headline throughput measurement)
# --------------------------------------------------------------------------
def make_static(width=1920, height=1080, n_clusters=256, per_cluster=256, n_boxes=4096,
                M=64, spp=1, frames=32, seed=SEED_BASE + 2, capacity=1 << 19, max_cells=1 << 14,
                **overrides) -> Scene:
    rng = np.random.default_rng(seed)
    tri, emit, _, _ = _clustered_lights(rng, n_clusters, per_cluster,
                                        [0.05, 0.90, 0.05], [0.95, 0.98, 0.95])
    n_louvre = (n_boxes * 3) // 32
    n_air = n_boxes // 16
    n_floor = n_boxes - n_louvre - n_air
    boxes = np.concatenate([
        _random_boxes(rng, n_floor, [0.0, 0.0, 0.0], [1.0, 0.12, 1.0]),
        _random_boxes(rng, n_louvre, [0.0, 0.78, 0.0], [1.0, 0.86, 1.0]),
        _random_boxes(rng, n_air, [0.0, 0.15, 0.2], [1.0, 0.7, 1.0]),
    ]).astype(np.float32)
    pos, nrm, fp = _primary_hits(boxes, width, height, cam=(0.1, 0.7, 0.05), look=(0.7, 0.1, 0.8))
    order = tiled_pixel_order(width, height)
    params = params_for(M=M, spp=spp, frames=frames, grid_dims=(64, 64, 64), hashed=1,
                        capacity=capacity, max_cells=max_cells, seed=seed, occ_grid_res=64)
    params.update(overrides)
    return Scene("static", tri, emit, boxes, np.ascontiguousarray(pos[order]), np.ascontiguousarray(nrm[order]),
                 params, image_size=(height, width), pixel=order.astype(np.int64),
                 footprint=np.ascontiguousarray(fp[order]))


# --------------------------------------------------------------------------
# dynamic: walled compartments, each with its own animated light
# --------------------------------------------------------------------------
def make_dynamic(n_points=1 << 20, per_cluster=65536, grid=4, n_bricks=16384, M=64, spp=1,
                 frames=60, seed=SEED_BASE + 3, capacity=1 << 19, max_cells=1 << 17, **overrides) -> Scene:
    rng = np.random.default_rng(seed)
    n_comp = grid * grid
    cw = 1.0 / grid
    # lights: one cluster per compartment, centred under its ceiling
    cx = (np.arange(grid) + 0.5) * cw
    centres = np.array([[cx[i], 0.93, cx[j]] for j in range(grid) for i in range(grid)], np.float64)
    spread = np.array([0.15 * cw, 0.01, 0.15 * cw])
    cen = centres[:, None, :] + spread * rng.standard_normal((n_comp, per_cluster, 3))
    verts = cen[:, :, None, :] + rng.uniform(-0.002, 0.002, size=(n_comp, per_cluster, 3, 3))
    tri = _f32(verts.reshape(n_comp * per_cluster, 9))
    base = rng.random((n_comp, 3))
    freq = rng.uniform(0.1, 1.0, size=n_comp)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_comp)

    def emission_at(frame: int) -> np.ndarray:
        # Le (1 + sin(2 pi f t + phi)) per compartment, t = frame index
        s = 1.0 + np.sin(2.0 * np.pi * freq * float(frame) + phase)
        return _f32(np.repeat(base * s[:, None], per_cluster, axis=0))

    emit = emission_at(0)
    # walls: bricks tiling the interior partition planes x = k/grid and
    # z = k/grid (k = 1..grid-1), floor to ceiling, 0.02 thick
    th = 0.01
    n_planes = 2 * (grid - 1)
    bricks = []
    if n_planes:
        per_plane = n_bricks // n_planes
        rows = max(1, int(round(math.sqrt(per_plane))))
        cols = max(1, per_plane // rows)
        for axis in (0, 2):
            for k in range(1, grid):
                w = k * cw
                for r in range(rows):
                    y0, y1 = r / rows, (r + 1) / rows
                    for c in range(cols):
                        u0, u1 = c / cols, (c + 1) / cols
                        if axis == 0:
                            bricks.append([w - th, y0, u0, w + th, y1, u1])
                        else:
                            bricks.append([u0, y0, w - th, u1, y1, w + th])
    while len(bricks) < n_bricks:  # pad with small boxes under the floor
        bricks.append([0.0, -0.02, 0.0, 0.001, -0.01, 0.001])
    boxes = _f32(np.array(bricks[:n_bricks]).reshape(-1, 6))
    # points: half on compartment floors, half on compartment walls
    comp = rng.integers(0, n_comp, size=n_points)
    ci = comp % grid
    cj = comp // grid
    lo_x = ci * cw + th
    lo_z = cj * cw + th
    span = cw - 2 * th
    u = rng.random(n_points)
    v = rng.random(n_points)
    side = rng.integers(0, 4, size=n_points)
    floor = np.arange(n_points) < n_points // 2
    pos = np.zeros((n_points, 3))
    nrm = np.zeros((n_points, 3))
    # floor points
    pos[:, 0] = lo_x + u * span
    pos[:, 2] = lo_z + v * span
    nrm[:, 1] = 1.0
    # wall points: side 0/1 = -x/+x wall, 2/3 = -z/+z wall
    wall = ~floor
    h = v * 0.9
    px = np.where(side == 0, lo_x, np.where(side == 1, lo_x + span, lo_x + u * span))
    pz = np.where(side == 2, lo_z, np.where(side == 3, lo_z + span, lo_z + u * span))
    pos[wall, 0] = px[wall]
    pos[wall, 1] = h[wall]
    pos[wall, 2] = pz[wall]
    nrm[wall] = 0.0
    nrm[wall, 0] = np.where(side[wall] == 0, 1.0, np.where(side[wall] == 1, -1.0, 0.0))
    nrm[wall, 2] = np.where(side[wall] == 2, 1.0, np.where(side[wall] == 3, -1.0, 0.0))
    # delivered in Morton order of their 1/64 cells, as a renderer's screen
    # tiles deliver neighbouring surface points together
    order = np.argsort(_morton_key(pos, 64), kind="stable")
    pos, nrm = pos[order], nrm[order]
    params = params_for(M=M, spp=spp, frames=frames, grid_dims=(64, 64, 64), hashed=1,
                        capacity=capacity, max_cells=max_cells, seed=seed, occ_grid_res=64)
    params.update(overrides)
    return Scene("dynamic", tri, emit, boxes, _f32(pos), _f32(nrm), params, emission_at=emission_at)


def _morton_key(pos: np.ndarray, res: int) -> np.ndarray:
    """Morton (Z-order) index of the res^3 cell of each point of [0, 1]^3."""
    c = np.clip(np.floor(pos * res), 0, res - 1).astype(np.uint64)
    key = np.zeros(pos.shape[0], np.uint64)
    for b in range(int(res - 1).bit_length()):
        for a in range(3):
            key |= ((c[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + a)
    return key


# --------------------------------------------------------------------------
# batched: uneven static-style scenes rendered together
# --------------------------------------------------------------------------
def _log_uniform(rng, lo, hi):
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def make_batch(n_scenes=16, seed=SEED_BASE + 4, capacity=1 << 16, frames=16, **overrides):
    """n_scenes scenes in the style of the static workload with log-uniform
    sizes: emitters in [4,096, 1,048,576] (256 clusters), shading points in
    [65,536, 2,097,152] (primary hits of a 16:9 camera), box occluders in
    [64, 16,384]; cut sizes 16, 32, 64 in turn; scene i has scene id i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_scenes):
        N = int(round(_log_uniform(rng, 4096, 1 << 20)))
        P = int(round(_log_uniform(rng, 65536, 1 << 21)))
        K = int(round(_log_uniform(rng, 64, 16384)))
        M = (16, 32, 64)[i % 3]
        width = max(16, int(round(math.sqrt(P * 16.0 / 9.0))))
        height = max(9, int(round(P / width)))
        per_cluster = max(1, int(round(N / 256)))
        s = make_static(width=width, height=height, n_clusters=256, per_cluster=per_cluster, n_boxes=K, M=M,
                        spp=1, frames=frames, seed=int(rng.integers(1 << 40)), capacity=capacity, scene_id=i,
                        **overrides)
        s.name = "batch%d" % i
        out.append(s)
    return out


WORKLOADS = {"tiny": make_tiny, "static": make_static, "dynamic": make_dynamic}


def make(name: str, **kw) -> Scene:
    return WORKLOADS[name](**kw)
