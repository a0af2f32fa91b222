"""Seeded synthetic scenes, cameras and deferred-MLP weights.

This module only *produces inputs*: feature textures of ground-partitioned
MERF-style blocks (a low-res 3D grid plus three high-res planes per block and
LOD, Sec. 4.1 "Rendering Stage"), pinhole cameras and the weights of the tiny
deferred MLP (Eq. "deferred").  It holds none of the rendering arithmetic
(no occupancy, no ray marching, no compositing), so both the HIP path and the
CPU oracle can be fed from it without sharing any of the method's code.

Stand-in data.  The paper measures on trained assets of its Campus scene
(Sec. 5, Table 2), which are not available; the scenes below keep the paper's
structure: blocks partition the ground plane without a z split (Eq. "blocks"),
each block is a sparse grid + triplanes (Sec. 3), textures are 8-bit with a
per-channel scale/offset (Sec. 4.5 baking to PNG), content sits near the ground
and views are aerial.

Conventions (shared by every consumer):
  * block (bx, by) is the unit cube [bx, bx+1] x [by, by+1] x [0, 1];
    block_id = by * nbx + bx.  A merged LOD asset (quadtree LOD) spans
    2^l x 2^l blocks; resolutions are texels per unit length, so a texture
    holds R * extent texels along each axis (below, for a unit block).
  * grid texture  : array [R][R][R][8]  indexed [z][y][x][channel]
  * plane xy      : array [Rp][Rp][8]   indexed [y][x][channel]
  * plane xz      : array [Rp][Rp][8]   indexed [z][x][channel]
  * plane yz      : array [Rp][Rp][8]   indexed [z][y][channel]
  * channel 0 is pre-activation density, 1-3 diffuse, 4-7 specular features.
  * scale/offset  : float32 [4][8] (texture 0 grid, 1 xy, 2 xz, 3 yz);
    a uint8 texel q decodes to q * scale + offset.
  * camera        : OpenCV axes (x right, y down, z forward); R is
    camera-to-world with columns (right, down, forward), stored row-major.
  * MLP weights   : flat float32[499] = W1[16][10], b1[16], W2[16][16], b2[16],
    W3[3][16], b3[3] (row-major, out x in).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

NCH = 8
MLP_SIZES = ((16, 10), (16, 16), (3, 16))
MLP_NPARAM = sum(o * i + o for o, i in MLP_SIZES)  # 499

U8 = 0
F32 = 1


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclass
class BlockLod:
    block_id: int
    lod: int
    aabb_min: np.ndarray  # float32[3]
    aabb_max: np.ndarray  # float32[3]
    grid_res: int
    plane_res: int
    occ_res: int
    dtype: int  # U8 or F32
    grid: np.ndarray  # [R][R][R][8] uint8 or float32
    planes: list  # 3 x [Rp][Rp][8]
    scale: np.ndarray  # float32[4][8]
    offset: np.ndarray  # float32[4][8]
    contracted: bool = False  # boundary block whose textures cover the contracted cube

    def decoded(self):
        """Float32 texture values (grid, [xy, xz, yz]) after the uint8 decode."""
        if self.dtype == F32:
            return self.grid, list(self.planes)
        g = self.grid.astype(np.float32) * self.scale[0] + self.offset[0]
        ps = [p.astype(np.float32) * self.scale[1 + i] + self.offset[1 + i]
              for i, p in enumerate(self.planes)]
        return g.astype(np.float32), [p.astype(np.float32) for p in ps]


@dataclass
class Scene:
    nbx: int
    nby: int
    blocks: list = field(default_factory=list)  # list[BlockLod]

    def get(self, block_id, lod):
        for b in self.blocks:
            if b.block_id == block_id and b.lod == lod:
                return b
        raise KeyError((block_id, lod))

    @property
    def n_lods(self):
        return 1 + max(b.lod for b in self.blocks)


@dataclass
class View:
    W: int
    H: int
    eye: np.ndarray  # float32[3]
    R: np.ndarray  # float32[3][3], columns right, down, forward
    fx: float
    fy: float
    cx: float
    cy: float
    crop: tuple = None  # (x0, y0, w, h); None = full image

    def __post_init__(self):
        if self.crop is None:
            self.crop = (0, 0, self.W, self.H)
        self.eye = np.asarray(self.eye, np.float32)
        self.R = np.asarray(self.R, np.float32).reshape(3, 3)
        self.fx = float(np.float32(self.fx))
        self.fy = float(np.float32(self.fy))
        self.cx = float(np.float32(self.cx))
        self.cy = float(np.float32(self.cy))

    @property
    def n_pixels(self):
        return int(self.crop[2]) * int(self.crop[3])

    def with_crop(self, x0, y0, w, h):
        return View(self.W, self.H, self.eye.copy(), self.R.copy(), self.fx, self.fy,
                    self.cx, self.cy, (int(x0), int(y0), int(w), int(h)))


@dataclass
class RenderParams:
    mode: int = 1  # 0 = mode A (n_steps midpoints over the block chord), 1 = mode B
    n_steps: int = 128  # mode A
    delta: float = 1.0 / 512.0  # mode B step
    max_steps: int = 2048  # mode B cap, counted from scene entry
    t_min: float = 0.0  # early ray termination threshold on the transmittance (0: off)
    pe_freqs: int = 0  # deferred MLP input [C_d, F, PE(d)] with this many frequencies (0-4)
    ext_delta: float = 0.0  # exterior step scale of contracted boundary blocks (0: no exterior)
    ext_max_steps: int = 0  # exterior steps per segment


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def look_rotation(forward, up=(0.0, 0.0, 1.0)):
    """Camera-to-world rotation with columns (right, down, forward)."""
    f = np.asarray(forward, np.float64)
    f = f / np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r = r / np.linalg.norm(r)
    dn = np.cross(f, r)
    return np.stack([r, dn, f], axis=1)


def pinhole(W, H, eye, R, vfov_deg=60.0):
    f = (H / 2.0) / math.tan(math.radians(vfov_deg) / 2.0)
    return View(W, H, np.asarray(eye, np.float32), np.asarray(R, np.float32), f, f, W / 2.0, H / 2.0)


def yaw_pitch_forward(yaw, pitch_down):
    """Unit forward vector; yaw measured from +x toward +y, pitch below horizon."""
    c = math.cos(pitch_down)
    return np.array([c * math.cos(yaw), c * math.sin(yaw), -math.sin(pitch_down)])


# --------------------------------------------------------------------------
# textures
# --------------------------------------------------------------------------
def _box3(a, axis):
    """Separable 3-tap box [1,1,1]/3 with replicated edges along one axis."""
    a = np.moveaxis(a, axis, 0)
    out = np.empty_like(a)
    out[1:-1] = a[:-2] + a[1:-1]
    out[1:-1] += a[2:]
    out[0] = a[0] + a[0] + a[1]
    out[-1] = a[-2] + a[-1] + a[-1]
    out *= np.float32(1.0 / 3.0)
    return np.ascontiguousarray(np.moveaxis(out, 0, axis))


def smoothed_noise(rng, shape, axes):
    a = rng.standard_normal(shape, dtype=np.float32)
    for ax in axes:
        a = _box3(a, ax)
    return a


def blob_density_raw(centers_xyz, blobs, peak, shift):
    """raw = ln(1e-6 + sum_b peak*exp(-|p-mu_b|^2 / (2 s_b^2))) - shift on a
    separable lattice of points given by centers_xyz = (xs, ys, zs).
    Returns array [len(zs)][len(ys)][len(xs)] float32."""
    xs, ys, zs = centers_xyz
    if len(blobs) == 0:
        dens = np.zeros((len(zs), len(ys), len(xs)), np.float64)
    else:
        mu = blobs[:, 0:3]
        s = blobs[:, 3]
        inv = 1.0 / (2.0 * s * s)
        gx = np.exp(-((xs[None, :] - mu[:, 0:1]) ** 2) * inv[:, None])
        gy = np.exp(-((ys[None, :] - mu[:, 1:2]) ** 2) * inv[:, None])
        gz = np.exp(-((zs[None, :] - mu[:, 2:3]) ** 2) * inv[:, None])
        m = (gy[:, :, None] * gx[:, None, :]).reshape(len(blobs), -1)  # [B, ny*nx]
        dens = (gz.T @ m).reshape(len(zs), len(ys), len(xs)) * peak
    return (np.log(1e-6 + dens) - shift).astype(np.float32)


def quantize(v):
    """Per-channel uint8 quantisation: offset = min, scale = (max-min)/255."""
    flat = v.reshape(-1, v.shape[-1]).astype(np.float64)
    lo = flat.min(axis=0)
    hi = flat.max(axis=0)
    scale = (hi - lo) / 255.0
    scale[scale == 0] = 1.0
    scale32 = scale.astype(np.float32)
    off32 = lo.astype(np.float32)
    q = np.rint((v.astype(np.float64) - off32.astype(np.float64)) / scale32.astype(np.float64))
    q = np.clip(q, 0, 255).astype(np.uint8)
    return q, scale32, off32


def downsample2(a, ndim):
    """2x box downsample of the first `ndim` axes."""
    if ndim == 3:
        r = a.shape[0] // 2
        return a.reshape(r, 2, r, 2, r, 2, -1).mean(axis=(1, 3, 5)).astype(np.float32)
    r = a.shape[0] // 2
    return a.reshape(r, 2, r, 2, -1).mean(axis=(1, 3)).astype(np.float32)


def make_blobs(rng, nbx, nby, per_block, z_range, s_range):
    """Blob list per block: rows (mu_x, mu_y, mu_z, s)."""
    out = {}
    for by in range(nby):
        for bx in range(nbx):
            mu = np.stack([
                rng.uniform(bx, bx + 1, per_block),
                rng.uniform(by, by + 1, per_block),
                rng.uniform(z_range[0], z_range[1], per_block),
            ], axis=1)
            s = rng.uniform(s_range[0], s_range[1], per_block)
            out[(bx, by)] = np.concatenate([mu, s[:, None]], axis=1)
    return out


def make_scene(nbx=1, nby=1, lods=((32, 128, 8),), dtype=F32, blobs_per_block=20,
               blob_xy_inset=0.0, blob_z=(0.0, 1.0), blob_s=(0.05, 0.2), peak=50.0,
               shift=5.0, seed=0, plane_density_amp=0.3, single_block_blob_box=None):
    """Build a block scene.

    lods: sequence of (grid_res, plane_res, occ_res), finest first; level l>0 is
    a 2x box downsample of level l-1 (as the paper's "downsample" LOD baseline,
    Table 5) when the resolutions halve, otherwise generated afresh.
    """
    ss = np.random.SeedSequence(seed)
    blob_ss, tex_ss = ss.spawn(2)
    brng = np.random.default_rng(blob_ss)
    if single_block_blob_box is not None:
        lo, hi = single_block_blob_box
        mu = brng.uniform(lo, hi, size=(blobs_per_block, 3))
        s = brng.uniform(blob_s[0], blob_s[1], blobs_per_block)
        blobs = {(0, 0): np.concatenate([mu, s[:, None]], axis=1)}
    else:
        blobs = make_blobs(brng, nbx, nby, blobs_per_block, blob_z, blob_s)
    tex_streams = tex_ss.spawn(nbx * nby)

    def one_block(bid):
        bx, by = bid % nbx, bid // nbx
        rng = np.random.default_rng(tex_streams[bid])
        near = [blobs[(x, y)] for y in range(by - 1, by + 2) for x in range(bx - 1, bx + 2)
                if (x, y) in blobs]
        bl = np.concatenate(near, axis=0) if near else np.zeros((0, 4))
        R0, Rp0, _ = lods[0]
        c = (np.arange(R0) + 0.5) / R0
        raw = blob_density_raw((bx + c, by + c, c), bl, peak, shift)
        grid = np.empty((R0, R0, R0, NCH), np.float32)
        grid[..., 0] = raw
        grid[..., 1:] = smoothed_noise(rng, (R0, R0, R0, NCH - 1), (0, 1, 2))
        planes = []
        for _ in range(3):
            p = smoothed_noise(rng, (Rp0, Rp0, NCH), (0, 1))
            p[..., 0] *= np.float32(plane_density_amp)
            planes.append(p)
        out = []
        lvl_grid, lvl_planes = grid, planes
        for l, (R, Rp, O) in enumerate(lods):
            if l > 0:
                pR, pRp, _ = lods[l - 1]
                lvl_grid = downsample2(lvl_grid, 3) if R * 2 == pR else lvl_grid
                lvl_planes = [downsample2(p, 2) if Rp * 2 == pRp else p for p in lvl_planes]
                assert lvl_grid.shape[0] == R and lvl_planes[0].shape[0] == Rp
            if dtype == U8:
                qg, sg, og = quantize(lvl_grid)
                qp = [quantize(p) for p in lvl_planes]
                scale = np.stack([sg] + [x[1] for x in qp]).astype(np.float32)
                offset = np.stack([og] + [x[2] for x in qp]).astype(np.float32)
                g_store, p_store = qg, [x[0] for x in qp]
            else:
                scale = np.ones((4, NCH), np.float32)
                offset = np.zeros((4, NCH), np.float32)
                g_store, p_store = lvl_grid.copy(), [p.copy() for p in lvl_planes]
            out.append(BlockLod(
                bid, l, np.array([bx, by, 0], np.float32), np.array([bx + 1, by + 1, 1], np.float32),
                R, Rp, O, dtype, np.ascontiguousarray(g_store),
                [np.ascontiguousarray(p) for p in p_store], scale, offset))
        return out

    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(nbx * nby, os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(workers) as ex:
        per_block = list(ex.map(one_block, range(nbx * nby)))
    scene = Scene(nbx, nby)
    for lst in per_block:
        scene.blocks.extend(lst)
    return scene


def homogeneous_block(R=8, Rp=8, O=4, sigma=2.0, color=(0.2, 0.5, 0.8), feat=(0.1, 0.3, 0.6, 0.9),
                      block_id=0, origin=(0, 0, 0), dtype=F32):
    """A block whose field is constant: density sigma, colour/feature values
    given after activation (the raw values are their logits)."""
    def logit(v):
        return math.log(v / (1.0 - v))
    g = np.zeros((R, R, R, NCH), np.float32)
    g[..., 0] = math.log(sigma)
    for i, c in enumerate(color):
        g[..., 1 + i] = logit(c)
    for i, f in enumerate(feat):
        g[..., 4 + i] = logit(f)
    planes = [np.zeros((Rp, Rp, NCH), np.float32) for _ in range(3)]
    o = np.asarray(origin, np.float32)
    return BlockLod(block_id, 0, o, o + 1, R, Rp, O, dtype, g, planes,
                    np.ones((4, NCH), np.float32), np.zeros((4, NCH), np.float32))


def mlp_sizes(pe=0):
    """(out, in) of the three layers over 10 + 6 pe inputs."""
    return ((16, 10 + 6 * pe), (16, 16), (3, 16))


def mlp_nparam(pe=0):
    return sum(o * i + o for o, i in mlp_sizes(pe))


def xavier_mlp(seed, pe=0):
    """Xavier-uniform weights a = sqrt(6/(fan_in+fan_out)), zero biases."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[1])
    parts = []
    for o, i in mlp_sizes(pe):
        a = math.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-a, a, size=(o, i)).reshape(-1))
        parts.append(np.zeros(o))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == mlp_nparam(pe)
    return w


def random_mlp(seed, scale=1.0, pe=0):
    """Weights and biases all drawn from U(-scale, scale) (for tests that need
    non-zero biases)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, mlp_nparam(pe)).astype(np.float32)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def c1_scene(seed=0):
    """One unit block, fp32 32^3 grid + 128^2 planes, occupancy 8^3, 20 blobs."""
    return make_scene(1, 1, ((32, 128, 8),), F32, blobs_per_block=20,
                      single_block_blob_box=(0.1, 0.9), seed=seed)


def c1_view():
    c = np.array([0.5, 0.5, 0.5])
    d = np.array([1.0, -2.0, 1.0])
    eye = c + 1.5 * d / np.linalg.norm(d)
    return pinhole(128, 128, eye, look_rotation(c - eye))


def c1_params():
    return RenderParams(mode=0, n_steps=128)


def city_scene(nb, seed, dtype=U8, lods=((128, 1024, 16),), blobs_per_block=200):
    """Ground-partitioned city-like scene: nb x nb unit blocks, blobs at heights 0-0.3."""
    return make_scene(nb, nb, lods, dtype, blobs_per_block=blobs_per_block, blob_z=(0.0, 0.3),
                      seed=seed)


def c2_scene(seed=1):
    return city_scene(4, seed)


def c2_view(W=1920, H=1080):
    return pinhole(W, H, (2.0, -0.5, 1.2), look_rotation(yaw_pitch_forward(math.pi / 2, math.radians(30))))


def cityb_params():
    return RenderParams(mode=1, delta=1.0 / 512.0, max_steps=2048)


C3_LODS = ((128, 1024, 16), (64, 512, 8), (32, 256, 4))


def c3_scene(seed=2, lods=C3_LODS):
    return city_scene(8, seed, U8, lods)


def aerial_views(seed, n, resolutions, xy=(1.0, 7.0), h=(2.0, 6.0), pitch=(35.0, 65.0)):
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
    views = []
    for _ in range(n):
        W, H = resolutions[rng.integers(len(resolutions))]
        ex, ey = rng.uniform(xy[0], xy[1], 2)
        hh = rng.uniform(h[0], h[1])
        yaw = rng.uniform(0, 2 * math.pi)
        pd = math.radians(rng.uniform(pitch[0], pitch[1]))
        views.append(pinhole(int(W), int(H), (ex, ey, hh), look_rotation(yaw_pitch_forward(yaw, pd))))
    return views


def c3_views(seed=2):
    return aerial_views(seed, 16, [(1920, 1080)])


C4_RESOLUTIONS = [(256, 256), (800, 800), (1280, 720), (1920, 1080)]


# Trajectory ranges for the batched workload.  With the aerial ranges of the
# 16-view workload some views hold 1-3 or 50+ blocks after LOD selection
# (thresholds 2/4/8) and culling; these seeded ranges keep every view within
# 4-40 blocks (realised 8-38, mean 21.5) without changing the selection rule.
C4_TRAJECTORY = dict(xy=(3.0, 5.0), h=(1.2, 2.8), pitch=(45.0, 75.0))


def c4_views(seed=3):
    return aerial_views(seed, 64, C4_RESOLUTIONS, **C4_TRAJECTORY)


def _box_down(a, f, ndim):
    """Box downsample of the first `ndim` axes by an integer factor f."""
    if f == 1:
        return a.astype(np.float32)
    sh = []
    for n in a.shape[:ndim]:
        sh += [n // f, f]
    return a.reshape(*sh, a.shape[-1]).mean(axis=tuple(range(1, 2 * ndim, 2)), dtype=np.float32)


def merged_lods(finest, nbx, nby, n_lods, dtype=U8):
    """Merged LOD assets (Sec. 4.4 LOD generation, Sec. 4.5 baking): the
    entry of LOD l covers 2^l x 2^l blocks of the finest level, at 1/2^l of
    its texel density, as one asset.  Its grid and xy plane are the 2^l box
    downsample of the finest blocks' decoded textures laid side by side; its
    xz (yz) plane is the mean over the blocks along y (x) of their
    downsampled xz (yz) planes, laid side by side along x (y).  Resolutions
    are per unit length; block_id is that of the asset's lowest block.
    finest: the LOD-0 BlockLod of every block (block_id = by * nbx + bx)."""
    from concurrent.futures import ThreadPoolExecutor
    by_id = {b.block_id: b for b in finest if b.lod == 0}

    def downs(bid):  # per level l >= 1: downsampled (grid, xy, xz, yz) of one block
        g, ps = by_id[bid].decoded()
        return [(_box_down(g, 1 << l, 3), [_box_down(p, 1 << l, 2) for p in ps]) for l in range(1, n_lods)]

    workers = max(1, min(len(by_id), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(workers) as ex:
        down = dict(zip(by_id, ex.map(downs, list(by_id))))

    def asset(job):
        l, gx, gy = job
        f = 1 << l
        ids = [[(gy + j) * nbx + (gx + i) for i in range(f)] for j in range(f)]
        b0 = by_id[ids[0][0]]
        R, Rp, O = b0.grid_res // f, b0.plane_res // f, b0.occ_res // f
        d = {i: down[i][l - 1] for row in ids for i in row}
        grid = np.concatenate([np.concatenate([d[i][0] for i in row], axis=2) for row in ids], axis=1)
        xy = np.concatenate([np.concatenate([d[i][1][0] for i in row], axis=1) for row in ids], axis=0)
        xz = np.concatenate([np.mean([d[ids[j][i]][1][1] for j in range(f)], axis=0, dtype=np.float32)
                             for i in range(f)], axis=1)
        yz = np.concatenate([np.mean([d[ids[j][i]][1][2] for i in range(f)], axis=0, dtype=np.float32)
                             for j in range(f)], axis=1)
        planes = [xy, xz, yz]
        if dtype == U8:
            qg, sg, og = quantize(grid)
            qp = [quantize(p) for p in planes]
            scale = np.stack([sg] + [x[1] for x in qp]).astype(np.float32)
            offset = np.stack([og] + [x[2] for x in qp]).astype(np.float32)
            g_store, p_store = qg, [x[0] for x in qp]
        else:
            scale = np.ones((4, NCH), np.float32)
            offset = np.zeros((4, NCH), np.float32)
            g_store, p_store = grid, planes
        lo = np.array([gx, gy, 0], np.float32)
        hi = np.array([gx + f, gy + f, 1], np.float32)
        return BlockLod(ids[0][0], l, lo, hi, R, Rp, O, dtype, np.ascontiguousarray(g_store),
                        [np.ascontiguousarray(p) for p in p_store], scale, offset)

    # groups that fit the grid entirely (an incomplete group at the edge has no merged asset)
    jobs = [(l, gx, gy) for l in range(1, n_lods) for gy in range(0, nby - (1 << l) + 1, 1 << l)
            for gx in range(0, nbx - (1 << l) + 1, 1 << l)]
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(asset, jobs))


def c3q_scene(seed=2, lod_city=None):
    """The 8x8 city with quadtree LODs: the finest blocks of the LOD city
    (128^3 grid, 1024^2 planes, 16^3 occupancy per unit block) plus merged
    assets of 2x2 blocks (LOD 1: 64 texels per unit, 128 x 128 x 64 grid) and
    4x4 blocks (LOD 2: 32 per unit, 128 x 128 x 32), uint8.  lod_city: an
    already generated c3_scene(seed) whose finest level is reused."""
    if lod_city is not None:
        fine = [b for b in lod_city.blocks if b.lod == 0]
    else:
        fine = city_scene(8, seed, U8, (C3_LODS[0],)).blocks
    return Scene(8, 8, fine + merged_lods(fine, 8, 8, 3))


QUADTREE_THRESHOLDS = (2.0, 4.0)


def c5_scenes(seed=4, target_seed=5, lods=((128, 1024, 16),), nb=4):
    learn = city_scene(nb, seed, F32, lods)
    target = city_scene(nb, target_seed, F32, lods)
    return learn, target


def c5_views(seed=4, n=8, W=800, H=800, center=(2.0, 2.0)):
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
    views = []
    for _ in range(n):
        rad = rng.uniform(2.5, 3.5)
        ang = rng.uniform(0, 2 * math.pi)
        hh = rng.uniform(1.2, 2.0)
        pd = math.radians(rng.uniform(20.0, 45.0))
        dx, dy = rng.uniform(-0.5, 0.5, 2)
        eye = (center[0] + rad * math.cos(ang), center[1] + rad * math.sin(ang), hh)
        yaw = math.atan2(center[1] + dy - eye[1], center[0] + dx - eye[0])
        views.append(pinhole(W, H, eye, look_rotation(yaw_pitch_forward(yaw, pd))))
    return views


def contract_boundary(blocks):
    """The same entries with every unit block on the footprint's edge marked
    contracted (the implementation details' boundary blocks): their textures
    are then read as covering the contracted cube [-2, 2]^3 of the box, so
    the outer part of each texture holds the exterior (synthetic content,
    as for every block here)."""
    import dataclasses
    lo = np.min([b.aabb_min for b in blocks], axis=0)
    hi = np.max([b.aabb_max for b in blocks], axis=0)
    out = []
    for b in blocks:
        ext = np.asarray(b.aabb_max) - np.asarray(b.aabb_min)
        edge = (b.aabb_min[0] == lo[0] or b.aabb_max[0] == hi[0] or b.aabb_min[1] == lo[1] or b.aabb_max[1] == hi[1])
        unit = ext[0] == 1 and ext[1] == 1 and b.aabb_min[2] == lo[2] and b.aabb_max[2] == hi[2]
        out.append(dataclasses.replace(b, contracted=bool(edge and unit)))
    return out
