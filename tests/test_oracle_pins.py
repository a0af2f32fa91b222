"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code: closed forms, the
paper's equivalence theorem (Sec. 4.2 and Appendix A), library routines
(scipy interpolation, torch.nn layers), an independent numpy brute force, and
finite differences.  A plausible mistake in the oracle -- a dropped term, a
wrong sign, a transposed plane axis, an off-by-one in the sample window --
fails at least one of them.

Parity unpinned: only the absolute appearance of the synthetic scenes (their
recipe is a reading of the workload description, not a value the paper
prints).
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
from paper_2312_16457_amd import scenegen as sg


def axis_view(eye, forward):
    """1x1 image whose single ray is exactly `forward` (axis-aligned)."""
    return sg.View(1, 1, np.asarray(eye, np.float32), sg.look_rotation(forward), 1.0, 1.0, 0.5, 0.5)


def zero_mlp():
    return np.zeros(sg.MLP_NPARAM, np.float32)


def sig(x):
    return 1.0 / (1.0 + np.exp(-x))


def stored_constants(b):
    """(sigma, colour[3], feature[4]) that a homogeneous block really holds
    after its fp32 storage."""
    g = b.grid[0, 0, 0].astype(np.float64)
    return math.exp(g[0]), sig(g[1:4]), sig(g[4:8])


# ---------------------------------------------------------------------------
# P1: homogeneous block -> T = exp(-sigma d), C_d = (1 - T) c   (Eq. alpha)
# ---------------------------------------------------------------------------
def test_homogeneous_closed_form_axis_ray():
    b = sg.homogeneous_block(sigma=2.0)
    ob = O.OracleScene([b])
    occ = O.occupancy(ob, 0)
    assert occ.all()
    v = axis_view((-0.25, 0.5, 0.5), (1.0, 0.0, 0.0))
    r = O.render(ob, [occ], v, [0], sg.RenderParams(mode=1), zero_mlp())
    s, c, f = stored_constants(b)
    T = math.exp(-s * 1.0)  # chord length 1 = 512 steps of 1/512
    assert r["n_eval"][0] == 512
    assert abs(r["trans"][0] - T) < 1e-12
    np.testing.assert_allclose(r["aux"][0, :3], (1 - T) * c, atol=1e-12)
    np.testing.assert_allclose(r["aux"][0, 3:7], (1 - T) * f, atol=1e-12)
    # zero MLP -> sigmoid(0) = 1/2 added to the diffuse colour (Eq. deferred)
    np.testing.assert_allclose(r["rgb"][0], (1 - T) * c + 0.5, atol=1e-12)


def slab64(o, d, lo, hi):
    t0, t1 = 0.0, math.inf
    for a in range(3):
        if d[a] == 0:
            if not lo[a] <= o[a] <= hi[a]:
                return None
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return (t0, t1) if t0 < t1 else None


def test_homogeneous_closed_form_mode_a_oblique():
    b = sg.homogeneous_block(sigma=3.0)
    ob = O.OracleScene([b])
    occ = O.occupancy(ob, 0)
    v = sg.pinhole(16, 16, (1.7, -0.9, 1.4), sg.look_rotation(np.array([0.5, 0.5, 0.5]) - [1.7, -0.9, 1.4]))
    r = O.render(ob, [occ], v, [0], sg.RenderParams(mode=0, n_steps=128), zero_mlp())
    s, c, _ = stored_constants(b)
    pix = O.pixels_of(v)
    hits = 0
    for n, (i, j) in enumerate(pix):
        x = (i + 0.5 - v.cx) / v.fx
        y = (j + 0.5 - v.cy) / v.fy
        d = v.R.astype(np.float64) @ np.array([x, y, 1.0])
        d /= np.linalg.norm(d)
        h = slab64(v.eye.astype(np.float64), d, [0, 0, 0], [1, 1, 1])
        L = 0.0 if h is None else h[1] - h[0]
        T = math.exp(-s * L)
        hits += h is not None
        # fp32 chord endpoints: ~1e-7 relative error in the optical depth
        assert abs(r["trans"][n] - T) < 2e-6
        np.testing.assert_allclose(r["aux"][n, :3], (1 - r["trans"][n]) * c, atol=1e-12)
    assert hits > 50


# ---------------------------------------------------------------------------
# P2: blocks along a ray composite as Porter-Duff "over" (Eq. across blocks)
# ---------------------------------------------------------------------------
def test_over_closed_form_three_blocks():
    blocks = [sg.homogeneous_block(sigma=s, color=col, block_id=k, origin=(k, 0, 0))
              for k, (s, col) in enumerate([(1.0, (0.9, 0.1, 0.1)), (2.0, (0.1, 0.9, 0.1)),
                                            (0.5, (0.1, 0.1, 0.9))])]
    ob = O.OracleScene(blocks)
    occs = [O.occupancy(ob, k) for k in range(3)]
    v = axis_view((-0.25, 0.5, 0.5), (1.0, 0.0, 0.0))
    r = O.render(ob, occs, v, [2, 0, 1], sg.RenderParams(mode=1), zero_mlp())
    C = np.zeros(3)
    T = 1.0
    for b in blocks:
        s, c, _ = stored_constants(b)
        Tk = math.exp(-s)
        C += T * (1 - Tk) * c
        T *= Tk
    assert r["n_eval"][0] == 3 * 512
    assert abs(r["trans"][0] - T) < 1e-12
    np.testing.assert_allclose(r["aux"][0, :3], C, atol=1e-12)
    # the reversed merge is the classic occlusion error (Fig. 2a): it must differ
    rr = O.render(ob, occs, v, [2, 0, 1], sg.RenderParams(mode=1), zero_mlp(), composite=O.REVERSED)
    assert np.abs(rr["aux"][0, :3] - C).max() > 0.05


# ---------------------------------------------------------------------------
# P3: block-merged == monolithic (the paper's equivalence theorem, App. A)
# ---------------------------------------------------------------------------
def tiny_city(seed=11, nb=2, lods=((16, 32, 4),), dtype=sg.F32, shift=3.0, blobs=12):
    return sg.make_scene(nb, nb, lods, dtype, blobs_per_block=blobs, blob_z=(0.0, 0.4),
                         seed=seed, shift=shift)


def tiny_view(W=40, H=30, eye=(1.0, -1.2, 1.3), target=(1.0, 1.0, 0.2)):
    return sg.pinhole(W, H, eye, sg.look_rotation(np.asarray(target) - np.asarray(eye)))


@pytest.mark.parametrize("case", ["c1", "tiny_b", "tiny_u8_a"])
def test_merged_equals_monolithic(case):
    if case == "c1":
        scene, v, p = sg.c1_scene(), sg.c1_view(), sg.c1_params()
    elif case == "tiny_b":
        scene, v, p = tiny_city(), tiny_view(), sg.cityb_params()
    else:
        scene, v, p = tiny_city(dtype=sg.U8), tiny_view(), sg.RenderParams(mode=0, n_steps=64)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    w = sg.random_mlp(3)
    setv = list(range(ob.n))
    a = O.render(ob, occs, v, setv, p, w)
    b = O.render(ob, occs, v, setv, p, w, composite=O.MONOLITHIC)
    assert a["n_eval"].sum() > 1000
    np.testing.assert_allclose(a["aux"], b["aux"], atol=1e-12, rtol=0)
    np.testing.assert_allclose(a["rgb"], b["rgb"], atol=1e-12, rtol=0)


@pytest.fixture(scope="module")
def c2():
    scene = sg.c2_scene()
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    v = sg.c2_view()
    sel = O.select(v, scene.blocks, zt, thresholds=(1e30,), cull=True)
    return scene, ob, occs, zt, v, sel


def test_c2_equivalence_and_negative_controls(c2):
    """P3 on the 4x4-block 1080p workload (sampled rows) and P4: the paper's
    failure modes -- no depth sort, reversed order, alpha_i / sum alpha_j
    weights (Fig. 2a, Table 4) -- must differ by far more than 1e-4."""
    scene, ob, occs, zt, v, sel = c2
    pix = O.pixels_of(v, rows=np.arange(3, 1080, 97))
    w = sg.xavier_mlp(1)
    p = sg.cityb_params()
    a = O.render(ob, occs, v, sel, p, w, pix=pix)
    b = O.render(ob, occs, v, sel, p, w, pix=pix, composite=O.MONOLITHIC)
    np.testing.assert_allclose(a["rgb"], b["rgb"], atol=1e-12, rtol=0)
    # per-view xy-distance order == per-ray entry order on every sampled pixel
    assert a["order_ok"].all()
    for comp in (O.REVERSED, O.BY_ID, O.ALPHA_NORM):
        c = O.render(ob, occs, v, sel, p, w, pix=pix, composite=comp)
        assert np.abs(c["rgb"] - a["rgb"]).max() > 1e-2, comp


# ---------------------------------------------------------------------------
# P5: quadrature -- an independent numpy field + a 2^20-step integral
# ---------------------------------------------------------------------------
def decoded64(b):
    """Texture values in fp64: the uint8 decode q * scale + offset taken in
    double precision (the fp32 scale/offset are exact in fp64)."""
    if b.dtype == sg.F32:
        return b.grid.astype(np.float64), [p.astype(np.float64) for p in b.planes]
    s = b.scale.astype(np.float64)
    o = b.offset.astype(np.float64)
    return (b.grid * s[0] + o[0], [p * s[1 + i] + o[1 + i] for i, p in enumerate(b.planes)])


def np_field(b, pts):
    """Independent numpy evaluation of grid (trilinear) + planes (bilinear),
    cell-centred, clamp-to-edge, decoded values, summed ((G+XY)+XZ)+YZ."""
    grid, planes = decoded64(b)
    q = pts - b.aabb_min.astype(np.float64)

    def taps(x, R):
        u = x * R - 0.5
        i0 = np.floor(u)
        f = u - i0
        i0 = i0.astype(np.int64)
        return np.clip(i0, 0, R - 1), np.clip(i0 + 1, 0, R - 1), f

    R, Rp = b.grid_res, b.plane_res
    gx, gy, gz = (taps(q[:, a], R) for a in range(3))
    G = 0
    for wz, iz in ((1 - gz[2], gz[0]), (gz[2], gz[1])):
        for wy, iy in ((1 - gy[2], gy[0]), (gy[2], gy[1])):
            for wx, ix in ((1 - gx[2], gx[0]), (gx[2], gx[1])):
                G = G + (wz * wy * wx)[:, None] * grid[iz, iy, ix]
    px, py, pz = (taps(q[:, a], Rp) for a in range(3))

    def bil(P, tu, tv):
        out = 0
        for wv, iv in ((1 - tv[2], tv[0]), (tv[2], tv[1])):
            for wu, iu in ((1 - tu[2], tu[0]), (tu[2], tu[1])):
                out = out + (wv * wu)[:, None] * P[iv, iu]
        return out

    return ((G + bil(planes[0], px, py)) + bil(planes[1], px, pz)) + bil(planes[2], py, pz)


def test_field_against_scipy_and_numpy():
    from scipy.ndimage import map_coordinates
    scene = tiny_city(dtype=sg.U8)
    ob = O.OracleScene(scene.blocks)
    b = scene.blocks[3]
    rng = np.random.default_rng(0)
    pts = (b.aabb_min + rng.uniform(0, 1, (500, 3))).astype(np.float32)
    raw = O.field(ob, 3, pts)
    np.testing.assert_allclose(raw, np_field(b, pts.astype(np.float64)), atol=1e-12)
    grid, planes = decoded64(b)
    q = pts.astype(np.float64) - b.aabb_min
    R, Rp = b.grid_res, b.plane_res
    ref = np.zeros((500, 8))
    for ch in range(8):
        g = map_coordinates(grid[..., ch].astype(np.float64), [q[:, 2] * R - .5, q[:, 1] * R - .5,
                                                                q[:, 0] * R - .5], order=1, mode="nearest")
        xy = map_coordinates(planes[0][..., ch].astype(np.float64), [q[:, 1] * Rp - .5, q[:, 0] * Rp - .5],
                             order=1, mode="nearest")
        xz = map_coordinates(planes[1][..., ch].astype(np.float64), [q[:, 2] * Rp - .5, q[:, 0] * Rp - .5],
                             order=1, mode="nearest")
        yz = map_coordinates(planes[2][..., ch].astype(np.float64), [q[:, 2] * Rp - .5, q[:, 1] * Rp - .5],
                             order=1, mode="nearest")
        ref[:, ch] = ((g + xy) + xz) + yz
    np.testing.assert_allclose(raw, ref, atol=1e-9)


def test_linear_field_reproduced_exactly():
    """P6: a field linear in x, y, z stored at texel centres is reproduced in
    the interior [1/2R, 1 - 1/2R]."""
    R = 8
    b = sg.homogeneous_block(R=R, Rp=8)
    c = (np.arange(R) + 0.5) / R
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    b.grid[..., 2] = (0.75 * xx - 0.5 * yy + 0.25 * zz + 0.125).astype(np.float32)
    ob = O.OracleScene([b])
    rng = np.random.default_rng(1)
    pts = rng.uniform(0.5 / R, 1 - 0.5 / R, (300, 3)).astype(np.float32)
    raw = O.field(ob, 0, pts)
    p = pts.astype(np.float64)
    np.testing.assert_allclose(raw[:, 2], 0.75 * p[:, 0] - 0.5 * p[:, 1] + 0.25 * p[:, 2] + 0.125, atol=1e-6)


@pytest.mark.parametrize("plane", [0, 1, 2])
def test_plane_impulse_axes(plane):
    """P6: a single-texel impulse in plane xy / xz / yz (index [v][u]) appears
    exactly at the texel centre and vanishes one texel away along u and v,
    whatever the third coordinate is."""
    Rp = 16
    b = sg.homogeneous_block(R=4, Rp=Rp)
    b.grid[...] = 0
    u0, v0 = 5, 11
    b.planes[plane][v0, u0, 3] = 1.0
    ob = O.OracleScene([b])
    axes = [(0, 1), (0, 2), (1, 2)][plane]
    third = ({0, 1, 2} - set(axes)).pop()
    rng = np.random.default_rng(plane)
    for _ in range(20):
        p = np.zeros(3, np.float32)
        p[axes[0]] = (u0 + 0.5) / Rp
        p[axes[1]] = (v0 + 0.5) / Rp
        p[third] = rng.uniform(0, 1)
        assert abs(O.field(ob, 0, p[None])[0, 3] - 1.0) < 1e-12
        q = p.copy()
        q[axes[0]] = (u0 + 1.5) / Rp
        assert abs(O.field(ob, 0, q[None])[0, 3]) < 1e-12
        q = p.copy()
        q[axes[1]] = (v0 - 1 + 0.5) / Rp
        assert abs(O.field(ob, 0, q[None])[0, 3]) < 1e-12
        assert abs(O.field(ob, 0, p[None])[0, 2]) < 1e-12  # other channels untouched


def brute_ray(blocks, o, d, t0, t1, n):
    """Continuous volume-rendering integral of the block field along a ray,
    midpoint rule with n steps between t0 and t1 (fp64, numpy)."""
    dt = (t1 - t0) / n
    A = np.zeros(7)
    T = 1.0
    chunk = 1 << 16
    for s in range(0, n, chunk):
        t = t0 + (np.arange(s, min(n, s + chunk)) + 0.5) * dt
        p = o[None, :] + t[:, None] * d[None, :]
        sigma = np.zeros(len(t))
        v = np.zeros((len(t), 7))
        for b in blocks:
            m = np.all((p >= b.aabb_min) & (p < b.aabb_max), axis=1)
            if m.any():
                raw = np_field(b, p[m])
                sigma[m] = np.exp(raw[:, 0])
                v[m] = sig(raw[:, 1:])
        tau = sigma * dt
        Tin = T * np.exp(-np.concatenate([[0.0], np.cumsum(tau)[:-1]]))
        w = Tin * -np.expm1(-tau)
        A += (w[:, None] * v).sum(0)
        T = Tin[-1] * math.exp(-tau[-1])
    return A, T


def test_quadrature_converges_and_discrete_sum_exact():
    """P5: occupancy forced to 1 (continuous field), axis-aligned rays whose
    block faces fall on step boundaries.  The renderer converges to the
    continuous integral at second order and the discrete sum equals an
    independent numpy evaluation of the same samples to 1e-12."""
    scene = tiny_city(nb=2, lods=((4, 8, 4),), shift=1.0, blobs=6, seed=5)
    ob = O.OracleScene(scene.blocks)
    ones = [np.ones((4, 4, 4), np.uint8) for _ in range(ob.n)]
    w = zero_mlp()
    rays = [((-0.25, 0.3, 0.2), (1, 0, 0)), ((-0.25, 1.7, 0.1), (1, 0, 0)), ((0.6, -0.25, 0.15), (0, 1, 0))]
    for eye, fwd in rays:
        v = axis_view(eye, fwd)
        o = np.asarray(eye, np.float32).astype(np.float64)
        d = np.asarray(fwd, np.float64)
        h = slab64(o, d, [0, 0, 0], [2, 2, 1])
        A_ref, T_ref = brute_ray(scene.blocks, o, d, h[0], h[1], 1 << 20)
        errs = []
        for inv in (64, 128, 256, 512, 1024):
            p = sg.RenderParams(mode=1, delta=1.0 / inv, max_steps=1 << 20)
            r = O.render(ob, ones, v, list(range(ob.n)), p, w)
            errs.append(max(abs(r["trans"][0] - T_ref), np.abs(r["aux"][0, :7] - A_ref).max()))
            if inv == 256:
                # exact enumeration of the discrete sum at the same sample points
                ks = np.arange(int(round(h[0] * inv)), int(round(h[1] * inv)))
                t = (ks + 0.5) / inv
                pts = o[None] + t[:, None] * d[None]
                A = np.zeros(7)
                T = 1.0
                for pt in pts:
                    b = next(b for b in scene.blocks if np.all((pt >= b.aabb_min) & (pt < b.aabb_max)))
                    raw = np_field(b, pt[None])[0]
                    a = -math.expm1(-math.exp(raw[0]) / inv)
                    A += T * a * sig(raw[1:])
                    T *= 1 - a
                assert abs(r["trans"][0] - T) < 1e-12
                np.testing.assert_allclose(r["aux"][0, :7], A, atol=1e-12)
        errs = np.array(errs)
        order = np.log2(errs[:-1] / errs[1:])
        assert errs[-1] < 1e-4, errs
        assert order.mean() > 1.5, (errs, order)


# ---------------------------------------------------------------------------
# P7: MLP against torch.nn in fp64
# ---------------------------------------------------------------------------
def test_mlp_against_torch():
    import torch
    w = sg.random_mlp(7, scale=0.8).astype(np.float64)
    net = torch.nn.Sequential(torch.nn.Linear(10, 16), torch.nn.ReLU(), torch.nn.Linear(16, 16),
                              torch.nn.ReLU(), torch.nn.Linear(16, 3), torch.nn.Sigmoid()).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.tensor(w[0:160].reshape(16, 10)))
        net[0].bias.copy_(torch.tensor(w[160:176]))
        net[2].weight.copy_(torch.tensor(w[176:432].reshape(16, 16)))
        net[2].bias.copy_(torch.tensor(w[432:448]))
        net[4].weight.copy_(torch.tensor(w[448:496].reshape(3, 16)))
        net[4].bias.copy_(torch.tensor(w[496:499]))
    rng = np.random.default_rng(0)
    for _ in range(50):
        x = rng.uniform(-1, 1, 10)
        ref = net(torch.tensor(x)[None]).detach().numpy()[0]
        np.testing.assert_allclose(O.mlp(w, x), ref, atol=1e-14)
    w2 = w.copy()
    w2[448:496] = 0
    np.testing.assert_allclose(O.mlp(w2, rng.uniform(-1, 1, 10)), sig(w[496:499]), atol=1e-15)


# ---------------------------------------------------------------------------
# P8: occupancy soundness -- density <= 0.01 everywhere in an empty cell
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [sg.F32, sg.U8])
def test_occupancy_sound(dtype):
    scene = sg.make_scene(1, 1, ((32, 64, 8),), dtype, blobs_per_block=6, blob_z=(0.0, 0.3), seed=9)
    ob = O.OracleScene(scene.blocks)
    occ = O.occupancy(ob, 0)
    assert 0 < occ.mean() < 1
    n = 17
    g = (np.arange(n) / (n - 1)) * (1 - 1e-7)
    worst = -np.inf
    for cz, cy, cx in zip(*np.nonzero(occ == 0)):
        zz, yy, xx = np.meshgrid((cz + g) / 8, (cy + g) / 8, (cx + g) / 8, indexing="ij")
        pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.float32)
        worst = max(worst, O.field(ob, 0, pts)[:, 0].max())
    assert math.exp(worst) <= 0.01
    # and the rule is not vacuous: some occupied cell does exceed 0.01
    cz, cy, cx = np.argwhere(occ == 1)[0]
    zz, yy, xx = np.meshgrid((cz + g) / 8, (cy + g) / 8, (cx + g) / 8, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.float32)
    assert occ.sum() > 0 and np.exp(O.field(ob, 0, pts)[:, 0]).max() > 0


def test_occupancy_skip_changes_little():
    """Samples skipped in empty cells carry density <= 0.01: the render with
    the occupancy mask stays within 1 - exp(-0.01 * chord) of the unmasked one."""
    scene = sg.make_scene(1, 1, ((32, 64, 8),), sg.F32, blobs_per_block=6, blob_z=(0.0, 0.3), seed=9)
    ob = O.OracleScene(scene.blocks)
    occ = O.occupancy(ob, 0)
    v = tiny_view(24, 24, eye=(0.5, -1.0, 1.0), target=(0.5, 0.5, 0.2))
    w = zero_mlp()
    a = O.render(ob, [occ], v, [0], sg.cityb_params(), w)
    b = O.render(ob, [np.ones_like(occ)], v, [0], sg.cityb_params(), w)
    assert np.abs(a["trans"] - b["trans"]).max() <= 1 - math.exp(-0.01 * math.sqrt(3))


# ---------------------------------------------------------------------------
# P8 (exact rule): the occupancy bit is the max-bound of the density over the
# cell's interpolation support (Sec. 4.5 "Baking", read as a conservative
# bound), recomputed here in numpy from the definition alone
# ---------------------------------------------------------------------------
THRESH32 = np.float32(math.log(0.01))


def np_occupancy(b):
    """Per axis a cell c reads the texel indices [c s - 1, (c + 1) s] (clamped
    to the texture), s = texels per cell; bound = ((max G + max XY) + max XZ) +
    max YZ over the density channel in fp32, each uint8 texel decoded as
    fl(fl(q s) + o); the cell is occupied iff bound > fl32(ln 0.01)."""
    ext = [int(round(float(b.aabb_max[a] - b.aabb_min[a]))) for a in range(3)]

    def ch0(arr, t):
        v = arr[..., 0]
        if b.dtype == sg.U8:
            return v.astype(np.float32) * np.float32(b.scale[t, 0]) + np.float32(b.offset[t, 0])
        return v.astype(np.float32)

    g = ch0(b.grid, 0)
    pl = [ch0(p, 1 + i) for i, p in enumerate(b.planes)]
    C = [b.occ_res * e for e in ext]  # cells along x, y, z
    s, sp = b.grid_res // b.occ_res, b.plane_res // b.occ_res

    def rng(c, step, n):
        return max(c * step - 1, 0), min((c + 1) * step, n - 1) + 1

    out = np.zeros((C[2], C[1], C[0]), np.uint8)
    for cz in range(C[2]):
        for cy in range(C[1]):
            for cx in range(C[0]):
                c = (cx, cy, cz)
                gr = [rng(c[a], s, g.shape[2 - a]) for a in range(3)]
                mg = g[gr[2][0]:gr[2][1], gr[1][0]:gr[1][1], gr[0][0]:gr[0][1]].max()
                # planes indexed [v][u]: xy (u=x, v=y), xz (u=x, v=z), yz (u=y, v=z)
                m = []
                for p, (au, av) in zip(pl, ((0, 1), (0, 2), (1, 2))):
                    u0, u1 = rng(c[au], sp, p.shape[1])
                    v0, v1 = rng(c[av], sp, p.shape[0])
                    m.append(p[v0:v1, u0:u1].max())
                bound = np.float32(np.float32(np.float32(mg + m[0]) + m[1]) + m[2])
                out[cz, cy, cx] = 1 if bound > THRESH32 else 0
    return out


@pytest.mark.parametrize("kind", ["f32", "u8", "merged_u8", "merged_f32"])
def test_occupancy_exact_rule_against_numpy(kind):
    if kind.startswith("merged"):
        dt = sg.U8 if kind.endswith("u8") else sg.F32
        fine = sg.make_scene(2, 2, ((32, 64, 8),), dt, blobs_per_block=3, blob_z=(0.0, 0.3), blob_s=(0.03, 0.08),
                             seed=5).blocks
        blocks = sg.merged_lods(fine, 2, 2, 2, dtype=dt)
        b = [x for x in blocks if x.lod == 1][0]
    else:
        dt = sg.F32 if kind == "f32" else sg.U8
        b = sg.make_scene(1, 1, ((32, 64, 8),), dt, blobs_per_block=6, blob_z=(0.0, 0.5), seed=13).blocks[0]
    ob = O.OracleScene([b])
    occ = O.occupancy(ob, 0)
    ref = np_occupancy(b)
    assert 0.05 < ref.mean() < 0.95  # both states present, so the comparison has teeth
    assert np.array_equal(occ, ref)


def test_occupancy_support_range_and_strict_threshold():
    """Impulses place the texel range exactly: grid texel i along x (s = 4
    texels per cell) is read by the cells c with 4c - 1 <= i <= 4c + 4, so
    texel 5 by cell 1 alone and texels 3, 4, 7, 8 by two cells; a range
    grown or shrunk by one texel fails.  A bound equal to fl32(ln 0.01) is
    empty and the next float up is occupied (strict >)."""
    R, Rp, Oc = 32, 32, 8
    lo = np.zeros(3, np.float32)

    def block(grid0, plane0=0.0):
        grid = np.zeros((R, R, R, 8), np.float32)
        grid[..., 0] = grid0
        planes = [np.zeros((Rp, Rp, 8), np.float32) for _ in range(3)]
        for p in planes:
            p[..., 0] = plane0
        return sg.BlockLod(0, 0, lo, lo + 1, R, Rp, Oc, sg.F32, grid, planes,
                           np.ones((4, 8), np.float32), np.zeros((4, 8), np.float32))

    expect = {3: {0, 1}, 4: {0, 1}, 5: {1}, 7: {1, 2}, 8: {1, 2}, 0: {0}, 31: {7}}
    for i, cells in expect.items():
        g = np.full((R, R, R), -20.0, np.float32)
        g[12, 17, i] = 5.0  # z = 12 (cells 2 and 3), y = 17 (cell 4 alone), x = i
        occ = O.occupancy(O.OracleScene([block(g)]), 0)
        hit = set(np.nonzero(occ.any(axis=(0, 1)))[0].tolist())
        assert hit == cells, (i, hit)
        assert set(np.nonzero(occ.any(axis=(0, 2)))[0].tolist()) == {4}
        assert set(np.nonzero(occ.any(axis=(1, 2)))[0].tolist()) == {2, 3}
    # strict threshold
    edge = O.occupancy(O.OracleScene([block(THRESH32)]), 0)
    assert not edge.any()
    g = np.full((R, R, R), THRESH32, np.float32)
    g[0, 0, 0] = np.nextafter(THRESH32, np.float32(1))
    up = O.occupancy(O.OracleScene([block(g)]), 0)
    assert up.sum() == 1 and up[0, 0, 0] == 1
    # the four textures add: a plane value lifts every cell over the threshold
    assert O.occupancy(O.OracleScene([block(np.full((R, R, R), THRESH32, np.float32), 1e-3)]), 0).all()


# ---------------------------------------------------------------------------
# z_top (Appendix D: the height of a block's content, which sets its LOD
# distance and its culling box): the top face of the highest occupied cell
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ext_z,O_res", [(1, 8), (1, 16), (2, 2)])
def test_ztop_closed_form(ext_z, O_res):
    rng = np.random.default_rng(ext_z * 31 + O_res)
    lo = np.array([3.0, -2.0, 0.0], np.float32)
    hi = lo + np.array([1.0, 1.0, float(ext_z)], np.float32)
    R = 2 * O_res
    b = sg.BlockLod(0, 0, lo, hi, R, R, O_res, sg.F32, np.zeros((R * ext_z, R, R, 8), np.float32),
                    [np.zeros((R, R, 8), np.float32), np.zeros((R * ext_z, R, 8), np.float32),
                     np.zeros((R * ext_z, R, 8), np.float32)],
                    np.ones((4, 8), np.float32), np.zeros((4, 8), np.float32))
    ob = O.OracleScene([b])
    nz = O_res * ext_z
    shape = (nz, O_res, O_res)
    assert O.ztop(ob, 0, np.zeros(shape, np.uint8)) == float(lo[2])  # empty: the floor
    for _ in range(6):
        occ = np.zeros(shape, np.uint8)
        k = int(rng.integers(nz))
        occ[k, rng.integers(O_res), rng.integers(O_res)] = 1
        below = int(rng.integers(k + 1))  # cells below the top change nothing
        occ[below, rng.integers(O_res), rng.integers(O_res)] = 1
        assert O.ztop(ob, 0, occ) == float(lo[2]) + (k + 1) / nz * ext_z
    # a contracted block's texture z is not world z: its top is its box's top
    bc = dataclasses.replace(b, contracted=True)
    occ = np.zeros(shape, np.uint8)
    occ[0, 0, 0] = 1
    assert O.ztop(O.OracleScene([bc]), 0, occ) == float(hi[2])


# ---------------------------------------------------------------------------
# P10/P11: selection -- culling is conservative, per-view order == per-ray order
# ---------------------------------------------------------------------------
def test_culling_conservative_and_order_on_lod_scene():
    lods = ((16, 32, 8), (8, 16, 4), (4, 8, 2))
    scene = sg.make_scene(6, 6, lods, sg.U8, blobs_per_block=8, blob_z=(0.0, 0.3), seed=21)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    views = sg.aerial_views(8, 6, [(48, 32)], xy=(0.5, 5.5), h=(1.5, 4.0))
    w = sg.xavier_mlp(2)
    thr = (1.5, 3.0, 6.0)
    n_culled = 0
    for v in views:
        sel = O.select(v, scene.blocks, zt, thresholds=thr, cull=True)
        allb = O.select(v, scene.blocks, zt, thresholds=thr, cull=False)
        assert set(sel) <= set(allb)
        n_culled += len(allb) - len(sel)
        a = O.render(ob, occs, v, sel, sg.cityb_params(), w)
        b = O.render(ob, occs, v, allb, sg.cityb_params(), w)
        assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["trans"], b["trans"])
        assert a["order_ok"].all()
        # LOD rule: distance to (centre_xy, z_top of the finest level)
        for k in sel:
            e = scene.blocks[k]
            k0 = ob.index(e.block_id, 0)
            c = np.array([(e.aabb_min[0] + e.aabb_max[0]) / 2, (e.aabb_min[1] + e.aabb_max[1]) / 2, zt[k0]])
            dist = np.linalg.norm(v.eye.astype(np.float64) - c)
            assert e.lod == next(l for l, t in enumerate(thr) if dist < t)
        # order: nondecreasing xy distance
        dxy = [np.hypot(v.eye[0] - (scene.blocks[k].aabb_min[0] + .5), v.eye[1] - (scene.blocks[k].aabb_min[1] + .5))
               for k in sel]
        assert all(dxy[i] <= dxy[i + 1] for i in range(len(dxy) - 1))
    assert n_culled > 0


# ---------------------------------------------------------------------------
# P13: fp64 adjoint vs central finite differences
# ---------------------------------------------------------------------------
def kink_free_mlp(seed):
    """Weights whose ReLU pre-activations stay > 0 for inputs in [0, 1]^10 and
    unit directions, so central differences never straddle a kink."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-0.3, 0.3, (16, 10))
    b1 = np.full(16, 4.0)
    W2 = rng.uniform(-0.05, 0.05, (16, 16))
    b2 = np.full(16, 7.0)
    W3 = rng.uniform(-0.02, 0.02, (3, 16))
    b3 = rng.uniform(-0.5, 0.5, 3)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def test_adjoint_matches_finite_differences():
    scene = tiny_city(nb=2, lods=((8, 16, 4),), shift=1.5, blobs=8, seed=13)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    v = tiny_view(12, 10, eye=(1.0, -0.8, 1.1), target=(1.0, 1.0, 0.15))
    p = sg.RenderParams(mode=1, delta=1.0 / 128, max_steps=4096)
    w = kink_free_mlp(3)
    setv = list(range(ob.n))
    pix = O.pixels_of(v)
    target = np.random.default_rng(4).uniform(0, 1, (len(pix), 3))

    def loss():
        r = O.render(ob, occs, v, setv, p, w, pix=pix)
        return np.mean((r["rgb"] - target) ** 2), r

    L0, r0 = loss()
    g_rgb = 2 * (r0["rgb"] - target) / target.size
    g_tr = np.random.default_rng(5).uniform(-0.1, 0.1, len(pix))
    grads, gm = O.adjoint(ob, occs, v, setv, p, w, pix, g_rgb)
    gmax = max(max(np.abs(g).max(), max(np.abs(q).max() for q in ps)) for g, ps in grads.values())
    assert gmax > 0
    rng = np.random.default_rng(6)
    h = 1e-3
    checked = 0
    picks = []
    for k, (g, ps) in grads.items():
        for arr_i, arr in enumerate([g] + ps):
            nz = np.argwhere(np.abs(arr) > 1e-3 * gmax)
            for _ in range(3 if arr_i == 0 else 1):
                picks.append((k, arr_i, tuple(nz[rng.integers(len(nz))])))
    for k, arr_i, idx in picks:
        fg, fps = ob.f64[k]
        arr = fg if arr_i == 0 else fps[arr_i - 1]
        ga = (grads[k][0] if arr_i == 0 else grads[k][1][arr_i - 1])[idx]
        old = arr[idx]
        arr[idx] = old + h
        Lp, _ = loss()
        arr[idx] = old - h
        Lm, _ = loss()
        arr[idx] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(ga - fd) <= 1e-4 * abs(fd) + 1e-6 * gmax, (k, arr_i, idx, ga, fd)
        checked += 1
    for i in rng.choice(499, 16, replace=False):
        old = w[i]
        w[i] = old + h
        Lp, _ = loss()
        w[i] = old - h
        Lm, _ = loss()
        w[i] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(gm[i] - fd) <= 1e-4 * abs(fd) + 1e-8, (i, gm[i], fd)
        checked += 1
    assert checked >= 40

    # transmittance output: L = sum g_tr * T  ->  dL/dtheta through T alone
    grads_t, _ = O.adjoint(ob, occs, v, setv, p, w, pix, np.zeros_like(g_rgb), g_tr)
    k = next(iter(grads_t))
    g = grads_t[k][0]
    idx = tuple(np.argwhere(np.abs(g) > 1e-3 * np.abs(g).max())[0])
    arr = ob.f64[k][0]
    old = arr[idx]
    arr[idx] = old + h
    Tp = O.render(ob, occs, v, setv, p, w, pix=pix)["trans"]
    arr[idx] = old - h
    Tm = O.render(ob, occs, v, setv, p, w, pix=pix)["trans"]
    arr[idx] = old
    fd = np.sum(g_tr * (Tp - Tm)) / (2 * h)
    assert abs(g[idx] - fd) <= 1e-4 * abs(fd) + 1e-9


def test_contracted_adjoint_matches_finite_differences():
    """P13 over contracted boundary blocks (implementation details, the
    contraction equation): the exterior samples, each with its own step and
    read through the contraction, join the single-chain adjoint in ray order.
    Central differences of the loss agree with the fp64 adjoint on texels
    that only the exterior's samples reach and on texels of the blocks' own
    samples, with dL/dT included."""
    scene = tiny_city(nb=2, lods=((8, 16, 4),), shift=1.5, blobs=8, seed=13)
    blocks = sg.contract_boundary(scene.blocks)
    assert all(b.contracted for b in blocks)
    ob = O.OracleScene(blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    v = tiny_view(12, 10, eye=(1.0, -1.5, 1.0), target=(1.0, 1.0, 0.15))
    p = sg.RenderParams(mode=1, delta=1.0 / 128, max_steps=4096, ext_delta=1.0 / 32, ext_max_steps=128)
    p0 = sg.RenderParams(mode=1, delta=1.0 / 128, max_steps=4096)
    w = kink_free_mlp(3)
    setv = list(range(ob.n))
    pix = O.pixels_of(v)
    target = np.random.default_rng(4).uniform(0, 1, (len(pix), 3))
    g_tr = np.random.default_rng(5).uniform(-0.1, 0.1, len(pix))

    def loss():
        r = O.render(ob, occs, v, setv, p, w, pix=pix)
        return np.mean((r["rgb"] - target) ** 2) + np.sum(g_tr * r["trans"]), r

    L0, r0 = loss()
    g_rgb = 2 * (r0["rgb"] - target) / target.size
    grads, gm = O.adjoint(ob, occs, v, setv, p, w, pix, g_rgb, g_tr)
    grads0, _ = O.adjoint(ob, occs, v, setv, p0, w, pix, g_rgb, g_tr)
    gmax = max(max(np.abs(g).max(), max(np.abs(q).max() for q in ps)) for g, ps in grads.values())
    assert gmax > 0
    rng = np.random.default_rng(6)
    h = 1e-3
    picks = []
    n_ext = 0
    for k, (g, ps) in grads.items():
        for arr_i, arr in enumerate([g] + ps):
            arr0 = grads0[k][0] if arr_i == 0 else grads0[k][1][arr_i - 1]
            big = np.abs(arr) > 1e-3 * gmax
            ext_only = np.argwhere(big & (arr0 == 0))  # reached by exterior samples alone
            own = np.argwhere(big & (arr0 != 0))
            if len(ext_only):
                picks.append((k, arr_i, tuple(ext_only[rng.integers(len(ext_only))])))
                n_ext += 1
            if len(own):
                picks.append((k, arr_i, tuple(own[rng.integers(len(own))])))
    assert n_ext >= 8, n_ext
    for k, arr_i, idx in picks:
        fg, fps = ob.f64[k]
        arr = fg if arr_i == 0 else fps[arr_i - 1]
        ga = (grads[k][0] if arr_i == 0 else grads[k][1][arr_i - 1])[idx]
        old = arr[idx]
        arr[idx] = old + h
        Lp, _ = loss()
        arr[idx] = old - h
        Lm, _ = loss()
        arr[idx] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(ga - fd) <= 1e-4 * abs(fd) + 1e-6 * gmax, (k, arr_i, idx, ga, fd)
    for i in rng.choice(499, 8, replace=False):
        old = w[i]
        w[i] = old + h
        Lp, _ = loss()
        w[i] = old - h
        Lm, _ = loss()
        w[i] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(gm[i] - fd) <= 1e-4 * abs(fd) + 1e-8, (i, gm[i], fd)
    # the opacity term and per-block MLPs are not defined over contracted blocks
    with pytest.raises(ValueError):
        O.adjoint(ob, occs, v, setv, p, w, pix, g_rgb, g_tr, w_opacity=np.ones(len(pix)))
    with pytest.raises(ValueError):
        O.adjoint_block_mlp(ob, occs, v, setv, p, [w] * ob.n, pix, g_rgb)


def test_sparsity_over_contracted_blocks():
    """The sparsity term over contracted blocks (Sec. 4.3 sparsity loss; the
    contraction equation): a point in a contracted block's box reads the
    block's textures at the contracted coordinate.  Independently: q from the
    fp64 contraction (pinned by P22), the field by numpy interpolation at q,
    alpha = 1 - exp(-exp(raw_0) delta) in occupied cells; points outside every
    box take zero."""
    scene = tiny_city(nb=2, lods=((8, 16, 4),), shift=1.0, blobs=8, seed=29)
    blocks = sg.contract_boundary(scene.blocks)
    assert all(b.contracted for b in blocks)
    ob = O.OracleScene(blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    rng = np.random.default_rng(31)
    pts = np.concatenate([rng.uniform(0, 2, (3000, 2)), rng.uniform(0, 1, (3000, 1))], 1).astype(np.float32)
    pts = np.concatenate([pts, np.array([[2.5, 0.5, 0.5], [0.5, -0.1, 0.5], [0.5, 0.5, 1.2]], np.float32)])
    delta = 1.0 / 64
    _, _, a = O.sparsity(ob, occs, list(range(ob.n)), pts, delta, 1.0, want_alpha=True, want_grad=False)
    assert (a[-3:] == 0).all()
    want = np.zeros(len(pts) - 3)
    occupied = np.zeros(len(pts) - 3, bool)
    for k, b in enumerate(blocks):
        lo, hi = np.asarray(b.aabb_min, np.float64), np.asarray(b.aabb_max, np.float64)
        p64 = pts[:-3].astype(np.float64)
        sel = np.all((p64 >= lo) & (p64 < hi), axis=1)
        x = (p64[sel] - (lo + hi) / 2) * 2 / (hi - lo)
        q = (np.array([O.contract(xi) for xi in x]) + 2) * (hi - lo) / 4
        raw = np_field(b, lo + q)
        O_ = b.occ_res
        cell = np.clip(np.floor(q * O_).astype(np.int64), 0, O_ - 1)
        occ = occs[k].reshape(O_, O_, O_)[cell[:, 2], cell[:, 1], cell[:, 0]] != 0
        want[sel] = np.where(occ, -np.expm1(-np.exp(raw[:, 0]) * delta), 0.0)
        occupied[sel] = occ
    got = a[:-3]
    same = (got != 0) == occupied
    assert same.mean() > 0.995, same.mean()  # cell decisions: fp32 here, fp64 in the check
    assert occupied.sum() > 1000
    assert np.abs(got - want)[same].max() <= 1e-5


# ---------------------------------------------------------------------------
# Early ray termination: the ray stops after the first evaluated sample whose
# transmittance is below t_min; what it skips is bounded by that transmittance
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [0, 1])
def test_early_termination_bound_and_equivalence(mode):
    scene = tiny_city(shift=0.0, blobs=12, seed=17)  # opaque variant
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    v = tiny_view()
    w = sg.random_mlp(3)
    setv = list(range(ob.n))
    base = sg.RenderParams(mode=1) if mode == 1 else sg.RenderParams(mode=0, n_steps=96)
    full = O.render(ob, occs, v, setv, base, w)
    t_min = 1e-3
    p = sg.RenderParams(mode=base.mode, n_steps=base.n_steps, t_min=t_min)
    term = O.render(ob, occs, v, setv, p, w)
    mono = O.render(ob, occs, v, setv, p, w, composite=O.MONOLITHIC)
    stopped = term["n_eval"] < full["n_eval"]
    assert stopped.sum() > 50
    # merged and monolithic composites stop at the same sample
    assert np.array_equal(term["n_eval"], mono["n_eval"])
    np.testing.assert_allclose(term["aux"], mono["aux"], atol=1e-12)
    # a stopped ray ended below t_min; the skipped remainder is at most its T
    assert (term["trans"][stopped] < t_min).all()
    assert (term["trans"][~stopped] == full["trans"][~stopped]).all()
    gap = np.abs(term["aux"][:, :7] - full["aux"][:, :7]).max(axis=1)
    assert (gap <= term["trans"] + 1e-12).all()
    # the stopping sample is the first below t_min: a threshold just under the
    # final T of a stopped ray would have stopped it no later
    lower = sg.RenderParams(mode=base.mode, n_steps=base.n_steps, t_min=t_min / 4)
    later = O.render(ob, occs, v, setv, lower, w)
    assert (later["n_eval"] >= term["n_eval"]).all() and (later["n_eval"] <= full["n_eval"]).all()


# ---------------------------------------------------------------------------
# Regularisers (Sec. 4.3): the opacity loss of homogeneous blocks is the
# binary entropy of exp(-sigma L); its gradient and the sparsity loss's match
# finite differences; the sparsity loss of a homogeneous block is 1 - exp(-sigma delta)
# ---------------------------------------------------------------------------
def bernoulli_entropy(a):
    from scipy.special import entr
    return float(entr(a) + entr(1.0 - a))


def test_opacity_closed_form_three_blocks():
    sigmas = [0.7, 2.0, 30.0]  # the last is fully opaque: its entropy is the clamp's
    blocks = [sg.homogeneous_block(sigma=s, block_id=k, origin=(k, 0, 0)) for k, s in enumerate(sigmas)]
    ob = O.OracleScene(blocks)
    occs = [O.occupancy(ob, k) for k in range(3)]
    v = axis_view((-0.25, 0.5, 0.5), (1.0, 0.0, 0.0))
    L = O.opacity(ob, occs, v, [0, 1, 2], sg.RenderParams(mode=1), O.pixels_of(v))[0]
    want = 0.0
    for b in blocks:
        s, _, _ = stored_constants(b)
        a = 1.0 - math.exp(-s)  # chord 1
        want += bernoulli_entropy(min(max(a, 1e-6), 1 - 1e-6))
    assert abs(L - want) < 1e-12
    # the entropy vanishes only at the clamp: an opaque block contributes ~1.5e-5
    assert bernoulli_entropy(1 - 1e-6) < 2e-5 and L > bernoulli_entropy(1 - math.exp(-0.7))


def test_opacity_gradient_matches_finite_differences():
    scene = tiny_city(nb=2, lods=((8, 16, 4),), shift=0.5, blobs=8, seed=21)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    v = tiny_view(10, 8, eye=(1.0, -0.8, 1.1), target=(1.0, 1.0, 0.15))
    p = sg.RenderParams(mode=1, delta=1.0 / 128, max_steps=4096)
    w = kink_free_mlp(3)
    setv = list(range(ob.n))
    pix = O.pixels_of(v)
    wo = np.random.default_rng(7).uniform(0.5, 1.5, len(pix))
    L0 = O.opacity(ob, occs, v, setv, p, pix)
    assert (L0 > 0.05).sum() > 10  # semi-transparent blocks are present
    grads, gm = O.adjoint(ob, occs, v, setv, p, w, pix, np.zeros((len(pix), 3)), None, wo)
    assert not gm.any()  # the opacity loss does not touch the MLP
    gmax = max(np.abs(g).max() for g, _ in grads.values())
    rng = np.random.default_rng(8)
    h = 1e-4
    checked = 0
    for k, (g, ps) in grads.items():
        for arr_i, arr_g in enumerate([g] + ps):
            nz = np.argwhere(np.abs(arr_g) > 1e-3 * gmax)
            if len(nz) == 0:
                continue
            assert not np.abs(arr_g[..., 1:]).any()  # density channel only
            for _ in range(2):
                idx = tuple(nz[rng.integers(len(nz))])
                fg, fps = ob.f64[k]
                arr = fg if arr_i == 0 else fps[arr_i - 1]
                old = arr[idx]
                arr[idx] = old + h
                Lp = np.sum(wo * O.opacity(ob, occs, v, setv, p, pix))
                arr[idx] = old - h
                Lm = np.sum(wo * O.opacity(ob, occs, v, setv, p, pix))
                arr[idx] = old
                fd = (Lp - Lm) / (2 * h)
                assert abs(arr_g[idx] - fd) <= 1e-4 * abs(fd) + 1e-6 * gmax, (k, arr_i, idx, arr_g[idx], fd)
                checked += 1
    assert checked >= 12


def test_sparsity_closed_form_and_gradient():
    b = sg.homogeneous_block(sigma=5.0)
    ob = O.OracleScene([b])
    occ = O.occupancy(ob, 0)
    rng = np.random.default_rng(9)
    inside = rng.uniform(0.0, 1.0, (300, 3)).astype(np.float32)
    outside = rng.uniform(1.0, 2.0, (100, 3)).astype(np.float32)
    pts = np.concatenate([inside, outside])
    delta = 1.0 / 512
    L, _ = O.sparsity(ob, [occ], [0], pts, delta, weight=2.0)
    s, _, _ = stored_constants(b)
    assert abs(L - 2.0 * 300 / 400 * -math.expm1(-s * delta)) < 1e-15
    # gradient against finite differences on a textured scene
    scene = tiny_city(nb=2, lods=((8, 16, 4),), shift=0.5, blobs=8, seed=23)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    pts = np.concatenate([rng.uniform(0, 2, (2000, 2)), rng.uniform(0, 1, (2000, 1))], 1).astype(np.float32)
    setv = list(range(ob.n))
    L, grads = O.sparsity(ob, occs, setv, pts, 1.0 / 64, weight=1.0)
    assert L > 0
    gmax = max(max(np.abs(g).max(), max(np.abs(q).max() for q in ps)) for g, ps in grads.values())
    h = 1e-4
    checked = 0
    for k, (g, ps) in grads.items():
        for arr_i, arr_g in enumerate([g] + ps):
            assert not np.abs(arr_g[..., 1:]).any()
            nz = np.argwhere(np.abs(arr_g) > 1e-3 * gmax)
            idx = tuple(nz[rng.integers(len(nz))])
            fg, fps = ob.f64[k]
            arr = fg if arr_i == 0 else fps[arr_i - 1]
            old = arr[idx]
            arr[idx] = old + h
            Lp, _ = O.sparsity(ob, occs, setv, pts, 1.0 / 64)
            arr[idx] = old - h
            Lm, _ = O.sparsity(ob, occs, setv, pts, 1.0 / 64)
            arr[idx] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(arr_g[idx] - fd) <= 1e-5 * abs(fd) + 1e-8 * gmax, (k, arr_i, idx, arr_g[idx], fd)
            checked += 1
    assert checked == 4 * ob.n


# ---------------------------------------------------------------------------
# Per-block deferred shading before the merge (Eq. across as written, each
# block with its own MLP): one block reduces to the single-MLP render;
# homogeneous blocks with constant-output MLPs give the closed form
# sum_k prod_{j<k} T^j ((1 - T^k) c^k + sigmoid(b3^k)); the adjoint matches
# finite differences in textures and in every block's MLP weights
# ---------------------------------------------------------------------------
def constant_mlp(b3):
    w = np.zeros(sg.MLP_NPARAM)
    w[496:499] = b3
    return w


def test_block_mlp_single_block_equals_global():
    scene = sg.c1_scene()
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, 0)]
    v = sg.c1_view()
    w = sg.random_mlp(3, 0.6).astype(np.float64)
    g = O.render(ob, occs, v, [0], sg.c1_params(), w)
    b = O.render(ob, occs, v, [0], sg.c1_params(), w.reshape(1, -1), composite=O.BLOCK_MLP)
    hit = g["n_march"] > 0
    assert hit.sum() > 1000 and (~hit).sum() > 100
    np.testing.assert_allclose(b["rgb"][hit], g["rgb"][hit], atol=1e-13)
    assert (b["rgb"][~hit] == 0).all() and (b["trans"] == g["trans"]).all()
    assert np.abs(b["aux"][:, :3] - b["rgb"]).max() == 0 and (b["aux"][:, 7] == b["trans"]).all()


def test_block_mlp_closed_form_three_blocks():
    sig_col = [(0.7, (0.9, 0.1, 0.1)), (2.0, (0.1, 0.9, 0.1)), (0.4, (0.1, 0.1, 0.9))]
    blocks = [sg.homogeneous_block(sigma=s, color=c, block_id=k, origin=(k, 0, 0)) for k, (s, c) in enumerate(sig_col)]
    ob = O.OracleScene(blocks)
    occs = [O.occupancy(ob, k) for k in range(3)]
    v = axis_view((-0.25, 0.5, 0.5), (1.0, 0.0, 0.0))
    b3 = np.array([[0.3, -1.0, 2.0], [-0.5, 0.5, 0.0], [1.5, 1.0, -2.0]])
    mlps = np.stack([constant_mlp(b3[k]) for k in range(3)])
    r = O.render(ob, occs, v, [2, 0, 1], sg.RenderParams(mode=1), mlps, composite=O.BLOCK_MLP)
    C = np.zeros(3)
    P = 1.0
    for k, blk in enumerate(blocks):
        s, c, _ = stored_constants(blk)
        Tk = math.exp(-s)
        C += P * ((1 - Tk) * c + sig(b3[k]))
        P *= Tk
    np.testing.assert_allclose(r["rgb"][0], C, atol=1e-12)
    assert abs(r["trans"][0] - P) < 1e-12
    # the single-MLP render of the same rays adds the specular term once, not per block
    g = O.render(ob, occs, v, [2, 0, 1], sg.RenderParams(mode=1), mlps[0])
    assert np.abs(g["rgb"][0] - r["rgb"][0]).max() > 0.1


@pytest.mark.parametrize("extra", ["rgb", "trans_opacity"])
def test_block_mlp_adjoint_matches_finite_differences(extra):
    scene = tiny_city(nb=2, lods=((8, 16, 4),), shift=1.5, blobs=8, seed=13)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    v = tiny_view(10, 8, eye=(1.0, -0.8, 1.1), target=(1.0, 1.0, 0.15))
    p = sg.RenderParams(mode=1, delta=1.0 / 128, max_steps=4096)
    mlps = np.stack([kink_free_mlp(20 + k) for k in range(ob.n)])
    setv = list(range(ob.n))
    pix = O.pixels_of(v)
    rng = np.random.default_rng(4)
    target = rng.uniform(0, 1, (len(pix), 3))
    g_tr = rng.uniform(-0.5, 0.5, len(pix)) if extra != "rgb" else None
    w_op = rng.uniform(0.1, 1.0, len(pix)) if extra != "rgb" else None

    def loss():
        r = O.render(ob, occs, v, setv, p, mlps, pix=pix, composite=O.BLOCK_MLP)
        L = np.mean((r["rgb"] - target) ** 2)
        if extra != "rgb":
            L += np.sum(g_tr * r["trans"]) + np.sum(w_op * O.opacity(ob, occs, v, setv, p, pix))
        return L, r

    L0, r0 = loss()
    g_rgb = 2 * (r0["rgb"] - target) / target.size
    grads, gm = O.adjoint_block_mlp(ob, occs, v, setv, p, mlps, pix, g_rgb, g_tr, w_op)
    gmax = max(max(np.abs(g).max(), max(np.abs(q).max() for q in ps)) for g, ps in grads.values())
    h = 1e-4
    checked = 0
    for k, (g, ps) in grads.items():
        for arr_i, arr_g in enumerate([g] + ps):
            nz = np.argwhere(np.abs(arr_g) > 1e-3 * gmax)
            for _ in range(2):
                idx = tuple(nz[rng.integers(len(nz))])
                fg, fps = ob.f64[k]
                arr = fg if arr_i == 0 else fps[arr_i - 1]
                old = arr[idx]
                arr[idx] = old + h
                Lp, _ = loss()
                arr[idx] = old - h
                Lm, _ = loss()
                arr[idx] = old
                fd = (Lp - Lm) / (2 * h)
                assert abs(arr_g[idx] - fd) <= 1e-4 * abs(fd) + 1e-6 * gmax, (k, arr_i, idx, arr_g[idx], fd)
                checked += 1
    for k in range(ob.n):  # every block's own MLP
        assert np.abs(gm[k]).max() > 0
        for i in rng.choice(499, 6, replace=False):
            old = mlps[k, i]
            mlps[k, i] = old + h
            Lp, _ = loss()
            mlps[k, i] = old - h
            Lm, _ = loss()
            mlps[k, i] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(gm[k, i] - fd) <= 1e-4 * abs(fd) + 1e-8, (k, i, gm[k, i], fd)
            checked += 1
    assert checked >= 40


# ---------------------------------------------------------------------------
# Quadtree LOD (Sec. 4.5 "Baking": an entry of LOD l is one asset over
# 2^l x 2^l blocks; Appendix D: coarse-to-fine selection, depth order)
# ---------------------------------------------------------------------------
def merged_block(R=4, Rp=8, O=2, ext=(2, 2, 1), seed=0, dtype=sg.F32):
    """A block of extent ext with random smooth textures (resolutions per unit length)."""
    rng = np.random.default_rng(seed)
    gx, gy, gz = (R * e for e in ext)
    px, py, pz = (Rp * e for e in ext)
    grid = rng.normal(0, 1, (gz, gy, gx, 8)).astype(np.float32)
    planes = [rng.normal(0, 1, s + (8,)).astype(np.float32) for s in ((py, px), (pz, px), (pz, py))]
    lo = np.zeros(3, np.float32)
    return sg.BlockLod(0, 1, lo, lo + np.array(ext, np.float32), R, Rp, O, dtype, grid, planes,
                       np.ones((4, 8), np.float32), np.zeros((4, 8), np.float32))


def test_merged_block_field_against_scipy():
    """Texture addressing of a non-cubic (4 x 2 x 1) asset: every texture is
    interpolated at u = q R - 1/2 per unit length over its own extent, with
    x (u) fastest; checked against scipy's map_coordinates."""
    from scipy.ndimage import map_coordinates
    b = merged_block(ext=(4, 2, 1))  # three different extents: a swapped row length fails
    ob = O.OracleScene([b])
    rng = np.random.default_rng(3)
    pts = (rng.uniform(0, 1, (400, 3)) * np.array([4, 2, 1])).astype(np.float32)
    raw = O.field(ob, 0, pts)
    q = pts.astype(np.float64)
    R, Rp = b.grid_res, b.plane_res
    ref = np.zeros((400, 8))
    for ch in range(8):
        g = map_coordinates(b.grid[..., ch].astype(np.float64), [q[:, 2] * R - .5, q[:, 1] * R - .5,
                                                                 q[:, 0] * R - .5], order=1, mode="nearest")
        xy = map_coordinates(b.planes[0][..., ch].astype(np.float64), [q[:, 1] * Rp - .5, q[:, 0] * Rp - .5],
                             order=1, mode="nearest")
        xz = map_coordinates(b.planes[1][..., ch].astype(np.float64), [q[:, 2] * Rp - .5, q[:, 0] * Rp - .5],
                             order=1, mode="nearest")
        yz = map_coordinates(b.planes[2][..., ch].astype(np.float64), [q[:, 2] * Rp - .5, q[:, 1] * Rp - .5],
                             order=1, mode="nearest")
        ref[:, ch] = ((g + xy) + xz) + yz
    np.testing.assert_allclose(raw, ref, atol=1e-9)


def test_merged_block_occupancy_sound():
    b = merged_block(R=8, Rp=16, O=2, seed=4)
    b.grid[..., 0] = -9.0  # empty but for a few dense texels
    b.grid[3, 5, 12, 0] = b.grid[6, 13, 2, 0] = 2.0
    for p in b.planes:
        p[..., 0] *= 0.1
    ob = O.OracleScene([b])
    occ = O.occupancy(ob, 0)
    assert occ.shape == (2, 4, 4) and 0 < occ.mean() < 1
    n = 9
    g = (np.arange(n) / (n - 1)) * (1 - 1e-7)
    worst = -np.inf
    for cz, cy, cx in zip(*np.nonzero(occ == 0)):
        zz, yy, xx = np.meshgrid((cz + g) / 2, (cy + g) / 2, (cx + g) / 2, indexing="ij")
        pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.float32)
        worst = max(worst, O.field(ob, 0, pts)[:, 0].max())
    assert math.exp(worst) <= 0.01


@pytest.fixture(scope="module")
def quad_city():
    fine = sg.city_scene(4, 7, sg.U8, ((16, 64, 4),), blobs_per_block=20)
    scene = sg.Scene(4, 4, fine.blocks + sg.merged_lods(fine.blocks, 4, 4, 3))
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    return scene, ob, occs, zt


def quad_views():
    views = sg.aerial_views(31, 6, [(40, 24)], xy=(0.0, 4.0), h=(1.0, 3.0), pitch=(30.0, 60.0))
    views.append(sg.pinhole(48, 32, (1.0, -1.5, 2.0), sg.look_rotation(sg.yaw_pitch_forward(math.pi / 2.5, math.radians(40)))))
    return views


def test_merged_assets_are_downsampled_finest_level(quad_city):
    """The LOD-1 asset over blocks (0,0)-(1,1) holds the 2x box downsample of
    the four finest grids side by side (up to uint8 re-quantisation)."""
    scene, ob, occs, zt = quad_city
    a = scene.get(0, 1)
    g, _ = a.decoded()
    fine = {bid: scene.get(bid, 0).decoded()[0].astype(np.float64) for bid in (0, 1, 4, 5)}
    def down(x):
        r = x.shape[0] // 2
        return x.reshape(r, 2, r, 2, r, 2, 8).mean(axis=(1, 3, 5))
    ref = np.concatenate([np.concatenate([down(fine[0]), down(fine[1])], axis=2),
                          np.concatenate([down(fine[4]), down(fine[5])], axis=2)], axis=1)
    assert g.shape == ref.shape == (8, 16, 16, 8)
    assert np.abs(g - ref).max() <= 0.51 * a.scale[0].max() + 1e-5


def test_quadtree_selection_rule_and_partition(quad_city):
    """Selected footprints are disjoint; without culling they tile the whole
    scene; a chosen LOD-l entry (l > 0) has every child at distance >=
    thresholds[l-1] and its parent has some child nearer (coarse to fine);
    huge thresholds give every finest block, zero thresholds the roots."""
    scene, ob, occs, zt = quad_city
    B = scene.blocks

    def dist(k):
        e = B[k]
        inside = [j for j, f in enumerate(B) if f.lod == 0 and f.aabb_min[0] >= e.aabb_min[0] and
                  f.aabb_max[0] <= e.aabb_max[0] and f.aabb_min[1] >= e.aabb_min[1] and f.aabb_max[1] <= e.aabb_max[1]]
        c = np.array([(e.aabb_min[0] + e.aabb_max[0]) / 2.0, (e.aabb_min[1] + e.aabb_max[1]) / 2.0,
                      max(zt[j] for j in inside)], np.float64)
        return float(np.linalg.norm(v.eye.astype(np.float64) - c))

    def kids(k):
        e = B[k]
        return [j for j, f in enumerate(B) if f.lod == e.lod - 1 and f.aabb_min[0] >= e.aabb_min[0] and
                f.aabb_max[0] <= e.aabb_max[0] and f.aabb_min[1] >= e.aabb_min[1] and f.aabb_max[1] <= e.aabb_max[1]]

    thr = (1.8, 3.2)
    mixed = 0
    for v in quad_views():
        sel = list(O.select(v, B, zt, thresholds=thr, cull=False, quadtree=True))
        area = np.zeros((4, 4), np.int32)
        for k in sel:
            e = B[k]
            area[int(e.aabb_min[1]):int(e.aabb_max[1]), int(e.aabb_min[0]):int(e.aabb_max[0])] += 1
            if e.lod > 0:
                assert all(dist(j) >= thr[e.lod - 1] for j in kids(k))
            parent = [j for j, f in enumerate(B) if f.lod == e.lod + 1 and k in kids(j)]
            for j in parent:
                assert any(dist(i) < thr[e.lod] for i in kids(j))
        assert (area == 1).all()
        mixed += len({B[k].lod for k in sel}) > 1
        assert [B[k].lod for k in O.select(v, B, zt, thresholds=(1e9, 1e9), cull=False, quadtree=True)] == [0] * 16
        assert [B[k].lod for k in O.select(v, B, zt, thresholds=(0.0, 0.0), cull=False, quadtree=True)] == [2]
    assert mixed >= 2


def test_quadtree_order_is_per_ray_order_and_culling_exact(quad_city):
    """On every pixel the per-view quadtree order equals the per-ray entry
    order (so the block merge is the monolithic composite, Appendix A), and
    culling removes only entries no ray reaches."""
    scene, ob, occs, zt = quad_city
    w = sg.xavier_mlp(3)
    p = sg.cityb_params()
    for v in quad_views():
        sel = list(O.select(v, scene.blocks, zt, thresholds=(1.8, 3.2), cull=True, quadtree=True))
        allb = list(O.select(v, scene.blocks, zt, thresholds=(1.8, 3.2), cull=False, quadtree=True))
        a = O.render(ob, occs, v, sel, p, w)
        assert a["order_ok"].all()
        m = O.render(ob, occs, v, sel, p, w, composite=O.MONOLITHIC)
        assert np.abs(a["rgb"] - m["rgb"]).max() < 1e-12 and np.abs(a["trans"] - m["trans"]).max() < 1e-12
        if {scene.blocks[k].lod for k in sel} == {scene.blocks[k].lod for k in allb}:
            b = O.render(ob, occs, v, allb, p, w)
            assert np.array_equal(a["rgb"], b["rgb"])


def np_pool(occ, level):
    """Max-pool by numpy's reshape-and-reduce: 2^level cells per axis, or the
    whole axis when it is shorter."""
    s = [min(1 << level, n) for n in occ.shape]
    z, y, x = occ.shape
    return occ.reshape(z // s[0], s[0], y // s[1], s[1], x // s[2], s[2]).max(axis=(1, 3, 5))


def test_occupancy_pyramid_against_numpy_pooling(quad_city):
    """The multi-level occupancy grid (Sec. 3 rendering stage, Sec. 4.5 max-pool
    downsampling) of cubic blocks and non-cubic merged assets: every level
    equals numpy's reshape-max of the base grid, each level is the 2x pool of
    the one below, the top level is one cell holding any(base), and a single
    occupied base cell lands in exactly one coarse cell at (x, y, z) >> l."""
    scene, ob, occs, zt = quad_city
    rng = np.random.default_rng(12)
    kinds = {}
    for k, b in enumerate(scene.blocks):
        kinds.setdefault(occs[k].shape, k)
    assert len(kinds) >= 3  # 16^3, 32x32x16, 64x64x16 cells
    for shape, k in kinds.items():
        nl = O.occupancy_levels(occs[k])
        assert 1 << nl == max(shape)
        grids = [occs[k]] + [(rng.random(shape) < p).astype(np.uint8) for p in (0.002, 0.05, 0.5)]
        for g in grids:
            prev = g
            for l in range(nl + 1):
                lv = O.occupancy_level(ob, k, g, l)
                assert np.array_equal(lv, np_pool(g, l)), (shape, l)
                if l:
                    assert np.array_equal(lv, np_pool(prev, 1)), (shape, l)
                prev = lv
            assert lv.shape == (1, 1, 1) and lv[0, 0, 0] == int(g.any())
        for _ in range(12):
            z, y, x = (int(rng.integers(n)) for n in shape)
            g = np.zeros(shape, np.uint8)
            g[z, y, x] = 1
            for l in range(nl + 1):
                lv = O.occupancy_level(ob, k, g, l)
                assert lv.sum() == 1
                cz, cy, cx = (min(i >> l, n - 1) for i, n in zip((z, y, x), lv.shape))
                assert lv[cz, cy, cx] == 1


# ---------------------------------------------------------------------------
# P21: positional encoding of the view direction in the deferred MLP
# (Eq. deferred): [d, sin(2^l d), cos(2^l d) for l < L]
# ---------------------------------------------------------------------------
def test_posenc_identities_and_values():
    """The identity part is d; every (sin, cos) pair lies on the unit circle;
    each frequency doubles the previous one (double-angle identities, which a
    wrong scale, a swapped sin/cos or a misplaced block breaks); the first
    frequency is 1 (closed-form values at pi/6, pi/2, 0)."""
    rng = np.random.default_rng(21)
    for pe in range(5):
        assert O.mlp_params(pe) == 499 + 96 * pe
        for _ in range(20):
            d = rng.standard_normal(3)
            d /= np.linalg.norm(d)
            g = O.posenc(d, pe)
            assert g.size == 3 + 6 * pe
            np.testing.assert_array_equal(g[:3], d)
            for l in range(pe):
                s, c = g[3 + 6 * l:6 + 6 * l], g[6 + 6 * l:9 + 6 * l]
                np.testing.assert_allclose(s * s + c * c, 1.0, atol=1e-15)
                if l + 1 < pe:
                    s2, c2 = g[9 + 6 * l:12 + 6 * l], g[12 + 6 * l:15 + 6 * l]
                    np.testing.assert_allclose(s2, 2 * s * c, atol=1e-14)
                    np.testing.assert_allclose(c2, c * c - s * s, atol=1e-14)
    g = O.posenc(np.array([np.pi / 6, np.pi / 2, 0.0]), 2)
    np.testing.assert_allclose(g[3:6], [0.5, 1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(g[6:9], [np.sqrt(3) / 2, 0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(g[9:12], [np.sqrt(3) / 2, 0.0, 0.0], atol=1e-15)
    with pytest.raises(ValueError):
        O.posenc(np.zeros(3), 5)


def test_mlp_with_posenc_against_torch():
    import torch
    pe = 4
    ni = 10 + 6 * pe
    w = sg.random_mlp(8, scale=0.5, pe=pe).astype(np.float64)
    o1 = 16 * ni
    net = torch.nn.Sequential(torch.nn.Linear(ni, 16), torch.nn.ReLU(), torch.nn.Linear(16, 16),
                              torch.nn.ReLU(), torch.nn.Linear(16, 3), torch.nn.Sigmoid()).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.tensor(w[0:o1].reshape(16, ni)))
        net[0].bias.copy_(torch.tensor(w[o1:o1 + 16]))
        net[2].weight.copy_(torch.tensor(w[o1 + 16:o1 + 272].reshape(16, 16)))
        net[2].bias.copy_(torch.tensor(w[o1 + 272:o1 + 288]))
        net[4].weight.copy_(torch.tensor(w[o1 + 288:o1 + 336].reshape(3, 16)))
        net[4].bias.copy_(torch.tensor(w[o1 + 336:o1 + 339]))
    rng = np.random.default_rng(1)
    for _ in range(30):
        x = rng.uniform(-1, 1, ni)
        ref = net(torch.tensor(x)[None]).detach().numpy()[0]
        np.testing.assert_allclose(O.mlp(w, x, pe), ref, atol=1e-14)


def widened(w0, pe):
    """The 10-input MLP w0 as an MLP over 10 + 6 pe inputs whose extra
    first-layer columns are zero."""
    ni = 10 + 6 * pe
    W1 = np.zeros((16, ni))
    W1[:, :10] = w0[:160].reshape(16, 10)
    return np.concatenate([W1.ravel(), w0[160:]])


@pytest.mark.parametrize("composite", [O.MERGED, O.BLOCK_MLP])
def test_posenc_render_reduces_to_plain_direction(composite):
    """With the encoding's first-layer columns zero, a render with PE(d)
    equals the render with the plain direction (both composites)."""
    scene = tiny_city(nb=2, lods=((8, 16, 4),), shift=2.0, blobs=8, seed=31)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    v = tiny_view(10, 8)
    p0 = sg.RenderParams(mode=1, delta=1.0 / 128, max_steps=4096)
    p4 = sg.RenderParams(mode=1, delta=1.0 / 128, max_steps=4096, pe_freqs=4)
    if composite == O.MERGED:
        w0 = sg.random_mlp(3, 0.6).astype(np.float64)
        w4 = widened(w0, 4)
    else:
        w0 = np.stack([sg.random_mlp(40 + k, 0.6) for k in range(ob.n)]).astype(np.float64)
        w4 = np.stack([widened(x, 4) for x in w0])
    a = O.render(ob, occs, v, list(range(ob.n)), p0, w0, composite=composite)
    b = O.render(ob, occs, v, list(range(ob.n)), p4, w4, composite=composite)
    assert np.abs(a["rgb"]).max() > 0.1
    np.testing.assert_allclose(b["rgb"], a["rgb"], atol=1e-15)
    w4x = w4.copy()
    w4x.reshape(-1, w4.shape[-1])[:, 10] += 0.5  # a first sin column: the colour changes
    c = O.render(ob, occs, v, list(range(ob.n)), p4, w4x, composite=composite)
    assert np.abs(c["rgb"] - a["rgb"]).max() > 1e-4


def test_adjoint_with_posenc_matches_finite_differences():
    pe = 4
    ni = 10 + 6 * pe
    scene = tiny_city(nb=2, lods=((8, 16, 4),), shift=1.5, blobs=8, seed=13)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    v = tiny_view(12, 10, eye=(1.0, -0.8, 1.1), target=(1.0, 1.0, 0.15))
    p = sg.RenderParams(mode=1, delta=1.0 / 128, max_steps=4096, pe_freqs=pe)
    rng = np.random.default_rng(3)
    # kink-free: |W1 x| <= 34 * 0.1 < b1 = 4 for inputs in [-1, 1]
    w = np.concatenate([rng.uniform(-0.1, 0.1, 16 * ni), np.full(16, 4.0), rng.uniform(-0.05, 0.05, 256),
                        np.full(16, 7.0), rng.uniform(-0.02, 0.02, 48), rng.uniform(-0.5, 0.5, 3)])
    setv = list(range(ob.n))
    pix = O.pixels_of(v)
    target = np.random.default_rng(4).uniform(0, 1, (len(pix), 3))

    def loss():
        return np.mean((O.render(ob, occs, v, setv, p, w, pix=pix)["rgb"] - target) ** 2)

    r0 = O.render(ob, occs, v, setv, p, w, pix=pix)
    g_rgb = 2 * (r0["rgb"] - target) / target.size
    grads, gm = O.adjoint(ob, occs, v, setv, p, w, pix, g_rgb)
    assert gm.size == O.mlp_params(pe)
    h = 1e-3
    # row 0 of W1 at encoding columns, then anywhere
    picks = [int(c) for c in rng.choice(np.arange(10, ni), 8, replace=False)]
    picks += [int(i) for i in rng.choice(gm.size, 10, replace=False)]
    for i in picks:
        old = w[i]
        w[i] = old + h
        Lp = loss()
        w[i] = old - h
        Lm = loss()
        w[i] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(gm[i] - fd) <= 1e-4 * abs(fd) + 1e-8, (i, gm[i], fd)
    k = next(iter(grads))
    g = grads[k][1][0]
    idx = tuple(np.argwhere(np.abs(g) > 1e-3 * np.abs(g).max())[0])
    arr = ob.f64[k][1][0]
    old = arr[idx]
    arr[idx] = old + h
    Lp = loss()
    arr[idx] = old - h
    Lm = loss()
    arr[idx] = old
    fd = (Lp - Lm) / (2 * h)
    assert abs(g[idx] - fd) <= 1e-4 * abs(fd) + 1e-9


# ---------------------------------------------------------------------------
# P22: contraction of boundary blocks (implementation details, the MERF
# contraction equation) and the exterior they own
# ---------------------------------------------------------------------------
def test_contraction_closed_forms():
    """Values the contraction equation fixes: identity inside the unit cube;
    outside, the coordinate(s) attaining the max norm m go to (2 - 1/m) with
    their sign and the others are divided by m; odd symmetry; all of space
    lands strictly inside the cube of radius 2; continuous across |x| = 1."""
    assert np.allclose(O.contract([0.5, -1.0, 0.2]), [0.5, -1.0, 0.2], atol=0, rtol=0)
    assert np.allclose(O.contract([3.0, 0.0, 0.0]), [5.0 / 3.0, 0.0, 0.0], rtol=1e-15)
    assert np.allclose(O.contract([3.0, 1.5, -0.5]), [5.0 / 3.0, 0.5, -1.0 / 6.0], rtol=1e-15)
    assert np.allclose(O.contract([-4.0, 4.0, 1.0]), [-1.75, 1.75, 0.25], rtol=1e-15)
    rng = np.random.default_rng(22)
    for _ in range(200):
        x = rng.normal(size=3) * np.exp(rng.uniform(-2, 6))
        y = O.contract(x)
        m = np.abs(x).max()
        assert np.allclose(O.contract(-x), -y, rtol=0, atol=0)
        assert np.abs(y).max() < 2.0
        if m > 1:
            # a ray from the origin: the contracted radius is 2 - 1/m, the direction kept
            assert np.isclose(np.abs(y).max(), 2.0 - 1.0 / m, rtol=1e-14)
            j = np.argmax(np.abs(x))
            k = [c for c in range(3) if c != j]
            assert np.allclose(y[k] / y[j], x[k] / x[j] * (1.0 / m) / (2.0 - 1.0 / m) * m, rtol=1e-12)
    u = np.array([1.0, 0.3, -0.7])
    for eps in (1e-6, 1e-9):
        assert np.allclose(O.contract(u * (1 + eps)), u, atol=3 * eps)


def test_contracted_local_coordinate_is_the_definition_in_fp32():
    """The fp32 decision sequence of a contracted block's texture coordinate
    agrees with q = (contract((p - centre) 2/extent) + 2) extent/4 in fp64 to
    a few fp32 ulps; a plain block's is p - lo exactly."""
    b = sg.homogeneous_block(origin=(2, -1, 0))
    cb = sg.contract_boundary([b])[0]
    assert cb.contracted
    ob = O.OracleScene([b, dataclasses.replace(cb, block_id=1)])
    rng = np.random.default_rng(23)
    ctr = np.array([2.5, -0.5, 0.5])
    for _ in range(300):
        p = (ctr + rng.normal(size=3) * np.exp(rng.uniform(-3, 4))).astype(np.float32)
        q0, m0 = O.local_q(ob, 0, p)
        assert np.array_equal(q0, (p - np.float32([2, -1, 0])).astype(np.float32)) and m0 == 0.0
        q1, m1 = O.local_q(ob, 1, p)
        x = (p.astype(np.float64) - ctr) * 2.0
        assert np.isclose(m1, np.abs(x).max(), rtol=1e-6)
        assert np.allclose(q1, (O.contract(x) + 2.0) / 4.0, atol=4e-7)


def _shell_block(sig_shell, sig_box, col_shell, col_box, R=8):
    """A contracted unit block whose texels in the outer shell (contracted
    |y|_inf > 1) hold one constant field and those of the box another."""
    b = sg.contract_boundary([sg.homogeneous_block(R=R, Rp=8, O=4)])[0]
    y = (np.arange(R) + 0.5) / R * 4.0 - 2.0
    shell = np.maximum(np.maximum(np.abs(y)[:, None, None], np.abs(y)[None, :, None]), np.abs(y)[None, None, :]) > 1
    g = b.grid.copy()
    logit = lambda v: math.log(v / (1.0 - v))
    for mask, s, col in ((shell, sig_shell, col_shell), (~shell, sig_box, col_box)):
        g[mask, 0] = math.log(s)
        for i, c in enumerate(col):
            g[mask, 1 + i] = logit(c)
    return dataclasses.replace(b, grid=g)


def test_exterior_is_composited_before_and_after_the_city():
    """Camera outside the footprint looking at the block: an opaque shell in
    front hides the box, so the accumulated colour is the shell's own colour
    (one sample with alpha = 1).  Looking away, the ray never enters the
    footprint and sees only the exterior: for a homogeneous medium the
    accumulated colour is (1 - T) times the medium's colour (the telescoping
    sum of T_i alpha_i), with 0 < T < 1."""
    shell_col, box_col = (0.9, 0.2, 0.1), (0.1, 0.7, 0.3)
    blk = _shell_block(1e4, 5.0, shell_col, box_col)
    ob = O.OracleScene([blk])
    occs = [O.occupancy(ob, 0)]
    w = sg.random_mlp(3, 0.5)
    p = sg.RenderParams(mode=1, ext_delta=1.0 / 64, ext_max_steps=4096)
    inward = sg.pinhole(3, 3, (2.5, 0.5, 0.5), sg.look_rotation([-1.0, 0.0, 0.0]), 20.0)
    ref = O.render(ob, occs, inward, [0], p, w, pix=np.array([[1, 1]], np.int32))
    assert ref["trans"][0] < 1e-12
    assert np.allclose(ref["aux"][0, :3], shell_col, atol=1e-9)
    assert ref["n_march"][0] >= 1
    # no exterior sampling: the box's colour shows instead
    p0 = sg.RenderParams(mode=1)
    ref0 = O.render(ob, occs, inward, [0], p0, w, pix=np.array([[1, 1]], np.int32))
    assert not np.allclose(ref0["aux"][0, :3], shell_col, atol=1e-2)
    thin = _shell_block(0.05, 5.0, shell_col, box_col)
    ob2 = O.OracleScene([thin])
    outward = sg.pinhole(3, 3, (2.5, 0.5, 0.5), sg.look_rotation([1.0, 0.0, 0.0]), 20.0)
    ref2 = O.render(ob2, [O.occupancy(ob2, 0)], outward, [0], p, w, pix=np.array([[1, 1]], np.int32))
    T = ref2["trans"][0]
    assert 0.0 < T < 1.0
    assert np.allclose(ref2["aux"][0, :3], (1.0 - T) * np.array(shell_col), rtol=1e-9)
    # a plain (uncontracted) block owns no exterior: nothing is sampled
    plain = dataclasses.replace(thin, contracted=False)
    ob3 = O.OracleScene([plain])
    ref3 = O.render(ob3, [O.occupancy(ob3, 0)], outward, [0], p, w, pix=np.array([[1, 1]], np.int32))
    assert ref3["trans"][0] == 1.0 and ref3["n_march"][0] == 0


def test_exterior_steps_are_about_uniform_in_contracted_space():
    """Along a ray leaving a contracted unit block's centre through its +x
    face, the exterior samples' contracted x-coordinate y = 4 q - 2 grows by
    2 delta / (1 + 2 delta m) per step, so by a step within [2 delta / 3,
    2 delta] while m runs from 1 to the far limit 1/delta (a step rule in m
    instead of m^2, or a wrong factor, leaves that band); the samples cover the
    shell up to within 2 delta of its outer face, and the y and z coordinates
    stay at the centre.  A ray leaving along a face diagonal keeps equal x and
    y contracted coordinates."""
    blk = sg.contract_boundary([sg.homogeneous_block()])[0]
    ob = O.OracleScene([blk])
    occs = [O.occupancy(ob, 0)]
    for delta in (1.0 / 32, 1.0 / 64):
        p = sg.RenderParams(mode=1, ext_delta=delta, ext_max_steps=100000)
        q, dl = O.ext_samples(ob, occs, [0], p, (0.5, 0.5, 0.5), (1.0, 0.0, 0.0), 0.5, np.inf, 1)
        y = 4.0 * q[:, 0].astype(np.float64) - 2.0
        assert len(y) > 10
        dy = np.diff(y)
        assert (dy > 2 * delta / 3 * (1 - 1e-4)).all() and (dy < 2 * delta * (1 + 1e-4)).all()
        assert y[0] > 1.0 and y[-1] > 2.0 - 2 * delta
        assert np.allclose(q[:, 1:], 0.5, atol=1e-6)
        # the step lengths are the world distances between consecutive samples
        m = 1.0 / (2.0 - y)
        assert np.allclose(dl, delta * m * m, rtol=1e-5)
    u = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)
    q, _ = O.ext_samples(ob, occs, [0], sg.RenderParams(mode=1, ext_delta=1 / 64, ext_max_steps=100000),
                         (0.5, 0.5, 0.5), u, 0.5 * np.sqrt(2.0), np.inf, 1)
    assert len(q) > 10 and np.allclose(q[:, 0], q[:, 1], atol=1e-6)


# ---------------------------------------------------------------------------
# Selection with contracted boundary blocks: such a block also owns the space
# beyond its outer faces (Eq. "blocks" in the max norm), so neither the
# frustum test of its box nor the far cut may drop it (Appendix D culling,
# read conservatively)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def contraction_city():
    scene = sg.make_scene(4, 4, ((8, 16, 4),), sg.U8, blobs_per_block=4, blob_z=(0.0, 0.3), seed=31)
    blocks = sg.contract_boundary(scene.blocks)
    ob = O.OracleScene(blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    return blocks, ob, occs, zt


CONTRACTION_VIEWS = {
    # inside the city, looking out over the +x edge
    "looking_out": ((2.2, 2.0, 0.6), (1.0, 0.15, 0.05)),
    # low inside the city, looking up past the -y edge: the content (and the
    # boxes up to its top) lie below the frustum, the exterior does not
    "looking_up": ((2.0, 1.0, 0.35), (0.0, -0.35, 1.0)),
    # ten widths beyond the far edge's opposite side, looking at the city
    "far": ((-6.0, 2.0, 1.5), (1.0, 0.0, -0.12)),
}


@pytest.mark.parametrize("name", sorted(CONTRACTION_VIEWS))
def test_selection_keeps_contracted_blocks(contraction_city, name):
    blocks, ob, occs, zt = contraction_city
    eye, fwd = CONTRACTION_VIEWS[name]
    v = sg.pinhole(40, 24, eye, sg.look_rotation(np.asarray(fwd)))
    thr = (8.0,)
    p = sg.RenderParams(mode=1, ext_delta=1.0 / 32, ext_max_steps=256)
    w = sg.random_mlp(5, 0.6)
    contracted = {k for k, b in enumerate(blocks) if b.contracted}
    sel = list(O.select(v, blocks, zt, thresholds=thr, cull=True))
    unculled = list(O.select(v, blocks, zt, thresholds=thr, cull=False))
    assert contracted <= set(sel)  # never culled, never beyond the far cut
    # culling stays exact with the exterior: the culled set renders bitwise
    # like every block within the far cut
    a = O.render(ob, occs, v, sel, p, w)
    b = O.render(ob, occs, v, unculled, p, w)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["trans"], b["trans"])
    assert (a["n_march"] > 0).mean() > 0.3
    if name == "far":
        # the plain inner blocks are all nearer than the far edge, yet the far
        # edge's contracted blocks (more than 8 widths away) are drawn
        far = [k for k in contracted
               if np.hypot(eye[0] - blocks[k].aabb_min[0] - 0.5, eye[1] - blocks[k].aabb_min[1] - 0.5) > 8.5]
        assert far and set(far) <= set(sel)
        c = O.render(ob, occs, v, [k for k in sel if k not in far], p, w)
        assert np.abs(c["trans"] - a["trans"]).max() > 1e-3  # and they matter: they own the exterior there
    else:
        assert len(unculled) > len(sel)  # some plain block was culled
    if name == "looking_up":
        # the old rule (contracted blocks culled by their box, z_top read from
        # texture z) drops blocks whose exterior this view sees
        plain = [dataclasses.replace(x, contracted=False) for x in blocks]
        obp = O.OracleScene(plain)
        old = set(O.select(v, plain, [O.ztop(obp, j, occs[j]) for j in range(len(plain))], thresholds=(1e30,),
                           cull=True))
        boxes_out = [k for k in contracted if k not in old]
        assert boxes_out
        c = O.render(ob, occs, v, [k for k in sel if k not in boxes_out], p, w)
        assert np.abs(c["trans"] - a["trans"]).max() > 1e-3


def test_quadtree_selection_opens_assets_holding_contracted_blocks():
    """Quadtree LOD over an 8x8 city with contracted edge columns: a merged
    asset whose footprint holds a contracted block is always opened down to
    that block (the merged asset owns no exterior), inner assets still merge,
    and the chosen footprints tile the city exactly once."""
    scene = sg.make_scene(8, 8, ((8, 16, 4),), sg.U8, blobs_per_block=2, blob_z=(0.0, 0.3), seed=33)
    fine = sg.contract_boundary(scene.blocks)
    blocks = fine + sg.merged_lods(scene.blocks, 8, 8, 3)
    ob = O.OracleScene(blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    contracted = {k for k, b in enumerate(blocks) if b.contracted}
    assert len(contracted) == 28
    p = sg.RenderParams(mode=1, ext_delta=1.0 / 32, ext_max_steps=256)
    w = sg.random_mlp(6, 0.6)
    merged_seen = 0
    for eye, fwd in (((4.0, -9.0, 6.0), (0.0, 1.0, -0.55)), ((4.2, 3.9, 7.0), (0.1, 0.05, -1.0))):
        v = sg.pinhole(32, 24, eye, sg.look_rotation(np.asarray(fwd)))
        sel = list(O.select(v, blocks, zt, thresholds=(1.0, 2.0), cull=True, quadtree=True))
        assert contracted <= set(sel)
        cover = np.zeros((8, 8), int)
        for k in sel:
            b = blocks[k]
            x0, y0 = int(b.aabb_min[0]), int(b.aabb_min[1])
            x1, y1 = int(b.aabb_max[0]), int(b.aabb_max[1])
            cover[y0:y1, x0:x1] += 1
            merged_seen += b.lod > 0
            if b.lod > 0:
                assert not any(blocks[c].aabb_min[0] >= x0 and blocks[c].aabb_max[0] <= x1 and
                               blocks[c].aabb_min[1] >= y0 and blocks[c].aabb_max[1] <= y1 for c in contracted)
        assert cover.max() <= 1
        unculled = list(O.select(v, blocks, zt, thresholds=(1.0, 2.0), cull=False, quadtree=True))
        a = O.render(ob, occs, v, sel, p, w)
        b = O.render(ob, occs, v, unculled, p, w)
        assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["trans"], b["trans"])
        assert a["order_ok"].all()
    assert merged_seen > 0


def test_step_cap_truncates_the_exterior_behind_it(contraction_city):
    """The cap of max_steps steps from scene entry truncates a ray: when it
    ends before the ray leaves the footprint's column, the exterior beyond
    the column is not sampled either (no hole followed by more samples).  An
    axis ray at y = 0.5, z = 0.2 from x = -0.5 crosses the 4-wide city from
    t = 0.5 to t = 4.5 (2048 steps of 1/512 in the box): with a cap of 1024
    its samples are the exterior before the column plus 1024 box steps; with
    a cap of 4096 they add the 2048 box steps and the exterior after it."""
    blocks, ob, occs, zt = contraction_city
    v = axis_view((-0.5, 0.5, 0.2), (1.0, 0.0, 0.0))
    allb = list(range(len(blocks)))
    o, d = (-0.5, 0.5, 0.2), (1.0, 0.0, 0.0)
    base = dict(mode=1, ext_delta=1.0 / 32, ext_max_steps=256)
    pre, _ = O.ext_samples(ob, occs, allb, sg.RenderParams(**base), o, d, 0.0, 0.5, 0)
    post, _ = O.ext_samples(ob, occs, allb, sg.RenderParams(**base), o, d, 4.5, np.inf, 1)
    assert len(pre) > 0 and len(post) > 0
    capped = O.render(ob, occs, v, allb, sg.RenderParams(max_steps=1024, **base), zero_mlp())
    full = O.render(ob, occs, v, allb, sg.RenderParams(max_steps=4096, **base), zero_mlp())
    assert capped["n_march"][0] == len(pre) + 1024
    assert full["n_march"][0] == len(pre) + 2048 + len(post)


def test_touched_texels_closed_form():
    """The texels a frame's evaluated samples read (its compulsory texture
    bytes): an axis ray along +x at y = z = 0.5 through a homogeneous block
    (8 texels per axis, every cell occupied) samples x over the whole chord,
    so the grid taps are x = 0..7 at y, z in {3, 4} (u = 0.5 R - 1/2 = 3.5),
    the xy plane u = 0..7 at v = y in {3, 4}, the xz plane u = 0..7 at v = z in
    {3, 4}, the yz plane the 2 x 2 texels (3..4, 3..4); a ray that misses the
    block reads nothing."""
    b = sg.homogeneous_block(R=8, Rp=8, O=4, sigma=2.0)
    ob = O.OracleScene([b])
    occs = [O.occupancy(ob, 0)]
    assert occs[0].all()
    v = axis_view((-0.25, 0.5, 0.5), (1.0, 0.0, 0.0))
    m = O.touched_texels(ob, occs, v, [0], sg.RenderParams(mode=1))[0]
    g = np.zeros((8, 8, 8), np.uint8)
    g[3:5, 3:5, :] = 1
    xy = np.zeros((8, 8), np.uint8)
    xy[3:5, :] = 1
    yz = np.zeros((8, 8), np.uint8)
    yz[3:5, 3:5] = 1
    assert np.array_equal(m[0], g) and np.array_equal(m[1], xy) and np.array_equal(m[2], xy)
    assert np.array_equal(m[3], yz)
    miss = axis_view((-0.25, 1.5, 0.5), (1.0, 0.0, 0.0))
    assert all(not x.any() for x in O.touched_texels(ob, occs, miss, [0], sg.RenderParams(mode=1))[0])
    # empty cells read nothing: the same ray through a block whose cells are all empty
    assert all(not x.any() for x in O.touched_texels(ob, [np.zeros_like(occs[0])], v, [0],
                                                     sg.RenderParams(mode=1))[0])


# ---------------------------------------------------------------------------
# P13 at the differentiable workload's size: central differences on the
# 64 x 64 crop (Sec. 4.2, consistent training through the block merge)
# ---------------------------------------------------------------------------
def _pixel_dirs(view, pix):
    """Unit world directions of the given pixels (fp64 of the camera model)."""
    R = np.asarray(view.R, np.float64).reshape(3, 3)
    x = (pix[:, 0] + 0.5 - float(view.cx)) / float(view.fx)
    y = (pix[:, 1] + 0.5 - float(view.cy)) / float(view.fy)
    u = np.stack([x, y, np.ones_like(x)], 1) @ R.T
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def _kink_risk(w, X, i, h):
    """Whether moving MLP weight i by +-h may carry some pixel's ReLU
    pre-activation across zero (layout W1 [16][10], b1, W2 [16][16], b2,
    W3 [3][16], b3; inputs X [n][10])."""
    W1, b1 = w[:160].reshape(16, 10), w[160:176]
    W2, b2 = w[176:432].reshape(16, 16), w[432:448]
    pre1 = X @ W1.T + b1
    h1 = np.maximum(pre1, 0.0)
    pre2 = h1 @ W2.T + b2
    if i < 176:  # W1[o][j] or b1[o]
        o = (i // 10) if i < 160 else i - 160
        dx = np.abs(X[:, i % 10]) if i < 160 else np.ones(len(X))
        if (np.abs(pre1[:, o]) <= 2 * h * dx).any():
            return True
        return bool((np.abs(pre2) <= 2 * h * dx[:, None] * np.abs(W2[:, o])[None, :]).any())
    if i < 448:  # W2[j][o] or b2[j]
        j = ((i - 176) // 16) if i < 432 else i - 432
        dx = h1[:, (i - 176) % 16] if i < 432 else np.ones(len(X))
        return bool((np.abs(pre2[:, j]) <= 2 * h * dx).any())
    return False  # W3, b3: after the last ReLU


@pytest.mark.slow
def test_c5_crop_adjoint_against_finite_differences():
    """The differentiable workload (4x4 fp32 blocks of 128^3 + 3 x 1024^2,
    view 0 of its eight 800x800 views): on the 64 x 64 window with the most
    evaluated samples among 16 seeded candidates (counted by the oracle), the
    fp64 adjoint of the MSE against the target scene's image matches central
    differences (h = 1e-3, fp64) on 64 seeded parameters the crop touches:
    24 grid texel-channels, 8 texel-channels per plane, 16 MLP weights (a
    weight whose perturbation could carry a ReLU pre-activation of some
    pixel across zero is redrawn)."""
    learn, target = sg.c5_scenes()
    v0 = sg.c5_views()[0]
    p = sg.cityb_params()
    w = sg.xavier_mlp(4).astype(np.float64)
    ob = O.OracleScene(learn.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    setv = list(range(ob.n))
    rng = np.random.default_rng(0)
    cands = [(int(rng.integers(0, 800 - 64)), int(rng.integers(0, 800 - 64))) for _ in range(16)]

    def score(c):
        pix = np.array([[c[0] + i, c[1] + j] for j in range(0, 64, 8) for i in range(0, 64, 8)], np.int32)
        return int(O.render(ob, occs, v0, setv, p, w, pix=pix)["n_eval"].sum())
    x0, y0 = max(cands, key=score)
    crop = v0.with_crop(x0, y0, 64, 64)
    pix = O.pixels_of(crop)
    ob_t = O.OracleScene(target.blocks)
    tgt = O.render(ob_t, [O.occupancy(ob_t, k) for k in range(ob_t.n)], crop, list(range(ob_t.n)), p,
                   sg.xavier_mlp(5), pix=pix)["rgb"]
    del ob_t, target

    def loss():
        r = O.render(ob, occs, crop, setv, p, w, pix=pix)
        return np.mean((r["rgb"] - tgt) ** 2), r
    L0, r0 = loss()
    assert r0["n_eval"].sum() > 1_000_000
    g_rgb = 2 * (r0["rgb"] - tgt) / tgt.size
    grads, gm = O.adjoint(ob, occs, crop, setv, p, w, pix, g_rgb)
    gmax = max(max(np.abs(g).max(), max(np.abs(q).max() for q in ps)) for g, ps in grads.values())
    assert gmax > 0
    h = 1e-3
    picks = []
    for arr_i, n_pick in ((0, 24), (1, 8), (2, 8), (3, 8)):
        cand = [(k, tuple(i)) for k, (g, ps) in grads.items()
                for i in np.argwhere(np.abs(g if arr_i == 0 else ps[arr_i - 1]) > 1e-3 * gmax)]
        for c in rng.choice(len(cand), n_pick, replace=False):
            picks.append((cand[c][0], arr_i, cand[c][1]))
    for k, arr_i, idx in picks:
        fg, fps = ob.f64[k]
        arr = fg if arr_i == 0 else fps[arr_i - 1]
        ga = (grads[k][0] if arr_i == 0 else grads[k][1][arr_i - 1])[idx]
        old = arr[idx]
        arr[idx] = old + h
        Lp, _ = loss()
        arr[idx] = old - h
        Lm, _ = loss()
        arr[idx] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(ga - fd) <= 1e-4 * abs(fd) + 1e-6 * gmax, (k, arr_i, idx, ga, fd)
    X = np.concatenate([r0["aux"][:, :7], _pixel_dirs(crop, pix)], 1)
    mlp_picks = []
    while len(mlp_picks) < 16:
        i = int(rng.integers(499))
        if i not in mlp_picks and not _kink_risk(w, X, i, h):
            mlp_picks.append(i)
    assert any(i < 448 for i in mlp_picks)  # hidden layers are exercised, not only the output layer
    gmm = np.abs(gm).max()
    for i in mlp_picks:
        old = w[i]
        w[i] = old + h
        Lp, _ = loss()
        w[i] = old - h
        Lm, _ = loss()
        w[i] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(gm[i] - fd) <= 1e-4 * abs(fd) + 1e-6 * gmm, (i, gm[i], fd)
    assert len(picks) + len(mlp_picks) == 64
