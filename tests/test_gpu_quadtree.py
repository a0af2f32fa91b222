"""GPU parity of the quadtree LOD path (merged assets over 2^l x 2^l blocks,
coarse-to-fine selection, recursive-quadrant depth order): occupancy of the
non-cubic assets and the per-view selection bit-exact against the oracle,
renders within 1e-4 with bit-exact sample counts, launch variants bitwise
equal, the adjoint on merged fp32 assets within 1e-3 of the fp64 adjoint,
and invalid sets (overlapping or misaligned entries) rejected."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2312_16457_amd import scenegen as sg

pytestmark = pytest.mark.gpu
THR = (1.8, 3.2)
TOL = 1e-4


def small_quad_city(dtype=sg.U8, seed=7):
    fine = sg.city_scene(4, seed, dtype, ((16, 64, 4),), blobs_per_block=20)
    return sg.Scene(4, 4, fine.blocks + sg.merged_lods(fine.blocks, 4, 4, 3, dtype=dtype))


def views_small():
    views = sg.aerial_views(31, 6, [(40, 24)], xy=(0.0, 4.0), h=(1.0, 3.0), pitch=(30.0, 60.0))
    views.append(sg.pinhole(48, 32, (1.0, -1.5, 2.0),
                            sg.look_rotation(sg.yaw_pitch_forward(math.pi / 2.5, math.radians(40)))))
    return views


def entry_index(scene, refs):
    look = {(b.block_id, b.lod): k for k, b in enumerate(scene.blocks)}
    return [look[tuple(x)] for x in refs]


@pytest.fixture(scope="module")
def quad(have_gpu):
    import torch
    from paper_2312_16457_amd import Renderer
    scene = small_quad_city()
    r = Renderer(0).load_blocks(scene.blocks)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    return torch, scene, r, ob, occs, zt


def test_occupancy_of_merged_assets_bit_exact(quad):
    torch, scene, r, ob, occs, zt = quad
    for k, b in enumerate(scene.blocks):
        got = r.occupancy(b.block_id, b.lod)
        assert got.shape == occs[k].shape and np.array_equal(got, occs[k]), (b.block_id, b.lod)


def test_quadtree_selection_bitwise(quad):
    torch, scene, r, ob, occs, zt = quad
    views = views_small() + sg.aerial_views(12, 300, [(64, 48), (160, 90)], xy=(-2.0, 6.0), h=(0.5, 6.0),
                                            pitch=(0.0, 89.0))
    # cameras straight above an LOD-0 block at exactly a threshold above its top
    rng = np.random.default_rng(2)
    for bid in rng.choice(16, 8, replace=False):
        k0 = entry_index(scene, [(int(bid), 0)])[0]
        b = scene.blocks[k0]
        for dz in THR:
            eye = np.array([b.aabb_min[0] + 0.5, b.aabb_min[1] + 0.5, zt[k0] + dz], np.float32)
            views.append(sg.pinhole(64, 48, eye, sg.look_rotation((0.3, 0.2, -1.0))))
    mixed = 0
    for v in views:
        for cull in (True, False):
            ref = [(scene.blocks[k].block_id, scene.blocks[k].lod)
                   for k in O.select(v, scene.blocks, zt, THR, cull, quadtree=True)]
            got = r.select(v, thresholds=THR, cull=cull, quadtree=True)
            assert got == ref
            mixed += len({l for _, l in got}) > 1
    assert mixed > 20


@pytest.mark.parametrize("vi", range(7))
def test_quadtree_render_parity(quad, vi):
    torch, scene, r, ob, occs, zt = quad
    from paper_2312_16457_amd import F_GRAPH, F_PER_BLOCK
    v = views_small()[vi]
    w = sg.xavier_mlp(4)
    mlp = torch.tensor(w, device="cuda")
    p = sg.cityb_params()
    sel = r.select(v, thresholds=THR, cull=True, quadtree=True)
    out = r.render([v], [sel], p, mlp, counts=True)
    shuffled = r.render([v], [sel[::-1]], p, mlp, counts=True)  # the library orders the set itself
    per_block = r.render([v], [sel], p, mlp, counts=True, flags=F_PER_BLOCK)
    graph = r.render([v], [sel], p, mlp, counts=True, flags=F_GRAPH)
    torch.cuda.synchronize()
    for o in (shuffled, per_block, graph):
        for key in ("rgb", "trans", "counts"):
            assert torch.equal(o[key], out[key]), key
    ref = O.render(ob, occs, v, entry_index(scene, sel), p, w)
    assert ref["order_ok"].all()
    assert np.array_equal(out["counts"].cpu().numpy()[:, 0], ref["n_eval"])
    assert np.abs(out["rgb"].cpu().numpy() - ref["rgb"]).max() <= TOL
    assert np.abs(out["trans"].cpu().numpy() - ref["trans"]).max() <= TOL


def test_sparse_bricks_of_merged_assets_bitwise(quad):
    """Block-sparse grids of the non-cubic merged assets (bricks around each
    occupied cell) render the same bits as the dense grids."""
    torch, scene, r, ob, occs, zt = quad
    from paper_2312_16457_amd import F_SPARSE
    assert r.pack_bricks() > 0
    mlp = torch.tensor(sg.xavier_mlp(4), device="cuda")
    p = sg.cityb_params()
    for v in views_small()[:3] + views_small()[6:]:
        sel = r.select(v, thresholds=THR, cull=True, quadtree=True)
        a = r.render([v], [sel], p, mlp, counts=True)
        b = r.render([v], [sel], p, mlp, counts=True, flags=F_SPARSE)
        torch.cuda.synchronize()
        for key in ("rgb", "trans", "aux", "counts"):
            assert torch.equal(a[key], b[key]), key


def test_quadtree_with_per_block_mlps(quad):
    """Each merged asset has its own deferred MLP (the paper retrains one per
    merged block): per-block shading before the merge over a mixed-LOD set,
    against the oracle's per-block composite."""
    torch, scene, r, ob, occs, zt = quad
    mlps = np.stack([sg.random_mlp(300 + k, 0.6) for k in range(len(scene.blocks))]).astype(np.float32)
    bm = torch.tensor(mlps, device="cuda")
    p = sg.cityb_params()
    for vi in (0, 1, 6):
        v = views_small()[vi]
        sel = r.select(v, thresholds=THR, cull=True, quadtree=True)
        out = r.render([v], [sel], p, None, counts=True, block_mlp=bm)
        torch.cuda.synchronize()
        ref = O.render(ob, occs, v, entry_index(scene, sel), p, mlps.astype(np.float64), composite=O.BLOCK_MLP)
        assert np.array_equal(out["counts"].cpu().numpy()[:, 0], ref["n_eval"])
        assert np.abs(out["rgb"].cpu().numpy() - ref["rgb"]).max() <= TOL
        assert np.abs(out["trans"].cpu().numpy() - ref["trans"]).max() <= TOL


def test_invalid_sets_rejected(quad):
    torch, scene, r, ob, occs, zt = quad
    from paper_2312_16457_amd import CowError
    v = views_small()[0]
    mlp = torch.tensor(sg.xavier_mlp(4), device="cuda")
    with pytest.raises(CowError):  # LOD-1 asset (0) overlaps block 5
        r.render([v], [[(0, 1), (5, 0)]], sg.cityb_params(), mlp)


def test_quadtree_adjoint_on_merged_fp32_assets(have_gpu):
    import torch
    from paper_2312_16457_amd import Renderer
    scene = small_quad_city(sg.F32, seed=9)
    r = Renderer(0).load_blocks(scene.blocks)
    v = views_small()[0]  # LOD-0 blocks and merged LOD-1 assets
    p = sg.cityb_params()
    sel = r.select(v, thresholds=THR, cull=True, quadtree=True)
    assert len({l for _, l in sel}) > 1
    rng = np.random.default_rng(5)
    w = sg.random_mlp(6, 0.3)
    mlp = torch.tensor(w, device="cuda")
    out = r.render([v], [sel], p, mlp)
    g_rgb = rng.uniform(-1, 1, (v.n_pixels, 3))
    gg = [torch.zeros_like(t[0]) for t in r.textures]
    gp = [[torch.zeros_like(q) for q in t[1]] for t in r.textures]
    gm = torch.zeros(499, device="cuda")
    r.render_backward([v], [sel], p, mlp, out["aux"], torch.tensor(g_rgb, dtype=torch.float32, device="cuda"),
                      None, gg, gp, gm)
    torch.cuda.synchronize()
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    idx = entry_index(scene, sel)
    grads, gm_ref = O.adjoint(ob, occs, v, idx, p, w.astype(np.float64), O.pixels_of(v), g_rgb)
    merged_checked = 0
    for k, (g, ps) in grads.items():
        for a, b in [(gg[k], g)] + [(gp[k][i], ps[i]) for i in range(3)]:
            den = np.abs(b).max()
            if den == 0:
                assert not a.any().item()
                continue
            e = np.abs(a.cpu().numpy() - b).max() / den
            assert e <= 1e-3, (k, e)
        merged_checked += scene.blocks[k].lod > 0
    assert merged_checked > 0
    e = np.abs(gm.cpu().numpy() - gm_ref).max() / np.abs(gm_ref).max()
    assert e <= 1e-3


@pytest.fixture(scope="module")
def c3q(have_gpu):
    import torch
    from paper_2312_16457_amd import Renderer
    scene = sg.c3q_scene()
    r = Renderer(0).load_blocks(scene.blocks)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    return torch, scene, r, ob, occs, zt


def test_c3q_selection_and_sampled_parity(c3q):
    """The 8x8 city with merged 2x2 and 4x4 LOD assets, the 64 batched views:
    selection bitwise, the batched launch bitwise equal to per-block
    launches, sampled rows of several views against the oracle."""
    torch, scene, r, ob, occs, zt = c3q
    from paper_2312_16457_amd import F_PER_BLOCK
    views = sg.c4_views()
    thr = sg.QUADTREE_THRESHOLDS
    sets = []
    for v in views:
        ref = [(scene.blocks[k].block_id, scene.blocks[k].lod)
               for k in O.select(v, scene.blocks, zt, thr, True, quadtree=True)]
        got = r.select(v, thresholds=thr, cull=True, quadtree=True)
        assert got == ref
        sets.append(got)
    w = sg.xavier_mlp(3)
    mlp = torch.tensor(w, device="cuda")
    p = sg.cityb_params()
    batched = r.render(views, sets, p, mlp, counts=True)
    per_block = r.render(views, sets, p, mlp, counts=True, flags=F_PER_BLOCK)
    torch.cuda.synchronize()
    for key in ("rgb", "trans", "counts"):
        assert torch.equal(per_block[key], batched[key]), key
    off = 0
    for vi, v in enumerate(views):
        n = v.n_pixels
        if vi % 16 == 0:
            rows = np.array([0, v.H // 3, v.H - 1])
            pix = O.pixels_of(v, rows=rows)
            ref = O.render(ob, occs, v, entry_index(scene, sets[vi]), p, w, pix=pix)
            assert ref["order_ok"].all()
            lin = off + pix[:, 1] * v.W + pix[:, 0]
            assert np.array_equal(batched["counts"].cpu().numpy()[lin, 0], ref["n_eval"])
            assert np.abs(batched["rgb"].cpu().numpy()[lin] - ref["rgb"]).max() <= TOL
            assert np.abs(batched["trans"].cpu().numpy()[lin] - ref["trans"]).max() <= TOL
        off += n
