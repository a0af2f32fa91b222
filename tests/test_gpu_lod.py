"""GPU parity on the 8x8-block, 3-LOD scene: occupancy of every LOD and the
per-view selection bit-exact against the oracle, culling exact, sampled
pixels of full 1080p renders, and the 64-view batched launch bitwise equal
to per-view and per-block launches."""
import numpy as np
import pytest

import oracle as O
from paper_2312_16457_amd import scenegen as sg

pytestmark = pytest.mark.gpu
THR = (2.0, 4.0, 8.0)


@pytest.fixture(scope="module")
def c3(have_gpu):
    import torch
    from paper_2312_16457_amd import Renderer
    scene = sg.c3_scene()
    r = Renderer(0).load_blocks(scene.blocks)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    return torch, scene, r, ob, occs, zt


def entry_index(scene, refs):
    look = {(b.block_id, b.lod): k for k, b in enumerate(scene.blocks)}
    return [look[tuple(x)] for x in refs]


def test_occupancy_all_lods_bit_exact(c3):
    torch, scene, r, ob, occs, zt = c3
    for k, b in enumerate(scene.blocks):
        assert np.array_equal(r.occupancy(b.block_id, b.lod), occs[k]), (b.block_id, b.lod)


def test_selection_bitwise(c3):
    torch, scene, r, ob, occs, zt = c3
    rng = np.random.default_rng(5)
    views = sg.c3_views() + sg.c4_views() + sg.aerial_views(11, 400, [(640, 360), (96, 96)], xy=(-2, 10),
                                                            h=(0.5, 9.0), pitch=(0.0, 89.0))
    # cameras exactly on an LOD threshold: straight above a block centre at
    # z_top + 2 (or + 4), an exact fp32 distance, which must go to the coarser LOD
    for k in rng.choice(64, 40, replace=False):
        b = scene.blocks[entry_index(scene, [(int(k), 0)])[0]]
        k0 = entry_index(scene, [(int(k), 0)])[0]
        for dz in (2.0, 4.0):
            eye = np.array([b.aabb_min[0] + 0.5, b.aabb_min[1] + 0.5, zt[k0] + dz], np.float32)
            views.append(sg.pinhole(64, 48, eye, sg.look_rotation((0.3, 0.2, -1.0))))
    n_exact = 0
    for v in views:
        ref = [(scene.blocks[k].block_id, scene.blocks[k].lod) for k in O.select(v, scene.blocks, zt, THR, True)]
        got = r.select(v, thresholds=THR, cull=True)
        assert got == ref
        unc = [(scene.blocks[k].block_id, scene.blocks[k].lod) for k in O.select(v, scene.blocks, zt, THR, False)]
        assert r.select(v, thresholds=THR, cull=False) == unc
        n_exact += 1
    assert n_exact > 500


def test_c3_views_sampled_parity_and_culling(c3):
    torch, scene, r, ob, occs, zt = c3
    views = sg.c3_views()
    w = sg.xavier_mlp(2)
    mlp = torch.tensor(w, device="cuda")
    p = sg.cityb_params()
    for vi in (0, 5, 9, 14):
        v = views[vi]
        sel = r.select(v, thresholds=THR, cull=True)
        out = r.render([v], [sel], p, mlp, counts=True)
        # culling is exact: the unculled set renders the same bits
        allb = r.select(v, thresholds=THR, cull=False)
        assert len(allb) >= len(sel)
        out2 = r.render([v], [allb], p, mlp, counts=True)
        torch.cuda.synchronize()
        for key in ("rgb", "trans", "counts"):
            assert torch.equal(out[key], out2[key]), (vi, key)
        rows = np.array([0, 333, 700, 1079])
        pix = O.pixels_of(v, rows=rows)
        ref = O.render(ob, occs, v, entry_index(scene, sel), p, w, pix=pix)
        lin = pix[:, 1] * v.W + pix[:, 0]
        assert np.array_equal(out["counts"].cpu().numpy()[lin, 0], ref["n_eval"])
        assert np.abs(out["rgb"].cpu().numpy()[lin] - ref["rgb"]).max() <= 1e-4
        assert np.abs(out["trans"].cpu().numpy()[lin] - ref["trans"]).max() <= 1e-4
        assert ref["order_ok"].all()


def test_c4_batched_equals_per_view_and_per_block(c3):
    """The 64-view batch (mixed resolutions, 8-38 blocks each) in one launch,
    in a replayed graph, view by view, and one launch per view per block:
    bitwise identical; sampled pixels of several views against the oracle."""
    torch, scene, r, ob, occs, zt = c3
    from paper_2312_16457_amd import F_GRAPH, F_PER_BLOCK
    views = sg.c4_views()
    sets = [r.select(v, thresholds=THR, cull=True) for v in views]
    w = sg.xavier_mlp(3)
    mlp = torch.tensor(w, device="cuda")
    p = sg.cityb_params()
    batched = r.render(views, sets, p, mlp, counts=True)
    graph = r.render(views, sets, p, mlp, counts=True, flags=F_GRAPH)
    graph2 = r.render(views, sets, p, mlp, counts=True, flags=F_GRAPH)
    per_block = r.render(views, sets, p, mlp, counts=True, flags=F_PER_BLOCK)
    torch.cuda.synchronize()
    for o in (graph, graph2, per_block):
        for key in ("rgb", "trans", "aux", "counts"):
            assert torch.equal(o[key], batched[key]), key
    off = 0
    for vi, v in enumerate(views):
        n = v.n_pixels
        if vi % 13 == 0:
            single = r.render([v], [sets[vi]], p, mlp, counts=True)
            torch.cuda.synchronize()
            assert torch.equal(single["rgb"], batched["rgb"][off:off + n])
            assert torch.equal(single["counts"], batched["counts"][off:off + n])
            rows = np.array([0, v.H // 2, v.H - 1])
            pix = O.pixels_of(v, rows=rows)
            ref = O.render(ob, occs, v, entry_index(scene, sets[vi]), p, w, pix=pix)
            lin = off + pix[:, 1] * v.W + pix[:, 0]
            assert np.array_equal(batched["counts"].cpu().numpy()[lin, 0], ref["n_eval"])
            assert np.abs(batched["rgb"].cpu().numpy()[lin] - ref["rgb"]).max() <= 1e-4
        off += n


def test_autotune_invariance(c3):
    torch, scene, r, ob, occs, zt = c3
    views = sg.c4_views()[:6]
    sets = [r.select(v, thresholds=THR, cull=True) for v in views]
    mlp = torch.tensor(sg.xavier_mlp(3), device="cuda")
    p = sg.cityb_params()
    r.set_config(8, 4, -1)
    base = r.render(views, sets, p, mlp)
    cfg = r.autotune(views, sets, p, mlp)
    tuned = r.render(views, sets, p, mlp)
    torch.cuda.synchronize()
    assert torch.equal(base["rgb"], tuned["rgb"]) and torch.equal(base["aux"], tuned["aux"])
    r.set_config(8, 4, -1)
    print("autotuned config", cfg)


def test_every_launch_configuration_bitwise(c3):
    """Every configuration the autotuner may pick (packet width 4-32, 1-4
    waves per workgroup, persistent or not) renders the same bits, forward
    counts included, for a batch of views of mixed size and block counts."""
    torch, scene, r, ob, occs, zt = c3
    views = [v.with_crop(0, 0, min(v.W, 200), min(v.H, 120)) for v in sg.c4_views()[:5]]
    sets = [r.select(v, thresholds=THR, cull=True) for v in views]
    mlp = torch.tensor(sg.xavier_mlp(3), device="cuda")
    p = sg.cityb_params()
    r.set_config(8, 4, -1)
    base = r.render(views, sets, p, mlp, counts=True)
    torch.cuda.synchronize()
    for persistent in (0, 1):
        for tw in (4, 8, 16, 32):
            for wv in (1, 2, 4):
                r.set_config(tw, wv, persistent)
                o = r.render(views, sets, p, mlp, counts=True)
                torch.cuda.synchronize()
                for key in ("rgb", "trans", "aux", "counts"):
                    assert torch.equal(o[key], base[key]), (tw, wv, persistent, key)
    r.set_config(8, 4, -1)
