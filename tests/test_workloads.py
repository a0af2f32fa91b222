"""CPU checks of the synthetic workloads' structure (no GPU): block counts
per view after selection, view-set sizes, LOD mix."""
import numpy as np
import pytest

import oracle as O
from paper_2312_16457_amd import scenegen as sg


@pytest.fixture(scope="module")
def c3_small():
    # the 8x8x3-LOD layout at reduced texture resolution: selection only needs
    # the AABBs and each block's z_top, which the occupancy rule sets
    lods = ((32, 64, 16), (16, 32, 8), (8, 16, 4))
    scene = sg.make_scene(8, 8, lods, sg.U8, blobs_per_block=40, blob_z=(0.0, 0.3), seed=2)
    ob = O.OracleScene(scene.blocks)
    zt = [O.ztop(ob, k, O.occupancy(ob, k)) for k in range(ob.n)]
    return scene, zt


def test_c4_views_hold_4_to_40_blocks(c3_small):
    scene, zt = c3_small
    views = sg.c4_views()
    assert len(views) == 64
    res = {(v.W, v.H) for v in views}
    assert res <= set(sg.C4_RESOLUTIONS) and len(res) == 4
    counts = [len(O.select(v, scene.blocks, zt, thresholds=(2, 4, 8), cull=True)) for v in views]
    hist = np.bincount(counts)
    print("blocks per view histogram:", {i: int(c) for i, c in enumerate(hist) if c})
    assert min(counts) >= 4 and max(counts) <= 40, counts


def test_c3_views_and_lod_mix(c3_small):
    scene, zt = c3_small
    views = sg.c3_views()
    assert len(views) == 16 and all((v.W, v.H) == (1920, 1080) for v in views)
    lods = np.zeros(3, int)
    for v in views:
        for k in O.select(v, scene.blocks, zt, thresholds=(2, 4, 8), cull=True):
            lods[scene.blocks[k].lod] += 1
    assert (lods > 0).all(), lods  # every LOD is exercised


def test_contract_boundary_marks_the_edge_columns():
    """The contraction workload: of a 4x4 city's 16 unit blocks the 12 on the
    footprint's edge are contracted, the 4 inner ones stay plain, and the
    textures are untouched; merged (2x2) assets are never contracted."""
    from paper_2312_16457_amd import scenegen as sg
    scene = sg.make_scene(4, 4, ((8, 16, 4),), sg.U8, blobs_per_block=2, seed=3)
    out = sg.contract_boundary(scene.blocks)
    edge = [b.aabb_min[0] in (0, 3) or b.aabb_min[1] in (0, 3) for b in scene.blocks]
    assert [b.contracted for b in out] == edge and sum(edge) == 12
    assert all(a.grid is b.grid for a, b in zip(scene.blocks, out))
    merged = sg.merged_lods(scene.blocks, 4, 4, 2)
    big = [b for b in sg.contract_boundary(merged) if b.aabb_max[0] - b.aabb_min[0] > 1]
    assert big and not any(b.contracted for b in big)
