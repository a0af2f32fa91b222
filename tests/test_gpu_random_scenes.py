"""Seeded random sweep of the forward path: small scenes of random size,
texel type (uint8 / fp32), grid and occupancy resolution, blob count and
height, with or without merged 2x2 LOD assets (quadtree selection), seen
from random cameras (a fifth of them along a coordinate axis) with or
without early termination.

Bars: rgb and transmittance within 1e-4 of the oracle; the render with
occupancy-pyramid jumps bitwise equal to the one-step march (COW_F_FLAT_OCC).
Sample counts: bit-exact without early termination.  With t_min > 0 the
kernel compares its fp32 transmittance with t_min and the oracle its fp64
one, so where the two straddle t_min a ray may stop one evaluated sample
earlier or later: at most max(1, 1e-3 of the rays) differ, each by one
evaluated sample, and every other ray has both counts equal."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2312_16457_amd import scenegen as sg

pytestmark = pytest.mark.gpu
TOL = 1e-4


def random_scene(rng):
    dtype = sg.U8 if rng.random() < 0.6 else sg.F32
    occ = int(rng.choice([2, 4, 8, 16]))
    R = max(int(rng.choice([16, 32])), occ)
    nb = int(rng.integers(1, 4))
    scene = sg.make_scene(nb, nb, ((R, 4 * R, occ),), dtype, blobs_per_block=int(rng.integers(1, 8)),
                          blob_z=(0.0, float(rng.uniform(0.3, 1.0))), blob_s=(0.03, 0.12),
                          seed=int(rng.integers(1 << 30)))
    if nb >= 2 and rng.random() < 0.5:
        scene = sg.Scene(nb, nb, scene.blocks + sg.merged_lods(scene.blocks, nb, nb, 2, dtype=dtype))
    return scene, nb


def random_view(rng, nb):
    eye = np.array([rng.uniform(-1, nb + 1), rng.uniform(-1, nb + 1), rng.uniform(0.05, 2.5)])
    fwd = np.array([rng.uniform(0, nb), rng.uniform(0, nb), rng.uniform(0, 0.5)]) - eye
    if rng.random() < 0.2:  # along an axis, exactly or nearly
        fwd = np.zeros(3)
        fwd[int(rng.integers(3))] = rng.choice([-1.0, 1.0])
        if rng.random() < 0.5:
            fwd += 1e-7 * rng.standard_normal(3)
    if abs(fwd[2]) > 0.999 * np.linalg.norm(fwd):
        fwd[0] += 1e-3  # keep the camera's up vector usable
    return sg.pinhole(int(rng.integers(8, 40)), int(rng.integers(8, 40)), eye, sg.look_rotation(fwd))


def check_counts(cnt, ref, t_min):
    if t_min == 0.0:
        assert np.array_equal(cnt[:, 0], ref["n_eval"])
        assert np.array_equal(cnt[:, 1], ref["n_march"])
        return
    diff = cnt[:, 0] != ref["n_eval"]
    assert diff.sum() <= max(1, int(1e-3 * len(diff))), int(diff.sum())
    assert np.abs(cnt[:, 0] - ref["n_eval"]).max() <= 1
    assert np.array_equal(cnt[~diff, 1], ref["n_march"][~diff])


@pytest.mark.parametrize("seed", [11, 12])
def test_random_scenes_and_cameras(have_gpu, seed):
    import torch
    from paper_2312_16457_amd import F_FLAT_OCC, Renderer
    rng = np.random.default_rng(seed)
    cases = 0
    for _ in range(12):
        scene, nb = random_scene(rng)
        r = Renderer(0).load_blocks(scene.blocks)
        ob = O.OracleScene(scene.blocks)
        occs = [O.occupancy(ob, k) for k in range(ob.n)]
        look = {(b.block_id, b.lod): k for k, b in enumerate(scene.blocks)}
        quad = len({b.lod for b in scene.blocks}) > 1
        w = sg.xavier_mlp(int(rng.integers(100)))
        mlp = torch.tensor(w, device="cuda")
        for _ in range(4):
            v = random_view(rng, nb)
            sel = r.select(v, thresholds=(1.5, 3.0) if quad else (1e30,), cull=True, quadtree=quad)
            p = sg.cityb_params()
            if rng.random() < 0.3:
                p = dataclasses.replace(p, t_min=float(rng.choice([1e-3, 0.05, 0.3])))
            if not sel:
                continue
            out = r.render([v], [sel], p, mlp, counts=True)
            flat = r.render([v], [sel], p, mlp, counts=True, flags=F_FLAT_OCC)
            torch.cuda.synchronize()
            for key in ("rgb", "trans", "counts"):
                assert torch.equal(out[key], flat[key]), key
            ref = O.render(ob, occs, v, [look[tuple(x)] for x in sel], p, w)
            cnt = out["counts"].cpu().numpy()
            check_counts(cnt, ref, p.t_min)
            assert np.abs(out["rgb"].cpu().numpy() - ref["rgb"]).max() <= TOL
            assert np.abs(out["trans"].cpu().numpy() - ref["trans"]).max() <= TOL
            cases += 1
    assert cases >= 30
