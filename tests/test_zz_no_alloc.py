"""cow_render_noalloc, the render entry point for callers that cannot
allocate device memory, against cow_render: the same kernels over tables
held in the library's fixed scratch instead of a workspace, so the same
bits.  Two calls in a row, the second smaller than the first (the scratch
keeps the first call's tables beyond what the second writes), one of them
with the persistent launch (whose counters the call clears); the limits are
refused before anything is enqueued."""
import numpy as np
import pytest

from paper_2312_16457_amd import scenegen as sg

pytestmark = pytest.mark.gpu


def _view(W, H, eye, target):
    return sg.pinhole(W, H, eye, sg.look_rotation(np.asarray(target, float) - np.asarray(eye, float)))


def test_noalloc_matches_render_on_two_calls(have_gpu):
    import torch
    from paper_2312_16457_amd import F_PERSISTENT, Renderer
    scene = sg.make_scene(3, 3, ((16, 64, 8),), sg.U8, blobs_per_block=10, blob_z=(0.0, 0.3), seed=7)
    r = Renderer(0).load_blocks(scene.blocks)
    refs = [(b.block_id, b.lod) for b in scene.blocks]
    mlp = torch.tensor(sg.xavier_mlp(2), device="cuda")
    p = sg.cityb_params()
    first = ([_view(64, 48, (1.5, -1.1, 1.3), (1.5, 1.5, 0.1)), _view(40, 24, (3.6, 1.4, 1.1), (1.0, 1.6, 0.2))],
             [refs, refs[:6]], 0)
    second = ([_view(24, 16, (0.4, 2.9, 0.9), (1.8, 1.0, 0.1))], [refs[:4]], F_PERSISTENT)
    for views, sets, flags in (first, second):
        ref = r.render(views, sets, p, mlp, counts=True, flags=flags)
        out = {k: torch.full_like(ref[k], float("nan")) for k in ("rgb", "trans", "aux")}
        out["counts"] = torch.full_like(ref["counts"], -1)
        r.render_noalloc(views, sets, p, mlp, out, flags=flags)
        torch.cuda.synchronize()
        print("noalloc call:", len(views), "views,", ref["rgb"].shape[0], "pixels, flags", flags, flush=True)
        for k in ("rgb", "trans", "aux", "counts"):
            assert torch.equal(out[k], ref[k]), k
        assert int(ref["counts"][:, 0].sum()) > 0


def test_noalloc_fp32_blocks_default_launch(have_gpu):
    """fp32 blocks take persistent launches by default: their work counters
    live in the scratch too (two calls, the second smaller)."""
    import torch
    from paper_2312_16457_amd import Renderer
    scene = sg.make_scene(2, 2, ((16, 32, 4),), sg.F32, blobs_per_block=10, blob_z=(0.0, 0.4), seed=8, shift=2.0)
    r = Renderer(0).load_blocks(scene.blocks)
    assert r.get_config() == (8, 4, -1)
    refs = [(b.block_id, b.lod) for b in scene.blocks]
    mlp = torch.tensor(sg.xavier_mlp(3), device="cuda")
    p = sg.cityb_params()
    calls = (([_view(48, 40, (1.0, -1.1, 1.3), (1.0, 1.0, 0.1))], [refs]),
             ([_view(16, 12, (2.6, 1.0, 1.0), (0.8, 1.1, 0.2))], [refs[:2]]))
    for views, sets in calls:
        ref = r.render(views, sets, p, mlp, counts=True)
        out = {k: torch.full_like(ref[k], float("nan")) for k in ("rgb", "trans", "aux")}
        out["counts"] = torch.full_like(ref["counts"], -1)
        r.render_noalloc(views, sets, p, mlp, out)
        torch.cuda.synchronize()
        print("noalloc fp32 call:", ref["rgb"].shape[0], "pixels", flush=True)
        for k in ("rgb", "trans", "aux", "counts"):
            assert torch.equal(out[k], ref[k]), k
        assert int(ref["counts"][:, 0].sum()) > 0


def test_noalloc_limits_are_refused(have_gpu):
    import torch
    from paper_2312_16457_amd import F_GRAPH, CowError, Renderer
    scene = sg.make_scene(1, 1, ((16, 32, 4),), sg.U8, blobs_per_block=4, seed=3)
    r = Renderer(0).load_blocks(scene.blocks)
    mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
    p = sg.cityb_params()
    v = _view(8, 8, (0.5, -1.0, 0.8), (0.5, 0.5, 0.2))

    def outputs(n):
        return dict(rgb=torch.zeros((n, 3), device="cuda"), trans=torch.zeros(n, device="cuda"),
                    aux=torch.zeros((n, 8), device="cuda"))
    with pytest.raises(CowError) as ei:  # more views than the scratch holds
        r.render_noalloc([v] * 257, [[(0, 0)]] * 257, p, mlp, outputs(257 * 64))
    assert ei.value.status == 1
    o = outputs(64)
    o["aux"] = None
    with pytest.raises(CowError) as ei:  # aux is required
        r.render_noalloc([v], [[(0, 0)]], p, mlp, o)
    assert ei.value.status == 1
    with pytest.raises(CowError) as ei:  # no graph replay
        r.render_noalloc([v], [[(0, 0)]], p, mlp, outputs(64), flags=F_GRAPH)
    assert ei.value.status == 4
    # 256 views is within the limit and renders like cow_render
    ref = r.render([v] * 256, [[(0, 0)]] * 256, p, mlp)
    out = outputs(256 * 64)
    r.render_noalloc([v] * 256, [[(0, 0)]] * 256, p, mlp, out)
    torch.cuda.synchronize()
    assert torch.equal(out["rgb"], ref["rgb"]) and torch.equal(out["trans"], ref["trans"])
