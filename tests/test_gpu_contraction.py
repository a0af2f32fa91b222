"""Contracted boundary blocks and the exterior they own (implementation
details, the contraction equation; Eq. "blocks" for ownership): the HIP
march against the oracle, element by element, with the sample counts
bit-exact (every decision on both sides is the same fp32 sequence)."""
import types

import numpy as np
import pytest

import oracle as O
from paper_2312_16457_amd import scenegen as sg

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_cuda(have_gpu):
    import torch
    return torch


def city(dtype, seed=7):
    scene = sg.make_scene(3, 3, ((16, 64, 8),), dtype, blobs_per_block=10, blob_z=(0, 0.3), seed=seed)
    return types.SimpleNamespace(blocks=sg.contract_boundary(scene.blocks))


VIEWS = {
    "outside_looking_in": ((1.5, -1.1, 1.3), (0.0, 2.6, -1.2)),
    "above_looking_out": ((1.5, 1.5, 1.4), (3.5, 2.5, -1.0)),
    "outside_looking_away": ((-0.5, 1.5, 0.5), (-1.0, 0.2, -0.1)),
}


def render_both(torch, sc, view, p, w, flags=0):
    from paper_2312_16457_amd import Renderer
    r = Renderer(0).load_blocks(sc.blocks)
    refs = [(b.block_id, b.lod) for b in sc.blocks]
    out = r.render([view], [refs], p, torch.tensor(w, device="cuda"), counts=True, flags=flags)
    torch.cuda.synchronize()
    ob = O.OracleScene(sc.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    ref = O.render(ob, occs, view, list(range(ob.n)), p, w)
    return out, ref


def check(out, ref):
    cnt = out["counts"].cpu().numpy()
    assert np.array_equal(cnt[:, 1], ref["n_march"]), "marched samples differ"
    assert np.array_equal(cnt[:, 0], ref["n_eval"]), "evaluated samples differ"
    for k in ("rgb", "trans", "aux"):
        e = np.abs(out[k].cpu().numpy() - ref[k]).max()
        assert e <= TOL, (k, e)


@pytest.mark.parametrize("name", sorted(VIEWS))
@pytest.mark.parametrize("dtype", [sg.U8, sg.F32])
def test_contracted_city_matches_oracle(torch_cuda, name, dtype):
    eye, fwd = VIEWS[name]
    view = sg.pinhole(37, 29, eye, sg.look_rotation(np.asarray(fwd)))
    p = sg.RenderParams(mode=1, ext_delta=1.0 / 64, ext_max_steps=512)
    sc = city(dtype)
    out, ref = render_both(torch_cuda, sc, view, p, sg.random_mlp(2, 0.7))
    print(name, dtype, "exterior-only samples:", int(ref["n_march"].sum()), flush=True)
    check(out, ref)
    # the exterior was sampled and changed the picture
    p0 = sg.RenderParams(mode=1)
    out0, ref0 = render_both(torch_cuda, sc, view, p0, sg.random_mlp(2, 0.7))
    check(out0, ref0)
    assert (ref["n_march"] > ref0["n_march"]).mean() > 0.3
    assert np.abs(ref["trans"] - ref0["trans"]).max() > 1e-3


def test_contracted_city_sparse_and_persistent(torch_cuda):
    from paper_2312_16457_amd import F_PERSISTENT, F_SPARSE
    eye, fwd = VIEWS["outside_looking_in"]
    view = sg.pinhole(33, 21, eye, sg.look_rotation(np.asarray(fwd)))
    p = sg.RenderParams(mode=1, ext_delta=1.0 / 48, ext_max_steps=300, t_min=0.0)
    sc = city(sg.U8, seed=9)
    for flags in (F_SPARSE, F_PERSISTENT):
        from paper_2312_16457_amd import Renderer
        r = Renderer(0).load_blocks(sc.blocks)
        if flags == F_SPARSE:
            r.pack_bricks()
        refs = [(b.block_id, b.lod) for b in sc.blocks]
        w = sg.random_mlp(4, 0.7)
        out = r.render([view], [refs], p, torch_cuda.tensor(w, device="cuda"), counts=True, flags=flags)
        torch_cuda.cuda.synchronize()
        ob = O.OracleScene(sc.blocks)
        ref = O.render(ob, [O.occupancy(ob, k) for k in range(ob.n)], view, list(range(ob.n)), p, w)
        check(out, ref)


def test_contracted_blocks_reject_unsupported_calls(torch_cuda):
    from paper_2312_16457_amd import F_PER_BLOCK, CowError, Renderer
    sc = city(sg.F32)
    r = Renderer(0).load_blocks(sc.blocks)
    refs = [(b.block_id, b.lod) for b in sc.blocks]
    view = sg.pinhole(16, 8, (1.5, -1.1, 1.3), sg.look_rotation(np.asarray((0.0, 2.6, -1.2))))
    mlp = torch_cuda.tensor(sg.random_mlp(2, 0.7), device="cuda")
    for p, flags in ((sg.RenderParams(mode=0, n_steps=64), 0), (sg.RenderParams(mode=1), F_PER_BLOCK)):
        with pytest.raises(CowError) as ei:
            r.render([view], [refs], p, mlp, flags=flags)
        assert ei.value.status == 4
    with pytest.raises(CowError) as ei:
        r.render([view], [refs], sg.RenderParams(mode=1, ext_delta=-1.0, ext_max_steps=8), mlp)
    assert ei.value.status == 1
    # a contracted block must span the scene's full height
    low = sg.contract_boundary([sg.homogeneous_block(block_id=0)])[0]
    top = sg.homogeneous_block(block_id=1, origin=(0, 0, 1))
    with pytest.raises(CowError) as ei:
        Renderer(0).load_blocks([low, top])
    assert ei.value.status == 1
