"""The per-block composites the forward hands to the backward (block_aux):
what the forward writes, and that the adjoint reading them gives the
gradients of the adjoint that re-composites each block itself.

Bars: the slots re-merged front to back give the forward's aux and
transmittance to fp32 rounding (1e-6); slots past a view's set and pixels
of other calls are untouched; gradients with and without the buffer agree
to 1e-6 relative (only the order of the fp32 atomic sums differs)."""
import numpy as np
import pytest

from paper_2312_16457_amd import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda(have_gpu):
    import torch
    return torch


def small_scene(dtype, seed):
    return sg.make_scene(2, 2, ((16, 32, 4),), dtype, blobs_per_block=10, blob_z=(0, 0.4), seed=seed, shift=1.0)


def views():
    eye = (1.0, -1.0, 1.2)
    return [sg.pinhole(33, 21, eye, sg.look_rotation(np.array([1.0, 1.0, 0.2]) - eye)),
            sg.pinhole(16, 12, (2.5, 1.0, 0.6), sg.look_rotation((-1.0, 0.1, -0.2)))]


@pytest.mark.parametrize("graph", [False, True])
def test_block_aux_content(torch_cuda, graph):
    torch = torch_cuda
    from paper_2312_16457_amd import F_GRAPH, Renderer
    scene = small_scene(sg.F32, 4)
    r = Renderer(0).load_blocks(scene.blocks)
    vs = views()
    sets = [[(b.block_id, 0) for b in scene.blocks], [(scene.blocks[1].block_id, 0), (scene.blocks[3].block_id, 0)]]
    mlp = torch.tensor(sg.random_mlp(2, 0.5), device="cuda")
    n_pix = sum(v.n_pixels for v in vs)
    slots = 5  # one more than the largest set: the last slot is never written
    ba = torch.full((n_pix, slots, 8), 7.0, device="cuda")
    out = r.render(vs, sets, sg.cityb_params(), mlp, block_aux=ba, flags=F_GRAPH if graph else 0)
    if graph:  # the replayed graph writes the buffer too
        ba.fill_(7.0)
        out = r.render(vs, sets, sg.cityb_params(), mlp, block_aux=ba, flags=F_GRAPH)
    torch.cuda.synchronize()
    b = ba.cpu().numpy()
    aux, trans = out["aux"].cpu().numpy(), out["trans"].cpu().numpy()
    p0 = 0
    for v, s in zip(vs, sets):
        blk = b[p0:p0 + v.n_pixels]
        assert np.all(blk[:, len(s):] == 7.0)  # slots past the set untouched
        T = np.ones(v.n_pixels, np.float64)
        A = np.zeros((v.n_pixels, 7), np.float64)
        marched = 0
        for j in range(len(s)):
            Tk = blk[:, j, 7].astype(np.float64)
            Ak = blk[:, j, :7].astype(np.float64)
            none = Tk == -1.0
            assert np.all((Tk >= 0.0) & (Tk <= 1.0) | none)
            assert np.all(Ak[none] == 0.0)
            marched += int((~none).sum())
            Tk = np.where(none, 1.0, Tk)
            A += T[:, None] * Ak
            T *= Tk
        assert marched > 0
        np.testing.assert_allclose(T, trans[p0:p0 + v.n_pixels], atol=1e-6)
        np.testing.assert_allclose(A, aux[p0:p0 + v.n_pixels, :7], atol=1e-6)
        np.testing.assert_allclose(T, aux[p0:p0 + v.n_pixels, 7], atol=1e-6)
        p0 += v.n_pixels


def grads(torch, r, vs, sets, params, mlp, out, g_rgb, w_op, bm, block_aux):
    gg = [torch.zeros_like(t[0]) for t in r.textures]
    gp = [[torch.zeros_like(q) for q in t[1]] for t in r.textures]
    gm = None if bm is not None else torch.zeros(499, device="cuda")
    gbm = None if bm is None else torch.zeros_like(bm)
    r.render_backward(vs, sets, params, mlp, out["aux"], g_rgb, None, gg, gp, gm, opacity_weight=w_op,
                      block_mlp=bm, grad_block_mlp=gbm, block_aux=block_aux)
    torch.cuda.synchronize()
    return [t for e in range(len(gg)) for t in [gg[e]] + gp[e]] + [gm if bm is None else gbm]


@pytest.mark.parametrize("case", ["block_mlp", "opacity", "block_mlp_opacity_tmin"])
def test_backward_from_block_aux(torch_cuda, case):
    torch = torch_cuda
    from paper_2312_16457_amd import Renderer
    scene = small_scene(sg.F32, 5)
    r = Renderer(0).load_blocks(scene.blocks)
    vs = views()
    sets = [[(b.block_id, 0) for b in scene.blocks], [(scene.blocks[1].block_id, 0), (scene.blocks[3].block_id, 0)]]
    params = sg.RenderParams(mode=1, t_min=1e-3) if case.endswith("tmin") else sg.cityb_params()
    n_pix = sum(v.n_pixels for v in vs)
    rng = np.random.default_rng(6)
    bm = None
    mlp = torch.tensor(sg.random_mlp(3, 0.6), device="cuda")
    if case.startswith("block_mlp"):
        bm = torch.tensor(np.stack([sg.random_mlp(40 + k, 0.6) for k in range(len(scene.blocks))]).astype(np.float32),
                          device="cuda")
        mlp = None
    w_op = None
    if "opacity" in case:
        w_op = torch.tensor(rng.uniform(0.2, 1.0, n_pix), dtype=torch.float32, device="cuda")
    ba = torch.zeros((n_pix, 4, 8), device="cuda")
    out = r.render(vs, sets, params, mlp, block_mlp=bm, block_aux=ba)
    g_rgb = torch.tensor(rng.uniform(-1, 1, (n_pix, 3)), dtype=torch.float32, device="cuda")
    ref = grads(torch, r, vs, sets, params, mlp, out, g_rgb, w_op, bm, None)
    got = grads(torch, r, vs, sets, params, mlp, out, g_rgb, w_op, bm, ba)
    nonzero = 0
    for a, b in zip(got, ref):
        scale = b.abs().max().item()
        if scale == 0:
            assert a.abs().max().item() == 0
            continue
        nonzero += 1
        assert (a - b).abs().max().item() <= 1e-6 * scale
    assert nonzero >= 8


def test_block_aux_refused(torch_cuda):
    torch = torch_cuda
    from paper_2312_16457_amd import CowError, Renderer
    from paper_2312_16457_amd.binding import COW_E_INVALID, COW_E_UNSUPPORTED
    scene = small_scene(sg.F32, 4)
    r = Renderer(0).load_blocks(scene.blocks)
    v = views()[0]
    s = [(b.block_id, 0) for b in scene.blocks]
    mlp = torch.tensor(sg.random_mlp(2, 0.5), device="cuda")
    small = torch.zeros((v.n_pixels, 3, 8), device="cuda")  # four blocks in the set
    with pytest.raises(CowError) as ei:
        r.render([v], [s], sg.cityb_params(), mlp, block_aux=small)
    assert ei.value.status == COW_E_INVALID
    raw = torch.zeros(v.n_pixels * 4 * 8 + 64, device="cuda")
    off = (-raw.data_ptr() // 4) % 16 + 1  # 4 bytes past a 64-byte boundary
    shifted = raw[off:off + v.n_pixels * 4 * 8].view(v.n_pixels, 4, 8)
    with pytest.raises(CowError) as ei:
        r.render([v], [s], sg.cityb_params(), mlp, block_aux=shifted)
    assert ei.value.status == COW_E_INVALID
    # uint8 blocks take no part in the backward, so they hand nothing to it
    u8 = small_scene(sg.U8, 4)
    ru = Renderer(0).load_blocks(u8.blocks)
    with pytest.raises(CowError) as ei:
        ru.render([v], [s], sg.cityb_params(), mlp, block_aux=torch.zeros((v.n_pixels, 4, 8), device="cuda"))
    assert ei.value.status == COW_E_UNSUPPORTED


def test_block_aux_every_launch_form(torch_cuda):
    """Fused, graph-replayed, persistent, one launch per view per block, and
    the entry point that allocates nothing write the same per-block
    composites, bit for bit."""
    torch = torch_cuda
    from paper_2312_16457_amd import F_GRAPH, F_PER_BLOCK, F_PERSISTENT, Renderer
    scene = small_scene(sg.F32, 4)
    r = Renderer(0).load_blocks(scene.blocks)
    vs = views()
    sets = [[(b.block_id, 0) for b in scene.blocks], [(scene.blocks[1].block_id, 0), (scene.blocks[3].block_id, 0)]]
    mlp = torch.tensor(sg.random_mlp(2, 0.5), device="cuda")
    n_pix = sum(v.n_pixels for v in vs)
    got = []
    for flags in (0, F_GRAPH, F_PERSISTENT, F_PER_BLOCK):
        ba = torch.full((n_pix, 4, 8), 7.0, device="cuda")
        r.render(vs, sets, sg.cityb_params(), mlp, flags=flags, block_aux=ba)
        got.append(ba)
    out = r.render(vs, sets, sg.cityb_params(), mlp)
    ba = torch.full((n_pix, 4, 8), 7.0, device="cuda")
    r.render_noalloc(vs, sets, sg.cityb_params(), mlp, out, block_aux=ba)
    got.append(ba)
    torch.cuda.synchronize()
    for b in got[1:]:
        assert torch.equal(b, got[0])
