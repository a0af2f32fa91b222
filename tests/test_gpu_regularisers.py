"""GPU parity of the two regularisers of the training objective (Sec. 4.3)
against the fp64 oracle, which is pinned to closed forms and finite
differences in tests/test_oracle_pins.py.

Bars.  Opacity entropy per ray: |H - H_ref| <= 1e-4 + 1e-4 |H_ref|.  The
entropy's slope |log((1 - a) / a)| is at most 14 on the clamped range, and
the fp32 block transmittance of a few hundred samples carries ~1e-6 relative
error, so each block contributes well under 2e-5.  Gradients: normwise
1e-3 as for the render's adjoint.  Sparsity: the occupancy and block
decisions are exact, so alpha differs only by fp32 rounding (<= 1e-5
absolute); the loss sum by fp32 atomics (<= 1e-5 relative)."""
import numpy as np
import pytest

import oracle as O
from paper_2312_16457_amd import scenegen as sg

pytestmark = pytest.mark.gpu
REL = 1e-3


@pytest.fixture(scope="module")
def torch_cuda(have_gpu):
    import torch
    return torch


def small_scene(seed, dtype=sg.F32, shift=0.5):
    return sg.make_scene(2, 2, ((16, 32, 4),), dtype, blobs_per_block=10, blob_z=(0, 0.4), seed=seed, shift=shift)


def small_view(W=33, H=21):
    eye = (1.0, -1.0, 1.2)
    return sg.pinhole(W, H, eye, sg.look_rotation(np.array([1.0, 1.0, 0.2]) - eye))


def zero_grads(torch, r):
    gg = [torch.zeros_like(t[0]) for t in r.textures]
    gp = [[torch.zeros_like(p) for p in t[1]] for t in r.textures]
    return gg, gp


def compare_grads(gg, gp, grads, rel=REL):
    worst = 0.0
    for k, (g, ps) in grads.items():
        for a, b in [(gg[k], g)] + [(gp[k][i], ps[i]) for i in range(3)]:
            a = a.cpu().numpy()
            den = np.abs(b).max()
            if den == 0:
                assert np.abs(a).max() == 0
                continue
            e = np.abs(a - b).max() / den
            worst = max(worst, e)
            assert e <= rel, (k, e)
    return worst


@pytest.mark.parametrize("case", ["grid", "chord", "grid_tmin"])
def test_opacity_forward_parity(torch_cuda, case):
    torch = torch_cuda
    from paper_2312_16457_amd import Renderer
    if case == "chord":
        scene = sg.c1_scene()
        view = sg.c1_view().with_crop(40, 30, 48, 40)
        params = sg.c1_params()
    else:
        scene = small_scene(3, shift=0.0 if case == "grid_tmin" else 0.5)
        view = small_view()
        params = sg.RenderParams(mode=1, t_min=1e-3) if case == "grid_tmin" else sg.cityb_params()
    r = Renderer(0).load_blocks(scene.blocks)
    sets = [[(b.block_id, b.lod) for b in scene.blocks]]
    mlp = torch.tensor(sg.random_mlp(5, 0.6), device="cuda")
    out = r.render([view], sets, params, mlp, opacity=True, counts=True)
    plain = r.render([view], sets, params, mlp)
    torch.cuda.synchronize()
    # the regulariser leaves the render untouched
    assert torch.equal(out["rgb"], plain["rgb"]) and torch.equal(out["aux"], plain["aux"])
    H = out["opacity"].cpu().numpy().astype(np.float64)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    ref = O.opacity(ob, occs, view, list(range(ob.n)), params, O.pixels_of(view))
    err = np.abs(H - ref)
    assert (err <= 1e-4 + 1e-4 * np.abs(ref)).all(), (err.max(), int(err.argmax()))
    assert (ref > 0.1).sum() > 20  # semi-transparent blocks are exercised
    no_march = out["counts"].cpu().numpy()[:, 1] == 0
    assert (H[no_march] == 0).all() and no_march.sum() < len(H)


def test_opacity_launch_variants_bitwise(torch_cuda):
    torch = torch_cuda
    from paper_2312_16457_amd import F_GRAPH, F_PER_BLOCK, F_PERSISTENT, Renderer
    scene = small_scene(4)
    views = [small_view(), small_view(20, 17).with_crop(3, 2, 12, 11)]
    params = sg.cityb_params()
    r = Renderer(0).load_blocks(scene.blocks)
    sets = [[(b.block_id, b.lod) for b in scene.blocks]] * 2
    mlp = torch.tensor(sg.random_mlp(5, 0.6), device="cuda")
    base = r.render(views, sets, params, mlp, opacity=True)["opacity"].clone()
    for flags in (F_GRAPH, F_PERSISTENT, F_PER_BLOCK, F_GRAPH | F_PER_BLOCK):
        for _ in range(2):  # graph replays
            o = r.render(views, sets, params, mlp, opacity=True, flags=flags)["opacity"]
            torch.cuda.synchronize()
            assert torch.equal(o, base), flags


@pytest.mark.parametrize("with_rgb", [False, True])
def test_opacity_backward_parity(torch_cuda, with_rgb):
    torch = torch_cuda
    from paper_2312_16457_amd import Renderer
    scene = small_scene(6)
    view = small_view()
    params = sg.cityb_params()
    r = Renderer(0).load_blocks(scene.blocks)
    sets = [[(b.block_id, b.lod) for b in scene.blocks]]
    w = sg.random_mlp(5, 0.6)
    mlp = torch.tensor(w, device="cuda")
    out = r.render([view], sets, params, mlp)
    rng = np.random.default_rng(12)
    wo = rng.uniform(0.2, 1.5, view.n_pixels)
    g_rgb = rng.uniform(-1, 1, (view.n_pixels, 3)) if with_rgb else np.zeros((view.n_pixels, 3))
    gg, gp = zero_grads(torch, r)
    gm = torch.zeros(499, device="cuda")
    r.render_backward([view], sets, params, mlp, out["aux"], torch.tensor(g_rgb, dtype=torch.float32, device="cuda"),
                      None, gg, gp, gm, opacity_weight=torch.tensor(wo, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    grads, gm_ref = O.adjoint(ob, occs, view, list(range(ob.n)), params, w, O.pixels_of(view), g_rgb, None, wo)
    compare_grads(gg, gp, grads)
    if not with_rgb:
        assert not gm.any().item()
        for k in range(len(gg)):  # density channel only
            assert not gg[k][..., 1:].any().item()


def test_opacity_autograd(torch_cuda):
    torch = torch_cuda
    from paper_2312_16457_amd import Renderer, make_render_fn
    scene = small_scene(8)
    view = small_view(24, 16)
    params = sg.cityb_params()
    r = Renderer(0).load_blocks(scene.blocks)
    sets = [[(b.block_id, b.lod) for b in scene.blocks]]
    mlp = torch.tensor(sg.random_mlp(9, 0.5), device="cuda", requires_grad=True)
    tex = []
    for g, ps in r.textures:
        g.requires_grad_(True)
        for p in ps:
            p.requires_grad_(True)
        tex += [g] + ps
    fn = make_render_fn(with_opacity=True)
    rgb, trans, H = fn.apply(r, [view], sets, params, mlp, *tex)
    loss = 0.05 * H.mean()
    gs = torch.autograd.grad(loss, tex)
    gg, gp = zero_grads(torch, r)
    with torch.no_grad():
        out = r.render([view], sets, params, mlp.detach())
        r.render_backward([view], sets, params, mlp.detach(), out["aux"], torch.zeros_like(out["rgb"]), None, gg, gp,
                          None, opacity_weight=torch.full_like(out["trans"], 0.05 / view.n_pixels))
    torch.cuda.synchronize()
    assert (gs[0] - gg[0]).abs().max().item() <= 1e-6 * gg[0].abs().max().item()
    assert gg[0].abs().max().item() > 0


def sparsity_points(rng, n_in, lo, hi):
    pts = rng.uniform(lo, hi, (n_in, 3))
    # boundary cases: on a shared block face (x = 1 belongs to the block
    # above), on the scene's upper faces (outside), below the ground (outside)
    edge = np.array([[1.0, 0.5, 0.2], [0.5, 1.0, 0.2], [1.0, 1.0, 0.1], [2.0, 0.5, 0.2], [0.5, 0.5, -0.01],
                     [0.0, 0.0, 0.0], [1.999999, 1.999999, 0.999999]])
    return np.concatenate([pts, edge]).astype(np.float32)


@pytest.mark.parametrize("dtype", [sg.F32, sg.U8])
def test_sparsity_parity(torch_cuda, dtype):
    torch = torch_cuda
    from paper_2312_16457_amd import Renderer
    scene = small_scene(10, dtype=dtype)
    r = Renderer(0).load_blocks(scene.blocks)
    refs = [(b.block_id, b.lod) for b in scene.blocks]
    rng = np.random.default_rng(3)
    pts = sparsity_points(rng, 5000, (-0.2, -0.2, -0.1), (2.2, 2.2, 1.1))
    delta, weight = 1.0 / 64, 0.01
    grads_on = dtype == sg.F32
    gg, gp = zero_grads(torch, r) if grads_on else (None, None)
    loss, alpha = r.sparsity(refs, torch.tensor(pts, device="cuda"), delta, weight, alpha=True,
                             grad_grid=gg, grad_plane=gp)
    torch.cuda.synchronize()
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    L_ref, grads, a_ref = O.sparsity(ob, occs, list(range(ob.n)), pts, delta, weight, want_alpha=True,
                                     want_grad=grads_on)
    a = alpha.cpu().numpy()
    assert ((a == 0) == (a_ref == 0)).all()  # the same points fall in occupied cells
    assert np.abs(a - a_ref).max() <= 1e-5
    assert (a_ref > 0).sum() > 500 and (a_ref == 0).sum() > 500
    assert abs(loss.item() - L_ref) <= 1e-5 * L_ref
    if grads_on:
        compare_grads(gg, gp, grads)
        for k in range(len(gg)):
            assert not gg[k][..., 1:].any().item()


def test_sparsity_edges_and_autograd(torch_cuda):
    torch = torch_cuda
    from paper_2312_16457_amd import CowError, Renderer, make_sparsity_fn
    scene = small_scene(11)
    r = Renderer(0).load_blocks(scene.blocks)
    refs = [(b.block_id, b.lod) for b in scene.blocks]
    # no points: the loss is left as it was
    loss = torch.full((1,), 0.25, device="cuda")
    r.sparsity(refs, torch.zeros((0, 3), device="cuda"), 1.0 / 64, 1.0, loss=loss)
    # no entries: every alpha is zero
    pts = torch.tensor(sparsity_points(np.random.default_rng(5), 300, (0, 0, 0), (2, 2, 1)), device="cuda")
    l2, a2 = r.sparsity([], pts, 1.0 / 64, 1.0, alpha=True)
    torch.cuda.synchronize()
    assert loss.item() == 0.25 and l2.item() == 0.0 and not a2.any().item()
    # a subset of the entries: points of the others count as empty space
    l_sub, a_sub = r.sparsity(refs[:1], pts, 1.0 / 64, 1.0, alpha=True)
    l_all, a_all = r.sparsity(refs, pts, 1.0 / 64, 1.0, alpha=True)
    torch.cuda.synchronize()
    inside0 = ((pts < 1.0).all(dim=1) & (pts[:, 2] >= 0)).cpu()
    assert torch.equal(a_sub.cpu()[inside0], a_all.cpu()[inside0])
    assert not a_sub.cpu()[~inside0].any()
    with pytest.raises(CowError):
        r.sparsity([(99, 0)], pts, 1.0 / 64, 1.0)
    with pytest.raises(CowError):
        r.sparsity(refs, pts, 0.0, 1.0)
    # autograd: gradient of 3 * L equals the direct call with weight 3
    tex = []
    for g, ps in r.textures:
        g.requires_grad_(True)
        for p in ps:
            p.requires_grad_(True)
        tex += [g] + ps
    fn = make_sparsity_fn()
    L = fn.apply(r, refs, pts, 1.0 / 64, 0.5, *tex)
    gs = torch.autograd.grad(3.0 * L, tex)
    gg, gp = zero_grads(torch, r)
    r.sparsity(refs, pts, 1.0 / 64, 1.5, grad_grid=gg, grad_plane=gp)
    torch.cuda.synchronize()
    assert abs(L.item() - 0.5 * l_all.item()) <= 1e-6 * l_all.item()
    assert (gs[0] - gg[0]).abs().max().item() <= 1e-6 * gg[0].abs().max().item()
    assert gg[0].abs().max().item() > 0
