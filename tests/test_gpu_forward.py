"""GPU forward parity: the HIP path through the C ABI against the CPU oracle.

Bars: occupancy, LOD selection, block order and per-pixel sample counts are
bit-exact; rgb and transmittance within 1e-4 max-abs (fp32 kernel vs fp64
oracle); batched, per-block, persistent, graph-replayed, sparse and
autotuned launches are bitwise identical to the fused launch."""
import math

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


def make_renderer(blocks):
    from paper_2312_16457_amd import Renderer
    return Renderer(0).load_blocks(blocks)


def all_refs(scene):
    return [(b.block_id, b.lod) for b in scene.blocks if b.lod == 0]


def check_against_oracle(torch, r, scene, view, params, w, sets_gpu, set_idx, pix_rows=None, tol=TOL):
    mlp = torch.tensor(w, device="cuda")
    out = r.render([view], [sets_gpu], params, mlp, counts=True)
    torch.cuda.synchronize()
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    pix = O.pixels_of(view) if pix_rows is None else O.pixels_of(view, rows=pix_rows)
    ref = O.render(ob, occs, view, set_idx, params, w, pix=pix)
    x0, y0, wd, _ = view.crop
    lin = (pix[:, 1] - y0) * wd + (pix[:, 0] - x0)
    rgb = out["rgb"].cpu().numpy()[lin]
    tr = out["trans"].cpu().numpy()[lin]
    cnt = out["counts"].cpu().numpy()[lin]
    assert np.array_equal(cnt[:, 0], ref["n_eval"]), "evaluated samples differ"
    assert np.array_equal(cnt[:, 1], ref["n_march"]), "marched samples differ"
    e_rgb = np.abs(rgb - ref["rgb"]).max()
    e_t = np.abs(tr - ref["trans"]).max()
    assert e_rgb <= tol and e_t <= tol, (e_rgb, e_t)
    aux = out["aux"].cpu().numpy()[lin]
    assert np.abs(aux - ref["aux"]).max() <= tol
    return out, ref, e_rgb, e_t


# ---------------------------------------------------------------------------
def test_occupancy_bit_exact_small(torch_cuda):
    for dtype in (sg.F32, sg.U8):
        scene = sg.make_scene(2, 2, ((16, 64, 8), (8, 32, 4)), dtype, blobs_per_block=8, blob_z=(0, 0.3), seed=4)
        r = make_renderer(scene.blocks)
        ob = O.OracleScene(scene.blocks)
        for k, b in enumerate(scene.blocks):
            ref = O.occupancy(ob, k)
            assert 0 < ref.mean() < 1
            assert np.array_equal(r.occupancy(b.block_id, b.lod), ref), (dtype, k)


def test_c1_single_block_chord_mode(torch_cuda):
    scene, view, params = sg.c1_scene(), sg.c1_view(), sg.c1_params()
    r = make_renderer(scene.blocks)
    ob = O.OracleScene(scene.blocks)
    assert np.array_equal(r.occupancy(0, 0), O.occupancy(ob, 0))
    w = sg.xavier_mlp(0)
    check_against_oracle(torch_cuda, r, scene, view, params, w, [(0, 0)], [0])


def test_homogeneous_closed_form(torch_cuda):
    """P1 on the GPU: T = exp(-sigma L), C_d = (1 - T) c for axis rays."""
    torch = torch_cuda
    b = sg.homogeneous_block(sigma=2.0)
    r = make_renderer([b])
    v = sg.View(1, 1, np.array([-0.25, 0.5, 0.5], np.float32), sg.look_rotation((1.0, 0.0, 0.0)), 1.0, 1.0, 0.5, 0.5)
    out = r.render([v], [[(0, 0)]], sg.RenderParams(mode=1), torch.zeros(499, device="cuda"), counts=True)
    g = b.grid[0, 0, 0].astype(np.float64)
    T = math.exp(-math.exp(g[0]))
    c = 1 / (1 + np.exp(-g[1:4]))
    assert out["counts"][0, 0].item() == 512
    assert abs(out["trans"][0].item() - T) <= TOL
    np.testing.assert_allclose(out["aux"][0, :3].cpu().numpy(), (1 - T) * c, atol=TOL)
    np.testing.assert_allclose(out["rgb"][0].cpu().numpy(), (1 - T) * c + 0.5, atol=TOL)


@pytest.mark.parametrize("dtype", [sg.U8, sg.F32])
def test_small_city_grid_mode(torch_cuda, dtype):
    """Several tiles and a ragged edge (37 x 29), 3x3 blocks, both dtypes."""
    scene = sg.make_scene(3, 3, ((16, 64, 8),), dtype, blobs_per_block=10, blob_z=(0, 0.3), seed=7)
    view = sg.pinhole(37, 29, (1.5, -1.1, 1.3), sg.look_rotation(np.array([1.5, 1.5, 0.1]) - [1.5, -1.1, 1.3]))
    r = make_renderer(scene.blocks)
    w = sg.random_mlp(2, 0.7)
    refs = all_refs(scene)
    ob_set = list(range(len(scene.blocks)))
    _, ref, _, _ = check_against_oracle(torch_cuda, r, scene, view, sg.cityb_params(), w, refs, ob_set)
    assert ref["n_eval"].sum() > 10000


def test_empty_crop_and_empty_set(torch_cuda):
    torch = torch_cuda
    scene = sg.make_scene(2, 2, ((8, 16, 4),), sg.U8, blobs_per_block=4, seed=1)
    r = make_renderer(scene.blocks)
    v = sg.pinhole(16, 16, (1.0, -1.0, 1.0), sg.look_rotation((0.0, 1.0, -0.5)))
    mlp = torch.tensor(sg.random_mlp(0, 0.5), device="cuda")
    # an empty set renders T = 1, C_d = 0: rgb = sigmoid(Phi(0, 0, d))
    out = r.render([v, v.with_crop(3, 4, 0, 5), v.with_crop(2, 2, 5, 3)], [[], [(0, 0)], []],
                   sg.cityb_params(), mlp)
    torch.cuda.synchronize()
    assert out["rgb"].shape[0] == 16 * 16 + 15
    assert torch.all(out["trans"] == 1.0)
    d = O.pixels_of(v)
    ref = []
    for (i, j) in d[:3]:
        x = (np.float32(i) + np.float32(0.5) - np.float32(v.cx)) / np.float32(v.fx)
        y = (np.float32(j) + np.float32(0.5) - np.float32(v.cy)) / np.float32(v.fy)
        u = v.R.astype(np.float64) @ np.array([x, y, 1.0])
        ref.append(O.mlp(sg.random_mlp(0, 0.5), np.concatenate([np.zeros(7), u / np.linalg.norm(u)])))
    np.testing.assert_allclose(out["rgb"][:3].cpu().numpy(), np.array(ref), atol=1e-5)


# ---------------------------------------------------------------------------
# the 4x4-block 1080p workload (the benchmark's configuration)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c2(torch_cuda):
    scene = sg.c2_scene()
    r = make_renderer(scene.blocks)
    return scene, r


def test_c2_occupancy_and_selection(c2):
    scene, r = c2
    ob = O.OracleScene(scene.blocks)
    zt = []
    for k, b in enumerate(scene.blocks):
        ref = O.occupancy(ob, k)
        assert np.array_equal(r.occupancy(b.block_id, b.lod), ref), k
        zt.append(O.ztop(ob, k, ref))
    v = sg.c2_view()
    sel_ref = O.select(v, scene.blocks, zt, thresholds=(1e30,), cull=True)
    sel = r.select(v, thresholds=(1e30,), cull=True)
    assert sel == [(scene.blocks[k].block_id, scene.blocks[k].lod) for k in sel_ref]


def test_c2_full_frame_sampled_rows(c2, torch_cuda):
    """Full 1920x1080 launch as benchmarked; every pixel finite, sampled rows
    (spanning the frame, both edges) against the oracle one by one."""
    scene, r = c2
    v = sg.c2_view()
    sel = r.select(v, thresholds=(1e30,), cull=True)
    set_idx = [next(k for k, b in enumerate(scene.blocks) if (b.block_id, b.lod) == s) for s in sel]
    rows = np.array([0, 1, 211, 540, 777, 1078, 1079])
    out, ref, e_rgb, e_t = check_against_oracle(torch_cuda, r, scene, v, sg.cityb_params(), sg.xavier_mlp(1),
                                                sel, set_idx, pix_rows=rows)
    assert torch_cuda.isfinite(out["rgb"]).all()
    assert ref["n_eval"].sum() > 1e6


def test_c2_full_frame_jumps_equal_flat(c2, torch_cuda):
    """The benchmarked 1920x1080 frame with jumps over empty occupancy-pyramid
    cells renders the same bits and sample counts as a one-step march."""
    torch = torch_cuda
    from paper_2312_16457_amd import F_FLAT_OCC
    scene, r = c2
    v = sg.c2_view()
    sel = r.select(v, thresholds=(1e30,), cull=True)
    mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
    a = r.render([v], [sel], sg.cityb_params(), mlp, counts=True)
    b = r.render([v], [sel], sg.cityb_params(), mlp, counts=True, flags=F_FLAT_OCC)
    torch.cuda.synchronize()
    for key in ("rgb", "trans", "aux", "counts"):
        assert torch.equal(a[key], b[key]), key
    c = a["counts"]
    assert (c[:, 1] - c[:, 0]).sum().item() > 1e7  # empty steps the jumps replace


def test_launch_variants_bitwise(c2, torch_cuda):
    """Per-block launches + blend, persistent, graph replay, packet shapes and
    waves per workgroup all give bit-identical outputs (P12)."""
    torch = torch_cuda
    from paper_2312_16457_amd import F_GRAPH, F_PER_BLOCK, F_PERSISTENT
    scene, r = c2
    v = sg.c2_view(W=480, H=270)
    views = [v, v.with_crop(17, 9, 301, 111)]
    sel = r.select(v, thresholds=(1e30,), cull=True)
    sets = [sel, sel[:7]]
    mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
    p = sg.cityb_params()
    r.set_config(8, 4, -1)
    base = r.render(views, sets, p, mlp, counts=True)
    torch.cuda.synchronize()
    variants = []
    for flags in (F_PER_BLOCK, F_PERSISTENT, F_GRAPH, F_GRAPH | F_PERSISTENT, F_GRAPH | F_PER_BLOCK):
        variants.append((flags, r.render(views, sets, p, mlp, counts=True, flags=flags)))
    for tw, wv, ps in ((16, 2, 0), (4, 1, 1), (32, 4, 0), (64, 1, 0), (1, 2, 0)):
        r.set_config(tw, wv, ps)
        variants.append(((tw, wv, ps), r.render(views, sets, p, mlp, counts=True)))
    r.set_config(8, 4, -1)
    # replay the cached graph a second time
    variants.append(("graph-replay", r.render(views, sets, p, mlp, counts=True, flags=F_GRAPH)))
    torch.cuda.synchronize()
    for name, o in variants:
        for key in ("rgb", "trans", "aux", "counts"):
            assert torch.equal(o[key], base[key]), (name, key)


def test_determinism(c2, torch_cuda):
    torch = torch_cuda
    scene, r = c2
    v = sg.c2_view(W=320, H=180)
    sel = r.select(v, thresholds=(1e30,), cull=True)
    mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
    a = r.render([v], [sel], sg.cityb_params(), mlp)
    b = r.render([v], [sel], sg.cityb_params(), mlp)
    torch.cuda.synchronize()
    assert torch.equal(a["rgb"], b["rgb"]) and torch.equal(a["aux"], b["aux"])


def test_sparse_bricks_bitwise(c2, torch_cuda):
    torch = torch_cuda
    from paper_2312_16457_amd import F_SPARSE
    scene, r = c2
    nbytes = r.pack_bricks()
    dense = sum(b.grid.nbytes for b in scene.blocks)
    assert 0 < nbytes
    v = sg.c2_view(W=480, H=270)
    sel = r.select(v, thresholds=(1e30,), cull=True)
    mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
    a = r.render([v], [sel], sg.cityb_params(), mlp, counts=True)
    b = r.render([v], [sel], sg.cityb_params(), mlp, counts=True, flags=F_SPARSE)
    torch.cuda.synchronize()
    for key in ("rgb", "trans", "aux", "counts"):
        assert torch.equal(a[key], b[key]), key
    print(f"brick atlas {nbytes / 2**20:.1f} MiB vs dense grids {dense / 2**20:.1f} MiB")


def test_negative_controls_differ(c2, torch_cuda):
    """Reversing the per-view block order (no depth sort) changes the image
    by far more than the parity tolerance (Fig. 2a)."""
    torch = torch_cuda
    scene, r = c2
    v = sg.c2_view(W=240, H=135)
    sel = r.select(v, thresholds=(1e30,), cull=True)
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    set_idx = [next(k for k, b in enumerate(scene.blocks) if (b.block_id, b.lod) == s) for s in sel]
    w = sg.xavier_mlp(1)
    out = r.render([v], [sel], sg.cityb_params(), torch.tensor(w, device="cuda"))
    pix = O.pixels_of(v, rows=np.arange(0, 135, 9))
    lin = pix[:, 1] * 240 + pix[:, 0]
    gpu = out["rgb"].cpu().numpy()[lin]
    for comp in (O.REVERSED, O.ALPHA_NORM):
        bad = O.render(ob, occs, v, set_idx, sg.cityb_params(), w, pix=pix, composite=comp)
        assert np.abs(bad["rgb"] - gpu).max() > 1e-2


def test_invalid_arguments_have_no_side_effects(c2, torch_cuda):
    torch = torch_cuda
    from paper_2312_16457_amd import CowError
    from paper_2312_16457_amd.binding import COW_E_INVALID, COW_E_NOT_LOADED, COW_E_UNSUPPORTED
    scene, r = c2
    v = sg.c2_view(W=64, H=36)
    mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
    cases = [
        ([(0, 0), (0, 0)], sg.cityb_params(), COW_E_INVALID),  # duplicate block
        ([(99, 0)], sg.cityb_params(), COW_E_NOT_LOADED),  # unknown block
        ([(0, 1)], sg.cityb_params(), COW_E_NOT_LOADED),  # unknown LOD
        ([(0, 0)], sg.RenderParams(mode=1, delta=-1.0), COW_E_INVALID),
        ([(0, 0)], sg.RenderParams(mode=7), COW_E_INVALID),
    ]
    for s, p, code in cases:
        with pytest.raises(CowError) as ei:
            r.render([v], [s], p, mlp)
        assert ei.value.status == code
    bad = v.with_crop(0, 0, 65, 36)
    with pytest.raises(CowError):
        r.render([bad], [[(0, 0)]], sg.cityb_params(), mlp)
    nan = sg.View(64, 36, np.array([np.nan, 0, 1], np.float32), v.R, v.fx, v.fy, v.cx, v.cy)
    with pytest.raises(CowError):
        r.render([nan], [[(0, 0)]], sg.cityb_params(), mlp)
    # backward through uint8 textures is unsupported
    out = r.render([v], [[(0, 0)]], sg.cityb_params(), mlp)
    with pytest.raises(CowError) as ei:
        r.render_backward([v], [[(0, 0)]], sg.cityb_params(), mlp, out["aux"], torch.zeros_like(out["rgb"]))
    assert ei.value.status == COW_E_UNSUPPORTED


@pytest.mark.parametrize("mode", [0, 1])
def test_early_termination_parity(torch_cuda, mode):
    """Opaque variant (density shift 0) with t_min = 1e-5: the kernel stops
    each ray at the same sample as the oracle (fp32 vs fp64 transmittance may
    differ by one sample where T meets t_min within rounding; the extra
    contribution is below t_min)."""
    torch = torch_cuda
    scene = sg.make_scene(3, 3, ((16, 64, 8),), sg.U8, blobs_per_block=10, blob_z=(0, 0.3), seed=7, shift=0.0)
    view = sg.pinhole(37, 29, (1.5, -1.1, 1.3), sg.look_rotation(np.array([1.5, 1.5, 0.1]) - [1.5, -1.1, 1.3]))
    p = sg.RenderParams(mode=1, t_min=1e-5) if mode == 1 else sg.RenderParams(mode=0, n_steps=128, t_min=1e-5)
    r = make_renderer(scene.blocks)
    w = sg.random_mlp(2, 0.7)
    refs = all_refs(scene)
    mlp = torch.tensor(w, device="cuda")
    out = r.render([view], [refs], p, mlp, counts=True)
    full = r.render([view], [refs], sg.RenderParams(mode=p.mode, n_steps=p.n_steps), mlp, counts=True)
    torch.cuda.synchronize()
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    ref = O.render(ob, occs, view, list(range(ob.n)), p, w)
    cnt = out["counts"].cpu().numpy()
    diff = cnt[:, 0] != ref["n_eval"]
    assert diff.mean() <= 1e-3 and np.abs(cnt[:, 0] - ref["n_eval"]).max() <= 1
    assert np.abs(out["rgb"].cpu().numpy() - ref["rgb"]).max() <= TOL
    assert np.abs(out["trans"].cpu().numpy() - ref["trans"]).max() <= TOL
    stopped = cnt[:, 0] < full["counts"].cpu().numpy()[:, 0]
    assert stopped.mean() > 0.2  # the opaque scene does terminate rays early
    gap = (out["aux"][:, :7] - full["aux"][:, :7]).abs().max(dim=1).values.cpu().numpy()
    assert (gap <= out["trans"].cpu().numpy() + 1e-6).all()


def test_mixed_dtype_scene(torch_cuda):
    """A loaded scene may hold uint8 and fp32 entries side by side; each
    call's sets must use one dtype.  A set of either dtype renders bit for bit
    as in a scene of that block alone, and a call mixing the two is refused
    (COW_E_UNSUPPORTED) with its outputs untouched."""
    torch = torch_cuda
    from paper_2312_16457_amd import CowError, Renderer
    from paper_2312_16457_amd.binding import COW_E_UNSUPPORTED
    u8 = sg.make_scene(2, 1, ((16, 32, 4),), sg.U8, blobs_per_block=8, seed=31, shift=2.0).blocks
    f32 = sg.make_scene(2, 1, ((16, 32, 4),), sg.F32, blobs_per_block=8, seed=32, shift=2.0).blocks
    both = [u8[0], f32[1]]
    v = sg.pinhole(40, 24, (1.0, -1.2, 0.8), sg.look_rotation(np.array([1.0, 0.5, 0.3]) - [1.0, -1.2, 0.8]))
    params = sg.cityb_params()
    mlp = torch.tensor(sg.random_mlp(2, 0.5), device="cuda")
    r = Renderer(0).load_blocks(both)
    for blk in both:
        alone = Renderer(0).load_blocks([blk])
        ref = alone.render([v], [[(blk.block_id, 0)]], params, mlp, counts=True)
        got = r.render([v], [[(blk.block_id, 0)]], params, mlp, counts=True)
        torch.cuda.synchronize()
        assert ref["counts"][:, 0].sum().item() > 0
        for k in ("rgb", "trans", "aux", "counts"):
            assert torch.equal(got[k], ref[k]), (blk.dtype, k)
    out = {k: t.clone().fill_(7.0) for k, t in r.render([v], [[(0, 0)]], params, mlp).items() if t is not None}
    before = {k: t.clone() for k, t in out.items()}
    with pytest.raises(CowError) as ei:
        r.render([v], [[(0, 0), (1, 0)]], params, mlp, out=out)
    assert ei.value.status == COW_E_UNSUPPORTED
    torch.cuda.synchronize()
    for k in out:
        assert torch.equal(out[k], before[k]), k
