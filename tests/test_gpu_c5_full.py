"""The differentiable workload at full size, in the launch the benchmark
times: the fp32 4x4-block city, all 8 views at 800x800 in one call (5.12 M
rays, persistent one-wave-per-SIMD forward; the adjoint with its LDS cache
of grid pairs), checked against the oracle where it can compute one by one:
sampled rows of every view for the forward (rgb and T <= 1e-4, evaluated
and marched sample counts exact), and for the adjoint an upstream gradient
that is zero except on 48 seeded pixels spread over the views (every other
ray scatters zeros), against the fp64 adjoint of those pixels (<= 1e-3
normwise per tensor).  The same with the edge blocks contracted and the
exterior sampled."""
import numpy as np
import pytest

import oracle as O
from paper_2312_16457_amd import scenegen as sg

pytestmark = pytest.mark.gpu


def compare(gg, gp, gm, grads, gm_ref, rel=1e-3):
    """max|g - g_ref| <= rel max|g_ref| per gradient tensor."""
    for k, (g, ps) in grads.items():
        for a, b in [(gg[k], g)] + [(gp[k][i], ps[i]) for i in range(3)]:
            den = np.abs(b).max()
            if den == 0:
                assert np.abs(a.cpu().numpy()).max() == 0
                continue
            assert np.abs(a.cpu().numpy() - b).max() / den <= rel, k
    assert np.abs(gm.cpu().numpy() - gm_ref).max() / np.abs(gm_ref).max() <= rel


@pytest.fixture(scope="module")
def c5(have_gpu):
    import torch
    from paper_2312_16457_amd import Renderer
    learn, _ = sg.c5_scenes()
    views = sg.c5_views()
    params = sg.cityb_params()
    w = sg.xavier_mlp(4)
    r = Renderer(0).load_blocks(learn.blocks)
    sets = [[(b.block_id, 0) for b in learn.blocks]] * len(views)
    mlp = torch.tensor(w, device="cuda")
    out = r.render(views, sets, params, mlp, counts=True)
    torch.cuda.synchronize()
    ob = O.OracleScene(learn.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    return torch, learn, views, params, w, r, sets, mlp, out, ob, occs


def test_c5_full_size_forward_sampled_rows(c5):
    torch, learn, views, params, w, r, sets, mlp, out, ob, occs = c5
    assert r.get_config()[2] == -1  # the default: persistent for fp32 blocks
    rgb, trans, counts = out["rgb"].cpu().numpy(), out["trans"].cpu().numpy(), out["counts"].cpu().numpy()
    assert np.isfinite(rgb).all() and np.isfinite(trans).all()
    rows = np.array([0, 1, 157, 399, 400, 613, 798, 799])
    base, n_eval = 0, 0
    for v in views:
        pix = O.pixels_of(v, rows=rows)
        ref = O.render(ob, occs, v, list(range(ob.n)), params, w, pix=pix)
        idx = base + pix[:, 1].astype(np.int64) * v.W + pix[:, 0]
        assert np.abs(rgb[idx] - ref["rgb"]).max() <= 1e-4
        assert np.abs(trans[idx] - ref["trans"]).max() <= 1e-4
        assert np.array_equal(counts[idx, 0], ref["n_eval"])
        assert np.array_equal(counts[idx, 1], ref["n_march"])
        n_eval += int(ref["n_eval"].sum())
        base += v.n_pixels
    assert n_eval > 1e6


def test_c5_full_size_adjoint_sparse_upstream(c5):
    torch, learn, views, params, w, r, sets, mlp, out, ob, occs = c5
    rng = np.random.default_rng(11)
    n_pix = out["rgb"].shape[0]
    g_rgb = np.zeros((n_pix, 3))
    grads, gm_ref = None, None
    base = 0
    for v in views:
        pix = np.stack([rng.integers(0, v.W, 6), rng.integers(200, 700, 6)], axis=1).astype(np.int32)
        g = rng.uniform(-1, 1, (6, 3))
        idx = base + pix[:, 1].astype(np.int64) * v.W + pix[:, 0]
        g_rgb[idx] = g
        gr, gmr = O.adjoint(ob, occs, v, list(range(ob.n)), params, w, pix, g)
        if grads is None:
            grads, gm_ref = gr, gmr
        else:
            for k, (gg_k, gp_k) in gr.items():
                grads[k][0][...] += gg_k
                for i in range(3):
                    grads[k][1][i][...] += gp_k[i]
            gm_ref = gm_ref + gmr
        base += v.n_pixels
    gg = [torch.zeros_like(t[0]) for t in r.textures]
    gp = [[torch.zeros_like(x) for x in t[1]] for t in r.textures]
    gm = torch.zeros(499, device="cuda")
    r.render_backward(views, sets, params, mlp, out["aux"], torch.tensor(g_rgb, dtype=torch.float32, device="cuda"),
                      None, gg, gp, gm)
    torch.cuda.synchronize()
    touched = [k for k, (g, ps) in grads.items() if np.abs(g).max() > 0]
    assert len(touched) >= 4
    compare(gg, gp, gm, {k: grads[k] for k in touched}, gm_ref)
    for k in set(range(len(learn.blocks))) - set(touched):
        assert gg[k].abs().max().item() == 0


def test_c5_contracted_full_size_forward_rows_and_adjoint(c5):
    """The same workload with its 12 edge blocks contracted and the exterior
    sampled (ext_delta 1/64, at most 512 steps per segment), as the benchmark
    times it: two sampled rows of every view (rgb and T <= 1e-4, sample
    counts exact), and the adjoint of an upstream gradient on 48 seeded
    pixels against the fp64 adjoint of those pixels."""
    from dataclasses import replace

    from paper_2312_16457_amd import Renderer
    torch, learn, views, params, w, _, sets, mlp, _, _, _ = c5
    blocks = sg.contract_boundary(learn.blocks)
    assert sum(b.contracted for b in blocks) == 12
    p = replace(params, ext_delta=1.0 / 64, ext_max_steps=512)
    r = Renderer(0).load_blocks(blocks)
    out = r.render(views, sets, p, mlp, counts=True)
    torch.cuda.synchronize()
    ob = O.OracleScene(blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    rgb, trans, counts = out["rgb"].cpu().numpy(), out["trans"].cpu().numpy(), out["counts"].cpu().numpy()
    rows = np.array([3, 611])
    base = 0
    for v in views:
        pix = O.pixels_of(v, rows=rows)
        ref = O.render(ob, occs, v, list(range(ob.n)), p, w, pix=pix)
        idx = base + pix[:, 1].astype(np.int64) * v.W + pix[:, 0]
        assert np.abs(rgb[idx] - ref["rgb"]).max() <= 1e-4
        assert np.abs(trans[idx] - ref["trans"]).max() <= 1e-4
        assert np.array_equal(counts[idx, 0], ref["n_eval"])
        assert np.array_equal(counts[idx, 1], ref["n_march"])
        base += v.n_pixels
    rng = np.random.default_rng(12)
    g_rgb = np.zeros((out["rgb"].shape[0], 3))
    grads, gm_ref, base = None, None, 0
    for v in views:
        pix = np.stack([rng.integers(0, v.W, 6), rng.integers(0, v.H, 6)], axis=1).astype(np.int32)
        g = rng.uniform(-1, 1, (6, 3))
        g_rgb[base + pix[:, 1].astype(np.int64) * v.W + pix[:, 0]] = g
        gr, gmr = O.adjoint(ob, occs, v, list(range(ob.n)), p, w, pix, g)
        if grads is None:
            grads, gm_ref = gr, gmr
        else:
            for k, (gg_k, gp_k) in gr.items():
                grads[k][0][...] += gg_k
                for i in range(3):
                    grads[k][1][i][...] += gp_k[i]
            gm_ref = gm_ref + gmr
        base += v.n_pixels
    gg = [torch.zeros_like(t[0]) for t in r.textures]
    gp = [[torch.zeros_like(x) for x in t[1]] for t in r.textures]
    gm = torch.zeros(499, device="cuda")
    r.render_backward(views, sets, p, mlp, out["aux"], torch.tensor(g_rgb, dtype=torch.float32, device="cuda"),
                      None, gg, gp, gm)
    torch.cuda.synchronize()
    touched = [k for k, (g, ps) in grads.items() if np.abs(g).max() > 0]
    assert len(touched) >= 4
    compare(gg, gp, gm, {k: grads[k] for k in touched}, gm_ref)
    for k in set(range(len(learn.blocks))) - set(touched):
        assert gg[k].abs().max().item() == 0
