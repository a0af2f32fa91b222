"""Benchmark of the block-merged ray-march render path on one MI355X.

Workload (N=1): 4x4 ground-partitioned uint8 blocks (128^3 grid + three
1024^2 planes, 16^3 occupancy per block), one 1920x1080 view, camera-anchored
steps of 1/512 block width, at most 2048 steps per ray, deferred MLP
10->16->16->3.  One step = one full render of the frame (forward march with
per-block composite and front-to-back merge, then the MFMA MLP pass), inputs
resident in HBM.

Prints one JSON line: metric/value (forward Msamples/s of evaluated samples),
FPS, the roofline of the march kernel (timed with HIP events on its own
stream inside the library), the CPU oracle baseline on a bounded sample, and
optional extra measurements (backward, batched vs per-block launches).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# MI355X published peaks
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# algorithmic fp32 flops of one evaluated sample of the uint8 path:
#   trilinear grid 8 taps x 8 ch x 2 = 128, three bilinear planes 3 x 4 x 8 x 2 = 192,
#   interpolation weights 30, decode q*s+o 4 x 8 x 2 = 64, texture sum 3 x 8 = 24,
#   activations (exp + 7 sigmoid) 22, alpha / weight / composite of 7 values / T 20
FLOPS_PER_SAMPLE = 128 + 192 + 30 + 64 + 24 + 22 + 20  # 480
# the same sample counted as vector-ALU operations (an FMA is one), the
# measure of the work a sample needs quoted beside the flop count: about 200
# FMA (interpolation, weights, decode, composite), 160 byte conversions,
# 9 exp + 7 rcp, rounded to 450
VALU_OPS_PER_SAMPLE = 450
BYTES_PER_SAMPLE_U8 = 160  # 20 texels x 8 uint8 channels gathered per evaluated sample


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20; 3 with --profile)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 5; 1 with --profile)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the backward and batched measurements")
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3 (no CPU leg, no extras)")
    ap.add_argument("--leg", choices=["fwd", "bwd", "batched", "quadtree", "variants", "opaque", "empty", "contract"],
                    default="fwd",
                    help="with --profile: the leg to run (one timed repetition of bwd / batched / quadtree / "
                         "the forward's options)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a 1 GiB device copy, to scale HBM byte counters")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the render path shards by view or by block with no "
              "inter-GPU exchange in the forward pass, and the benchmark runs on a single MI355X.", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_each_way": src.numel() * 4, "launches": 3}))
        return
    import __graft_entry__
    __graft_entry__._ensure_built()
    from paper_2312_16457_amd import Renderer, scenegen as sg
    if args.profile and args.leg != "fwd":
        fn = {"bwd": lambda *a, **k: leg_backward(*a, **k)[0], "batched": lambda *a, **k: leg_batched(*a, **k)[0],
              "quadtree": leg_quadtree,
              "variants": leg_variants, "opaque": leg_opaque, "empty": leg_empty_space,
              "contract": leg_contracted}
        print(json.dumps({"leg": args.leg, **fn[args.leg](torch, sg, Renderer, reps=1)}), flush=True)
        return

    t0 = time.time()
    scene = sg.c2_scene()
    view = sg.c2_view()
    params = sg.cityb_params()
    w = sg.xavier_mlp(1)
    log(f"scene generated in {time.time() - t0:.1f}s")
    r = Renderer(0)
    r.load_blocks(scene.blocks)
    sel = r.select(view, thresholds=(1e30,), cull=True)
    mlp = torch.tensor(w, device="cuda")
    # evaluated-sample count from the kernel's own counters (untimed run)
    out = r.render([view], [sel], params, mlp, counts=True)
    torch.cuda.synchronize()
    n_eval = int(out["counts"][:, 0].sum().item())
    n_march = int(out["counts"][:, 1].sum().item())
    out = r.render([view], [sel], params, mlp, want_aux=False)
    steps = args.steps if args.steps is not None else (3 if args.profile else 20)
    warm = args.warmup if args.warmup is not None else (1 if args.profile else 5)
    for _ in range(warm):
        r.render([view], [sel], params, mlp, out=out)
    torch.cuda.synchronize()
    # march-kernel duration: HIP events recorded by the library around the
    # kernel on the call's stream
    r.set_timing(True)
    march_ms = []
    for _ in range(steps):
        r.render([view], [sel], params, mlp, out=out)
        march_ms.append(r.last_timing()[0])
    r.set_timing(False)
    torch.cuda.synchronize()
    # one step = the whole per-frame path: the view's block set (selection on
    # the host: culling and depth order), then the render
    t_start = time.perf_counter()
    for _ in range(steps):
        sel_t = r.select(view, thresholds=(1e30,), cull=True)
        r.render([view], [sel_t], params, mlp, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t_start) * 1e3 / steps
    t_sel = time.perf_counter()
    for _ in range(100):
        r.select(view, thresholds=(1e30,), cull=True)
    select_ms = (time.perf_counter() - t_sel) * 1e3 / 100
    msamples = n_eval / (ms * 1e-3) / 1e6
    fps = 1000.0 / ms
    k_ms = float(np.mean(march_ms))
    achieved = FLOPS_PER_SAMPLE * n_eval / (k_ms * 1e-3) / 1e12
    res = {
        "metric": "forward Msamples/s (evaluated samples), 4x4 uint8 blocks, 1920x1080",
        "value": round(msamples, 2),
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "4x4 ground blocks, uint8 128^3 grid + 3x1024^2 planes, 16^3 occupancy, "
                               "one 1920x1080 view, delta 1/512, <=2048 steps, MLP 10-16-16-3",
                   "pixels": view.n_pixels, "evaluated_samples": n_eval, "marched_samples": n_march,
                   "blocks": len(sel)},
        "fps_1080p": round(fps, 2),
        "select_ms": round(select_ms, 4),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "kernel": "march_fwd_kernel<1,false> (uint8, grid sampling)", "kernel_ms": round(k_ms, 4),
                     "algorithmic_tflop_per_launch": round(FLOPS_PER_SAMPLE * n_eval / 1e12, 4),
                     "flops_per_sample": FLOPS_PER_SAMPLE,
                     "frac_basis": "480 algorithmic fp32 flops per evaluated sample (an FMA counts 2)",
                     "valu_ops_per_sample": VALU_OPS_PER_SAMPLE,
                     "frac_at_valu_ops": round(VALU_OPS_PER_SAMPLE * n_eval / (k_ms * 1e-3) / 1e12 /
                                               PEAK_FP32_TFLOPS, 4),
                     "gathered_GBps": round(BYTES_PER_SAMPLE_U8 * n_eval / (k_ms * 1e-3) / 1e9, 1)},
    }
    log(f"forward {ms:.2f} ms per frame")
    if not args.profile:
        res["gather"] = gather_ceiling(torch, view, n_eval, res["roofline"]["gathered_GBps"])
        log("gather probe done")
    if not args.no_cpu_baseline and not args.profile:
        res["cpu_baseline"] = cpu_baseline(scene, view, sel, params, w)
        log("cpu baseline done")
    res["roofline"]["traffic"] = recorded_traffic()
    comp = compulsory_bytes()
    if comp:
        res["roofline"]["hbm_compulsory_bytes"] = comp
        if res["roofline"]["traffic"]:
            res["roofline"]["traffic_over_compulsory"] = round(res["roofline"]["traffic"] / comp, 2)
    if not args.no_extras and not args.profile:
        res["variants"] = forward_variants(torch, sg, r, view, sel, params, mlp, ms)
        del r, out
        torch.cuda.empty_cache()
        res["extras"] = extras(torch, sg, Renderer, cpu=res.get("cpu_baseline"))
    print(json.dumps(res), flush=True)


def source_digest():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2312_16457_amd", "csrc")
    for f in ("cow_internal.h", "cow_device.h", "cow_march.hip"):  # the march kernel's sources
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per march launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (scaled by a 1 GiB copy), or None when the kernel
    sources changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_march_fwd_4x4_1080p.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_digest") != source_digest():
        return None
    return rec.get("hbm_bytes_per_launch")


def compulsory_bytes():
    """The march's compulsory HBM bytes per launch on the bench frame: the
    unique 128-byte texture lines its evaluated samples read, the occupancy
    bytes and its outputs, as counted by the oracle's committed script
    (oracle/compulsory_bytes.py; the record names its command)."""
    path = os.path.join(ROOT, "profiles", "compulsory_bytes_4x4_1080p.json")
    if not os.path.exists(path):
        return None
    return json.load(open(path)).get("compulsory_bytes_march")


def gather_ceiling(torch, view, n_eval, march_GBps):
    """Achievable texel-gather rate for the march's access pattern: the
    library's gather microbenchmark (the march's ten 16-byte pair loads per
    sample, no arithmetic) on the same view, at the mean evaluated samples per
    ray, over random uint8 textures of three footprints: L2-resident, Infinity
    Cache-resident and the frame's own 640 MiB.  frac = the march's gathered
    bytes per second over the probe's at the frame's footprint."""
    from paper_2312_16457_amd import COW_U8
    from paper_2312_16457_amd.binding import gather_probe
    steps = max(1, int(round(n_eval / view.n_pixels)))
    out = {"steps_per_ray": steps}
    cases = (("l2_1block_32_128", 1, 32, 128), ("mall_2x2_64_512", 2, 64, 512), ("frame_4x4_128_1024", 4, 128, 1024))
    for name, nb, R, Rp in cases:
        nbytes = nb * nb * (R ** 3 + 3 * Rp * Rp) * 8
        tex = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
        gather_probe(view, tex, nb, nb, R, Rp, COW_U8, steps, 1.0 / 512)  # warm-up
        best = min(gather_probe(view, tex, nb, nb, R, Rp, COW_U8, steps, 1.0 / 512)[0] for _ in range(3))
        gbytes = view.n_pixels * steps * BYTES_PER_SAMPLE_U8
        out[name] = {"footprint_MiB": round(nbytes / 2 ** 20, 1), "ms": round(best, 3),
                     "GBps": round(gbytes / (best * 1e-3) / 1e9, 1)}
        del tex
    out["march_GBps"] = march_GBps
    out["frac_of_frame_footprint"] = round(march_GBps / out["frame_4x4_128_1024"]["GBps"], 4)
    return out


def _threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))


def host_cpu():
    """CPU model, cores and SMT of the host, from lscpu."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except Exception:
        pass
    return {"model": info.get("Model name"), "sockets": info.get("Socket(s)"),
            "cores_per_socket": info.get("Core(s) per socket"), "threads_per_core": info.get("Thread(s) per core"),
            "logical_cpus": info.get("CPU(s)"), "threads_used": _threads()}


def _oracle_rate(O, ob, occs, view, set_idx, params, w, pix, fp32=False, threads=None):
    t = time.perf_counter()
    ref = O.render(ob, occs, view, set_idx, params, w, pix=pix, nthreads=threads or _threads(), fp32=fp32)
    dt = time.perf_counter() - t
    n = int(ref["n_eval"].sum())
    return {"Msamples_per_s": round(n / dt / 1e6, 3), "seconds": round(dt, 2), "evaluated_samples": n,
            "rays": int(len(pix))}


def cpu_baseline(scene, view, sel, params, w):
    """The CPU oracle, as it stands, on every second row of the same frame
    (about 10 s of work on 16 host threads), in fp64 (the oracle) and in its
    single-precision build (the same decisions, continuous per-sample math in
    float); plus the single-block frame in full."""
    import oracle as O
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    set_idx = [next(k for k, b in enumerate(scene.blocks) if (b.block_id, b.lod) == s) for s in sel]
    rows = np.arange(0, view.H, 2)
    pix = O.pixels_of(view, rows=rows)
    threads = _threads()
    f64 = _oracle_rate(O, ob, occs, view, set_idx, params, w, pix)
    f32 = _oracle_rate(O, ob, occs, view, set_idx, params, w, pix, fp32=True)
    res = {"value": f64["Msamples_per_s"], "unit": "Msamples/s", "cores": threads,
           "kind": "oracle", "sample": f"every second row of the 1920x1080 frame ({len(rows)} rows, "
                                       f"{len(pix)} rays, {f64['evaluated_samples']} evaluated samples), "
                                       f"fp64, {f64['seconds']:.1f}s",
           "host": host_cpu(), "fp32": f32,
           "note": "the oracle is a plain per-ray reference, not a tuned CPU renderer; Msamples/s counts "
                   "evaluated samples"}
    del ob, occs
    from paper_2312_16457_amd import scenegen as sg
    c1 = sg.c1_scene()
    ob1 = O.OracleScene(c1.blocks)
    occ1 = [O.occupancy(ob1, 0)]
    v1 = sg.c1_view()
    pix1 = O.pixels_of(v1)
    w1 = sg.xavier_mlp(0)
    res["legs"] = {"single_block_128x128_full_frame": {
        "fp64": _oracle_rate(O, ob1, occ1, v1, [0], sg.c1_params(), w1, pix1),
        "fp32": _oracle_rate(O, ob1, occ1, v1, [0], sg.c1_params(), w1, pix1, fp32=True)}}
    return res


def cpu_baseline_lod(scene, sg):
    """The oracle on the 8x8x3-LOD city: the 16 aerial 1080p views (two of
    them, every 16th row) and the 64-view batch (every 512th row of every
    view), fp64 and fp32; rates are evaluated samples per second on that
    sample, which equal the whole workload's by construction of the unit
    (extrapolated, labelled)."""
    import oracle as O
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    p = sg.cityb_params()
    w = sg.xavier_mlp(3)
    out = {}
    for name, views, every in (("lod_city_aerial_16x1080p", sg.c3_views()[:2], 16),
                               ("batched_64_views", sg.c4_views(), 512)):
        legs = {}
        for fp32 in (False, True):
            t = time.perf_counter()
            n = rays = 0
            for v in views:
                sel = O.select(v, scene.blocks, zt, thresholds=(2.0, 4.0, 8.0), cull=True)
                pix = O.pixels_of(v, rows=np.arange(0, v.H, every))
                r = O.render(ob, occs, v, sel, p, w, pix=pix, nthreads=_threads(), fp32=fp32)
                n += int(r["n_eval"].sum())
                rays += len(pix)
            dt = time.perf_counter() - t
            legs["fp32" if fp32 else "fp64"] = {"Msamples_per_s": round(n / dt / 1e6, 3), "seconds": round(dt, 2),
                                                "evaluated_samples": n, "rays": rays}
        legs["sample"] = (f"{len(views)} views, every {every}th row (extrapolated: the rate over this sample "
                          "stands for the whole workload)")
        out[name] = legs
    return out


def cpu_baseline_adjoint(learn, sg):
    """The fp64 adjoint (one thread: the oracle's adjoint is serial) on the
    64x64 crop of the differentiable workload's view 0 with the most evaluated
    samples among 16 seeded windows (counted by the oracle)."""
    import oracle as O
    ob = O.OracleScene(learn.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    setv = list(range(ob.n))
    v0 = sg.c5_views()[0]
    p = sg.cityb_params()
    w = sg.xavier_mlp(4)
    rng = np.random.default_rng(0)
    cands = [(int(rng.integers(0, 800 - 64)), int(rng.integers(0, 800 - 64))) for _ in range(16)]

    def score(c):
        pix = np.array([[c[0] + i, c[1] + j] for j in range(0, 64, 8) for i in range(0, 64, 8)], np.int32)
        return int(O.render(ob, occs, v0, setv, p, w, pix=pix)["n_eval"].sum())
    x0, y0 = max(cands, key=score)
    crop = v0.with_crop(x0, y0, 64, 64)
    pix = O.pixels_of(crop)
    r = O.render(ob, occs, crop, setv, p, w, pix=pix)
    n = int(r["n_eval"].sum())
    g = np.random.default_rng(1).uniform(-1e-3, 1e-3, (len(pix), 3))
    t = time.perf_counter()
    O.adjoint(ob, occs, crop, setv, p, w, pix, g)
    dt = time.perf_counter() - t
    return {"Msamples_per_s": round(n / dt / 1e6, 3), "seconds": round(dt, 2), "evaluated_samples": n,
            "cores": 1, "sample": f"64x64 crop at ({x0}, {y0}) of view 0, fp64 adjoint"}


def log(msg, t0=[time.time()]):
    print(f"[bench {time.time() - t0[0]:7.1f}s] {msg}", file=sys.stderr, flush=True)


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / reps


def forward_variants(torch, sg, r, view, sel, params, mlp, base_ms, reps=5):
    """The bench frame with the render's options: early ray termination
    (t_min = 1e-3, the oracle applies the same rule), one deferred MLP per
    block before the merge (the across-block equation as written), and the
    per-ray opacity-entropy output."""
    from dataclasses import replace
    from paper_2312_16457_amd import F_FLAT_OCC
    res = {"base_ms": None if base_ms is None else round(base_ms, 3)}
    p_t = replace(params, t_min=1e-3)
    cnt = r.render([view], [sel], p_t, mlp, counts=True)
    n_t = int(cnt["counts"][:, 0].sum().item())
    out = r.render([view], [sel], p_t, mlp, want_aux=False)
    ms = _timed(torch, lambda: r.render([view], [sel], p_t, mlp, out=out), reps)
    res["early_termination_1e-3"] = {"ms": round(ms, 3), "evaluated_samples": n_t,
                                     "Msamples_per_s": round(n_t / (ms * 1e-3) / 1e6, 1)}
    bm = torch.tensor(np.stack([sg.xavier_mlp(100 + k) for k in range(len(r.blocks))]), device="cuda")
    out = r.render([view], [sel], params, None, want_aux=False, block_mlp=bm)
    ms = _timed(torch, lambda: r.render([view], [sel], params, None, out=out, block_mlp=bm), reps)
    res["per_block_mlps"] = {"ms": round(ms, 3), "blocks": len(sel)}
    out = r.render([view], [sel], params, mlp, want_aux=False, opacity=True)
    ms = _timed(torch, lambda: r.render([view], [sel], params, mlp, out=out), reps)
    res["with_opacity_entropy"] = {"ms": round(ms, 3)}
    out = r.render([view], [sel], params, mlp, want_aux=False)
    ms = _timed(torch, lambda: r.render([view], [sel], params, mlp, out=out, flags=F_FLAT_OCC), reps)
    res["one_step_empty_space"] = {"ms": round(ms, 3)}
    # the deferred MLPs over the positional encoding of the direction (Eq. deferred, 4 frequencies)
    p_pe = replace(params, pe_freqs=4)
    mlp_pe = torch.tensor(sg.xavier_mlp(1, pe=4), device="cuda")
    out = r.render([view], [sel], p_pe, mlp_pe, want_aux=False)
    ms = _timed(torch, lambda: r.render([view], [sel], p_pe, mlp_pe, out=out), reps)
    res["mlp_with_posenc"] = {"ms": round(ms, 3)}
    bm_pe = torch.tensor(np.stack([sg.xavier_mlp(100 + k, pe=4) for k in range(len(r.blocks))]), device="cuda")
    out = r.render([view], [sel], p_pe, None, want_aux=False, block_mlp=bm_pe)
    ms = _timed(torch, lambda: r.render([view], [sel], p_pe, None, out=out, block_mlp=bm_pe), reps)
    res["per_block_mlps_with_posenc"] = {"ms": round(ms, 3)}
    log("forward variants done")
    return res


def leg_empty_space(torch, sg, Renderer, reps=3):
    """Jumps over empty cells of the max-pooled occupancy pyramid against a
    one-step march (COW_F_FLAT_OCC; same samples evaluated, same bits) on a
    sparse city: the bench layout with 12 blobs per block spread over the whole
    block height instead of 200 near the ground, one 1920x1080 view."""
    from paper_2312_16457_amd import F_FLAT_OCC
    log("empty space: generating the sparse 4x4 city")
    scene = sg.make_scene(4, 4, ((128, 1024, 16),), sg.U8, blobs_per_block=12, blob_z=(0.0, 0.9),
                          blob_s=(0.04, 0.1), seed=1)
    view = sg.c2_view()
    r = Renderer(0)
    r.load_blocks(scene.blocks)
    sel = r.select(view, thresholds=(1e30,), cull=True)
    p = sg.cityb_params()
    mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
    cnt = r.render([view], [sel], p, mlp, counts=True)["counts"]
    n_eval, n_march = int(cnt[:, 0].sum().item()), int(cnt[:, 1].sum().item())
    res = {"workload": "4x4 uint8 blocks, 12 blobs per block over heights 0-0.9, one 1920x1080 view",
           "evaluated_samples": n_eval, "marched_samples": n_march}
    out = r.render([view], [sel], p, mlp, want_aux=False)
    for name, flags in (("one_step", F_FLAT_OCC), ("pyramid_jumps", 0)):
        ms = _timed(torch, lambda: r.render([view], [sel], p, mlp, out=out, flags=flags), reps)
        res[name] = {"ms": round(ms, 3), "Msamples_per_s": round(n_eval / (ms * 1e-3) / 1e6, 1)}
    res["speedup_from_jumps"] = round(res["one_step"]["ms"] / res["pyramid_jumps"]["ms"], 2)
    del r
    torch.cuda.empty_cache()
    return res


def leg_contracted(torch, sg, Renderer, reps=3):
    """Contracted boundary blocks (the 12 edge blocks of the bench city) with
    their exterior sampled (ext_delta 1/64, at most 512 steps per segment),
    against the same city with plain blocks, from the bench camera and from
    one outside the footprint looking across it (1920x1080 each)."""
    import numpy as np
    from dataclasses import replace
    log("contracted: generating the 4x4 city")
    scene = sg.c2_scene()
    cams = {"bench_view": sg.c2_view(),
            "outside_view": sg.pinhole(1920, 1080, (2.0, -2.5, 1.6),
                                       sg.look_rotation(np.asarray((0.0, 1.0, -0.45))))}
    res = {"workload": "4x4 uint8 blocks (128^3 + 3 x 1024^2), 12 edge blocks contracted, 1920x1080 views",
           "ext_delta": 1.0 / 64, "ext_max_steps": 512}
    for label, blocks, p in (("plain", scene.blocks, sg.cityb_params()),
                             ("contracted", sg.contract_boundary(scene.blocks),
                              replace(sg.cityb_params(), ext_delta=1.0 / 64, ext_max_steps=512))):
        r = Renderer(0)
        r.load_blocks(blocks)
        mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
        for cam, view in cams.items():
            sel = r.select(view, thresholds=(1e30,), cull=False)
            cnt = r.render([view], [sel], p, mlp, counts=True)["counts"]
            n_eval, n_march = int(cnt[:, 0].sum().item()), int(cnt[:, 1].sum().item())
            out = r.render([view], [sel], p, mlp, want_aux=False)
            ms = _timed(torch, lambda: r.render([view], [sel], p, mlp, out=out), reps)
            res[f"{label}_{cam}"] = {"ms": round(ms, 3), "evaluated_samples": n_eval, "marched_samples": n_march,
                                     "Msamples_per_s": round(n_eval / (ms * 1e-3) / 1e6, 1)}
        del r
        torch.cuda.empty_cache()
    return res


def leg_opaque(torch, sg, Renderer, reps=3):
    """The bench frame over the opaque variant of the city (the density
    recipe without its shift of 5: peak density 50), with and without early
    ray termination (t_min = 1e-3; the oracle applies the same rule)."""
    from dataclasses import replace
    log("opaque: generating the opaque 4x4 city")
    scene = sg.make_scene(4, 4, ((128, 1024, 16),), sg.U8, blobs_per_block=200, blob_z=(0.0, 0.3), seed=1,
                          shift=0.0)
    view = sg.c2_view()
    r = Renderer(0)
    r.load_blocks(scene.blocks)
    sel = r.select(view, thresholds=(1e30,), cull=True)
    mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
    res = {"workload": "4x4 uint8 blocks, opaque density (shift 0), one 1920x1080 view"}
    for name, tmin in (("no_termination", 0.0), ("t_min_1e-3", 1e-3)):
        p = replace(sg.cityb_params(), t_min=tmin)
        cnt = r.render([view], [sel], p, mlp, counts=True)["counts"]
        n_eval, n_march = int(cnt[:, 0].sum().item()), int(cnt[:, 1].sum().item())
        out = r.render([view], [sel], p, mlp, want_aux=False)
        ms = _timed(torch, lambda: r.render([view], [sel], p, mlp, out=out), reps)
        res[name] = {"ms": round(ms, 3), "evaluated_samples": n_eval, "marched_samples": n_march,
                     "fps": round(1e3 / ms, 1)}
    res["speedup_from_termination"] = round(res["no_termination"]["ms"] / res["t_min_1e-3"]["ms"], 2)
    del r
    torch.cuda.empty_cache()
    return res


def leg_variants(torch, sg, Renderer, reps=1):
    """forward_variants on the bench frame, for the profiler."""
    scene = sg.c2_scene()
    view = sg.c2_view()
    r = Renderer(0)
    r.load_blocks(scene.blocks)
    sel = r.select(view, thresholds=(1e30,), cull=True)
    mlp = torch.tensor(sg.xavier_mlp(1), device="cuda")
    return forward_variants(torch, sg, r, view, sel, sg.cityb_params(), mlp, None, reps=reps)


def leg_backward(torch, sg, Renderer, reps=2):
    """Backward throughput on the fp32 4x4 scene, 8 views at 800x800."""
    log("backward: generating the fp32 4x4 scene")
    learn, _ = sg.c5_scenes()
    views = sg.c5_views()
    p = sg.cityb_params()
    r = Renderer(0)
    r.load_blocks(learn.blocks)
    sets = [[(b.block_id, 0) for b in learn.blocks]] * len(views)
    mlp = torch.tensor(sg.xavier_mlp(4), device="cuda")
    out = r.render(views, sets, p, mlp, counts=True)
    n_eval = int(out["counts"][:, 0].sum().item())
    fwd_ms = _timed(torch, lambda: r.render(views, sets, p, mlp, out=out), reps)
    g = torch.randn_like(out["rgb"]) * 1e-3
    log(f"backward: first call ({n_eval} samples)")
    gg = [torch.zeros_like(t[0]) for t in r.textures]
    gp = [[torch.zeros_like(x) for x in t[1]] for t in r.textures]
    gm = torch.zeros(499, device="cuda")
    r.render_backward(views, sets, p, mlp, out["aux"], g, None, gg, gp, gm)
    torch.cuda.synchronize()
    r.set_timing(True)
    bt = []
    for _ in range(reps):
        r.render_backward(views, sets, p, mlp, out["aux"], g, None, gg, gp, gm)
        bt.append(r.last_timing()[1])
    r.set_timing(False)
    t = time.perf_counter()
    for _ in range(reps):
        r.render_backward(views, sets, p, mlp, out["aux"], g, None, gg, gp, gm)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / reps
    log(f"backward {ms:.1f} ms")
    res = {"Msamples_per_s": round(n_eval / (ms * 1e-3) / 1e6, 2), "ms": round(ms, 3),
           "march_bwd_ms": round(float(np.mean(bt)), 3), "evaluated_samples": n_eval,
           "workload": "4x4 fp32 blocks 128^3 + 3x1024^2, 8 views 800x800",
           "fwd_ms": round(fwd_ms, 3), "fwd_Msamples_per_s": round(n_eval / (fwd_ms * 1e-3) / 1e6, 1),
           "fwd_gathered_GBps": round(640 * n_eval / (fwd_ms * 1e-3) / 1e9, 1)}
    # the backward's options: the opacity-entropy gradient, per-block MLPs,
    # and the sparsity regulariser at 2^14 points (forward and gradient)
    w_op = torch.full((out["rgb"].shape[0],), 1e-3, device="cuda")
    ms = _timed(torch, lambda: r.render_backward(views, sets, p, mlp, out["aux"], g, None, gg, gp, gm,
                                                 opacity_weight=w_op), 1)
    res["with_opacity_entropy_ms"] = round(ms, 3)
    # the same two options with the forward's per-block composites handed over
    # (block_aux): the adjoint then marches each block once
    ba = torch.empty((out["rgb"].shape[0], max(len(s) for s in sets), 8), dtype=torch.float32, device="cuda")
    r.render(views, sets, p, mlp, out=out, block_aux=ba)
    ms = _timed(torch, lambda: r.render_backward(views, sets, p, mlp, out["aux"], g, None, gg, gp, gm,
                                                 opacity_weight=w_op, block_aux=ba), 1)
    res["with_opacity_entropy_block_aux_ms"] = round(ms, 3)
    bm = torch.tensor(np.stack([sg.xavier_mlp(200 + k) for k in range(len(r.blocks))]), device="cuda")
    gbm = torch.zeros_like(bm)
    out_b = r.render(views, sets, p, None, block_mlp=bm)
    ms = _timed(torch, lambda: r.render_backward(views, sets, p, None, out_b["aux"], g, None, gg, gp, None,
                                                 block_mlp=bm, grad_block_mlp=gbm), 1)
    res["per_block_mlps_ms"] = round(ms, 3)
    r.render(views, sets, p, None, block_mlp=bm, out=out_b, block_aux=ba)
    ms = _timed(torch, lambda: r.render_backward(views, sets, p, None, out_b["aux"], g, None, gg, gp, None,
                                                 block_mlp=bm, grad_block_mlp=gbm, block_aux=ba), 1)
    res["per_block_mlps_block_aux_ms"] = round(ms, 3)
    del out_b, ba
    pts = torch.rand((1 << 14, 3), device="cuda") * torch.tensor([4.0, 4.0, 1.0], device="cuda")
    refs = [(b.block_id, 0) for b in learn.blocks]
    ms = _timed(torch, lambda: r.sparsity(refs, pts, 1.0 / 512, 1e-3, grad_grid=gg, grad_plane=gp), 5)
    res["sparsity_2e14_points_ms"] = round(ms, 4)
    log("backward variants done")
    del r, gg, gp, out
    torch.cuda.empty_cache()
    # the same scene with its 12 edge blocks contracted and the exterior
    # sampled (ext_delta 1/64, at most 512 steps per segment): forward and
    # backward of the contraction kernels
    from dataclasses import replace
    rc = Renderer(0)
    rc.load_blocks(sg.contract_boundary(learn.blocks))
    pc = replace(p, ext_delta=1.0 / 64, ext_max_steps=512)
    oc = rc.render(views, sets, pc, mlp, counts=True)
    n_ct = int(oc["counts"][:, 0].sum().item())
    ct_fwd = _timed(torch, lambda: rc.render(views, sets, pc, mlp, out=oc), reps)
    gg = [torch.zeros_like(t[0]) for t in rc.textures]
    gp = [[torch.zeros_like(x) for x in t[1]] for t in rc.textures]
    ct_bwd = _timed(torch, lambda: rc.render_backward(views, sets, pc, mlp, oc["aux"], g, None, gg, gp, gm), reps)
    res["contracted"] = {"workload": "the same 4x4 fp32 scene, 12 edge blocks contracted, exterior ext_delta 1/64, "
                                     "<= 512 steps per segment", "evaluated_samples": n_ct,
                         "fwd_ms": round(ct_fwd, 3), "bwd_ms": round(ct_bwd, 3),
                         "bwd_Msamples_per_s": round(n_ct / (ct_bwd * 1e-3) / 1e6, 2)}
    log(f"backward, contracted: {ct_bwd:.1f} ms")
    del rc, gg, gp, oc, g
    torch.cuda.empty_cache()
    # the fp32 forward's gather rate against the probe at the same footprint
    from paper_2312_16457_amd import COW_F32
    from paper_2312_16457_amd.binding import gather_probe
    steps = max(1, int(round(n_eval / sum(v.n_pixels for v in views))))
    nbytes = 16 * (128 ** 3 + 3 * 1024 * 1024) * 32
    tex = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
    gather_probe(views[0], tex, 4, 4, 128, 1024, COW_F32, steps, 1.0 / 512)
    pms = min(gather_probe(views[0], tex, 4, 4, 128, 1024, COW_F32, steps, 1.0 / 512)[0] for _ in range(3))
    probe = views[0].n_pixels * steps * 640 / (pms * 1e-3) / 1e9
    res["fwd_gather_probe_GBps"] = round(probe, 1)
    res["fwd_gather_frac"] = round(res["fwd_gathered_GBps"] / probe, 4)
    # the fp32 forward's HBM reads per launch from its committed rocprofv3
    # FETCH_SIZE pass (null when the kernel's sources changed since)
    path = os.path.join(ROOT, "profiles", "traffic_march_fwd_f32_8x800.json")
    if os.path.exists(path):
        rec = json.load(open(path))
        if rec.get("source_digest") == source_digest():
            hbm = rec["hbm_read_bytes_per_launch"] / (fwd_ms * 1e-3) / 1e9
            res["fwd_hbm_read_GBps"] = round(hbm, 1)
            res["fwd_hbm_frac_of_peak"] = round(hbm / PEAK_HBM_GBS, 4)
    del tex
    torch.cuda.empty_cache()
    return res, learn


def _time_launches(torch, r, views, sets, p, mlp, reps, tag):
    """The batch three ways: one graph-replayed launch over every view, one
    fused launch (march + MLP) per view, and one launch per view per block
    (the paper's one-shader-per-block design)."""
    from paper_2312_16457_amd import F_GRAPH, F_PER_BLOCK
    out = r.render(views, sets, p, mlp, want_aux=False)
    timings = {}
    for name, flags in (("batched_graph", F_GRAPH), ("per_block_launches", F_PER_BLOCK)):
        log(f"{tag}: timing {name}")
        r.render(views, sets, p, mlp, out=out, flags=flags)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r.render(views, sets, p, mlp, out=out, flags=flags)
        torch.cuda.synchronize()
        timings[name] = (time.perf_counter() - t) * 1e3 / reps
    del out
    log(f"{tag}: timing per_view_launches")
    outs = [r.render([v], [s], p, mlp, want_aux=False) for v, s in zip(views, sets)]

    def per_view():
        for v, s, o in zip(views, sets, outs):
            r.render([v], [s], p, mlp, out=o)
    timings["per_view_launches"] = _timed(torch, per_view, reps)
    del outs
    return timings


def leg_batched(torch, sg, Renderer, reps=2):
    """64 views of mixed resolution over the 8x8x3-LOD scene in one
    graph-replayed launch vs one launch per view per block."""
    log("batched: generating the 8x8x3-LOD scene")
    scene = sg.c3_scene()
    views = sg.c4_views()
    p = sg.cityb_params()
    r = Renderer(0)
    r.load_blocks(scene.blocks)
    sets = [r.select(v, thresholds=(2.0, 4.0, 8.0), cull=True) for v in views]
    mlp = torch.tensor(sg.xavier_mlp(3), device="cuda")
    cnt = r.render(views, sets, p, mlp, counts=True)
    n_eval = int(cnt["counts"][:, 0].sum().item())
    n_pix = cnt["rgb"].shape[0]
    del cnt
    timings = _time_launches(torch, r, views, sets, p, mlp, reps, "batched")
    # the 16 aerial 1080p views of the LOD city, one launch per frame
    v16 = sg.c3_views()
    s16 = [r.select(v, thresholds=(2.0, 4.0, 8.0), cull=True) for v in v16]
    n16 = sum(int(r.render([v], [s], p, mlp, counts=True)["counts"][:, 0].sum().item()) for v, s in zip(v16, s16))
    outs = [r.render([v], [s], p, mlp, want_aux=False) for v, s in zip(v16, s16)]

    def frames():
        for v, s, o in zip(v16, s16, outs):
            r.render([v], [s], p, mlp, out=o)
    ms16 = _timed(torch, frames, reps)
    del outs
    tb = timings["batched_graph"]
    del r
    torch.cuda.empty_cache()
    # gather rate of the batch and of the 16 aerial frames against the probe
    # at the LOD city's footprint class (HBM-resident: 8 x 8 blocks of 128^3
    # + 3 x 1024^2, 2.5 GiB, at the batch's mean evaluated samples per ray)
    gat = lod_city_gather(torch, sg, n_eval / n_pix, {"batched_64_views": (n_eval, tb), "aerial_16x1080p": (n16, ms16)})
    res = {"views": len(views), "pixels": n_pix, "evaluated_samples": n_eval,
           "blocks_per_view": [min(len(s) for s in sets), max(len(s) for s in sets)],
           "launches_per_block_mode": sum(max(len(s), 1) for s in sets) + 1,
           "ms_batched": round(tb, 2), "ms_per_block": round(timings["per_block_launches"], 2),
           "ms_per_view": round(timings["per_view_launches"], 2),
           "speedup_vs_per_block": round(timings["per_block_launches"] / tb, 3),
           "speedup_vs_per_view": round(timings["per_view_launches"] / tb, 3),
           "Msamples_per_s": round(n_eval / (tb * 1e-3) / 1e6, 1),
           "fps_1080p_equivalent": round(n_pix / (tb * 1e-3) / 2073600, 2),
           "workload": "8x8 blocks x 3 LODs uint8, 64 views {256^2, 800^2, 1280x720, 1920x1080}",
           "aerial_16x1080p": {"ms_per_frame": round(ms16 / len(v16), 3), "fps": round(1e3 * len(v16) / ms16, 2),
                               "evaluated_samples": n16, "Msamples_per_s": round(n16 / (ms16 * 1e-3) / 1e6, 1),
                               "blocks_per_view": [min(len(x) for x in s16), max(len(x) for x in s16)]},
           "gather": gat}
    return res, scene


def lod_city_gather(torch, sg, steps_per_ray, legs):
    """The texel-gather probe on a 1920x1080 view over an 8 x 8 field of
    uint8 blocks of 128^3 + 3 x 1024^2 (2.5 GiB, the footprint class of the
    8x8x3-LOD city's 3.1 GiB), at the given mean evaluated samples per ray;
    each leg's gathered bytes per second (160 B per evaluated sample) as a
    fraction of it."""
    from paper_2312_16457_amd import COW_U8
    from paper_2312_16457_amd.binding import gather_probe
    view = sg.c2_view()
    steps = max(1, int(round(steps_per_ray)))
    nbytes = 64 * (128 ** 3 + 3 * 1024 * 1024) * 8
    tex = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
    gather_probe(view, tex, 8, 8, 128, 1024, COW_U8, steps, 1.0 / 512)
    best = min(gather_probe(view, tex, 8, 8, 128, 1024, COW_U8, steps, 1.0 / 512)[0] for _ in range(3))
    probe = view.n_pixels * steps * BYTES_PER_SAMPLE_U8 / (best * 1e-3) / 1e9
    del tex
    torch.cuda.empty_cache()
    out = {"probe_footprint_GiB": round(nbytes / 2 ** 30, 2), "probe_steps_per_ray": steps,
           "probe_GBps": round(probe, 1)}
    for name, (n, ms) in legs.items():
        gb = BYTES_PER_SAMPLE_U8 * n / (ms * 1e-3) / 1e9
        out[name] = {"gathered_GBps": round(gb, 1), "frac_of_probe": round(gb / probe, 4)}
    return out


def leg_single_block(torch, sg, Renderer, reps=20):
    """One fp32 block (32^3 grid, 128^2 planes), one 128x128 view, 128 chord
    steps per ray."""
    scene = sg.c1_scene()
    view = sg.c1_view()
    p = sg.c1_params()
    r = Renderer(0)
    r.load_blocks(scene.blocks)
    sets = [[(0, 0)]]
    mlp = torch.tensor(sg.xavier_mlp(0), device="cuda")
    n_eval = int(r.render([view], sets, p, mlp, counts=True)["counts"][:, 0].sum().item())
    out = r.render([view], sets, p, mlp, want_aux=False)
    ms = _timed(torch, lambda: r.render([view], sets, p, mlp, out=out), reps)
    from paper_2312_16457_amd import F_GRAPH
    ms_g = _timed(torch, lambda: r.render([view], sets, p, mlp, out=out, flags=F_GRAPH), reps)
    res = {"ms": round(ms, 4), "evaluated_samples": n_eval, "Msamples_per_s": round(n_eval / (ms * 1e-3) / 1e6, 1),
           "ms_graph": round(ms_g, 4), "Msamples_per_s_graph": round(n_eval / (ms_g * 1e-3) / 1e6, 1),
           "workload": "1 fp32 block 32^3 + 3x128^2, one 128x128 view, 128 chord steps"}
    del r
    return res


def leg_quadtree(torch, sg, Renderer, lod_city=None, reps=2):
    """The same 64 views over quadtree LODs: merged assets of 2x2 and 4x4 blocks."""
    log("quadtree: building the quadtree-LOD city")
    scene = sg.c3q_scene(lod_city=lod_city)
    views = sg.c4_views()
    p = sg.cityb_params()
    r = Renderer(0)
    r.load_blocks(scene.blocks)
    thr = sg.QUADTREE_THRESHOLDS
    sets = [r.select(v, thresholds=thr, cull=True, quadtree=True) for v in views]
    mlp = torch.tensor(sg.xavier_mlp(3), device="cuda")
    cnt = r.render(views, sets, p, mlp, counts=True)
    n_eval = int(cnt["counts"][:, 0].sum().item())
    n_pix = cnt["rgb"].shape[0]
    del cnt
    timings = _time_launches(torch, r, views, sets, p, mlp, reps, "quadtree")
    tb = timings["batched_graph"]
    res = {"views": len(views), "pixels": n_pix, "evaluated_samples": n_eval,
           "entries_per_view": [min(len(s) for s in sets), max(len(s) for s in sets)],
           "entries_by_lod": [sum(1 for s in sets for _, l in s if l == k) for k in range(3)],
           "ms_batched": round(tb, 2), "ms_per_block": round(timings["per_block_launches"], 2),
           "ms_per_view": round(timings["per_view_launches"], 2),
           "speedup_vs_per_block": round(timings["per_block_launches"] / tb, 3),
           "speedup_vs_per_view": round(timings["per_view_launches"] / tb, 3),
           "Msamples_per_s": round(n_eval / (tb * 1e-3) / 1e6, 1),
           "fps_1080p_equivalent": round(n_pix / (tb * 1e-3) / 2073600, 2),
           "workload": "8x8 blocks, quadtree LODs (merged 2x2 and 4x4 assets) uint8, thresholds "
                       "2 and 4, the same 64 views"}
    del r
    torch.cuda.empty_cache()
    return res


def extras(torch, sg, Renderer, cpu=None):
    """Backward throughput, the batched-vs-per-block comparison on the
    8x8x3-LOD scene and the same views over quadtree LODs.  cpu: the CPU
    baseline's dict, whose legs on these workloads' scenes are added here."""
    ex = {"single_block": leg_single_block(torch, sg, Renderer), "opaque": leg_opaque(torch, sg, Renderer),
          "empty_space": leg_empty_space(torch, sg, Renderer), "contracted": leg_contracted(torch, sg, Renderer)}
    ex["bwd"], learn = leg_backward(torch, sg, Renderer)
    if cpu is not None:
        cpu.setdefault("legs", {})["fp64_adjoint_c5_crop"] = cpu_baseline_adjoint(learn, sg)
        log("cpu baseline: adjoint leg done")
    del learn
    ex["batched"], lod_city = leg_batched(torch, sg, Renderer)
    if cpu is not None:
        cpu.setdefault("legs", {}).update(cpu_baseline_lod(lod_city, sg))
        log("cpu baseline: LOD city legs done")
    ex["quadtree"] = leg_quadtree(torch, sg, Renderer, lod_city=lod_city)
    return ex


if __name__ == "__main__":
    main()
