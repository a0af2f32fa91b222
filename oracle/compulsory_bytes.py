"""Compulsory HBM bytes of the 4x4 uint8 bench frame, counted by the oracle.

Run from the repository root: python -m oracle.compulsory_bytes [--rows-every N]
Writes profiles/compulsory_bytes_4x4_1080p.json.

The compulsory bytes of one render are the texture bytes its evaluated
samples read at least once, plus the occupancy bytes and the outputs.  The
oracle takes the same sample decisions as the render (exact fp32), so its
touched-texel masks are those of the frame.  Two granularities: unique
texels (8 bytes each, uint8 x 8 channels) and unique 128-byte lines of each
texture (the L2/HBM transfer unit), each texture starting on a line boundary.
This is test and measurement infrastructure: only this script, the tests and
the benchmark's CPU leg call the oracle."""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2312_16457_amd import scenegen as sg  # noqa: E402

LINE = 128


def count(masks, texel_bytes):
    texels = 0
    lines = 0
    per_line = LINE // texel_bytes
    for ms in masks.values():
        for m in ms:
            flat = m.reshape(-1)
            texels += int(flat.sum())
            n = flat.size
            pad = (-n) % per_line
            lines += int(np.pad(flat, (0, pad)).reshape(-1, per_line).any(axis=1).sum())
    return texels * texel_bytes, lines * LINE


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rows-every", type=int, default=1, help="count over every Nth image row only")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "compulsory_bytes_4x4_1080p.json"))
    args = ap.parse_args()
    t0 = time.time()
    scene = sg.c2_scene()
    view = sg.c2_view()
    params = sg.cityb_params()
    ob = O.OracleScene(scene.blocks)
    occs = [O.occupancy(ob, k) for k in range(ob.n)]
    zt = [O.ztop(ob, k, occs[k]) for k in range(ob.n)]
    sel = [int(k) for k in O.select(view, scene.blocks, zt, thresholds=(1e30,), cull=True)]
    rows = np.arange(0, view.H, args.rows_every)
    pix = O.pixels_of(view, rows=rows)
    masks = O.touched_texels(ob, occs, view, sel, params, pix=pix)
    tex_b, line_b = count(masks, 8)
    all_tex = sum(b.grid.nbytes + sum(p.nbytes for p in b.planes) for k, b in enumerate(scene.blocks) if k in sel)
    occ_b = sum(o.size for k, o in enumerate(occs) if k in sel)
    n_pix = len(pix)
    rec = {
        "workload": "4x4 uint8 blocks (128^3 grid + 3 x 1024^2 planes, 16^3 occupancy), one 1920x1080 view, "
                    "delta 1/512, <= 2048 steps",
        "rows": "all" if args.rows_every == 1 else f"every {args.rows_every}th row",
        "pixels": n_pix,
        "blocks": len(sel),
        "texture_bytes_loaded": int(all_tex),
        "touched_texel_bytes": tex_b,
        "touched_line_bytes": line_b,
        "occupancy_bytes": int(2 * occ_b),
        "output_bytes_march": 36 * n_pix,
        "output_bytes_frame": 48 * n_pix + 32 * n_pix,
        "compulsory_bytes_march": int(line_b + 2 * occ_b + 36 * n_pix),
        "note": "march: touched 128-byte texture lines + occupancy and skip bytes + aux (32 B) and T (4 B) "
                "written per pixel; the frame adds the MLP pass (reads aux 32 B, writes rgb 12 B)",
        "command": "python -m oracle.compulsory_bytes" + ("" if args.rows_every == 1 else
                                                          f" --rows-every {args.rows_every}"),
        "seconds": round(time.time() - t0, 1),
    }
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
