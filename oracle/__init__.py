"""CPU oracle for block-merged ray marching (City-on-Web, arXiv 2312.16457).

TEST INFRASTRUCTURE ONLY: the plain definition that the GPU renderer is
checked against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the renderer never does, and the
two share no code.  The C source (oracle.c) holds the arithmetic; this module
only marshals numpy arrays.

Pinning status of each function (what fixes it other than itself) is listed
in tests/test_oracle_pins.py; there is no "parity unpinned" function here
except the scene-level appearance (see the module docstring of those tests).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
# the same source with single-precision continuous arithmetic, for timing only
LIB32 = os.path.join(HERE, "liboracle_f32.so")

MERGED, MONOLITHIC, REVERSED, BY_ID, ALPHA_NORM, BLOCK_MLP = range(6)


def build():
    """Compile oracle.c with gcc: fp32 decisions must not be contracted.  Also
    the single-precision build (continuous per-sample arithmetic in float,
    the same decisions), which only the benchmark's CPU baseline times."""
    base = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]
    src = os.path.join(HERE, "oracle.c")
    subprocess.check_call(base + ["-o", LIB, src, "-lm"])
    subprocess.check_call(base + ["-DORC_REAL=float", "-o", LIB32, src, "-lm"])


class _Block(C.Structure):
    _fields_ = [
        ("block_id", C.c_int), ("lod", C.c_int),
        ("lo", C.c_float * 3), ("hi", C.c_float * 3),
        ("R", C.c_int), ("Rp", C.c_int), ("O", C.c_int),
        ("dtype", C.c_int),
        ("g8", C.c_void_p), ("p8", C.c_void_p * 3),
        ("gf", C.c_void_p), ("pf", C.c_void_p * 3),
        ("scale", (C.c_float * 8) * 4), ("offset", (C.c_float * 8) * 4),
        ("contracted", C.c_int),
    ]


class _View(C.Structure):
    _fields_ = [
        ("W", C.c_int), ("H", C.c_int), ("x0", C.c_int), ("y0", C.c_int), ("w", C.c_int), ("h", C.c_int),
        ("eye", C.c_float * 3), ("R", C.c_float * 9),
        ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
    ]


class _Params(C.Structure):
    _fields_ = [("mode", C.c_int), ("n_steps", C.c_int), ("delta", C.c_float), ("max_steps", C.c_int),
                ("t_min", C.c_float), ("pe", C.c_int), ("ext_delta", C.c_float), ("ext_max_steps", C.c_int)]


_libs = {}


def lib(fp32=False):
    """The oracle library; fp32=True: its single-precision build (timing only)."""
    path = LIB32 if fp32 else LIB
    if path not in _libs:
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
        L.orc_occupancy.argtypes = [C.POINTER(_Block), vp]
        L.orc_ztop.argtypes = [C.POINTER(_Block), vp]
        L.orc_occupancy_level.argtypes = [C.POINTER(_Block), vp, C.c_int, vp]
        L.orc_ztop.restype = C.c_double
        L.orc_render.argtypes = [C.POINTER(_Block), C.c_int, C.POINTER(C.c_void_p), C.POINTER(_View),
                                 vp, C.c_int, C.POINTER(_Params), vp, vp, C.c_int, C.c_int,
                                 vp, vp, vp, vp, vp, vp, C.c_int]
        L.orc_ray_blocks.argtypes = [C.POINTER(_Block), C.c_int, C.POINTER(_View), vp, C.c_int,
                                     C.POINTER(_Params), C.c_int, C.c_int, vp, C.c_int]
        L.orc_adjoint.argtypes = [C.POINTER(_Block), C.c_int, C.POINTER(C.c_void_p), C.POINTER(_View),
                                  vp, C.c_int, C.POINTER(_Params), vp, vp, C.c_int, vp, vp, vp,
                                  C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), vp]
        L.orc_adjoint_block_mlp.argtypes = [C.POINTER(_Block), C.c_int, C.POINTER(C.c_void_p), C.POINTER(_View),
                                            vp, C.c_int, C.POINTER(_Params), vp, vp, C.c_int, vp, vp, vp,
                                            C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), vp]
        L.orc_opacity.argtypes = [C.POINTER(_Block), C.c_int, C.POINTER(C.c_void_p), C.POINTER(_View),
                                  vp, C.c_int, C.POINTER(_Params), vp, C.c_int, vp]
        L.orc_sparsity.argtypes = [C.POINTER(_Block), C.c_int, C.POINTER(C.c_void_p), vp, C.c_int, vp,
                                   C.c_int, C.c_double, C.c_double, vp, C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_void_p)]
        L.orc_sparsity.restype = C.c_double
        L.orc_select.argtypes = [C.POINTER(_View), C.c_int, vp, vp, vp, vp, vp, vp, vp, C.c_int, C.c_int,
                                 vp, C.c_int]
        L.orc_select_quadtree.argtypes = L.orc_select.argtypes
        L.orc_touched_texels.argtypes = [C.POINTER(_Block), C.c_int, C.POINTER(C.c_void_p), C.POINTER(_View), vp,
                                         C.c_int, C.POINTER(_Params), vp, C.c_long, C.POINTER(C.c_void_p), C.c_int]
        L.orc_mlp.argtypes = [vp, vp, vp]
        L.orc_mlp_pe.argtypes = [vp, C.c_int, vp, vp]
        L.orc_mlp_params.argtypes = [C.c_int]
        L.orc_mlp_params.restype = C.c_long
        L.orc_posenc.argtypes = [vp, C.c_int, vp]
        L.orc_contract.argtypes = [vp, vp]
        L.orc_contract.restype = None
        L.orc_local_q.argtypes = [C.POINTER(_Block), vp, vp]
        L.orc_local_q.restype = C.c_float
        L.orc_ext_samples.argtypes = [C.POINTER(_Block), C.c_int, C.POINTER(C.c_void_p), vp, C.c_int,
                                      C.POINTER(_Params), vp, vp, C.c_float, C.c_float, C.c_int, vp, vp, C.c_long]
        L.orc_ext_samples.restype = C.c_long
        L.orc_field.argtypes = [C.POINTER(_Block), C.c_int, vp, vp]
        _libs[path] = L
    return _libs[path]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_view(v):
    s = _View()
    s.W, s.H = int(v.W), int(v.H)
    s.x0, s.y0, s.w, s.h = (int(x) for x in v.crop)
    s.eye[:] = [float(x) for x in np.asarray(v.eye, np.float32)]
    s.R[:] = [float(x) for x in np.asarray(v.R, np.float32).reshape(-1)]
    s.fx, s.fy, s.cx, s.cy = v.fx, v.fy, v.cx, v.cy
    return s


def make_params(p):
    s = _Params()
    s.mode, s.n_steps, s.delta, s.max_steps = int(p.mode), int(p.n_steps), float(p.delta), int(p.max_steps)
    s.t_min = float(getattr(p, "t_min", 0.0))
    s.pe = int(getattr(p, "pe_freqs", 0))
    s.ext_delta = float(getattr(p, "ext_delta", 0.0))
    s.ext_max_steps = int(getattr(p, "ext_max_steps", 0))
    return s


def mlp_params(pe=0):
    """Weights of the deferred MLP over 10 + 6 pe inputs (499 for pe = 0)."""
    return int(lib().orc_mlp_params(int(pe)))


def contract(x):
    """MERF's contraction (max norm) of one point, fp64: identity inside the
    unit cube, everything else into the cube of radius 2."""
    y = np.zeros(3, np.float64)
    lib().orc_contract(_ptr(np.ascontiguousarray(x, np.float64)), _ptr(y))
    return y


def local_q(ob, k, p):
    """fp32 texture-space coordinate of world point p in block k (the
    decision sequence) and the max norm of its box-normalised coordinate."""
    q = np.zeros(3, np.float32)
    m = lib().orc_local_q(C.byref(ob.arr[k]), _ptr(np.ascontiguousarray(p, np.float32)), _ptr(q))
    return q, float(m)


def ext_samples(ob, occs, set_idx, params, o, d, t_start, t_end, post, cap=4096):
    """Texture coordinates and step lengths of the samples of one exterior
    segment of the ray (o, d)."""
    q = np.zeros((cap, 3), np.float32)
    dl = np.zeros(cap, np.float64)
    s = np.ascontiguousarray(set_idx, np.int32)
    pr = make_params(params)
    n = lib().orc_ext_samples(ob.arr, ob.n, _occ_ptrs(ob, occs), _ptr(s), len(s), C.byref(pr),
                              _ptr(np.ascontiguousarray(o, np.float32)), _ptr(np.ascontiguousarray(d, np.float32)),
                              float(t_start), float(t_end), int(post), _ptr(q), _ptr(dl), cap)
    return q[:n], dl[:n]


def posenc(d, pe):
    """[d, sin(2^l d), cos(2^l d) for l < pe] of one direction (3 + 6 pe values)."""
    out = np.zeros(3 + 6 * pe, np.float64)
    if lib().orc_posenc(_ptr(np.ascontiguousarray(d, np.float64)), int(pe), _ptr(out)) < 0:
        raise ValueError("pe must be 0-4")
    return out


class OracleScene:
    """ctypes view of a list of BlockLod entries.

    uint8 blocks are passed as bytes plus their fp32 scale/offset; float blocks
    are held as fp64 copies (exact), which tests may perturb in place for
    finite differences.  `need` restricts which blocks get textures (others
    only contribute their AABB to the scene box)."""

    def __init__(self, blocks, need=None):
        self.blocks = list(blocks)
        self.n = len(self.blocks)
        self.arr = (_Block * self.n)()
        self.keep = []
        self.f64 = {}
        for k, b in enumerate(self.blocks):
            s = self.arr[k]
            s.block_id, s.lod = int(b.block_id), int(b.lod)
            s.lo[:] = [float(x) for x in b.aabb_min]
            s.hi[:] = [float(x) for x in b.aabb_max]
            s.R, s.Rp, s.O = int(b.grid_res), int(b.plane_res), int(b.occ_res)
            s.contracted = int(bool(getattr(b, "contracted", False)))
            for t in range(4):
                s.scale[t][:] = [float(x) for x in b.scale[t]]
                s.offset[t][:] = [float(x) for x in b.offset[t]]
            if need is not None and k not in need:
                s.dtype = 1 if b.dtype == 1 else 0
                continue
            if b.dtype == 0:
                s.dtype = 0
                g = np.ascontiguousarray(b.grid)
                ps = [np.ascontiguousarray(p) for p in b.planes]
                self.keep += [g] + ps
                s.g8 = g.ctypes.data
                for i in range(3):
                    s.p8[i] = ps[i].ctypes.data
            else:
                s.dtype = 1
                g = np.ascontiguousarray(b.grid, dtype=np.float64)
                ps = [np.ascontiguousarray(p, dtype=np.float64) for p in b.planes]
                self.f64[k] = (g, ps)
                s.gf = g.ctypes.data
                for i in range(3):
                    s.pf[i] = ps[i].ctypes.data

    def index(self, block_id, lod):
        for k, b in enumerate(self.blocks):
            if b.block_id == block_id and b.lod == lod:
                return k
        raise KeyError((block_id, lod))


def dims(b, res):
    """(z, y, x) texel or cell counts of a block: res per unit length times
    the block's extent on each axis."""
    ext = [int(round(float(b.aabb_max[c]) - float(b.aabb_min[c]))) for c in range(3)]
    return (res * ext[2], res * ext[1], res * ext[0])


def occupancy(ob, k):
    b = ob.blocks[k]
    out = np.zeros(dims(b, b.occ_res), np.uint8)
    r = lib().orc_occupancy(C.byref(ob.arr[k]), _ptr(out))
    if r != 0:
        raise ValueError("bad resolutions")
    return out


def occupancy_level(ob, k, occ, level):
    """Level `level` of the max-pooled occupancy pyramid of entry k, shape
    (max(Cz >> l, 1), max(Cy >> l, 1), max(Cx >> l, 1))."""
    shape = tuple(max(n >> level, 1) for n in occ.shape)
    out = np.zeros(shape, np.uint8)
    r = lib().orc_occupancy_level(C.byref(ob.arr[k]), _ptr(np.ascontiguousarray(occ, np.uint8)), level, _ptr(out))
    if r != 0:
        raise ValueError("bad level")
    return out


def occupancy_levels(occ):
    """Number of pyramid levels above the base: log2 of the largest axis."""
    return int(max(occ.shape)).bit_length() - 1


def ztop(ob, k, occ):
    return lib().orc_ztop(C.byref(ob.arr[k]), _ptr(np.ascontiguousarray(occ)))


def _occ_ptrs(ob, occs):
    arr = (C.c_void_p * ob.n)()
    for k in range(ob.n):
        o = occs.get(k) if isinstance(occs, dict) else occs[k]
        arr[k] = None if o is None else o.ctypes.data
    return arr


def pixels_of(view, rows=None, stride=1):
    """Absolute pixel coordinates of a view's crop, row-major (optionally a
    subset of rows)."""
    x0, y0, w, h = view.crop
    ys = np.arange(y0, y0 + h) if rows is None else np.asarray(rows)
    ys = ys[::stride] if rows is None else ys
    xs = np.arange(x0, x0 + w)
    jj, ii = np.meshgrid(ys, xs, indexing="ij")
    return np.stack([ii.reshape(-1), jj.reshape(-1)], axis=1).astype(np.int32)


def render(ob, occs, view, set_idx, params, mlp, pix=None, composite=MERGED, nthreads=0, fp32=False):
    """fp32=True runs the single-precision build (for timing; not the oracle)."""
    L = lib(fp32)
    if pix is None:
        pix = pixels_of(view)
    pix = np.ascontiguousarray(pix, np.int32)
    n = pix.shape[0]
    setv = np.ascontiguousarray(set_idx, np.int32)
    w = np.ascontiguousarray(mlp, np.float64)
    npar = mlp_params(getattr(params, "pe_freqs", 0))
    if composite == BLOCK_MLP and w.size != npar * ob.n:
        raise ValueError("BLOCK_MLP needs one MLP per entry of the scene")
    if composite != BLOCK_MLP and w.size != npar:
        raise ValueError("the MLP has %d weights" % npar)
    out = dict(rgb=np.zeros((n, 3)), trans=np.zeros(n), aux=np.zeros((n, 8)),
               n_eval=np.zeros(n, np.int64), n_march=np.zeros(n, np.int64),
               order_ok=np.zeros(n, np.int32))
    vs, ps = make_view(view), make_params(params)
    L.orc_render(ob.arr, ob.n, _occ_ptrs(ob, occs), C.byref(vs), _ptr(setv), len(setv), C.byref(ps),
                 _ptr(w), _ptr(pix), n, composite, _ptr(out["rgb"]), _ptr(out["trans"]),
                 _ptr(out["aux"]), _ptr(out["n_eval"]), _ptr(out["n_march"]),
                 _ptr(out["order_ok"]), int(nthreads))
    return out


def touched_texels(ob, occs, view, set_idx, params, pix=None, nthreads=0):
    """Per entry of set_idx: four uint8 masks (grid [z][y][x], then the xy,
    xz, yz planes [v][u]) with 1 at every texel the evaluated samples of the
    given pixels read (t_min = 0, plain blocks)."""
    if pix is None:
        pix = pixels_of(view)
    pix = np.ascontiguousarray(pix, np.int32)
    setv = np.ascontiguousarray(set_idx, np.int32)
    masks = {}
    arr = (C.c_void_p * (4 * ob.n))()
    for k in setv:
        b = ob.blocks[int(k)]
        ms = [np.zeros(b.grid.shape[:3], np.uint8)] + [np.zeros(p.shape[:2], np.uint8) for p in b.planes]
        masks[int(k)] = ms
        for t in range(4):
            arr[4 * int(k) + t] = ms[t].ctypes.data
    vs, ps = make_view(view), make_params(params)
    r = lib().orc_touched_texels(ob.arr, ob.n, _occ_ptrs(ob, occs), C.byref(vs), _ptr(setv), len(setv), C.byref(ps),
                                 _ptr(pix), pix.shape[0], arr, int(nthreads))
    if r != 0:
        raise ValueError("touched texels need t_min = 0 and plain blocks")
    return masks


def ray_blocks(ob, view, set_idx, params, i, j, cap=128):
    setv = np.ascontiguousarray(set_idx, np.int32)
    out = np.zeros(cap, np.int32)
    vs, ps = make_view(view), make_params(params)
    m = lib().orc_ray_blocks(ob.arr, ob.n, C.byref(vs), _ptr(setv), len(setv), C.byref(ps), int(i),
                             int(j), _ptr(out), cap)
    return out[:m]


def _grad_arrays(ob, idx):
    grads = {}
    gg = (C.c_void_p * ob.n)()
    gp = (C.c_void_p * (3 * ob.n))()
    for k in idx:
        b = ob.blocks[k]
        g = np.zeros(b.grid.shape, np.float64)
        ps = [np.zeros(p.shape, np.float64) for p in b.planes]
        grads[k] = (g, ps)
        gg[k] = g.ctypes.data
        for i in range(3):
            gp[3 * k + i] = ps[i].ctypes.data
    return grads, gg, gp


def opacity(ob, occs, view, set_idx, params, pix):
    """Per-ray block-opacity entropy."""
    pix = np.ascontiguousarray(pix, np.int32)
    setv = np.ascontiguousarray(set_idx, np.int32)
    out = np.zeros(pix.shape[0])
    vs, ps = make_view(view), make_params(params)
    lib().orc_opacity(ob.arr, ob.n, _occ_ptrs(ob, occs), C.byref(vs), _ptr(setv), len(setv), C.byref(ps),
                      _ptr(pix), pix.shape[0], _ptr(out))
    return out


def sparsity(ob, occs, set_idx, pts, delta, weight=1.0, want_alpha=False, want_grad=True):
    """L1 opacity sparsity at points; returns (loss, {block: (grad_grid,
    [grad_planes])}), plus alpha per point with want_alpha.  Gradients need
    fp64 blocks (want_grad=False for others)."""
    setv = np.ascontiguousarray(set_idx, np.int32)
    pts = np.ascontiguousarray(pts, np.float32)
    alpha = np.zeros(pts.shape[0])
    if want_grad:
        grads, gg, gp = _grad_arrays(ob, set(int(s) for s in setv))
    else:
        grads, gg, gp = {}, None, None
    loss = lib().orc_sparsity(ob.arr, ob.n, _occ_ptrs(ob, occs), _ptr(setv), len(setv), _ptr(pts), pts.shape[0],
                              float(delta), float(weight), _ptr(alpha), gg, gp)
    return (loss, grads, alpha) if want_alpha else (loss, grads)


def adjoint(ob, occs, view, set_idx, params, mlp, pix, grad_rgb, grad_trans=None, w_opacity=None):
    """fp64 adjoint; returns ({block index: (grad_grid, [grad_planes])}, grad_mlp)."""
    L = lib()
    pix = np.ascontiguousarray(pix, np.int32)
    setv = np.ascontiguousarray(set_idx, np.int32)
    grads = {}
    gg = (C.c_void_p * ob.n)()
    gp = (C.c_void_p * (3 * ob.n))()
    for k in set(int(s) for s in setv):
        b = ob.blocks[k]
        g = np.zeros(b.grid.shape, np.float64)
        ps = [np.zeros(p.shape, np.float64) for p in b.planes]
        grads[k] = (g, ps)
        gg[k] = g.ctypes.data
        for i in range(3):
            gp[3 * k + i] = ps[i].ctypes.data
    gm = np.zeros(mlp_params(getattr(params, "pe_freqs", 0)), np.float64)
    if np.asarray(mlp).size != gm.size:
        raise ValueError("the MLP has %d weights" % gm.size)
    gr = np.ascontiguousarray(grad_rgb, np.float64)
    gt = None if grad_trans is None else np.ascontiguousarray(grad_trans, np.float64)
    wo = None if w_opacity is None else np.ascontiguousarray(w_opacity, np.float64)
    vs, ps_ = make_view(view), make_params(params)
    r = L.orc_adjoint(ob.arr, ob.n, _occ_ptrs(ob, occs), C.byref(vs), _ptr(setv), len(setv),
                      C.byref(ps_), _ptr(np.ascontiguousarray(mlp, np.float64)), _ptr(pix), pix.shape[0],
                      _ptr(gr), _ptr(gt), _ptr(wo), gg, gp, _ptr(gm))
    if r != 0:
        raise ValueError("adjoint needs float blocks (contracted ones: valid extents, no opacity term)")
    return grads, gm


def adjoint_block_mlp(ob, occs, view, set_idx, params, mlps, pix, grad_rgb, grad_trans=None, w_opacity=None):
    """fp64 adjoint of the per-block deferred composite (BLOCK_MLP);
    mlps [ob.n][P] (P = mlp_params(params.pe_freqs)); returns ({block: (grad_grid,
    [grad_planes])}, grad_mlps [ob.n][P])."""
    L = lib()
    pix = np.ascontiguousarray(pix, np.int32)
    setv = np.ascontiguousarray(set_idx, np.int32)
    grads, gg, gp = _grad_arrays(ob, set(int(s) for s in setv))
    w = np.ascontiguousarray(mlps, np.float64).reshape(-1)
    npar = mlp_params(getattr(params, "pe_freqs", 0))
    if w.size != npar * ob.n:
        raise ValueError("one MLP per entry of the scene")
    gm = np.zeros(npar * ob.n, np.float64)
    gr = np.ascontiguousarray(grad_rgb, np.float64)
    gt = None if grad_trans is None else np.ascontiguousarray(grad_trans, np.float64)
    wo = None if w_opacity is None else np.ascontiguousarray(w_opacity, np.float64)
    vs, ps_ = make_view(view), make_params(params)
    r = L.orc_adjoint_block_mlp(ob.arr, ob.n, _occ_ptrs(ob, occs), C.byref(vs), _ptr(setv), len(setv),
                                C.byref(ps_), _ptr(w), _ptr(pix), pix.shape[0], _ptr(gr), _ptr(gt), _ptr(wo),
                                gg, gp, _ptr(gm))
    if r != 0:
        raise ValueError("adjoint needs float blocks, none of them contracted")
    return grads, gm.reshape(ob.n, npar)


def select(view, entries, ztops, thresholds=(2.0, 4.0, 8.0), cull=True, cap=4096, quadtree=False):
    """entries: list of BlockLod (or objects with block_id, lod, aabb_min, aabb_max
    and optionally contracted); ztops: per entry.  Returns chosen entry indices
    in front-to-back order.
    quadtree: entries of LOD l are merged assets over 2^l x 2^l blocks."""
    n = len(entries)
    ids = np.array([e.block_id for e in entries], np.int32)
    lods = np.array([e.lod for e in entries], np.int32)
    lo = np.array([e.aabb_min for e in entries], np.float32).reshape(-1)
    hi = np.array([e.aabb_max for e in entries], np.float32).reshape(-1)
    zt = np.ascontiguousarray(ztops, np.float64)
    ct = np.array([int(bool(getattr(e, "contracted", False))) for e in entries], np.int32)
    thr = np.ascontiguousarray(thresholds, np.float64)
    out = np.zeros(cap, np.int32)
    vs = make_view(view)
    fn = lib().orc_select_quadtree if quadtree else lib().orc_select
    m = fn(C.byref(vs), n, _ptr(ids), _ptr(lods), _ptr(lo), _ptr(hi), _ptr(zt), _ptr(ct), _ptr(thr),
           len(thr), int(cull), _ptr(out), cap)
    if m == -3:
        raise ValueError("quadtree selection needs a threshold for every LOD below the coarsest")
    if m < 0:
        raise KeyError("selected (block, LOD) not loaded")
    return out[:m]


def mlp(w, x, pe=0):
    """sigmoid(Phi(x)) for x = [C_d, F, PE(d)] (10 + 6 pe values)."""
    x = np.ascontiguousarray(x, np.float64)
    if x.size != 10 + 6 * pe or np.asarray(w).size != mlp_params(pe):
        raise ValueError("input or weight count does not match pe")
    out = np.zeros(3)
    lib().orc_mlp_pe(_ptr(np.ascontiguousarray(w, np.float64)), int(pe), _ptr(x), _ptr(out))
    return out


def field(ob, k, pts):
    """Pre-activation features (8 channels, fp64) at world points pts[n][3]."""
    pts = np.ascontiguousarray(pts, np.float32)
    out = np.zeros((pts.shape[0], 8))
    lib().orc_field(C.byref(ob.arr[k]), pts.shape[0], _ptr(pts), _ptr(out))
    return out
