"""ctypes binding of libcow.so (include/cow.h) with torch tensors as the
device-memory and stream plumbing.  Argument marshalling only: every step of
the render runs in the HIP library, and a missing library is an error."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcow.so")

COW_OK, COW_E_INVALID, COW_E_NOT_LOADED, COW_E_WORKSPACE, COW_E_UNSUPPORTED, COW_E_HIP, COW_E_INTERNAL = range(7)
COW_U8, COW_F32 = 0, 1
MODE_CHORD, MODE_GRID = 0, 1
F_NONE, F_GRAPH, F_PERSISTENT, F_PER_BLOCK, F_SPARSE, F_FLAT_OCC = 0, 1, 2, 4, 8, 16
BLOCK_CONTRACTED = 1  # cow_block_desc.flags: boundary block over the contracted cube

EXPORTS = ["cow_create", "cow_destroy", "cow_last_error", "cow_query_workspace", "cow_load_blocks",
           "cow_get_occupancy", "cow_get_occupancy_level", "cow_select_blocks", "cow_query_bricks", "cow_pack_bricks", "cow_render", "cow_render_noalloc",
           "cow_render_backward", "cow_sparsity", "cow_autotune", "cow_get_config", "cow_set_config",
           "cow_set_timing", "cow_last_timing", "cow_gather_probe"]


class CowError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"cow status {status}: {msg}")
        self.status = status


class BlockDesc(C.Structure):
    _fields_ = [("block_id", C.c_int32), ("lod", C.c_int32),
                ("aabb_min", C.c_float * 3), ("aabb_max", C.c_float * 3),
                ("grid_res", C.c_int32), ("plane_res", C.c_int32), ("occ_res", C.c_int32),
                ("dtype", C.c_int32), ("grid", C.c_void_p), ("plane", C.c_void_p * 3),
                ("scale", (C.c_float * 8) * 4), ("offset", (C.c_float * 8) * 4), ("flags", C.c_int32)]


class View(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("crop_x0", C.c_int32), ("crop_y0", C.c_int32),
                ("crop_w", C.c_int32), ("crop_h", C.c_int32), ("eye", C.c_float * 3), ("R", C.c_float * 9),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float)]


class BlockRef(C.Structure):
    _fields_ = [("block_id", C.c_int32), ("lod", C.c_int32)]


class BlockSet(C.Structure):
    _fields_ = [("refs", C.POINTER(BlockRef)), ("n", C.c_int32)]


class LodPolicy(C.Structure):
    _fields_ = [("thresholds", C.c_double * 3), ("n_thresholds", C.c_int32), ("cull", C.c_int32),
                ("quadtree", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_steps", C.c_int32), ("delta", C.c_float), ("max_steps", C.c_int32),
                ("t_min", C.c_float), ("flags", C.c_int32), ("counts", C.c_void_p), ("opacity", C.c_void_p),
                ("opacity_weight", C.c_void_p), ("block_mlp", C.c_void_p), ("grad_block_mlp", C.c_void_p),
                ("pe_freqs", C.c_int32), ("ext_delta", C.c_float), ("ext_max_steps", C.c_int32),
                ("block_aux", C.c_void_p), ("block_aux_n", C.c_int32)]


_lib = None


def lib():
    """Load the built library; raise if it is absent (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        P, vp = C.POINTER, C.c_void_p
        L.cow_create.argtypes = [P(vp), C.c_int]
        L.cow_destroy.argtypes = [vp]
        L.cow_last_error.argtypes = [vp]
        L.cow_last_error.restype = C.c_char_p
        L.cow_query_workspace.argtypes = [vp, P(BlockDesc), C.c_int, C.c_int, C.c_int64, P(C.c_size_t),
                                          P(C.c_size_t), P(C.c_size_t)]
        L.cow_load_blocks.argtypes = [vp, P(BlockDesc), C.c_int, vp, C.c_size_t, vp]
        L.cow_get_occupancy.argtypes = [vp, C.c_int, C.c_int, vp, C.c_size_t]
        L.cow_get_occupancy_level.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, C.c_size_t]
        L.cow_select_blocks.argtypes = [vp, P(View), P(LodPolicy), P(BlockRef), C.c_int, P(C.c_int)]
        L.cow_query_bricks.argtypes = [vp, P(C.c_size_t)]
        L.cow_pack_bricks.argtypes = [vp, vp, C.c_size_t, vp]
        L.cow_render.argtypes = [vp, P(View), C.c_int, P(BlockSet), P(Params), vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.cow_render_noalloc.argtypes = [vp, P(View), C.c_int, P(BlockSet), P(Params), vp, vp, vp, vp, vp]
        L.cow_render_backward.argtypes = [vp, P(View), C.c_int, P(BlockSet), P(Params), vp, vp, vp, vp,
                                          P(vp), P(vp), vp, vp, C.c_size_t, vp]
        L.cow_sparsity.argtypes = [vp, P(BlockSet), vp, C.c_int64, C.c_float, C.c_float, vp, vp, vp, vp, vp,
                                   C.c_size_t, vp]
        L.cow_autotune.argtypes = [vp, P(View), C.c_int, P(BlockSet), P(Params), vp, vp, C.c_size_t, C.c_char_p, vp]
        L.cow_get_config.argtypes = [vp, P(C.c_int), P(C.c_int), P(C.c_int)]
        L.cow_set_config.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.cow_set_timing.argtypes = [vp, C.c_int]
        L.cow_last_timing.argtypes = [vp, P(C.c_float), P(C.c_float)]
        L.cow_gather_probe.argtypes = [P(View), vp, C.c_size_t, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                       C.c_int, C.c_float, vp, P(C.c_float), vp]
        for name in EXPORTS:
            if name != "cow_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def make_view(v):
    s = View()
    s.W, s.H = int(v.W), int(v.H)
    s.crop_x0, s.crop_y0, s.crop_w, s.crop_h = (int(x) for x in v.crop)
    s.eye[:] = [float(x) for x in np.asarray(v.eye, np.float32)]
    s.R[:] = [float(x) for x in np.asarray(v.R, np.float32).reshape(-1)]
    s.fx, s.fy, s.cx, s.cy = float(v.fx), float(v.fy), float(v.cx), float(v.cy)
    return s


def make_params(p, flags=0, counts=None, opacity=None, opacity_weight=None, block_mlp=None, grad_block_mlp=None,
                block_aux=None):
    s = Params()
    s.mode, s.n_steps, s.delta, s.max_steps = int(p.mode), int(p.n_steps), float(p.delta), int(p.max_steps)
    s.t_min = float(getattr(p, "t_min", 0.0))
    s.flags = int(flags)
    s.counts = None if counts is None else counts.data_ptr()
    s.opacity = None if opacity is None else opacity.data_ptr()
    s.opacity_weight = None if opacity_weight is None else opacity_weight.data_ptr()
    s.block_mlp = None if block_mlp is None else block_mlp.data_ptr()
    s.grad_block_mlp = None if grad_block_mlp is None else grad_block_mlp.data_ptr()
    s.pe_freqs = int(getattr(p, "pe_freqs", 0))
    s.ext_delta = float(getattr(p, "ext_delta", 0.0))
    s.ext_max_steps = int(getattr(p, "ext_max_steps", 0))
    if block_aux is not None:
        s.block_aux = block_aux.data_ptr()
        s.block_aux_n = int(block_aux.shape[1])
    return s


def mlp_params(pe=0):
    """Weights of the deferred MLP over 10 + 6 pe inputs (499 for pe = 0)."""
    return 499 + 96 * int(pe)


def _dims(d, res):
    """(z, y, x) texel or cell counts of a block descriptor: res per unit
    length times the extent on each axis."""
    ext = [int(round(d.aabb_max[a] - d.aabb_min[a])) for a in range(3)]
    return res * ext[2], res * ext[1], res * ext[0]


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Renderer:
    """One library context on one GPU.  Device memory (textures, workspaces,
    outputs) is held as torch tensors; the library only sees pointers."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.L = lib()
        h = C.c_void_p()
        st = self.L.cow_create(C.byref(h), int(device))
        if st != COW_OK:
            raise CowError(st, "cow_create failed")
        self.h = h
        self.blocks = []  # (block_id, lod) in load order
        self.textures = []
        self.load_ws = None
        self.render_ws = None
        self.bwd_ws = None
        self.brick_ws = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.L.cow_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _check(self, st):
        if st != COW_OK:
            raise CowError(st, self.L.cow_last_error(self.h).decode())

    # -- loading ----------------------------------------------------------------
    def load_blocks(self, blocks):
        """blocks: sequence of scenegen.BlockLod (numpy textures are copied to
        the GPU) or of dicts with torch textures already on the device."""
        torch = self.torch
        descs = (BlockDesc * len(blocks))()
        keep = []
        self.blocks = []
        for k, b in enumerate(blocks):
            d = descs[k]
            get = (lambda n: b[n]) if isinstance(b, dict) else (lambda n: getattr(b, n))
            d.block_id, d.lod = int(get("block_id")), int(get("lod"))
            d.aabb_min[:] = [float(x) for x in get("aabb_min")]
            d.aabb_max[:] = [float(x) for x in get("aabb_max")]
            d.grid_res, d.plane_res, d.occ_res = int(get("grid_res")), int(get("plane_res")), int(get("occ_res"))
            d.dtype = int(get("dtype"))
            contracted = b.get("contracted", False) if isinstance(b, dict) else getattr(b, "contracted", False)
            d.flags = BLOCK_CONTRACTED if contracted else 0
            g = get("grid")
            ps = list(get("planes"))
            if not torch.is_tensor(g):
                g = torch.from_numpy(np.ascontiguousarray(g)).to(self.device)
                ps = [torch.from_numpy(np.ascontiguousarray(p)).to(self.device) for p in ps]
            want = torch.uint8 if d.dtype == COW_U8 else torch.float32
            for t in [g] + ps:
                if t.dtype != want or not t.is_contiguous() or t.device != self.device:
                    raise ValueError("textures must be contiguous device tensors of the block's dtype")
            gz, gy, gx = _dims(d, d.grid_res)
            pz, py, px = _dims(d, d.plane_res)
            sizes = [gz * gy * gx, py * px, pz * px, pz * py]
            if [t.numel() for t in [g] + ps] != [8 * n for n in sizes]:
                raise ValueError(f"block {d.block_id} lod {d.lod}: texture sizes do not match the "
                                 f"resolutions times the block extents")
            d.grid = g.data_ptr()
            for i in range(3):
                d.plane[i] = ps[i].data_ptr()
            sc, of = np.asarray(get("scale"), np.float32), np.asarray(get("offset"), np.float32)
            for t in range(4):
                d.scale[t][:] = [float(x) for x in sc[t]]
                d.offset[t][:] = [float(x) for x in of[t]]
            keep.append((g, ps))
            self.blocks.append((d.block_id, d.lod))
        lb, rb, bb = C.c_size_t(), C.c_size_t(), C.c_size_t()
        self._check(self.L.cow_query_workspace(self.h, descs, len(blocks), 1, 0, C.byref(lb), C.byref(rb), C.byref(bb)))
        self.load_ws = torch.empty(max(lb.value, 1), dtype=torch.uint8, device=self.device)
        self._check(self.L.cow_load_blocks(self.h, descs, len(blocks), self.load_ws.data_ptr(), lb.value, _stream()))
        self.textures = keep
        self.descs = descs
        self.brick_ws = None
        return self

    def occupancy(self, block_id, lod):
        k = self.blocks.index((block_id, lod))
        shape = _dims(self.descs[k], self.descs[k].occ_res)
        out = np.zeros(int(np.prod(shape)), np.uint8)
        self._check(self.L.cow_get_occupancy(self.h, block_id, lod, out.ctypes.data, out.size))
        return out.reshape(shape)

    def occupancy_level(self, block_id, lod, level):
        """Level `level` of the max-pooled occupancy pyramid, shape
        (max(Oz >> l, 1), max(Oy >> l, 1), max(Ox >> l, 1))."""
        k = self.blocks.index((block_id, lod))
        shape = tuple(max(n >> max(level, 0), 1) for n in _dims(self.descs[k], self.descs[k].occ_res))
        out = np.zeros(int(np.prod(shape)), np.uint8)
        self._check(self.L.cow_get_occupancy_level(self.h, block_id, lod, level, out.ctypes.data, out.size))
        return out.reshape(shape)

    def pack_bricks(self):
        n = C.c_size_t()
        self._check(self.L.cow_query_bricks(self.h, C.byref(n)))
        self.brick_ws = self.torch.empty(max(n.value, 1), dtype=self.torch.uint8, device=self.device)
        self._check(self.L.cow_pack_bricks(self.h, self.brick_ws.data_ptr(), n.value, _stream()))
        return n.value

    def select(self, view, thresholds=(2.0, 4.0, 8.0), cull=True, cap=4096, quadtree=False):
        pol = LodPolicy()
        for i, t in enumerate(thresholds):
            pol.thresholds[i] = float(t)
        pol.n_thresholds = len(thresholds)
        pol.cull = int(bool(cull))
        pol.quadtree = int(bool(quadtree))
        out = (BlockRef * cap)()
        n = C.c_int()
        v = make_view(view)
        self._check(self.L.cow_select_blocks(self.h, C.byref(v), C.byref(pol), out, cap, C.byref(n)))
        return [(out[i].block_id, out[i].lod) for i in range(n.value)]

    # -- rendering --------------------------------------------------------------
    def _sets(self, sets):
        arrs = []
        cs = (BlockSet * len(sets))()
        for i, s in enumerate(sets):
            a = (BlockRef * max(len(s), 1))()
            for k, (bid, lod) in enumerate(s):
                a[k].block_id, a[k].lod = int(bid), int(lod)
            cs[i].refs = C.cast(a, C.POINTER(BlockRef))
            cs[i].n = len(s)
            arrs.append(a)
        return cs, arrs

    def _ws(self, attr, n_views, n_pix, backward=False):
        lb, rb, bb = C.c_size_t(), C.c_size_t(), C.c_size_t()
        self._check(self.L.cow_query_workspace(self.h, self.descs, len(self.descs), n_views, n_pix,
                                               C.byref(lb), C.byref(rb), C.byref(bb)))
        need = bb.value if backward else rb.value
        cur = getattr(self, attr)
        if cur is None or cur.numel() < need:
            cur = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
            setattr(self, attr, cur)
        return cur

    def _check_block_mlp(self, block_mlp, pe=0):
        torch = self.torch
        if block_mlp is None:
            return None
        n = mlp_params(pe)
        if (block_mlp.dtype != torch.float32 or block_mlp.device != self.device
                or block_mlp.numel() != n * len(self.blocks)):
            raise ValueError(f"block_mlp must be [loaded entries][{n}] float32 on the device")
        return block_mlp.contiguous()

    def _check_block_aux(self, block_aux, n_pix):
        torch = self.torch
        if block_aux is None:
            return None
        if (block_aux.dtype != torch.float32 or block_aux.device != self.device or block_aux.dim() != 3
                or block_aux.shape[0] != n_pix or block_aux.shape[2] != 8 or not block_aux.is_contiguous()):
            raise ValueError("block_aux must be a contiguous float32 device tensor [pixels][slots][8]")
        return block_aux

    def render(self, views, sets, params, mlp, want_aux=True, counts=False, flags=0, out=None, opacity=False,
               block_mlp=None, block_aux=None):
        """block_mlp: [loaded entries][P] per-block deferred MLPs (shading
        before the merge); mlp is then unused and may be None.  P =
        mlp_params(params.pe_freqs): 499, or 883 with four encoding
        frequencies of the direction.  block_aux: [pixels][slots][8] float32,
        filled with each block's composite (A^k, T^k) for render_backward
        (slots: at least the largest set size), or None."""
        torch = self.torch
        vs = (View * len(views))(*[make_view(v) for v in views])
        cs, keep = self._sets(sets)
        n_pix = sum(int(v.crop[2]) * int(v.crop[3]) for v in views)
        if out is None:
            out = dict(rgb=torch.empty((n_pix, 3), dtype=torch.float32, device=self.device),
                       trans=torch.empty(n_pix, dtype=torch.float32, device=self.device),
                       aux=torch.empty((n_pix, 8), dtype=torch.float32, device=self.device) if want_aux else None,
                       counts=torch.zeros((n_pix, 2), dtype=torch.int64, device=self.device) if counts else None,
                       opacity=torch.zeros(n_pix, dtype=torch.float32, device=self.device) if opacity else None)
        ws = self._ws("render_ws", len(views), n_pix)
        pe = int(getattr(params, "pe_freqs", 0))
        bm = self._check_block_mlp(block_mlp, pe)
        p = make_params(params, flags, out.get("counts"), out.get("opacity"), block_mlp=bm,
                        block_aux=self._check_block_aux(block_aux, n_pix))
        if bm is None and (mlp is None or mlp.dtype != torch.float32 or mlp.device != self.device
                           or mlp.numel() != mlp_params(pe)):
            raise ValueError(f"mlp must be {mlp_params(pe)} float32 values on the device")
        aux = out.get("aux")
        self._check(self.L.cow_render(self.h, vs, len(views), cs, C.byref(p), None if mlp is None else mlp.data_ptr(),
                                      out["rgb"].data_ptr(), out["trans"].data_ptr(),
                                      None if aux is None else aux.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
        return out

    def render_noalloc(self, views, sets, params, mlp, out, flags=0, block_aux=None):
        """cow_render_noalloc into caller-given outputs `out` (rgb, trans, aux
        and optionally counts, as returned by render): no workspace."""
        vs = (View * len(views))(*[make_view(v) for v in views])
        cs, keep = self._sets(sets)
        n_pix = sum(int(v.crop[2]) * int(v.crop[3]) for v in views)
        p = make_params(params, flags, out.get("counts"), out.get("opacity"),
                        block_aux=self._check_block_aux(block_aux, n_pix))
        aux = out.get("aux")
        self._check(self.L.cow_render_noalloc(self.h, vs, len(views), cs, C.byref(p), mlp.data_ptr(),
                                              out["rgb"].data_ptr(), out["trans"].data_ptr(),
                                              None if aux is None else aux.data_ptr(), _stream()))
        return out

    def _grad_tables(self, grad_grid, grad_plane):
        ne = len(self.blocks)
        gg = (C.c_void_p * ne)()
        gp = (C.c_void_p * (3 * ne))()
        for e in range(ne):
            if grad_grid is not None and grad_grid[e] is not None:
                gg[e] = grad_grid[e].data_ptr()
            if grad_plane is not None and grad_plane[e] is not None:
                for k in range(3):
                    if grad_plane[e][k] is not None:
                        gp[3 * e + k] = grad_plane[e][k].data_ptr()
        return gg, gp

    def render_backward(self, views, sets, params, mlp, aux, grad_rgb, grad_trans=None, grad_grid=None,
                        grad_plane=None, grad_mlp=None, opacity_weight=None, block_mlp=None, grad_block_mlp=None,
                        flags=0, ws=None, block_aux=None):
        """grad_grid[e] / grad_plane[e][k]: torch fp32 tensors (or None) per
        loaded entry e, accumulated in place; grad_mlp likewise.
        opacity_weight: per-pixel dL/d(opacity regulariser) or None.
        ws: a caller's uint8 device workspace (cow_query_workspace's backward
        size), or None for one the renderer keeps.  block_aux: the buffer the
        forward filled for the same views and sets, or None (the adjoint then
        re-composites each block where it needs A^k or T^k)."""
        vs = (View * len(views))(*[make_view(v) for v in views])
        cs, keep = self._sets(sets)
        n_pix = sum(int(v.crop[2]) * int(v.crop[3]) for v in views)
        if ws is None:
            ws = self._ws("bwd_ws", len(views), n_pix, backward=True)
        gg, gp = self._grad_tables(grad_grid, grad_plane)
        ow = None if opacity_weight is None else opacity_weight.contiguous()
        pe = int(getattr(params, "pe_freqs", 0))
        n = mlp_params(pe)
        bm = self._check_block_mlp(block_mlp, pe)
        if grad_block_mlp is not None and grad_block_mlp.numel() != n * len(self.blocks):
            raise ValueError(f"grad_block_mlp must be [loaded entries][{n}]")
        if bm is None and mlp is not None and mlp.numel() != n:
            raise ValueError(f"mlp must hold {n} weights")
        if grad_mlp is not None and grad_mlp.numel() != n:
            raise ValueError(f"grad_mlp must hold {n} values")
        p = make_params(params, flags=flags, opacity_weight=ow, block_mlp=bm, grad_block_mlp=grad_block_mlp,
                        block_aux=self._check_block_aux(block_aux, n_pix))
        self._check(self.L.cow_render_backward(
            self.h, vs, len(views), cs, C.byref(p), None if mlp is None else mlp.data_ptr(), aux.data_ptr(),
            grad_rgb.contiguous().data_ptr(),
            None if grad_trans is None else grad_trans.contiguous().data_ptr(), gg, gp,
            None if grad_mlp is None else grad_mlp.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))

    def sparsity(self, refs, pts, delta, weight=1.0, loss=None, alpha=False, grad_grid=None, grad_plane=None):
        """Sparsity regulariser at points pts [n][3] (device fp32) over the
        (block, lod) entries `refs` (first match wins).  Adds the loss to
        `loss` (a device fp32 scalar tensor, created if None) and returns
        (loss, alpha or None); gradients accumulate into grad_grid/plane."""
        torch = self.torch
        pts = pts.contiguous()
        if pts.dtype != torch.float32 or pts.device != self.device or pts.dim() != 2 or pts.shape[1] != 3:
            raise ValueError("pts must be [n][3] float32 on the device")
        n = pts.shape[0]
        if loss is None:
            loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        a = torch.empty(n, dtype=torch.float32, device=self.device) if alpha else None
        cs, keep = self._sets([refs])
        ws = self._ws("bwd_ws", 1, 1, backward=True)
        if ws.numel() < 256 + 4 * len(refs) + 32 * len(self.blocks):
            ws = self.torch.empty(256 + 4 * len(refs) + 32 * len(self.blocks), dtype=torch.uint8, device=self.device)
        gg = gp = None
        if grad_grid is not None or grad_plane is not None:
            gg, gp = self._grad_tables(grad_grid, grad_plane)
        self._check(self.L.cow_sparsity(self.h, cs, pts.data_ptr(), n, float(delta), float(weight),
                                        None if a is None else a.data_ptr(), loss.data_ptr(), gg, gp,
                                        ws.data_ptr(), ws.numel(), _stream()))
        return loss, a

    def autotune(self, views, sets, params, mlp, cache_path=None):
        vs = (View * len(views))(*[make_view(v) for v in views])
        cs, keep = self._sets(sets)
        n_pix = sum(int(v.crop[2]) * int(v.crop[3]) for v in views)
        need = self._ws("render_ws", len(views), n_pix).numel() + 16 * n_pix + 512
        ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        p = make_params(params)
        self._check(self.L.cow_autotune(self.h, vs, len(views), cs, C.byref(p), mlp.data_ptr(), ws.data_ptr(),
                                        ws.numel(), None if cache_path is None else cache_path.encode(), _stream()))
        return self.get_config()

    def get_config(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        self._check(self.L.cow_get_config(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def set_config(self, tile_w, waves, persistent):
        self._check(self.L.cow_set_config(self.h, int(tile_w), int(waves), int(persistent)))

    def set_timing(self, on=True):
        self._check(self.L.cow_set_timing(self.h, int(on)))

    def last_timing(self):
        f, b = C.c_float(), C.c_float()
        self._check(self.L.cow_last_timing(self.h, C.byref(f), C.byref(b)))
        return f.value, b.value


def _zero_grads(torch, r):
    gg, gp = [], []
    for e in range(len(r.blocks)):
        g, ps = r.textures[e]
        gg.append(torch.zeros_like(g))
        gp.append([torch.zeros_like(p) for p in ps])
    return gg, gp


def _tex_grads(gg, gp, n_tex):
    out = []
    for e in range(len(gg)):
        out += [gg[e]] + gp[e]
    return tuple(out[:n_tex])


def make_render_fn(with_opacity=False, per_block_mlp=False):
    """torch.autograd.Function over cow_render / cow_render_backward.
    Differentiable inputs: the MLP weights and every fp32 texture of the
    loaded blocks (grid, xy, xz, yz per entry, in load order).  Outputs rgb
    and trans, plus the per-ray opacity regulariser with with_opacity.  With
    per_block_mlp the MLP input is [loaded entries][P], one deferred MLP
    per block applied before the merge (P = mlp_params(params.pe_freqs)).
    With either option the forward keeps each block's composite (32 bytes
    per pixel and set entry) for the backward, which then does not march
    the blocks a second time."""
    import torch

    class RenderFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, renderer, views, sets, params, mlp, *textures):
            ba = None
            if with_opacity or per_block_mlp:
                n_pix = sum(int(v.crop[2]) * int(v.crop[3]) for v in views)
                ba = torch.empty((n_pix, max(1, max(len(x) for x in sets)), 8), dtype=torch.float32,
                                 device=renderer.device)
            if per_block_mlp:
                out = renderer.render(views, sets, params, None, want_aux=True, opacity=with_opacity, block_mlp=mlp,
                                      block_aux=ba)
            else:
                out = renderer.render(views, sets, params, mlp, want_aux=True, opacity=with_opacity, block_aux=ba)
            ctx.renderer, ctx.views, ctx.sets, ctx.params = renderer, views, sets, params
            ctx.block_aux = ba
            ctx.save_for_backward(mlp, out["aux"])
            ctx.n_tex = len(textures)
            if with_opacity:
                return out["rgb"], out["trans"], out["opacity"]
            return out["rgb"], out["trans"]

        @staticmethod
        def backward(ctx, g_rgb, g_trans, g_opacity=None):
            mlp, aux = ctx.saved_tensors
            r = ctx.renderer
            gg, gp = _zero_grads(torch, r)
            gm = torch.zeros_like(mlp)
            g_rgb = g_rgb if g_rgb is not None else torch.zeros((aux.shape[0], 3), device=aux.device)
            if per_block_mlp:
                r.render_backward(ctx.views, ctx.sets, ctx.params, None, aux, g_rgb, g_trans, gg, gp, None,
                                  opacity_weight=g_opacity, block_mlp=mlp, grad_block_mlp=gm, block_aux=ctx.block_aux)
            else:
                r.render_backward(ctx.views, ctx.sets, ctx.params, mlp, aux, g_rgb, g_trans, gg, gp, gm,
                                  opacity_weight=g_opacity, block_aux=ctx.block_aux)
            return (None, None, None, None, gm) + _tex_grads(gg, gp, ctx.n_tex)

    return RenderFn


def make_sparsity_fn():
    """torch.autograd.Function over cow_sparsity: the scalar sparsity loss of
    points pts over entries refs; differentiable in the fp32 textures."""
    import torch

    class SparsityFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, renderer, refs, pts, delta, weight, *textures):
            loss, _ = renderer.sparsity(refs, pts, delta, weight)
            ctx.renderer, ctx.refs, ctx.delta, ctx.weight = renderer, refs, delta, weight
            ctx.save_for_backward(pts)
            ctx.n_tex = len(textures)
            return loss[0]

        @staticmethod
        def backward(ctx, g_loss):
            (pts,) = ctx.saved_tensors
            r = ctx.renderer
            gg, gp = _zero_grads(torch, r)
            # the loss is linear in its weight: d(g L)/dtheta = gradient of weight g
            scratch = torch.zeros(1, dtype=torch.float32, device=pts.device)
            r.sparsity(ctx.refs, pts, ctx.delta, float(ctx.weight) * float(g_loss), loss=scratch,
                       grad_grid=gg, grad_plane=gp)
            return (None, None, None, None, None) + _tex_grads(gg, gp, ctx.n_tex)

    return SparsityFn


def gather_probe(view, tex, blocks_x, blocks_y, grid_res, plane_res, dtype, steps, delta):
    """cow_gather_probe: the march's texel-pair loads without its arithmetic.
    tex is a device uint8 tensor holding the block field; returns
    (kernel ms, gathered bytes)."""
    import torch
    v = make_view(view)
    tiles = (v.crop_w // 8) * (v.crop_h // 8)
    sink = torch.empty(tiles * 64, dtype=torch.int32, device=tex.device)
    ms = C.c_float(0.0)
    st = lib().cow_gather_probe(C.byref(v), C.c_void_p(tex.data_ptr()), tex.numel() * tex.element_size(),
                                int(blocks_x), int(blocks_y), int(grid_res), int(plane_res), int(dtype), int(steps),
                                float(delta), C.c_void_p(sink.data_ptr()), C.byref(ms), _stream())
    if st != COW_OK:
        raise CowError(st, "cow_gather_probe: invalid arguments or HIP error")
    per_sample = 160 if dtype == COW_U8 else 640
    return float(ms.value), tiles * 64 * int(steps) * per_sample
