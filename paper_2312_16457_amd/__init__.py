"""MI355X-native block-merged ray-march renderer (City-on-Web, arXiv 2312.16457).

The render path lives in libcow.so (HIP kernels for gfx950 behind the C ABI
in include/cow.h); this package is its Python binding plus the seeded
synthetic-scene generator used by the tests and the benchmark."""
from .binding import (BLOCK_CONTRACTED, COW_F32, COW_U8, F_FLAT_OCC, F_GRAPH, F_NONE, F_PER_BLOCK, F_PERSISTENT, F_SPARSE,
                      MODE_CHORD, MODE_GRID, CowError, Renderer, lib, make_render_fn, make_sparsity_fn, mlp_params)

__all__ = ["Renderer", "CowError", "lib", "make_render_fn", "make_sparsity_fn", "COW_U8", "COW_F32", "MODE_CHORD", "MODE_GRID",
           "F_NONE", "F_GRAPH", "F_PERSISTENT", "F_PER_BLOCK", "F_SPARSE", "F_FLAT_OCC", "BLOCK_CONTRACTED", "mlp_params"]
