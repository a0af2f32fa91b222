"""Descriptor limits at their edges: texel offsets are 32-bit, so a texture
must stay below 2 GiB and a resolution within 1024 (grid) and 8192 (plane)
texels per axis.  cow_query_workspace validates descriptors on the host
before anything touches their memory, so the textures here are placeholder
addresses; each case sits on one side of one limit."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer(have_gpu):
    from paper_2312_16457_amd import Renderer
    return Renderer(0)


def desc(dtype, grid_res, plane_res, occ_res=4, extent=(1, 1, 1)):
    from paper_2312_16457_amd import binding
    d = binding.BlockDesc()
    d.block_id, d.lod = 0, 0
    d.aabb_min[:] = [0.0, 0.0, 0.0]
    d.aabb_max[:] = [float(e) for e in extent]
    d.grid_res, d.plane_res, d.occ_res, d.dtype = grid_res, plane_res, occ_res, dtype
    d.grid = 0x10000
    for k in range(3):
        d.plane[k] = 0x20000 + 0x10000 * k
    for t in range(4):
        d.scale[t][:] = [1.0] * 8
        d.offset[t][:] = [0.0] * 8
    return d


def query(r, d):
    from paper_2312_16457_amd import binding
    lb, rb, bb = C.c_size_t(), C.c_size_t(), C.c_size_t()
    arr = (binding.BlockDesc * 1)(d)
    st = r.L.cow_query_workspace(r.h, arr, 1, 1, 1, C.byref(lb), C.byref(rb), C.byref(bb))
    return st, r.L.cow_last_error(r.h).decode(), bb.value


@pytest.mark.parametrize("dtype,grid_res,plane_res,extent,msg", [
    # fp32 plane of 8192^2 texels: 2 GiB exactly, one byte past what a signed 32-bit offset reaches
    (1, 16, 8192, (1, 1, 1), "larger than 2 GiB"),
    # fp32 grid of 512 x 512 x 256 texels: 2 GiB
    (1, 256, 256, (2, 2, 1), "larger than 2 GiB"),
    # uint8 grid of 1024^3 texels: 8 GiB
    (0, 1024, 256, (1, 1, 1), "larger than 2 GiB"),
    # more than 8192 plane texels or 1024 grid texels along one axis
    (0, 16, 16384, (1, 1, 1), "resolution too large"),
    (0, 1024, 1024, (2, 1, 1), "resolution too large"),
])
def test_limits_refused(renderer, dtype, grid_res, plane_res, extent, msg):
    from paper_2312_16457_amd import binding
    st, err, _ = query(renderer, desc(dtype, grid_res, plane_res, extent=extent))
    assert st == binding.COW_E_INVALID and msg in err, (st, err)


@pytest.mark.parametrize("dtype,grid_res,plane_res,extent", [
    (0, 16, 8192, (1, 1, 1)),    # uint8 plane of 8192^2 texels: 512 MiB
    (1, 16, 4096, (1, 1, 1)),    # fp32 plane 4096^2: 512 MiB
    (1, 256, 256, (2, 1, 1)),    # fp32 grid 512 x 256 x 256: 1 GiB
    (0, 512, 256, (1, 1, 1)),    # uint8 grid 512^3: 1 GiB
])
def test_limits_accepted(renderer, dtype, grid_res, plane_res, extent):
    from paper_2312_16457_amd import binding
    st, err, bwd = query(renderer, desc(dtype, grid_res, plane_res, extent=extent))
    assert st == binding.COW_OK, err
    if dtype == 1:
        # the backward workspace holds a 64-byte pair slot per fp32 texel
        gx, gy, gz = (grid_res * e for e in extent)
        px, py, pz = (plane_res * e for e in extent)
        assert bwd >= 64 * (gx * gy * gz + px * py + px * pz + py * pz)
