"""CPU checks of the C ABI: the library loads, exports exactly what
include/cow.h declares, and the ctypes structures match the C layout."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cow.h")


@pytest.fixture(scope="module")
def libcow():
    from paper_2312_16457_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return binding.lib()


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"COW_API\s+[\w\s\*]+?\b(cow_\w+)\s*\(", src)))


def test_header_declarations_exported(libcow):
    from paper_2312_16457_amd import binding
    names = declared()
    assert len(names) >= 16
    assert sorted(binding.EXPORTS) == names
    for n in names:
        assert hasattr(libcow, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == names, "the library exports exactly the declared entry points"


def test_every_export_has_a_ctypes_signature(libcow):
    """Each entry point is called with declared argument types (floats and
    64-bit sizes would otherwise be passed wrongly or rejected), and the
    declared count matches the header's parameter list."""
    from paper_2312_16457_amd import binding
    src = open(HEADER).read()
    for n in binding.EXPORTS:
        f = getattr(libcow, n)
        assert f.argtypes is not None, n
        m = re.search(r"\b" + n + r"\s*\(([^)]*)\)", src)
        params = [p for p in m.group(1).split(",") if p.strip() and p.strip() != "void"]
        assert len(f.argtypes) == len(params), (n, len(f.argtypes), len(params))


def test_struct_layouts_match_c():
    from paper_2312_16457_amd import binding as B
    prog = r"""
    #include <stdio.h>
    #include <stddef.h>
    #include "cow.h"
    int main(void) {
      printf("%zu %zu %zu %zu %zu\n", sizeof(cow_block_desc), offsetof(cow_block_desc, grid),
             offsetof(cow_block_desc, scale), offsetof(cow_block_desc, offset), offsetof(cow_block_desc, flags));
      printf("%zu %zu %zu\n", sizeof(cow_view), offsetof(cow_view, eye), offsetof(cow_view, fx));
      printf("%zu %zu\n", sizeof(cow_block_ref), sizeof(cow_block_set));
      printf("%zu %zu\n", sizeof(cow_lod_policy), offsetof(cow_lod_policy, cull));
      printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(cow_render_params), offsetof(cow_render_params, flags),
             offsetof(cow_render_params, counts), offsetof(cow_render_params, opacity),
             offsetof(cow_render_params, opacity_weight), offsetof(cow_render_params, ext_delta),
             offsetof(cow_render_params, ext_max_steps));
      return 0;
    }
    """
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                               "-I", "/opt/rocm/include", src, "-o", exe])
        vals = [list(map(int, l.split())) for l in subprocess.check_output([exe], text=True).splitlines()]
    assert vals[0] == [C.sizeof(B.BlockDesc), B.BlockDesc.grid.offset, B.BlockDesc.scale.offset,
                       B.BlockDesc.offset.offset, B.BlockDesc.flags.offset]
    assert vals[1] == [C.sizeof(B.View), B.View.eye.offset, B.View.fx.offset]
    assert vals[2] == [C.sizeof(B.BlockRef), C.sizeof(B.BlockSet)]
    assert vals[3] == [C.sizeof(B.LodPolicy), B.LodPolicy.cull.offset]
    assert vals[4] == [C.sizeof(B.Params), B.Params.flags.offset, B.Params.counts.offset, B.Params.opacity.offset,
                       B.Params.opacity_weight.offset, B.Params.ext_delta.offset, B.Params.ext_max_steps.offset]


def test_null_context_and_no_device(libcow):
    from paper_2312_16457_amd import binding as B
    assert libcow.cow_last_error(None) == b"null context"
    assert libcow.cow_destroy(None) == B.COW_E_INVALID
    assert libcow.cow_create(None, 0) == B.COW_E_INVALID
    try:
        import torch
        gpu = torch.cuda.is_available()
    except Exception:
        gpu = False
    if not gpu:
        h = C.c_void_p()
        assert libcow.cow_create(C.byref(h), 0) != B.COW_OK


def test_renderer_without_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2312_16457_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        binding.lib()
