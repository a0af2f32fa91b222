"""The texel-gather microbenchmark (cow_gather_probe), a measurement aid for
the march's gather rate: it runs, rejects bad arguments before launching,
is deterministic, and reads the texture it is given (all-zero texels XOR to
zero; random texels do not)."""
import pytest

from paper_2312_16457_amd import COW_F32, COW_U8, CowError, scenegen as sg
from paper_2312_16457_amd.binding import gather_probe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda(have_gpu):
    import torch
    return torch


def small_view():
    return sg.c2_view().with_crop(800, 400, 64, 32)


@pytest.mark.parametrize("dtype", [COW_U8, COW_F32])
def test_probe_runs_and_reads_texture(torch_cuda, dtype):
    torch = torch_cuda
    nb, R, Rp = 2, 16, 64
    texel = 8 if dtype == COW_U8 else 32
    nbytes = nb * nb * (R ** 3 + 3 * Rp * Rp) * texel
    g = torch.Generator(device="cuda").manual_seed(3)
    tex = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    view = small_view()
    ms, gbytes = gather_probe(view, tex, nb, nb, R, Rp, dtype, 300, 1.0 / 512)
    assert ms > 0 and gbytes == view.n_pixels * 300 * (20 * texel)
    from paper_2312_16457_amd import binding
    import ctypes as C
    sinks = []
    for t in (tex, tex, torch.zeros_like(tex)):
        v = binding.make_view(view)
        sink = torch.full((view.n_pixels,), -1, dtype=torch.int32, device="cuda")
        out_ms = C.c_float(0)
        st = binding.lib().cow_gather_probe(C.byref(v), C.c_void_p(t.data_ptr()), t.numel(), nb, nb, R, Rp, dtype,
                                            300, 1.0 / 512, C.c_void_p(sink.data_ptr()), C.byref(out_ms),
                                            binding._stream())
        assert st == 0
        sinks.append(sink.cpu())
    assert (sinks[0] == sinks[1]).all()
    assert (sinks[2] == 0).all()
    assert (sinks[0] != 0).float().mean().item() > 0.9


def test_probe_rejects_bad_arguments(torch_cuda):
    torch = torch_cuda
    tex = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    view = small_view()
    with pytest.raises(CowError):  # texture too small for 2x2 blocks of 64^3
        gather_probe(view, tex, 2, 2, 64, 64, COW_U8, 10, 1.0 / 512)
    with pytest.raises(CowError):  # not a power of two
        gather_probe(view, tex, 1, 1, 12, 16, COW_U8, 10, 1.0 / 512)
    with pytest.raises(CowError):  # crop not a multiple of 8
        gather_probe(sg.c2_view().with_crop(0, 0, 20, 16), tex, 1, 1, 8, 16, COW_U8, 10, 1.0 / 512)
