"""The allocation-free C2R entry point (arche_k_fft_c2r_noalloc) against the
allocating one (arche_k_fft_c2r) through the C ABI: the same kernels on the
same twiddles, so the outputs are bit-identical; two calls in a row, the
second on a smaller grid (the shared scratch keeps the first call's
contents); the input is left unchanged; sizes beyond the scratch and
unsupported sizes are rejected before anything is enqueued."""
import sys

import numpy as np
import pytest

from paper_2606_13283_amd import arche

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    arche.load()
    return torch


def spectrum(torch, shape, seed):
    Nx, Ny, Nz = shape
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    # the half spectrum of a real field
    X = np.fft.rfftn(x)
    return torch.from_numpy(X).to("cuda"), x


@pytest.mark.parametrize("shapes", [((128, 128, 128), (48, 40, 36), (20, 16, 12))])
def test_noalloc_c2r_matches_allocating_entry_point(torch_gpu, shapes):
    torch = torch_gpu
    for i, shape in enumerate(shapes):
        say("noalloc c2r call", i, shape)
        X, x = spectrum(torch, shape, 100 + i)
        X0 = X.clone()
        ref = arche.fft_c2r(X, shape[2])
        out = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
        arche.fft_c2r_noalloc(X, shape[2], out)
        torch.cuda.synchronize()
        assert torch.equal(X, X0), "input spectrum modified"
        assert torch.equal(out, ref), (shape, float((out - ref).abs().max()))
        ng = int(np.prod(shape))
        assert np.max(np.abs(out.cpu().numpy() / ng - x)) <= 1e-13 * np.max(np.abs(x))


def test_noalloc_rejects_sizes(torch_gpu):
    torch = torch_gpu
    X = torch.zeros((4, 4, 3), dtype=torch.complex128, device="cuda")
    out = torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda")
    L = arche.load()
    import ctypes
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = arche._grid_arr((256, 128, 128))  # half spectrum above ARCHE_NOALLOC_MAX_NH
    assert L.arche_k_fft_c2r_noalloc(big, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     stream) == arche.EINVAL
    odd = arche._grid_arr((4, 4, 26 * 5))  # 130 = 2 * 5 * 13 has no plan
    assert L.arche_k_fft_c2r_noalloc(odd, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     stream) == arche.EINVAL
    assert L.arche_k_fft_c2r_noalloc(arche._grid_arr((4, 4, 4)), None, ctypes.c_void_p(out.data_ptr()),
                                     stream) == arche.EINVAL
    assert arche.NOALLOC_MAX_NH == 128 * 128 * 65
