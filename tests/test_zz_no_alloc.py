"""dwt2_fwd_noalloc (the forward with the library's own scratch array, for
callers that cannot allocate) against dwt2_fwd with a caller's workspace,
through the C ABI: bit-identical on two calls in a row (the second on a
smaller input), in both modes, and across replays of a captured graph."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1708_07853_amd import _lib, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _fwd(lib, x, out, levels, mode):
    h, w = x.shape
    nbytes = lib.dwt2_workspace_size(w, h, 1, levels, mode)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    st = lib.dwt2_fwd(x.data_ptr(), x.stride(0), 0, out.data_ptr(), out.stride(0), 0, w, h, 1, levels, mode, 0,
                      ws.data_ptr(), nbytes, _stream())
    assert st == 0, lib.dwt2_last_error()
    return out


def _noalloc(lib, x, out, levels, mode):
    h, w = x.shape
    st = lib.dwt2_fwd_noalloc(x.data_ptr(), x.stride(0), 0, out.data_ptr(), out.stride(0), 0, w, h, 1, levels,
                              mode, 0, _stream())
    assert st == 0, lib.dwt2_last_error()
    return out


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_equals_fwd_two_calls_second_smaller(mode):
    lib = _lib.load()
    dt = np.float32 if mode == 0 else np.int32
    for (w, h, levels) in [(1531, 1103, 5), (301, 177, 3)]:   # the second call is smaller
        x = torch.from_numpy(synth.image(w, h, w + h, dt)).cuda()
        ref = _fwd(lib, x, torch.empty_like(x), levels, mode)
        got = _noalloc(lib, x, torch.full_like(x, 7), levels, mode)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (w, h, levels)


def test_noalloc_full_benchmark_image():
    """The 8192^2, 6-level image the scratch array is sized for."""
    lib = _lib.load()
    x = synth.image_device(8192, 8192, 2)
    ref = _fwd(lib, x, torch.empty_like(x), 6, 0)
    got = _noalloc(lib, x, torch.empty_like(x), 6, 0)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    lib = _lib.load()
    x = torch.zeros((8, 8), device="cuda")
    st = lib.dwt2_fwd_noalloc(x.data_ptr(), 16384, 0, x.data_ptr() + 4, 16384, 0, 16384, 16384, 1, 6, 0, 0,
                              _stream())
    assert st == -4 and b"scratch" in lib.dwt2_last_error()


def test_noalloc_replays_from_a_captured_graph():
    lib = _lib.load()
    h, w, L = 700, 1300, 5
    x = torch.from_numpy(synth.image(w, h, 12)).cuda()
    ref = _fwd(lib, x, torch.empty_like(x), L, 0)
    out = torch.empty_like(x)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):       # first call on the capture stream: looks up the array
        _noalloc(lib, x, out, L, 0)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        _noalloc(lib, x, out, L, 0)
    for rep in range(3):
        out.fill_(0)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        _noalloc(lib, x[:300, :400].contiguous(), torch.empty((300, 400), device="cuda"), 3, 0)  # eager use between
        torch.cuda.synchronize()
