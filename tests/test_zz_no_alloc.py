"""abf_fast_noalloc (the entry point for callers that cannot allocate
device memory) through the C ABI: on two calls in a row, the second on a
smaller image, its output equals abf_fast's bit for bit (the same kernels,
workspace in the library's fixed per-GPU array instead of caller memory);
a request larger than ABF_NOALLOC_BYTES is refused before any device work
and leaves the output untouched."""
import numpy as np
import pytest

from synth import rect_scene, smooth_field

pytestmark = pytest.mark.gpu

ABF_E_WORKSPACE = -5
NOALLOC_BYTES = 64 << 20


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def abf():
    import paper_1811_02308_amd as m
    m.lib()
    return m


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _noalloc(torch, abf, fd, sd, td, kernel, R, N, precision, out):
    h, w = fd.shape
    s = torch.cuda.current_stream().cuda_stream
    return abf.lib().abf_fast_noalloc(
        fd.data_ptr(), 0 if td is None else td.data_ptr(), sd.data_ptr(), h, w, fd.stride(0),
        abf.KERNELS[kernel], 0.0, R, N, abf.PRECISIONS[precision], abf.FLAG_CLAMP,
        out.data_ptr(), out.stride(0), s)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("kernel,R,N", [("box", 5, 6), ("gaussian", 9, 5), ("box", 30, 8)])
def test_noalloc_equals_fast_twice(torch, abf, precision, kernel, R, N):
    for seed, (h, w) in ((1, (700, 900)), (2, (130, 210))):       # second call smaller
        f = rect_scene(900 + seed, h, w, n_rect=7, noise=8, side_lo=8, side_hi=200)
        sg = smooth_field(np.random.default_rng(seed), h, w, 8, 40)
        th = (f + smooth_field(np.random.default_rng(seed + 5), h, w, -15, 15)).astype(np.float32)
        fd, sd, td = _dev(torch, f), _dev(torch, sg), _dev(torch, th)
        assert abf.lib().abf_workspace_bytes(h, w, R, N, abf.PRECISIONS[precision]) <= NOALLOC_BYTES
        dt = torch.float32 if precision == "mixed" else torch.float64
        out = torch.full((h, w), -1.0, dtype=dt, device="cuda")
        st = _noalloc(torch, abf, fd, sd, td, kernel, R, N, precision, out)
        assert st == 0, abf.lib().abf_status_string(st)
        ref = abf.fast(fd, sd, theta=td, kernel=kernel, rho=R, N=N, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (seed, h, w)


def test_noalloc_refuses_oversized_request(torch, abf):
    h, w, R, N = 2048, 2048, 5, 8
    assert abf.lib().abf_workspace_bytes(h, w, R, N, abf.PRECISIONS["mixed"]) > NOALLOC_BYTES
    fd = torch.zeros((h, w), dtype=torch.float32, device="cuda")
    sd = torch.full((h, w), 20.0, dtype=torch.float32, device="cuda")
    out = torch.full((h, w), 7.0, dtype=torch.float32, device="cuda")
    assert _noalloc(torch, abf, fd, sd, None, "box", R, N, "mixed", out) == ABF_E_WORKSPACE
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
