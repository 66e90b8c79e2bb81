"""GPU parity of the recursive kernel (ABF_KERNEL_RECURSIVE: Deriche's
recursive approximation of the Gaussian truncated to the window, O(1) per
pixel in rho) against the CPU oracle's value of record for the same kernel
(oracle.fast_abf with kernel "recursive": direct window sums with the
kernel's weights). Every pixel on small images (one and several row and
column segments of the passes, single rows and columns, rho from 0 to
beyond the image), sampled pixels on a large one, to the mixed path's bar
of 0.05 on [0, 255] (the kernel has no FP64 path, see abf.h)."""
import numpy as np
import pytest

import oracle
from synth import gauss_field, rect_scene, smooth_field, voronoi

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-6, "mixed": 0.05}


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


def dev(torch, a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


CASES = [((64, 80), 5, 5), ((37, 530), 12, 6), ((530, 41), 7, 8), ((1, 200), 3, 4),
         ((150, 1), 3, 4), ((20, 30), 40, 6), ((90, 120), 0, 5), ((600, 700), 30, 6),
         ((128, 1100), 60, 3), ((70, 90), 1, 1)]     # segments of 512: one, several, partial


@pytest.mark.parametrize("precision", ["mixed"])
@pytest.mark.parametrize("shape,R,N", CASES)
def test_recursive_every_pixel(torch, abf, precision, shape, R, N):
    h, w = shape
    f = rect_scene(500 + R + N, h, w, n_rect=6, noise=6.0, side_lo=2, side_hi=max(3, min(h, w)))
    sg = smooth_field(np.random.default_rng(R + 1), h, w, 8, 40)
    th = None
    if N % 2 == 0:       # theta away from f on half the cases (t0 outside [0, 1] on some pixels)
        th = (f + smooth_field(np.random.default_rng(N), h, w, -15, 15)).astype(np.float32)
    out = abf.fast(dev(torch, f), dev(torch, sg), theta=dev(torch, th), kernel="recursive", rho=R,
                   N=N, precision=precision).cpu().numpy().astype(np.float64)
    if h * w * (2 * R + 1) ** 2 <= 4e7:
        ref = oracle.fast_abf(f, th, sg, "recursive", R, N)
        err = float(np.max(np.abs(out - ref)))
    else:            # wide windows: every border row and column, and random pixels
        rng = np.random.default_rng(R)
        ys = np.concatenate([np.arange(h), np.arange(h), np.zeros(w, int), np.full(w, h - 1),
                             rng.integers(0, h, 1500)])
        xs = np.concatenate([np.zeros(h, int), np.full(h, w - 1), np.arange(w), np.arange(w),
                             rng.integers(0, w, 1500)])
        ref = oracle.fast_abf(f, th, sg, "recursive", R, N, pixels=(ys, xs))
        err = float(np.max(np.abs(out[ys, xs] - ref)))
    assert err < TOL[precision], err


@pytest.mark.parametrize("precision", ["mixed"])
def test_recursive_large_sampled(torch, abf, precision):
    """2048 x 1536 Voronoi cells with noise at rho = 48: several segments of
    both passes, ill-conditioned windows far from the image's one origin
    recomputed from their windows; sampled pixels plus the borders."""
    h, w, R, N = 2048, 1536, 48, 6
    f = voronoi(77, h, w, n_seed=40, noise=4.0)
    sg = smooth_field(np.random.default_rng(5), h, w, 5, 30)
    out = abf.fast(dev(torch, f), dev(torch, sg), kernel="recursive", rho=R, N=N,
                   precision=precision).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(11)
    ys = np.concatenate([rng.integers(0, h, 300), [0, 0, h - 1, h - 1, h // 2, 511, 512, 1023]])
    xs = np.concatenate([rng.integers(0, w, 300), [0, w - 1, 0, w - 1, 511, 512, 513, w - 2]])
    ref = oracle.fast_abf(f, None, sg, "recursive", R, N, pixels=(ys, xs))
    assert np.max(np.abs(out[ys, xs] - ref)) < TOL[precision]


def test_recursive_scope(torch, abf):
    """The FP64 path and the entry points that do not take the kernel
    return their status codes before any device work."""
    f = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    s = torch.full((16, 16), 10.0, dtype=torch.float32, device="cuda")
    for N in (1, 6):
        with pytest.raises(abf.ABFError):
            abf.fast(f, s, kernel="recursive", rho=3, N=N, precision="fp64")
    with pytest.raises(abf.ABFError):
        abf.bruteforce(f, s, kernel="recursive", rho=3)
    field = gauss_field(3, 64, 64)
    out = abf.fast(dev(torch, field), s.new_full((64, 64), 20.0), kernel="recursive", rho=4, N=7,
                   precision="mixed")
    assert out.shape == (64, 64)
