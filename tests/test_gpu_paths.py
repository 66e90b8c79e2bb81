"""GPU parity of every moment kernel abf_fast dispatches to, each case pinned
to the kernel it exercises (abf_stack_kernel), against the CPU oracle.

The moment step of Algorithm 1 (window moments by convolution, Prop. 2,
shifted to [alpha_i, beta_i], Prop. 3) has four kernels: box running sums,
the 2-D tile kernel with LDS row stride 160 or 256, and the matrix-core
kernel for wide Gaussian windows on large images. Each test below first
asserts which of them its configuration takes, then compares the filtered
output with ``oracle.fast_abf`` at every pixel (small images) or at sampled
pixels that include the corners, the edges and the last partial row block
and column strip (large images). Bars: FP64 path 1e-6, mixed path 0.05 on
[0, 255].
"""
import numpy as np
import pytest

import oracle
from synth import gauss_field, rect_scene, smooth_field, voronoi, workload

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


def edge_samples(H, W, n, seed):
    """Random pixels plus corners, edge midpoints, and the last rows and
    columns (the partial 16-row block / 16-column strip of the matrix-core
    kernel and the partial tiles of the tile kernel)."""
    rng = np.random.default_rng(seed)
    ys = list(rng.integers(0, H, n))
    xs = list(rng.integers(0, W, n))
    fixed = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, 0), (0, W // 2),
             (H - 1, W // 2), (H // 2, W - 1)]
    for d in range(1, 17):
        fixed += [(H - d, int(rng.integers(0, W))), (int(rng.integers(0, H)), W - d)]
    for y, x in fixed:
        ys.append(y)
        xs.append(x)
    return np.array(ys), np.array(xs)


def compare_sampled(torch, abf, f, th, sg, kernel, R, N, precision, ys, xs, sigma_s):
    out = abf.fast(dev(torch, f), dev(torch, sg), theta=dev(torch, th), kernel=kernel, rho=R, N=N,
                   sigma_s=sigma_s, precision=precision)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)[ys, xs]
    ref = oracle.fast_abf(f, th, sg, kernel, R, N, sigma_s=sigma_s, pixels=(ys, xs))
    return float(np.max(np.abs(got - ref)))


# ----------------------------------------------------------------- matrix cores
# (h, w, R, N): images of at least 2^22 pixels; both orientations of a
# 2048 x 2731 request put a partial 16-column strip or a partial 16-row block
# at the far edge
MFMA_CASES = [(2048, 2048, 8, 1), (2048, 2731, 8, 5), (2731, 2048, 10, 6), (2048, 2731, 10, 2),
              (2048, 2048, 12, 3), (2731, 2048, 12, 4), (2048, 2731, 16, 6), (2731, 2048, 16, 5)]


@pytest.fixture(scope="module")
def mfma_images():
    imgs = {}
    for (h, w) in {(c[0], c[1]) for c in MFMA_CASES}:
        f = rect_scene(4000 + h, h, w, n_rect=40, noise=10, side_lo=h // 16, side_hi=h // 2)
        zeta = smooth_field(np.random.default_rng(h + 1), h, w, -20, 20)
        imgs[(h, w)] = (f, (f + zeta).astype(np.float32),
                        smooth_field(np.random.default_rng(h + 2), h, w, 10, 30))
    return imgs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("h,w,R,N", MFMA_CASES)
def test_mfma_moment_kernel_matches_oracle(torch, abf, mfma_images, precision, h, w, R, N):
    # the matrix cores serve the mixed path; the FP64 path takes the tile kernel at these sizes
    assert abf.stack_kernel(h, w, "gaussian", R, N, precision) == (
        "mfma" if precision == "mixed" else "tile")
    f, th, sg = mfma_images[(h, w)]
    ys, xs = edge_samples(h, w, 300, seed=R * 10 + N)
    # theta = f on even N, theta = f + zeta (t0 outside [0, 1] at some pixels) on odd N
    err = compare_sampled(torch, abf, f, th if N % 2 else None, sg, "gaussian", R, N, precision,
                          ys, xs, R / 3.0)
    assert err < TOL[precision], err


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mfma_stack_planes_match_oracle(torch, abf, mfma_images, precision):
    """The matrix-core kernel's stored Legendre moments against the oracle's
    at sampled pixels (the range stage excluded)."""
    h, w, R, N = 2048, 2731, 12, 6
    assert abf.stack_kernel(h, w, "gaussian", R, N, precision) == (
        "mfma" if precision == "mixed" else "tile")
    f, _, _ = mfma_images[(h, w)]
    st = abf.moment_stack(dev(torch, f), kernel="gaussian", rho=R, N=N, sigma_s=R / 3.0,
                          precision=precision)
    torch.cuda.synchronize()
    a, b, mom = abf.stack_planes(st, h, w, N, precision)
    ys, xs = edge_samples(h, w, 300, seed=5)
    _, aux = oracle.fast_abf(f, None, np.full(f.shape, 20.0), "gaussian", R, N, sigma_s=R / 3.0,
                             pixels=(ys, xs), aux=True)
    assert np.array_equal(a.cpu().numpy()[ys, xs], aux["alpha"].astype(np.float32))
    assert np.array_equal(b.cpu().numpy()[ys, xs], aux["beta"].astype(np.float32))
    live = aux["alpha"] != aux["beta"]
    for k in range(N):
        got = mom[k].cpu().numpy().astype(np.float64)[ys, xs]
        assert np.max(np.abs(got[live] - aux["amom"][:, k + 1][live])) < 2e-6, k


# ----------------------------------------------------------------- tile kernel, wide LDS stride
WIDE_SMALL = [(17, 6), (20, 8), (24, 5), (20, 3)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("R,N", WIDE_SMALL)
def test_gaussian_wide_tile_every_pixel(torch, abf, precision, R, N):
    h, w = 70, 333
    assert abf.stack_kernel(h, w, "gaussian", R, N, precision) == "tile_wide"
    f = rect_scene(800 + R, h, w, n_rect=6, noise=10, side_lo=6, side_hi=60)
    sg = smooth_field(np.random.default_rng(R + N), h, w, 5, 50)
    th = (f + smooth_field(np.random.default_rng(R), h, w, -20, 20)).astype(np.float32)
    out = abf.fast(dev(torch, f), dev(torch, sg), theta=dev(torch, th), kernel="gaussian", rho=R,
                   N=N, precision=precision)
    torch.cuda.synchronize()
    ref = oracle.fast_abf(f, th, sg, "gaussian", R, N)
    err = np.abs(out.cpu().numpy().astype(np.float64) - ref)
    assert err.max() < TOL[precision], float(err.max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("h,w,R,N", [(2048, 2048, 20, 6), (1100, 1500, 40, 7), (2048, 2731, 24, 8)])
def test_gaussian_wide_tile_large_sampled(torch, abf, precision, h, w, R, N):
    """Gaussian windows above radius 16 (the 256-wide LDS row stride) on images
    of up to 5.6 Mpix, including a config-4-shaped 2048 x 2731 request."""
    assert abf.stack_kernel(h, w, "gaussian", R, N, precision) == "tile_wide"
    f = gauss_field(900 + R, h, w)
    sg = smooth_field(np.random.default_rng(R), h, w, 5, 60)
    th = (f + smooth_field(np.random.default_rng(R + 3), h, w, -20, 20)).astype(np.float32)
    ys, xs = edge_samples(h, w, 250, seed=R)
    err = compare_sampled(torch, abf, f, th, sg, "gaussian", R, N, precision, ys, xs, R / 3.0)
    assert err < TOL[precision], err


# ----------------------------------------------------------------- box kernel paths
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("N", [5, 6, 7, 8])
def test_box_paths_by_precision_and_degree(torch, abf, precision, N):
    """The box kernel takes running sums except on the FP64 path at N >= 7,
    where the tile kernel with unit weights replaces it; both against the
    oracle on a high-contrast image with a partial last strip."""
    h, w, R = 200, 517, 5
    want = "tile" if (precision == "fp64" and N >= 7) else "box"
    assert abf.stack_kernel(h, w, "box", R, N, precision) == want
    f = voronoi(1300 + N, h, w, n_seed=30, noise=15.0)
    sg = smooth_field(np.random.default_rng(N), h, w, 10, 40)
    out = abf.fast(dev(torch, f), dev(torch, sg), kernel="box", rho=R, N=N, precision=precision)
    torch.cuda.synchronize()
    ref = oracle.fast_abf(f, None, sg, "box", R, N)
    err = np.abs(out.cpu().numpy().astype(np.float64) - ref)
    assert err.max() < TOL[precision], float(err.max())


# ----------------------------------------------------------------- full-size configs
@pytest.fixture(scope="module")
def texture():
    return workload("texture1080_box8_n6")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_texture_full_size_first_pass_sampled(torch, abf, texture, precision):
    """Texture workload at its full size (96 planes of 1920 x 1080): one pass
    of sigma map + strided fast filter over all planes, sampled pixels of
    four planes against the oracle fed the GPU's sigma map; the sigma map
    itself against the oracle's rule at the same pixels."""
    from oracle.spatial import local_std_sigma
    fr = texture["frames"]
    n, h, w = fr.shape
    assert abf.stack_kernel(h, w, "box", texture["R"], texture["N"], precision) == "box"
    x = torch.from_numpy(fr).cuda()
    sig = abf.sigma_local_std(x, **texture["sigma_rule"])
    y = abf.fast_strided(x, sig, kernel="box", rho=texture["R"], N=texture["N"], precision=precision)
    torch.cuda.synchronize()
    for c in (0, 37, 64, n - 1):
        ys, xs = edge_samples(h, w, 120, seed=c)
        sc = sig[c].cpu().numpy()
        # the sigma map on the top-left 40 x 40 corner (clamped borders
        # included: the oracle's window clamps at the image's own edges there)
        sr = texture["sigma_rule"]
        ref_sig = local_std_sigma(fr[c][:44, :44], sr["radius"], sr["scale"], sr["lo"], sr["hi"])
        assert np.max(np.abs(sc[:40, :40] - ref_sig[:40, :40])) <= 1e-5 * 80
        ref = oracle.fast_abf(fr[c], None, sc, "box", texture["R"], texture["N"], pixels=(ys, xs))
        got = y[c].cpu().numpy().astype(np.float64)[ys, xs]
        assert np.max(np.abs(got - ref)) < TOL[precision], c


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_texture_full_size_third_pass_sampled(torch, abf, texture, precision):
    """The texture workload's third pass at full size. Its input (two passes
    of smoothing) is nearly flat in places, so many windows are narrow and
    far from their wave's origin: their shifts are ill-conditioned and are
    accepted by the FP32 stack's width-aware rule or recomputed from their
    windows. Sampled pixels of three planes, plus each plane's 64 windows of
    smallest non-zero range, against the oracle fed the GPU's pass-3 input
    and sigma map."""
    from scipy.ndimage import maximum_filter, minimum_filter
    fr = texture["frames"]
    n, h, w = fr.shape
    R, N, sr = texture["R"], texture["N"], texture["sigma_rule"]
    x = torch.from_numpy(fr).cuda()
    x3 = abf.texture_filter(x, 2, R, N, precision=precision, **sr).float()
    sig = abf.sigma_local_std(x3, **sr)
    y = abf.fast_strided(x3, sig, kernel="box", rho=R, N=N, precision=precision)
    torch.cuda.synchronize()
    for c in (0, 41, n - 1):
        f3, sc = x3[c].cpu().numpy(), sig[c].cpu().numpy()
        d = (maximum_filter(f3, 2 * R + 1, mode="nearest").astype(np.float64)
             - minimum_filter(f3, 2 * R + 1, mode="nearest"))
        flat = np.argsort(np.where(d > 0, d, np.inf), axis=None)[:64]
        ys, xs = edge_samples(h, w, 150, seed=100 + c)
        ys = np.concatenate([ys, flat // w])
        xs = np.concatenate([xs, flat % w])
        ref = oracle.fast_abf(f3, None, sc, "box", R, N, pixels=(ys, xs))
        got = y[c].cpu().numpy().astype(np.float64)[ys, xs]
        assert np.max(np.abs(got - ref)) < TOL[precision], c


# ----------------------------------------------------------------- large images
@pytest.fixture(scope="module")
def large_image():
    base = voronoi(1003, 4096, 4096)
    f = np.ascontiguousarray(np.tile(base, (4, 4))[:12292, :12290])
    sg = np.ascontiguousarray(np.tile(smooth_field(np.random.default_rng(9), 1024, 1024, 10, 40),
                                      (13, 13))[:12292, :12290])
    return f, sg


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_image_sampled(torch, abf, large_image, precision):
    """A 12292 x 12290 image (151 Mpix; 0.6 GB per float plane, an 11 GB FP64
    stack at N = 8): the 4096^2 Voronoi scene tiled 3 x 3 plus a ragged
    border, box R = 5, N = 8 (mixed: the fused path; FP64: the tile
    kernel), sampled pixels against the oracle, corners and the last rows
    and columns included. Every index of the kernels beyond 2^31 bytes of a
    plane's start runs here."""
    f, sg = large_image
    h, w = f.shape
    R, N = 5, 8
    out = abf.fast(dev(torch, f), dev(torch, sg), kernel="box", rho=R, N=N, precision=precision)
    torch.cuda.synchronize()
    ys, xs = edge_samples(h, w, 300, seed=12)
    got = out[torch.from_numpy(ys).cuda(), torch.from_numpy(xs).cuda()].cpu().numpy().astype(np.float64)
    del out
    torch.cuda.empty_cache()
    ref = oracle.fast_abf(f, None, sg, "box", R, N, pixels=(ys, xs))
    assert np.max(np.abs(got - ref)) < TOL[precision]


# ----------------------------------------------------------------- streams
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_non_current_stream(torch, abf, precision):
    """Calls issued on a side stream while the current stream is busy with
    other work: the binding allocates its temporaries on the side stream, so
    results equal those of the same calls on the current stream, for the
    plain call, the strided batch and the texture helper."""
    f = rect_scene(61, 300, 500, n_rect=8, noise=10, side_lo=10, side_hi=120)
    sg = smooth_field(np.random.default_rng(61), 300, 500, 8, 40)
    fd, sd = dev(torch, f), dev(torch, sg)
    ref = abf.fast(fd, sd, kernel="box", rho=5, N=6, precision=precision)
    ref_b = abf.fast_strided(torch.stack([fd, fd.flip(0)]), torch.stack([sd, sd]), kernel="gaussian",
                             rho=7, N=5, precision=precision)
    ref_t = abf.texture_filter(torch.stack([fd, fd.flip(1)]), passes=2, precision=precision)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    big = torch.randn(4096, 4096, device="cuda")
    outs = []
    for _ in range(4):
        big = big @ big.T * 1e-3                  # keeps the current stream busy
        side.wait_stream(torch.cuda.current_stream())
        fb = torch.stack([fd, fd.flip(0)])
        sb = torch.stack([sd, sd])
        ft = torch.stack([fd, fd.flip(1)])
        side.wait_stream(torch.cuda.current_stream())
        a = abf.fast(fd, sd, kernel="box", rho=5, N=6, precision=precision, stream=side)
        b = abf.fast_strided(fb, sb, kernel="gaussian", rho=7, N=5, precision=precision, stream=side)
        c = abf.texture_filter(ft, passes=2, precision=precision, stream=side)
        # (the inputs made on the current stream stay referenced until the end)
        outs.append((a, b, c, fb, sb, ft))
        torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for a, b, c, *_ in outs:
        assert torch.equal(a, ref) and torch.equal(b, ref_b) and torch.equal(c, ref_t)
