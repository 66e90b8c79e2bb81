"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on
the same seeded inputs.

Bars: window bounds and passthrough pixels bit-exact; FP64 path within
1e-6 and mixed path within 0.05 intensity units (on [0, 255]) of the
oracle's fast filter; brute force within 1e-9 (FP64) / 2e-3 (FP32).
Small images are compared at every pixel; full-size workloads at sampled
pixels (corners, edges and a seeded random set) that the oracle evaluates
one by one on the full image.
"""
import numpy as np
import pytest

import oracle
from oracle.spatial import window_minmax
from synth import WORKLOADS, rect_scene, smooth_field, voronoi, workload

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
    m.lib()          # fails loudly if the library is missing
    return m


def dev(torch, a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def sample_pixels(H, W, n=1500, seed=0):
    rng = np.random.default_rng(seed)
    ys = list(rng.integers(0, H, n)) + [0, 0, H - 1, H - 1, H // 2, 0, H - 1, H // 2]
    xs = list(rng.integers(0, W, n)) + [0, W - 1, 0, W - 1, 0, W // 2, W // 2, W - 1]
    return np.array(ys), np.array(xs)


def run_fast(torch, abf, wl, precision, **kw):
    out = abf.fast(dev(torch, wl["f"]), dev(torch, wl["sigma"]), theta=dev(torch, wl["theta"]),
                   kernel=wl["kernel"], rho=wl["R"], N=wl["N"], sigma_s=wl["sigma_s"],
                   precision=precision, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


# ----------------------------------------------------------------- bounds
@pytest.mark.parametrize("shape,R", [((256, 256), 3), ((37, 300), 5), ((300, 37), 20), ((1, 129), 4),
                                     ((129, 1), 4), ((5, 7), 20), ((1, 1), 3), ((70, 90), 0),
                                     ((200, 333), 96), ((64, 100), 1), ((33, 70), 2), ((65, 130), 6),
                                     ((100, 150), 24), ((97, 200), 25)])
def test_minmax_bit_exact(torch, abf, shape, R):
    f = rect_scene(11, *shape, n_rect=4, noise=10, side_lo=1, side_hi=max(2, min(shape)))
    a, b = abf.minmax(dev(torch, f), R)
    torch.cuda.synchronize()
    lo, hi = window_minmax(f, R)
    assert np.array_equal(a.cpu().numpy(), lo)
    assert np.array_equal(b.cpu().numpy(), hi)


def test_minmax_voronoi_full(torch, abf):
    f = voronoi(1003, 1024, 1536, n_seed=64)
    for R in (5, 20):
        a, b = abf.minmax(dev(torch, f), R)
        torch.cuda.synchronize()
        lo, hi = window_minmax(f, R)
        assert np.array_equal(a.cpu().numpy(), lo) and np.array_equal(b.cpu().numpy(), hi)



@pytest.mark.parametrize("R", [2, 5, 15, 30])
def test_bounds_mixed_sign_bit_exact(torch, abf, R):
    """Window bounds of finite inputs of both signs, with -0, +0, subnormal
    and near-FP32-max magnitudes (the kernels take each min/max as the
    median against an infinity): minmax_tile bit for bit, and the Gaussian
    tile kernel's own bounds (on values of moderate size, whose power sums
    stay finite) bit for bit where it takes them."""
    rng = np.random.default_rng(4321 + R)
    h, w = 97, 301
    f = (rng.standard_normal((h, w)) * 1e3).astype(np.float32)
    f[rng.random((h, w)) < 0.05] = np.float32(-0.0)
    f[rng.random((h, w)) < 0.02] = np.float32(1e-40)
    f[rng.random((h, w)) < 0.02] = np.float32(-1e-40)
    big = f.copy()
    big[rng.random((h, w)) < 0.02] = np.float32(3.0e38)
    big[rng.random((h, w)) < 0.02] = np.float32(-3.0e38)
    a, b = abf.minmax(dev(torch, big), R)
    torch.cuda.synchronize()
    lo, hi = window_minmax(big, R)
    assert np.array_equal(a.cpu().numpy().view(np.uint32), lo.view(np.uint32))
    assert np.array_equal(b.cpu().numpy().view(np.uint32), hi.view(np.uint32))
    if abf.stack_single_pass(h, w, "gaussian", R, 4):
        st = abf.moment_stack(dev(torch, f), kernel="gaussian", rho=R, N=4, precision="mixed")
        torch.cuda.synchronize()
        pl = abf.stack_planes(st, h, w, 4, "mixed")
        lo, hi = window_minmax(f, R)
        assert np.array_equal(pl[0].cpu().numpy().view(np.uint32), lo.view(np.uint32))
        assert np.array_equal(pl[1].cpu().numpy().view(np.uint32), hi.view(np.uint32))

# ----------------------------------------------------------------- stack
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel,R,N", [("box", 3, 5), ("box", 20, 8), ("gaussian", 6, 6)])
def test_moment_stack_matches_oracle(torch, abf, precision, kernel, R, N):
    f = rect_scene(21, 96, 280, n_rect=6, noise=10, side_lo=8, side_hi=64)
    st = abf.moment_stack(dev(torch, f), kernel=kernel, rho=R, N=N, precision=precision)
    torch.cuda.synchronize()
    a, b, mom = abf.stack_planes(st, *f.shape, N, precision)
    _, aux = oracle.fast_abf(f, None, np.full(f.shape, 20.0), kernel, R, N, aux=True)
    assert np.array_equal(a.cpu().numpy(), aux["alpha"].astype(np.float32))
    assert np.array_equal(b.cpu().numpy(), aux["beta"].astype(np.float32))
    live = aux["alpha"] != aux["beta"]
    # The power sums are shifted from the wave's origin to each window's
    # mid-range (Prop. 3); the shift amplifies FP64 rounding by about
    # ((|mid - origin| + half) / half)^k, which reaches ~1e7 at k = 5 for the
    # narrowest windows of this image (range ~10 units, origin ~100 away):
    # 1e-7 on a~_k. The end-to-end tests below bound what this does to g^.
    tol = 1e-6 if precision == "fp64" else 2e-6
    for k in range(N):
        got = mom[k].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got[live] - aux["amom"][..., k + 1][live])) < tol, k
        assert np.all(got[~live] == 0)


# ----------------------------------------------------------------- range alone
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_range_stage_on_oracle_stack(torch, abf, precision):
    """Feed the oracle's own bounds and Legendre moments to abf_range, which
    isolates the range kernel's error (integrals, fit, ratio)."""
    f = rect_scene(5, 64, 200, n_rect=5, noise=10, side_lo=8, side_hi=40)
    zeta = smooth_field(np.random.default_rng(3), *f.shape, -20, 20)
    th = (f + zeta).astype(np.float32)
    sg = smooth_field(np.random.default_rng(4), *f.shape, 3, 90)
    sg[:8, :8] = np.inf
    N, R = 8, 4
    ref, aux = oracle.fast_abf(f, th, sg, "box", R, N, aux=True)
    st = abf.moment_stack(dev(torch, f), kernel="box", rho=R, N=N, precision=precision)
    a, b, mom = abf.stack_planes(st, *f.shape, N, precision)
    mdt = torch.float64 if precision == "fp64" else torch.float32
    for k in range(N):
        mom[k].copy_(torch.from_numpy(np.nan_to_num(aux["amom"][..., k + 1]) * (aux["alpha"] != aux["beta"])).to(mdt))
    out = abf.range_from_stack(st, dev(torch, sg), img=dev(torch, f), theta=dev(torch, th), N=N,
                               precision=precision)
    torch.cuda.synchronize()
    err = np.abs(out.cpu().numpy().astype(np.float64) - ref)
    assert np.max(err) < (2e-7 if precision == "fp64" else 1e-3), np.max(err)


# ----------------------------------------------------------------- end to end
# (Gaussian R = 1 and 16: the tile kernel's split tail wave with its shortest
# halves, 3 rows, and its widest tail, 32 columns)
SMALL = [("box", 3, 5), ("box", 1, 0), ("box", 2, 1), ("box", 5, 8), ("gaussian", 4, 6), ("gaussian", 9, 3),
         ("gaussian", 1, 4), ("gaussian", 16, 5)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel,R,N", SMALL)
def test_fast_small_images_every_pixel(torch, abf, precision, kernel, R, N):
    f = rect_scene(7 + R, 72, 301, n_rect=6, noise=10, side_lo=6, side_hi=48)
    sg = smooth_field(np.random.default_rng(R), *f.shape, 10, 30)
    wl = dict(f=f, theta=None, sigma=sg, kernel=kernel, R=R, N=N, sigma_s=0.0)
    got = run_fast(torch, abf, wl, precision)
    ref = oracle.fast_abf(f, None, sg, kernel, R, N)
    lo, hi = window_minmax(f, R)
    flat = lo == hi
    assert np.array_equal(got[flat], f[flat].astype(np.float64))
    assert np.max(np.abs(got - ref)) < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fast_rects256_full(torch, abf, precision):
    wl = workload("rects256_box3_n5")
    got = run_fast(torch, abf, wl, precision)
    ref = oracle.fast_abf(wl["f"], wl["theta"], wl["sigma"], wl["kernel"], wl["R"], wl["N"])
    assert np.max(np.abs(got - ref)) < TOL[precision]


@pytest.fixture(scope="module")
def sharpen():
    return workload("sharpen1024_gauss15_n6")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fast_sharpen1024_sampled(torch, abf, sharpen, precision):
    wl = sharpen
    got = run_fast(torch, abf, wl, precision)
    ys, xs = sample_pixels(*wl["f"].shape, n=1500, seed=2)
    ref = oracle.fast_abf(wl["f"], wl["theta"], wl["sigma"], wl["kernel"], wl["R"], wl["N"],
                          sigma_s=wl["sigma_s"], pixels=(ys, xs))
    assert np.max(np.abs(got[ys, xs] - ref)) < TOL[precision]


@pytest.fixture(scope="module")
def vor4096():
    return voronoi(1003, 4096, 4096)


@pytest.mark.parametrize("R", [5, 20])
@pytest.mark.parametrize("N", [5, 6, 7, 8])
def test_fast_voronoi4096_sampled(torch, abf, vor4096, R, N):
    wl = WORKLOADS[f"voronoi4096_box{R}_n{N}"]()
    assert np.array_equal(wl["f"], vor4096)
    ys, xs = sample_pixels(4096, 4096, n=800, seed=R + N)
    ref = oracle.fast_abf(wl["f"], None, wl["sigma"], "box", R, N, pixels=(ys, xs))
    for precision in ("fp64", "mixed"):
        got = run_fast(torch, abf, wl, precision)
        assert np.max(np.abs(got[ys, xs] - ref)) < TOL[precision], precision


# ----------------------------------------------------------------- edge cases
def test_edge_constant_and_tiny(torch, abf):
    for shape in [(1, 1), (1, 17), (17, 1), (3, 4)]:
        f = np.full(shape, 12.5, dtype=np.float32)
        for prec in ("fp64", "mixed"):
            out = abf.fast(dev(torch, f), dev(torch, np.full(shape, 9.0)), rho=5, N=6, precision=prec)
            assert np.array_equal(out.cpu().numpy().astype(np.float64), f.astype(np.float64))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_edge_sigma_inf_and_theta_far(torch, abf, precision):
    f = rect_scene(3, 40, 50, n_rect=4, noise=10, side_lo=4, side_hi=20)
    sg = np.full(f.shape, np.inf, dtype=np.float32)
    got = abf.fast(dev(torch, f), dev(torch, sg), rho=2, N=5, precision=precision).cpu().numpy()
    ref = oracle.fast_abf(f, None, sg, "box", 2, 5)
    assert np.max(np.abs(got - ref)) < TOL[precision]
    th = (f + 300.0).astype(np.float32)   # centre far above every window
    sg2 = np.full(f.shape, 15.0, dtype=np.float32)
    got = abf.fast(dev(torch, f), dev(torch, sg2), theta=dev(torch, th), rho=2, N=5,
                   precision=precision).cpu().numpy()
    ref = oracle.fast_abf(f, th, sg2, "box", 2, 5)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref)) < TOL[precision]


@pytest.mark.parametrize("amp", [0.05, 0.08])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_narrow_windows_far_from_origin(torch, abf, precision, amp):
    """Plateaus at 90 and 110 (alternating every 48 columns, so every wave's
    samples span both) with noise of +-amp: the windows inside a plateau
    are about 2 amp wide and 10 away from the wave's origin (rho about 200
    and 125), so their shift is ill-conditioned at N = 6 and 7. On the FP32
    stack they are taken through the width-aware acceptance or recomputed
    from their windows, on the FP64 path recomputed; every pixel within the
    bar of the oracle."""
    h, w = 64, 400
    rng = np.random.default_rng(int(amp * 1000))
    base = np.where((np.arange(w) // 48) % 2 == 0, 90.0, 110.0)
    f = (base[None, :] + rng.uniform(-amp, amp, (h, w))).astype(np.float32)
    sg = smooth_field(np.random.default_rng(2), h, w, 0.05, 30.0)
    for N in (6, 7):
        got = abf.fast(dev(torch, f), dev(torch, sg), rho=5, N=N, precision=precision)
        ref = oracle.fast_abf(f, None, sg, "box", 5, N)
        assert np.max(np.abs(got.cpu().numpy().astype(np.float64) - ref)) < TOL[precision], N


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_edge_window_larger_than_image(torch, abf, precision):
    f = rect_scene(9, 9, 23, n_rect=3, noise=10, side_lo=2, side_hi=6)
    sg = np.full(f.shape, 25.0, dtype=np.float32)
    got = abf.fast(dev(torch, f), dev(torch, sg), rho=30, N=6, precision=precision).cpu().numpy()
    ref = oracle.fast_abf(f, None, sg, "box", 30, 6)
    assert np.max(np.abs(got - ref)) < TOL[precision]


# ----------------------------------------------------------------- brute force
@pytest.mark.parametrize("kernel,R", [("box", 3), ("gaussian", 7)])
def test_bruteforce_matches_oracle(torch, abf, kernel, R):
    f = rect_scene(13, 80, 140, n_rect=5, noise=10, side_lo=6, side_hi=40)
    zeta = smooth_field(np.random.default_rng(1), *f.shape, -20, 20)
    th = (f + zeta).astype(np.float32)
    sg = smooth_field(np.random.default_rng(2), *f.shape, 5, 40)
    ref = oracle.brute_abf(f, th, sg, kernel, R)
    g64 = abf.bruteforce(dev(torch, f), dev(torch, sg), theta=dev(torch, th), kernel=kernel, rho=R,
                         precision="fp64").cpu().numpy()
    g32 = abf.bruteforce(dev(torch, f), dev(torch, sg), theta=dev(torch, th), kernel=kernel, rho=R,
                         precision="mixed").cpu().numpy()
    assert np.max(np.abs(g64 - ref)) < 1e-9
    assert np.max(np.abs(g32 - ref)) < 2e-3


# ----------------------------------------------------------------- API properties
def test_batched_equals_single_and_deterministic(torch, abf):
    items, singles = [], []
    for i, (h, w, kernel, R, N) in enumerate([(64, 100, "box", 3, 5), (130, 70, "gaussian", 5, 6),
                                              (33, 257, "box", 20, 8)]):
        f = rect_scene(100 + i, h, w, n_rect=4, noise=10, side_lo=4, side_hi=30)
        sg = smooth_field(np.random.default_rng(i), h, w, 10, 30)
        it = dict(img=dev(torch, f), sigma=dev(torch, sg), kernel=kernel, rho=R, N=N)
        items.append(it)
        singles.append(abf.fast(it["img"], it["sigma"], kernel=kernel, rho=R, N=N))
    outs = abf.fast_batched(items)
    outs2 = abf.fast_batched(items)
    torch.cuda.synchronize()
    for a, b, c in zip(outs, singles, outs2):
        assert torch.equal(a, b) and torch.equal(a, c)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batched_groups_equal_single(torch, abf, precision):
    """Requests that share launches (one shape and parameter set, each with
    its own buffers, some as row-pitched views) give exactly abf_fast's
    output: box kernel (strip kernel), Gaussian (tile kernel taking the
    bounds), a radius above the bounds kernel's tile limit (its per-image
    host loop), theta given or not, mixed with single requests and the
    recursive kernel (one image per launch)."""
    specs = [(60, 90, "box", 4, 5, False), (60, 90, "box", 4, 5, False), (41, 130, "gaussian", 6, 6, True),
             (60, 90, "box", 4, 5, False), (41, 130, "gaussian", 6, 6, True), (70, 50, "box", 30, 7, False),
             (70, 50, "box", 30, 7, False), (33, 47, "box", 2, 3, False), (41, 130, "gaussian", 6, 6, True)]
    if precision == "mixed":
        specs += [(50, 60, "recursive", 5, 6, False), (50, 60, "recursive", 5, 6, False)]
    items, singles = [], []
    for i, (h, w, kernel, R, N, with_theta) in enumerate(specs):
        f = rect_scene(300 + i, h, w, n_rect=4, noise=8, side_lo=4, side_hi=30)
        sg = smooth_field(np.random.default_rng(i), h, w, 8, 35)
        img = dev(torch, f)
        if i % 3 == 1:       # a row-pitched view into a wider buffer
            wide = torch.zeros((h, w + 13), dtype=torch.float32, device="cuda")
            wide[:, 3:3 + w] = img
            img = wide[:, 3:3 + w]
            sgw = torch.zeros((h, w + 13), dtype=torch.float32, device="cuda")
            sgw[:, 3:3 + w] = dev(torch, sg)
            sgd = sgw[:, 3:3 + w]
        else:
            sgd = dev(torch, sg)
        th = None
        if with_theta:
            th = img + dev(torch, smooth_field(np.random.default_rng(50 + i), h, w, -15, 15))
            if i % 3 == 1:
                thw = torch.zeros((h, w + 13), dtype=torch.float32, device="cuda")
                thw[:, 3:3 + w] = th
                th = thw[:, 3:3 + w]
        it = dict(img=img, sigma=sgd, theta=th, kernel=kernel, rho=R, N=N)
        items.append(it)
        singles.append(abf.fast(img, sgd, theta=th, kernel=kernel, rho=R, N=N, precision=precision))
    outs = abf.fast_batched(items, precision=precision)
    outs2 = abf.fast_batched(items, precision=precision)
    torch.cuda.synchronize()
    for i, (a, b, c) in enumerate(zip(outs, singles, outs2)):
        assert torch.equal(a, b) and torch.equal(a, c), i


def test_stack_reuse_for_new_theta_sigma(torch, abf):
    f = rect_scene(41, 90, 120, n_rect=5, noise=10, side_lo=6, side_hi=40)
    st = abf.moment_stack(dev(torch, f), rho=4, N=6, precision="mixed")
    for seed in range(3):
        sg = smooth_field(np.random.default_rng(seed), *f.shape, 5, 50)
        th = (f + smooth_field(np.random.default_rng(seed + 9), *f.shape, -10, 10)).astype(np.float32)
        a = abf.range_from_stack(st, dev(torch, sg), img=dev(torch, f), theta=dev(torch, th), N=6)
        b = abf.fast(dev(torch, f), dev(torch, sg), theta=dev(torch, th), rho=4, N=6)
        assert torch.equal(a, b)


SINGLE_PASS = [((256, 300), 15, 6), ((37, 300), 5, 8), ((300, 37), 20, 5), ((1, 129), 4, 6),
               ((129, 1), 4, 6), ((5, 7), 20, 3), ((1, 1), 3, 2), ((70, 90), 0, 6), ((70, 90), 1, 7),
               ((130, 517), 2, 1), ((150, 700), 12, 8), ((120, 400), 40, 7), ((90, 260), 60, 8),
               ((64, 390), 16, 6)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel,shape,R,N", [("gaussian",) + c for c in SINGLE_PASS])
def test_single_pass_stack_equals_two_pass(torch, abf, precision, kernel, shape, R, N):
    """Where the Gaussian tile kernel takes the window bounds itself
    (abf_stack_single_pass), abf_moment_stack equals abf_minmax followed by
    abf_stack_moments bit for bit, and its bounds are the exact window
    min/max (with -0 stored as +0). The image has noisy rectangles, a
    near-flat patch (exact recompute of ill-conditioned shifts) and -0."""
    h, w = shape
    f = rect_scene(300 + R + N, h, w, n_rect=6, noise=0.7, side_lo=2, side_hi=60)
    f[h // 3: h // 3 + 20, w // 4: w // 4 + 40] = np.float32(250.0)
    f[h // 3: h // 3 + 20, w // 4: w // 4 + 40] += (np.arange(min(40, w - w // 4), dtype=np.float32) % 3) * np.float32(0.25)
    f[::7, ::5] = np.float32(-0.0)
    assert abf.stack_single_pass(h, w, kernel, R, N)
    img = dev(torch, f)
    one = abf.moment_stack(img, kernel=kernel, rho=R, N=N, precision=precision)
    two = torch.zeros_like(one)
    abf.minmax_into_stack(img, two, R, N, precision=precision)
    abf.stack_moments(img, two, kernel=kernel, rho=R, N=N, precision=precision)
    torch.cuda.synchronize()
    p1 = abf.stack_planes(one, h, w, N, precision)
    p2 = abf.stack_planes(two, h, w, N, precision)
    for a, b in zip((p1[0], p1[1], *p1[2]), (p2[0], p2[1], *p2[2])):
        assert torch.equal(a, b)
    lo, hi = window_minmax(f, R)
    assert np.array_equal(p1[0].cpu().numpy().view(np.uint32), lo.astype(np.float32).view(np.uint32))
    assert np.array_equal(p1[1].cpu().numpy().view(np.uint32), hi.astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("kernel,R,N", [("box", 3, 8), ("gaussian", 7, 8), ("box", 5, 7),
                                        ("gaussian", 12, 7)])
def test_fp64_every_pixel_high_contrast(torch, abf, kernel, R, N):
    """FP64 path at N = 7, 8 on clipped, high-contrast content (Voronoi cells at
    levels U[0, 255] plus noise, clipped): every pixel within 1e-6 of the
    oracle. Strips and tiles there span dark and bright cells, so one origin
    for a region's power sums is far from many windows, and the box
    kernel's running sums carry the rounding of the strip's extreme values;
    with a single origin and the N <= 5 threshold at every degree, the FP64
    path missed the bound on 13 (box) and 239 (Gaussian) pixels of this
    image at N = 8."""
    from synth.generators import block_constant
    h, w = 256, 512
    f = voronoi(1201, h, w, n_seed=24, noise=15.0)
    sg = block_constant(np.random.default_rng(1202), h, w, 10, 40)
    ss = R / 3.0 if kernel == "gaussian" else 0.0
    out = abf.fast(dev(torch, f), dev(torch, sg), kernel=kernel, rho=R, N=N, sigma_s=ss,
                   precision="fp64")
    torch.cuda.synchronize()
    ref = oracle.fast_abf(f, None, sg, kernel, R, N, sigma_s=ss)
    err = np.abs(out.cpu().numpy() - ref)
    assert err.max() <= TOL["fp64"], (float(err.max()), int((err > TOL["fp64"]).sum()))


FUSED_CASES = [("box", 3, 5), ("box", 20, 8), ("box", 5, 1), ("gaussian", 15, 6), ("gaussian", 4, 8),
               ("gaussian", 40, 7)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel,R,N", FUSED_CASES)
def test_fused_equals_stack_path(torch, abf, precision, kernel, R, N):
    """abf_moments_range (moments and range stage in one kernel) against the
    stack path (abf_moment_stack + abf_range, as in abf_fast): bit-identical,
    with and without keeping the stack. The image mixes noisy rectangles with
    near-flat bright patches, whose windows take the exact recompute for
    ill-conditioned shifts."""
    f = rect_scene(60 + R, 150, 700, n_rect=10, noise=0.7, side_lo=10, side_hi=90)
    f[40:90, 100:400] = np.float32(250.0) + (np.arange(300, dtype=np.float32) % 3) * np.float32(0.25)
    sg = smooth_field(np.random.default_rng(R + N), *f.shape, 4, 60)
    th = (f + smooth_field(np.random.default_rng(R), *f.shape, -15, 15)).astype(np.float32)
    img, sgd, thd = dev(torch, f), dev(torch, sg), dev(torch, th)
    st = abf.moment_stack(img, kernel=kernel, rho=R, N=N, precision=precision)
    ref = abf.range_from_stack(st, sgd, img=img, theta=thd, N=N, precision=precision)
    out = abf.fast(img, sgd, theta=thd, kernel=kernel, rho=R, N=N, precision=precision)
    st1 = torch.zeros_like(st)
    abf.minmax_into_stack(img, st1, R, N, precision=precision)
    out1 = abf.moments_range(img, st1, sgd, theta=thd, kernel=kernel, rho=R, N=N,
                             precision=precision)
    # keep_stack: the fused kernel's stored moments equal the stack path's
    st2 = torch.zeros_like(st)
    abf.minmax_into_stack(img, st2, R, N, precision=precision)
    out2 = abf.moments_range(img, st2, sgd, theta=thd, kernel=kernel, rho=R, N=N,
                             precision=precision, keep_stack=True)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert torch.equal(out1, ref)
    assert torch.equal(out2, ref)
    for p, q in zip(abf.stack_planes(st, *f.shape, N, precision)[2],
                    abf.stack_planes(st2, *f.shape, N, precision)[2]):
        assert torch.equal(p, q)


FUSED_EDGE = [((1, 1), 0, 1), ((1, 1), 8, 8), ((1, 300), 5, 6), ((300, 1), 5, 6), ((5, 7), 8, 8),
              ((70, 90), 0, 6), ((70, 90), 1, 7), ((257, 513), 8, 1), ((64, 250), 4, 5),
              ((90, 450), 20, 8), ((41, 37), 32, 6), ((200, 200), 13, 5)]


@pytest.mark.parametrize("shape,R,N", FUSED_EDGE)
def test_fused_default_edges(torch, abf, shape, R, N):
    """abf_fast's fused path (box kernel, mixed, rho <= 32) on single pixels,
    single rows and columns, rho = 0 and 1, N = 1, and strips with a partial
    last chunk: equal to the stack path bit for bit, and within the mixed
    bar of the oracle at every pixel."""
    h, w = shape
    assert abf.fast_fused(h, w, "box", R, N, "mixed")
    f = rect_scene(700 + R + N, h, w, n_rect=4, noise=9.0, side_lo=1, side_hi=max(2, min(h, w)))
    sg = smooth_field(np.random.default_rng(R + 3 * N), h, w, 6, 45)
    th = (f + smooth_field(np.random.default_rng(N), h, w, -12, 12)).astype(np.float32)
    img, sgd, thd = dev(torch, f), dev(torch, sg), dev(torch, th)
    out = abf.fast(img, sgd, theta=thd, kernel="box", rho=R, N=N, precision="mixed")
    st = abf.moment_stack(img, kernel="box", rho=R, N=N, precision="mixed")
    ref = abf.range_from_stack(st, sgd, img=img, theta=thd, N=N, precision="mixed")
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    want = oracle.fast_abf(f, th, sg, "box", R, N)
    assert np.max(np.abs(out.cpu().numpy().astype(np.float64) - want)) < TOL["mixed"]


GAUSS_ONE = [((1, 1), 3, 6), ((7, 300), 5, 8), ((70, 90), 15, 6), ((130, 257), 20, 5),
             ((64, 200), 1, 1), ((33, 47), 40, 7), ((600, 520), 12, 6)]


@pytest.mark.parametrize("shape,R,N", GAUSS_ONE)
def test_gaussian_one_kernel_default(torch, abf, shape, R, N):
    """abf_fast's Gaussian path on the mixed path, where the tile kernel
    takes the window bounds itself: one kernel for the whole filter (bounds,
    moments, range stage). Equal to the stack path bit for bit and within
    the mixed bar of the oracle at every pixel; single pixels and rows,
    ragged tiles, both LDS strides (R up to 16 and above)."""
    h, w = shape
    assert abf.fast_fused(h, w, "gaussian", R, N, "mixed")
    f = rect_scene(900 + R + N, h, w, n_rect=4, noise=7.0, side_lo=1, side_hi=max(2, min(h, w)))
    sg = smooth_field(np.random.default_rng(R + 5 * N), h, w, 6, 45)
    th = (f + smooth_field(np.random.default_rng(N + 1), h, w, -10, 10)).astype(np.float32)
    img, sgd, thd = dev(torch, f), dev(torch, sg), dev(torch, th)
    out = abf.fast(img, sgd, theta=thd, kernel="gaussian", rho=R, N=N, precision="mixed")
    st = abf.moment_stack(img, kernel="gaussian", rho=R, N=N, precision="mixed")
    ref = abf.range_from_stack(st, sgd, img=img, theta=thd, N=N, precision="mixed")
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    if h * w * (2 * R + 1) ** 2 <= 3e7:
        want = oracle.fast_abf(f, th, sg, "gaussian", R, N)
        assert np.max(np.abs(out.cpu().numpy().astype(np.float64) - want)) < TOL["mixed"]
    else:
        rng = np.random.default_rng(R)
        ys, xs = rng.integers(0, h, 800), rng.integers(0, w, 800)
        want = oracle.fast_abf(f, th, sg, "gaussian", R, N, pixels=(ys, xs))
        got = out.cpu().numpy().astype(np.float64)[ys, xs]
        assert np.max(np.abs(got - want)) < TOL["mixed"]


@pytest.mark.parametrize("R,N", [(5, 8), (8, 6), (3, 5), (20, 8)])
def test_fused_default_equals_stack_path_4096(torch, abf, vor4096, R, N):
    """At 4096^2 the box kernel's segment geometry fills the device in whole
    rounds of waves; where abf_fast takes the fused path (mixed, rho <= 32)
    the geometry is sized for both instantiations, so abf_fast's output
    equals the stack path's bit for bit on a full-size image too."""
    assert abf.fast_fused(4096, 4096, "box", R, N, "mixed")
    sg = smooth_field(np.random.default_rng(R * 10 + N), 4096, 4096, 10, 40)
    img, sgd = dev(torch, vor4096), dev(torch, sg)
    out = abf.fast(img, sgd, kernel="box", rho=R, N=N, precision="mixed")
    st = abf.moment_stack(img, kernel="box", rho=R, N=N, precision="mixed")
    ref = abf.range_from_stack(st, sgd, img=img, N=N, precision="mixed")
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("R,N", [(12, 8), (8, 5), (16, 6)])
def test_fast_gaussian_large_image_sampled(torch, abf, precision, R, N):
    """Wide Gaussian windows on a 2048 x 2040 image, just below the size at
    which the moment stage moves to the matrix cores: the tile kernel at a
    large size, sampled pixels against the oracle, edges, corners and the
    last partial tile included. (The matrix-core kernel has its own tests.)"""
    from synth import gauss_field
    assert abf.stack_kernel(2048, 2040, "gaussian", R, N, precision) in ("tile", "tile_wide")
    f = gauss_field(77 + R, 2048, 2040)
    sg = smooth_field(np.random.default_rng(R), *f.shape, 5, 60)
    th = (f + smooth_field(np.random.default_rng(R + 1), *f.shape, -20, 20)).astype(np.float32)
    wl = dict(f=f, theta=th, sigma=sg, kernel="gaussian", R=R, N=N, sigma_s=R / 3.0)
    out = run_fast(torch, abf, wl, precision)
    ys, xs = sample_pixels(*f.shape, n=400, seed=R)
    ys = np.concatenate([ys, [2047, 2047, 2040, 15, 16]])
    xs = np.concatenate([xs, [2039, 1000, 7, 2039, 0]])
    ref = oracle.fast_abf(f, th, sg, "gaussian", R, N, sigma_s=R / 3.0, pixels=(ys, xs))
    err = np.abs(out[ys, xs] - ref)
    assert np.max(err) < TOL[precision], np.max(err)
