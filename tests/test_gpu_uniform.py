"""GPU parity of the uniform-prior comparison variant (abf_uniform_prior,
abf_range_uniform) against oracle/uniform.py, and the classical-filter
observations of Sec. III-B on the GPU path."""
import numpy as np
import pytest

import oracle
from oracle.uniform import uniform_prior_abf, window_mean
from synth import rect_scene, smooth_field

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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel,R", [("box", 2), ("box", 5), ("gaussian", 6), ("box", 20)])
def test_uniform_prior_every_pixel(torch, abf, precision, kernel, R):
    f = rect_scene(31 + R, 70, 203, n_rect=6, noise=10, side_lo=6, side_hi=48)
    th = (f + smooth_field(np.random.default_rng(R), *f.shape, -15, 15)).astype(np.float32)
    sg = smooth_field(np.random.default_rng(R + 1), *f.shape, 4, 60)
    ref = uniform_prior_abf(f, th, sg, kernel, R)
    out = abf.uniform_prior(dev(torch, f), dev(torch, sg), theta=dev(torch, th), kernel=kernel,
                            rho=R, precision=precision)
    torch.cuda.synchronize()
    err = np.abs(out.cpu().numpy().astype(np.float64) - ref)
    assert np.max(err) < TOL[precision], (np.max(err), np.unravel_index(np.argmax(err), err.shape))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_uniform_prior_infinite_sigma_and_constant(torch, abf, precision):
    f = rect_scene(8, 40, 90, n_rect=4, noise=10, side_lo=6, side_hi=30)
    sg = np.full(f.shape, np.inf, np.float32)
    out = abf.uniform_prior(dev(torch, f), dev(torch, sg), kernel="box", rho=3, precision=precision)
    torch.cuda.synchronize()
    assert np.max(np.abs(out.cpu().numpy() - window_mean(f, "box", 3))) < TOL[precision]
    c = np.full((33, 47), 91.0, np.float32)
    out = abf.uniform_prior(dev(torch, c), dev(torch, np.full(c.shape, 20.0, np.float32)), rho=4,
                            precision=precision)
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 91.0)


def test_uniform_from_resident_stack(torch, abf):
    f = rect_scene(12, 64, 150, n_rect=5, noise=10, side_lo=6, side_hi=40)
    sg = smooth_field(np.random.default_rng(5), *f.shape, 5, 50)
    img, sgd = dev(torch, f), dev(torch, sg)
    st = abf.moment_stack(img, kernel="gaussian", rho=5, N=6, precision="fp64")
    a = abf.range_uniform_from_stack(st, img, sgd, N=6, precision="fp64")
    b = abf.uniform_prior(img, sgd, kernel="gaussian", rho=5, precision="fp64")
    torch.cuda.synchronize()
    assert np.max(np.abs(a.cpu().numpy() - b.cpu().numpy())) < 1e-6
    with pytest.raises(abf.ABFError):
        abf.range_uniform_from_stack(st, img, sgd, N=0, precision="fp64")


def test_classical_filter_observations_on_gpu(torch, abf):
    """Classical filter (theta = f, sigma = 40), GPU brute force as the
    reference: the PSNR of Algorithm 1 rises with N, and from N = 1 on it
    beats the uniform prior (Sec. III-B)."""
    f = rect_scene(21, 256, 256)
    img = dev(torch, f)
    sg = torch.full_like(img, 40.0)
    for R in (3, 5, 10):
        b = abf.bruteforce(img, sg, kernel="box", rho=R, precision="fp64").cpu().numpy()
        psnr = lambda g: 10 * np.log10(255.0 ** 2 / np.mean((g.cpu().numpy().astype(np.float64) - b) ** 2))
        ours = [psnr(abf.fast(img, sg, kernel="box", rho=R, N=N, precision="fp64")) for N in range(7)]
        u = psnr(abf.uniform_prior(img, sg, kernel="box", rho=R, precision="fp64"))
        assert ours[1] > u, (R, ours[1], u)
        assert all(y > x for x, y in zip(ours, ours[1:])), (R, ours)
