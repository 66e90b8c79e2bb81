"""GPU tests of the batched entry points, the sigma map and the texture
pipeline against the oracle and against single-image calls."""
import numpy as np
import pytest

import oracle
from oracle.spatial import local_std_sigma
from synth import rect_scene, smooth_field, texture_frames

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


@pytest.mark.parametrize("kernel,R,N", [("box", 3, 5), ("box", 30, 6), ("gaussian", 5, 4), ("box", 2, 0),
                                         ("gaussian", 15, 6), ("gaussian", 20, 8)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_strided_equals_single_calls(torch, abf, kernel, R, N, precision):
    n, h, w = 5, 61, 97
    f = np.stack([rect_scene(300 + i, h, w, n_rect=4, noise=10, side_lo=4, side_hi=30) for i in range(n)])
    sg = np.stack([smooth_field(np.random.default_rng(i), h, w, 8, 40) for i in range(n)])
    fd = torch.from_numpy(f).cuda()
    sd = torch.from_numpy(sg).cuda()
    out = abf.fast_strided(fd, sd, kernel=kernel, rho=R, N=N, precision=precision)
    for i in range(n):
        single = abf.fast(fd[i], sd[i], kernel=kernel, rho=R, N=N, precision=precision)
        assert torch.equal(out[i], single), i
    # a strided view with a row pitch larger than w
    big = torch.zeros((n, h, w + 13), dtype=torch.float32, device="cuda")
    big[:, :, :w] = fd
    bs = torch.zeros_like(big)
    bs[:, :, :w] = sd
    out2 = abf.fast_strided(big[:, :, :w], bs[:, :, :w], kernel=kernel, rho=R, N=N, precision=precision)
    assert torch.equal(out2, out)


def test_sigma_map_matches_oracle(torch, abf):
    f = np.stack([rect_scene(50 + i, 70, 110, n_rect=5, noise=12, side_lo=4, side_hi=40) for i in range(3)])
    for r in (0, 1, 4):
        got = abf.sigma_local_std(torch.from_numpy(f).cuda(), radius=r).cpu().numpy()
        for i in range(3):
            ref = local_std_sigma(f[i], r)
            assert np.max(np.abs(got[i] - ref)) <= 1e-5 * 80


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_texture_pipeline_pass_by_pass(torch, abf, precision):
    fr = texture_frames(77, n_frames=2, h=72, w=120).reshape(6, 72, 120)
    x = torch.from_numpy(fr).cuda()
    for p in range(3):
        sig = abf.sigma_local_std(x, radius=4)
        y = abf.fast_strided(x, sig, kernel="box", rho=8, N=6, precision=precision)
        xs, ss, ys = x.cpu().numpy(), sig.cpu().numpy(), y.cpu().numpy().astype(np.float64)
        for i in (0, 3, 5):
            ref = oracle.fast_abf(xs[i], None, ss[i], "box", 8, 6)
            assert np.max(np.abs(ys[i] - ref)) < TOL[precision], (p, i)
        x = y.float()
    full = abf.texture_filter(torch.from_numpy(fr).cuda(), passes=3, precision=precision)
    assert torch.equal(full.float(), x)
