"""GPU parity of the application parameter maps (abf_sharpen_maps,
abf_mrtv_sigma, abf_grey) against oracle/maps.py, and the Sec. IV-C texture
procedure pass by pass against the oracle's filter fed the same maps."""
import numpy as np
import pytest

import oracle
from oracle import maps
from synth import rect_scene, texture_frames

pytestmark = pytest.mark.gpu


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
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("shape,r,s", [((70, 131), 5, 1.0), ((33, 40), 2, 0.7), ((16, 17), 0, 2.0),
                                       ((90, 77), 12, 3.0)])
def test_sharpen_maps(torch, abf, shape, r, s):
    f = rect_scene(r + 3, *shape, n_rect=5, noise=8, side_lo=4, side_hi=30)
    th, sg = abf.sharpen_maps(dev(torch, f), radius=r, log_sigma=s, lo=5.0, hi=40.0, v_ref=15.0)
    torch.cuda.synchronize()
    rth, rsg = maps.sharpen_maps(f, r, s, 5.0, 40.0, 15.0)
    assert np.max(np.abs(th.cpu().numpy()[0] - rth)) < 1e-4
    assert np.max(np.abs(sg.cpu().numpy()[0] - rsg)) < 1e-4


@pytest.mark.parametrize("shape,r", [((70, 131), 2), ((33, 40), 1), ((50, 61), 6), ((20, 23), 0)])
def test_mrtv_sigma(torch, abf, shape, r):
    f = rect_scene(r + 11, *shape, n_rect=6, noise=8, side_lo=4, side_hi=30)
    sg = abf.mrtv_sigma(dev(torch, f), radius=r, eps=1e-3, lo=5.0, hi=80.0, v_ref=20.0)
    torch.cuda.synchronize()
    ref = maps.mrtv_sigma(f, r, 1e-3, 5.0, 80.0, 20.0)
    assert np.max(np.abs(sg.cpu().numpy()[0] - ref)) < 1e-4


def test_grey_and_batches(torch, abf):
    fr = texture_frames(3, n_frames=2, h=40, w=57)
    g = abf.grey(dev(torch, fr))
    torch.cuda.synchronize()
    for i in range(2):
        assert np.max(np.abs(g.cpu().numpy()[i] - maps.grey(fr[i]))) < 1e-4
    # a batch gives the per-image maps
    x = dev(torch, fr.reshape(6, 40, 57))
    sb = abf.mrtv_sigma(x, radius=2)
    th, sg = abf.sharpen_maps(x, radius=3)
    torch.cuda.synchronize()
    for k in range(6):
        assert torch.equal(sb[k], abf.mrtv_sigma(x[k], radius=2)[0])
        t1, s1 = abf.sharpen_maps(x[k], radius=3)
        assert torch.equal(th[k], t1[0]) and torch.equal(sg[k], s1[0])


def test_map_argument_checks(torch, abf):
    x = dev(torch, np.zeros((8, 8)))
    with pytest.raises(abf.ABFError):
        abf.sharpen_maps(x, radius=40)
    with pytest.raises(abf.ABFError):
        abf.mrtv_sigma(x, radius=2, eps=0.0)
    with pytest.raises(abf.ABFError):
        abf.mrtv_sigma(x, radius=2, lo=50.0, hi=10.0)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_texture_procedure_pass_by_pass(torch, abf, precision):
    fr = texture_frames(9, n_frames=1, h=48, w=72)
    R, N = 4, 6
    k = abf.texture_filter_paper(dev(torch, fr), rho=R, N=N, precision=precision, keep=True)
    torch.cuda.synchronize()
    tol = 1e-6 if precision == "fp64" else 0.05
    # maps against the oracle's maps of the same inputs
    g0 = maps.grey(fr[0])
    assert np.max(np.abs(k["grey0"].cpu().numpy()[0] - g0)) < 1e-4
    s1 = maps.mrtv_sigma(k["grey0"].cpu().numpy()[0], 2, 1e-3, 5.0, 80.0, 20.0)
    assert np.max(np.abs(k["sigma1"].cpu().numpy()[0, 0] - s1)) < 1e-4
    assert np.max(np.abs(k["sigma2"].cpu().numpy()[0, 0] - 0.8 * s1)) < 1e-4
    # each pass against the oracle's filter fed the GPU's own input and maps
    src = [fr[0], k["pass1"].cpu().numpy()[0].astype(np.float32),
           k["pass2"].cpu().numpy()[0].astype(np.float32)]
    outs = [k["pass1"], k["pass2"], k["pass3"]]
    sig = [k["sigma1"], k["sigma2"], k["sigma3"]]
    th3 = k["theta3"].cpu().numpy()[0]
    for p in range(3):
        for c in range(3):
            ref = oracle.fast_abf(src[p][c], th3[c] if p == 2 else None,
                                  sig[p].cpu().numpy()[0, c], "box", R, N)
            got = outs[p].cpu().numpy()[0, c].astype(np.float64)
            assert np.max(np.abs(got - ref)) < tol, (p, c, np.max(np.abs(got - ref)))
    # pass 3's maps: theta from each channel, sigma from the grey image
    g2 = maps.grey(src[2])
    rth, _ = maps.sharpen_maps(src[2][1], R, 1.0, 5.0, 40.0, 20.0)
    _, rsg = maps.sharpen_maps(k["grey2"].cpu().numpy()[0], R, 1.0, 5.0, 40.0, 20.0)
    assert np.max(np.abs(k["grey2"].cpu().numpy()[0] - g2)) < 1e-3
    assert np.max(np.abs(th3[1] - rth)) < 1e-3
    assert np.max(np.abs(k["sigma3"].cpu().numpy()[0, 2] - rsg)) < 1e-4
