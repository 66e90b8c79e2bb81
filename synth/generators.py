"""Seeded generators of images, theta maps and sigma maps (see package docstring)."""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _f32(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a + np.float32(0.0)          # -0.0 -> +0.0


def smooth_field(rng: np.random.Generator, h: int, w: int, lo: float, hi: float,
                 grid: int = 8) -> np.ndarray:
    """An 8x8 grid of U[lo, hi] values, bilinearly upsampled to h x w.

    Grid node (a, b) sits on pixel ((h-1) a / (grid-1), (w-1) b / (grid-1))
    (align-corners interpolation), so every value lies in [lo, hi].
    """
    g = rng.uniform(lo, hi, size=(grid, grid))
    ys = np.linspace(0.0, grid - 1.0, h) if h > 1 else np.zeros(1)
    xs = np.linspace(0.0, grid - 1.0, w) if w > 1 else np.zeros(1)
    y0 = np.minimum(np.floor(ys).astype(np.int64), grid - 2)
    x0 = np.minimum(np.floor(xs).astype(np.int64), grid - 2)
    ty = (ys - y0)[:, None]
    tx = (xs - x0)[None, :]
    g00 = g[y0][:, x0]
    g01 = g[y0][:, x0 + 1]
    g10 = g[y0 + 1][:, x0]
    g11 = g[y0 + 1][:, x0 + 1]
    out = (1 - ty) * ((1 - tx) * g00 + tx * g01) + ty * ((1 - tx) * g10 + tx * g11)
    return _f32(out)


def rect_scene(seed: int, h: int = 256, w: int = 256, n_rect: int = 8,
               noise: float = 10.0, side_lo: int | None = None,
               side_hi: int | None = None) -> np.ndarray:
    """Uniform background, ``n_rect`` axis-aligned constant rectangles painted
    in order, plus i.i.d. N(0, noise^2); clipped to [0, 255]."""
    rng = _rng(seed)
    side_lo = 16 if side_lo is None else side_lo
    side_hi = 128 if side_hi is None else side_hi
    img = np.full((h, w), rng.uniform(0, 255), dtype=np.float64)
    for _ in range(n_rect):
        rh = int(min(h, rng.integers(side_lo, side_hi + 1)))
        rw = int(min(w, rng.integers(side_lo, side_hi + 1)))
        y0 = int(rng.integers(0, h - rh + 1))
        x0 = int(rng.integers(0, w - rw + 1))
        img[y0:y0 + rh, x0:x0 + rw] = rng.uniform(0, 255)
    img += rng.normal(0.0, noise, size=(h, w))
    return _f32(np.clip(img, 0, 255))


def gauss_field(seed: int, h: int = 1024, w: int = 1024, n_blob: int = 20,
                noise: float = 5.0) -> np.ndarray:
    """Sum of ``n_blob`` isotropic Gaussian blobs (amplitude U[0,255], centre
    uniform, width U[32,256] px), rescaled so its maximum is 255, plus
    N(0, noise^2); clipped to [0, 255]."""
    rng = _rng(seed)
    yy = np.arange(h, dtype=np.float64)[:, None]
    xx = np.arange(w, dtype=np.float64)[None, :]
    img = np.zeros((h, w))
    for _ in range(n_blob):
        a = rng.uniform(0, 255)
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        s = rng.uniform(32, 256)
        img += a * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
    img *= 255.0 / img.max()
    img += rng.normal(0.0, noise, size=(h, w))
    return _f32(np.clip(img, 0, 255))


def voronoi(seed: int, h: int = 4096, w: int = 4096, n_seed: int = 256,
            noise: float = 15.0) -> np.ndarray:
    """Nearest-seed Voronoi cells with levels U[0,255] plus N(0, noise^2),
    clipped to [0, 255]."""
    from scipy.spatial import cKDTree
    rng = _rng(seed)
    seeds = np.stack([rng.uniform(0, h, n_seed), rng.uniform(0, w, n_seed)], axis=1)
    levels = rng.uniform(0, 255, n_seed)
    tree = cKDTree(seeds)
    out = np.empty((h, w), dtype=np.float64)
    xs = np.arange(w, dtype=np.float64)
    step = max(1, (1 << 20) // max(w, 1))
    for y0 in range(0, h, step):
        ys = np.arange(y0, min(h, y0 + step), dtype=np.float64)
        pts = np.stack(np.meshgrid(ys, xs, indexing="ij"), axis=-1).reshape(-1, 2)
        _, idx = tree.query(pts)
        out[y0:y0 + len(ys)] = levels[idx].reshape(len(ys), w)
    out += rng.normal(0.0, noise, size=(h, w))
    return _f32(np.clip(out, 0, 255))


def block_constant(rng: np.random.Generator, h: int, w: int, lo: float, hi: float,
                   block: int = 16) -> np.ndarray:
    """A map that is constant U[lo, hi] on each block x block tile."""
    g = rng.uniform(lo, hi, size=((h + block - 1) // block, (w + block - 1) // block))
    return _f32(np.repeat(np.repeat(g, block, axis=0), block, axis=1)[:h, :w])


def texture_frames(seed: int, n_frames: int = 32, h: int = 1080, w: int = 1920,
                   n_region: int = 12, contrast: float = 40.0) -> np.ndarray:
    """``n_frames`` RGB frames as an (n_frames, 3, h, w) float32 array.

    Each frame has ``n_region`` Voronoi regions; each region has a per-channel
    base level U[40, 215] and one texture among checkerboard, horizontal,
    vertical and diagonal stripes, with a period of 4..16 px, a random phase
    and a square-wave amplitude of +-contrast/2.
    """
    from scipy.spatial import cKDTree
    rng = _rng(seed)
    out = np.empty((n_frames, 3, h, w), dtype=np.float32)
    yy = np.arange(h)[:, None]
    xx = np.arange(w)[None, :]
    grid = np.stack(np.meshgrid(np.arange(h, dtype=np.float64),
                                np.arange(w, dtype=np.float64), indexing="ij"),
                    axis=-1).reshape(-1, 2)
    for fi in range(n_frames):
        seeds = np.stack([rng.uniform(0, h, n_region), rng.uniform(0, w, n_region)], 1)
        _, idx = cKDTree(seeds).query(grid)
        idx = idx.reshape(h, w)
        frame = np.empty((3, h, w))
        for r in range(n_region):
            base = rng.uniform(40, 215, size=3)
            kind = int(rng.integers(0, 4))
            period = int(rng.integers(4, 17))
            phase = int(rng.integers(0, period))
            half = period // 2 if period > 1 else 1
            if kind == 0:
                wave = (((yy + phase) // half + (xx + phase) // half) % 2)
            elif kind == 1:
                wave = ((yy + phase) // half % 2) + 0 * xx
            elif kind == 2:
                wave = ((xx + phase) // half % 2) + 0 * yy
            else:
                wave = ((xx + yy + phase) // half % 2)
            sq = (2.0 * wave - 1.0) * (contrast / 2.0)
            m = idx == r
            for c in range(3):
                frame[c][m] = (base[c] + sq)[m]
        out[fi] = np.clip(frame, 0, 255)
    return _f32(out)


# ---------------------------------------------------------------------------
# Named workloads. Each returns a dict with the image ``f`` (float32 H x W),
# ``theta`` (None means theta = f), ``sigma`` (float32 H x W) and the filter
# parameters (kernel kind, sigma_s, R, N).
# ---------------------------------------------------------------------------

def _rects_256(seed: int = 1001):
    f = rect_scene(seed, 256, 256)
    rng = _rng(seed + 7)
    return dict(f=f, theta=None, sigma=smooth_field(rng, 256, 256, 10, 30),
                kernel="box", sigma_s=0.0, R=3, N=5)


def _sharpen_1024(seed: int = 1002):
    f = gauss_field(seed, 1024, 1024)
    rng = _rng(seed + 7)
    zeta = smooth_field(rng, 1024, 1024, -20, 20)
    sigma = smooth_field(rng, 1024, 1024, 5, 60)
    return dict(f=f, theta=_f32(f + zeta), sigma=sigma, kernel="gaussian",
                sigma_s=5.0, R=15, N=6)


def _voronoi(seed: int = 1003, size: int = 4096, R: int = 5, N: int = 5):
    f = voronoi(seed, size, size)
    rng = _rng(seed + 7)
    return dict(f=f, theta=None, sigma=block_constant(rng, size, size, 10, 40, 16),
                kernel="box", sigma_s=0.0, R=R, N=N)


WORKLOADS = {
    # 256 x 256 rectangles + noise 10, box R=3, N=5, sigma smooth in [10, 30]
    "rects256_box3_n5": _rects_256,
    # 1024 x 1024 smooth field + noise 5, Gaussian sigma_s=5 R=15, N=6,
    # theta = f + zeta (zeta smooth in [-20, 20]), sigma smooth in [5, 60]
    "sharpen1024_gauss15_n6": _sharpen_1024,
}
for _R in (5, 20):
    for _N in (5, 6, 7, 8):
        WORKLOADS[f"voronoi4096_box{_R}_n{_N}"] = (
            lambda seed=1003, size=4096, R=_R, N=_N: _voronoi(seed, size, R, N))


def _texture(seed: int = 1005, n_frames: int = 32, h: int = 1080, w: int = 1920):
    frames = texture_frames(seed, n_frames, h, w)
    return dict(frames=frames.reshape(n_frames * 3, h, w), kernel="box", sigma_s=0.0, R=8, N=6,
                passes=3, sigma_rule=dict(radius=4, scale=3.0, lo=5.0, hi=80.0))


# 32 RGB 1920 x 1080 frames of textured Voronoi regions, filtered channel by
# channel (96 planes), box R=8, N=6, 3 passes, sigma = clip(3 * std_9x9, 5, 80)
WORKLOADS["texture1080_box8_n6"] = _texture


def _classical_512(seed: int = 1006):
    f = rect_scene(seed, 512, 512)
    return dict(f=f, theta=None, sigma=np.full((512, 512), 40.0, np.float32), kernel="box",
                sigma_s=0.0, R=5, N=5)


# classical filter (theta = f, sigma = sigma_0 = 40 everywhere) on a 512 x 512
# rectangle scene: the setting of the paper's timing and PSNR sweeps over
# rho and N (Sec. III-B); R and N here are the defaults, the sweep varies them
WORKLOADS["classical512_box5_n5"] = _classical_512


def workload(name: str, **kw):
    """Return the named workload dict (see ``WORKLOADS``)."""
    return WORKLOADS[name](**kw)


def serving_requests(seed: int, n: int, rate_per_s: float):
    """A Poisson stream of filter requests of mixed sizes and parameters.

    Each request: short side U{256, 512, 1024, 2048}, aspect 1:1 or 4:3,
    R in {3, 5, 10, 20}, N in {5, 6, 8}, box or Gaussian (sigma_s = R/3),
    a rectangle scene image (rectangle sides U{H/16..H/2}), theta = f and a
    smooth sigma map in [10, 30]. Returns a list of dicts with the arrival
    time (seconds from start) and the arrays.
    """
    rng = _rng(seed)
    t = 0.0
    reqs = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        s = int(rng.choice([256, 512, 1024, 2048]))
        h, w = (s, s) if rng.random() < 0.5 else (s, int(round(4 * s / 3)))
        R = int(rng.choice([3, 5, 10, 20]))
        N = int(rng.choice([5, 6, 8]))
        gauss = bool(rng.random() < 0.5)
        img_seed = int(rng.integers(0, 2**31 - 1))
        f = rect_scene(img_seed, h, w, side_lo=max(1, h // 16), side_hi=max(2, h // 2))
        sigma = smooth_field(_rng(img_seed + 1), h, w, 10, 30)
        reqs.append(dict(t=t, f=f, theta=None, sigma=sigma,
                         kernel="gaussian" if gauss else "box",
                         sigma_s=R / 3.0 if gauss else 0.0, R=R, N=N, id=i))
    return reqs
