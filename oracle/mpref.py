"""Algorithm 1 exactly as printed, in 60-digit mpmath arithmetic, for tiny
images (pins the FP64 routes of ``fast``). Steps, in the paper's order:

  1. alpha_i, beta_i: window min/max (eq. bounds);
  2. A^-1 from eq. (inv) (exact integers);
  3. gamma_k(i) = sum_j omega(j) f(i-j)^k (Prop. 2, its definition);
  4. mu from m by the binomial shift of Prop. 3;
  5. c = A^-1 mu;
  6. t0, lambda (eq. sub);
  7. I_0 by eq. (I_0) (two erf), I_1 by eq. (I_1);
  8. I_2..I_{N+1} by eq. (F_forward);
  9. T1, T2 and g^ = alpha + (beta - alpha) T1/T2 (eq. BFfinal).

Clamp-to-edge windows and normalised weights as in ``spatial``. With 60
digits the forward recursion's loss (at most a factor of about
(N+1)!/(2 lambda)^(N+1)) leaves far more than FP64 accuracy for the
lambda >= 1e-4 used in the pins. No post-rules are applied.
"""
from __future__ import annotations

from math import comb

import mpmath as mp
import numpy as np

from .hilbert import hilbert_inverse


def _weights(kind, R, sigma_s):
    js = range(-R, R + 1)
    if kind == "box":
        w1 = [mp.mpf(1) for _ in js]
    else:
        s = mp.mpf(R) / 3 if (sigma_s is None or sigma_s <= 0) else mp.mpf(sigma_s)
        w1 = [mp.e ** (-(mp.mpf(j) ** 2) / (2 * s * s)) for j in js]
    tot = sum(w1)
    w1 = [x / tot for x in w1]
    return [[a * b for b in w1] for a in w1]


def fast_abf_mp(f, theta=None, sigma=None, kernel="box", R=1, N=2, sigma_s=None,
                dps: int = 60):
    """Returns an (H, W) float64 array of g^ computed at ``dps`` digits."""
    f = np.asarray(f, dtype=np.float32) + np.float32(0)
    H, W = f.shape
    th = f if theta is None else np.asarray(theta, dtype=np.float32) + np.float32(0)
    sg = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (H, W))
    out = np.empty((H, W))
    with mp.workdps(dps):
        w = _weights(kernel, R, sigma_s)
        Ainv = hilbert_inverse(N)
        for i in range(H):
            for j in range(W):
                win = [[mp.mpf(float(f[min(H - 1, max(0, i + dy)), min(W - 1, max(0, j + dx))]))
                        for dx in range(-R, R + 1)] for dy in range(-R, R + 1)]
                flat = [v for row in win for v in row]
                a, b = min(flat), max(flat)
                if a == b:
                    out[i, j] = float(f[i, j])
                    continue
                m = [sum(w[p][q] * win[p][q] ** k for p in range(2 * R + 1)
                         for q in range(2 * R + 1)) for k in range(N + 1)]
                d = b - a
                mu = [sum(comb(k, r) * (-a) ** (k - r) * m[r] for r in range(k + 1)) / d ** k
                      for k in range(N + 1)]
                c = [sum(Ainv[p][q] * mu[q] for q in range(N + 1)) for p in range(N + 1)]
                t0 = (mp.mpf(float(th[i, j])) - a) / d
                s = mp.mpf(float(sg[i, j]))
                if mp.isinf(s):
                    # lambda = 0: psi = 1 and I_k = 1/(k+1) (the recursion's
                    # limit); the integrals are then elementary.
                    I = [mp.mpf(1) / (k + 1) for k in range(N + 2)]
                else:
                    lam = d * d / (2 * s * s)
                    sl = mp.sqrt(lam)
                    I0 = mp.sqrt(mp.pi / lam) / 2 * (mp.erf(sl * (1 - t0)) - mp.erf(-sl * t0))
                    e0, e1 = mp.e ** (-lam * t0 ** 2), mp.e ** (-lam * (1 - t0) ** 2)
                    I = [I0, t0 * I0 + (e0 - e1) / (2 * lam)]
                    for k in range(2, N + 2):
                        I.append(t0 * I[k - 1] + (k - 1) / (2 * lam) * I[k - 2] - e1 / (2 * lam))
                T1 = sum(c[k] * I[k + 1] for k in range(N + 1))
                T2 = sum(c[k] * I[k] for k in range(N + 1))
                out[i, j] = float(a + d * T1 / T2)
    return out
