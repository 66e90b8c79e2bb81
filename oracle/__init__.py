"""CPU oracle for the fast adaptive bilateral filter (Gavaskar & Chaudhury,
"Fast Adaptive Bilateral Filtering", arXiv:1811.02308).

TEST INFRASTRUCTURE ONLY. Nothing in the GPU library imports, calls or links
this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code with the HIP
path: the two meet only at the seeded input generators of ``synth/``.

Contents
--------
``hilbert``    exact integer tables: the Hilbert-matrix inverse of eq. (inv)
               (Sec. II-B, Theorem) and the shifted-Legendre coefficients.
``spatial``    clamp-to-edge windows, window min/max (eq. bounds), spatial
               weights (eq. sp_kernel / box), moments (Prop. 2 and the
               stretched-histogram moments of eq. hist_moments_new).
``integrals``  the range integrals I_k of eq. (integrals): the paper's
               closed forms and recursion (eqs. I_0, I_1, F_forward) and an
               accurate composite Gauss-Legendre evaluation of the same
               definite integrals.
``fast``       Algorithm 1 end to end, two routes (see ``fast.fast_abf``).
``brute``      the brute-force adaptive bilateral filter of eqs.
               (BF_adaptive1), (BF_adaptive2).
``mpref``      Algorithm 1 in 60-digit mpmath arithmetic for tiny images,
               used to pin the FP64 routes.
``uniform``    the uniform-prior comparison variant of Sec. III-B (the
               N = 0 estimator on [f, 2 fbar - f]).

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against a closed form, an exact identity, brute force on tiny inputs or a
high-precision evaluation. The paper's printed PSNR values (Table 1, Fig. 3)
need its test image, which is not available, so those numbers are
**parity unpinned**; only their trend is checked.
"""
from . import hilbert, spatial, integrals, fast, brute, uniform  # noqa: F401
from .fast import fast_abf, fast_abf_literal  # noqa: F401
from .brute import brute_abf  # noqa: F401
from .spatial import window_minmax  # noqa: F401
from .uniform import uniform_prior_abf  # noqa: F401
