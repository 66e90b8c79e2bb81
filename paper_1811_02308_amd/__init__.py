"""MI355X (gfx950) fast adaptive bilateral filter: thin Python binding.

Every function here marshals arguments for one C-ABI entry point of
``libabf.so`` (declared in ``include/abf.h``) and runs nothing else: all
filtering happens in the library's HIP kernels. PyTorch provides device
memory and the current HIP stream. If the library is not built, calls
raise ``RuntimeError``; there is no fallback path.

Functions mirror the C names: ``fast`` (abf_fast), ``bruteforce``
(abf_bruteforce), ``minmax`` (abf_minmax), ``moment_stack``
(abf_moment_stack), ``range_from_stack`` (abf_range), ``fast_batched``
(abf_fast_batched).
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "lib", "library_path", "fast", "bruteforce", "minmax", "moment_stack",
    "range_from_stack", "fast_batched", "minmax_into_stack", "stack_moments",
    "fast_strided", "sigma_local_std", "moments_range", "uniform_prior", "range_uniform_from_stack",
    "sharpen_maps", "mrtv_sigma", "grey", "texture_filter_paper", "workspace_bytes", "stack_bytes",
    "stack_planes", "stack_kernel", "Request", "KERNELS", "PRECISIONS", "ABFError",
]

KERNELS = {"box": 0, "gaussian": 1, "recursive": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
FLAG_CLAMP = 1
FLAG_KEEP_STACK = 2
N_MAX = 8
RHO_MAX = 96

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class ABFError(RuntimeError):
    pass


def library_path() -> str:
    return os.path.join(_HERE, "libabf.so")


class Request(ctypes.Structure):
    _fields_ = [
        ("img", ctypes.c_void_p), ("theta", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
        ("h", ctypes.c_int), ("w", ctypes.c_int), ("pitch", ctypes.c_longlong),
        ("kernel_kind", ctypes.c_int), ("sigma_s", ctypes.c_double), ("rho", ctypes.c_int),
        ("N", ctypes.c_int), ("out", ctypes.c_void_p), ("out_pitch", ctypes.c_longlong),
    ]


def lib():
    """Load libabf.so (built in-tree by ``paper_1811_02308_amd.build``)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_1811_02308_amd.build` (no fallback exists)")
    L = ctypes.CDLL(path)
    vp, i, ll, d, sz, u = (ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_double,
                           ctypes.c_size_t, ctypes.c_uint)
    sig = {
        "abf_status_string": ([i], ctypes.c_char_p),
        "abf_version": ([], i),
        "abf_stack_pitch": ([i], ll),
        "abf_stack_bytes": ([i, i, i, i], sz),
        "abf_stack_plane_offset": ([i, i, i, i, i], sz),
        "abf_scratch_bytes": ([i, i, i], sz),
        "abf_workspace_bytes": ([i, i, i, i, i], sz),
        "abf_kernel_scratch_bytes": ([i, i, i, i, i], sz),
        "abf_kernel_workspace_bytes": ([i, i, i, i, i, i], sz),
        "abf_minmax": ([vp, i, i, ll, i, vp, vp, ll, vp, sz, vp], i),
        "abf_moment_stack": ([vp, i, i, ll, i, d, i, i, i, vp, sz, vp, sz, vp], i),
        "abf_stack_single_pass": ([i, i, i, i, i], i),
        "abf_fast_noalloc": ([vp, vp, vp, i, i, ll, i, d, i, i, i, u, vp, ll, vp], i),
        "abf_stack_kernel": ([i, i, i, i, i, i], i),
        "abf_fast_fused": ([i, i, i, i, i, i], i),
        "abf_stack_moments": ([vp, i, i, ll, i, d, i, i, i, vp, sz, vp], i),
        "abf_range": ([vp, sz, vp, vp, vp, i, i, ll, i, i, u, vp, ll, vp], i),
        "abf_moments_range": ([vp, vp, vp, i, i, ll, i, d, i, i, i, u, vp, sz, vp, ll, vp], i),
        "abf_uniform_prior": ([vp, vp, vp, i, i, ll, i, d, i, i, u, vp, ll, vp, sz, vp], i),
        "abf_range_uniform": ([vp, sz, vp, vp, vp, i, i, ll, i, i, u, vp, ll, vp], i),
        "abf_fast": ([vp, vp, vp, i, i, ll, i, d, i, i, i, u, vp, ll, vp, sz, vp], i),
        "abf_bruteforce": ([vp, vp, vp, i, i, ll, i, d, i, i, vp, ll, vp], i),
        "abf_batched_workspace_bytes": ([ctypes.POINTER(Request), i, i], sz),
        "abf_fast_batched": ([ctypes.POINTER(Request), i, i, u, vp, sz, vp], i),
        "abf_strided_workspace_bytes": ([i, i, i, i, i, i], sz),
        "abf_fast_strided": ([vp, vp, vp, i, i, i, ll, ll, i, d, i, i, i, u, vp, ll, ll, vp, sz, vp], i),
        "abf_sigma_local_std": ([vp, i, i, i, ll, ll, i, d, d, d, vp, ll, ll, vp], i),
        "abf_sharpen_maps": ([vp, i, i, i, ll, ll, i, d, d, d, d, vp, vp, ll, ll, vp], i),
        "abf_mrtv_sigma": ([vp, i, i, i, ll, ll, i, d, d, d, d, vp, ll, ll, vp], i),
        "abf_grey": ([vp, i, i, i, ll, ll, ll, vp, ll, ll, vp], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = L
    return L


def _check(status: int, what: str):
    if status != 0:
        msg = lib().abf_status_string(status).decode()
        raise ABFError(f"{what} failed: {msg} (status {status})")


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _on(stream):
    """Context in which the binding allocates outputs and temporaries: the
    stream the call's kernels run on. Torch's caching allocator ties a block
    to the stream current at allocation, and only reuses it for work ordered
    after that stream's pending kernels; a workspace dropped at return while
    the kernels still run on another stream could otherwise be handed out
    again on the current stream and overwritten mid-flight."""
    import contextlib
    if stream is None:
        return contextlib.nullcontext()
    return _torch().cuda.stream(stream)


def _plane(t, name):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ABFError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or t.dim() != 2 or t.stride(1) != 1:
        raise ABFError(f"{name} must be a 2-D float32 tensor with unit column stride")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _prec(p):
    if p not in PRECISIONS:
        raise ABFError(f"precision must be one of {list(PRECISIONS)}")
    return PRECISIONS[p]


def _kind(k):
    if k not in KERNELS:
        raise ABFError(f"kernel must be one of {list(KERNELS)}")
    return KERNELS[k]


def _common_pitch(img, *others):
    p = img.stride(0)
    for o in others:
        if o is not None and (o.shape != img.shape or o.stride(0) != p):
            raise ABFError("theta/sigma must have the image's shape and row pitch")
    return p


def _alloc_bytes(nbytes, device, stream=None):
    torch = _torch()
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    with _on(stream):
        return torch.empty(max(1, int(nbytes)), dtype=torch.uint8, device=device)


def _empty(shape, dtype, device, stream=None):
    """torch.empty on the stream the call's kernels run on (see _on)."""
    torch = _torch()
    with _on(stream):
        return torch.empty(shape, dtype=dtype, device=device)


def _out_dtype(p):
    torch = _torch()
    return torch.float64 if p == 0 else torch.float32


def workspace_bytes(h, w, rho, N, precision="mixed", kernel="box"):
    return int(lib().abf_kernel_workspace_bytes(h, w, rho, N, _prec(precision), _kind(kernel)))


def stack_bytes(h, w, N, precision="mixed"):
    return int(lib().abf_stack_bytes(h, w, N, _prec(precision)))


def fast(img, sigma, theta=None, kernel="box", rho=3, N=5, sigma_s=0.0, precision="mixed",
         clamp=True, out=None, workspace=None, stream=None):
    """abf_fast: Algorithm 1 on one image. Returns ``out`` (float32 for
    'mixed', float64 for 'fp64')."""
    torch = _torch()
    img, sigma, theta = _plane(img, "img"), _plane(sigma, "sigma"), _plane(theta, "theta")
    h, w = img.shape
    pitch = _common_pitch(img, sigma, theta)
    p = _prec(precision)
    if out is None:
        out = _empty((h, w), _out_dtype(p), img.device, stream)
    need = lib().abf_kernel_workspace_bytes(h, w, rho, N, p, _kind(kernel))
    if workspace is None:
        workspace = _alloc_bytes(need, img.device, stream)
    st = lib().abf_fast(_ptr(img), _ptr(theta), _ptr(sigma), h, w, pitch, _kind(kernel),
                        float(sigma_s), int(rho), int(N), p, FLAG_CLAMP if clamp else 0,
                        _ptr(out), out.stride(0), _ptr(workspace), workspace.numel(), _stream(stream))
    _check(st, "abf_fast")
    return out


def bruteforce(img, sigma, theta=None, kernel="box", rho=3, sigma_s=0.0, precision="fp64",
               out=None, stream=None):
    """abf_bruteforce: eqs. (BF_adaptive1), (BF_adaptive2) directly."""
    torch = _torch()
    img, sigma, theta = _plane(img, "img"), _plane(sigma, "sigma"), _plane(theta, "theta")
    h, w = img.shape
    pitch = _common_pitch(img, sigma, theta)
    p = _prec(precision)
    if out is None:
        out = _empty((h, w), _out_dtype(p), img.device, stream)
    st = lib().abf_bruteforce(_ptr(img), _ptr(theta), _ptr(sigma), h, w, pitch, _kind(kernel),
                              float(sigma_s), int(rho), p, _ptr(out), out.stride(0), _stream(stream))
    _check(st, "abf_bruteforce")
    return out


def minmax(img, rho, stream=None):
    """abf_minmax: window bounds (alpha, beta) as two float32 planes."""
    torch = _torch()
    img = _plane(img, "img")
    h, w = img.shape
    a = _empty((h, w), torch.float32, img.device, stream)
    b = _empty((h, w), torch.float32, img.device, stream)
    ws = _alloc_bytes(lib().abf_scratch_bytes(h, w, rho), img.device, stream)
    st = lib().abf_minmax(_ptr(img), h, w, img.stride(0), int(rho), _ptr(a), _ptr(b), a.stride(0),
                          _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "abf_minmax")
    return a, b


def moment_stack(img, kernel="box", rho=3, N=5, sigma_s=0.0, precision="mixed", stack=None,
                 workspace=None, stream=None):
    """abf_moment_stack: returns the raw stack buffer (uint8 tensor)."""
    img = _plane(img, "img")
    h, w = img.shape
    p = _prec(precision)
    if stack is None:
        stack = _alloc_bytes(lib().abf_stack_bytes(h, w, N, p), img.device, stream)
    if workspace is None:
        workspace = _alloc_bytes(lib().abf_kernel_scratch_bytes(h, w, rho, N, _kind(kernel)),
                                 img.device, stream)
    st = lib().abf_moment_stack(_ptr(img), h, w, img.stride(0), _kind(kernel), float(sigma_s),
                                int(rho), int(N), p, _ptr(stack), stack.numel(), _ptr(workspace),
                                workspace.numel(), _stream(stream))
    _check(st, "abf_moment_stack")
    return stack


def stack_single_pass(h, w, kernel="box", rho=3, N=5):
    """abf_stack_single_pass: True if moment_stack / fast build the stack of
    an h x w image in one kernel launch (bounds taken by the moment kernel)."""
    return bool(lib().abf_stack_single_pass(int(h), int(w), _kind(kernel), int(rho), int(N)))


STACK_KERNELS = {0: "bounds_only", 1: "box", 2: "tile", 3: "tile_wide", 4: "mfma"}


def stack_kernel(h, w, kernel="box", rho=3, N=5, precision="mixed"):
    """abf_stack_kernel: name of the moment kernel that builds the stack of an
    h x w image with these parameters ('box', 'tile', 'tile_wide', 'mfma',
    'bounds_only' for N = 0)."""
    k = int(lib().abf_stack_kernel(int(h), int(w), _kind(kernel), int(rho), int(N), _prec(precision)))
    if k < 0:
        raise ABFError("abf_stack_kernel: invalid arguments")
    return STACK_KERNELS[k]


def fast_fused(h, w, kernel="box", rho=3, N=5, precision="mixed"):
    """abf_fast_fused: whether abf_fast runs the moment and range stages fused
    in one kernel for these arguments (else the stack path)."""
    return bool(lib().abf_fast_fused(int(h), int(w), _kind(kernel), int(rho), int(N), _prec(precision)))


def minmax_into_stack(img, stack, rho, N, precision="mixed", workspace=None, stream=None):
    """abf_minmax writing alpha/beta into planes 0 and 1 of a stack buffer."""
    img = _plane(img, "img")
    h, w = img.shape
    p = _prec(precision)
    L = lib()
    if stack.numel() < L.abf_stack_bytes(h, w, N, p):
        raise ABFError("stack buffer too small")
    if workspace is None:
        workspace = _alloc_bytes(L.abf_scratch_bytes(h, w, rho), img.device, stream)
    a = ctypes.c_void_p(stack.data_ptr())
    b = ctypes.c_void_p(stack.data_ptr() + int(L.abf_stack_plane_offset(h, w, N, p, 1)))
    st = L.abf_minmax(_ptr(img), h, w, img.stride(0), int(rho), a, b, L.abf_stack_pitch(w),
                      _ptr(workspace), workspace.numel(), _stream(stream))
    _check(st, "abf_minmax")
    return stack


def stack_moments(img, stack, kernel="box", rho=3, N=5, sigma_s=0.0, precision="mixed",
                  stream=None):
    """abf_stack_moments: moment planes of a stack whose bounds are present."""
    img = _plane(img, "img")
    h, w = img.shape
    st = lib().abf_stack_moments(_ptr(img), h, w, img.stride(0), _kind(kernel), float(sigma_s),
                                 int(rho), int(N), _prec(precision), _ptr(stack), stack.numel(),
                                 _stream(stream))
    _check(st, "abf_stack_moments")
    return stack


def stack_planes(stack, h, w, N, precision="mixed"):
    """Views (alpha, beta, [a~_1..a~_N]) into a stack buffer, each (h, w)."""
    torch = _torch()
    p = _prec(precision)
    L = lib()
    P = int(L.abf_stack_pitch(w))

    def view(plane, dtype):
        off = int(L.abf_stack_plane_offset(h, w, N, p, plane))
        esz = torch.tensor([], dtype=dtype).element_size()
        flat = stack[off: off + P * h * esz].view(dtype)
        return flat.view(h, P)[:, :w]

    mdt = torch.float64 if p == 0 else torch.float32
    return view(0, torch.float32), view(1, torch.float32), [view(2 + k, mdt) for k in range(N)]


def range_from_stack(stack, sigma, img=None, theta=None, N=5, precision="mixed", clamp=True,
                     out=None, stream=None):
    """abf_range: the range stage from a moment stack built for the same image."""
    torch = _torch()
    sigma, img, theta = _plane(sigma, "sigma"), _plane(img, "img"), _plane(theta, "theta")
    h, w = sigma.shape
    ref = theta if theta is not None else img
    if ref is None:
        raise ABFError("either theta or img is required")
    pitch = _common_pitch(sigma, img, theta)
    p = _prec(precision)
    if out is None:
        out = _empty((h, w), _out_dtype(p), sigma.device, stream)
    st = lib().abf_range(_ptr(stack), stack.numel(), _ptr(img), _ptr(theta), _ptr(sigma), h, w,
                         pitch, int(N), p, FLAG_CLAMP if clamp else 0, _ptr(out), out.stride(0),
                         _stream(stream))
    _check(st, "abf_range")
    return out


def moments_range(img, stack, sigma, theta=None, kernel="box", rho=3, N=5, sigma_s=0.0,
                  precision="mixed", clamp=True, keep_stack=False, out=None, stream=None):
    """abf_moments_range: moments and range stage in one pass from a stack
    whose bound planes are present (``minmax_into_stack``); with
    ``keep_stack`` the moment planes are stored too."""
    torch = _torch()
    img, sigma, theta = _plane(img, "img"), _plane(sigma, "sigma"), _plane(theta, "theta")
    h, w = img.shape
    pitch = _common_pitch(img, sigma, theta)
    p = _prec(precision)
    if out is None:
        out = _empty((h, w), _out_dtype(p), img.device, stream)
    flags = (FLAG_CLAMP if clamp else 0) | (FLAG_KEEP_STACK if keep_stack else 0)
    st = lib().abf_moments_range(_ptr(img), _ptr(theta), _ptr(sigma), h, w, pitch, _kind(kernel),
                                 float(sigma_s), int(rho), int(N), p, flags, _ptr(stack),
                                 stack.numel(), _ptr(out), out.stride(0), _stream(stream))
    _check(st, "abf_moments_range")
    return out


def uniform_prior(img, sigma, theta=None, kernel="box", rho=3, sigma_s=0.0, precision="mixed",
                  clamp=True, out=None, workspace=None, stream=None):
    """abf_uniform_prior: the uniform-prior comparison variant (N = 0 on
    [f, 2 fbar - f])."""
    torch = _torch()
    img, sigma, theta = _plane(img, "img"), _plane(sigma, "sigma"), _plane(theta, "theta")
    h, w = img.shape
    pitch = _common_pitch(img, sigma, theta)
    p = _prec(precision)
    L = lib()
    if out is None:
        out = _empty((h, w), _out_dtype(p), img.device, stream)
    if workspace is None:
        workspace = _alloc_bytes(L.abf_workspace_bytes(h, w, int(rho), 1, p), img.device, stream)
    st = L.abf_uniform_prior(_ptr(img), _ptr(theta), _ptr(sigma), h, w, pitch, _kind(kernel),
                             float(sigma_s), int(rho), p, FLAG_CLAMP if clamp else 0, _ptr(out),
                             out.stride(0), _ptr(workspace), workspace.numel(), _stream(stream))
    _check(st, "abf_uniform_prior")
    return out


def range_uniform_from_stack(stack, img, sigma, theta=None, N=5, precision="mixed", clamp=True,
                             out=None, stream=None):
    """abf_range_uniform: the uniform-prior variant from a resident stack."""
    torch = _torch()
    img, sigma, theta = _plane(img, "img"), _plane(sigma, "sigma"), _plane(theta, "theta")
    h, w = img.shape
    pitch = _common_pitch(img, sigma, theta)
    p = _prec(precision)
    if out is None:
        out = _empty((h, w), _out_dtype(p), img.device, stream)
    st = lib().abf_range_uniform(_ptr(stack), stack.numel(), _ptr(img), _ptr(theta), _ptr(sigma),
                                 h, w, pitch, int(N), p, FLAG_CLAMP if clamp else 0, _ptr(out),
                                 out.stride(0), _stream(stream))
    _check(st, "abf_range_uniform")
    return out


def fast_batched(items, precision="mixed", clamp=True, workspace=None, stream=None):
    """abf_fast_batched. ``items``: list of dicts with keys img, sigma, theta
    (optional), kernel, rho, N, sigma_s (optional), out (optional).
    Returns the list of outputs."""
    torch = _torch()
    p = _prec(precision)
    reqs = (Request * max(1, len(items)))()
    outs = []
    for i, it in enumerate(items):
        img, sg, th = _plane(it["img"], "img"), _plane(it["sigma"], "sigma"), _plane(it.get("theta"), "theta")
        h, w = img.shape
        pitch = _common_pitch(img, sg, th)
        out = it.get("out")
        if out is None:
            out = _empty((h, w), _out_dtype(p), img.device, stream)
        outs.append(out)
        reqs[i] = Request(img.data_ptr(), th.data_ptr() if th is not None else None, sg.data_ptr(),
                          h, w, pitch, _kind(it.get("kernel", "box")), float(it.get("sigma_s", 0.0)),
                          int(it["rho"]), int(it["N"]), out.data_ptr(), out.stride(0))
    need = lib().abf_batched_workspace_bytes(reqs, len(items), p)
    if workspace is None and items:
        workspace = _alloc_bytes(need, items[0]["img"].device, stream)
    st = lib().abf_fast_batched(reqs, len(items), p, FLAG_CLAMP if clamp else 0,
                                _ptr(workspace) if workspace is not None else None,
                                workspace.numel() if workspace is not None else 0, _stream(stream))
    _check(st, "abf_fast_batched")
    return outs


def _batch3(t, name):
    """A (n, h, w) float32 CUDA tensor with unit column stride -> (n, h, w, pitch, stride)."""
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
        raise ABFError(f"{name} must be a float32 CUDA tensor")
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3 or t.stride(2) != 1:
        raise ABFError(f"{name} must be (n, h, w) with unit column stride")
    return t


def fast_strided(img, sigma, theta=None, kernel="box", rho=3, N=5, sigma_s=0.0,
                 precision="mixed", clamp=True, out=None, workspace=None, stream=None):
    """abf_fast_strided: the fast filter on a stack of n images (n, h, w) of
    one shape and parameter set, one launch per stage for the whole batch."""
    torch = _torch()
    img, sigma, theta = _batch3(img, "img"), _batch3(sigma, "sigma"), _batch3(theta, "theta")
    n, h, w = img.shape
    for o in (sigma, theta):
        if o is not None and (o.shape != img.shape or o.stride() != img.stride()):
            raise ABFError("theta/sigma must have the image batch's shape and strides")
    p = _prec(precision)
    if out is None:
        out = _empty((n, h, w), _out_dtype(p), img.device, stream)
    need = lib().abf_strided_workspace_bytes(n, h, w, rho, N, p)
    if workspace is None:
        workspace = _alloc_bytes(need, img.device, stream)
    st = lib().abf_fast_strided(_ptr(img), _ptr(theta), _ptr(sigma), n, h, w, img.stride(1),
                                img.stride(0), _kind(kernel), float(sigma_s), int(rho), int(N), p,
                                FLAG_CLAMP if clamp else 0, _ptr(out), out.stride(1), out.stride(0),
                                _ptr(workspace), workspace.numel(), _stream(stream))
    _check(st, "abf_fast_strided")
    return out


def sigma_local_std(img, radius=4, scale=3.0, lo=5.0, hi=80.0, out=None, stream=None):
    """abf_sigma_local_std: sigma = clamp(scale * local std over (2r+1)^2, lo, hi)."""
    torch = _torch()
    img = _batch3(img, "img")
    n, h, w = img.shape
    if out is None:
        out = _empty((n, h, w), torch.float32, img.device, stream)
    st = lib().abf_sigma_local_std(_ptr(img), n, h, w, img.stride(1), img.stride(0), int(radius),
                                   float(scale), float(lo), float(hi), _ptr(out), out.stride(1),
                                   out.stride(0), _stream(stream))
    _check(st, "abf_sigma_local_std")
    return out


def texture_filter(frames, passes=3, rho=8, N=6, radius=4, scale=3.0, lo=5.0, hi=80.0,
                   precision="mixed", stream=None):
    """Iterated adaptive filtering of a batch of planar channel-images
    (n, h, w) as in the texture-removal use (Sec. IV-C: the filter applied
    repeatedly, channel by channel): each pass recomputes sigma from the
    current input's local contrast (abf_sigma_local_std) and filters the
    whole batch with one abf_fast_strided call (theta = f, box kernel).
    Returns the output of the last pass (float32 for 'mixed'). Every torch
    operation in between runs on ``stream`` as well."""
    with _on(stream):
        return _texture_filter(frames, passes, rho, N, radius, scale, lo, hi, precision, stream)


def _texture_filter(frames, passes, rho, N, radius, scale, lo, hi, precision, stream):
    torch = _torch()
    x = _batch3(frames, "frames")
    n, h, w = x.shape
    p = _prec(precision)
    ws = _alloc_bytes(lib().abf_strided_workspace_bytes(n, h, w, rho, N, p), x.device, stream)
    sig = _empty(x.shape, torch.float32, x.device, stream)
    outs = [_empty((n, h, w), _out_dtype(p), x.device, stream) for _ in range(2)]
    cur = x
    for i in range(passes):
        sigma_local_std(cur if cur.dtype == torch.float32 else cur.float(), radius, scale, lo, hi,
                        out=sig, stream=stream)
        src = cur if cur.dtype == torch.float32 else cur.float()
        fast_strided(src, sig, kernel="box", rho=rho, N=N, precision=precision,
                     out=outs[i % 2], workspace=ws, stream=stream)
        cur = outs[i % 2]
    return cur


# ---------------------------------------------------------------- application maps (Sec. IV)
def _out3(t, n, h, w, like, stream=None):
    torch = _torch()
    if t is None:
        return _empty((n, h, w), torch.float32, like.device, stream)
    t = _batch3(t, "out")
    if tuple(t.shape) != (n, h, w):
        raise ABFError("output maps must have the input batch's shape")
    return t


def sharpen_maps(img, radius=5, log_sigma=1.0, lo=5.0, hi=40.0, v_ref=20.0, theta=None,
                 sigma=None, stream=None):
    """abf_sharpen_maps: (theta, sigma) of the sharpening application for a
    batch (n, h, w) or one image: theta = 2 f - fbar, sigma = affine(|LoG f|)."""
    x = _batch3(img, "img")
    n, h, w = x.shape
    theta = _out3(theta, n, h, w, x, stream)
    sigma = _out3(sigma, n, h, w, x, stream)
    if theta.stride() != sigma.stride():
        raise ABFError("theta and sigma outputs must share strides")
    st = lib().abf_sharpen_maps(_ptr(x), n, h, w, x.stride(1), x.stride(0), int(radius),
                                float(log_sigma), float(lo), float(hi), float(v_ref), _ptr(theta),
                                _ptr(sigma), theta.stride(1), theta.stride(0), _stream(stream))
    _check(st, "abf_sharpen_maps")
    return theta, sigma


def mrtv_sigma(img, radius=2, eps=1e-3, lo=5.0, hi=80.0, v_ref=20.0, out=None, stream=None):
    """abf_mrtv_sigma: sigma = affine(mRTV) for a batch (n, h, w) or one image."""
    x = _batch3(img, "img")
    n, h, w = x.shape
    out = _out3(out, n, h, w, x, stream)
    st = lib().abf_mrtv_sigma(_ptr(x), n, h, w, x.stride(1), x.stride(0), int(radius), float(eps),
                              float(lo), float(hi), float(v_ref), _ptr(out), out.stride(1),
                              out.stride(0), _stream(stream))
    _check(st, "abf_mrtv_sigma")
    return out


def grey(rgb, out=None, stream=None):
    """abf_grey: 0.299 R + 0.587 G + 0.114 B of planar colour images
    (n, 3, h, w) or (3, h, w); returns (n, h, w)."""
    torch = _torch()
    if not isinstance(rgb, torch.Tensor) or rgb.device.type != "cuda" or rgb.dtype != torch.float32:
        raise ABFError("rgb must be a float32 CUDA tensor")
    if rgb.dim() == 3:
        rgb = rgb.unsqueeze(0)
    if rgb.dim() != 4 or rgb.shape[1] != 3 or rgb.stride(3) != 1:
        raise ABFError("rgb must be (n, 3, h, w) with unit column stride")
    n, _, h, w = rgb.shape
    out = _out3(out, n, h, w, rgb, stream)
    st = lib().abf_grey(_ptr(rgb), n, h, w, rgb.stride(2), rgb.stride(1), rgb.stride(0), _ptr(out),
                        out.stride(1), out.stride(0), _stream(stream))
    _check(st, "abf_grey")
    return out


def texture_filter_paper(frames, rho=8, N=6, mrtv_radius=2, eps=1e-3, lo=5.0, hi=80.0,
                         v_ref=20.0, shrink=0.8, log_sigma=1.0, sharpen_lo=5.0, sharpen_hi=40.0,
                         sharpen_v_ref=20.0, precision="mixed", stream=None, keep=False):
    """The texture-removal procedure of Sec. IV-C on planar colour frames
    (n, 3, h, w), every step in the library's kernels:
      sigma_1 = affine(mRTV) of the grey input (abf_grey, abf_mrtv_sigma);
      pass 1: the fast filter, theta = f, sigma_1, channel by channel;
      pass 2: the same on pass 1's output with sigma_1 scaled by `shrink`;
      pass 3: sharpening (Sec. IV-A) of pass 2's output: theta = f + zeta per
              channel, sigma from |LoG| of its grey image (abf_sharpen_maps).
    The maps of all three channels of a frame are the grey image's (written
    once per channel plane). Returns pass 3's output (n, 3, h, w), or with
    ``keep`` a dict of every intermediate. Every torch operation in between
    (layout copies, dtype conversions) runs on ``stream`` as well."""
    with _on(stream):
        return _texture_filter_paper(frames, rho, N, mrtv_radius, eps, lo, hi, v_ref, shrink,
                                     log_sigma, sharpen_lo, sharpen_hi, sharpen_v_ref, precision,
                                     stream, keep)


def _texture_filter_paper(frames, rho, N, mrtv_radius, eps, lo, hi, v_ref, shrink, log_sigma,
                          sharpen_lo, sharpen_hi, sharpen_v_ref, precision, stream, keep):
    torch = _torch()
    if frames.dim() != 4 or frames.shape[1] != 3:
        raise ABFError("frames must be (n, 3, h, w)")
    n, _, h, w = frames.shape
    x = frames.contiguous()
    planes = x.view(n * 3, h, w)
    p = _prec(precision)
    ws = _alloc_bytes(lib().abf_strided_workspace_bytes(n * 3, h, w, rho, N, p), x.device, stream)
    sig3 = _empty((n, 3, h, w), torch.float32, x.device, stream)
    g0 = grey(x, stream=stream)
    for c in range(3):
        mrtv_sigma(g0, mrtv_radius, eps, lo, hi, v_ref, out=sig3[:, c], stream=stream)
    y1 = fast_strided(planes, sig3.view(n * 3, h, w), kernel="box", rho=rho, N=N,
                      precision=precision, workspace=ws, stream=stream)
    y1f = y1 if y1.dtype == torch.float32 else y1.float()
    sig3b = _empty((n, 3, h, w), torch.float32, x.device, stream)
    for c in range(3):
        mrtv_sigma(g0, mrtv_radius, eps, shrink * lo, shrink * hi, v_ref, out=sig3b[:, c],
                   stream=stream)
    y2 = fast_strided(y1f, sig3b.view(n * 3, h, w), kernel="box", rho=rho, N=N,
                      precision=precision, workspace=ws, stream=stream)
    y2f = y2 if y2.dtype == torch.float32 else y2.float()
    th, scratch = sharpen_maps(y2f, rho, log_sigma, sharpen_lo, sharpen_hi, sharpen_v_ref,
                               stream=stream)
    g2 = grey(y2f.view(n, 3, h, w), stream=stream)
    sig3c = _empty((n, 3, h, w), torch.float32, x.device, stream)
    for c in range(3):
        sharpen_maps(g2, rho, log_sigma, sharpen_lo, sharpen_hi, sharpen_v_ref,
                     theta=scratch.view(n, 3, h, w)[:, c], sigma=sig3c[:, c], stream=stream)
    y3 = fast_strided(y2f, sig3c.view(n * 3, h, w), theta=th, kernel="box", rho=rho, N=N,
                      precision=precision, workspace=ws, stream=stream)
    out = y3.view(n, 3, h, w)
    if keep:
        return dict(grey0=g0, sigma1=sig3, pass1=y1.view(n, 3, h, w), sigma2=sig3b,
                    pass2=y2.view(n, 3, h, w), theta3=th.view(n, 3, h, w), grey2=g2,
                    sigma3=sig3c, pass3=out)
    return out
