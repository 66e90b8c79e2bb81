"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/abf.h, and rejects bad arguments synchronously (before
any HIP call) with the documented status codes."""
import ctypes
import os
import re

import pytest

import paper_1811_02308_amd as abf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abf.h")

pytestmark = pytest.mark.skipif(not os.path.exists(abf.library_path()),
                                reason="libabf.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(abf_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 14
    L = ctypes.CDLL(abf.library_path())
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = abf.lib()
    assert L.abf_status_string(0) == b"ok"
    assert b"invalid" in L.abf_status_string(-1)
    assert b"workspace" in L.abf_status_string(-5)
    assert L.abf_version() >= 100


def test_stack_layout_arithmetic():
    L = abf.lib()
    assert L.abf_stack_pitch(1) == 64 and L.abf_stack_pitch(64) == 64 and L.abf_stack_pitch(65) == 128
    h, w, N = 100, 130, 6
    P = 192 * h
    assert L.abf_stack_plane_offset(h, w, N, 1, 0) == 0
    assert L.abf_stack_plane_offset(h, w, N, 1, 1) == 4 * P
    assert L.abf_stack_plane_offset(h, w, N, 1, 2) == 8 * P
    assert L.abf_stack_plane_offset(h, w, N, 0, 3) == 8 * P + 8 * P
    sb = L.abf_stack_bytes(h, w, N, 1)
    assert sb >= 4 * P * (N + 2) and sb % 256 == 0
    assert L.abf_stack_bytes(h, w, N, 0) >= 8 * P + 8 * P * N
    assert L.abf_workspace_bytes(h, w, 5, N, 1) == sb + L.abf_scratch_bytes(h, w, 5)
    assert L.abf_workspace_bytes(0, w, 5, N, 1) == 0


def _fast(L, **kw):
    a = dict(img=1, theta=None, sigma=1, h=8, w=8, pitch=8, kind=0, ss=0.0, rho=2, N=5, prec=1,
             flags=1, out=1, opitch=8, ws=256, wsb=1 << 20, stream=None)
    a.update(kw)
    v = lambda x: ctypes.c_void_p(x) if x is not None else None
    return L.abf_fast(v(a["img"]), v(a["theta"]), v(a["sigma"]), a["h"], a["w"], a["pitch"],
                      a["kind"], a["ss"], a["rho"], a["N"], a["prec"], a["flags"], v(a["out"]),
                      a["opitch"], v(a["ws"]), a["wsb"], a["stream"])


def test_invalid_arguments_rejected_before_any_launch():
    L = abf.lib()
    assert _fast(L, img=None) == -1
    assert _fast(L, sigma=None) == -1
    assert _fast(L, out=None) == -1
    assert _fast(L, h=0) == -1
    assert _fast(L, pitch=7) == -1
    assert _fast(L, opitch=7) == -1
    assert _fast(L, rho=-1) == -1
    assert _fast(L, N=-1) == -1
    assert _fast(L, prec=7) == -1
    assert _fast(L, kind=3) == -1
    assert _fast(L, N=9) == -4
    assert _fast(L, rho=97) == -4
    assert _fast(L, ws=None) == -5
    assert _fast(L, ws=257) == -5          # misaligned
    assert _fast(L, wsb=16) == -5          # too small


def test_other_entry_points_validate():
    L = abf.lib()
    vp = ctypes.c_void_p
    assert L.abf_bruteforce(None, None, vp(1), 4, 4, 4, 0, 0.0, 1, 0, vp(1), 4, None) == -1
    assert L.abf_bruteforce(vp(1), None, vp(1), 4, 4, 4, 0, 0.0, 200, 0, vp(1), 4, None) == -4
    assert L.abf_minmax(vp(1), 4, 4, 4, 1, vp(1), vp(1), 4, None, 0, None) == -5
    assert L.abf_minmax(vp(1), 4, 4, 3, 1, vp(1), vp(1), 4, vp(256), 1 << 20, None) == -1
    assert L.abf_range(vp(256), 1 << 20, None, None, vp(1), 4, 4, 4, 5, 1, 1, vp(1), 4, None) == -1
    assert L.abf_moment_stack(vp(1), 4, 4, 4, 0, 0.0, 1, 5, 1, vp(256), 16, vp(256), 1 << 20, None) == -5
    reqs = (abf.Request * 1)()
    reqs[0] = abf.Request(1, None, 1, 4, 4, 4, 0, 0.0, 1, 5, 1, 4)
    assert L.abf_fast_batched(reqs, 1, 1, 1, None, 0, None) == -5
    reqs[0] = abf.Request(1, None, 1, 4, 4, 4, 0, 0.0, 1, 12, 1, 4)
    assert L.abf_fast_batched(reqs, 1, 1, 1, None, 0, None) == -4
    assert L.abf_fast_batched(reqs, 0, 1, 1, None, 0, None) == 0


def test_stack_single_pass_query():
    """The bounds are taken inside the Gaussian tile kernel; the box kernel
    and the matrix-core kernel (8 <= rho <= 16 on images of 4 Mpix or more)
    read them from a separate bounds pass. No device call is made."""
    L = abf.lib()
    assert L.abf_stack_single_pass(1024, 1024, 1, 15, 6) == 1
    assert L.abf_stack_single_pass(333, 340, 1, 3, 5) == 1
    assert L.abf_stack_single_pass(1024, 1024, 0, 15, 6) == 0      # box
    assert L.abf_stack_single_pass(2048, 2048, 1, 15, 6) == 0      # matrix cores
    assert L.abf_stack_single_pass(2048, 2048, 1, 20, 6) == 1
    assert L.abf_stack_single_pass(1024, 1024, 1, 40, 7) == 1
    assert L.abf_stack_single_pass(1024, 1024, 1, 90, 8) == 1
    assert L.abf_stack_single_pass(1024, 1024, 1, 15, 0) == 0      # no moments
    assert L.abf_stack_single_pass(0, 1024, 1, 15, 6) == 0
    assert L.abf_stack_single_pass(16, 16, 1, -1, 6) == 0
    assert L.abf_stack_single_pass(16, 16, 1, 3, 9) == 0
    assert L.abf_stack_single_pass(16, 16, 5, 3, 6) == 0


def test_fast_fused_query():
    """abf_fast_fused: the box kernel on the mixed path at rho <= 32 runs the
    moment and range stages fused, and so does the Gaussian tile kernel on
    the mixed path where it takes the window bounds itself (one kernel for
    the whole filter); everything else, and invalid arguments, the stack
    path."""
    L = abf.lib()
    assert L.abf_fast_fused(4096, 4096, 0, 5, 8, 1) == 1
    assert L.abf_fast_fused(4096, 4096, 0, 8, 5, 1) == 1
    assert L.abf_fast_fused(4096, 4096, 0, 20, 8, 1) == 1
    assert L.abf_fast_fused(4096, 4096, 0, 32, 5, 1) == 1
    assert L.abf_fast_fused(4096, 4096, 0, 33, 5, 1) == 0
    assert L.abf_fast_fused(4096, 4096, 0, 5, 8, 0) == 0          # FP64
    assert L.abf_fast_fused(4096, 4096, 1, 5, 8, 1) == 1          # Gaussian tile, bounds taken
    assert L.abf_fast_fused(1024, 1024, 1, 15, 6, 1) == 1
    assert L.abf_fast_fused(4096, 4096, 1, 10, 6, 1) == 0         # matrix-core stack
    assert L.abf_fast_fused(1024, 1024, 1, 15, 6, 0) == 0         # FP64
    assert L.abf_fast_fused(4096, 4096, 2, 5, 8, 1) == 0          # recursive
    assert L.abf_fast_fused(64, 64, 0, 3, 0, 1) == 0              # N = 0: bounds only
    assert L.abf_fast_fused(0, 64, 0, 3, 5, 1) == 0
    assert L.abf_fast_fused(64, 64, 0, 3, 5, 2) == 0
    assert abf.fast_fused(64, 64, "box", 3, 5) and not abf.fast_fused(64, 64, "box", 3, 5, "fp64")


def test_stack_kernel_query():
    """abf_stack_kernel names the moment kernel of a configuration: box
    running sums, the tile kernel (LDS stride 160 or 256) or the matrix-core
    kernel; -1 for invalid arguments."""
    L = abf.lib()
    BOUNDS, BOX, TILE, WIDE, MFMA = 0, 1, 2, 3, 4
    assert L.abf_stack_kernel(4096, 4096, 0, 5, 8, 1) == BOX
    assert L.abf_stack_kernel(4096, 4096, 0, 20, 6, 0) == BOX
    assert L.abf_stack_kernel(4096, 4096, 0, 5, 7, 0) == TILE          # FP64 box, N >= 7
    assert L.abf_stack_kernel(4096, 4096, 0, 40, 8, 0) == WIDE
    assert L.abf_stack_kernel(1024, 1024, 1, 15, 6, 1) == TILE
    assert L.abf_stack_kernel(2048, 2048, 1, 15, 6, 1) == MFMA
    assert L.abf_stack_kernel(2048, 2048, 1, 15, 6, 0) == TILE          # FP64 keeps the tile kernel
    assert L.abf_stack_kernel(2048, 2047, 1, 15, 6, 1) == TILE         # below 2^22 pixels
    assert L.abf_stack_kernel(2048, 2048, 1, 15, 7, 1) == TILE         # N = 7 stays on the tile
    assert L.abf_stack_kernel(2048, 2048, 1, 7, 6, 1) == TILE          # R < 8
    assert L.abf_stack_kernel(2048, 2048, 1, 17, 6, 1) == WIDE
    assert L.abf_stack_kernel(64, 64, 1, 16, 5, 1) == TILE
    assert L.abf_stack_kernel(64, 64, 1, 17, 5, 1) == WIDE
    assert L.abf_stack_kernel(64, 64, 1, 96, 8, 0) == WIDE
    assert L.abf_stack_kernel(64, 64, 0, 3, 0, 1) == BOUNDS
    assert L.abf_stack_kernel(0, 64, 0, 3, 5, 1) == -1
    assert L.abf_stack_kernel(64, 64, 2, 3, 5, 1) == -1
    assert L.abf_stack_kernel(64, 64, 0, 3, 9, 1) == -1
    assert L.abf_stack_kernel(64, 64, 0, 97, 5, 1) == -1
    assert L.abf_stack_kernel(64, 64, 0, 3, 5, 2) == -1
