// Sanitizer driver for the C ABI of libabf (include/abf.h): argument checks,
// status codes and the workspace / stack layout arithmetic of api.cpp, run
// against host-only launcher stand-ins (stub_launchers.cpp) under
// AddressSanitizer and UndefinedBehaviorSanitizer. Every buffer is host
// memory registered with the stand-ins, which report any plane a kernel
// would touch outside it. Exit status 0 when every check holds.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/abf.h"
#include "stub_registry.h"

static int g_fail = 0;
#define CHECK(c)                                                             \
  do {                                                                       \
    if (!(c)) {                                                              \
      std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);      \
      ++g_fail;                                                              \
    }                                                                        \
  } while (0)

// A 256-byte aligned host buffer of `bytes` bytes, registered with the stubs.
struct Buf {
  std::vector<unsigned char> raw;
  void* p = nullptr;
  size_t bytes = 0;
  explicit Buf(size_t n) : raw(n + 256), bytes(n) {
    uintptr_t a = reinterpret_cast<uintptr_t>(raw.data());
    p = reinterpret_cast<void*>((a + 255) / 256 * 256);
    stub_register(p, n);
  }
  float* f() { return static_cast<float*>(p); }
};

static void sizes() {
  CHECK(abf_stack_pitch(0) == 0 && abf_stack_pitch(-3) == 0);
  CHECK(abf_stack_pitch(1) == 64 && abf_stack_pitch(64) == 64 && abf_stack_pitch(65) == 128);
  CHECK(abf_stack_bytes(0, 5, 3, ABF_PREC_MIXED) == 0 && abf_stack_bytes(5, 0, 3, 1) == 0);
  CHECK(abf_stack_bytes(5, 5, -1, ABF_PREC_MIXED) == 0);
  CHECK(abf_scratch_bytes(0, 5, 3) == 0 && abf_workspace_bytes(5, 5, 3, -1, 1) == 0);
  // planes: alpha, beta (float32), then N moment planes of the precision
  for (int prec = 0; prec <= 1; ++prec)
    for (int N = 0; N <= ABF_N_MAX; ++N) {
      const int h = 37, w = 70;
      const size_t P = (size_t)abf_stack_pitch(w) * h, e = prec == ABF_PREC_FP64 ? 8 : 4;
      CHECK(abf_stack_plane_offset(h, w, N, prec, 1) == 4 * P);
      CHECK(abf_stack_plane_offset(h, w, N, prec, 2) == 8 * P);
      CHECK(abf_stack_plane_offset(h, w, N, prec, N + 2) == 8 * P + N * P * e);
      CHECK(abf_stack_bytes(h, w, N, prec) >= 8 * P + N * P * e);
      CHECK(abf_stack_bytes(h, w, N, prec) % 256 == 0);
    }
  // large images: 2^32 pixels, sizes in size_t without wrap-around
  const size_t big = abf_stack_bytes(65536, 65536, 8, ABF_PREC_FP64);
  CHECK(big == (size_t)65536 * 65536 * (8 + 8 * 8));
  CHECK(abf_workspace_bytes(65536, 65536, 5, 8, ABF_PREC_FP64) > big);
  for (int s = -6; s <= 0; ++s) CHECK(std::strlen(abf_status_string(s)) > 0);
  CHECK(std::strlen(abf_status_string(42)) > 0);
  CHECK(abf_version() > 0);
}

static void entry_points() {
  const int h = 40, w = 53;
  const long long pitch = 56;
  Buf img(sizeof(float) * pitch * h), th(sizeof(float) * pitch * h), sg(sizeof(float) * pitch * h);
  Buf out(sizeof(double) * pitch * h);
  for (int prec = 0; prec <= 1; ++prec)
    for (int kind = 0; kind <= 1; ++kind)
      for (int N : {0, 1, 5, 8})
        for (int rho : {0, 3, 30, (int)ABF_RHO_MAX}) {
          const size_t wsb = abf_workspace_bytes(h, w, rho, N, prec);
          const size_t sb = abf_stack_bytes(h, w, N, prec);
          Buf ws(wsb), st(sb), scr(abf_scratch_bytes(h, w, rho));
          const unsigned fl = ABF_FLAG_CLAMP;
          CHECK(abf_fast(img.f(), th.f(), sg.f(), h, w, pitch, kind, 0.0, rho, N, prec, fl, out.p,
                         pitch, ws.p, wsb, nullptr) == ABF_OK);
          CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, pitch, kind, 0.0, rho, N, prec, fl,
                         out.p, pitch, ws.p, wsb, nullptr) == ABF_OK);
          CHECK(abf_moment_stack(img.f(), h, w, pitch, kind, 0.0, rho, N, prec, st.p, sb, scr.p,
                                 scr.bytes, nullptr) == ABF_OK);
          CHECK(abf_range(st.p, sb, img.f(), nullptr, sg.f(), h, w, pitch, N, prec, fl, out.p,
                          pitch, nullptr) == ABF_OK);
          // too small or misaligned workspaces and stacks
          CHECK(abf_fast(img.f(), th.f(), sg.f(), h, w, pitch, kind, 0.0, rho, N, prec, fl, out.p,
                         pitch, ws.p, wsb - 1, nullptr) == ABF_E_WORKSPACE);
          CHECK(abf_fast(img.f(), th.f(), sg.f(), h, w, pitch, kind, 0.0, rho, N, prec, fl, out.p,
                         pitch, static_cast<char*>(ws.p) + 8, wsb, nullptr) == ABF_E_WORKSPACE);
          CHECK(abf_range(st.p, sb - 1, img.f(), nullptr, sg.f(), h, w, pitch, N, prec, fl,
                          out.p, pitch, nullptr) == ABF_E_WORKSPACE);
          if (N >= 1) {
            CHECK(abf_stack_moments(img.f(), h, w, pitch, kind, 0.0, rho, N, prec, st.p, sb,
                                    nullptr) == ABF_OK);
            CHECK(abf_moments_range(img.f(), th.f(), sg.f(), h, w, pitch, kind, 0.0, rho, N, prec,
                                    fl, st.p, sb, out.p, pitch, nullptr) == ABF_OK);
            CHECK(abf_range_uniform(st.p, sb, img.f(), nullptr, sg.f(), h, w, pitch, N, prec, fl,
                                    out.p, pitch, nullptr) == ABF_OK);
          }
        }
  // the recursive kernel: its own workspace size, abf_fast and abf_moment_stack only
  for (int prec = 0; prec <= 1; ++prec)
    for (int N : {1, 5, 6, 7})
      for (int rho : {0, 3, 30}) {
        const int k = ABF_KERNEL_RECURSIVE;
        const size_t wsb = abf_kernel_workspace_bytes(h, w, rho, N, prec, k);
        const size_t sb = abf_stack_bytes(h, w, N, prec);
        CHECK(wsb > abf_workspace_bytes(h, w, rho, N, prec));
        CHECK(abf_kernel_workspace_bytes(h, w, rho, N, prec, 0) ==
              abf_workspace_bytes(h, w, rho, N, prec));
        Buf ws(wsb), st(sb), scr(abf_kernel_scratch_bytes(h, w, rho, N, k));
        const abf_status want = prec == ABF_PREC_FP64 ? ABF_E_UNSUPPORTED : ABF_OK;
        CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, pitch, k, 0.0, rho, N, prec, 1, out.p,
                       pitch, ws.p, wsb, nullptr) == want);
        CHECK(abf_moment_stack(img.f(), h, w, pitch, k, 0.0, rho, N, prec, st.p, sb, scr.p,
                               scr.bytes, nullptr) == want);
        if (want == ABF_OK) {
          CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, pitch, k, 0.0, rho, N, prec, 1, out.p,
                         pitch, ws.p, abf_workspace_bytes(h, w, rho, N, prec),
                         nullptr) == ABF_E_WORKSPACE);
        }
        CHECK(abf_stack_moments(img.f(), h, w, pitch, k, 0.0, rho, N, prec, st.p, sb, nullptr) ==
              ABF_E_INVALID);
        CHECK(abf_bruteforce(img.f(), nullptr, sg.f(), h, w, pitch, k, 0.0, rho, prec, out.p,
                             pitch, nullptr) == ABF_E_INVALID);
      }
  const size_t wsb = abf_workspace_bytes(h, w, 3, 5, ABF_PREC_MIXED);
  Buf ws(wsb);
  // invalid arguments: refused before any launch
  const int calls = stub_calls();
  CHECK(abf_fast(nullptr, nullptr, nullptr, h, w, pitch, 0, 0.0, 3, 5, 1, 1, out.p, pitch, ws.p,
                 wsb, nullptr) == ABF_E_INVALID);
  CHECK(abf_fast(img.f(), nullptr, sg.f(), 0, w, pitch, 0, 0.0, 3, 5, 1, 1, out.p, pitch, ws.p,
                 wsb, nullptr) == ABF_E_INVALID);
  CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, w - 1, 0, 0.0, 3, 5, 1, 1, out.p, pitch, ws.p,
                 wsb, nullptr) == ABF_E_INVALID);
  CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, pitch, 3, 0.0, 3, 5, 1, 1, out.p, pitch, ws.p,
                 wsb, nullptr) == ABF_E_INVALID);
  CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, pitch, 0, 0.0, -1, 5, 1, 1, out.p, pitch, ws.p,
                 wsb, nullptr) == ABF_E_INVALID);
  CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, pitch, 0, 0.0, 3, 5, 7, 1, out.p, pitch, ws.p,
                 wsb, nullptr) == ABF_E_INVALID);
  CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, pitch, 1, 1.0 / 0.0, 3, 5, 1, 1, out.p, pitch,
                 ws.p, wsb, nullptr) == ABF_E_INVALID);
  CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, pitch, 0, 0.0, 3, ABF_N_MAX + 1, 1, 1, out.p,
                 pitch, ws.p, wsb, nullptr) == ABF_E_UNSUPPORTED);
  CHECK(abf_fast(img.f(), nullptr, sg.f(), h, w, pitch, 0, 0.0, ABF_RHO_MAX + 1, 5, 1, 1, out.p,
                 pitch, ws.p, wsb, nullptr) == ABF_E_UNSUPPORTED);
  CHECK(abf_minmax(img.f(), h, w, pitch, 3, out.f(), out.f(), w - 1, ws.p, wsb, nullptr) ==
        ABF_E_INVALID);
  CHECK(abf_bruteforce(img.f(), nullptr, nullptr, h, w, pitch, 0, 0.0, 3, 1, out.p, pitch,
                       nullptr) == ABF_E_INVALID);
  CHECK(stub_calls() == calls);
  CHECK(abf_bruteforce(img.f(), nullptr, sg.f(), h, w, pitch, 1, 0.0, 3, 0, out.p, pitch,
                       nullptr) == ABF_OK);
  CHECK(abf_sigma_local_std(img.f(), 1, h, w, pitch, 0, 4, 3.0, 5.0, 80.0, out.f(), pitch, 0,
                            nullptr) == ABF_OK);
}

static void batches() {
  // requests of different sizes and parameters, each with its own buffers
  const int n = 5;
  std::vector<Buf*> keep;
  std::vector<abf_request> reqs(n);
  for (int i = 0; i < n; ++i) {
    const int h = 9 + 13 * i, w = 17 + 7 * i;
    const long long pitch = w + i;
    Buf* a = new Buf(sizeof(float) * pitch * h);
    Buf* s = new Buf(sizeof(float) * pitch * h);
    Buf* o = new Buf(sizeof(double) * (w + 3) * h);
    keep.insert(keep.end(), {a, s, o});
    reqs[i] = abf_request{a->f(), nullptr, s->f(), h, w, pitch, i % 2, 0.0, 2 + 9 * i,
                          1 + (i * 3) % 8, o->p, w + 3};
  }
  for (int prec = 0; prec <= 1; ++prec) {
    const size_t wsb = abf_batched_workspace_bytes(reqs.data(), n, prec);
    Buf ws(wsb);
    CHECK(abf_fast_batched(reqs.data(), n, prec, ABF_FLAG_CLAMP, ws.p, wsb, nullptr) == ABF_OK);
    CHECK(abf_fast_batched(reqs.data(), n, prec, ABF_FLAG_CLAMP, ws.p, wsb - 1, nullptr) ==
          ABF_E_WORKSPACE);
    CHECK(abf_fast_batched(reqs.data(), 0, prec, ABF_FLAG_CLAMP, nullptr, 0, nullptr) == ABF_OK);
  }
  // requests that share launches: groups of one shape and parameter set
  // (theta given by all or none), each request with its own buffers, mixed
  // with single requests; radii on both sides of the bounds kernel's tile
  // limit (the larger ones loop over the images on the host)
  for (int rho : {3, 40}) {
    std::vector<abf_request> g;
    for (int i = 0; i < 7; ++i) {
      const bool odd = i % 3 == 2;
      const int h = odd ? 30 : 23, w = odd ? 19 : 41;
      const long long pitch = w + 5;
      Buf* a = new Buf(sizeof(float) * pitch * h);
      Buf* t = new Buf(sizeof(float) * pitch * h);
      Buf* s = new Buf(sizeof(float) * pitch * h);
      Buf* o = new Buf(sizeof(double) * (w + 2) * h);
      keep.insert(keep.end(), {a, t, s, o});
      g.push_back(abf_request{a->f(), i % 2 ? t->f() : nullptr, s->f(), h, w, pitch, i % 2 ? 0 : 1,
                              0.0, rho, 5, o->p, w + 2});
    }
    for (int prec = 0; prec <= 1; ++prec) {
      const size_t wsb = abf_batched_workspace_bytes(g.data(), (int)g.size(), prec);
      Buf ws(wsb);
      const int before = stub_calls();
      CHECK(abf_fast_batched(g.data(), (int)g.size(), prec, ABF_FLAG_CLAMP, ws.p, wsb, nullptr) ==
            ABF_OK);
      CHECK(stub_calls() > before);
      CHECK(abf_fast_batched(g.data(), (int)g.size(), prec, ABF_FLAG_CLAMP, ws.p, wsb - 1,
                             nullptr) == ABF_E_WORKSPACE);
    }
  }
  {  // four requests of one group: the offset table, then one launch per stage for all four
    std::vector<abf_request> g;
    for (int i = 0; i < 4; ++i) {
      Buf* a = new Buf(sizeof(float) * 64 * 20);
      Buf* s = new Buf(sizeof(float) * 64 * 20);
      Buf* o = new Buf(sizeof(float) * 64 * 20);
      keep.insert(keep.end(), {a, s, o});
      g.push_back(abf_request{a->f(), nullptr, s->f(), 20, 60, 64, 0, 0.0, 3, 5, o->p, 64});
    }
    const size_t wsb = abf_batched_workspace_bytes(g.data(), 4, 1);
    Buf ws(wsb);
    const int before = stub_calls();
    CHECK(abf_fast_batched(g.data(), 4, 1, ABF_FLAG_CLAMP, ws.p, wsb, nullptr) == ABF_OK);
    // the table, then bounds and fused moments-and-range, or bounds, moments, range
    CHECK(stub_calls() - before == (abf_fast_fused(20, 60, 0, 3, 5, 1) ? 3 : 4));
  }
  abf_request bad = reqs[1];
  bad.N = ABF_N_MAX + 1;
  CHECK(abf_batched_workspace_bytes(&bad, 1, 1) == 0 ||
        abf_fast_batched(&bad, 1, 1, 1, nullptr, 0, nullptr) != ABF_OK);
  // strided: n images of one shape at a fixed stride
  const int m = 3, h = 21, w = 34;
  const long long pitch = 40, stride = pitch * h + 16;
  Buf img(sizeof(float) * stride * m), sg(sizeof(float) * stride * m);
  Buf out(sizeof(double) * stride * m);
  for (int prec = 0; prec <= 1; ++prec)
    for (int rho : {1, 8, 40}) {
      const size_t wsb = abf_strided_workspace_bytes(m, h, w, rho, 6, prec);
      Buf ws(wsb);
      CHECK(abf_fast_strided(img.f(), nullptr, sg.f(), m, h, w, pitch, stride, 0, 0.0, rho, 6,
                             prec, ABF_FLAG_CLAMP, out.p, pitch, stride, ws.p, wsb,
                             nullptr) == ABF_OK);
      CHECK(abf_fast_strided(img.f(), nullptr, sg.f(), m, h, w, pitch, stride, 0, 0.0, rho, 6,
                             prec, ABF_FLAG_CLAMP, out.p, pitch, stride, ws.p, wsb - 1,
                             nullptr) == ABF_E_WORKSPACE);
    }
  Buf t2(sizeof(float) * stride * m), s2(sizeof(float) * stride * m);
  CHECK(abf_sharpen_maps(img.f(), m, h, w, pitch, stride, 5, 1.0, 5.0, 40.0, 20.0, t2.f(), s2.f(),
                         pitch, stride, nullptr) == ABF_OK);
  CHECK(abf_mrtv_sigma(img.f(), m, h, w, pitch, stride, 2, 1e-3, 5.0, 80.0, 20.0, s2.f(), pitch,
                       stride, nullptr) == ABF_OK);
  CHECK(abf_sharpen_maps(img.f(), m, h, w, pitch, stride, 5, 1.0, 50.0, 40.0, 20.0, t2.f(),
                         s2.f(), pitch, stride, nullptr) == ABF_E_INVALID);      // lo > hi
  for (Buf* b : keep) delete b;
}

int main() {
  sizes();
  entry_points();
  batches();
  const int v = stub_violations();
  if (v) std::fprintf(stderr, "%d plane(s) outside their buffers\n", v);
  std::printf("abi driver: %d failed checks, %d out-of-buffer planes, %d launches\n", g_fail, v,
              stub_calls());
  return (g_fail || v) ? 1 : 0;
}
