/*
 * abf.h -- C ABI of the MI355X (gfx950) fast adaptive bilateral filter.
 *
 * Implements the filter of Gavaskar & Chaudhury, "Fast Adaptive Bilateral
 * Filtering" (arXiv:1811.02308):
 *
 *   brute force  g(i) = sum_j w(j) phi_i(f(i-j) - theta(i)) f(i-j) / eta(i)
 *                eqs. (BF_adaptive1), (BF_adaptive2), (r_kernel)
 *   fast         Algorithm 1 (Sec. II-D): window bounds alpha, beta
 *                (eq. bounds), moments of the local histogram by
 *                convolution (Prop. 2), the shift to [alpha, beta]
 *                (Prop. 3), the Hilbert-inverse fit (Theorem, eq. inv),
 *                the range integrals I_k (eqs. I_0, I_1, F_forward) and the
 *                ratio of eq. (BFfinal).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Images are single-channel, row-major float32 planes on the DEVICE,
 *   h rows by w columns; `pitch` is the distance between rows in elements
 *   (pitch >= w). The caller owns every buffer; the library never frees or
 *   keeps a pointer after a call returns.
 * - Border rule: windows are clamp-to-edge (replicate) in every stage.
 * - Window: `rho` is the integer radius R; the window is [-R, R]^2. The box
 *   kernel weighs every tap 1/(2R+1)^2. The Gaussian kernel weighs tap j by
 *   exp(-|j|^2 / (2 sigma_s^2)) (eq. sp_kernel), normalised to sum to 1;
 *   sigma_s <= 0 selects sigma_s = R/3 (the paper's window [-3 rho, 3 rho]).
 * - theta may be NULL, meaning theta = f (the classical filter, Sec. III).
 *   sigma must hold values > 0 (or +inf, which gives the spatial mean);
 *   this is not checked on the device, violations give NaN at that pixel.
 * - All calls are asynchronous on `stream` (a hipStream_t, NULL = default
 *   stream). Argument errors are reported synchronously, before any HIP
 *   call, as ABF_E_INVALID / ABF_E_UNSUPPORTED / ABF_E_WORKSPACE; a failed
 *   launch is reported as ABF_E_HIP. Nothing is synchronised.
 * - Precision: ABF_PREC_FP64 computes and stores everything in FP64 and
 *   writes a double output. ABF_PREC_MIXED computes in FP64 but keeps the
 *   moment stack and the output in FP32 (see abf_moment_stack).
 * - Calls on different streams with different workspaces may run
 *   concurrently; the library holds no mutable device state.
 */
#ifndef ABF_H
#define ABF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ABF_OK = 0,
    ABF_E_INVALID = -1,      /* null pointer, bad size, pitch < w, ...      */
    ABF_E_NOMEM = -2,        /* reserved (the library never allocates)      */
    ABF_E_HIP = -3,          /* a HIP launch or runtime call failed         */
    ABF_E_UNSUPPORTED = -4,  /* valid but outside what is built (N, rho)    */
    ABF_E_WORKSPACE = -5     /* workspace/stack too small or misaligned     */
} abf_status;

/* ABF_KERNEL_RECURSIVE: the recursive approximation of the Gaussian that
 * Sec. II-D names as the O(1)-per-pixel option for the convolutions of
 * Algorithm 1 -- Deriche's fourth-order sum of two damped complex
 * exponentials (sigma_s as for the Gaussian, <= 0 meaning rho/3), taken on
 * the window [-rho, rho] only and normalised to sum 1 per axis, so that
 * every weight lies inside the window of the bounds. Its moments cost O(1)
 * per pixel for any rho (truncated first-order recursions along rows and
 * columns). Taken by abf_fast and abf_moment_stack only, with the workspace
 * of abf_kernel_workspace_bytes / abf_kernel_scratch_bytes, on the mixed
 * path only: the passes run along whole rows and columns, so the power
 * sums share one origin for the image, and under the FP64 path's
 * conditioning limits the windows far from it (recomputed directly, O(rho^2)
 * each) made a 4096 x 4096 call take seconds; ABF_PREC_FP64 returns
 * ABF_E_UNSUPPORTED. Every other entry point taking kernel_kind returns
 * ABF_E_INVALID for it. */
enum { ABF_KERNEL_BOX = 0, ABF_KERNEL_GAUSSIAN = 1, ABF_KERNEL_RECURSIVE = 2 };
enum { ABF_PREC_FP64 = 0, ABF_PREC_MIXED = 1 };
/* ABF_FLAG_CLAMP: clip the output to [alpha_i, beta_i] (the fitted
 * polynomial may go negative, Sec. II-B); recommended, used by tests.     */
enum { ABF_FLAG_CLAMP = 1u };
/* ABF_FLAG_KEEP_STACK (abf_moments_range only): also store the moment
 * planes in the stack, so that abf_range can reuse them later.            */
enum { ABF_FLAG_KEEP_STACK = 2u };
enum { ABF_N_MAX = 8, ABF_RHO_MAX = 96 };

/* Human-readable name of a status code (static string). */
const char* abf_status_string(int status);

/* Library version: major*10000 + minor*100 + patch. */
int abf_version(void);

/*
 * Moment stack (the resident intermediate of Algorithm 1).
 * Layout: plane pitch P = abf_stack_pitch(w) elements (a multiple of 64);
 *   plane 0  alpha_i  float32 (exact window minimum of f)
 *   plane 1  beta_i   float32 (exact window maximum of f)
 *   planes 2..N+1     a~_k, k = 1..N: the shifted-Legendre moments of the
 *            stretched histogram H_i (eqs. Lambda_tilde, mhist),
 *            a~_k = sum_j w(j) P_k(2 y_j - 1) with y_j = (f(i-j)-alpha_i)/
 *            (beta_i-alpha_i); they equal sum_r ell_kr mu_r for the moments
 *            mu_r of eq. (hist_moments_new), and lie in [-1, 1].
 *            float32 for ABF_PREC_MIXED, float64 for ABF_PREC_FP64.
 * Plane k starts at byte offset abf_stack_plane_offset(h, w, N, prec, k).
 * Where alpha_i == beta_i the moment planes hold 0.
 * The stack depends on (f, kernel, rho, N) only, not on theta or sigma.
 */
long long abf_stack_pitch(int w);
size_t abf_stack_bytes(int h, int w, int N, int precision);
size_t abf_stack_plane_offset(int h, int w, int N, int precision, int plane);

/* Scratch needed by abf_fast / abf_moment_stack / abf_minmax besides the
 * stack (bytes). abf_fast's workspace = abf_stack_bytes + this. */
size_t abf_scratch_bytes(int h, int w, int rho);
size_t abf_workspace_bytes(int h, int w, int rho, int N, int precision);
/* The same for a given spatial kernel: equal to the two above for the box
 * and Gaussian kernels; for ABF_KERNEL_RECURSIVE the scratch also holds
 * 2N FP64 planes of h x w (the row pass's sums and the column pass's causal
 * half) plus the origin and the kernel's weights. */
size_t abf_kernel_scratch_bytes(int h, int w, int rho, int N, int kernel_kind);
size_t abf_kernel_workspace_bytes(int h, int w, int rho, int N, int precision, int kernel_kind);

/*
 * abf_minmax -- eq. (bounds): alpha_i / beta_i = min / max of f over the
 * clamp-to-edge window [-rho, rho]^2 (eq. bounds; Prop. 1). Exact
 * (bit-identical to any correct evaluation). alpha/beta: device float32
 * planes with row pitch out_pitch. workspace: >= abf_scratch_bytes(h,w,rho)
 * bytes, 256-byte aligned. rho in [0, ABF_RHO_MAX].
 */
abf_status abf_minmax(const float* img, int h, int w, long long pitch, int rho,
                      float* alpha, float* beta, long long out_pitch,
                      void* workspace, size_t workspace_bytes, void* stream);

/*
 * abf_moment_stack -- window bounds and moment steps of Algorithm 1 (Props. 1-3): writes the
 * moment stack described above into `stack` (>= abf_stack_bytes, 256-byte
 * aligned). The power images are accumulated in FP64 about a local origin
 * and shifted to [alpha_i, beta_i] per pixel. N in [0, ABF_N_MAX].
 * Where abf_stack_single_pass() is 1 the bounds are taken inside the moment
 * kernel (one launch, workspace unused); otherwise abf_minmax runs first.
 * The stack is the same either way, and equals abf_minmax followed by
 * abf_stack_moments bit for bit. abf_fast builds its stack this way too.
 */
abf_status abf_moment_stack(const float* img, int h, int w, long long pitch,
                            int kernel_kind, double sigma_s, int rho, int N,
                            int precision, void* stack, size_t stack_bytes,
                            void* workspace, size_t workspace_bytes, void* stream);

/*
 * abf_stack_single_pass -- 1 if abf_moment_stack (and abf_fast) build the
 * stack of an h x w image with this kernel, rho and N in a single kernel
 * launch (the Gaussian tile kernel computes the window bounds of eq. bounds
 * itself), 0 if they launch the bounds kernel and then the moment kernel
 * (and for invalid arguments). Lets a caller time or plan the launches.
 */
int abf_stack_single_pass(int h, int w, int kernel_kind, int rho, int N);

/*
 * abf_stack_kernel -- which moment kernel abf_moment_stack (and so abf_fast,
 * abf_fast_strided, abf_fast_batched) runs for an h x w image with this
 * kernel, rho, N and precision: the step of Algorithm 1 that forms the
 * local-histogram moments by convolution (Prop. 2) and shifts them to
 * [alpha_i, beta_i] (Prop. 3). Values:
 *   ABF_STACK_BOUNDS_ONLY  N = 0: no moment planes, window bounds only
 *   ABF_STACK_BOX          box kernel, running sums (O(1) per pixel in rho)
 *   ABF_STACK_TILE         2-D tile kernel, direct separable sums (Gaussian
 *                          weights, or unit weights for the FP64 box path
 *                          at N >= 7), LDS row stride 160 (tile + 2 rho fit)
 *   ABF_STACK_TILE_WIDE    the same kernel with LDS row stride 256
 *   ABF_STACK_MFMA         Gaussian sums as banded FP64 matrix products
 * Returns -1 for invalid arguments. Host only; lets callers and tests
 * confirm which kernel a configuration exercises.
 */
enum { ABF_STACK_BOUNDS_ONLY = 0, ABF_STACK_BOX = 1, ABF_STACK_TILE = 2,
       ABF_STACK_TILE_WIDE = 3, ABF_STACK_MFMA = 4 };
int abf_stack_kernel(int h, int w, int kernel_kind, int rho, int N, int precision);

/*
 * abf_fast_fused -- 1 if abf_fast (and abf_fast_strided, and the shared
 * launches of abf_fast_batched) run the moment and range stages of
 * Algorithm 1 fused in one kernel for these arguments: the box kernel on
 * the mixed path at rho <= 32, and the Gaussian kernel on the mixed path
 * wherever its tile kernel builds the stack (there the same kernel takes
 * the window bounds as well: the whole filter in one launch), where the
 * fused kernels were measured faster on MI355X. 0 for the stack path and
 * for invalid arguments. Host only.
 */
int abf_fast_fused(int h, int w, int kernel_kind, int rho, int N, int precision);

/*
 * abf_stack_moments -- the second half of abf_moment_stack: given a stack
 * whose planes 0 and 1 already hold alpha_i and beta_i for this image and
 * rho (e.g. written by abf_minmax with out_pitch = abf_stack_pitch(w)),
 * writes the moment planes 2..N+1 (moment steps of Algorithm 1, Props. 2-3).
 * Needs no scratch. Lets a caller time or schedule the two spatial
 * kernels separately; abf_minmax + abf_stack_moments gives the stack of
 * abf_moment_stack.
 */
abf_status abf_stack_moments(const float* img, int h, int w, long long pitch,
                             int kernel_kind, double sigma_s, int rho, int N,
                             int precision, void* stack, size_t stack_bytes,
                             void* stream);

/*
 * abf_range -- Algorithm 1's per-pixel steps (eqs. inv, sub, I_0, I_1,
 * F_forward, BFfinal) from a moment stack: the fit
 * c = A^-1 mu (eq. inv, evaluated through the Legendre moments), t0 and
 * lambda (eq. sub), the integrals I_0..I_{N+1} (eqs. I_0, I_1 and the
 * recursion F_forward; for lambda below a threshold where that recursion
 * loses accuracy, the same definite integrals by Gauss-Legendre
 * quadrature), and g^ = alpha + (beta - alpha) T1/T2 (eq. BFfinal).
 * img is read only when theta is NULL. If T2 <= 0 or the ratio is not
 * finite the N = 0 estimate I_1/I_0 is used. Where alpha_i == beta_i the
 * output is f(i) (Algorithm 1's flat-window case). out: float32 (MIXED) or float64 (FP64) with
 * row pitch out_pitch (elements).
 */
abf_status abf_range(const void* stack, size_t stack_bytes, const float* img,
                     const float* theta, const float* sigma, int h, int w,
                     long long pitch, int N, int precision, unsigned flags,
                     void* out, long long out_pitch, void* stream);

/*
 * abf_moments_range -- Algorithm 1 from the moments on, in one pass per pixel: given
 * a stack whose planes 0 and 1 hold alpha_i and beta_i (abf_minmax with
 * out_pitch = abf_stack_pitch(w)), forms each pixel's moments (Props. 2-3)
 * and finishes the filter from them in registers (the fit of eq. inv, the
 * integrals, eq. BFfinal), without writing the moment planes unless flags
 * has ABF_FLAG_KEEP_STACK. The output equals abf_stack_moments followed by
 * abf_range, bit for bit. Arguments as for those two calls (theta and
 * sigma share `pitch` with img; theta NULL means theta = img).
 * It moves fewer bytes than the stack path but holds the range stage's
 * registers through the moment pass, which lowers occupancy; on MI355X it
 * is the slower of the two, so abf_fast uses the stack path.
 */
abf_status abf_moments_range(const float* img, const float* theta, const float* sigma,
                             int h, int w, long long pitch, int kernel_kind,
                             double sigma_s, int rho, int N, int precision,
                             unsigned flags, void* stack, size_t stack_bytes,
                             void* out, long long out_pitch, void* stream);

/*
 * abf_fast -- the whole fast filter (Algorithm 1) on one image:
 * abf_moment_stack into the front of `workspace`, then abf_range; or, where
 * abf_fast_fused() is 1, abf_minmax into the stack's bounds planes and then
 * abf_moments_range (moments and range stage in one kernel, the moment
 * planes never written), the Gaussian tile kernel writing the bounds
 * planes itself in that same kernel instead. All give the same output bit
 * for bit.
 * workspace >= abf_workspace_bytes(h, w, rho, N, precision), 256-byte
 * aligned. theta, sigma share `pitch` with img. Only ABF_FLAG_CLAMP of
 * `flags` is used.
 */
abf_status abf_fast(const float* img, const float* theta, const float* sigma,
                    int h, int w, long long pitch, int kernel_kind, double sigma_s,
                    int rho, int N, int precision, unsigned flags,
                    void* out, long long out_pitch,
                    void* workspace, size_t workspace_bytes, void* stream);

/*
 * abf_fast_noalloc -- abf_fast for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Its workspace is a fixed array of
 * ABF_NOALLOC_BYTES bytes (64 MiB) that the library holds on every GPU it
 * runs on until the process ends; the call itself allocates nothing. A
 * request whose abf_workspace_bytes(h, w, rho, N, precision) exceeds
 * ABF_NOALLOC_BYTES returns ABF_E_WORKSPACE before any device work (about
 * 16 + 4N bytes per pixel mixed, 16 + 8N FP64: 1024 x 1024 fits at every N
 * mixed and up to N = 6 in FP64). Calls on one GPU share that GPU's array:
 * calls that overlap on one GPU, on any streams, race, so the caller
 * serialises them.
 * Other arguments, checks and results are those of abf_fast (the same
 * kernels: the output is bit-identical).
 */
enum { ABF_NOALLOC_BYTES = 64 << 20 };
abf_status abf_fast_noalloc(const float* img, const float* theta, const float* sigma,
                            int h, int w, long long pitch, int kernel_kind,
                            double sigma_s, int rho, int N, int precision,
                            unsigned flags, void* out, long long out_pitch,
                            void* stream);

/*
 * abf_uniform_prior -- the uniform-prior comparison variant of Sec. III-B
 * (classical filtering, Fig. 3 and the discussion beside Table 1): the
 * N = 0 estimator of Algorithm 1 with the constant fitted on
 * [f(i), 2 fbar(i) - f(i)] (ordered) instead of [alpha_i, beta_i], fbar the
 * window mean under the same spatial kernel:
 *   g^ = lo + (hi - lo) I_1 / I_0,  t0 = (theta - lo)/(hi - lo),
 *   lambda = (hi - lo)^2 / (2 sigma^2);   g^ = f(i) where lo = hi.
 * Builds an N = 1 moment stack in `workspace` (>= abf_workspace_bytes(h,
 * w, rho, 1, precision)) and calls abf_range_uniform. Arguments and output
 * types as for abf_fast.
 *
 * abf_range_uniform -- the same from a resident stack built with any
 * N in [1, ABF_N_MAX] for this image, kernel and rho (fbar is recovered as
 * (alpha+beta)/2 + (beta-alpha)/2 a~_1). img is always read (f(i) sets the
 * interval); theta NULL means theta = img.
 */
abf_status abf_uniform_prior(const float* img, const float* theta, const float* sigma,
                             int h, int w, long long pitch, int kernel_kind, double sigma_s,
                             int rho, int precision, unsigned flags, void* out,
                             long long out_pitch, void* workspace, size_t workspace_bytes,
                             void* stream);
abf_status abf_range_uniform(const void* stack, size_t stack_bytes, const float* img,
                             const float* theta, const float* sigma, int h, int w,
                             long long pitch, int N, int precision, unsigned flags, void* out,
                             long long out_pitch, void* stream);

/*
 * abf_bruteforce -- eqs. (BF_adaptive1), (BF_adaptive2) directly, O(rho^2)
 * per pixel; the plain reference the fast path is compared with.
 * ABF_PREC_FP64: FP64 arithmetic, double output. ABF_PREC_MIXED: FP32
 * arithmetic, float output. The exponent of each window is shifted by its
 * smallest value (the common factor cancels in the ratio).
 */
abf_status abf_bruteforce(const float* img, const float* theta, const float* sigma,
                          int h, int w, long long pitch, int kernel_kind,
                          double sigma_s, int rho, int precision,
                          void* out, long long out_pitch, void* stream);

/* One image (or one channel) of a batch. */
typedef struct abf_request {
    const float* img;
    const float* theta;      /* NULL: theta = f */
    const float* sigma;
    int h, w;
    long long pitch;
    int kernel_kind;
    double sigma_s;
    int rho;
    int N;
    void* out;               /* float32 (MIXED) / float64 (FP64) */
    long long out_pitch;
} abf_request;

/*
 * abf_fast_batched -- abf_fast over n independent requests (images or
 * colour channels of any sizes and parameters; kernel_kind box, Gaussian or
 * recursive, under the same rules as abf_fast) in one call on one stream.
 * Requests that agree in h, w, pitch, out_pitch, kernel_kind, sigma_s, rho,
 * N and in whether theta is given form a group (at most 65535 requests; in
 * order of first appearance) whose images share each stage's launch: a
 * table of every member's byte offsets from the group's first request (its
 * image, theta, sigma, output and stack) is written to the workspace, and
 * each kernel finds its image through it, so each member may live in its
 * own allocation. A group of one, and every recursive request, runs as
 * abf_fast. The results are bit-identical to abf_fast on each request.
 * Pointers of one group must share the alignment of the group's first
 * (any caller-allocated float32 / float64 planes do).
 * workspace (device, 256-byte aligned) >= abf_batched_workspace_bytes(reqs,
 * n, precision): the offset table (40 bytes per request, rounded up to 256),
 * then one 256-byte aligned slice per request for its stack and scratch.
 * Validation as abf_fast for every request before any launch; n = 0 returns
 * ABF_OK without touching the workspace.
 */
size_t abf_batched_workspace_bytes(const abf_request* reqs, int n, int precision);
abf_status abf_fast_batched(const abf_request* reqs, int n, int precision,
                            unsigned flags, void* workspace, size_t workspace_bytes,
                            void* stream);

/*
 * abf_fast_strided -- abf_fast on n images of one shape and one parameter
 * set laid out at a fixed stride: image z is img + z*image_stride (theta
 * and sigma use the same stride), its output out + z*out_image_stride
 * (elements of the output type). Each stage of Algorithm 1 is ONE launch
 * whose grid covers all n images (e.g. the channels of a batch of colour
 * frames, filtered channel by channel as in Sec. IV-C).
 * workspace >= abf_strided_workspace_bytes(n, h, w, rho, N, precision):
 * n moment stacks followed by one scratch area. n in [1, 65535].
 */
size_t abf_strided_workspace_bytes(int n, int h, int w, int rho, int N, int precision);
abf_status abf_fast_strided(const float* img, const float* theta, const float* sigma, int n,
                            int h, int w, long long pitch, long long image_stride,
                            int kernel_kind, double sigma_s, int rho, int N, int precision,
                            unsigned flags, void* out, long long out_pitch,
                            long long out_image_stride, void* workspace,
                            size_t workspace_bytes, void* stream);

/*
 * Parameter maps of the applications (Sec. IV). n images at image_stride
 * (elements) in, maps at out_image_stride out (float32, row pitch
 * out_pitch); every border clamp-to-edge; sums in FP64. The affine map of a
 * measure v to sigma is sigma = hi - (hi - lo) min(v / v_ref, 1) (hi for
 * v = 0, falling to lo at v >= v_ref; the paper specifies only that low
 * values map to high sigma). lo <= hi, v_ref > 0.
 *
 * abf_sharpen_maps -- sharpening and noise removal (Sec. IV-A):
 *   theta = f + zeta, zeta = f - fbar, fbar the mean of f over the
 *   (2 radius + 1)^2 window; sigma = affine(|LoG * f|), the LoG being the sum
 *   over both axes of the second derivative (x^2/s^4 - 1/s^2) g(x) of the
 *   sampled Gaussian g of std s = log_sigma (radius round(4 s), normalised to
 *   sum 1) along one axis times g along the other. radius and round(4 s) at
 *   most 32.
 * abf_mrtv_sigma -- texture filtering (Sec. IV-C): sigma = affine(mRTV),
 *   mRTV = Delta max|grad f| / (sum|grad f| + eps) over the (2 radius + 1)^2
 *   window, Delta = window max - window min of f, grad f by central
 *   differences. radius at most 31, eps > 0.
 * abf_grey -- 0.299 R + 0.587 G + 0.114 B of planar colour images (channel
 *   planes channel_stride elements apart), the grey image the texture
 *   application computes its maps on.
 */
abf_status abf_sharpen_maps(const float* img, int n, int h, int w, long long pitch,
                            long long image_stride, int radius, double log_sigma, double lo,
                            double hi, double v_ref, float* theta, float* sigma,
                            long long out_pitch, long long out_image_stride, void* stream);
abf_status abf_mrtv_sigma(const float* img, int n, int h, int w, long long pitch,
                          long long image_stride, int radius, double eps, double lo, double hi,
                          double v_ref, float* sigma, long long out_pitch,
                          long long out_image_stride, void* stream);
abf_status abf_grey(const float* rgb, int n, int h, int w, long long pitch,
                    long long channel_stride, long long image_stride, float* out,
                    long long out_pitch, long long out_image_stride, void* stream);

/*
 * abf_sigma_local_std -- a per-pixel range width from local contrast for
 * texture filtering: sigma(i) = clamp(scale * sd(i), lo, hi), sd(i) the
 * population standard deviation of f over the clamp-to-edge window
 * [-radius, radius]^2 (FP64). The paper drives sigma from a local texture
 * measure through an affine map (Sec. IV-C); this is the contrast rule of
 * the texture benchmark. n images at image_stride / out_image_stride
 * (elements). radius in [0, 32]; lo <= hi.
 */
abf_status abf_sigma_local_std(const float* img, int n, int h, int w, long long pitch,
                               long long image_stride, int radius, double scale, double lo,
                               double hi, float* out, long long out_pitch,
                               long long out_image_stride, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ABF_H */
