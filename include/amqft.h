/*
 * amqft -- batched power-of-two complex DFT by the AM-QFT recursion on AMD
 * MI355X (gfx950).  C ABI: plain pointers and sizes, status codes, no
 * exceptions, no printing.
 *
 * Method: L. Pasquini, "A class of AM-QFT algorithms for power-of-two FFT"
 * (arXiv:1404.1810).  The transform computed is the CDFT of eq. qft_0A,
 *
 *     X(k) = sum_{n=0}^{N-1} x(n) exp(-i 2 pi n k / N),   k = 0..N-1,
 *
 * unnormalised, with input and output in natural ("growing") order
 * (Sec. 2.4, Table tab:implementation).  The eight variants of Sec. 5-6 are
 * selected by amqft_variant; all of them compute the same DFT and differ only
 * in rounding (Sec. 7.3).  N = 1 (identity) is accepted as an extension; the
 * paper's recursion starts at N = 2 (Sec. 4).
 *
 * Memory layout: complex values are interleaved (re, im) pairs of the storage
 * type; every signal is contiguous.  Device pointers come from the caller
 * (hipMalloc, or torch.empty(..., device="cuda") on ROCm) and must stay valid
 * until the work queued on the stream has completed.  in == out (in place) is
 * allowed for every entry point below unless stated otherwise.
 *
 * Errors: every entry point validates its arguments before any HIP call and
 * returns AMQFT_ERR_INVALID_ARG / AMQFT_ERR_NOT_POW2 / AMQFT_ERR_UNSUPPORTED
 * without touching the GPU; AMQFT_ERR_ALLOC reports a failed device
 * allocation and AMQFT_ERR_HIP a failed launch or copy (the HIP error string
 * is kept per thread and returned by amqft_last_hip_error()).
 */
#ifndef AMQFT_H
#define AMQFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Variant = skeleton x odd-to-even conversion M1..M8 (Sec. 5, Sec. 6):
 * 1, 4, 5, 8 split time indices first (dct_ot/dst_ot functions); 2, 3, 6, 7
 * split harmonics first (dct_to/dst_to).  4 is the improved QFT. */
typedef enum {
    AMQFT_V1 = 1, AMQFT_V2 = 2, AMQFT_V3 = 3, AMQFT_V4 = 4,
    AMQFT_V5 = 5, AMQFT_V6 = 6, AMQFT_V7 = 7, AMQFT_V8 = 8
} amqft_variant;

/* Storage type of the complex data; arithmetic is FP64 for AMQFT_C128,
 * FP32 for AMQFT_C64 / C32H / C32B and 32-bit fixed point for AMQFT_C32I. */
typedef enum {
    AMQFT_C128 = 0, /* complex double: 16 bytes per point            */
    AMQFT_C64 = 1,  /* complex float: 8 bytes per point              */
    AMQFT_C32H = 2, /* FP16 (re, im) pairs, FP32 arithmetic: 4 bytes */
    AMQFT_C32B = 3, /* BF16 (re, im) pairs, FP32 arithmetic: 4 bytes */
    /* Fixed point (Sec. 7.2: halvings are binary translations; Sec. 7.4:
     * fixed-point implementations): (re, im) int32 pairs, 8 bytes per point,
     * in units of the input's last bit; the output is the unnormalized DFT in
     * the same units.  Constants are round(f 2^29) (Q2.29), so only the
     * variants whose constants are 2cos / 2sin (1, 3, 5, 7) have this form;
     * 2^8 <= n <= 2^14.  Sums are exact and wrap modulo 2^32; a product with
     * a constant k is round(a k / 2^29), a halving round(a / 2), both to
     * nearest with ties away from zero.  The caller picks the input scale
     * (measured with the oracle on random, sign, tone and constant inputs):
     * variant 1 keeps every value inside int32 for |x| <= 2^15 up to
     * n = 2^14; variant 3 scales values near harmonic n/4 up by about
     * n/(4 pi) and needs |x| <= 2^12 at n = 2^12, 2^10 at 2^13 and 2^8 at
     * 2^14; variants 5 and 7 grow as their floating-point versions do and
     * wrap at |x| <= 2^15 from n = 2^12 (variant 5) and 2^10 (variant 7). */
    AMQFT_C32I = 4
} amqft_dtype;

typedef enum {
    AMQFT_OK = 0,
    AMQFT_ERR_INVALID_ARG = 1, /* null pointer, bad enum, bad batch/offsets */
    AMQFT_ERR_NOT_POW2 = 2,    /* a length is not a power of two or is < 1  */
    AMQFT_ERR_UNSUPPORTED = 3, /* length above AMQFT_MAX_LOG2N, or a flag
                                  combination this build does not provide   */
    AMQFT_ERR_ALLOC = 4,       /* device or host allocation failed          */
    AMQFT_ERR_HIP = 5          /* a HIP call failed                         */
} amqft_status;

/* Plan flags. */
enum {
    /* Generate the trigonometric constants (Sec. 7.1) on the device in FP64,
     * rounded once to the working precision: the LDS-resident kernels do so
     * inside every workgroup; for the paths that read constants from global
     * memory (N above one workgroup's LDS) the plan's table is generated on
     * the device at plan creation instead of being uploaded from the host. */
    AMQFT_FLAG_ONTHEFLY_CONSTANTS = 1u,
    /* Do not consult the tuning table; use the default launch shape. */
    AMQFT_FLAG_NO_AUTOTUNE = 2u,
    /* Use the multi-pass (global-memory) path even when a signal fits LDS.
     * For tests of that path at sizes where every variant is accurate. */
    AMQFT_FLAG_FORCE_MULTIPASS = 4u,
    /* Use the large-N path of variants 4 and 8 (top levels, rows, back
     * levels and chain over a global workspace) even when a signal fits
     * LDS: from N = 2^11, FP64 and FP32 storage only (AMQFT_ERR_UNSUPPORTED
     * otherwise, and together with AMQFT_FLAG_FORCE_MULTIPASS).  For tests of
     * that path at sizes where every variant is accurate. */
    AMQFT_FLAG_FORCE_LARGE = 8u,
    /* amqft_exec_adjoint runs the transposed flow graph of the plan's
     * variant instead of conjugating around its forward program.  The real
     * transpose of a program for F computes F^H (F is symmetric,
     * eq. qft_0A), and the transpose of variant 4's program is variant 2's
     * with the sign of i in the combine flipped (M4^T = M2, M8^T = M6,
     * M1^T = M3, M5^T = M7; skeleton A <-> B, Sec. 5-6), so the adjoint of a
     * variant-v plan runs the compile-time kernel of its dual variant.  For
     * N = 2^8 .. 2^14 (2^13 in FP64), where both kernels exist
     * (AMQFT_ERR_UNSUPPORTED otherwise and for many-length plans); the
     * forward transform is unchanged. */
    AMQFT_FLAG_TRANSPOSED_ADJOINT = 16u,
    /* In-place execution (Sec. 7.1: every variant can run in place; an
     * efficient in-place form is left open there).  amqft_exec,
     * amqft_exec_adjoint and amqft_exec_graph then require in == out
     * (AMQFT_ERR_INVALID_ARG otherwise).  Up to one workgroup's LDS (2^14
     * points, 2^13 in FP64) the kernels read each signal once and write it
     * once, with no workspace.  Above it, variants 4 and 8 with FP32
     * storage at N = 2^15 .. 2^17 (FP64 2^14 .. 2^16; with
     * AMQFT_FLAG_FORCE_LARGE from 2^11) keep the recursion's intermediate
     * rows in the signal's own buffer: the workspace is about 0.24 N values
     * a signal (the blocks the chain reads at folded indices, N/8 values,
     * and the row slots that two chain workgroups share) instead of 2 N,
     * and the transform moves the out-of-place path's bytes plus one copy
     * of those shared slots.  Other variants, sizes and storage types give
     * AMQFT_ERR_UNSUPPORTED above one workgroup's LDS, as do many-length
     * plans. */
    AMQFT_FLAG_IN_PLACE = 32u
};

/* Environment (read at plan creation):
 *   AMQFT_TUNE_CACHE   path of a JSON-lines file that keeps autotuned launch
 *                      shapes across processes (see amqft_plan_create_many);
 *   AMQFT_LARGE_WS_MB  size in MiB (1 .. 2^20) of each of the two workspace
 *                      buffers of the large-N plans of variants 4 and 8
 *                      (default 128; signals run in chunks that fit them). */

/* Largest supported log2(N). */
#define AMQFT_MAX_LOG2N 24

typedef struct amqft_plan_s *amqft_plan;

/* Plan for `batch` signals of length n stored back to back (stride n).
 * The plan owns the constant table and any workspace; it may be used for
 * any number of amqft_exec/amqft_exec_adjoint calls but not concurrently on
 * two streams (workspace is per plan).  batch = 0 is allowed (exec is then
 * a no-op).  On error *out is set to NULL. */
amqft_status amqft_plan_create(amqft_plan *out, int64_t n, int64_t batch,
                               amqft_variant variant, amqft_dtype dtype,
                               unsigned flags);

/* Real transforms of the same recursion (Sec. 3.1, Sec. 7.4: the CDFT is
 * D_c / D_r, one DCT-0, one DST-0 and the combine of eqs. qft_17-21; these
 * are the parts of it). */
typedef enum {
    /* R(k) = sum_n r(n) exp(-i 2 pi n k / n), k = 0 .. n/2, of a real signal
     * (eqs. qft_22 - qft_25: D_c / D_r, dct[n] and dst[n]): in n reals, out
     * n/2 + 1 interleaved complex values per signal. */
    AMQFT_RDFT = 0,
    /* The dct[n] function: S(k) = sum_{m=0}^{n/2} s(m) cos(2 pi m k / n),
     * k = 0 .. n/2: in and out n/2 + 1 reals per signal (eq. qft_0B). */
    AMQFT_DCT0 = 1,
    /* The dst[n] function: S(k) = sum_{m=1}^{n/2-1} s(m) sin(2 pi m k / n),
     * k = 1 .. n/2 - 1: in and out n/2 - 1 reals per signal (eq. qft_0C). */
    AMQFT_DST0 = 2
} amqft_real_kind;

/* Plan for `batch` real signals of one real transform of length n (the
 * periodization, a power of two, 4 <= n <= 2^14 for AMQFT_C64 = FP32 reals
 * and 2^13 for AMQFT_C128 = FP64 reals; AMQFT_ERR_UNSUPPORTED for other sizes
 * and storage types, and for the force flags).  Signals are stored back to
 * back with the strides given above, for input and output alike.  Executed by
 * amqft_exec; amqft_exec_adjoint gives the same result as amqft_exec for
 * AMQFT_DCT0 and AMQFT_DST0 (real symmetric matrices) and
 * AMQFT_ERR_UNSUPPORTED for AMQFT_RDFT.  Two real signals share one complex
 * lane of the recursion (its coefficients are real), so a batch costs about
 * half the complex transforms of its size. */
amqft_status amqft_plan_create_real(amqft_plan *out, int64_t n, int64_t batch,
                                    amqft_real_kind kind, amqft_variant variant,
                                    amqft_dtype dtype, unsigned flags);

/* Plan for `count` signals of (possibly different) power-of-two lengths in
 * one buffer: signal i has lengths_host[i] points and starts at complex
 * element offsets_host[i]; offsets_host has count+1 entries, is
 * non-decreasing, and offsets_host[i+1] - offsets_host[i] >= lengths_host[i]
 * (signals must not overlap).  Both arrays are host memory and are copied
 * into the plan.  Execution: the short lengths (up to 2^7 for variants 1, 2,
 * 4, 5, 6 and 8, up to 2^12 for 3 and 7) run in one persistent launch over a
 * work list sorted longest first; every longer length runs as one batched
 * launch sequence per length class over the same buffer (the classes that
 * need a global workspace on a second stream forked from, and joined back
 * into, `stream`).  The first out-of-place execution autotunes the
 * persistent grid, the multi-pass sub-block sizes and the signals per chunk
 * of the large-N classes (synchronising `stream`); an in-place execution
 * before it runs the default shapes. */
amqft_status amqft_plan_create_many(amqft_plan *out, int64_t count,
                                    const int64_t *lengths_host,
                                    const int64_t *offsets_host,
                                    amqft_variant variant, amqft_dtype dtype,
                                    unsigned flags);

/* X = F x (eq. qft_0A) for every signal of the plan, asynchronously on
 * `stream` (a hipStream_t; NULL = the default stream).  in_dev and out_dev
 * are device pointers to the interleaved complex data in the plan's dtype. */
amqft_status amqft_exec(amqft_plan plan, const void *in_dev, void *out_dev,
                        void *stream);

/* y = F^H g, the conjugate transpose (unnormalised): the inverse DFT times N.
 * Because the DFT matrix is symmetric, F^H g = conj(F conj(g)). */
amqft_status amqft_exec_adjoint(amqft_plan plan, const void *in_dev,
                                void *out_dev, void *stream);

/* Fused loss and gradient for loss = sum_b sum_k |w(b,k) * (F x_b)(k)|^2:
 * reads x (batch, n) and w (batch, n) (both in the plan's dtype), writes
 * grad_x = 2 F^H(|w|^2 * F x) (same layout) and the per-signal losses
 * loss_dev[b] (FP32, or FP64 for AMQFT_C128).  grad = dL/dRe + i dL/dIm.
 * Only plans made by amqft_plan_create with n >= 4 (AMQFT_ERR_UNSUPPORTED
 * otherwise); grad_dev may alias x_dev but not w_dev. */
amqft_status amqft_power_loss_grad(amqft_plan plan, const void *x_dev,
                                   const void *w_dev, void *grad_dev,
                                   void *loss_dev, void *stream);

/* Capture the plan's forward (adjoint = 0) or adjoint (adjoint = 1)
 * execution on the given buffers into a HIP graph owned by the plan, and
 * launch it on `stream`; later calls with the same buffers replay the graph.
 * The buffers are part of the graph: passing different pointers re-captures. */
amqft_status amqft_exec_graph(amqft_plan plan, const void *in_dev,
                              void *out_dev, int adjoint, void *stream);

/* Free the plan and its device memory.  The caller must have synchronised
 * every stream the plan ran on.  NULL is accepted. */
amqft_status amqft_plan_destroy(amqft_plan plan);

/* Write a one-line, NUL-terminated description of what the plan launches
 * (kernel name, grid, block, LDS bytes; or the multi-pass / many-length
 * structure) into buf[0 .. len).  Host only; no GPU work.  For reports and
 * profiles: the kernel name matches the one a profiler lists. */
amqft_status amqft_plan_describe(amqft_plan plan, char *buf, size_t len);

/* Bytes of device workspace owned by the plan (0 when none). */
amqft_status amqft_plan_workspace_size(amqft_plan plan, size_t *bytes);

/* Copy the plan's constant table for length n (n/4 entries, widened to
 * FP64 from the working precision the kernels read them in) into host
 * memory table_host[0 .. n/4).  Entry p holds f(2 pi p / n) for the
 * variant's family f in {2cos, 1/(2cos), 2sin, 1/(2sin)} (Sec. 7.1); entry 0
 * is unused.  Without AMQFT_FLAG_ONTHEFLY_CONSTANTS these are the host
 * values (long double, rounded once to the working precision); with it, the
 * values the device generated in FP64 (the same ones the LDS-resident
 * kernels generate per workgroup), read back with a synchronous copy
 * (AMQFT_ERR_HIP if it fails).  For tests of the constant generation. */
amqft_status amqft_plan_constants(amqft_plan plan, int64_t n, double *table_host,
                                  int64_t entries);

/* Bytes of the device array each GPU holds for amqft_exec_noalloc. */
#define AMQFT_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): X = F x (adjoint = 0) or
 * y = F^H g (adjoint = 1) of `batch` signals of length n (stride n) on the
 * current device, asynchronously on `stream`, with no plan and no
 * allocation of any kind.  Same kernels, same results (bit for bit) as a
 * plan made by amqft_plan_create with AMQFT_FLAG_ONTHEFLY_CONSTANTS:
 * constants are always generated on the device in FP64.  The paths above
 * one workgroup's LDS keep their workspace and constant table in a
 * file-scope device array of AMQFT_NOALLOC_SCRATCH_BYTES per GPU (held
 * until the process ends); signals run in chunks that fit it, and a length
 * whose single signal does not fit (n above 2^21 for FP32 storage, 2^20 for
 * FP64) returns AMQFT_ERR_UNSUPPORTED before any HIP call.  Every call on
 * one GPU uses the same array and leaves its contents behind (nothing in it
 * needs to start at zero): calls that overlap on one GPU (two streams, or
 * two host threads) race and must be serialised by the caller.  The first
 * call on a device resolves the array's address and sets kernel attributes
 * (no allocation).  in_dev == out_dev is allowed.  Errors as for
 * amqft_plan_create / amqft_exec. */
amqft_status amqft_exec_noalloc(int64_t n, int64_t batch, amqft_variant variant,
                                amqft_dtype dtype, int adjoint,
                                const void *in_dev, void *out_dev,
                                void *stream);

/* Static description of a status code. */
const char *amqft_status_string(amqft_status status);

/* Last HIP error string seen by this thread ("" if none). */
const char *amqft_last_hip_error(void);

/* Library version string. */
const char *amqft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AMQFT_H */
