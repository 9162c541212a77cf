/*
 * stockfft: batched complex-to-complex single-precision 1D FFTs on AMD
 * Instinct MI355X (gfx950), by Stockham autosort passes with radix-16/8/4/2
 * butterflies and, beside them, a four-step split through device memory.
 *
 * What is computed (arXiv 2603.27569, Section II-A, the DFT definition):
 *   forward  (FFT_FORWARD  = -1):  X[k] = sum_n x[n] exp(-2 pi i n k / N)
 *   backward (FFT_BACKWARD = +1):  X[k] = sum_n x[n] exp(+2 pi i n k / N)
 * Neither direction is scaled: backward(forward(x)) = N x.  The backward
 * transform is also the adjoint F^H of the forward one (F is symmetric).
 *
 * Data layout: interleaved complex64 (re, im as two float32), rows stored
 * one after another with no padding: element n of row b is at byte offset
 * (b * N + n) * 8.  Device pointers are device memory owned by the caller;
 * they must be 8-byte aligned.  Output is in natural order.
 *
 * Streams: every exec entry point takes a hipStream_t passed as void*
 * (NULL = the null stream), enqueues its kernels on it and returns without
 * synchronising.  Exec calls never allocate memory.
 *
 * Errors: every entry point returns an FFT_* status code; 0 is success.
 * Argument checks happen before any HIP call.  When a HIP call fails the
 * status is FFT_HIP_ERROR and fft_last_hip_error() returns the raw
 * hipError_t value of the calling thread.
 */
#ifndef STOCKFFT_H
#define STOCKFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stockfft_plan_s *fft_plan_t;
typedef struct stockfft_ragged_s *fft_ragged_plan_t;

enum fft_status {
  FFT_SUCCESS = 0,
  FFT_INVALID_SIZE = 1,      /* N not a power of two in [256, 2^20] ([256, 16384] ragged) */
  FFT_INVALID_BATCH = 2,     /* batch < 1, or batch * N * 8 overflows */
  FFT_INVALID_DIRECTION = 3, /* direction not FFT_FORWARD / FFT_BACKWARD */
  FFT_INVALID_POINTER = 4,   /* a required pointer is NULL */
  FFT_MISALIGNED = 5,        /* a data pointer is not 8-byte aligned */
  FFT_OVERLAP = 6,           /* input and output partially overlap */
  FFT_INVALID_PLAN = 7,      /* NULL, destroyed or foreign plan handle */
  FFT_NO_DEVICE = 8,         /* no HIP device is visible */
  FFT_ALLOC_FAILED = 9,      /* device allocation failed */
  FFT_HIP_ERROR = 10,        /* a HIP call failed; see fft_last_hip_error() */
  FFT_INVALID_ARGUMENT = 11, /* another argument is out of range */
  FFT_UNSUPPORTED = 12       /* the plan cannot run this operation */
};

#define FFT_FORWARD (-1)
#define FFT_BACKWARD (+1)

/* Algorithm selection for fft_plan_config. */
#define FFT_ALGO_AUTO 0        /* the tuned choice for (N, batch) */
#define FFT_ALGO_SINGLE_PASS 1 /* one dispatch, all passes on chip (Section IV-D rule 1) */
#define FFT_ALGO_FOUR_STEP 2   /* two dispatches through device memory (Section IV-B eq. (3)) */

/* Storage formats of fft_exec_io's buffers (arithmetic is FP32 in all). */
#define FFT_IO_C64 0   /* complex64: two float32 per value (fft_exec's format) */
#define FFT_IO_C16 1   /* two IEEE binary16 per value, real part first */
#define FFT_IO_BC16 2  /* two bfloat16 per value, real part first */
/* The same storage formats with the 16-point DFTs on the matrix cores (see
 * fft_exec_io). */
#define FFT_IO_C16_MMA 3
#define FFT_IO_BC16_MMA 4

/*
 * fft_plan -- create a plan for `batch` transforms of length `n`.
 * Section II-A (definition), Section IV-D (synthesis rules).
 *   plan       out: the new handle; set to NULL on any error.
 *   n          transform length, a power of two in [256, 1048576].  Up to
 *              16384 a whole transform fits in one CU's LDS and a single-pass
 *              kernel is available; above it only the four-step (eq. (3),
 *              Section IV-D rule 3) exists: N1 x 16384 with N1 <= 64, or
 *              N1 x N2 with N1, N2 in {256, 512, 1024}, whichever the tuned
 *              table names for (n, batch).
 *   batch      number of rows, >= 1.
 *   direction  FFT_FORWARD or FFT_BACKWARD.
 * The plan owns device memory for its twiddle tables (computed in FP64 on
 * the host and rounded once to FP32) and, for the four-step algorithm, a
 * workspace of batch * n * 8 bytes.  It belongs to the device that was
 * current when it was created.
 * With the environment variable STOCKFFT_LOG set (to anything but "" or
 * "0") every plan prints one line on stderr when it is created: its length,
 * batch, direction, algorithm, kernel variant, and the shapes of its fused,
 * matched-filter and 16-bit storage kernels.
 * Errors: FFT_INVALID_POINTER, FFT_INVALID_SIZE, FFT_INVALID_BATCH,
 * FFT_INVALID_DIRECTION, FFT_NO_DEVICE, FFT_ALLOC_FAILED, FFT_HIP_ERROR.
 */
int fft_plan(fft_plan_t *plan, int64_t n, int64_t batch, int direction);

/*
 * fft_plan_config -- fft_plan with an explicit algorithm and kernel variant.
 *   algorithm  FFT_ALGO_AUTO, FFT_ALGO_SINGLE_PASS or FFT_ALGO_FOUR_STEP.
 *   variant    NULL for the tuned choice, or a variant name listed by
 *              fft_variant_describe() of the matching kind and length.
 * Errors: as fft_plan, plus FFT_UNSUPPORTED (no four-step split for n, or
 * FFT_ALGO_SINGLE_PASS with n > 16384) and FFT_INVALID_ARGUMENT (unknown
 * algorithm or variant name).
 */
int fft_plan_config(fft_plan_t *plan, int64_t n, int64_t batch, int direction, int algorithm,
                    const char *variant);

/*
 * fft_exec -- run the plan: out = F in (or the backward transform).
 * Section II-B (Stockham autosort), Section V (passes and device bypass).
 *   in, out   caller-owned device buffers of batch * n complex64 values.
 *             in == out (in place) is allowed; any other overlap is not.
 *   stream    hipStream_t as void*, NULL for the null stream.
 * Asynchronous; does not allocate.  One plan must not run on two streams at
 * once (the four-step workspace is per plan); different plans are independent.
 * Errors: FFT_INVALID_PLAN, FFT_INVALID_POINTER, FFT_MISALIGNED,
 * FFT_OVERLAP, FFT_HIP_ERROR.
 */
int fft_exec(fft_plan_t plan, const void *in, void *out, void *stream);

/*
 * fft_exec_io -- fft_exec with 16-bit storage in HBM: in and out hold
 * batch * n complex values of `io` (FFT_IO_C16 or FFT_IO_BC16, 4 bytes per
 * value; FFT_IO_C64 is fft_exec itself).  Values are widened exactly on
 * load, every pass runs in FP32 with the plan's FP32 twiddles, and each
 * output is rounded once to the storage format (nearest even).  This halves
 * the bytes of a bandwidth-bound transform (the paper's future-work item on
 * mixed-precision storage, Section IX-A); the error is then that of one
 * rounding of the output, about 2^-11 (binary16) or 2^-8 (bfloat16) relative.
 * binary16 overflows to infinity above 65504: a bin can reach sqrt(n) times
 * the input row's 2-norm, so inputs must be scaled for that; bfloat16 has
 * float32's range.  Single-pass plans only (n <= 16384).  Asynchronous; does
 * not allocate.  in == out allowed.  The kernel shape is the plan's named
 * variant, else the 16-bit transform's own tuned choice
 * (fft_tune_query_storage16), which can differ from the FP32 one.
 * FFT_IO_C16_MMA / FFT_IO_BC16_MMA: the same storage for n = 16^P * RL
 * (512, 1024, 2048, 4096, 8192, 16384; any single-pass plan of those
 * lengths), with every 16-point DFT of the P radix-16 passes computed on the
 * matrix cores (the paper's matrix-multiply DFT, Sections V-C and VII-C,
 * with its batched and mixed-precision future-work items, Section IX-A)
 * and a last radix-RL pass (RL = 2, 4, 8) on the vector ALUs: twiddles are applied in FP32, then each
 * pass's inputs and the DFT matrix are rounded to the storage format and
 * multiplied with FP32 sums, so the error is that of one rounding per pass
 * plus the rounded matrix's instead of one rounding in all.
 * Errors: FFT_INVALID_PLAN, FFT_INVALID_ARGUMENT (unknown io),
 * FFT_UNSUPPORTED (four-step plan; for the MMA formats also another length),
 * FFT_INVALID_POINTER, FFT_MISALIGNED (not 4-byte aligned),
 * FFT_OVERLAP, FFT_HIP_ERROR.
 */
int fft_exec_io(fft_plan_t plan, const void *in, void *out, int io, void *stream);

/*
 * fft_destroy -- free the plan's device memory.  The caller must ensure no
 * exec that uses the plan is still in flight.  NULL is a no-op; a second
 * destroy of the same handle returns FFT_INVALID_PLAN.
 */
int fft_destroy(fft_plan_t plan);

/*
 * fft_exec_spectral_energy -- fused forward transform, weighting and adjoint
 * in one kernel, for L = sum_b sum_k w_k^2 |(F x_b)[k]|^2 (a differentiable
 * use of the transform; F^H is the adjoint of Section II-A's F).
 *   plan        a forward, single-pass plan of length n and batch rows.  The
 *               kernel's shape is the plan's variant when one was named, else
 *               this kernel's own tuned choice (fft_tune_query_fused): it runs
 *               two transforms per load and may prefer another shape than the
 *               plain transform.
 *   x           device, batch * n complex64.
 *   w           device, n float32 spectral weights shared by every row.
 *   grad_scale  device, one float32 multiplying the gradient, or NULL for 1.
 *   grad_x      device, batch * n complex64 output
 *               grad_scale * F^H(2 w^2 .* F x_b) = dL/dRe x + i dL/dIm x,
 *               or NULL to compute the loss only (forward passes only).
 *   row_loss    device, batch float32: the per-row sums.  Required.
 *   loss_total  device, one float32 receiving sum_b row_loss[b] (a fixed-order
 *               tree, bitwise reproducible), or NULL.  The kernel's last
 *               workgroup writes it, counting arrivals on counters the plan
 *               owns: calls on one plan must not run concurrently (different
 *               streams without ordering between them race).
 * Errors: FFT_INVALID_PLAN, FFT_INVALID_POINTER, FFT_MISALIGNED,
 * FFT_OVERLAP (grad_x partially overlapping x), FFT_UNSUPPORTED (backward or
 * four-step plan), FFT_HIP_ERROR.
 */
int fft_exec_spectral_energy(fft_plan_t plan, const void *x, const float *w,
                             const float *grad_scale, void *grad_x, float *row_loss,
                             float *loss_total, void *stream);

/*
 * fft_exec_spectral_energy_noalloc -- fft_exec_spectral_energy for callers
 * that cannot allocate device memory around the call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * per-row losses and the arrival counters of the loss total live in a
 * static device array of the library instead of a caller buffer and the
 * plan's counters.  The array is 4 MiB + 4 KiB, one copy on each GPU the
 * call runs on, held until the process ends; the first call on a GPU looks
 * up its address and clears its counters with a small kernel on `stream`.
 *   plan, x, w, grad_scale, grad_x, stream   as fft_exec_spectral_energy.
 *   loss_total  device, one float32 receiving sum_b of the row losses
 *               (required; the row losses themselves are not returned).
 * The plan's batch must be at most 1048576 rows (FFT_INVALID_ARGUMENT).
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (two streams without ordering, two host threads) race, and the
 * caller must order them.  Allocates nothing (no hipMalloc, hipFree or
 * allocating library routine); asynchronous.
 * Errors: FFT_INVALID_PLAN, FFT_INVALID_POINTER, FFT_INVALID_ARGUMENT,
 * FFT_MISALIGNED, FFT_OVERLAP, FFT_UNSUPPORTED (backward or four-step
 * plan), FFT_HIP_ERROR.
 */
int fft_exec_spectral_energy_noalloc(fft_plan_t plan, const void *x, const float *w,
                                     const float *grad_scale, void *grad_x, float *loss_total,
                                     void *stream);

/*
 * fft_exec_matched_filter -- fused range compression (the paper's future
 * work on SAR pipeline fusion, Section IX-A): out_b = F^{-1}(conj(h) .* F x_b)
 * with F^{-1} = backward / N, in one kernel.
 *   plan   a forward, single-pass plan; the kernel's shape is the plan's
 *          variant when one was named, else fft_tune_query_filter's choice
 *          (its twiddles are built with the plan).
 *   x      device, batch * n complex64;  h  device, n complex64 filter spectrum;
 *   out    device, batch * n complex64 (may equal x).
 * Errors: as fft_exec_spectral_energy.
 */
int fft_exec_matched_filter(fft_plan_t plan, const void *x, const void *h, void *out,
                            void *stream);

/*
 * fft_plan_ragged -- plan a ragged batch: `count` transforms of different
 * power-of-two lengths, packed one after another in one buffer (transform i
 * starts at element offset sum_{j<i} sizes[j]).  All run in one persistent
 * kernel launch, captured once in a hipGraph.  Each length runs with its
 * own tuned shape; the transforms are grouped into tasks of about equal
 * cost, dealt to the workgroups (two per CU) once, here, by a longest-first
 * list schedule on measured task costs (no device queue or atomic).
 *   sizes      host array of `count` lengths, each a power of two in
 *              [256, 16384]; copied, the caller keeps ownership.
 *   count      >= 1.
 *   direction  FFT_FORWARD or FFT_BACKWARD.
 * The plan owns its task lists, twiddle tables and graph.
 * Errors: FFT_INVALID_POINTER, FFT_INVALID_SIZE (with the first bad entry),
 * FFT_INVALID_BATCH (count < 1), FFT_INVALID_DIRECTION, FFT_NO_DEVICE,
 * FFT_ALLOC_FAILED, FFT_HIP_ERROR.
 */
int fft_plan_ragged(fft_ragged_plan_t *plan, const int64_t *sizes, int64_t count, int direction);

/*
 * fft_exec_ragged -- run a ragged plan: out = F in for every packed
 * transform.  in/out: device, sum(sizes) complex64, 8-byte aligned; in == out
 * allowed.  The first call on a stream instantiates the graph; later calls
 * update its pointer arguments and relaunch it.  Asynchronous; the plan must
 * not run on two streams at once (calls rewrite its one graph's arguments).
 * Errors: FFT_INVALID_PLAN, FFT_INVALID_POINTER, FFT_MISALIGNED, FFT_OVERLAP,
 * FFT_HIP_ERROR.
 */
int fft_exec_ragged(fft_ragged_plan_t plan, const void *in, void *out, void *stream);

/*
 * fft_exec_ragged_direct -- the same persistent kernel as fft_exec_ragged,
 * started with a plain kernel launch instead of the plan's graph (for callers
 * that capture it into a graph of their own, or that want the lower launch
 * cost: about 5 us less per call on ROCm 7 with one MI355X).  Same arguments,
 * results and errors as fft_exec_ragged; the plan's graph is not touched.
 */
int fft_exec_ragged_direct(fft_ragged_plan_t plan, const void *in, void *out, void *stream);

/*
 * fft_exec_ragged_plain -- the same ragged batch by plain launches: one
 * single-pass launch per transform size over rows that the caller has
 * grouped by size (the comparison baseline).  `in_by_size[s]`/`out_by_size[s]`
 * (s = log2(N) - 8, 7 entries, NULL when no transform has that size) each hold
 * the rows of one size contiguously, in plan order.
 */
int fft_exec_ragged_plain(fft_ragged_plan_t plan, const void *const *in_by_size,
                          void *const *out_by_size, void *stream);

/* fft_destroy_ragged -- free a ragged plan (NULL is a no-op). */
int fft_destroy_ragged(fft_ragged_plan_t plan);

/*
 * Ragged shapes.  Each size has one or more compiled shapes for the
 * persistent kernel (radix of the passes, lanes per transform, transforms
 * per task, hence the LDS tile); the autotuner picks one per size.
 * fft_ragged_shapes: comma-separated shape names for length n, into buf.
 * fft_tune_set_ragged: use `shape` for length n in ragged plans made later.
 * fft_tune_query_ragged: the shape ragged plans would use for n, into buf.
 * fft_tune_clear_ragged: back to the built-in shapes (the tuned MI355X choice).
 * Host only.  Errors: FFT_INVALID_POINTER, FFT_INVALID_SIZE,
 * FFT_INVALID_ARGUMENT (unknown shape, shape for another length, small buffer).
 */
int fft_ragged_shapes(int64_t n, char *buf, int64_t cap);
int fft_tune_set_ragged(int64_t n, const char *shape);
int fft_tune_query_ragged(int64_t n, char *buf, int64_t cap);
int fft_tune_clear_ragged(void);

/*
 * Tuning.  fft_tune_load reads a JSON file written by the project's
 * autotuner: {"arch": "gfx950", "entries": [{"n": N, "batch_min": a,
 * "batch_max": b, "variant": "<name>"}, ...]}, with "filter_entries" and
 * "fused_entries" of the same form for the two fused kernels and "ragged":
 * [{"n": N, "shape": "<name>"}, ...] for ragged plans.  A missing or unreadable
 * file, or one tuned for another architecture, leaves the built-in table in
 * force and returns FFT_INVALID_ARGUMENT; so does a file whose "cus" differs
 * from the device's compute-unit count.  Entries naming unknown variants
 * are skipped.  fft_tune_set adds one entry; fft_tune_clear drops all.
 * Later entries win.  Plans made before a change keep their variant.
 */
int fft_tune_load(const char *json_path);
int fft_tune_set(int64_t n, int64_t batch_min, int64_t batch_max, const char *variant);
int fft_tune_clear(void);

/*
 * fft_tune_query -- the single-pass variant name that fft_plan would choose
 * for (n, batch), written NUL-terminated into buf (cap bytes).  Host only.
 * Errors: FFT_INVALID_POINTER, FFT_INVALID_SIZE, FFT_INVALID_BATCH,
 * FFT_INVALID_ARGUMENT (buffer too small).
 */
int fft_tune_query(int64_t n, int64_t batch, char *buf, int64_t cap);

/*
 * fft_tune_query_filter -- the single-pass variant whose fused kernel
 * fft_exec_matched_filter would use for a forward plan of (n, batch) made
 * without an explicit variant (the matched filter is tuned on its own: it
 * runs two transforms per load and may prefer another shape than the plain
 * transform).  The tune file's "filter_entries" take precedence over the
 * built-in table.  Host only.  Errors: as fft_tune_query (n must be at most
 * 16384).
 */
int fft_tune_query_filter(int64_t n, int64_t batch, char *buf, int64_t cap);

/*
 * fft_tune_query_fused -- the same for the fused forward -> weight -> adjoint
 * kernel of fft_exec_spectral_energy, tuned on its own ("fused_entries" in a
 * tune file).  Host only.  Errors: as fft_tune_query_filter.
 */
int fft_tune_query_fused(int64_t n, int64_t batch, char *buf, int64_t cap);

/*
 * fft_tune_query_storage16 -- the same for fft_exec_io's 16-bit storage
 * formats FFT_IO_C16 and FFT_IO_BC16 ("storage16_entries" in a tune file),
 * for plans of either direction.  Host only.  Errors: as
 * fft_tune_query_filter.
 */
int fft_tune_query_storage16(int64_t n, int64_t batch, char *buf, int64_t cap);

/*
 * fft_set_launch_limit -- largest grid (in workgroups) one kernel launch may
 * use; bigger batches are split into several launches on the same stream.
 * Default 2^20; a value <= 0 restores it.  Affects launches made after the
 * call.  Exists so the splitting path can be exercised at small sizes.
 */
int fft_set_launch_limit(int64_t max_groups);

/*
 * Introspection (host only; the variant calls need no device).
 * fft_variant_count: number of compiled kernel variants.
 * fft_variant_describe: JSON text for variant `index` into buf (cap bytes,
 *   NUL-terminated); returns FFT_INVALID_ARGUMENT for a bad index or a
 *   buffer that is too small.  A single-pass variant states its shape
 *   (values_per_lane, lanes_per_transform, transforms_per_workgroup,
 *   radices, lds_layout, exchange_rounds, barriers, twiddle_schedule, ...),
 *   whether it has the fused forward -> weight -> adjoint kernel
 *   ("fused_kernel") and also the matched filter ("fused_kernels"), its
 *   persistent workgroups per CU ("streamed", 0 for a workgroup per row)
 *   and, for the in-wave exchange shapes at N = 4096, the groups and
 *   members of a group per lane ("wave_exchange", "wave_members"; 0 for
 *   shapes that exchange through the LDS only).
 * fft_variant_twiddles: the FP32 twiddle table of variant `index` as built
 *   for the device (interleaved re, im; forward direction), written into
 *   out[0 .. 2*count); *count receives the number of complex entries.
 *   With out == NULL only *count is set.
 * fft_plan_describe: JSON text describing a plan: its variant, and for a
 *   single-pass variant "variant_resources" (VGPRs, scratch bytes per lane,
 *   static LDS bytes and the largest workgroup of its forward FP32 kernel,
 *   as the HIP runtime reports them for the plan's device), the matched-
 *   filter, fused and 16-bit storage shapes.  Errors: FFT_INVALID_PLAN, or
 *   FFT_INVALID_ARGUMENT for a buffer that is too small.
 */
int fft_variant_count(void);
int fft_variant_describe(int index, char *buf, int64_t cap);
int fft_variant_twiddles(int index, float *out, int64_t cap_complex, int64_t *count);
int fft_plan_describe(fft_plan_t plan, char *buf, int64_t cap);

const char *fft_status_string(int status);
int fft_last_hip_error(void);
int fft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STOCKFFT_H */
