/*
 * stockref: measurement references beside the transform library (a separate
 * shared library, libstockref.so).  None of these calls is part of the
 * transform path; they exist so the transform's time can be compared with
 * kernels of known, simpler work on the same device, and so the time of a
 * transform's phases can be read off one workgroup at a time.
 *
 * The paper's methodology (Section VI-A) times the GPU kernels alone; these
 * references give the two figures that frame such a time on this device:
 * the cost of a launch that does nothing, and the time to move the same
 * bytes with no arithmetic, in the same launch shape.
 *
 * Conventions as in stockfft.h: device pointers are caller-owned device
 * memory, streams are hipStream_t passed as void* (NULL = null stream),
 * calls are asynchronous, never allocate, and return an FFT_* status code
 * (0 on success; FFT_INVALID_ARGUMENT / FFT_INVALID_POINTER /
 * FFT_MISALIGNED for bad arguments, checked before any HIP call;
 * FFT_HIP_ERROR when a launch fails, with the raw code from
 * ref_last_hip_error()).
 */
#ifndef STOCKREF_H
#define STOCKREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * ref_empty -- launch a kernel of `groups` workgroups of `threads` lanes
 * (1 <= threads <= 1024, 1 <= groups <= 2^31 - 1) whose body is empty: the
 * fixed cost of one dispatch.
 */
int ref_empty(int64_t groups, int threads, void *stream);

/*
 * ref_copy_rows -- copy `batch` rows of `n` complex64 values from `in` to
 * `out` in the single-pass transform's launch shape: one workgroup of
 * `lanes` lanes per row, lane t moving the values t + m * lanes (m < n /
 * lanes) with the transform's streaming 8-byte loads and stores.  Shapes:
 * (n, lanes) in {(4096, 256), (4096, 512), (4096, 1024), (1024, 64),
 * (16384, 1024)}; anything else gives FFT_INVALID_ARGUMENT.  in and out
 * must not overlap and must be 8-byte aligned.
 */
int ref_copy_rows(const void *in, void *out, int64_t n, int64_t batch, int lanes, void *stream);

/*
 * ref_copy_wide -- copy `bytes` bytes (a multiple of 16, >= 16) with
 * 16-byte streaming loads and stores, one per lane, 256 lanes per
 * workgroup, 16 values per lane: a grid of bytes / 65536 workgroups
 * (rounded up; the tail is bounds-checked).  16-byte aligned, no overlap.
 */
int ref_copy_wide(const void *in, void *out, int64_t bytes, void *stream);

/*
 * ref_weight_energy -- the middle step of the unfused gradient chain
 * (forward transform, this, adjoint transform) for the loss
 * L = sum_b sum_k w_k^2 |y_b[k]|^2: in place, y_b[k] <- 2 w_k^2 y_b[k], and
 * row_loss[b] = sum_k w_k^2 |y_b[k]|^2 (the values before scaling).
 *   y         device, batch * n complex64 (8-byte aligned);
 *   w         device, n float32;  row_loss  device, batch float32.
 * n a power of two in [256, 16384]; batch >= 1.
 */
int ref_weight_energy(void *y, const float *w, float *row_loss, int64_t n, int64_t batch,
                      void *stream);

/*
 * ref_filter_multiply -- the middle step of the unfused range-compression
 * chain: in place, y_b[k] <- conj(h_k) y_b[k] / n.  y: batch * n complex64,
 * h: n complex64, both device, 8-byte aligned; n a power of two in
 * [256, 16384]; batch >= 1.
 */
int ref_filter_multiply(void *y, const void *h, int64_t n, int64_t batch, void *stream);

/*
 * ref_lds_exchange -- the LDS roof of the transform's exchange: `groups`
 * workgroups of 256 lanes (1 <= groups <= 2^31 - 1), each doing `rounds`
 * (>= 0) exchanges of 32 KiB -- every lane writes 16 values of 8 bytes to
 * LDS, a barrier, every lane reads 16 values another lane wrote, a barrier
 * -- and nothing else.  Bank-conflict free.  Each round moves 64 KiB of LDS
 * traffic per workgroup (32 KiB written, 32 KiB read).  out: device,
 * groups * 256 float32 (4-byte aligned), caller-owned; out[g * 256 + t] =
 * 16 ((t + rounds) mod 256) + 120, the sum of the real parts lane t holds at
 * the end (lane t starts with t + m, m < 16, and every round passes each
 * lane's values to lane t - 1).
 */
int ref_lds_exchange(int64_t groups, int rounds, float *out, void *stream);

/*
 * ref_timeline -- run the single-pass transform of variant `variant` (one
 * of the names ref_timeline_variants lists) on `batch` rows, as fft_exec
 * would, with clock readings taken at the phase boundaries of every wave.
 *   tw       device, the variant's twiddle table (fft_variant_twiddles);
 *   inverse  0 forward, 1 backward;
 *   stamps   device, uint64_t[groups * waves * 32], groups = batch (one
 *            transform per workgroup), waves = the variant's lanes / 64.
 *            For wave v of workgroup g, stamps[(g * waves + v) * 32 + i]
 *            holds for i < 16 the 100 MHz real-time counter and for
 *            i >= 16 the shader clock counter, at mark i mod 16:
 *            0 entry, 1 input loads (and the twiddle loads a shape issues
 *            with them) landed, 2 .. 2P the pass marks (after
 *            pass p's arithmetic: 2p + 2; after the exchange that follows
 *            it: 2p + 3), 2P + 1 stores issued, 2P + 2 stores completed.
 *            Unused slots are 0.  For the in-wave exchange shapes (names
 *            ending in _wx1 or _wm2) the exchanges after passes 0 and 2 are
 *            the register transposes and the one after pass 1 the LDS.
 * The readings wait for the memory operations in flight at each mark, so
 * the timed kernel runs somewhat slower than the plain one.
 */
int ref_timeline(const char *variant, const void *in, void *out, const void *tw, int64_t batch,
                 int inverse, uint64_t *stamps, void *stream);

/* ref_timeline_variants -- comma-separated names into buf (cap bytes). */
int ref_timeline_variants(char *buf, int64_t cap);

int ref_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STOCKREF_H */
