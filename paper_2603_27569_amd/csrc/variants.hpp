// Host-visible description of every compiled kernel variant.
//
// A single-pass variant is one Stockham shape (N, values per lane E, lanes per
// transform T = N/E, transforms per workgroup, LDS pad, radix sequence)
// compiled for both directions.  The planner and the autotuner pick among
// them per size; the four-step, fused and ragged paths reuse the same shapes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stockfft {

constexpr int kMaxPasses = 8;

// Grids larger than this many workgroups are split into several launches.
constexpr int64_t kDefaultMaxGroupsPerLaunch = int64_t(1) << 20;
// Lengths: single pass up to kMaxSinglePassN (a whole transform in LDS), the
// four-step above it, up to kMaxN.
constexpr int64_t kMaxSinglePassN = 16384;
constexpr int64_t kMaxN = int64_t(1) << 20;
int64_t max_groups_per_launch();
void set_max_groups_per_launch(int64_t groups);
// Compute units of the current device (cached per device).
int device_cus();

using LaunchFn = hipError_t (*)(const void* in, void* out, const void* tw, int64_t batch,
                                bool inverse, hipStream_t s);

// Fused forward -> weight -> adjoint: grad = scale * F^H(2 w^2 .* F x) and
// row_loss[b] = sum_k w_k^2 |(F x_b)[k]|^2.  grad may be null (loss only).
// With total non-null the last workgroup to finish also writes sum_b
// row_loss[b] there; counters is plan-owned zeroed device memory of
// kTotalGroups * 64 + 1 words, left zeroed.
constexpr unsigned kTotalGroups = 16;  // first-level counters of the fused loss total
using FusedFn = hipError_t (*)(const void* x, const float* w, const float* scale, void* grad,
                               float* row_loss, float* total, unsigned* counters, const void* tw,
                               int64_t batch, hipStream_t s);

// Fused matched filter: out = (1/N) F^H(conj(h) .* F x).
using FilterFn = hipError_t (*)(const void* x, const void* h, void* out, const void* tw,
                                int64_t batch, hipStream_t s);

struct SingleVariant {
  const char* name;
  int n, e, t, tpb, padlog, npass;
  int radix[kMaxPasses];
  int chunks;  // exchange rounds per pass (the LDS holds N / chunks elements per transform)
  bool double_buffered;  // exchanges alternate between two LDS buffers
  int twiddle_schedule;  // 0 at their pass, 1 one pass ahead, 2 all with the input
  bool paired_twiddles;  // table layout: two twiddles per 16-byte entry (PairedTwiddles)
  bool paired_lanes;     // first/last pass in the paired butterfly order (PairedLanes)
  int streamed;          // 0: a workgroup per transform; k: k persistent workgroups per CU (Streamed)
  int wave_exchange;     // 0: every exchange through the LDS; G: in-wave exchanges, G groups per lane (WaveExchange)
  int wave_members;      // with in-wave exchanges: members of each group per lane (1 or 2)
  int threads;
  int lds_bytes;
  int tw_elems;
  LaunchFn launch;
  FusedFn fused;     // null when not compiled for this variant
  FilterFn filter;   // null when not compiled for this variant
  // The same transform with 16-bit storage (FP32 arithmetic): complex values
  // in HBM as IEEE half pairs (launch_f16) or bfloat16 pairs (launch_bf16).
  LaunchFn launch_f16;
  LaunchFn launch_bf16;
  // The forward FP32 kernel itself, for resource queries (hipFuncGetAttributes).
  const void* kernel;
};

extern const SingleVariant kSingleVariants[];
extern const int kNumSingleVariants;

// Four-step second stage: Z[b][k2 + N2 k1] = sum_{n1} W_N1^{n1 k1} W_N^{n1 k2} Y[b][n1][k2]
// (tw: the sub-transform table, used by second stages that run it too; tw4:
// the stage's own table).
using FourStepCombineFn = hipError_t (*)(const void* y, void* out, const void* tw, const void* tw4,
                                         int64_t batch, bool inverse, hipStream_t s);
// Four-step first stage: Y[b][n1][.] = FFT_N2(x[b][n1 + N1 m], m = 0..N2-1)
using FourStepColumnsFn = hipError_t (*)(const void* x, void* y, const void* tw, int64_t batch,
                                         bool inverse, hipStream_t s);

struct FourStepVariant {
  const char* name;
  int n, n1, n2;
  const char* sub_name;  // single-pass shape of the length-N2 sub-transforms
  int tw_sub_elems;
  FourStepColumnsFn columns;
  FourStepCombineFn combine;
  // Twiddle layout of the second stage: false -- the full table
  // [n1 - 1][k2] = W_N^{n1 k2}; true (large N) -- W_N^m as the product of
  // two short tables, lo[j] = W_N^j (j < 2^s) and hi[j] = W_N^{j 2^s}
  // (j < N / 2^s), s = floor(log2 N / 2), followed by W_N1^j (j < N1).
  bool two_level;
  // Tiled splits with N1 != N2: the N1-point single-pass shape whose table
  // the second stage runs on, appended to the stage table (else null).
  const char* sub2_name;
};

const FourStepVariant* four_step_variants(int* count);

}  // namespace stockfft
