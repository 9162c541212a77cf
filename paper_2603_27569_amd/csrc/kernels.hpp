// Kernels of the plain, 16-bit storage, fused and four-step paths, templated
// on a Stockham Shape (stockham.hpp).  Each kernel is launched by a small host wrapper that
// splits very large batches into several grids.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "stockham.hpp"
#include "variants.hpp"

namespace stockfft {

// Streaming (nontemporal) global accesses for the transform data: every input
// element is read once and every output element written once, so the hint
// keeps them from displacing the shared twiddle tables and lets the output
// drain to memory while the kernel still runs instead of at its end.  The
// four-step's stride-N1 column loads keep ordinary accesses (their cache
// lines are shared between workgroups; the hint there cost up to 1.5x at
// N = 2^20), and so does its workspace, which the second stage reads back;
// its final stores stream.
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ c32 load_stream(const c32* p) {
  const f32x2 v = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(p));
  return c32{v.x, v.y};
}
__device__ __forceinline__ void store_stream(c32* p, c32 a) {
  const f32x2 v = {a.x, a.y};
  __builtin_nontemporal_store(v, reinterpret_cast<f32x2*>(p));
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Row position of register slot m for the first pass's inputs (in_position)
// and the last pass's outputs (out_position): t + m T, or the paired order.
template <class S>
__device__ __forceinline__ int in_position(int t, int m) { return read_position<S, 0>(t, m); }
template <class S>
__device__ __forceinline__ int out_position(int t, int m) { return read_position<S, S::P - 1>(t, m); }

// Loads one row unconditionally: a slot past the last row is pointed at a
// row that exists (its result is never stored), which costs nothing, where
// zeroing its registers costs one instruction per register on every lane.
template <class S>
__device__ __forceinline__ void global_load_row(c32 (&a)[S::E], const c32* src, int t) {
  if constexpr (paired_pass<S, 0>()) {
    // slots m and m + 1 (m even) are adjacent elements: one 16-byte load
#pragma unroll
    for (int m = 0; m < S::E; m += 2) {
      const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(src + in_position<S>(t, m)));
      a[m] = c32{v.x, v.y};
      a[m + 1] = c32{v.z, v.w};
    }
  } else {
#pragma unroll
    for (int m = 0; m < S::E; ++m) a[m] = load_stream(src + t + m * S::T);
  }
}

// The same through one buffer descriptor over the workgroup's rows: lane_row
// is the lane's row offset from the descriptor's base in elements.  Both
// orders of register slots are lane part + slot part (position(t, m) =
// position(t, 0) + position(0, m)), the slot part a constant.
template <class S>
__device__ __forceinline__ void buffer_load_row(c32 (&a)[S::E], const Buf& b, int lane_row, int t) {
  const int voff = 8 * (lane_row + in_position<S>(t, 0));
  if constexpr (paired_pass<S, 0>()) {
#pragma unroll
    for (int m = 0; m < S::E; m += 2) {
      const u32x4 v = b.ld128<kNT>(voff, 8 * in_position<S>(0, m));
      a[m] = c32{__uint_as_float(v.x), __uint_as_float(v.y)};
      a[m + 1] = c32{__uint_as_float(v.z), __uint_as_float(v.w)};
    }
  } else {
#pragma unroll
    for (int m = 0; m < S::E; ++m) {
      const u32x2 v = b.ld64<kNT>(voff, 8 * in_position<S>(0, m));
      a[m] = c32{__uint_as_float(v.x), __uint_as_float(v.y)};
    }
  }
}
template <class S>
__device__ __forceinline__ void buffer_store_row(const c32 (&a)[S::E], const Buf& b, int lane_row,
                                                 int t, bool live) {
  if (!live) return;
  const int voff = 8 * (lane_row + out_position<S>(t, 0));
  if constexpr (paired_pass<S, S::P - 1>()) {
#pragma unroll
    for (int m = 0; m < S::E; m += 2)
      b.st128<kNT>(u32x4{__float_as_uint(a[m].x), __float_as_uint(a[m].y), __float_as_uint(a[m + 1].x),
                         __float_as_uint(a[m + 1].y)},
                   voff, 8 * out_position<S>(0, m));
  } else {
#pragma unroll
    for (int m = 0; m < S::E; ++m)
      b.st64<kNT>(u32x2{__float_as_uint(a[m].x), __float_as_uint(a[m].y)}, voff, 8 * out_position<S>(0, m));
  }
}

// Every launcher gives a workgroup TPB consecutive rows from a grid of
// ceil(rows / TPB) workgroups, so with one transform per workgroup every row
// is live; only the last workgroup of a TPB > 1 shape can hold dead slots.
// Those load the last row (row_src) and store nothing.
template <class S>
__device__ __forceinline__ bool row_live(int64_t row, int64_t rows) {
  return S::TPB == 1 || row < rows;
}
template <class S>
__device__ __forceinline__ int64_t row_src(int64_t row, int64_t rows) {
  return row_live<S>(row, rows) ? row : rows - 1;
}
// The element offset of a slot's source row from its workgroup's first row
// (below TPB N, so a 32-bit buffer offset).
template <class S>
__device__ __forceinline__ int slot_src(int slot, int64_t row, int64_t rows) {
  return S::TPB == 1 ? 0 : (int)(row_src<S>(row, rows) - (row - slot)) * S::N;
}

template <class S, bool STREAM = true>
__device__ __forceinline__ void global_store_row(const c32 (&a)[S::E], c32* dst, int t, bool live) {
  if (live) {
    if constexpr (paired_pass<S, S::P - 1>()) {
      static_assert(STREAM, "paired stores stream");
#pragma unroll
      for (int m = 0; m < S::E; m += 2) {
        const f32x4 v = {a[m].x, a[m].y, a[m + 1].x, a[m + 1].y};
        __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(dst + out_position<S>(t, m)));
      }
    } else {
#pragma unroll
      for (int m = 0; m < S::E; ++m) {
        if constexpr (STREAM)
          store_stream(dst + t + m * S::T, a[m]);
        else
          dst[t + m * S::T] = a[m];
      }
    }
  }
}

// ------------------------------------------------------------ single pass
// One dispatch per batch (the paper's synthesis rule 1, Section IV-D): each
// workgroup owns TPB whole transforms; every pass stays on chip.
template <class S, bool INV>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_stockham(const c32* in, c32* out,
                                                         const c32* tw, int64_t rows) {
  __shared__ alignas(16) c32 lds_all[S::TPB * S::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int slot = S::TPB == 1 ? 0 : tid / S::T;  // one transform: the row base is uniform
  const int t = tid - slot * S::T;
  const int64_t row = (int64_t)blockIdx.x * S::TPB + slot;
  const bool live = row_live<S>(row, rows);
  const int64_t row0 = (int64_t)blockIdx.x * S::TPB;
  c32* lds = lds_all + slot * S::LDS_ELEMS;
  c32 a[S::E];
  buffer_load_row<S>(a, Buf(in + row0 * S::N), slot_src<S>(slot, row, rows), t);
  run_passes<S, INV>(a, lds, tw, t);
  buffer_store_row<S>(a, Buf(out + row0 * S::N), slot * S::N, t, live);
}

template <class S>
hipError_t launch_single(const void* in, void* out, const void* tw, int64_t batch, bool inverse,
                         hipStream_t s) {
  const int64_t groups = (batch + S::TPB - 1) / S::TPB;
  const int64_t cap = max_groups_per_launch();
  for (int64_t g0 = 0; g0 < groups; g0 += cap) {
    const int64_t g = groups - g0 < cap ? groups - g0 : cap;
    const int64_t r0 = g0 * S::TPB;
    const c32* ip = static_cast<const c32*>(in) + r0 * S::N;
    c32* op = static_cast<c32*>(out) + r0 * S::N;
    const c32* twp = static_cast<const c32*>(tw);
    if (inverse)
      k_stockham<S, true><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(ip, op, twp, batch - r0);
    else
      k_stockham<S, false><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(ip, op, twp, batch - r0);
  }
  return hipGetLastError();
}

// ------------------------------------------------------ 16-bit storage
// 16-bit storage formats: one complex value in 4 bytes (real in the low
// half).  Loads widen exactly to FP32; stores round to nearest even.
struct IoF16 {
  static constexpr int BYTES = 4;
  __device__ __forceinline__ static c32 load(uint32_t v) {
    const float2 f = __half22float2(*reinterpret_cast<const __half2*>(&v));
    return c32{f.x, f.y};
  }
  __device__ __forceinline__ static uint32_t store(c32 a) {
    const __half2 h = __floats2half2_rn(a.x, a.y);
    return *reinterpret_cast<const uint32_t*>(&h);
  }
};

struct IoBF16 {
  static constexpr int BYTES = 4;
  __device__ __forceinline__ static c32 load(uint32_t v) {
    return c32{__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
  }
  // gfx950 converts a pair in one instruction (v_cvt_pk_bf16_f32), rounding
  // to nearest even.
  __device__ __forceinline__ static uint32_t store(c32 a) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{a.x, a.y}, b2));
  }
};

// The single-pass transform with 16-bit storage: the rows are widened on
// load, every pass runs in FP32, and the result is rounded once on store.
template <class S, bool INV, class IO>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_stockham_io(const uint32_t* in,
                                                                    uint32_t* out, const c32* tw,
                                                                    int64_t rows) {
  __shared__ alignas(16) c32 lds_all[S::TPB * S::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int slot = S::TPB == 1 ? 0 : tid / S::T;  // one transform: the row base is uniform
  const int t = tid - slot * S::T;
  const int64_t row = (int64_t)blockIdx.x * S::TPB + slot;
  const bool live = row_live<S>(row, rows);
  const int64_t row0 = (int64_t)blockIdx.x * S::TPB;
  c32* lds = lds_all + slot * S::LDS_ELEMS;
  c32 a[S::E];
  {
    // 4 bytes per value; lane part + constant slot part as in buffer_load_row
    const Buf src(in + row0 * S::N);
    const int voff = 4 * (slot_src<S>(slot, row, rows) + in_position<S>(t, 0));
    if constexpr (paired_pass<S, 0>()) {
      // slots m and m + 1 (m even) are adjacent values: one 8-byte load
#pragma unroll
      for (int m = 0; m < S::E; m += 2) {
        const u32x2 v = src.ld64<kNT>(voff, 4 * in_position<S>(0, m));
        a[m] = IO::load(v.x);
        a[m + 1] = IO::load(v.y);
      }
    } else {
#pragma unroll
      for (int m = 0; m < S::E; ++m) a[m] = IO::load(src.ld32<kNT>(voff, 4 * in_position<S>(0, m)));
    }
  }
  run_passes<S, INV>(a, lds, tw, t);
  if (live) {
    const Buf dst(out + row0 * S::N);
    const int voff = 4 * (slot * S::N + out_position<S>(t, 0));
    if constexpr (paired_pass<S, S::P - 1>()) {
#pragma unroll
      for (int m = 0; m < S::E; m += 2)
        dst.st64<kNT>(u32x2{IO::store(a[m]), IO::store(a[m + 1])}, voff, 4 * out_position<S>(0, m));
    } else {
#pragma unroll
      for (int m = 0; m < S::E; ++m) dst.st32<kNT>(IO::store(a[m]), voff, 4 * out_position<S>(0, m));
    }
  }
}

template <class S, class IO>
hipError_t launch_single_io(const void* in, void* out, const void* tw, int64_t batch,
                            bool inverse, hipStream_t s) {
  const int64_t groups = (batch + S::TPB - 1) / S::TPB;
  const int64_t cap = max_groups_per_launch();
  for (int64_t g0 = 0; g0 < groups; g0 += cap) {
    const int64_t g = groups - g0 < cap ? groups - g0 : cap;
    const int64_t r0 = g0 * S::TPB;
    const uint32_t* ip = static_cast<const uint32_t*>(in) + r0 * S::N;
    uint32_t* op = static_cast<uint32_t*>(out) + r0 * S::N;
    const c32* twp = static_cast<const c32*>(tw);
    if (inverse)
      k_stockham_io<S, true, IO><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(ip, op, twp, batch - r0);
    else
      k_stockham_io<S, false, IO><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(ip, op, twp, batch - r0);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ streaming
// Persistent form of the single-pass transform for large batches.  With one
// short-lived workgroup per row, every workgroup of a launch first waits for
// its whole row, then computes, then stores, so a batch that fills the chip
// once runs its loads, its arithmetic and its stores one after the other.
// Here G = k x CUs workgroups loop over the rows (row = blockIdx.x + i G):
// each loads its twiddles once and keeps them in registers, and issues the
// next row's loads before the current row's passes, so one row's loads
// overlap the previous row's arithmetic and its stores the next row's.
// The vector-memory counter lets the row's stores stay in flight while the
// next loop waits for the prefetched row, and the exchange barriers wait
// only for LDS traffic.

struct IoF32 {  // complex64 storage, for the streaming form's FP32 launch
  static constexpr int BYTES = 8;
  __device__ __forceinline__ static c32 load(u32x2 v) {
    return c32{__uint_as_float(v.x), __uint_as_float(v.y)};
  }
  __device__ __forceinline__ static u32x2 store(c32 a) {
    return u32x2{__float_as_uint(a.x), __float_as_uint(a.y)};
  }
};
template <class IO>
using io_raw = std::conditional_t<std::is_same_v<IO, IoF32>, u32x2, uint32_t>;

template <class Base, int WPC, int DEPTH = 1>
struct Streamed : Base {
  static_assert(Base::TPB == 1 && Base::PF == 2, "streamed shapes hold every twiddle in registers");
  static_assert(!paired_lanes<Base>::value, "streamed shapes use the t + m T order");
  static constexpr int STREAM_WPC = WPC;
  static constexpr int STREAM_DEPTH = DEPTH;
  // Waves per SIMD that WPC resident workgroups need (the register budget).
  static constexpr int WPE = WPC * Base::THREADS / 256 > 1 ? WPC * Base::THREADS / 256 : 1;
};
template <class S, class = void>
struct streamed : std::integral_constant<int, 0> {};
template <class S>
struct streamed<S, std::void_t<decltype(S::STREAM_WPC)>> : std::integral_constant<int, S::STREAM_WPC> {};

// One row of raw values: slot m at t + m T.
template <class S, class IO>
__device__ __forceinline__ void stream_load(io_raw<IO> (&r)[S::E], const Buf& b, int t) {
  constexpr int B = (int)sizeof(io_raw<IO>);
#pragma unroll
  for (int m = 0; m < S::E; ++m) {
    if constexpr (B == 8)
      r[m] = b.ld64<kNT>(B * t, B * m * S::T);
    else
      r[m] = b.ld32<kNT>(B * t, B * m * S::T);
  }
}

template <class S, bool INV, class IO>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_stockham_stream(const void* in, void* out,
                                                                 const c32* tw, int64_t rows,
                                                                 int64_t stride) {
  using R = io_raw<IO>;
  constexpr int B = (int)sizeof(R);
  constexpr int D = S::STREAM_DEPTH;  // rows in flight ahead of the one computed
  constexpr int NB = D + 1;           // register buffers, used round-robin
  static_assert(D * S::E + S::E <= 63, "in-flight accesses exceed the wave's memory counter");
  __shared__ alignas(16) c32 lds[S::LDS_ELEMS];
  const int t = threadIdx.x;
  const char* src = static_cast<const char*>(in);
  char* dst = static_cast<char*>(out);
  R buf[NB][S::E];
  int64_t row = blockIdx.x;  // the grid never exceeds rows
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (row + j * stride < rows) stream_load<S, IO>(buf[j], Buf(src + (row + j * stride) * (S::N * B)), t);
  c32 w[S::TW_REGS];
  preload_twiddles<S>(w, tw, t);
  // Wait for the twiddles here (the rows loaded before them are then in too):
  // otherwise the loop's wait counts must allow for their loads still being
  // in flight, and in later rows they would wait for the prefetches.
#pragma unroll
  for (int i = 0; i < S::TW_REGS; ++i) asm volatile("" ::"v"(w[i].x), "v"(w[i].y));
  for (;;) {
    // Unrolled NB times, so every buffer index is a constant and no loaded
    // register is copied (a copy would wait for its load).
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      const int64_t r = row + s * stride;
      if (r >= rows) return;  // uniform
      const int64_t ahead = r + D * stride;
      // buffer (s + D) mod NB held the row computed in the previous step
      if (ahead < rows) stream_load<S, IO>(buf[(s + D) % NB], Buf(src + ahead * (S::N * B)), t);
      c32 a[S::E];
#pragma unroll
      for (int m = 0; m < S::E; ++m) a[m] = IO::load(buf[s][m]);
      run_passes_preloaded<S, INV>(a, w, lds, tw, t);
      const Buf o(dst + r * (S::N * B));
#pragma unroll
      for (int m = 0; m < S::E; ++m) {
        if constexpr (B == 8)
          o.st64<kNT>(IO::store(a[m]), B * t, B * m * S::T);
        else
          o.st32<kNT>(IO::store(a[m]), B * t, B * m * S::T);
      }
      __syncthreads();  // this row's last exchange reads are done before the next row's writes
    }
    row += NB * stride;
  }
}

template <class S, class IO>
hipError_t launch_stream(const void* in, void* out, const void* tw, int64_t batch, bool inverse,
                         hipStream_t s) {
  int64_t g = (int64_t)device_cus() * streamed<S>::value;
  if (g > batch) g = batch;
  const c32* twp = static_cast<const c32*>(tw);
  if (inverse)
    k_stockham_stream<S, true, IO><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(in, out, twp, batch, g);
  else
    k_stockham_stream<S, false, IO><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(in, out, twp, batch, g);
  return hipGetLastError();
}

// Sum v over the lanes of one wave that own the same transform (all 64 lanes
// when a transform spans several waves).  Every one of those lanes returns
// the wave's sum; a transform wider than a wave adds its waves' sums
// afterwards.
template <class S>
__device__ __forceinline__ float wave_group_sum(float v) {
  constexpr int W = S::T < 64 ? S::T : 64;
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The loss total of the fused kernels: the last workgroup to count itself
// adds all rows in a fixed order (bitwise reproducible), reading them with
// device-scope atomic loads as they were published, so no cache write-back is
// needed.  fused_loss_count: thread 0 of a workgroup whose row losses have
// been published (and have completed) counts it; gi is its index among the
// groups_all workgroups that count; returns whether it came last.
__device__ __forceinline__ int fused_loss_count(unsigned* counters, unsigned groups_all, unsigned gi) {
  const unsigned grp = gi % kTotalGroups;
  const unsigned in_grp = groups_all / kTotalGroups + (grp < groups_all % kTotalGroups ? 1u : 0u);
  const unsigned ngrp = groups_all < kTotalGroups ? groups_all : kTotalGroups;
  unsigned* c1 = counters + grp * 64;
  unsigned* c2 = counters + kTotalGroups * 64;
  int last = 0;
  if (atomicAdd(c1, 1u) == in_grp - 1u) {
    atomicExch(c1, 0u);
    if (atomicAdd(c2, 1u) == ngrp - 1u) {
      atomicExch(c2, 0u);
      last = 1;
    }
  }
  return last;
}

// The sum itself, by every thread of the last workgroup; scratch is LDS for
// THREADS floats, free on entry.
template <class S>
__device__ __forceinline__ void fused_loss_sum(float* scratch, float* total_out,
                                               const float* row_loss_all, int64_t rows_all) {
  const int tid = threadIdx.x;
  // Summation order, whatever the workgroup size: 1024 lanes, lane v adds
  // rows v, v + 1024, ... in turn, then a halving tree (lane v adds lane
  // v + h for h = 512, 256, ..., 1).  Thread tid plays lanes tid + j THREADS.
  static_assert(1024 % S::THREADS == 0 && S::THREADS % 64 == 0, "lane mapping");
  static_assert(S::TPB * S::LDS_ELEMS * sizeof(c32) >= S::THREADS * sizeof(float), "tree");
  constexpr int V = 1024 / S::THREADS;
  float v[V];
#pragma unroll
  for (int j = 0; j < V; ++j) {
    v[j] = 0.f;
    for (int64_t i = tid + j * S::THREADS; i < rows_all; i += 1024)
      v[j] += __hip_atomic_load(row_loss_all + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
#pragma unroll
  for (int h = V / 2; h > 0; h >>= 1)  // tree steps h * THREADS, inside a thread
#pragma unroll
    for (int j = 0; j < h; ++j) v[j] += v[j + h];
  float part = v[0];
  if constexpr (S::THREADS > 64) {  // tree steps THREADS / 2 .. 64, across waves
    float* f = scratch;
    f[tid] = part;
    __syncthreads();
#pragma unroll
    for (int h = S::THREADS / 2; h >= 64; h >>= 1) {
      if (tid < h) f[tid] += f[tid + h];
      __syncthreads();
    }
    part = f[tid & 63];
  }
#pragma unroll
  for (int h = 32; h > 0; h >>= 1) part += __shfl_xor(part, h, 64);  // steps 32 .. 1
  if (tid == 0) total_out[0] = part;
}

// Both steps after the workgroup's last store: every workgroup of the launch
// calls it once, after publishing its rows.
template <class S>
__device__ __forceinline__ void fused_loss_total(float* scratch, int& is_last, float* total_out,
                                                 unsigned* counters, const float* row_loss_all,
                                                 int64_t rows_all, unsigned groups_all, unsigned gi) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this lane's publication has completed
  __syncthreads();  // ... for every lane; and the LDS is free
  if (threadIdx.x == 0) is_last = fused_loss_count(counters, groups_all, gi);
  __syncthreads();
  if (is_last) fused_loss_sum<S>(scratch, total_out, row_loss_all, rows_all);
}

// -------------------------------------------------- fused forward/adjoint
// x -> y = F x -> (row loss sum w^2 |y|^2, g = 2 w^2 y * scale) -> F^H g.
// Reads x once and writes the gradient once: 16 N bytes per row against the
// 48 N of three separate launches.
// Loss total: workgroups count themselves on kTotalGroups counters (by global
// index mod kTotalGroups, each on its own 256-byte line), and each group's
// last one on a second-level counter, so no single address takes every
// workgroup's atomic.  counters: kTotalGroups * 64 + 1 zeroed words, left zeroed.
template <class S>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_spectral_energy(
    const c32* x, const float* __restrict__ w, const float* __restrict__ scale, c32* grad,
    float* row_loss, const c32* tw, int64_t rows, float* total_out, unsigned* counters,
    float* row_loss_all, int64_t rows_all, unsigned groups_all, unsigned gbase) {
  static_assert(round_trip_layout<S>(), "the adjoint runs on the forward's output registers");
  __shared__ alignas(16) c32 lds_all[S::TPB * S::LDS_ELEMS];
  __shared__ float red[(S::THREADS + 63) / 64];
  __shared__ int is_last;
  const int tid = threadIdx.x;
  const int slot = S::TPB == 1 ? 0 : tid / S::T;  // one transform: the row base is uniform
  const int t = tid - slot * S::T;
  const int64_t row = (int64_t)blockIdx.x * S::TPB + slot;
  const bool live = row_live<S>(row, rows);
  const int64_t row0 = (int64_t)blockIdx.x * S::TPB;
  c32* lds = lds_all + slot * S::LDS_ELEMS;
  c32 a[S::E];
  buffer_load_row<S>(a, Buf(x + row0 * S::N), slot_src<S>(slot, row, rows), t);
  run_passes<S, false>(a, lds, tw, t);

  const float sc = scale ? 2.0f * scale[0] : 2.0f;
  float acc = 0.f;
  const Buf wb(w);
  const int wv = 4 * out_position<S>(t, 0);
#pragma unroll
  for (int m = 0; m < S::E; ++m) {
    const float wq = __uint_as_float(wb.ld32(wv, 4 * out_position<S>(0, m)));
    const float w2 = wq * wq;
    const c32 y = a[m];
    acc += w2 * (y.x * y.x + y.y * y.y);
    const float g = sc * w2;
    a[m] = c32{g * y.x, g * y.y};
  }
  acc = wave_group_sum<S>(acc);
  if constexpr (S::T > 64) {
    if ((tid & 63) == 0) red[tid >> 6] = acc;
  }
  __syncthreads();  // forward passes done with LDS; wave partials visible
  if (t == 0 && live) {
    float total = acc;
    if constexpr (S::T > 64) {
      total = 0.f;
      const int w0 = (slot * S::T) >> 6;
#pragma unroll
      for (int i = 0; i < S::T / 64; ++i) total += red[w0 + i];
    }
    if (total_out != nullptr)
      atomicExch(&row_loss[row], total);  // published where every XCD sees it
    else
      row_loss[row] = total;
  }
  if (grad != nullptr) {  // uniform across the launch
    run_passes<S, true>(a, lds, tw, t);
    buffer_store_row<S>(a, Buf(grad + row0 * S::N), slot * S::N, t, live);
  }
  if (total_out != nullptr)  // uniform across the launch
    fused_loss_total<S>(reinterpret_cast<float*>(lds_all), is_last, total_out, counters, row_loss_all,
                        rows_all, groups_all, gbase + blockIdx.x);
}

template <class S>
hipError_t launch_spectral_energy(const void* x, const float* w, const float* scale, void* grad,
                                  float* row_loss, float* total, unsigned* counters, const void* tw,
                                  int64_t batch, hipStream_t s) {
  const int64_t groups = (batch + S::TPB - 1) / S::TPB;
  const int64_t cap = max_groups_per_launch();
  for (int64_t g0 = 0; g0 < groups; g0 += cap) {
    const int64_t g = groups - g0 < cap ? groups - g0 : cap;
    const int64_t r0 = g0 * S::TPB;
    k_spectral_energy<S><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(
        static_cast<const c32*>(x) + r0 * S::N, w, scale,
        grad ? static_cast<c32*>(grad) + r0 * S::N : nullptr, row_loss + r0,
        static_cast<const c32*>(tw), batch - r0, total, counters, row_loss, batch,
        (unsigned)groups, (unsigned)g0);
  }
  return hipGetLastError();
}

// Persistent form of the fused kernel (Streamed shapes): G = k x CUs
// workgroups loop over the rows (row = blockIdx.x + i G) with the next D
// rows' loads in flight during the current row's forward passes, weight and
// adjoint passes, so one row's arithmetic overlaps other rows' HBM traffic
// where a workgroup per row runs every row's loads, arithmetic and stores in
// lockstep.  The twiddles and the squared weights of the lane's positions
// are loaded once per workgroup.  Same outputs as k_spectral_energy.
template <class S>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_spectral_energy_stream(
    const c32* x, const float* __restrict__ w, const float* __restrict__ scale, c32* grad,
    float* row_loss, const c32* tw, int64_t rows, int64_t stride, float* total_out,
    unsigned* counters) {
  static_assert(round_trip_layout<S>(), "the adjoint runs on the forward's output registers");
  constexpr int D = S::STREAM_DEPTH;
  constexpr int NB = D + 1;
  static_assert(D * S::E + S::E <= 63, "in-flight accesses exceed the wave's memory counter");
  __shared__ alignas(16) c32 lds[S::LDS_ELEMS];
  __shared__ float red[(S::THREADS + 63) / 64];
  __shared__ int is_last;
  const int t = threadIdx.x;
  u32x2 buf[NB][S::E];
  const int64_t row0 = blockIdx.x;  // the grid never exceeds rows
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (row0 + j * stride < rows) stream_load<S, IoF32>(buf[j], Buf(x + (row0 + j * stride) * S::N), t);
  c32 tws[S::TW_REGS];
  preload_twiddles<S>(tws, tw, t);
  float w2[S::E];
  {
    const Buf wb(w);
#pragma unroll
    for (int m = 0; m < S::E; ++m) {
      const float wq = __uint_as_float(wb.ld32(4 * t, 4 * m * S::T));
      w2[m] = wq * wq;
    }
  }
  // Wait for the twiddles and weights here (the rows loaded before them are
  // then in too), so that the loop's waits need not count them.
#pragma unroll
  for (int i = 0; i < S::TW_REGS; ++i) asm volatile("" ::"v"(tws[i].x), "v"(tws[i].y));
#pragma unroll
  for (int m = 0; m < S::E; ++m) asm volatile("" ::"v"(w2[m]));
  const float sc = scale ? 2.0f * scale[0] : 2.0f;
  bool done = false;
  for (int64_t row = row0; !done; row += NB * stride) {
    // Unrolled NB times, so every buffer index is a constant and no loaded
    // register is copied (a copy would wait for its load).
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      const int64_t r = row + s * stride;
      if (r >= rows) {  // uniform
        done = true;
        break;
      }
      const int64_t ahead = r + D * stride;
      if (ahead < rows) stream_load<S, IoF32>(buf[(s + D) % NB], Buf(x + ahead * S::N), t);
      c32 a[S::E];
#pragma unroll
      for (int m = 0; m < S::E; ++m) a[m] = IoF32::load(buf[s][m]);
      run_passes_preloaded<S, false>(a, tws, lds, tw, t);
      float acc = 0.f;
#pragma unroll
      for (int m = 0; m < S::E; ++m) {
        const c32 y = a[m];
        acc += w2[m] * (y.x * y.x + y.y * y.y);
        const float g = sc * w2[m];
        a[m] = c32{g * y.x, g * y.y};
      }
      acc = wave_group_sum<S>(acc);
      if constexpr (S::T > 64) {
        if ((t & 63) == 0) red[t >> 6] = acc;
      }
      __syncthreads();  // forward passes done with LDS; wave partials visible
      if (t == 0) {
        float total = acc;
        if constexpr (S::T > 64) {
          total = 0.f;
#pragma unroll
          for (int i = 0; i < S::T / 64; ++i) total += red[i];
        }
        if (total_out != nullptr)
          atomicExch(&row_loss[r], total);  // published where every XCD sees it
        else
          row_loss[r] = total;
      }
      if (grad != nullptr) {  // uniform across the launch
        run_passes_preloaded<S, true>(a, tws, lds, tw, t);
        const Buf o(grad + r * S::N);
#pragma unroll
        for (int m = 0; m < S::E; ++m) o.st64<kNT>(IoF32::store(a[m]), 8 * t, 8 * m * S::T);
      }
      __syncthreads();  // this row's exchange and partial reads are done before the next row's writes
    }
  }
  if (total_out != nullptr)  // uniform across the launch
    fused_loss_total<S>(reinterpret_cast<float*>(lds), is_last, total_out, counters, row_loss, rows,
                        gridDim.x, blockIdx.x);
}

template <class S>
hipError_t launch_spectral_energy_stream(const void* x, const float* w, const float* scale, void* grad,
                                         float* row_loss, float* total, unsigned* counters,
                                         const void* tw, int64_t batch, hipStream_t s) {
  int64_t g = (int64_t)device_cus() * streamed<S>::value;
  if (g > batch) g = batch;
  k_spectral_energy_stream<S><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(
      static_cast<const c32*>(x), w, scale, static_cast<c32*>(grad), row_loss,
      static_cast<const c32*>(tw), batch, g, total, counters);
  return hipGetLastError();
}

// ------------------------------------------------------- matched filter
// Range compression (the paper's future work on SAR pipeline fusion):
// out = (1/N) F^H(conj(h) .* F x) in one kernel.
template <class S>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_matched_filter(const c32* x, const c32* __restrict__ h,
                                                               c32* out, const c32* tw,
                                                               int64_t rows) {
  static_assert(round_trip_layout<S>(), "the inverse runs on the forward's output registers");
  __shared__ alignas(16) c32 lds_all[S::TPB * S::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int slot = S::TPB == 1 ? 0 : tid / S::T;  // one transform: the row base is uniform
  const int t = tid - slot * S::T;
  const int64_t row = (int64_t)blockIdx.x * S::TPB + slot;
  const bool live = row_live<S>(row, rows);
  const int64_t row0 = (int64_t)blockIdx.x * S::TPB;
  c32* lds = lds_all + slot * S::LDS_ELEMS;
  c32 a[S::E];
  buffer_load_row<S>(a, Buf(x + row0 * S::N), slot_src<S>(slot, row, rows), t);
  run_passes<S, false>(a, lds, tw, t);
  constexpr float inv_n = 1.0f / float(S::N);  // a power of two: exact
  const Buf hb(h);
  const int hv = 8 * out_position<S>(t, 0);
#pragma unroll
  for (int m = 0; m < S::E; ++m) {
    const u32x2 hw = hb.ld64(hv, 8 * out_position<S>(0, m));
    const c32 hq = c32{__uint_as_float(hw.x), __uint_as_float(hw.y)};
    const c32 y = cmulc(a[m], hq);
    a[m] = c32{y.x * inv_n, y.y * inv_n};
  }
  __syncthreads();
  run_passes<S, true>(a, lds, tw, t);
  buffer_store_row<S>(a, Buf(out + row0 * S::N), slot * S::N, t, live);
}

template <class S>
hipError_t launch_matched_filter(const void* x, const void* h, void* out, const void* tw,
                                 int64_t batch, hipStream_t s) {
  const int64_t groups = (batch + S::TPB - 1) / S::TPB;
  const int64_t cap = max_groups_per_launch();
  for (int64_t g0 = 0; g0 < groups; g0 += cap) {
    const int64_t g = groups - g0 < cap ? groups - g0 : cap;
    const int64_t r0 = g0 * S::TPB;
    k_matched_filter<S><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(
        static_cast<const c32*>(x) + r0 * S::N, static_cast<const c32*>(h),
        static_cast<c32*>(out) + r0 * S::N, static_cast<const c32*>(tw), batch - r0);
  }
  return hipGetLastError();
}

// -------------------------------------------------------------- four-step
// The paper's eq. (3) order: length-N2 sub-transforms of the N1 decimated
// sequences x[n1 + N1 m] (stage 1), then twiddle W_N^{n1 k2} and length-N1
// DFTs across the sub-transforms, stored at k2 + N2 k1 (stage 2).  The
// intermediate goes through device memory.
//
// Stage 1 mapping is XCD-aware: the workgroups are dealt round-robin to the 8
// XCDs, so block i serves row 8 (i div 8N1) + (i mod 8) and sub-sequence
// (i mod 8N1) div 8; all N1 readers of one row then share one L2, which
// absorbs the stride-N1 reads.
constexpr int kXcds = 8;

template <class S, int N1, bool INV>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_four_step_columns(const c32* x, c32* y,
                                                                  const c32* tw,
                                                                  int64_t rows) {
  static_assert(S::TPB == 1, "four-step sub-transforms use one transform per workgroup");
  static_assert(!paired_lanes<S>::value, "four-step sub-transforms use the plain lane order");
  __shared__ alignas(16) c32 lds[S::LDS_ELEMS];
  const int64_t i = blockIdx.x;
  const int64_t grp = i / (kXcds * N1);
  const int r = (int)(i - grp * kXcds * N1);
  const int n1 = r / kXcds;
  const int64_t row = grp * kXcds + (r - n1 * kXcds);
  if (row >= rows) return;  // whole workgroup, before any barrier
  constexpr int N = S::N * N1;
  const int t = threadIdx.x;
  const c32* src = x + row * N + n1;
  c32 a[S::E];
#pragma unroll
  for (int m = 0; m < S::E; ++m) a[m] = src[(int64_t)(t + m * S::T) * N1];
  run_passes<S, INV>(a, lds, tw, t);
  global_store_row<S, false>(a, y + (row * N1 + n1) * S::N, t, true);
}

// Length-N1 DFT in registers for the four-step second stage.  N1 <= 16: the
// exact radix-2 DIT of Dft.  N1 = 32, 64: N1 = P Q with P = 16, i.e. P-point
// DFTs of the Q interleaved sub-sequences v[Q p + q], twiddles W_N1^{q kp}
// (from wn, wn[j] = W_N1^j in the forward direction), then Q-point DFTs; the
// result X[k] is left in v[slot(k)].
template <int N1, bool INV>
struct RegDft {
  static constexpr int P = N1 <= 16 ? N1 : 16;
  static constexpr int Q = N1 / P;
  static constexpr int slot(int k) { return Q == 1 ? k : Q * (k % P) + k / P; }
  __device__ __forceinline__ static void run(c32 (&v)[N1], const c32* wn) {
    if constexpr (Q == 1) {
      Dft<N1, INV>::run(v);
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        c32 t[P];
#pragma unroll
        for (int p = 0; p < P; ++p) t[p] = v[Q * p + q];
        Dft<P, INV>::run(t);
#pragma unroll
        for (int kp = 0; kp < P; ++kp)
          v[Q * kp + q] = (q == 0 || kp == 0) ? t[kp] : ctw<INV>(t[kp], wn[q * kp]);
      }
#pragma unroll
      for (int kp = 0; kp < P; ++kp) {
        c32 u[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) u[q] = v[Q * kp + q];
        Dft<Q, INV>::run(u);
#pragma unroll
        for (int kq = 0; kq < Q; ++kq) v[Q * kp + kq] = u[kq];
      }
    }
  }
};

constexpr int half_log2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l / 2;
}

template <int N1, int N2, bool INV, bool TWO_LEVEL>
__global__ __launch_bounds__(256) void k_four_step_combine(const c32* y, c32* out,
                                                           const c32* __restrict__ tw4, int64_t rows) {
  constexpr int N = N1 * N2;
  static_assert(TWO_LEVEL || N1 <= 16, "the full twiddle table serves N1 <= 16");
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = gid / N2;
  const int k2 = (int)(gid - row * N2);
  if (row >= rows) return;
  const c32* src = y + row * N + k2;
  c32 v[N1];
  v[0] = src[0];
  const c32* wn = nullptr;
  if constexpr (TWO_LEVEL) {
    // W_N^{n1 k2} for n1 = RA j + i as W_N^{RA j k2} W_N^{i k2}: 2 (RA - 1 +
    // N1 / RA - 1) table reads per lane instead of 2 (N1 - 1); each factor is
    // hi[m >> SL] lo[m mod 2^SL] of two once-rounded entries.
    constexpr int SL = half_log2(N);
    constexpr int RA = N1 >= 16 ? 8 : N1;
    constexpr int RB = N1 / RA;
    const c32* lo = tw4;
    const c32* hi = tw4 + (1 << SL);
    wn = hi + (N >> SL);
    c32 bi[RA], cj[RB];
#pragma unroll
    for (int i = 1; i < RA; ++i) {
      const int m = i * k2;  // < N
      bi[i] = cmul(hi[m >> SL], lo[m & ((1 << SL) - 1)]);
    }
#pragma unroll
    for (int j = 1; j < RB; ++j) {
      const int m = RA * j * k2;  // < N
      cj[j] = cmul(hi[m >> SL], lo[m & ((1 << SL) - 1)]);
    }
#pragma unroll
    for (int n1 = 1; n1 < N1; ++n1) {
      const int i = n1 % RA, j = n1 / RA;
      const c32 w = j == 0 ? bi[i] : i == 0 ? cj[j] : cmul(cj[j], bi[i]);
      v[n1] = ctw<INV>(src[(int64_t)n1 * N2], w);
    }
  } else {
#pragma unroll
    for (int n1 = 1; n1 < N1; ++n1)
      v[n1] = ctw<INV>(src[(int64_t)n1 * N2], tw4[(n1 - 1) * N2 + k2]);
  }
  RegDft<N1, INV>::run(v, wn);
  c32* dst = out + row * N + k2;
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) store_stream(dst + (int64_t)k1 * N2, v[RegDft<N1, INV>::slot(k1)]);
}

template <class S, int N1>
hipError_t launch_four_step_columns(const void* x, void* y, const void* tw, int64_t batch,
                                    bool inverse, hipStream_t s) {
  // Rows are processed in chunks of kXcds * (max groups) so the block index fits.
  const int64_t units = max_groups_per_launch() / (kXcds * N1);
  const int64_t rows_per_launch = (units > 0 ? units : 1) * kXcds;
  for (int64_t r0 = 0; r0 < batch; r0 += rows_per_launch) {
    const int64_t rows = batch - r0 < rows_per_launch ? batch - r0 : rows_per_launch;
    const int64_t blocks = ((rows + kXcds - 1) / kXcds) * kXcds * N1;
    const c32* xp = static_cast<const c32*>(x) + r0 * S::N * N1;
    c32* yp = static_cast<c32*>(y) + r0 * S::N * N1;
    const c32* twp = static_cast<const c32*>(tw);
    if (inverse)
      k_four_step_columns<S, N1, true><<<dim3((unsigned)blocks), dim3(S::THREADS), 0, s>>>(xp, yp, twp, rows);
    else
      k_four_step_columns<S, N1, false><<<dim3((unsigned)blocks), dim3(S::THREADS), 0, s>>>(xp, yp, twp, rows);
  }
  return hipGetLastError();
}

template <int N1, int N2, bool TWO_LEVEL>
hipError_t launch_four_step_combine(const void* y, void* out, const void* /*tw*/, const void* tw4,
                                    int64_t batch, bool inverse, hipStream_t s) {
  static_assert(N2 % 256 == 0, "combine blocks cover 256 consecutive k2");
  const int64_t per = max_groups_per_launch() * 256 / N2;
  const int64_t rows_per_launch = per > 0 ? per : 1;
  for (int64_t r0 = 0; r0 < batch; r0 += rows_per_launch) {
    const int64_t rows = batch - r0 < rows_per_launch ? batch - r0 : rows_per_launch;
    const int64_t blocks = rows * N2 / 256;
    const c32* yp = static_cast<const c32*>(y) + r0 * N1 * N2;
    c32* op = static_cast<c32*>(out) + r0 * N1 * N2;
    const c32* twp = static_cast<const c32*>(tw4);
    if (inverse)
      k_four_step_combine<N1, N2, true, TWO_LEVEL>
          <<<dim3((unsigned)blocks), dim3(256), 0, s>>>(yp, op, twp, rows);
    else
      k_four_step_combine<N1, N2, false, TWO_LEVEL>
          <<<dim3((unsigned)blocks), dim3(256), 0, s>>>(yp, op, twp, rows);
  }
  return hipGetLastError();
}

}  // namespace stockfft
