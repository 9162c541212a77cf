// Measurement references beside the transform library (libstockref.so):
// an empty kernel, copies of the transform's bytes in its own launch shape
// and in a wide grid, the middle steps of the two unfused chains the fused
// kernels are compared with, and the single-pass transform with phase
// stamps.  Declarations and argument contracts: include/stockref.h.
#include "../../include/stockref.h"

#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "../../include/stockfft.h"
#include "../csrc/kernels.hpp"
#include "../csrc/wavex.hpp"

using namespace stockfft;

namespace {

thread_local int g_ref_hip_error = 0;

int launched() {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return FFT_SUCCESS;
  g_ref_hip_error = (int)e;
  return FFT_HIP_ERROR;
}

bool pow2_in(int64_t n, int64_t lo, int64_t hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

bool overlap(const void* a, const void* b, size_t bytes) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + bytes && y < x + bytes;
}

__global__ void k_empty() {}

// One workgroup of T lanes per row of N values, lane t moving x[t + m T].
template <int N, int T>
__global__ __launch_bounds__(T) void k_copy_rows(const c32* in, c32* out) {
  constexpr int E = N / T;
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * N;
  c32 a[E];
#pragma unroll
  for (int m = 0; m < E; ++m) a[m] = load_stream(in + base + t + m * T);
#pragma unroll
  for (int m = 0; m < E; ++m) store_stream(out + base + t + m * T, a[m]);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// 16 bytes per lane per access, 16 accesses per lane, 256 lanes.
__global__ __launch_bounds__(256) void k_copy_wide(const f32x4* in, f32x4* out, int64_t count) {
  const int64_t base = (int64_t)blockIdx.x * 4096 + threadIdx.x;
  f32x4 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int64_t i = base + m * 256;
    v[m] = i < count ? __builtin_nontemporal_load(in + i) : f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int64_t i = base + m * 256;
    if (i < count) __builtin_nontemporal_store(v[m], out + i);
  }
}

// One workgroup of 256 lanes per row: y <- 2 w^2 y, row loss by a wave
// shuffle tree and the LDS across the four waves.
__global__ __launch_bounds__(256) void k_weight_energy(c32* y, const float* __restrict__ w,
                                                       float* row_loss, int n) {
  __shared__ float part[4];
  const int t = threadIdx.x;
  c32* row = y + (int64_t)blockIdx.x * n;
  float acc = 0.f;
  for (int k = t; k < n; k += 256) {
    const float w2 = w[k] * w[k];
    const c32 v = load_stream(row + k);
    acc += w2 * (v.x * v.x + v.y * v.y);
    store_stream(row + k, c32{2.f * w2 * v.x, 2.f * w2 * v.y});
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((t & 63) == 0) part[t >> 6] = acc;
  __syncthreads();
  if (t == 0) row_loss[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

// The LDS exchange alone, in the radix-16 headline shape's size and access
// width: 256 lanes, 16 values of 8 bytes each, so every round writes and reads
// back 32 KiB per workgroup, with a barrier after the writes and one after the
// reads and nothing else in between.  Lane t writes slot t + 256 m and reads
// slot ((t + 1) mod 256) + 256 m: consecutive lanes on consecutive 8-byte
// slots (no bank conflicts), and every value moves to another lane, so after
// r rounds lane t holds lane ((t + r) mod 256)'s values.  out[g 256 + t] is
// the sum of lane t's final values (the caller can check it).
__global__ __launch_bounds__(256) void k_lds_exchange(int rounds, float* out) {
  __shared__ alignas(16) c32 buf[16 * 256];
  const int t = threadIdx.x;
  c32 a[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) a[m] = c32{(float)(t + m), (float)m};
  const int u = (t + 1) & 255;
  for (int r = 0; r < rounds; ++r) {
#pragma unroll
    for (int m = 0; m < 16; ++m) buf[t + 256 * m] = a[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; ++m) a[m] = buf[u + 256 * m];
    __syncthreads();
  }
  float s = 0.f;
#pragma unroll
  for (int m = 0; m < 16; ++m) s += a[m].x;
  out[(int64_t)blockIdx.x * 256 + t] = s;
}

// y <- conj(h) y / n over every element (n a power of two: 1/n is exact).
__global__ __launch_bounds__(256) void k_filter_multiply(c32* y, const c32* __restrict__ h,
                                                         int logn, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const float inv_n = 1.0f / (float)(1 << logn);
  const c32 v = load_stream(y + i);
  const c32 z = cmulc(v, h[i & ((int64_t(1) << logn) - 1)]);
  store_stream(y + i, c32{z.x * inv_n, z.y * inv_n});
}

// ------------------------------------------------------------ timeline

// Clock readings of one wave at the phase marks (see stockref.h).  Each
// mark waits for the LDS and scalar operations in flight, and the scheduler
// may not move work across it.
struct TimelineProbe {
  static constexpr bool on = true;
  uint64_t rt[16];
  uint64_t ct[16];
  __device__ __forceinline__ void read(int slot) {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    rt[slot] = __builtin_amdgcn_s_memrealtime();
    ct[slot] = __builtin_amdgcn_s_memtime();
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  }
  __device__ __forceinline__ void mark(int k) { read(k + 1); }
};

template <class S, bool INV>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_stockham_timeline(const c32* in, c32* out,
                                                                        const c32* tw,
                                                                        uint64_t* stamps) {
  static_assert(S::TPB == 1, "one transform per workgroup");
  __shared__ alignas(16) c32 lds[S::LDS_ELEMS];
  TimelineProbe pr;
#pragma unroll
  for (int i = 0; i < 16; ++i) pr.rt[i] = pr.ct[i] = 0;
  pr.read(0);
  const int t = threadIdx.x;
  const int64_t row = blockIdx.x;
  c32 a[S::E];
  c32 w[S::TW_REGS];
  buffer_load_row<S>(a, Buf(in + row * S::N), 0, t);
  preload_twiddles<S>(w, tw, t);  // in flight with the input, as in the plain kernel
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  pr.read(1);
  run_passes_preloaded<S, INV, TimelineProbe>(a, w, lds, tw, t, &pr);
  buffer_store_row<S>(a, Buf(out + row * S::N), 0, t, true);
  pr.read(2 * S::P + 1);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  pr.read(2 * S::P + 2);
  if ((t & 63) == 0) {
    uint64_t* dst = stamps + (row * (S::THREADS / 64) + (t >> 6)) * 32;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      dst[i] = pr.rt[i];
      dst[16 + i] = pr.ct[i];
    }
  }
}

// The same stamps around the in-wave exchange kernel's load, passes and
// store (marks 2p + 1 after pass p, 2p + 2 after the exchange that follows).
template <class S, bool INV>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_stockham_wx_timeline(const c32* in, c32* out,
                                                                           const c32* tw,
                                                                           uint64_t* stamps) {
  __shared__ alignas(16) c32 lds[S::LDS_ELEMS];
  TimelineProbe pr;
#pragma unroll
  for (int i = 0; i < 16; ++i) pr.rt[i] = pr.ct[i] = 0;
  pr.read(0);
  const int t = threadIdx.x;
  const int64_t row = blockIdx.x;
  const WxLane<S> L(t);
  WxRegs<S> R;
  wx_load<S, IoF32>(R, L, in, tw, row);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  pr.read(1);
  wx_passes<S, INV, TimelineProbe>(R, L, lds, &pr);
  wx_store<S, IoF32>(R, L, out, row);
  pr.read(2 * S::P + 1);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  pr.read(2 * S::P + 2);
  if ((t & 63) == 0) {
    uint64_t* dst = stamps + (row * (S::THREADS / 64) + (t >> 6)) * 32;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      dst[i] = pr.rt[i];
      dst[16 + i] = pr.ct[i];
    }
  }
}

struct TimelineVariant {
  const char* name;
  int n, threads;
  hipError_t (*launch)(const void*, void*, const void*, int64_t, bool, uint64_t*, hipStream_t);
};

template <class S>
hipError_t launch_timeline(const void* in, void* out, const void* tw, int64_t batch, bool inv,
                           uint64_t* stamps, hipStream_t s) {
  const dim3 grid((unsigned)batch), block(S::THREADS);
  const c32* ip = static_cast<const c32*>(in);
  c32* op = static_cast<c32*>(out);
  const c32* twp = static_cast<const c32*>(tw);
  if (inv)
    k_stockham_timeline<S, true><<<grid, block, 0, s>>>(ip, op, twp, stamps);
  else
    k_stockham_timeline<S, false><<<grid, block, 0, s>>>(ip, op, twp, stamps);
  return hipGetLastError();
}

template <class S>
hipError_t launch_timeline_wx(const void* in, void* out, const void* tw, int64_t batch, bool inv,
                              uint64_t* stamps, hipStream_t s) {
  const dim3 grid((unsigned)batch), block(S::THREADS);
  const c32* ip = static_cast<const c32*>(in);
  c32* op = static_cast<c32*>(out);
  const c32* twp = static_cast<const c32*>(tw);
  if (inv)
    k_stockham_wx_timeline<S, true><<<grid, block, 0, s>>>(ip, op, twp, stamps);
  else
    k_stockham_wx_timeline<S, false><<<grid, block, 0, s>>>(ip, op, twp, stamps);
  return hipGetLastError();
}

// The shapes of the N = 4096 variants of the library with one transform
// per workgroup (names as fft_variant_describe gives them); the first is
// the tuned shape at 256 rows.
const TimelineVariant kTimeline[] = {
    {"n4096_e16_b1_px_r8.8.8.8_pt_wm2", 4096, 256,
     &launch_timeline_wx<WaveExchange<PairedTwiddles<ShapeX<1, 2, 1, 4096, 16, 1, -1, 8, 8, 8, 8>>, 1, 2>>},
    {"n4096_e8_b1_px_r8.8.8.8_pt_wx1", 4096, 512,
     &launch_timeline_wx<WaveExchange<PairedTwiddles<ShapeX<1, 2, 1, 4096, 8, 1, -1, 8, 8, 8, 8>>, 1>>},
    {"n4096_e8_b1_p4_r8.8.8.8_pt", 4096, 512,
     &launch_timeline<PairedTwiddles<Shape<4096, 8, 1, 4, 8, 8, 8, 8>>>},
    {"n4096_e16_b1_px_r16.16.16_db_pt_tall", 4096, 256,
     &launch_timeline<DoubleBuffered<PairedTwiddles<ShapeX<1, 2, 1, 4096, 16, 1, -1, 16, 16, 16>>>>},
    {"n4096_e16_b1_px_r16.16.16_db_pt", 4096, 256,
     &launch_timeline<DoubleBuffered<PairedTwiddles<Shape<4096, 16, 1, -1, 16, 16, 16>>>>},
    {"n4096_e16_b1_px_r16.16.16_db", 4096, 256,
     &launch_timeline<DoubleBuffered<Shape<4096, 16, 1, -1, 16, 16, 16>>>},
    {"n4096_e16_b1_px_r16.16.16", 4096, 256, &launch_timeline<Shape<4096, 16, 1, -1, 16, 16, 16>>},
    {"n4096_e8_b1_p4_r8.8.8.8", 4096, 512, &launch_timeline<Shape<4096, 8, 1, 4, 8, 8, 8, 8>>},
};

}  // namespace

extern "C" int ref_empty(int64_t groups, int threads, void* stream) {
  if (groups < 1 || groups > 0x7fffffff || threads < 1 || threads > 1024) return FFT_INVALID_ARGUMENT;
  k_empty<<<dim3((unsigned)groups), dim3((unsigned)threads), 0, (hipStream_t)stream>>>();
  return launched();
}

extern "C" int ref_copy_rows(const void* in, void* out, int64_t n, int64_t batch, int lanes,
                             void* stream) {
  if (!in || !out) return FFT_INVALID_POINTER;
  if (batch < 1 || batch > 0x7fffffff) return FFT_INVALID_ARGUMENT;
  if (((uintptr_t)in & 7u) || ((uintptr_t)out & 7u)) return FFT_MISALIGNED;
  if (overlap(in, out, (size_t)n * (size_t)batch * 8)) return FFT_OVERLAP;
  const dim3 grid((unsigned)batch);
  hipStream_t s = (hipStream_t)stream;
  const c32* ip = static_cast<const c32*>(in);
  c32* op = static_cast<c32*>(out);
  if (n == 4096 && lanes == 256)
    k_copy_rows<4096, 256><<<grid, dim3(256), 0, s>>>(ip, op);
  else if (n == 4096 && lanes == 512)
    k_copy_rows<4096, 512><<<grid, dim3(512), 0, s>>>(ip, op);
  else if (n == 4096 && lanes == 1024)
    k_copy_rows<4096, 1024><<<grid, dim3(1024), 0, s>>>(ip, op);
  else if (n == 1024 && lanes == 64)
    k_copy_rows<1024, 64><<<grid, dim3(64), 0, s>>>(ip, op);
  else if (n == 16384 && lanes == 1024)
    k_copy_rows<16384, 1024><<<grid, dim3(1024), 0, s>>>(ip, op);
  else
    return FFT_INVALID_ARGUMENT;
  return launched();
}

extern "C" int ref_copy_wide(const void* in, void* out, int64_t bytes, void* stream) {
  if (!in || !out) return FFT_INVALID_POINTER;
  if (bytes < 16 || bytes % 16 != 0) return FFT_INVALID_ARGUMENT;
  if (((uintptr_t)in & 15u) || ((uintptr_t)out & 15u)) return FFT_MISALIGNED;
  if (overlap(in, out, (size_t)bytes)) return FFT_OVERLAP;
  const int64_t count = bytes / 16;
  const int64_t groups = (count + 4095) / 4096;
  if (groups > 0x7fffffff) return FFT_INVALID_ARGUMENT;
  k_copy_wide<<<dim3((unsigned)groups), dim3(256), 0, (hipStream_t)stream>>>(
      static_cast<const f32x4*>(in), static_cast<f32x4*>(out), count);
  return launched();
}

extern "C" int ref_lds_exchange(int64_t groups, int rounds, float* out, void* stream) {
  if (!out) return FFT_INVALID_POINTER;
  if (groups < 1 || groups > 0x7fffffff || rounds < 0) return FFT_INVALID_ARGUMENT;
  if ((uintptr_t)out & 3u) return FFT_MISALIGNED;
  k_lds_exchange<<<dim3((unsigned)groups), dim3(256), 0, (hipStream_t)stream>>>(rounds, out);
  return launched();
}

extern "C" int ref_weight_energy(void* y, const float* w, float* row_loss, int64_t n, int64_t batch,
                                 void* stream) {
  if (!y || !w || !row_loss) return FFT_INVALID_POINTER;
  if (!pow2_in(n, 256, 16384) || batch < 1 || batch > 0x7fffffff) return FFT_INVALID_ARGUMENT;
  if (((uintptr_t)y & 7u) || ((uintptr_t)w & 3u) || ((uintptr_t)row_loss & 3u)) return FFT_MISALIGNED;
  k_weight_energy<<<dim3((unsigned)batch), dim3(256), 0, (hipStream_t)stream>>>(
      static_cast<c32*>(y), w, row_loss, (int)n);
  return launched();
}

extern "C" int ref_filter_multiply(void* y, const void* h, int64_t n, int64_t batch, void* stream) {
  if (!y || !h) return FFT_INVALID_POINTER;
  if (!pow2_in(n, 256, 16384) || batch < 1) return FFT_INVALID_ARGUMENT;
  if (((uintptr_t)y & 7u) || ((uintptr_t)h & 7u)) return FFT_MISALIGNED;
  const int64_t total = n * batch;
  const int64_t groups = (total + 255) / 256;
  if (groups > 0x7fffffff) return FFT_INVALID_ARGUMENT;
  int logn = 0;
  while ((int64_t(1) << logn) < n) ++logn;
  k_filter_multiply<<<dim3((unsigned)groups), dim3(256), 0, (hipStream_t)stream>>>(
      static_cast<c32*>(y), static_cast<const c32*>(h), logn, total);
  return launched();
}

extern "C" int ref_timeline(const char* variant, const void* in, void* out, const void* tw,
                            int64_t batch, int inverse, uint64_t* stamps, void* stream) {
  if (!variant || !in || !out || !tw || !stamps) return FFT_INVALID_POINTER;
  if (batch < 1 || batch > 0x7fffffff || (inverse != 0 && inverse != 1)) return FFT_INVALID_ARGUMENT;
  for (const TimelineVariant& v : kTimeline) {
    if (std::strcmp(v.name, variant) != 0) continue;
    if (((uintptr_t)in & 7u) || ((uintptr_t)out & 7u) || ((uintptr_t)stamps & 7u))
      return FFT_MISALIGNED;
    if (overlap(in, out, (size_t)v.n * (size_t)batch * 8) && in != out) return FFT_OVERLAP;
    const hipError_t e = v.launch(in, out, tw, batch, inverse == 1, stamps, (hipStream_t)stream);
    if (e != hipSuccess) {
      g_ref_hip_error = (int)e;
      return FFT_HIP_ERROR;
    }
    return FFT_SUCCESS;
  }
  return FFT_INVALID_ARGUMENT;
}

extern "C" int ref_timeline_variants(char* buf, int64_t cap) {
  if (!buf) return FFT_INVALID_POINTER;
  std::string s;
  for (const TimelineVariant& v : kTimeline) {
    if (!s.empty()) s += ",";
    s += v.name;
  }
  if (cap < (int64_t)s.size() + 1) return FFT_INVALID_ARGUMENT;
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return FFT_SUCCESS;
}

extern "C" int ref_last_hip_error(void) { return g_ref_hip_error; }
