// Raw buffer accesses for workgroup-uniform arrays (a workgroup's rows, a
// twiddle table, a weight vector).  The base address sits in a buffer
// descriptor in scalar registers and an element's byte offset splits into a
// lane part (one vector register, computed once) and a constant part (a
// scalar register or the instruction's immediate), so the addressing of an
// unrolled row of loads takes no vector instructions, where 64-bit global
// addresses take two per distinct offset beyond the 4 KiB immediate range.
#pragma once

#include <hip/hip_runtime.h>

namespace stockfft {

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Descriptor word 3 for raw (stride 0) accesses on CDNA: 32-bit data format,
// no swizzle, no index.
constexpr int kRsrcWord3 = 0x00020000;
// Record count: offsets up to 2 GiB - 1 bytes stay in range.
constexpr int kRsrcBytes = 0x7fffffff;
// Cache policy of the access: 0 ordinary, kNT streamed once (nontemporal).
constexpr int kNT = 2;

struct Buf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ explicit Buf(const void* base)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, kRsrcBytes, kRsrcWord3)) {}

  // Byte offsets: voff varies by lane, soff is uniform (a constant after
  // unrolling).  Both must be non-negative and their sum below 2 GiB.
  template <int AUX = 0>
  __device__ __forceinline__ unsigned ld32(int voff, int soff) const {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX);
  }
  template <int AUX = 0>
  __device__ __forceinline__ u32x2 ld64(int voff, int soff) const {
    return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX);
  }
  template <int AUX = 0>
  __device__ __forceinline__ u32x4 ld128(int voff, int soff) const {
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX);
  }
  template <int AUX = 0>
  __device__ __forceinline__ void st32(unsigned v, int voff, int soff) const {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, voff, soff, AUX);
  }
  template <int AUX = 0>
  __device__ __forceinline__ void st64(u32x2 v, int voff, int soff) const {
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, AUX);
  }
  template <int AUX = 0>
  __device__ __forceinline__ void st128(u32x4 v, int voff, int soff) const {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, AUX);
  }
};

}  // namespace stockfft
