// Radix-16 Stockham passes whose 16-point DFTs run on the matrix cores
// (the paper's Section VI matrix-multiply DFT idea and its future-work item
// on combining it with half-precision storage, Section VIII), for N = 4096
// with binary16 or bfloat16 storage.
//
// One pass is 256 butterflies of 16 legs.  Written as real arithmetic, a
// 16-point DFT is a 32 x 32 matrix M acting on the 32 reals of a butterfly
// (real parts of the legs, then imaginary parts):
//   M = [[C, S], [-S, C]],  C[k][r] = cos(2 pi k r / 16),  S[k][r] = sin(...)
// (forward; the backward transform negates S).  A wave takes 32 butterflies
// as the 32 columns of a 32 x 32 operand and forms M times it with two
// v_mfma_f32_32x32x16 products (K = 32 split in two halves of 16): the
// operands are rounded to the 16-bit format, products are exact and the
// sums are FP32.  Twiddles are applied in FP32 on the vector ALUs before the
// rounding, and the exchange between passes keeps FP32 values in LDS.
//
// Lane layouts of the 32x32x16 products (checked on gfx950): lane l holds
// A[l % 32][8 (l / 32) + e] and B[8 (l / 32) + e][l % 32] for e < 8, and the
// result D[8 (g / 4) + 4 (l / 32) + g % 4][l % 32] in accumulator g < 16.
// So lane (j = l % 32, h = l / 32) supplies legs 8h .. 8h + 7 of butterfly j
// (real parts to the first product, imaginary parts to the second) and gets
// back bins 4h .. 4h + 3 and 8 + 4h .. 8 + 4h + 3 of the same butterfly, real
// parts in accumulators 0 .. 7 and imaginary parts in 8 .. 15.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "kernels.hpp"

namespace stockfft {
namespace {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kN = 4096;
constexpr int kNB = kN / 16;              // butterflies per pass
constexpr int kThreads = 256;             // four waves per transform
constexpr int kBlocks = kNB / 32 / (kThreads / 64);  // 32-butterfly blocks per wave
constexpr int kLds = kN + kN / 16;        // one pad element per 16 against bank conflicts

__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

// cos(2 pi m / 16), m = 0 .. 15, from the FP64 values; sin(2 pi m / 16) is
// entry (m + 12) mod 16.
__device__ __forceinline__ float cos16(int m) {
  constexpr float c1 = 0.92387953251128674, c2 = 0.70710678118654757, c3 = 0.38268343236508978;
  constexpr float t[16] = {1.f, c1, c2, c3, 0.f, -c3, -c2, -c1, -1.f, -c1, -c2, -c3, 0.f, c3, c2, c1};
  return t[m & 15];
}

// Entry (i, q) of M (rows: real bins 0..15, imaginary bins 16..31; columns:
// real legs, imaginary legs).
template <bool INV>
__device__ __forceinline__ float dft_entry(int i, int q) {
  const int m = ((i & 15) * (q & 15)) & 15;
  const float c = cos16(m);
  const float s = INV ? -cos16(m + 12) : cos16(m + 12);
  if (i < 16) return q < 16 ? c : s;
  return q < 16 ? -s : c;
}

// The 16-bit operand format: binary16 storage multiplies binary16 operands,
// bfloat16 storage bfloat16 operands.
template <class IO>
struct MmaOps;

template <>
struct MmaOps<IoF16> {
  typedef f16x8 V;
  __device__ __forceinline__ static V pack(const float (&v)[8]) {
    V r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (_Float16)v[e];
    return r;
  }
  __device__ __forceinline__ static f32x16 mma(V a, V b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct MmaOps<IoBF16> {
  typedef bf16x8 V;
  __device__ __forceinline__ static V pack(const float (&v)[8]) {
    V r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (__bf16)v[e];
    return r;
  }
  __device__ __forceinline__ static f32x16 mma(V a, V b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// Bin of the butterfly held in output slot q (q < 8) by half h of the wave.
__device__ __forceinline__ int out_bin(int q, int h) { return 4 * h + q + (q & 4); }

template <bool INV, class IO>
__global__ __launch_bounds__(kThreads) void k_stockham_mma(const uint32_t* in, uint32_t* out,
                                                           const c32* tw, int64_t rows) {
  using Ops = MmaOps<IO>;
  __shared__ alignas(16) c32 lds[kLds];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int jl = lane & 31;
  const int h = lane >> 5;
  const int64_t row = blockIdx.x;
  if (row >= rows) return;  // whole workgroup, before any barrier

  // The DFT matrix as the A operand: row jl, columns 8h + e (first product,
  // real legs) and 16 + 8h + e (second product, imaginary legs).
  typename Ops::V a_re, a_im;
  {
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      re[e] = dft_entry<INV>(jl, 8 * h + e);
      im[e] = dft_entry<INV>(jl, 16 + 8 * h + e);
    }
    a_re = Ops::pack(re);
    a_im = Ops::pack(im);
  }

  int j[kBlocks];
#pragma unroll
  for (int b = 0; b < kBlocks; ++b) j[b] = 32 * ((tid >> 6) * kBlocks + b) + jl;

  // Legs 8h + e of each butterfly, and every twiddle up front (passes 1, 2:
  // W_{16 Ns}^{r (j mod Ns)} for leg r, table entry (r - 1) Ns + j mod Ns).
  c32 d[kBlocks][8];
  c32 w1[kBlocks][8], w2[kBlocks][8];
  const uint32_t* src = in + row * kN;
#pragma unroll
  for (int b = 0; b < kBlocks; ++b)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = 8 * h + e;
      d[b][e] = IO::load(__builtin_nontemporal_load(src + j[b] + r * kNB));
      const int r1 = r > 0 ? r - 1 : 0;
      w1[b][e] = tw[r1 * 16 + (j[b] & 15)];
      w2[b][e] = tw[15 * 16 + r1 * 256 + j[b]];
      if (r == 0) w1[b][e] = w2[b][e] = c32{1.f, 0.f};
    }

  c32 o[kBlocks][8];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    // Operands of every block first, then the products block after block, so
    // that one block's products run while the next block's are issued.
    typename Ops::V b_re[kBlocks], b_im[kBlocks];
#pragma unroll
    for (int b = 0; b < kBlocks; ++b) {
      float re[8], im[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        c32 v = d[b][e];
        if (p == 1) v = ctw<INV>(v, w1[b][e]);
        if (p == 2) v = ctw<INV>(v, w2[b][e]);
        re[e] = v.x;
        im[e] = v.y;
      }
      b_re[b] = Ops::pack(re);
      b_im[b] = Ops::pack(im);
    }
    f32x16 acc[kBlocks];
#pragma unroll
    for (int b = 0; b < kBlocks; ++b) acc[b] = Ops::mma(a_re, b_re[b], f32x16{});
#pragma unroll
    for (int b = 0; b < kBlocks; ++b) acc[b] = Ops::mma(a_im, b_im[b], acc[b]);
#pragma unroll
    for (int b = 0; b < kBlocks; ++b)
#pragma unroll
      for (int q = 0; q < 8; ++q) o[b][q] = c32{acc[b][q], acc[b][8 + q]};
    if (p < 2) {
      // Bin k of butterfly j goes to x = (j / Ns) Ns 16 + j mod Ns + k Ns; the
      // next pass reads leg r of butterfly j at j + r N / 16.  With one pad
      // element per 16 the padded slots are affine in k and r: pidx(x) =
      // pidx(x at k = 0) + k for Ns = 1 (x = 16 j + k) and + 17 k for Ns = 16,
      // and pidx(j + 256 r) = pidx(j) + 272 r, so every access is a base
      // address plus a constant.
      const int ns = p == 0 ? 1 : 16;
      const int step = p == 0 ? 1 : 17;
#pragma unroll
      for (int b = 0; b < kBlocks; ++b) {
        c32* wr = lds + pidx((j[b] / ns) * ns * 16 + (j[b] & (ns - 1))) + step * 4 * h;
#pragma unroll
        for (int q = 0; q < 8; ++q) wr[step * (q + (q & 4))] = o[b][q];
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < kBlocks; ++b) {
        const c32* rd = lds + pidx(j[b]) + 272 * 8 * h;
#pragma unroll
        for (int e = 0; e < 8; ++e) d[b][e] = rd[272 * e];
      }
      __syncthreads();
    }
  }
  // Last pass (Ns = 256): bin k of butterfly j is element j + 256 k.
  uint32_t* dst = out + row * kN;
#pragma unroll
  for (int b = 0; b < kBlocks; ++b)
#pragma unroll
    for (int q = 0; q < 8; ++q)
      __builtin_nontemporal_store(IO::store(o[b][q]), dst + j[b] + out_bin(q, h) * kNB);
}

template <class IO>
hipError_t launch_mma(const void* in, void* out, const void* tw, int64_t batch, bool inverse,
                      hipStream_t s) {
  const int64_t cap = max_groups_per_launch();
  for (int64_t r0 = 0; r0 < batch; r0 += cap) {
    const int64_t g = batch - r0 < cap ? batch - r0 : cap;
    const uint32_t* ip = static_cast<const uint32_t*>(in) + r0 * kN;
    uint32_t* op = static_cast<uint32_t*>(out) + r0 * kN;
    const c32* twp = static_cast<const c32*>(tw);
    if (inverse)
      k_stockham_mma<true, IO><<<dim3((unsigned)g), dim3(kThreads), 0, s>>>(ip, op, twp, batch - r0);
    else
      k_stockham_mma<false, IO><<<dim3((unsigned)g), dim3(kThreads), 0, s>>>(ip, op, twp, batch - r0);
  }
  return hipGetLastError();
}

}  // namespace

bool mma_supported(const SingleVariant& v) {
  return v.n == kN && v.npass == 3 && v.radix[0] == 16 && v.radix[1] == 16 && v.radix[2] == 16;
}

hipError_t launch_mma_f16(const void* in, void* out, const void* tw, int64_t batch, bool inverse,
                          hipStream_t s) {
  return launch_mma<IoF16>(in, out, tw, batch, inverse, s);
}

hipError_t launch_mma_bf16(const void* in, void* out, const void* tw, int64_t batch,
                           bool inverse, hipStream_t s) {
  return launch_mma<IoBF16>(in, out, tw, batch, inverse, s);
}

}  // namespace stockfft
