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
// sums are FP32.  Each pass's outputs get the next pass's twiddles in FP32 on
// the vector ALUs and are rounded once to the 16-bit format as they go into
// LDS, so the exchange moves 16-bit pairs and the next pass reads its
// operands without converting (the first pass reads them from HBM as
// stored).
//
// Lane layouts of the 32x32x16 products (checked on gfx950): lane l holds
// A[l % 32][8 (l / 32) + e] and B[8 (l / 32) + e][l % 32] for e < 8, and the
// result D[8 (g / 4) + 4 (l / 32) + g % 4][l % 32] in accumulator g < 16.
// So lane (j = l % 32, h = l / 32) supplies legs 8h .. 8h + 7 of butterfly j
// (real parts to the first product, imaginary parts to the second) and gets
// back bins 4h .. 4h + 3 and 8 + 4h .. 8 + 4h + 3 of the same butterfly, real
// parts in accumulators 0 .. 7 and imaginary parts in 8 .. 15.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"
#include "kernels.hpp"

namespace stockfft {
namespace {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kN = 4096;
constexpr int kNB = kN / 16;              // butterflies per pass
constexpr int kLds = kN + kN / 16;        // one pad slot per 16 against bank conflicts

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

// The 8 real parts (lo) or imaginary parts (hi) of 8 stored 16-bit pairs as
// one operand: dword i of the operand is half 0 or 1 of pairs 2i and 2i + 1.
template <class V>
__device__ __forceinline__ V gather_halves(const uint32_t (&d)[8], bool hi) {
  const unsigned sel = hi ? 0x07060302u : 0x05040100u;
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = __builtin_amdgcn_perm(d[2 * i + 1], d[2 * i], sel);
  return __builtin_bit_cast(V, w);
}

// THREADS lanes per transform (one, two or four waves), each wave taking
// kBlocks blocks of 32 butterflies: fewer waves mean more independent
// products per wave and no barrier waits across waves, more waves fewer
// registers and more transforms in flight.  One wave per transform is held
// to two waves per SIMD (at most 256 VGPRs).
template <int THREADS, bool INV, class IO>
__global__ __launch_bounds__(THREADS, THREADS == 64 ? 2 : 1) void k_stockham_mma(
    const uint32_t* in, uint32_t* out, const c32* tw, int64_t rows) {
  constexpr int kBlocks = kNB / 32 / (THREADS / 64);
  using Ops = MmaOps<IO>;
  using V = typename Ops::V;
  __shared__ alignas(16) uint32_t lds[kLds];  // 16-bit pairs, one pad per 16
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int jl = lane & 31;
  const int h = lane >> 5;
  const int64_t row = blockIdx.x;
  if (row >= rows) return;  // whole workgroup, before any barrier

  // The DFT matrix as the A operand: row jl, columns 8h + e (first product,
  // real legs) and 16 + 8h + e (second product, imaginary legs).
  V a_re, a_im;
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
  for (int b = 0; b < kBlocks; ++b) j[b] = 32 * ((tid >> 6) * kBlocks + b) + jl;  // butterfly

  // Legs 8h + e of each butterfly as stored pairs: the first pass takes its
  // operands straight from HBM, the later ones from LDS, where the writer has
  // already applied their twiddles and rounded.
  uint32_t d[kBlocks][8];
  const uint32_t* src = in + row * kN;
#pragma unroll
  for (int b = 0; b < kBlocks; ++b)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      d[b][e] = __builtin_nontemporal_load(src + j[b] + (8 * h + e) * kNB);

#pragma unroll
  for (int p = 0; p < 3; ++p) {
    // Bin k of butterfly j goes to x = (j / Ns) Ns 16 + j mod Ns + k Ns, which
    // the next pass reads as leg r' = x / 256 = j / 16 of butterfly j' = x mod
    // 256; its twiddle there is W_{16 Ns'}^{r' (j' mod Ns')} (Ns' = 16 Ns):
    // table entry (r' - 1) 16 + k after the first pass, 240 + (r' - 1) 256 +
    // j mod 16 + 16 k after the second.  Loaded before the products.
    c32 wn[kBlocks][8];
    if (p < 2) {
#pragma unroll
      for (int b = 0; b < kBlocks; ++b) {
        const int r = j[b] >> 4;
        const int r1 = r > 0 ? r - 1 : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = out_bin(q, h);
          const int idx = p == 0 ? r1 * 16 + k : 240 + r1 * 256 + (j[b] & 15) + 16 * k;
          wn[b][q] = r > 0 ? tw[idx] : c32{1.f, 0.f};
        }
      }
    }
    f32x16 acc[kBlocks];
#pragma unroll
    for (int b = 0; b < kBlocks; ++b)
      acc[b] = Ops::mma(a_re, gather_halves<V>(d[b], false), f32x16{});
#pragma unroll
    for (int b = 0; b < kBlocks; ++b) acc[b] = Ops::mma(a_im, gather_halves<V>(d[b], true), acc[b]);
    if (p < 2) {
      // With one pad element per 16 the padded slots are affine in k and r:
      // pidx(x) = pidx(x at k = 0) + k for Ns = 1 (x = 16 j + k) and + 17 k
      // for Ns = 16, and pidx(j + 256 r) = pidx(j) + 272 r.
      const int ns = p == 0 ? 1 : 16;
      const int step = p == 0 ? 1 : 17;
#pragma unroll
      for (int b = 0; b < kBlocks; ++b) {
        uint32_t* wr = lds + pidx((j[b] / ns) * ns * 16 + (j[b] & (ns - 1))) + step * 4 * h;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          wr[step * (q + (q & 4))] = IO::store(ctw<INV>(c32{acc[b][q], acc[b][8 + q]}, wn[b][q]));
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < kBlocks; ++b) {
        const uint32_t* rd = lds + pidx(j[b]) + 272 * 8 * h;
#pragma unroll
        for (int e = 0; e < 8; ++e) d[b][e] = rd[272 * e];
      }
      __syncthreads();
    } else {
      // Last pass (Ns = 256): bin k of butterfly j is element j + 256 k.
      uint32_t* dst = out + row * kN;
#pragma unroll
      for (int b = 0; b < kBlocks; ++b)
#pragma unroll
        for (int q = 0; q < 8; ++q)
          __builtin_nontemporal_store(IO::store(c32{acc[b][q], acc[b][8 + q]}),
                                      dst + j[b] + out_bin(q, h) * kNB);
    }
  }
}

template <int THREADS, class IO>
hipError_t launch_mma_threads(const void* in, void* out, const void* tw, int64_t batch,
                              bool inverse, hipStream_t s) {
  const int64_t cap = max_groups_per_launch();
  for (int64_t r0 = 0; r0 < batch; r0 += cap) {
    const int64_t g = batch - r0 < cap ? batch - r0 : cap;
    const uint32_t* ip = static_cast<const uint32_t*>(in) + r0 * kN;
    uint32_t* op = static_cast<uint32_t*>(out) + r0 * kN;
    const c32* twp = static_cast<const c32*>(tw);
    const dim3 grid((unsigned)g), block(THREADS);
    if (inverse)
      k_stockham_mma<THREADS, true, IO><<<grid, block, 0, s>>>(ip, op, twp, batch - r0);
    else
      k_stockham_mma<THREADS, false, IO><<<grid, block, 0, s>>>(ip, op, twp, batch - r0);
  }
  return hipGetLastError();
}

// Lanes per transform by batch, from measurements at N = 4096 (binary16,
// microseconds per launch for 256 / 128 / 64 lanes): batch 256: 5.2 / 5.7 / 7.3,
// 2048: 23.0 / 17.1 / 17.5, 16384: 152 / 131 / 120.  The bfloat16 kernel
// needs more registers (its twiddle product and rounding do not fuse), and
// with one wave per transform it spills: it stops at two waves.
template <class IO>
hipError_t launch_mma(const void* in, void* out, const void* tw, int64_t batch, bool inverse,
                      hipStream_t s) {
  if (batch <= 512) return launch_mma_threads<256, IO>(in, out, tw, batch, inverse, s);
  if constexpr (std::is_same<IO, IoF16>::value)
    if (batch > 4096) return launch_mma_threads<64, IO>(in, out, tw, batch, inverse, s);
  return launch_mma_threads<128, IO>(in, out, tw, batch, inverse, s);
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
