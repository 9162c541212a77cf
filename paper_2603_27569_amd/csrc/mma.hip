// Radix-16 Stockham passes whose 16-point DFTs run on the matrix cores
// (the paper's matrix-multiply DFT of Sections V-C and VII-C, and its
// future-work items on batched matrix-core FFTs and mixed precision,
// Section IX-A), for N = 512 ... 16384 with binary16 or bfloat16 storage.
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

// N = 16^P * RL: P radix-16 passes on the matrix cores, then (RL > 1) one
// radix-RL pass on the vector ALUs.
template <int N>
struct MmaPlan {
  static constexpr int RL = N == 512 || N == 8192 ? 2 : N == 1024 || N == 16384 ? 4 : N == 2048 ? 8 : 1;
  static constexpr int P = N / RL == 256 ? 2 : 3;
  static constexpr int NB = N / 16;     // butterflies per radix-16 pass
  static constexpr int NL = N / RL;     // butterflies of the last pass (RL > 1)
  static constexpr int LDS = N + N / 16;  // one pad slot per 16 against bank conflicts
  static_assert(N / RL == (P == 2 ? 256 : 4096) && NB % 32 == 0, "unsupported length");
  // Offset of pass p's twiddle table (entries [r - 1][k], as the host builds it).
  static constexpr int tw_off(int p) {
    int o = 0, ns = 16;
    for (int i = 1; i < p; ++i, ns *= 16) o += 15 * ns;
    return o;
  }
};

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

// TPWG transforms per workgroup of THREADS lanes, each wave taking kBlocks
// blocks of 32 butterflies (of one transform or, for short transforms,
// several): fewer waves per block of work mean more independent products per
// wave and no barrier waits across waves, more waves fewer registers and more
// transforms in flight.  One wave per workgroup is held to two waves per SIMD.
template <int N, int THREADS, int TPWG, bool INV, class IO>
__global__ __launch_bounds__(THREADS, THREADS == 64 ? 2 : 1) void k_stockham_mma(
    const uint32_t* in, uint32_t* out, const c32* tw, int64_t rows) {
  using M = MmaPlan<N>;
  constexpr int NB = M::NB;
  constexpr int BPT = NB / 32;  // blocks per transform
  constexpr int kBlocks = TPWG * BPT / (THREADS / 64);
  static_assert(kBlocks >= 1 && kBlocks * (THREADS / 64) == TPWG * BPT, "lanes per transform");
  using Ops = MmaOps<IO>;
  using V = typename Ops::V;
  __shared__ alignas(16) uint32_t lds[TPWG * M::LDS];  // 16-bit pairs, one pad per 16
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int jl = lane & 31;
  const int h = lane >> 5;
  const int64_t row0 = (int64_t)blockIdx.x * TPWG;
  if (row0 >= rows) return;  // whole workgroup, before any barrier

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

  // Block b of this wave: transform tr[b] of the workgroup, butterfly j[b];
  // rows past the batch (a last, partial workgroup) compute on zeros and
  // store nothing.
  int j[kBlocks], tr[kBlocks];
  bool live[kBlocks];
#pragma unroll
  for (int b = 0; b < kBlocks; ++b) {
    const int g = (tid >> 6) * kBlocks + b;
    tr[b] = TPWG > 1 ? g / BPT : 0;
    j[b] = 32 * (g - tr[b] * BPT) + jl;
    live[b] = TPWG == 1 || row0 + tr[b] < rows;  // one transform: row0 < rows
  }

  // Legs 8h + e of each butterfly as stored pairs: the first pass takes its
  // operands straight from HBM, the later ones from LDS, where the writer has
  // already applied their twiddles and rounded.
  uint32_t d[kBlocks][8];
#pragma unroll
  for (int b = 0; b < kBlocks; ++b) {
    const uint32_t* src = in + (row0 + tr[b]) * N;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      d[b][e] = live[b] ? __builtin_nontemporal_load(src + j[b] + (8 * h + e) * NB) : 0u;
  }

#pragma unroll
  for (int p = 0; p < M::P; ++p) {
    const int ns = 1 << (4 * p);  // Ns of this pass
    const bool last16 = p == M::P - 1;
    // Bin k of butterfly j goes to x = (j / Ns) Ns 16 + j mod Ns + k Ns.  The
    // next pass (radix R', Ns' = 16 Ns, N / R' butterflies) reads it as leg
    // r' = x / (N / R') of butterfly j' = x mod (N / R'), whose twiddle there
    // is W_{Ns' R'}^{r' (j' mod Ns')}: table entry tw_off + (r' - 1) Ns' + j'
    // mod Ns'.  Loaded before the products.
    c32 wn[kBlocks][8];
    if (!last16 || M::RL > 1) {
      const int nsn = 16 * ns;
      const int span = last16 ? M::NL : NB;  // N / R' (a power of two)
      const int off = M::tw_off(p + 1);
#pragma unroll
      for (int b = 0; b < kBlocks; ++b) {
        const int base = (j[b] / ns) * ns * 16 + (j[b] & (ns - 1));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int x = base + out_bin(q, h) * ns;
          const int r = x / span, jn = x & (span - 1);
          wn[b][q] = r > 0 ? tw[off + (r - 1) * nsn + (jn & (nsn - 1))] : c32{1.f, 0.f};
        }
      }
    }
    f32x16 acc[kBlocks];
#pragma unroll
    for (int b = 0; b < kBlocks; ++b)
      acc[b] = Ops::mma(a_re, gather_halves<V>(d[b], false), f32x16{});
#pragma unroll
    for (int b = 0; b < kBlocks; ++b) acc[b] = Ops::mma(a_im, gather_halves<V>(d[b], true), acc[b]);
    if (last16 && M::RL == 1) {
      // Last pass (Ns = N / 16): bin k of butterfly j is element j + k N / 16.
#pragma unroll
      for (int b = 0; b < kBlocks; ++b) {
        if (!live[b]) continue;
        uint32_t* dst = out + (row0 + tr[b]) * N;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          __builtin_nontemporal_store(IO::store(c32{acc[b][q], acc[b][8 + q]}),
                                      dst + j[b] + out_bin(q, h) * NB);
      }
      return;
    }
    // With one pad element per 16 the padded slots are affine in k: pidx(x) =
    // pidx(x at k = 0) + k for Ns = 1 (x = 16 j + k) and + 17 Ns / 16 k for
    // Ns >= 16, so every write is a base address plus a constant.
    const int step = p == 0 ? 1 : 17 * ns / 16;
#pragma unroll
    for (int b = 0; b < kBlocks; ++b) {
      uint32_t* wr = lds + tr[b] * M::LDS + pidx((j[b] / ns) * ns * 16 + (j[b] & (ns - 1))) +
                     step * 4 * h;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        wr[step * (q + (q & 4))] = IO::store(ctw<INV>(c32{acc[b][q], acc[b][8 + q]}, wn[b][q]));
    }
    __syncthreads();
    if (!last16) {
      // pidx(j + r N / 16) = pidx(j) + 17 N / 256 r.
#pragma unroll
      for (int b = 0; b < kBlocks; ++b) {
        const uint32_t* rd = lds + tr[b] * M::LDS + pidx(j[b]) + (17 * NB / 16) * 8 * h;
#pragma unroll
        for (int e = 0; e < 8; ++e) d[b][e] = rd[(17 * NB / 16) * e];
      }
      __syncthreads();
    }
  }
  if constexpr (M::RL > 1) {
    // The radix-RL pass (Ns = N / RL) on the vector ALUs in FP32: butterfly j
    // reads legs j + r N / RL (twiddles already applied) and writes bin k to
    // element j + k N / RL.
    constexpr int R = M::RL, NL = M::NL;
#pragma unroll
    for (int i = tid; i < TPWG * NL; i += THREADS) {
      const int t = i / NL, jb = i - t * NL;
      if (row0 + t >= rows) continue;
      const uint32_t* rd = lds + t * M::LDS;
      c32 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = IO::load(rd[pidx(jb + r * NL)]);
      Dft<R, INV>::run(v);
      uint32_t* dst = out + (row0 + t) * N;
#pragma unroll
      for (int k = 0; k < R; ++k) __builtin_nontemporal_store(IO::store(v[k]), dst + jb + k * NL);
    }
  }
}

template <int N, int THREADS, class IO, int TPWG = 1>
hipError_t launch_mma_threads(const void* in, void* out, const void* tw, int64_t batch,
                              bool inverse, hipStream_t s) {
  const int64_t cap = max_groups_per_launch() * TPWG;  // rows per launch
  for (int64_t r0 = 0; r0 < batch; r0 += cap) {
    const int64_t rows = batch - r0 < cap ? batch - r0 : cap;
    const uint32_t* ip = static_cast<const uint32_t*>(in) + r0 * N;
    uint32_t* op = static_cast<uint32_t*>(out) + r0 * N;
    const c32* twp = static_cast<const c32*>(tw);
    const dim3 grid((unsigned)((rows + TPWG - 1) / TPWG)), block(THREADS);
    if (inverse)
      k_stockham_mma<N, THREADS, TPWG, true, IO><<<grid, block, 0, s>>>(ip, op, twp, rows);
    else
      k_stockham_mma<N, THREADS, TPWG, false, IO><<<grid, block, 0, s>>>(ip, op, twp, rows);
  }
  return hipGetLastError();
}

// Lanes per transform.  N = 4096 by batch, from measurements (binary16,
// microseconds per launch for 256 / 128 / 64 lanes): batch 256: 5.2 / 5.7 /
// 7.3, 2048: 23.0 / 17.1 / 17.5, 16384: 152 / 131 / 120.  The bfloat16 kernel
// needs more registers (its twiddle product and rounding do not fuse), and
// with one wave per transform it spills: it stops at two waves.  Other
// lengths (measured at about 64 MiB per launch): up to 2048 one wave per
// workgroup with four blocks of 32 butterflies (eight spill), so 512 and 1024
// take several transforms per workgroup (2048: 17.8 against 23.1 us with two
// waves of two blocks at 2048 x 4096), 8192
// four blocks per wave (23.1 against 24.3 with two), 16384 two blocks per
// wave (28.8 against 29.4 with four).
template <class IO>
hipError_t launch_mma(int64_t n, const void* in, void* out, const void* tw, int64_t batch,
                      bool inverse, hipStream_t s) {
  constexpr bool f16 = std::is_same<IO, IoF16>::value;
  switch (n) {
    case 512: return launch_mma_threads<512, 64, IO, 4>(in, out, tw, batch, inverse, s);
    case 1024: return launch_mma_threads<1024, 64, IO, 2>(in, out, tw, batch, inverse, s);
    case 2048: return launch_mma_threads<2048, 64, IO, 1>(in, out, tw, batch, inverse, s);
    case 8192: return launch_mma_threads<8192, 256, IO>(in, out, tw, batch, inverse, s);
    case 16384: return launch_mma_threads<16384, 1024, IO>(in, out, tw, batch, inverse, s);
    default: break;
  }
  if (batch <= 512) return launch_mma_threads<4096, 256, IO>(in, out, tw, batch, inverse, s);
  if constexpr (f16)
    if (batch > 4096) return launch_mma_threads<4096, 64, IO>(in, out, tw, batch, inverse, s);
  return launch_mma_threads<4096, 128, IO>(in, out, tw, batch, inverse, s);
}

}  // namespace

bool mma_supported(int64_t n) {
  return n == 512 || n == 1024 || n == 2048 || n == 4096 || n == 8192 || n == 16384;
}

const char* mma_table_variant(int64_t n) {
  switch (n) {
    case 512: return "n512_e16_b2_p4_r16.16.2";
    case 1024: return "n1024_e16_b1_p4_r16.16.4";
    case 2048: return "n2048_e16_b1_p4_r16.16.8";
    case 4096: return "n4096_e16_b1_p4_r16.16.16";
    case 8192: return "n8192_e32_b1_p4_r16.16.16.2";
    case 16384: return "n16384_e16_b1_p4_r16.16.16.4";
    default: return nullptr;
  }
}

hipError_t launch_mma_f16(int64_t n, const void* in, void* out, const void* tw, int64_t batch,
                          bool inverse, hipStream_t s) {
  return launch_mma<IoF16>(n, in, out, tw, batch, inverse, s);
}

hipError_t launch_mma_bf16(int64_t n, const void* in, void* out, const void* tw, int64_t batch,
                           bool inverse, hipStream_t s) {
  return launch_mma<IoBF16>(n, in, out, tw, batch, inverse, s);
}

}  // namespace stockfft
