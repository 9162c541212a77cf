// Two-tier exchange for N = 4096 = 8^4: the register-and-shuffle tier of the
// paper's two-tier model (Section III-B) re-derived for 64-lane waves.
//
// In a radix-8 Stockham plan of 4096 points (passes with Ns = 1, 8, 64, 512)
// the exchange after pass 0 and the exchange after pass 2 are each a set of
// independent 8 x 8 transposes:
//   after pass 0, butterfly j1 = 8 g + m of pass 1 takes leg r from output m
//   of pass-0 butterfly g + 64 r (g in [0, 64), m, r in [0, 8));
//   after pass 2, butterfly j3 = h + 64 m of pass 3 takes leg r from output m
//   of pass-2 butterfly h + 64 r (h in [0, 64)).
// So if the 8 butterflies of a group (g or h) sit in 8 lanes of one wave --
// lane bits 3..5 hold the member m, lane bits 0..2 and the wave the group --
// each of those exchanges is a transpose between the member bits of the lane
// and the leg index of the registers, done in registers with cross-lane
// moves and no LDS and no barrier: lane bit 5 by v_permlane32_swap, bit 4 by
// v_permlane16_swap (both gfx950), bit 3 by a DPP row rotation by 8 (lane
// xor 8 within each 16-lane row) and a select.  Only the exchange after pass
// 1 (butterfly 8 g + m writes 64 g + m + 8 r; butterfly h + 64 m of pass 2
// reads h + 64 m + 512 r) crosses waves and goes through the LDS: one write,
// one barrier, one read per transform, where the all-LDS schedule has three
// exchanges and five barriers.  The arithmetic is the Stockham pass of
// stockham.hpp unchanged (same twiddle tables, same DFT_8), only the
// butterfly-to-lane map differs per pass.
//
// The price is in the global accesses: a wave owns 8 G groups, so for one
// leg its loads cover G 8-byte values at 8 G consecutive positions for each
// of the 8 members (positions g + 64 m): runs of 64 G bytes instead of one
// 512-byte run.  G = 2 (two adjacent groups per lane, 16 values per lane)
// makes every run a whole 128-byte line and every access 16 bytes.
#pragma once

#include "stockham.hpp"

namespace stockfft {

template <class Base, int G_>
struct WaveExchange : Base {
  static_assert(Base::N == 4096 && Base::P == 4 && Base::radix(0) == 8 && Base::radix(1) == 8 &&
                    Base::radix(2) == 8 && Base::radix(3) == 8,
                "the in-wave exchange is derived for the radix-8 plan of 4096 points");
  static_assert(G_ == 1 || G_ == 2, "one or two groups per lane");
  static_assert(Base::E == 8 * G_ && Base::TPB == 1 && Base::C == 1, "shape");
  static constexpr int WX = G_;
  // The one LDS exchange uses its own swizzle over 4096 elements (wx_slot).
  static constexpr int LDS_ELEMS = 4096;
};

template <class S, class = void>
struct wave_exchange : std::integral_constant<int, 0> {};
template <class S>
struct wave_exchange<S, std::void_t<decltype(S::WX)>> : std::integral_constant<int, S::WX> {};

// Physical LDS slot of exchange position i = 64 q + 8 b + c (c, b in [0, 8)):
// bits 0..4 of i are xor-ed with bits 6..9, a bijection inside every block
// of 64.  For both access patterns of the exchange (writes at 64 g + m + 8 r,
// reads at h + 64 m + 512 r; lanes vary the group's low bits and the member)
// any 32 consecutive lanes then hit 32 different 8-byte slots modulo 32,
// i.e. all 64 four-byte banks once (checked on the CPU for every access).
__device__ __forceinline__ int wx_slot(int i) {
  const int q = i >> 6;
  return i ^ (q & 7) ^ (((q ^ (q >> 3)) & 1) << 3) ^ (((q >> 1) & 1) << 4);
}

// Swaps two 32-bit values between lane halves: lanes 32..63 of p with lanes
// 0..31 of q.
__device__ __forceinline__ void swap_lanes32(float& p, float& q) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(p), __float_as_uint(q), false, false);
  p = __uint_as_float(r[0]);
  q = __uint_as_float(r[1]);
}
// Lanes 16..31 and 48..63 of p with lanes 0..15 and 32..47 of q.
__device__ __forceinline__ void swap_lanes16(float& p, float& q) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(p), __float_as_uint(q), false, false);
  p = __uint_as_float(r[0]);
  q = __uint_as_float(r[1]);
}
// Lanes with bit 3 set trade their p for q of lane ^ 8, so (lane, p) and
// (lane ^ 8, q) are exchanged wherever bit 3 of the lane differs from the
// slot bit (p: 0, q: 1).  DPP row_ror:8 reads lane ^ 8 inside a 16-lane row.
__device__ __forceinline__ void swap_lanes8(float& p, float& q, bool hi) {
  const unsigned pu = __float_as_uint(p), qu = __float_as_uint(q);
  const unsigned from_q = __builtin_amdgcn_update_dpp(0u, qu, 0x128, 0xf, 0xf, false);
  const unsigned from_p = __builtin_amdgcn_update_dpp(0u, pu, 0x128, 0xf, 0xf, false);
  p = __uint_as_float(hi ? from_q : pu);
  q = __uint_as_float(hi ? qu : from_p);
}

// 8 x 8 transpose between lane bits 3..5 and the register index: afterwards
// lane (member m) register r holds what lane (member r) register m held, for
// the 8 lanes of the same lane bits 0..2.
__device__ __forceinline__ void transpose8(c32 (&v)[8], bool hi3) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    swap_lanes32(v[i].x, v[i + 4].x);
    swap_lanes32(v[i].y, v[i + 4].y);
  }
#pragma unroll
  for (int i = 0; i < 8; i += (i & 1) ? 3 : 1) {  // 0, 1, 4, 5
    swap_lanes16(v[i].x, v[i + 2].x);
    swap_lanes16(v[i].y, v[i + 2].y);
  }
#pragma unroll
  for (int i = 0; i < 8; i += 2) {
    swap_lanes8(v[i].x, v[i + 1].x, hi3);
    swap_lanes8(v[i].y, v[i + 1].y, hi3);
  }
}

// Raw storage of one value (8 bytes FP32, 4 bytes 16-bit) and of the G
// adjacent values a lane moves with one access.
template <class IO, int G>
struct WxAccess {
  static constexpr int B = IO::BYTES;
  static constexpr int BYTES = B * G;
  __device__ __forceinline__ static void load(c32 (&v)[G], const Buf& b, int voff, int soff) {
    if constexpr (BYTES == 16) {
      const u32x4 r = b.ld128<kNT>(voff, soff);
      v[0] = IO::load(u32x2{r.x, r.y});
      v[1] = IO::load(u32x2{r.z, r.w});
    } else if constexpr (BYTES == 8 && B == 8) {
      v[0] = IO::load(b.ld64<kNT>(voff, soff));
    } else if constexpr (BYTES == 8) {
      const u32x2 r = b.ld64<kNT>(voff, soff);
      v[0] = IO::load(r.x);
      v[1] = IO::load(r.y);
    } else {
      v[0] = IO::load(b.ld32<kNT>(voff, soff));
    }
  }
  __device__ __forceinline__ static void store(const c32 (&v)[G], const Buf& b, int voff, int soff) {
    if constexpr (BYTES == 16) {
      const u32x2 p = IO::store(v[0]), q = IO::store(v[1]);
      b.st128<kNT>(u32x4{p.x, p.y, q.x, q.y}, voff, soff);
    } else if constexpr (BYTES == 8 && B == 8) {
      b.st64<kNT>(IO::store(v[0]), voff, soff);
    } else if constexpr (BYTES == 8) {
      b.st64<kNT>(u32x2{IO::store(v[0]), IO::store(v[1])}, voff, soff);
    } else {
      b.st32<kNT>(IO::store(v[0]), voff, soff);
    }
  }
};

// One 4096-point transform per workgroup of 512 / G lanes.  Lane l of wave w
// is member m = l >> 3 of the groups G (8 w + (l & 7)) + u, u < G.
template <class S, bool INV, class IO>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_stockham_wx(const void* in, void* out,
                                                             const c32* tw, int64_t rows) {
  constexpr int G = S::WX;
  using A = WxAccess<IO, G>;
  constexpr int B = IO::BYTES;
  __shared__ alignas(16) c32 lds[S::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int m = lane >> 3;
  const int g0 = G * (8 * (tid >> 6) + (lane & 7));  // first group of the lane
  const bool hi3 = (lane & 8) != 0;
  const int64_t row = blockIdx.x;
  (void)rows;  // one row per workgroup: the grid is the batch

  // Pass 0 legs: butterfly g + 64 m reads x[g + 64 m + 512 r].
  c32 a[G][8];
  {
    const Buf src(static_cast<const char*>(in) + row * 4096 * B);
    const int voff = B * (g0 + 64 * m);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      c32 v[G];
      A::load(v, src, voff, B * 512 * r);
#pragma unroll
      for (int u = 0; u < G; ++u) a[u][r] = v[u];
    }
  }
  // Every twiddle, loaded behind the input: pass 1 (k = m, shared by the
  // lane's groups), pass 2 (k = h), pass 3 (k = h + 64 m).
  c32 w1[8], w2[G][8], w3[G][8];
  fetch_twiddles<S, 1>(w1, 0, tw + S::tw_off(1), m);
#pragma unroll
  for (int u = 0; u < G; ++u) {
    fetch_twiddles<S, 2>(w2[u], 0, tw + S::tw_off(2), g0 + u);
    fetch_twiddles<S, 3>(w3[u], 0, tw + S::tw_off(3), g0 + u + 64 * m);
  }

  // Pass 0, in-wave exchange, pass 1.
#pragma unroll
  for (int u = 0; u < G; ++u) {
    Dft<8, INV>::run(a[u]);
    transpose8(a[u], hi3);
#pragma unroll
    for (int r = 1; r < 8; ++r) a[u][r] = ctw<INV>(a[u][r], w1[r - 1]);
    Dft<8, INV>::run(a[u]);
  }
  // The LDS exchange: butterfly 8 g + m writes leg r to 64 g + m + 8 r;
  // butterfly h + 64 m of pass 2 reads h + 64 m + 512 r.  Both slot maps are
  // one xor of a lane value with the leg's bits (wx_slot leaves bits 5 and
  // up alone and is linear over the bits it mixes).
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const int base = 64 * (g0 + u) + m;
    const int sb = wx_slot(base);
#pragma unroll
    for (int r = 0; r < 8; ++r) lds[sb ^ (8 * r)] = a[u][r];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const int base = g0 + u + 64 * m;
    const int s0 = wx_slot(base), s1 = wx_slot(base + 512);
#pragma unroll
    for (int r = 0; r < 8; ++r) a[u][r] = lds[((r & 1) ? s1 - 512 : s0) + 512 * r];
  }
  // Pass 2, in-wave exchange, pass 3.
#pragma unroll
  for (int u = 0; u < G; ++u) {
#pragma unroll
    for (int r = 1; r < 8; ++r) a[u][r] = ctw<INV>(a[u][r], w2[u][r - 1]);
    Dft<8, INV>::run(a[u]);
    transpose8(a[u], hi3);
#pragma unroll
    for (int r = 1; r < 8; ++r) a[u][r] = ctw<INV>(a[u][r], w3[u][r - 1]);
    Dft<8, INV>::run(a[u]);
  }
  // Pass 3 output leg r of butterfly h + 64 m goes to h + 64 m + 512 r.
  {
    const Buf dst(static_cast<char*>(out) + row * 4096 * B);
    const int voff = B * (g0 + 64 * m);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      c32 v[G];
#pragma unroll
      for (int u = 0; u < G; ++u) v[u] = a[u][r];
      A::store(v, dst, voff, B * 512 * r);
    }
  }
}

template <class S, class IO>
hipError_t launch_wx(const void* in, void* out, const void* tw, int64_t batch, bool inverse,
                     hipStream_t s) {
  const int64_t cap = max_groups_per_launch();
  for (int64_t r0 = 0; r0 < batch; r0 += cap) {
    const int64_t g = batch - r0 < cap ? batch - r0 : cap;
    const char* ip = static_cast<const char*>(in) + r0 * 4096 * IO::BYTES;
    char* op = static_cast<char*>(out) + r0 * 4096 * IO::BYTES;
    const c32* twp = static_cast<const c32*>(tw);
    if (inverse)
      k_stockham_wx<S, true, IO><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(ip, op, twp, g);
    else
      k_stockham_wx<S, false, IO><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(ip, op, twp, g);
  }
  return hipGetLastError();
}

}  // namespace stockfft
