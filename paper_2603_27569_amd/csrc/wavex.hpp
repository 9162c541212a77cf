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
// The price is in the global accesses and in the moves: with one member per
// lane a wave owns 8 G groups, so for one leg its loads cover G 8-byte values
// at 8 G consecutive positions for each of the 8 members (positions
// g + 64 m): runs of 64 G bytes instead of one 512-byte run.  G = 2 (two
// adjacent groups per lane, 16 values per lane) makes every run a whole
// 128-byte line and every access 16 bytes; M = 2 (two members per lane) does
// it with 8-byte accesses and replaces the DPP step by a register rename.
// Each cross-lane step costs one VALU instruction per 32-bit value moved
// (permlane swaps: one per two values; DPP: a move and a select per value),
// where an LDS exchange costs two memory instructions per 64-bit value.
#pragma once

#include "kernels.hpp"

namespace stockfft {

// G adjacent groups per lane; M members of each group per lane (M = 1: the
// member is lane bits 3..5; M = 2: its low two bits are lane bits 4..5 and
// its top bit selects one of the lane's two butterflies of the group, so a
// wave holds 16 whole groups and one leg of a wave's loads covers four
// 128-byte lines with 8-byte accesses, and the transpose needs no DPP).
template <class Base, int G_, int M_ = 1>
struct WaveExchange : Base {
  static_assert(Base::N == 4096 && Base::P == 4 && Base::radix(0) == 8 && Base::radix(1) == 8 &&
                    Base::radix(2) == 8 && Base::radix(3) == 8,
                "the in-wave exchange is derived for the radix-8 plan of 4096 points");
  static_assert((G_ == 1 || G_ == 2) && (M_ == 1 || M_ == 2), "one or two groups / members per lane");
  static_assert(Base::E == 8 * G_ * M_ && Base::TPB == 1 && Base::C == 1, "shape");
  static constexpr int WX = G_;
  static constexpr int WXM = M_;
  // The one LDS exchange uses its own swizzle over 4096 elements (wx_slot).
  static constexpr int LDS_ELEMS = 4096;
};

template <class S, class = void>
struct wave_exchange : std::integral_constant<int, 0> {};
template <class S>
struct wave_exchange<S, std::void_t<decltype(S::WX)>> : std::integral_constant<int, S::WX> {};
template <class S, class = void>
struct wave_members : std::integral_constant<int, 0> {};
template <class S>
struct wave_members<S, std::void_t<decltype(S::WXM)>> : std::integral_constant<int, S::WXM> {};

// Physical LDS slot of exchange position i = 64 q + 8 b + c (c, b in [0, 8)):
// bits 0..4 of i are xor-ed with bits 6..9, a bijection inside every block
// of 64 that leaves bits 5 and up alone.  For both access patterns of the
// exchange (writes at 64 g + m + 8 r, reads at h + 64 m + 512 r; lanes vary
// the group's low bits and the member's lane bits) any 32 consecutive lanes
// then hit 32 different 8-byte slots modulo 32, i.e. all 64 four-byte banks
// once (checked on the CPU for every access of both layouts).
template <int M>
__device__ __forceinline__ int wx_slot(int i) {
  const int q = i >> 6;
  if constexpr (M == 1) {
    return i ^ (q & 7) ^ (((q ^ (q >> 3)) & 1) << 3) ^ (((q >> 1) & 1) << 4);
  } else {
    // Two members per lane: the lanes of one access vary the group's low four
    // bits and two member bits; bits 0..4 are xor-ed with bits 9, 6, 7, 8 and
    // 9 ^ 6 of i.
    return i ^ ((q >> 3) & 1) ^ ((q & 7) << 1) ^ ((((q >> 3) ^ q) & 1) << 4);
  }
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

// The same transpose with M members of the group per lane: member bit k
// pairs with leg bit k; member bits below LB = log2(8 / M) are lane bits
// 6 - LB + k (swapped across lanes), the others select the lane's butterfly
// (swapped between registers, which costs nothing).
template <int M>
__device__ __forceinline__ void transpose_members(c32 (&v)[M][8], bool hi3) {
  if constexpr (M == 1) {
    transpose8(v[0], hi3);
  } else {
    static_assert(M == 2, "members per lane");
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int r = 0; r < 8; r += 2) {  // member bit 0: lane bit 4, leg bit 0
        swap_lanes16(v[s][r].x, v[s][r + 1].x);
        swap_lanes16(v[s][r].y, v[s][r + 1].y);
      }
#pragma unroll
      for (int r = 0; r < 8; r += (r & 1) ? 3 : 1) {  // member bit 1: lane bit 5, leg bit 1
        swap_lanes32(v[s][r].x, v[s][r + 2].x);
        swap_lanes32(v[s][r].y, v[s][r + 2].y);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // member bit 2: the butterfly, leg bit 2
      const c32 t = v[1][r];
      v[1][r] = v[0][r + 4];
      v[0][r + 4] = t;
    }
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

// One 4096-point transform per workgroup of 512 / (G M) lanes.  Lane l of
// wave w holds, for u < G and s < M, member m = (l >> (6 - LB)) + 2^LB s of
// group G (GPW w + (l mod GPW)) + u, where LB = log2(8 / M) member bits sit
// at the top of the lane index and GPW = 64 / 2^LB groups share a wave.
template <class S>
struct WxLane {
  static constexpr int G = S::WX;
  static constexpr int M = S::WXM;
  static constexpr int LB = M == 1 ? 3 : 2;
  static constexpr int GPW = 64 >> LB;
  static constexpr int MS = 1 << LB;  // member stride between a lane's butterflies
  int m0;    // the lane's first member
  int g0;    // the lane's first group
  bool hi3;  // lane bit 3 (the DPP step of the one-member transpose)
  __device__ __forceinline__ explicit WxLane(int tid)
      : m0((tid & 63) >> (6 - LB)), g0(G * (GPW * (tid >> 6) + (tid & (GPW - 1)))),
        hi3((tid & 8) != 0) {}
  __device__ __forceinline__ int member(int s) const { return m0 + MS * s; }
};

// The lane's values (a[u][s][r]: leg r of its butterfly (u, s)) and every
// twiddle it applies: pass 1 (k = m, shared by the lane's groups), pass 2
// (k = h, shared by its members), pass 3 (k = h + 64 m).
template <class S>
struct WxRegs {
  c32 a[S::WX][S::WXM][8];
  c32 w1[S::WXM][8], w2[S::WX][8], w3[S::WX][S::WXM][8];
};

// Pass 0 legs (butterfly g + 64 m reads x[g + 64 m + 512 r]) and the
// twiddles, issued behind them.
template <class S, class IO>
__device__ __forceinline__ void wx_load(WxRegs<S>& R, const WxLane<S>& L, const void* in,
                                        const c32* tw, int64_t row) {
  constexpr int G = S::WX, M = S::WXM, B = IO::BYTES;
  const Buf src(static_cast<const char*>(in) + row * 4096 * B);
  const int voff = B * (L.g0 + 64 * L.m0);
#pragma unroll
  for (int s = 0; s < M; ++s)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      c32 v[G];
      WxAccess<IO, G>::load(v, src, voff, B * (64 * L.MS * s + 512 * r));
#pragma unroll
      for (int u = 0; u < G; ++u) R.a[u][s][r] = v[u];
    }
#pragma unroll
  for (int s = 0; s < M; ++s) fetch_twiddles<S, 1>(R.w1[s], 0, tw + S::tw_off(1), L.member(s));
#pragma unroll
  for (int u = 0; u < G; ++u) {
    fetch_twiddles<S, 2>(R.w2[u], 0, tw + S::tw_off(2), L.g0 + u);
#pragma unroll
    for (int s = 0; s < M; ++s)
      fetch_twiddles<S, 3>(R.w3[u][s], 0, tw + S::tw_off(3), L.g0 + u + 64 * L.member(s));
  }
}

template <class S, bool INV>
__device__ __forceinline__ void wx_dfts(WxRegs<S>& R) {
#pragma unroll
  for (int u = 0; u < S::WX; ++u)
#pragma unroll
    for (int s = 0; s < S::WXM; ++s) Dft<8, INV>::run(R.a[u][s]);
}

// The four passes.  Phase marks as run_passes sets them: 2p + 1 after pass
// p's arithmetic, 2p + 2 after the exchange that follows it.
template <class S, bool INV, class Pr>
__device__ __forceinline__ void wx_passes(WxRegs<S>& R, const WxLane<S>& L, c32* lds, Pr* pr) {
  constexpr int G = S::WX, M = S::WXM;
  if constexpr (kLdsPoison) {  // debug builds: the buffer starts as NaNs
#pragma unroll 1
    for (int i = threadIdx.x; i < S::LDS_ELEMS; i += S::THREADS) lds[i] = lds_poison();
    __syncthreads();
  }
  // Pass 0, in-wave exchange.
  wx_dfts<S, INV>(R);
  if constexpr (Pr::on) pr->mark(1);
#pragma unroll
  for (int u = 0; u < G; ++u) transpose_members<M>(R.a[u], L.hi3);
  if constexpr (Pr::on) pr->mark(2);
  // Pass 1 (Ns = 8).
#pragma unroll
  for (int u = 0; u < G; ++u)
#pragma unroll
    for (int s = 0; s < M; ++s)
#pragma unroll
      for (int r = 1; r < 8; ++r) R.a[u][s][r] = ctw<INV>(R.a[u][s][r], R.w1[s][r - 1]);
  wx_dfts<S, INV>(R);
  if constexpr (Pr::on) pr->mark(3);
  // The LDS exchange: butterfly 8 g + m writes leg r to 64 g + m + 8 r;
  // butterfly h + 64 m of pass 2 reads h + 64 m + 512 r.  Both slot maps are
  // one xor of a lane value with the leg's bits (wx_slot leaves bits 5 and
  // up alone and xors bits 0..4 with bits 6..9 only).
#pragma unroll
  for (int u = 0; u < G; ++u)
#pragma unroll
    for (int s = 0; s < M; ++s) {
      const int sb = wx_slot<M>(64 * (L.g0 + u) + L.member(s));
#pragma unroll
      for (int r = 0; r < 8; ++r) lds[sb ^ (8 * r)] = R.a[u][s][r];
    }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < G; ++u)
#pragma unroll
    for (int s = 0; s < M; ++s) {
      const int base = L.g0 + u + 64 * L.member(s);
      const int s0 = wx_slot<M>(base), s1 = wx_slot<M>(base + 512);
#pragma unroll
      for (int r = 0; r < 8; ++r) R.a[u][s][r] = lds[((r & 1) ? s1 - 512 : s0) + 512 * r];
      if constexpr (kLdsPoison)
#pragma unroll
        for (int r = 0; r < 8; ++r) lds[((r & 1) ? s1 - 512 : s0) + 512 * r] = lds_poison();
    }
  if constexpr (Pr::on) pr->mark(4);
  // Pass 2 (Ns = 64), in-wave exchange.
#pragma unroll
  for (int u = 0; u < G; ++u)
#pragma unroll
    for (int s = 0; s < M; ++s)
#pragma unroll
      for (int r = 1; r < 8; ++r) R.a[u][s][r] = ctw<INV>(R.a[u][s][r], R.w2[u][r - 1]);
  wx_dfts<S, INV>(R);
  if constexpr (Pr::on) pr->mark(5);
#pragma unroll
  for (int u = 0; u < G; ++u) transpose_members<M>(R.a[u], L.hi3);
  if constexpr (Pr::on) pr->mark(6);
  // Pass 3 (Ns = 512).
#pragma unroll
  for (int u = 0; u < G; ++u)
#pragma unroll
    for (int s = 0; s < M; ++s)
#pragma unroll
      for (int r = 1; r < 8; ++r) R.a[u][s][r] = ctw<INV>(R.a[u][s][r], R.w3[u][s][r - 1]);
  wx_dfts<S, INV>(R);
  if constexpr (Pr::on) pr->mark(7);
}

// Pass 3 output leg r of butterfly h + 64 m goes to h + 64 m + 512 r.
template <class S, class IO>
__device__ __forceinline__ void wx_store(const WxRegs<S>& R, const WxLane<S>& L, void* out,
                                         int64_t row) {
  constexpr int G = S::WX, M = S::WXM, B = IO::BYTES;
  const Buf dst(static_cast<char*>(out) + row * 4096 * B);
  const int voff = B * (L.g0 + 64 * L.m0);
#pragma unroll
  for (int s = 0; s < M; ++s)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      c32 v[G];
#pragma unroll
      for (int u = 0; u < G; ++u) v[u] = R.a[u][s][r];
      WxAccess<IO, G>::store(v, dst, voff, B * (64 * L.MS * s + 512 * r));
    }
}

template <class S, bool INV, class IO>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_stockham_wx(const void* in, void* out,
                                                             const c32* tw, int64_t rows) {
  __shared__ alignas(16) c32 lds[S::LDS_ELEMS];
  (void)rows;  // one row per workgroup: the grid is the batch
  const WxLane<S> L(threadIdx.x);
  WxRegs<S> R;
  wx_load<S, IO>(R, L, in, tw, blockIdx.x);
  wx_passes<S, INV, NoProbe>(R, L, lds, nullptr);
  wx_store<S, IO>(R, L, out, blockIdx.x);
}

// The fused forward -> weight -> adjoint kernel (k_spectral_energy's outputs)
// on the in-wave layout.  The forward's output register map (lane (h, m),
// leg r at h + 64 m + 512 r) is the input register map of the adjoint, so
// the adjoint runs on the registers in place; the weight of each value is
// read at its output position.
template <class S>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_spectral_energy_wx(
    const c32* x, const float* __restrict__ w, const float* __restrict__ scale, c32* grad,
    float* row_loss, const c32* tw, float* total_out, unsigned* counters, float* row_loss_all,
    int64_t rows_all, unsigned groups_all, unsigned gbase) {
  constexpr int G = S::WX, M = S::WXM;
  __shared__ alignas(16) c32 lds[S::LDS_ELEMS];
  __shared__ float red[S::THREADS / 64];
  __shared__ int is_last;
  const int tid = threadIdx.x;
  const int64_t row = blockIdx.x;  // one row per workgroup
  const WxLane<S> L(tid);
  WxRegs<S> R;
  wx_load<S, IoF32>(R, L, x, tw, row);
  wx_passes<S, false, NoProbe>(R, L, lds, nullptr);
  const float sc = scale ? 2.0f * scale[0] : 2.0f;
  float acc = 0.f;
  {
    const Buf wb(w);
    const int voff = 4 * (L.g0 + 64 * L.m0);
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int s = 0; s < M; ++s)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const float wq = __uint_as_float(wb.ld32(voff, 4 * (u + 64 * L.MS * s + 512 * r)));
          const float w2 = wq * wq;
          const c32 y = R.a[u][s][r];
          acc += w2 * (y.x * y.x + y.y * y.y);
          const float g = sc * w2;
          R.a[u][s][r] = c32{g * y.x, g * y.y};
        }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();  // forward passes done with the LDS; wave partials visible
  if (tid == 0) {
    float total = 0.f;
#pragma unroll
    for (int i = 0; i < S::THREADS / 64; ++i) total += red[i];
    if (total_out != nullptr) {
      // Published where every XCD sees it, then the workgroup counts itself
      // at once, so the counters' round trips overlap the adjoint instead of
      // waiting behind the gradient stores; this wave has nothing else in
      // flight here.
      atomicExch(&row_loss[row], total);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      is_last = fused_loss_count(counters, groups_all, gbase + blockIdx.x);
    } else {
      row_loss[row] = total;
    }
  }
  if (grad != nullptr) {  // uniform across the launch
    wx_passes<S, true, NoProbe>(R, L, lds, nullptr);
    wx_store<S, IoF32>(R, L, grad, row);
  }
  if (total_out != nullptr) {  // uniform across the launch
    __syncthreads();  // is_last visible; the LDS free for the sum's tree
    if (is_last) fused_loss_sum<S>(reinterpret_cast<float*>(lds), total_out, row_loss_all, rows_all);
  }
}

template <class S>
hipError_t launch_spectral_energy_wx(const void* x, const float* w, const float* scale, void* grad,
                                     float* row_loss, float* total, unsigned* counters,
                                     const void* tw, int64_t batch, hipStream_t s) {
  const int64_t cap = max_groups_per_launch();
  for (int64_t r0 = 0; r0 < batch; r0 += cap) {
    const int64_t g = batch - r0 < cap ? batch - r0 : cap;
    k_spectral_energy_wx<S><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(
        static_cast<const c32*>(x) + r0 * 4096, w, scale,
        grad ? static_cast<c32*>(grad) + r0 * 4096 : nullptr, row_loss + r0,
        static_cast<const c32*>(tw), total, counters, row_loss, batch, (unsigned)batch,
        (unsigned)r0);
  }
  return hipGetLastError();
}

// The fused matched filter (k_matched_filter's output, (1/N) F^H(conj(h) .*
// F x)) on the in-wave layout: the filter spectrum is read at each value's
// output position and the inverse runs on the registers in place.
template <class S>
__global__ __launch_bounds__(S::THREADS, S::WPE) void k_matched_filter_wx(const c32* x,
                                                                   const c32* __restrict__ h,
                                                                   c32* out, const c32* tw) {
  constexpr int G = S::WX, M = S::WXM;
  __shared__ alignas(16) c32 lds[S::LDS_ELEMS];
  const int64_t row = blockIdx.x;  // one row per workgroup
  const WxLane<S> L(threadIdx.x);
  WxRegs<S> R;
  wx_load<S, IoF32>(R, L, x, tw, row);
  wx_passes<S, false, NoProbe>(R, L, lds, nullptr);
  constexpr float inv_n = 1.0f / 4096.0f;  // a power of two: exact
  {
    const Buf hb(h);
    const int voff = 8 * (L.g0 + 64 * L.m0);
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int s = 0; s < M; ++s)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const u32x2 hw = hb.ld64(voff, 8 * (u + 64 * L.MS * s + 512 * r));
          const c32 y = cmulc(R.a[u][s][r], c32{__uint_as_float(hw.x), __uint_as_float(hw.y)});
          R.a[u][s][r] = c32{y.x * inv_n, y.y * inv_n};
        }
  }
  __syncthreads();  // the forward's LDS reads are done before the inverse's writes
  wx_passes<S, true, NoProbe>(R, L, lds, nullptr);
  wx_store<S, IoF32>(R, L, out, row);
}

template <class S>
hipError_t launch_matched_filter_wx(const void* x, const void* h, void* out, const void* tw,
                                    int64_t batch, hipStream_t s) {
  const int64_t cap = max_groups_per_launch();
  for (int64_t r0 = 0; r0 < batch; r0 += cap) {
    const int64_t g = batch - r0 < cap ? batch - r0 : cap;
    k_matched_filter_wx<S><<<dim3((unsigned)g), dim3(S::THREADS), 0, s>>>(
        static_cast<const c32*>(x) + r0 * 4096, static_cast<const c32*>(h),
        static_cast<c32*>(out) + r0 * 4096, static_cast<const c32*>(tw));
  }
  return hipGetLastError();
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
