// Device building blocks of the Stockham autosort FFT for gfx950.
//
// Notation follows the paper (Section II): W_N = exp(-2 pi i / N); one
// Stockham pass of radix R applies N/R butterflies; butterfly j reads its R
// legs at j + r N/R, multiplies leg r by W_{Ns R}^{(j mod Ns) r} (Ns = product
// of the radices of the earlier passes), takes a length-R DFT and writes leg
// k to (j div Ns) Ns R + (j mod Ns) + k Ns.  After the last pass the output
// is in natural order (Section II-B), with no bit reversal.
//
// Work split (the two-tier model of Section III-B, re-derived for gfx950):
// a transform is owned by T lanes; each lane keeps E = N/T complex values in
// VGPRs (tier 1) and does E/R butterflies per pass.  The LDS (tier 2) is only
// an exchange buffer between passes: one buffer per transform, reused by
// every pass (Section IV-A), with an optional pad of one element every
// 2^PADLOG elements against bank conflicts.  The first pass reads global
// memory straight into registers and the last pass writes global memory
// straight from registers (the device-memory bypass of Section V-A).
//
// Register index convention: for every pass, lane t holds in a[m] the element
// at position t + m T of the buffer being read, so leg r of the lane's b-th
// butterfly (j = t + b T) is a[b + r E/R].  With this convention the global
// load of the first pass and the global store of the last pass are both
// a[m] <-> x[t + m T]: consecutive lanes touch consecutive 8-byte elements.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "buffer.hpp"

namespace stockfft {

// ------------------------------------------------------------------ complex

// Interleaved complex64; 8-byte aligned so global and LDS accesses are single
// 64-bit operations.
struct alignas(8) c32 {
  float x, y;
};

__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c32 cmul(c32 a, c32 w) {
  return {a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
}
// a * conj(w)
__device__ __forceinline__ c32 cmulc(c32 a, c32 w) {
  return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}
template <bool INV>
__device__ __forceinline__ c32 ctw(c32 a, c32 w) {
  if constexpr (INV) return cmulc(a, w);
  else return cmul(a, w);
}
// multiply by -i (forward) or +i (backward): the root W_4^1 of the direction
template <bool INV>
__device__ __forceinline__ c32 mul_w4(c32 a) {
  if constexpr (INV) return {-a.y, a.x};
  else return {a.y, -a.x};
}

// cos/sin of k pi / 8, rounded once from their exact values.
constexpr float kC1 = 0.923879532511286756128f;  // cos(pi/8)
constexpr float kS1 = 0.382683432365089771728f;  // sin(pi/8)
constexpr float kR2 = 0.707106781186547524401f;  // cos(pi/4)

// v * W_R^k for the direction (W = e^{-2 pi i / R} forward, its conjugate
// backward), with k and R compile-time; exact roots need no multiply.
template <int R, int K, bool INV>
__device__ __forceinline__ c32 mul_root(c32 v) {
  constexpr int k16 = (K * 16 / R) & 15;  // the same root expressed in W_16
  static_assert((K * 16) % R == 0, "roots beyond W_16 are not tabulated");
  if constexpr (k16 == 0) {
    return v;
  } else if constexpr (k16 == 4) {
    return mul_w4<INV>(v);
  } else if constexpr (k16 == 8) {
    return {-v.x, -v.y};
  } else if constexpr (k16 == 12) {
    return mul_w4<!INV>(v);
  } else if constexpr (k16 == 2 || k16 == 6 || k16 == 10 || k16 == 14) {
    // (+-r2, +-r2) roots: two multiplies.
    constexpr float cr = (k16 == 2 || k16 == 14) ? kR2 : -kR2;
    constexpr float si = (k16 == 2 || k16 == 6) ? -kR2 : kR2;  // forward sign
    constexpr float s = INV ? -si : si;
    return {cr * v.x - s * v.y, cr * v.y + s * v.x};
  } else {
    // odd multiples of pi/8
    constexpr float c = (k16 == 1 || k16 == 15) ? kC1 : (k16 == 3 || k16 == 13) ? kS1
                        : (k16 == 5 || k16 == 11) ? -kS1 : -kC1;
    constexpr float sf = (k16 == 1 || k16 == 7) ? -kS1 : (k16 == 3 || k16 == 5) ? -kC1
                         : (k16 == 9 || k16 == 15) ? kS1 : kC1;
    constexpr float s = INV ? -sf : sf;
    return {c * v.x - s * v.y, c * v.y + s * v.x};
  }
}

// ---------------------------------------------------------------- DFT_R
// In-register length-R DFT, R in {2, 4, 8, 16}, natural-order in and out,
// by radix-2 decimation in time: DFT_R = combine(DFT_{R/2}(even),
// W_R^k * DFT_{R/2}(odd)).  For R = 8 this is the split DIT butterfly of
// Section V-B, eq. (4).

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(c32 (&v)[2]) {
    c32 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int R, bool INV>
struct Dft {
  template <int K>
  __device__ __forceinline__ static void combine(c32 (&v)[R], const c32 (&e)[R / 2],
                                                 const c32 (&o)[R / 2]) {
    if constexpr (K < R / 2) {
      c32 t = mul_root<R, K, INV>(o[K]);
      v[K] = cadd(e[K], t);
      v[K + R / 2] = csub(e[K], t);
      combine<K + 1>(v, e, o);
    }
  }
  __device__ __forceinline__ static void run(c32 (&v)[R]) {
    c32 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    Dft<R / 2, INV>::run(e);
    Dft<R / 2, INV>::run(o);
    combine<0>(v, e, o);
  }
};

// -------------------------------------------------------------- LDS poison
// Debug builds (STOCKFFT_LDS_POISON defined) fill each exchange buffer with
// NaNs before the first exchange and overwrite every slot with a NaN as soon
// as it has been read.  A read that a missing barrier lets run before its
// write then returns a NaN, and so does a slot whose next write a missing
// barrier lets run before its last read (the reader's poison lands on the new
// value): either way the transform's output turns NaN.
#ifdef STOCKFFT_LDS_POISON
constexpr bool kLdsPoison = true;
#else
constexpr bool kLdsPoison = false;
#endif
__device__ __forceinline__ c32 lds_poison() { return c32{__builtin_nanf(""), __builtin_nanf("")}; }

// ------------------------------------------------------------- plan shape

template <int... Rs>
struct RadixList {
  static constexpr int P = sizeof...(Rs);
  static constexpr int r[P] = {Rs...};
};

// N points, E values per lane, TPB transforms per workgroup, LDS layout
// PADLOG (> 0: a pad element every 2^PADLOG; 0: none; -1: XOR swizzle, see
// pidx), radices of the passes in order.
//
// C > 1 splits every exchange into C rounds through a buffer of N/C elements
// (plus pad): the transform stays whole in registers and the LDS is only the
// pipe between them, so a large transform needs a fraction of the LDS and
// several workgroups fit on one CU.  In the exchange after pass p, butterfly
// b of a lane writes only to chunk floor(b C / BPT_p) and read slot m comes
// from chunk floor(m C / E), both known at compile time, provided C divides
// BPT_p = E / R_p and Ns_{p+1} <= N / C (checked below).
//
// PF = 1 loads each pass's twiddles one pass ahead (latency hidden behind a
// pass, registers spent); PF = 2 loads every pass's twiddles together with the
// input (for one workgroup per CU, where registers are plentiful and a pass
// is too short to hide an L2 round trip); PF = 0 loads them at the start of
// their pass (for shapes that need the registers for occupancy).  WPE is the minimum
// number of waves per SIMD the compiler must allow for (1 = no constraint).
template <int C_, int PF_, int WPE_, int N_, int E_, int TPB_, int PADLOG_, int... Rs>
struct ShapeX {
  using L = RadixList<Rs...>;
  static constexpr int C = C_;
  static constexpr int PF = PF_;
  static constexpr int WPE = WPE_;
  static constexpr int N = N_;
  static constexpr int E = E_;
  static constexpr int T = N_ / E_;
  static constexpr int TPB = TPB_;
  static constexpr int PADLOG = PADLOG_;
  static constexpr int P = L::P;
  static constexpr int THREADS = T * TPB;
  static constexpr int CHUNK = N / C;
  static constexpr int LDS_ELEMS = CHUNK + (PADLOG > 0 ? (CHUNK >> PADLOG) : 0);
  static constexpr int radix(int p) { return L::r[p]; }
  static constexpr int ns(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= L::r[i];
    return s;
  }
  // Offset of pass p's table: entries [r-1][k], r in [1,R_p), k in [0,Ns_p).
  static constexpr int tw_off(int p) {
    int o = 0;
    for (int i = 1; i < p; ++i) o += (L::r[i] - 1) * ns(i);
    return o;
  }
  static constexpr int TW_ELEMS = tw_off(P);
  // Twiddles one lane applies in pass p: E/R_p butterflies x (R_p - 1) legs.
  static constexpr int tw_per_lane(int p) { return p == 0 ? 0 : (E / L::r[p]) * (L::r[p] - 1); }
  // Where pass p's twiddles sit in a lane's twiddle registers: one set reused
  // per pass, or (PF = 2) every pass's in turn.
  static constexpr int tw_lane_off(int p) {
    int o = 0;
    if (PF == 2)
      for (int i = 1; i < p; ++i) o += tw_per_lane(i);
    return o;
  }
  static constexpr int TW_REGS = [] {
    int m = 1;
    for (int i = 1; i < P; ++i) m = tw_per_lane(i) > m ? tw_per_lane(i) : m;
    if (PF == 2 && tw_lane_off(P) > 1) m = tw_lane_off(P);
    return m;
  }();
  static constexpr bool valid() {
    if (ns(P) != N || T * E != N || THREADS > 1024 || THREADS < 1) return false;
    if (C < 1 || N % C != 0) return false;
    for (int i = 0; i < P; ++i)
      if (E % L::r[i] != 0) return false;
    for (int i = 0; i + 1 < P; ++i)
      if ((E / L::r[i]) % C != 0 || ns(i + 1) > CHUNK) return false;
    return true;
  }
  static_assert(valid(), "inconsistent Stockham shape");
  static_assert(PF >= 0 && PF <= 2, "unknown twiddle schedule");
  static_assert(PADLOG >= -1 && (PADLOG >= 0 || (CHUNK % 16 == 0 && radix(0) % 2 == 0)),
                "unknown LDS layout");
  // Physical LDS slot of exchange position i.  The XOR swizzle permutes the
  // pairs of each 16-element row (one sweep of the LDS banks) by bits 4..6 of
  // i: the stride-16 writes of a radix-16 pass then spread over the banks as
  // with padding, while pairs (2k, 2k + 1) stay adjacent and in order, so
  // they can still move as one 16-byte access, and no space is added.
  __device__ __forceinline__ static int pidx(int i) {
    if constexpr (PADLOG > 0) return i + (i >> PADLOG);
    else if constexpr (PADLOG < 0) return i ^ (((i >> 4) & 7) << 1);
    else return i;
  }
  // pidx(l + c) for a lane part l >= 0 and a part c >= 0 that is a constant
  // once the caller's loops are unrolled.  With padding, the pad count of
  // l + c is that of l + (c mod 2^PADLOG) plus c / 2^PADLOG, so one shift of
  // the lane part serves every c with the same low bits (all of them when
  // the lane part's low bits are known zero), and the rest folds into the
  // access's immediate offset instead of costing two vector instructions
  // per access.
  __device__ __forceinline__ static int pidx(int l, int c) {
    if constexpr (PADLOG > 0) {
      constexpr int M = (1 << PADLOG) - 1;
      return l + c + ((l + (c & M)) >> PADLOG) + (c >> PADLOG);
    } else {
      return pidx(l + c);
    }
  }
};

// Double-buffered exchange: consecutive exchanges alternate between two LDS
// buffers, so a pass's writes never meet the previous exchange's reads and
// the barrier after each exchange's reads is not needed (P - 1 barriers per
// transform instead of 2P - 3), for twice the LDS.  Whole-transform
// exchanges only (C = 1).
template <class Base>
struct DoubleBuffered : Base {
  static_assert(Base::C == 1, "double buffering takes whole-transform exchanges");
  static constexpr bool DB = true;
  static constexpr int BUF = Base::LDS_ELEMS;
  static constexpr int LDS_ELEMS = 2 * Base::LDS_ELEMS;
};

template <class S, class = void>
struct double_buffered : std::false_type {};
template <class S>
struct double_buffered<S, std::void_t<decltype(S::DB)>> : std::integral_constant<bool, S::DB> {};

// Paired twiddle table: in every pass of radix R >= 4 the twiddles for
// r = 2q + 1 and 2q + 2 sit side by side, entry [q][k] = (W^{k (2q + 1)},
// W^{k (2q + 2)}) with W = W_{Ns R} (the last pair holds W^{k (R - 1)} and a
// zero), so a lane fetches two twiddles with one 16-byte load: R/2 load
// instructions per butterfly instead of R - 1.  For consecutive k the pairs
// are consecutive, so a wave's load still covers whole cache lines.  Radix-2
// passes keep the plain layout (one twiddle per butterfly).
template <class Base>
struct PairedTwiddles : Base {
  static constexpr bool PT = true;
  static constexpr int tw_pass_elems(int p) {
    return p == 0 ? 0
           : Base::radix(p) >= 4 ? (Base::radix(p) / 2) * 2 * Base::ns(p)
                                 : (Base::radix(p) - 1) * Base::ns(p);
  }
  static constexpr int tw_off(int p) {
    int o = 0;
    for (int i = 1; i < p; ++i) o += tw_pass_elems(i);
    return o;
  }
  static constexpr int TW_ELEMS = tw_off(Base::P);
};

// Paired lanes: in the first pass and in the last pass, where a lane does
// BPT = E / R >= 2 butterflies, it takes BPT consecutive ones, j = BPT t + b,
// instead of j = t + b T.  The legs it then reads from global memory (first
// pass, legs j + r N/R) and writes to it (last pass, outputs j + k N/R) are
// BPT adjacent elements: one 16-byte access carries two complex64 values (an
// 8- or 16-byte access two or four 16-bit pairs) where the plain convention
// needs one access per value.  The passes in between keep the plain
// convention; only the first exchange's writes and the last exchange's reads
// see the other butterfly order.  With exchange rounds (C > 1) the first
// exchange's round h is written by the lanes t in [h T / C, (h + 1) T / C),
// whole waves when T / C is a multiple of 64.
template <class Base>
struct PairedLanes : Base {
  static constexpr bool PL = true;
  static_assert(Base::E / Base::radix(0) >= 2 || Base::E / Base::radix(Base::P - 1) >= 2,
                "paired lanes need two butterflies per lane in the first or the last pass");
};

template <class S, class = void>
struct paired_lanes : std::false_type {};
template <class S>
struct paired_lanes<S, std::void_t<decltype(S::PL)>> : std::integral_constant<bool, S::PL> {};

// Whether pass p runs a lane's butterflies in the paired order.
template <class S, int p>
constexpr bool paired_pass() {
  if constexpr (!paired_lanes<S>::value) return false;
  else return (p == 0 || p == S::P - 1) && S::E / S::radix(p) >= 2;
}

// Butterfly index of a lane's b-th butterfly in pass p.
template <class S, int p>
__device__ __forceinline__ int bfly_index(int t, int b) {
  if constexpr (paired_pass<S, p>()) return (S::E / S::radix(p)) * t + b;
  else return t + b * S::T;
}

// Buffer position that pass p reads into register slot m: leg m / BPT of
// the lane's butterfly m mod BPT, at j + (m / BPT) N / R.
template <class S, int p>
__device__ __forceinline__ int read_position(int t, int m) {
  constexpr int BPT = S::E / S::radix(p);
  if constexpr (paired_pass<S, p>()) return BPT * t + (m % BPT) + (m / BPT) * (S::T * BPT);
  else return t + m * S::T;
}

// Whether a transform's output register layout (the last pass's) is the
// input layout of the first pass, so that a second transform can run on the
// registers in place (the fused kernels).
template <class S>
constexpr bool round_trip_layout() {
  if constexpr (!paired_lanes<S>::value) return true;
  else return paired_pass<S, 0>() == paired_pass<S, S::P - 1>() &&
              S::radix(0) == S::radix(S::P - 1);
}

template <class S, class = void>
struct paired_twiddles : std::false_type {};
template <class S>
struct paired_twiddles<S, std::void_t<decltype(S::PT)>> : std::integral_constant<bool, S::PT> {};

// The R - 1 twiddles of pass p for the butterfly with k = j mod Ns, from the
// pass's table twp, into dst[off + 0 .. off + R - 2] (dst[off + r - 1] is the
// twiddle of leg r; off is a constant once the caller's loops are unrolled).
template <class S, int p, int CAP>
__device__ __forceinline__ void fetch_twiddles(c32 (&dst)[CAP], int off, const c32* twp, int k) {
  constexpr int R = S::radix(p);
  constexpr int NS = S::ns(p);
  static_assert(R - 1 <= CAP, "twiddle registers");
  const Buf tb(twp);  // the lane part of every offset is k
  if constexpr (paired_twiddles<S>::value && R >= 4) {
#pragma unroll
    for (int q = 0; q < R / 2; ++q) {
      const u32x4 v = tb.ld128(16 * k, 16 * q * NS);
      dst[off + 2 * q] = c32{__uint_as_float(v.x), __uint_as_float(v.y)};
      if (2 * q + 1 < R - 1) dst[off + 2 * q + 1] = c32{__uint_as_float(v.z), __uint_as_float(v.w)};
    }
  } else {
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const u32x2 v = tb.ld64(8 * k, 8 * (r - 1) * NS);
      dst[off + r - 1] = c32{__uint_as_float(v.x), __uint_as_float(v.y)};
    }
  }
}

// The common case: whole-transform exchange buffer, twiddles one pass ahead.
template <int N_, int E_, int TPB_, int PADLOG_, int... Rs>
using Shape = ShapeX<1, true, 1, N_, E_, TPB_, PADLOG_, Rs...>;

// ------------------------------------------------------------ one pass

// Issues the global loads of the twiddles this lane needs in pass p into
// registers.  With prefetch the caller consumes them one pass later, so their
// latency hides behind a whole pass of arithmetic and exchange.
template <class S, int p>
__device__ __forceinline__ void load_twiddles(c32 (&w)[S::TW_REGS], const c32* tw, int t) {
  if constexpr (p > 0 && p < S::P) {
    constexpr int R = S::radix(p);
    constexpr int NS = S::ns(p);
    constexpr int BPT = S::E / R;
    const c32* twp = tw + S::tw_off(p);
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int k = bfly_index<S, p>(t, b) & (NS - 1);
      fetch_twiddles<S, p>(w, S::tw_lane_off(p) + b * (R - 1), twp, k);
    }
    // Keep prefetched loads here: the scheduler would otherwise sink them to
    // their use, past the exchange barriers, and expose their latency.
    if constexpr (S::PF) __builtin_amdgcn_sched_barrier(0);
  }
}

// Twiddle multiply and butterflies of pass p.  With prefetch, w[] holds the
// pass-p twiddles on entry and the pass-(p+1) loads are issued after they
// are applied; without, the pass-p twiddles are loaded here.
template <class S, int p, bool INV>
__device__ __forceinline__ void pass_compute(c32 (&a)[S::E], c32 (&w)[S::TW_REGS],
                                             const c32* tw, int t) {
  constexpr int R = S::radix(p);
  constexpr int BPT = S::E / R;
  if constexpr (!S::PF) {
    // One butterfly at a time: its R - 1 twiddles are loaded, applied and
    // dead before the next butterfly's are needed (fewest live registers).
    constexpr int NS = S::ns(p);
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      c32 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = a[b + r * BPT];
      if constexpr (p > 0) {
        c32 wb[R - 1];
        fetch_twiddles<S, p>(wb, 0, tw + S::tw_off(p), bfly_index<S, p>(t, b) & (NS - 1));
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = ctw<INV>(v[r], wb[r - 1]);
      }
      Dft<R, INV>::run(v);
#pragma unroll
      for (int r = 0; r < R; ++r) a[b + r * BPT] = v[r];
    }
    return;
  }
  if constexpr (p > 0) {
#pragma unroll
    for (int b = 0; b < BPT; ++b)
#pragma unroll
      for (int r = 1; r < R; ++r)
        a[b + r * BPT] = ctw<INV>(a[b + r * BPT], w[S::tw_lane_off(p) + b * (R - 1) + (r - 1)]);
  }
  if constexpr (S::PF == 1) load_twiddles<S, p + 1>(w, tw, t);
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    c32 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[b + r * BPT];
    Dft<R, INV>::run(v);
#pragma unroll
    for (int r = 0; r < R; ++r) a[b + r * BPT] = v[r];
  }
}

// Writes butterfly b's R outputs of pass p to their Stockham positions in
// the exchange buffer (offset by the round's chunk start).
template <class S, int p>
__device__ __forceinline__ void exchange_write(const c32 (&a)[S::E], c32* lds, int t, int b,
                                               int chunk0) {
  constexpr int R = S::radix(p);
  constexpr int NS = S::ns(p);
  constexpr int BPT = S::E / R;
  // Leg 0's position (j / Ns) Ns R + j mod Ns is the lane part at b = 0
  // plus the part of b (powers of two T and Ns: j = t + b T never carries
  // across a multiple of Ns that t alone would not, and the paired order
  // only writes in the first pass, where Ns = 1).
  const auto wpos = [](int j) { return (j / NS) * NS * R + (j & (NS - 1)); };
  const int l = wpos(bfly_index<S, p>(t, 0));
  const int c = wpos(bfly_index<S, p>(0, b)) - chunk0;
  if constexpr (S::PADLOG < 0 && NS == 1) {
    // The swizzle keeps the pairs of this butterfly's consecutive outputs
    // adjacent and 16-byte aligned: one 16-byte store per pair.
#pragma unroll
    for (int k = 0; k < R; k += 2) {
      const c32 u = a[b + k * BPT], v = a[b + (k + 1) * BPT];
      *reinterpret_cast<float4*>(lds + S::pidx(l + c + k)) = float4{u.x, u.y, v.x, v.y};
    }
  } else {
#pragma unroll
    for (int k = 0; k < R; ++k) lds[S::pidx(l, c + k * NS)] = a[b + k * BPT];
  }
}

// Exchange after pass p: write the outputs to their Stockham positions and
// read the next pass's inputs (positions t + m T, or the paired order when the
// next pass is a paired last pass), in C rounds of N/C elements.  The buffer
// must be free on entry; it is free again on return unless the next pass is
// the last (which reads nothing more from it).
template <class S, int p>
__device__ __forceinline__ void exchange(c32 (&a)[S::E], c32* lds, int t) {
  constexpr int R = S::radix(p);
  constexpr int BPT = S::E / R;
  constexpr int BPC = BPT / S::C;  // butterflies per chunk
  constexpr int MPC = S::E / S::C;  // read slots per chunk
  constexpr bool PW = paired_pass<S, p>();      // paired writes (first pass)
  constexpr bool PR = paired_pass<S, p + 1>();  // paired reads (for the last pass)
  static_assert(!PW || p == 0, "only the first pass writes in the paired order");
  static_assert(!PW || S::C == 1 || S::T % S::C == 0, "paired rounds split by lanes");
  static_assert(!PR || S::C == 1 || S::radix(p + 1) % S::C == 0, "paired rounds split by legs");
  c32 nxt[S::E];
#pragma unroll
  for (int h = 0; h < S::C; ++h) {
    if (h > 0) __syncthreads();  // the previous round's reads are done
    if constexpr (PW) {
      // Lane t's butterflies all fall in chunk t / (T / C).
      if (S::C == 1 || t / (S::T / S::C) == h) {
#pragma unroll
        for (int b = 0; b < BPT; ++b) exchange_write<S, p>(a, lds, t, b, h * S::CHUNK);
      }
    } else {
#pragma unroll
      for (int b = h * BPC; b < (h + 1) * BPC; ++b) exchange_write<S, p>(a, lds, t, b, h * S::CHUNK);
    }
    __syncthreads();
    if constexpr (PR) {
      const auto at = [&](int m) {
        return S::pidx(read_position<S, p + 1>(t, 0), read_position<S, p + 1>(0, m) - h * S::CHUNK);
      };
#pragma unroll
      for (int m = h * MPC; m < (h + 1) * MPC; ++m) nxt[m] = lds[at(m)];
      if constexpr (kLdsPoison)
#pragma unroll
        for (int m = h * MPC; m < (h + 1) * MPC; ++m) lds[at(m)] = lds_poison();
    } else if constexpr (S::PADLOG < 0 && S::T % 128 == 0 && S::CHUNK % 128 == 0) {
      // The swizzle leaves bits 7 and up alone, so the read positions
      // t + m T stay a constant stride apart after it.
      const int base = S::pidx(t);
#pragma unroll
      for (int m = h * MPC; m < (h + 1) * MPC; ++m) nxt[m] = lds[base + m * S::T - h * S::CHUNK];
      if constexpr (kLdsPoison)
#pragma unroll
        for (int m = h * MPC; m < (h + 1) * MPC; ++m) lds[base + m * S::T - h * S::CHUNK] = lds_poison();
    } else {
#pragma unroll
      for (int m = h * MPC; m < (h + 1) * MPC; ++m) nxt[m] = lds[S::pidx(t, m * S::T - h * S::CHUNK)];
      if constexpr (kLdsPoison)
#pragma unroll
        for (int m = h * MPC; m < (h + 1) * MPC; ++m) lds[S::pidx(t, m * S::T - h * S::CHUNK)] = lds_poison();
    }
  }
#pragma unroll
  for (int m = 0; m < S::E; ++m) a[m] = nxt[m];
  if constexpr (p + 2 < S::P && !double_buffered<S>::value)
    __syncthreads();  // all reads done before the next overwrite
}

// Phase marks of the pass pipeline.  The product kernels take NoProbe,
// whose marks compile to nothing; a timeline probe records a clock reading
// at each mark: mark 2p + 1 after pass p's arithmetic, 2p + 2 after the
// exchange that follows it.
struct NoProbe {
  static constexpr bool on = false;
  __device__ __forceinline__ void mark(int) {}
};

// Runs passes p..P-1.  On entry a[] holds the pass-p inputs in the register
// convention (and, with prefetch, w[] the pass-p twiddles).  On exit a[]
// holds the transform in natural order, a[m] at position t + m T.  The
// exchange buffer must be free to overwrite on entry (the caller's barrier).
template <class S, int p, bool INV, class Pr>
__device__ __forceinline__ void run_passes_from(c32 (&a)[S::E], c32 (&w)[S::TW_REGS], c32* lds,
                                                const c32* tw, int t, Pr* pr) {
  if constexpr (kLdsPoison && p == 0 && S::P > 1) {
    // The transform's whole exchange buffer (both halves when double
    // buffered) starts as NaNs.
#pragma unroll 1
    for (int i = t; i < S::LDS_ELEMS; i += S::T) lds[i] = lds_poison();
    __syncthreads();
  }
  pass_compute<S, p, INV>(a, w, tw, t);
  if constexpr (Pr::on) pr->mark(2 * p + 1);
  if constexpr (p + 1 < S::P) {
    if constexpr (double_buffered<S>::value)
      exchange<S, p>(a, lds + (p & 1) * S::BUF, t);
    else
      exchange<S, p>(a, lds, t);
    if constexpr (Pr::on) pr->mark(2 * p + 2);
    run_passes_from<S, p + 1, INV>(a, w, lds, tw, t, pr);
  }
}

// All passes of one transform.  Called right after the lane's input loads
// were issued, so the first twiddle loads queue behind them.
template <class S, int p>
__device__ __forceinline__ void load_all_twiddles(c32 (&w)[S::TW_REGS], const c32* tw, int t) {
  if constexpr (p < S::P) {
    load_twiddles<S, p>(w, tw, t);
    load_all_twiddles<S, p + 1>(w, tw, t);
  }
}

// The twiddle loads a shape issues together with the input (PF = 2: all of
// them); nothing for the other schedules.
template <class S>
__device__ __forceinline__ void preload_twiddles(c32 (&w)[S::TW_REGS], const c32* tw, int t) {
  if constexpr (S::PF == 2) load_all_twiddles<S, 1>(w, tw, t);
}

// All passes, with w[] as preload_twiddles left it.
template <class S, bool INV, class Pr = NoProbe>
__device__ __forceinline__ void run_passes_preloaded(c32 (&a)[S::E], c32 (&w)[S::TW_REGS],
                                                     c32* lds, const c32* tw, int t,
                                                     Pr* pr = nullptr) {
  run_passes_from<S, 0, INV>(a, w, lds, tw, t, pr);
}

template <class S, bool INV, class Pr = NoProbe>
__device__ __forceinline__ void run_passes(c32 (&a)[S::E], c32* lds, const c32* tw,
                                           int t, Pr* pr = nullptr) {
  c32 w[S::TW_REGS];
  preload_twiddles<S>(w, tw, t);
  run_passes_from<S, 0, INV>(a, w, lds, tw, t, pr);
}

}  // namespace stockfft
